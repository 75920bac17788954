"""Python binding of libnemdcl.so (include/nemdcl.h): argument marshalling only.

Every entry point of the C ABI is exposed under its own name (ncl_create,
ncl_set_lattice, ...); `Handle` bundles them for convenience.  Device buffers
are torch tensors on a ROCm device (torch supplies memory and streams only);
all arithmetic runs in the library's HIP kernels.  There is no CPU fallback:
if the library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnemdcl.so")

NCL_OK = 0
NCL_E_ARG, NCL_E_BOX_TOO_SMALL, NCL_E_LATTICE, NCL_E_CAPACITY = -1, -2, -3, -4
NCL_E_HIP, NCL_E_DEVICE_FLAG, NCL_E_STATE = -5, -6, -7
NCL_DYNAMIC_SIZE, NCL_DYNAMIC_OFFSET = 0, 1
NCL_PREC_FP64, NCL_PREC_FP32, NCL_PREC_FP32_KAHAN = 0, 1, 2
NCL_OPT_DO_TIGHT, NCL_OPT_CLOSE_RADIUS, NCL_OPT_BAND, NCL_OPT_SWEEP, NCL_OPT_DETERMINISTIC, NCL_OPT_SKIN = 0, 1, 2, 3, 4, 5
NCL_SWEEP_TILED, NCL_SWEEP_PARTICLE, NCL_SWEEP_AUTO, NCL_SWEEP_HALF, NCL_SWEEP_FUSED = 0, 1, 2, 3, 4

VARIANTS = {"ds": NCL_DYNAMIC_SIZE, "do": NCL_DYNAMIC_OFFSET}
PRECISIONS = {"fp64": NCL_PREC_FP64, "fp32": NCL_PREC_FP32, "fp32k": NCL_PREC_FP32_KAHAN}

EXPORTED = ["ncl_create", "ncl_destroy", "ncl_set_potential", "ncl_set_option", "ncl_set_lattice",
            "ncl_get_lattice", "ncl_cell_counts", "ncl_build_cells", "ncl_compute_forces",
            "ncl_debug_pairs", "ncl_get_stats", "ncl_last_error",
            "ncl_batch_create", "ncl_batch_destroy", "ncl_batch_set_potential", "ncl_batch_set_option",
            "ncl_batch_set_lattices", "ncl_batch_build_cells", "ncl_batch_compute_forces",
            "ncl_batch_debug_pairs", "ncl_batch_get_stats", "ncl_batch_get_lattices", "ncl_batch_sllod_run",
            "ncl_batch_last_error", "ncl_forces_noalloc"]
NCL_NOALLOC_MAX_N = 65536
NCL_NOALLOC_MAX_CELLS = 65536


class NclError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nemdcl error {code}: {msg}")
        self.code = code


class ncl_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("variant", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("cells", ctypes.c_int32 * 3), ("max_occupancy", ctypes.c_int32), ("ncells", ctypes.c_int64),
                ("candidates", ctypes.c_int64), ("pairs", ctypes.c_int64), ("fp64_pairs", ctypes.c_int64),
                ("neighbourhood", ctypes.c_int64), ("sweep", ctypes.c_int32), ("brick", ctypes.c_int32 * 3),
                ("tune_ms", ctypes.c_float * 5), ("list_rebuilds", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(there is no CPU fallback for the HIP path)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    sig = {
        "ncl_create": [ctypes.POINTER(P), I, P],
        "ncl_destroy": [P],
        "ncl_set_potential": [P, D, D, D, I],
        "ncl_set_option": [P, I, D],
        "ncl_set_lattice": [P, P, P, D, I, P],
        "ncl_get_lattice": [P, P, P, P],
        "ncl_cell_counts": [P, I, P],
        "ncl_build_cells": [P, I, P, I64, I, I],
        "ncl_compute_forces": [P, P, P, P],
        "ncl_debug_pairs": [P, P, P],
        "ncl_get_stats": [P, ctypes.POINTER(ncl_stats)],
        "ncl_last_error": [P],
        "ncl_batch_create": [ctypes.POINTER(P), I, P, ctypes.c_int32, P],
        "ncl_batch_destroy": [P],
        "ncl_batch_set_potential": [P, D, D, D, I],
        "ncl_batch_set_option": [P, I, D],
        "ncl_batch_set_lattices": [P, I, P, P, P, P, P],
        "ncl_batch_build_cells": [P, P, I, I],
        "ncl_batch_compute_forces": [P, P, P, P],
        "ncl_batch_debug_pairs": [P, P, P],
        "ncl_batch_get_stats": [P, ctypes.POINTER(ncl_stats)],
        "ncl_batch_get_lattices": [P, P, P],
        "ncl_batch_sllod_run": [P, P, P, P, P, P, D, D, I64, I, P],
        "ncl_batch_last_error": [P],
        "ncl_forces_noalloc": [I, P, P, P, D, I, P, P, I, I, P, I64, P, P, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = I
    lib.ncl_last_error.restype = ctypes.c_char_p
    lib.ncl_batch_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def _np(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(h, code: int) -> None:
    if code != NCL_OK:
        msg = _lib.ncl_last_error(h).decode() if h else ""
        raise NclError(code, msg)


# ---- the C entry points, one to one -------------------------------------
def ncl_create(device: int = 0, stream: int = 0):
    h = ctypes.c_void_p()
    _check(None, _lib.ncl_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream or None)))
    return h


def ncl_destroy(h) -> None:
    _check(h, _lib.ncl_destroy(h))


def ncl_set_potential(h, eps: float, sigma: float, rc: float, shift_energy: int) -> None:
    _check(h, _lib.ncl_set_potential(h, float(eps), float(sigma), float(rc), int(shift_energy)))


def ncl_set_option(h, option: int, value: float) -> None:
    _check(h, _lib.ncl_set_option(h, int(option), float(value)))


def ncl_set_lattice(h, L0, A, t: float, automorphisms=()) -> None:
    L0 = _np(L0, np.float64).reshape(9)
    A = _np(A, np.float64).reshape(9)
    auts = list(automorphisms or [])
    aut = np.zeros(18, dtype=np.int32)
    for k, M in enumerate(auts):
        aut[9 * k: 9 * k + 9] = _np(M, np.int32).reshape(9)
    _check(h, _lib.ncl_set_lattice(h, _ptr(L0), _ptr(A), float(t), len(auts), _ptr(aut) if auts else None))


def ncl_get_lattice(h) -> Tuple[np.ndarray, np.ndarray, Tuple[int, int]]:
    L = np.zeros(9)
    M = np.zeros(9, dtype=np.int32)
    c = np.zeros(2, dtype=np.int32)
    _check(h, _lib.ncl_get_lattice(h, _ptr(L), _ptr(M), _ptr(c)))
    return L.reshape(3, 3), M.reshape(3, 3), (int(c[0]), int(c[1]))


def ncl_cell_counts(h, variant: int) -> np.ndarray:
    c = np.zeros(3, dtype=np.int32)
    _check(h, _lib.ncl_cell_counts(h, int(variant), _ptr(c)))
    return c


def _dev_ptr(t, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def ncl_build_cells(h, variant: int, x, n: int, precision: int, debug: int = 0) -> None:
    import torch
    _check(h, _lib.ncl_build_cells(h, int(variant), _dev_ptr(x, torch.float64) if n else None, int(n),
                                   int(precision), int(debug)))


def ncl_compute_forces(h, F, U, W) -> None:
    import torch
    _check(h, _lib.ncl_compute_forces(h, _dev_ptr(F), _dev_ptr(U, torch.float64), _dev_ptr(W, torch.float64)))


def ncl_debug_pairs(h, count, hash_) -> None:
    import torch
    _check(h, _lib.ncl_debug_pairs(h, _dev_ptr(count, torch.int64), _dev_ptr(hash_, torch.int64)))


def ncl_get_stats(h) -> dict:
    s = ncl_stats()
    _check(h, _lib.ncl_get_stats(h, ctypes.byref(s)))
    return {"n": s.n, "variant": s.variant, "precision": s.precision, "cells": list(s.cells),
            "max_occupancy": s.max_occupancy, "ncells": s.ncells, "candidates": s.candidates,
            "pairs": s.pairs, "fp64_pairs": s.fp64_pairs, "neighbourhood": s.neighbourhood,
            "sweep": s.sweep, "brick": list(s.brick), "tune_ms": list(s.tune_ms),
            "list_rebuilds": s.list_rebuilds}


def ncl_last_error(h) -> str:
    return _lib.ncl_last_error(h).decode()


# ---- convenience wrapper -------------------------------------------------
class Handle:
    """One library handle bound to a device and a torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = ncl_create(device, self.stream.cuda_stream)
        self.n = 0
        self.precision = NCL_PREC_FP64

    def close(self):
        if self.h is not None:
            ncl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_potential(self, pot=None, *, eps=1.0, sigma=1.0, rc=2 ** (1 / 6), shift=1):
        if pot is not None:
            eps, sigma, rc, shift = pot.eps, pot.sigma, pot.rc, pot.shift
        ncl_set_potential(self.h, eps, sigma, rc, shift)

    def set_option(self, option: int, value: float):
        ncl_set_option(self.h, option, value)

    def set_lattice(self, L0, A, t, automorphisms=()):
        ncl_set_lattice(self.h, L0, A, t, automorphisms)

    def get_lattice(self):
        return ncl_get_lattice(self.h)

    def cell_counts(self, variant):
        return ncl_cell_counts(self.h, VARIANTS.get(variant, variant))

    def build_cells(self, variant, x, precision="fp64", debug=False):
        self.precision = PRECISIONS.get(precision, precision)
        self.n = int(x.shape[0])
        ncl_build_cells(self.h, VARIANTS.get(variant, variant), x, self.n, self.precision, int(debug))

    def compute_forces(self, F=None, U=None, W=None):
        import torch
        dt = torch.float64 if self.precision == NCL_PREC_FP64 else torch.float32
        if F is None:
            F = torch.empty((self.n, 3), dtype=dt, device=self.device)
        if U is None:
            U = torch.empty(1, dtype=torch.float64, device=self.device)
        if W is None:
            W = torch.empty(9, dtype=torch.float64, device=self.device)
        ncl_compute_forces(self.h, F, U, W)
        return F, U, W

    def debug_pairs(self):
        import torch
        c = torch.empty(self.n, dtype=torch.int64, device=self.device)
        hs = torch.empty(self.n, dtype=torch.int64, device=self.device)
        ncl_debug_pairs(self.h, c, hs)
        return c, hs

    def stats(self):
        return ncl_get_stats(self.h)


# ---- batched form ---------------------------------------------------------
def _bcheck(b, code: int) -> None:
    if code != NCL_OK:
        msg = _lib.ncl_batch_last_error(b).decode() if b else ""
        raise NclError(code, msg)


def ncl_batch_create(n_per_rep, device: int = 0, stream: int = 0):
    n = _np(n_per_rep, np.int64)
    b = ctypes.c_void_p()
    _bcheck(None, _lib.ncl_batch_create(ctypes.byref(b), int(device), ctypes.c_void_p(stream or None),
                                        len(n), _ptr(n)))
    return b


def ncl_batch_destroy(b) -> None:
    _bcheck(b, _lib.ncl_batch_destroy(b))


def ncl_batch_set_potential(b, eps, sigma, rc, shift_energy) -> None:
    _bcheck(b, _lib.ncl_batch_set_potential(b, float(eps), float(sigma), float(rc), int(shift_energy)))


def ncl_batch_set_option(b, option: int, value: float) -> None:
    _bcheck(b, _lib.ncl_batch_set_option(b, int(option), float(value)))


def ncl_batch_set_lattices(b, variant: int, L0s, As, ts, automorphisms) -> None:
    R = len(ts)
    L0 = _np(L0s, np.float64).reshape(R * 9)
    A = _np(As, np.float64).reshape(R * 9)
    t = _np(ts, np.float64).reshape(R)
    naut = np.zeros(R, dtype=np.int32)
    aut = np.zeros(R * 18, dtype=np.int32)
    for r, auts in enumerate(automorphisms):
        naut[r] = len(auts)
        for k, M in enumerate(auts):
            aut[18 * r + 9 * k: 18 * r + 9 * k + 9] = _np(M, np.int32).reshape(9)
    _bcheck(b, _lib.ncl_batch_set_lattices(b, int(variant), _ptr(L0), _ptr(A), _ptr(t), _ptr(naut), _ptr(aut)))


def ncl_batch_build_cells(b, x, precision: int, debug: int = 0) -> None:
    import torch
    _bcheck(b, _lib.ncl_batch_build_cells(b, _dev_ptr(x, torch.float64), int(precision), int(debug)))


def ncl_batch_compute_forces(b, F, U, W) -> None:
    import torch
    _bcheck(b, _lib.ncl_batch_compute_forces(b, _dev_ptr(F), _dev_ptr(U, torch.float64), _dev_ptr(W, torch.float64)))


def ncl_batch_debug_pairs(b, count, hash_) -> None:
    import torch
    _bcheck(b, _lib.ncl_batch_debug_pairs(b, _dev_ptr(count, torch.int64), _dev_ptr(hash_, torch.int64)))


def ncl_batch_get_stats(b) -> dict:
    s = ncl_stats()
    _bcheck(b, _lib.ncl_batch_get_stats(b, ctypes.byref(s)))
    return {"n": s.n, "variant": s.variant, "precision": s.precision, "max_occupancy": s.max_occupancy,
            "ncells": s.ncells, "candidates": s.candidates, "pairs": s.pairs, "fp64_pairs": s.fp64_pairs,
            "neighbourhood": s.neighbourhood, "list_rebuilds": s.list_rebuilds,
            "sweep": s.sweep, "tune_ms": list(s.tune_ms)}


def ncl_batch_get_lattices(b, nrep: int):
    L = np.zeros(9 * nrep)
    c = np.zeros(3 * nrep, dtype=np.int32)
    _bcheck(b, _lib.ncl_batch_get_lattices(b, _ptr(L), _ptr(c)))
    return L.reshape(nrep, 3, 3), c.reshape(nrep, 3)


def ncl_batch_sllod_run(b, x, p, F, U, W, h, mass, nsteps, use_graph, hist=None) -> None:
    import torch
    _bcheck(b, _lib.ncl_batch_sllod_run(b, _dev_ptr(x, torch.float64), _dev_ptr(p, torch.float64), _dev_ptr(F),
                                        _dev_ptr(U, torch.float64), _dev_ptr(W, torch.float64), float(h),
                                        float(mass), int(nsteps), int(use_graph),
                                        _dev_ptr(hist, torch.float64) if hist is not None else None))


def ncl_batch_last_error(b) -> str:
    return _lib.ncl_batch_last_error(b).decode()


def ncl_forces_noalloc(device: int, stream: int, L0, A, t: float, automorphisms, pot, variant: int,
                       precision: int, x, n: int, F, U, W) -> None:
    """The entry point that allocates nothing (see include/nemdcl.h): lattice,
    cells and forces of one box of at most NCL_NOALLOC_MAX_N particles.
    pot = (eps, sigma, r_c, shift flag); F, U, W are caller-owned device
    tensors."""
    import torch
    auts = list(automorphisms or [])
    aut = _np(np.concatenate([_np(M, np.int32).reshape(9) for M in auts]), np.int32) if auts else None
    L0a, Aa, pa = _np(L0, np.float64).reshape(9), _np(A, np.float64).reshape(9), _np(pot, np.float64).reshape(4)
    code = _lib.ncl_forces_noalloc(int(device), ctypes.c_void_p(stream or None), _ptr(L0a), _ptr(Aa), float(t),
                                   len(auts), _ptr(aut), _ptr(pa), int(variant), int(precision),
                                   _dev_ptr(x, torch.float64) if n else None, int(n),
                                   _dev_ptr(F) if n else None, _dev_ptr(U, torch.float64), _dev_ptr(W, torch.float64))
    if code != NCL_OK:
        raise NclError(code, "ncl_forces_noalloc")


class Batch:
    """A batch of independent replicas bound to a device and a torch stream."""

    def __init__(self, n_per_rep, device: int = 0, stream=None):
        import torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n = [int(v) for v in n_per_rep]
        self.nrep = len(self.n)
        self.ntot = int(sum(self.n))
        self.b = ncl_batch_create(self.n, device, self.stream.cuda_stream)
        self.precision = NCL_PREC_FP32

    def close(self):
        if self.b is not None:
            ncl_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_potential(self, pot):
        ncl_batch_set_potential(self.b, pot.eps, pot.sigma, pot.rc, pot.shift)

    def set_option(self, option, value):
        ncl_batch_set_option(self.b, option, value)

    def set_lattices(self, variant, L0s, As, ts, automorphisms):
        ncl_batch_set_lattices(self.b, VARIANTS.get(variant, variant), L0s, As, ts, automorphisms)

    def build_cells(self, x, precision="fp32", debug=False):
        self.precision = PRECISIONS.get(precision, precision)
        ncl_batch_build_cells(self.b, x, self.precision, int(debug))

    def _outputs(self, F, U, W):
        import torch
        dt = torch.float64 if self.precision == NCL_PREC_FP64 else torch.float32
        if F is None:
            F = torch.empty((self.ntot, 3), dtype=dt, device=self.device)
        if U is None:
            U = torch.empty(self.nrep, dtype=torch.float64, device=self.device)
        if W is None:
            W = torch.empty(self.nrep * 9, dtype=torch.float64, device=self.device)
        return F, U, W

    def compute_forces(self, F=None, U=None, W=None):
        F, U, W = self._outputs(F, U, W)
        ncl_batch_compute_forces(self.b, F, U, W)
        return F, U, W

    def debug_pairs(self):
        import torch
        c = torch.empty(self.ntot, dtype=torch.int64, device=self.device)
        hs = torch.empty(self.ntot, dtype=torch.int64, device=self.device)
        ncl_batch_debug_pairs(self.b, c, hs)
        return c, hs

    def stats(self):
        return ncl_batch_get_stats(self.b)

    def lattices(self):
        return ncl_batch_get_lattices(self.b, self.nrep)

    def sllod_run(self, x, p, h, mass, nsteps, use_graph=True, F=None, U=None, W=None, history=False):
        import torch
        F, U, W = self._outputs(F, U, W)
        hist = torch.zeros(((nsteps + 1) * self.nrep * 8,), dtype=torch.float64, device=self.device) if history else None
        ncl_batch_sllod_run(self.b, x, p, F, U, W, h, mass, nsteps, use_graph, hist)
        if hist is not None:
            hist = hist.view(nsteps + 1, self.nrep, 8)
        return F, U, W, hist
