"""FP64 CPU oracle for the deforming-box pair-force path (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1412_3784_amd``) and never imports it.  The numerical work is in
``oracle.c`` (plain C, FP64, OpenMP over particles); this module compiles it
with gcc and wraps it with ctypes.  Every function cites the passage of Dobson,
Fox & Saracino (arXiv:1412.3784) it follows; see the header of oracle.c.

Parity pins: tests/test_oracle_*.py.  Functions without an independent pin are
marked "parity unpinned" in their docstring (none at present).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

E_BAD_AUT, E_FLOW, E_BOX_TOO_SMALL, E_NOMEM = -1, -2, -3, -4


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    I = ctypes.c_int
    lib.orc_expm.argtypes = [P, D, P]
    lib.orc_lattice_at.argtypes = [P, P, D, P]
    lib.orc_reduce.argtypes = [P, P, D, I, P, P, P, P]
    lib.orc_heights.argtypes = [P, P]
    lib.orc_ds_counts.argtypes = [P, D, P]
    lib.orc_qr.argtypes = [P, P, P]
    lib.orc_do_counts.argtypes = [P, D, P]
    lib.orc_do_neighbourhood.argtypes = [P, P, D, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, P, ctypes.c_int32]
    lib.orc_pairs_brute.argtypes = [P, I64, P, D, I64, P]
    lib.orc_pairs_brute.restype = I64
    lib.orc_forces_brute.argtypes = [P, I64, P, P, P, P, P, P, P, P, P]
    lib.orc_forces_cells.argtypes = [P, I64, P, P, P, I, P, I64, P, P, P, P, P, P, P, P]
    lib.orc_sllod.argtypes = [P, P, I64, P, P, D, I, P, P, D, D, I64, I, P]
    lib.orc_max_threads.restype = I
    _lib = lib
    return lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().orc_max_threads())


# --------------------------------------------------------------------------
# lattice (Sec. 2.1-2.2)
# --------------------------------------------------------------------------
def expm(A, t: float) -> np.ndarray:
    """exp(tA) (Sec. 2.1: L_t = exp(At) L0)."""
    A = _d(A).reshape(3, 3)
    E = np.zeros((3, 3))
    _load().orc_expm(_p(A), float(t), _p(E))
    return E


def lattice_at(L0, A, t: float) -> np.ndarray:
    """Unreduced basis L_t = exp(tA) L0 (Sec. 2.1)."""
    L0, A = _d(L0).reshape(3, 3), _d(A).reshape(3, 3)
    L = np.zeros((3, 3))
    _load().orc_lattice_at(_p(L0), _p(A), float(t), _p(L))
    return L


def reduce(L0, A, t: float, automorphisms) -> Tuple[np.ndarray, np.ndarray, Tuple[int, int]]:
    """Reduced basis (Sec. 2.2, KR eq:kr and the generalised-KR diagonal stretch).

    Returns (Lred, Mtot, (p, q)) with Lred = exp(diag(theta - p mu1 - q mu2)) L0
    = L_t Mtot.  Raises ValueError on an invalid automorphism or flow.
    """
    L0, A = _d(L0).reshape(3, 3), _d(A).reshape(3, 3)
    auts = list(automorphisms or [])
    aut = np.zeros(18, dtype=np.int32)
    for k, M in enumerate(auts):
        aut[9 * k: 9 * k + 9] = _i32(M).reshape(9)
    Lred = np.zeros((3, 3))
    Mtot = np.zeros((3, 3), dtype=np.int32)
    coef = np.zeros(2, dtype=np.int32)
    rc = _load().orc_reduce(_p(L0), _p(A), float(t), len(auts), _p(aut), _p(Lred), _p(Mtot), _p(coef))
    if rc != 0:
        raise ValueError(f"orc_reduce failed with code {rc}")
    return Lred, Mtot, (int(coef[0]), int(coef[1]))


def heights(L) -> np.ndarray:
    """Box heights h_i = 1/|row_i(L^-1)| (Sec. 4.1, Fig. bh)."""
    L = _d(L).reshape(3, 3)
    h = np.zeros(3)
    _load().orc_heights(_p(L), _p(h))
    return h


def ds_counts(L, rc: float) -> np.ndarray:
    """Dynamic-size cell counts c_i = floor(h_i / d_cut) (Sec. 4.1)."""
    L = _d(L).reshape(3, 3)
    c = np.zeros(3, dtype=np.int32)
    _load().orc_ds_counts(_p(L), float(rc), _p(c))
    return c


def qr(L) -> Tuple[np.ndarray, np.ndarray]:
    """L = Q R, R upper triangular with positive diagonal (Sec. 4.2, eq. R)."""
    L = _d(L).reshape(3, 3)
    Q, R = np.zeros((3, 3)), np.zeros((3, 3))
    if _load().orc_qr(_p(L), _p(Q), _p(R)) != 0:
        raise ValueError("singular basis")
    return Q, R


def do_counts(L, rc: float) -> np.ndarray:
    """Dynamic-offset cell counts l_i = floor(r_ii / d_cut) (Sec. 5.2)."""
    L = _d(L).reshape(3, 3)
    l = np.zeros(3, dtype=np.int32)
    _load().orc_do_counts(_p(L), float(rc), _p(l))
    return l


def do_neighbourhood(R, l, rc: float, a: int, b: int, c: int, tight: bool = False) -> np.ndarray:
    """Dynamic-offset neighbourhood of cell (a,b,c) as rows (a',b',c',i,j,k) (Sec. 4.2).

    tight=False: the paper's rule (home cell grown by one cell width; 27/30/34/36
    cells); tight=True: grown by d_cut only (a subset that still covers r < d_cut)."""
    R = _d(R).reshape(3, 3)
    l = _i32(l)
    out = np.zeros((128, 6), dtype=np.int32)
    n = _load().orc_do_neighbourhood(_p(R), _p(l), float(rc), int(a), int(b), int(c), int(bool(tight)),
                                     _p(out), 128)
    return out[:min(n, 128)].copy()


# --------------------------------------------------------------------------
# pair set and forces (Sec. 2 images, Sec. 3 cut-off, Sec. 4.1 cell list)
# --------------------------------------------------------------------------
def pot_array(pot) -> np.ndarray:
    return np.array([pot.eps, pot.sigma, pot.rc, float(pot.shift)], dtype=np.float64)


def pairs_brute(x, L, rc: float) -> np.ndarray:
    """All (i, j, m0, m1, m2) of the interacting set P, by brute force over images."""
    x, L = _d(x).reshape(-1, 3), _d(L).reshape(3, 3)
    n = x.shape[0]
    lib = _load()
    npairs = lib.orc_pairs_brute(_p(x), n, _p(L), float(rc), 0, None)
    if npairs < 0:
        raise ValueError("singular basis")
    out = np.zeros((max(npairs, 1), 5), dtype=np.int64)
    lib.orc_pairs_brute(_p(x), n, _p(L), float(rc), npairs, _p(out))
    return out[:npairs]


class Result:
    """F (N x 3), u (N, per-particle energy, half of each pair), U, W (3 x 3),
    count and hash per particle (full-list view: every neighbour image of i),
    stats (candidates, directed in-range pairs) for the cell-list path."""

    def __init__(self, F, u, U, W, count, hash_, stats=None, fmag=None):
        self.F, self.u, self.U, self.W, self.count, self.hash, self.stats = F, u, U, W, count, hash_, stats
        self.fmag = fmag  # per-particle sum of |f_ij| (cell-list path only)


def forces_brute(x, L, pot, Mkey=None) -> Result:
    """Forces/energy/virial over P by brute force (the plain definition)."""
    x, L = _d(x).reshape(-1, 3), _d(L).reshape(3, 3)
    n = x.shape[0]
    F = np.zeros((n, 3))
    u = np.zeros(n)
    U = np.zeros(1)
    W = np.zeros((3, 3))
    cnt = np.zeros(n, dtype=np.int64)
    hsh = np.zeros(n, dtype=np.uint64)
    Mk = None if Mkey is None else _i32(Mkey).reshape(3, 3)
    rc = _load().orc_forces_brute(_p(x), n, _p(L), _p(pot_array(pot)), _p(Mk), _p(F), _p(u), _p(U),
                                  _p(W), _p(cnt), _p(hsh))
    if rc != 0:
        raise ValueError(f"orc_forces_brute failed with code {rc}")
    return Result(F, u, float(U[0]), W, cnt, hsh)


def forces_cells(x, L, pot, Mkey=None, threads: int = 0, want_hash: bool = True, subset=None) -> Result:
    """Forces/energy/virial via the plain dynamic-size cell list (Sec. 4.1), FP64.

    subset: optional particle indices; only those are swept and the
    per-particle outputs follow its order (U and W then cover only them)."""
    x, L = _d(x).reshape(-1, 3), _d(L).reshape(3, 3)
    n = x.shape[0]
    sub = None if subset is None else np.ascontiguousarray(np.asarray(subset, dtype=np.int64))
    rows = n if sub is None else len(sub)
    F = np.zeros((rows, 3))
    u = np.zeros(rows)
    U = np.zeros(1)
    W = np.zeros((3, 3))
    cnt = np.zeros(rows, dtype=np.int64)
    hsh = np.zeros(rows, dtype=np.uint64) if want_hash else None
    st = np.zeros(2, dtype=np.int64)
    fm = np.zeros(rows)
    Mk = None if Mkey is None else _i32(Mkey).reshape(3, 3)
    rc = _load().orc_forces_cells(_p(x), n, _p(L), _p(pot_array(pot)), _p(Mk), int(threads), _p(sub),
                                  0 if sub is None else len(sub), _p(F), _p(u), _p(U), _p(W), _p(cnt),
                                  _p(hsh), _p(st), _p(fm))
    if rc == E_BOX_TOO_SMALL:
        raise ValueError("box too small: some c_i < 1")
    if rc != 0:
        raise ValueError(f"orc_forces_cells failed with code {rc}")
    return Result(F, u, float(U[0]), W, cnt, hsh, (int(st[0]), int(st[1])), fm)


def sllod(x, p, L0, A, t0, automorphisms, pot, h, mass, nsteps, threads: int = 0):
    """FP64 SLLOD trajectory with peculiar momenta in the deforming box (the
    box follows the flow, Sec. 2.1; remaps by the automorphisms, Sec. 2.2),
    symmetric splitting with the exact streaming drift; see orc_sllod.

    Returns (x, p, hist): final wrapped positions and momenta, and hist of
    shape (nsteps + 1, 8) = (t, U, W_xx, W_yy, W_zz, K_xx, K_yy, K_zz)."""
    x = _d(x).reshape(-1, 3).copy()
    p = _d(p).reshape(-1, 3).copy()
    n = x.shape[0]
    auts = list(automorphisms or [])
    aut = _i32(np.concatenate([_i32(M).reshape(9) for M in auts])) if auts else None
    hist = np.zeros((int(nsteps) + 1, 8))
    rc = _load().orc_sllod(_p(x), _p(p), n, _p(_d(L0).reshape(9)), _p(_d(A).reshape(9)), float(t0), len(auts),
                           _p(aut), _p(pot_array(pot)), float(h), float(mass), int(nsteps), int(threads), _p(hist))
    if rc != 0:
        raise ValueError(f"orc_sllod failed with code {rc}")
    return x, p, hist


def energy_balance(hist, A):
    """H(t_n) - H(t_0) + trapezoid integral of sum_a A_aa (K_aa + W_aa): zero
    along exact SLLOD solutions (see orc_sllod)."""
    hist = np.asarray(hist)
    a = np.diag(np.asarray(A, dtype=np.float64).reshape(3, 3))
    H = 0.5 * hist[:, 5:8].sum(axis=1) + hist[:, 1]
    rate = (a * (hist[:, 5:8] + hist[:, 2:5])).sum(axis=1)
    dt = np.diff(hist[:, 0])
    integ = np.concatenate([[0.0], np.cumsum(0.5 * dt * (rate[1:] + rate[:-1]))])
    return H - H[0] + integ
