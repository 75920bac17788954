"""Helpers for GPU-vs-oracle parity tests: run one box through the HIP
library and through the FP64 oracle on the same seeded positions, and
compare pair sets (exactly) and forces / energy / virial (to a tolerance)."""
from __future__ import annotations

import numpy as np

import oracle
import workloads as wl

# Per-particle force error bound, relative to max(sum_j |f_ij|, eps/sigma),
# and relative L2 error over all particles.  The eps/sigma floor covers
# particles whose only neighbours sit where the pair force crosses zero (the
# WCA cut-off): there the force's relative condition number r f'/f grows
# without bound, so no FP32 evaluation can hold a purely relative bound.
# FP64 mode is compared with a positions-rounding allowance: the library
# works from wrapped positions x - L n, which differ from the inputs by an
# ulp, and close pairs amplify that by ~12.
TOL_F = {"fp64": 1e-10, "fp32": 1e-5, "fp32k": 1e-5}
# energy: relative to sum of |u_i|
TOL_U = {"fp64": 1e-10, "fp32": 1e-7, "fp32k": 1e-7}
FORCE_FLOOR = 1.0  # eps / sigma


def oracle_positions(box: wl.Box) -> np.ndarray:
    """Positions at the box's strain time: x = L_t s (+ jitter), L_t from the oracle."""
    return box.positions(oracle.lattice_at(box.L0, box.A, box.t))


def run_oracle(box: wl.Box, x: np.ndarray, subset=None, want_hash=True):
    Lr, Mt, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    return oracle.forces_cells(x, Lr, box.pot, Mkey=Mt, want_hash=want_hash, subset=subset)


def run_gpu(box: wl.Box, x: np.ndarray, variant: str, precision: str, debug: bool = True, options=None,
            handle=None, L0=None, A=None, t=None, auts=None):
    import torch
    from paper_1412_3784_amd import Handle
    h = handle or Handle(0)
    h.set_potential(box.pot)
    for k, v in (options or {}).items():
        h.set_option(k, v)
    h.set_lattice(box.L0 if L0 is None else L0, box.A if A is None else A, box.t if t is None else t,
                  box.automorphisms if auts is None else auts)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    h.build_cells(variant, xt, precision, debug=debug)
    F, U, W = h.compute_forces()
    out = {}
    if debug:
        c, hs = h.debug_pairs()
        out["count"] = c.cpu().numpy()
        out["hash"] = hs.cpu().numpy().view(np.uint64)
    torch.cuda.synchronize()
    out["F"] = F.cpu().numpy().astype(np.float64)
    out["U"] = float(U.cpu().numpy()[0])
    out["W"] = W.cpu().numpy().reshape(3, 3)
    out["stats"] = h.stats()
    out["lattice"] = h.get_lattice()
    if handle is None:
        h.close()
    return out


def compare(g: dict, r, precision: str, check_pairs=True, label=""):
    """Assert parity; returns a dict of the measured errors."""
    tolF, tolU = TOL_F[precision], TOL_U[precision]
    if check_pairs:
        bad = np.nonzero(g["count"] != r.count)[0]
        assert len(bad) == 0, f"{label}: pair counts differ at {bad[:10]} ({len(bad)} particles)"
        bad = np.nonzero(g["hash"] != r.hash)[0]
        assert len(bad) == 0, f"{label}: pair sets differ at {bad[:10]} ({len(bad)} particles)"
    dF = np.linalg.norm(g["F"] - r.F, axis=1)
    scale = np.maximum(r.fmag, FORCE_FLOOR)
    cond = dF / scale
    worst = int(np.argmax(cond)) if len(cond) else 0
    l2 = np.linalg.norm(g["F"] - r.F) / max(np.linalg.norm(r.F), 1e-300)
    Fn = np.linalg.norm(r.F, axis=1)
    unc = dF[Fn > 0] / Fn[Fn > 0]
    errs = {"max_cond_F": float(cond.max()) if len(cond) else 0.0, "rel_l2_F": float(l2),
            "max_unconditioned_F": float(unc.max()) if len(unc) else 0.0}
    assert errs["max_cond_F"] <= tolF, f"{label}: particle {worst} force error {cond[worst]:.3e} > {tolF}"
    assert l2 <= tolF, f"{label}: relative L2 force error {l2:.3e}"
    usum = np.abs(r.u).sum() + 1e-300
    errs["rel_U"] = abs(g["U"] - r.U) / usum
    assert errs["rel_U"] <= tolU, f"{label}: energy error {errs['rel_U']:.3e}"
    wscale = r.fmag.sum() + 1e-300  # sum_P |r_ij| |f_ij| <= r_c sum_i fmag_i / 2
    errs["rel_W"] = float(np.abs(g["W"] - r.W).max() / wscale)
    assert errs["rel_W"] <= max(tolF, 1e-10), f"{label}: virial error {errs['rel_W']:.3e}"
    return errs
