"""FP32 force accuracy near the WCA cut-off, where the pair force has
|f'| of about 60-75 eps/sigma^2 while |f| goes to zero (so the eps/sigma
floor of the per-particle bound applies).  46,656 isolated pairs, each at a
separation drawn from [1.103, 1.113] sigma (r_c = 1.1225 sigma; the FP32
error peaks there) in a random direction, sit on the sites of a dilute grid
of a deformed, remapped lattice; every particle has exactly one neighbour,
so its force error is that of one pair evaluation.  In a float32 emulation
with r^2 recomputed from the rounded FP32 components about 4 of these
particles exceed the bound; with r^2 carried from FP64 the worst is 6.7e-6.
The FP32 paths must keep the per-particle error within
1e-5 max(sum_j |f_ij|, eps/sigma) for every sweep schedule and both cell
lists, and the energy within 1e-7 of sum_i |u_i| with no floor."""
import functools

import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import run_gpu, run_oracle

pytestmark = pytest.mark.gpu

SWEEP_OPT = 3  # NCL_OPT_SWEEP: 0 tiled, 1 per particle, 3 half list
GRID = 36      # pairs on a GRID^3 grid of the reduced box


@functools.lru_cache(maxsize=1)
def pair_box():
    """Lattice of a planar-flow box at 0.35 of its period (after a remap
    step), sized so that grid sites are at least 3.3 sigma apart; one pair
    per site, centred on it."""
    n = 2 * GRID ** 3
    box = wl.make_box("planar", 0.5, n, density=2.0 / 3.7 ** 3, pot=wl.WCA, t_frac=0.35, seed=4321)
    Lr, _, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    g = np.random.default_rng(97531)
    ijk = np.stack(np.meshgrid(*[np.arange(GRID)] * 3, indexing="ij"), -1).reshape(-1, 3)
    sites = ((ijk + 0.5) / GRID) @ Lr.T
    u = g.normal(size=(len(sites), 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    r = g.uniform(1.103, 1.113, len(sites))
    half = 0.5 * r[:, None] * u
    x = np.empty((2 * len(sites), 3))
    x[0::2] = sites - half
    x[1::2] = sites + half
    return box, x


@functools.lru_cache(maxsize=1)
def pair_oracle():
    box, x = pair_box()
    return run_oracle(box, x, want_hash=False)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_3784_amd  # noqa: F401  (fails loudly if the library is missing)


@pytest.mark.parametrize("variant", ["ds", "do"])
@pytest.mark.parametrize("precision,sweep", [("fp32", 0), ("fp32", 1), ("fp32", 3), ("fp32k", 0), ("fp32k", 1)])
def test_isolated_pairs_near_wca_cutoff(variant, precision, sweep):
    box, x = pair_box()
    r = pair_oracle()
    assert (r.count == 1).all(), "grid sites too close: some particle has more than one neighbour"
    # every |F_i| is below 1.5 eps/sigma: the bound is close to its eps/sigma floor
    assert np.linalg.norm(r.F, axis=1).max() < 1.5
    g = run_gpu(box, x, variant, precision, debug=False, options={SWEEP_OPT: sweep})
    label = f"{variant}/{precision}/sweep{sweep}"
    assert g["stats"]["pairs"] == r.stats[1], label
    dF = np.linalg.norm(g["F"] - r.F, axis=1)
    cond = dF / np.maximum(r.fmag, 1.0)
    i = int(np.argmax(cond))
    assert cond[i] <= 1e-5, f"{label}: particle {i} force error {cond[i]:.3e}"
    assert np.linalg.norm(g["F"] - r.F) / np.linalg.norm(r.F) <= 1e-5, label
    # energy: the shifted WCA energy also vanishes at r_c (mean |u_i| here is
    # 0.003 eps); the FP32 paths evaluate the pair energy in FP64, so the
    # plain relative bound holds with no floor
    dU = abs(g["U"] - r.U)
    assert dU <= 1e-7 * np.abs(r.u).sum(), f"{label}: energy error {dU:.3e} (sum |u_i| {np.abs(r.u).sum():.3e})"
    assert np.abs(g["W"] - r.W).max() <= 1e-5 * r.fmag.sum(), label
