"""GPU parity on seeded random boxes: flow (planar, uniaxial, biaxial, shear
or none), strain rate and time, particle count (300 to 30,000), density
(0.05 to 0.95, so sparse boxes with long runs of empty cells occur), WCA or
LJ, cell-list variant, precision and sweep schedule (LDS-tiled, per
particle, autotuned, or the half list in FP32) are drawn per case, and the
pair sets, forces, energy and virial are compared with the FP64 oracle.
The cell counts of these boxes (6- to 18-bit keys) take one radix pass of a
6- to 10-bit digit or two passes of up to 9 bits.  Each case is built
twice: with pair digests (debug = 1; the pair sets come from the digest
sweep) and without; both times forces, energy and virial come from the
production sweep."""
import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import compare, oracle_positions, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

SWEEP_OPT = 3  # NCL_OPT_SWEEP: 0 tiled, 1 per particle, 2 autotuned, 3 half list
FLOWS = ("planar", "uniaxial", "biaxial", "shear", "none")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_3784_amd  # noqa: F401  (fails loudly if the library is missing)


def draw_case(seed):
    g = np.random.default_rng(8800 + seed)
    flow = FLOWS[int(g.integers(0, len(FLOWS)))]
    pot = wl.WCA if g.random() < 0.5 else wl.LJ25
    n = int(round(np.exp(g.uniform(np.log(300), np.log(30000)))))
    density = float(np.exp(g.uniform(np.log(0.05), np.log(0.95))))
    variant = ("ds", "do")[int(g.integers(0, 2))]
    precision = ("fp64", "fp32", "fp32k")[int(g.integers(0, 3))]
    sweeps = [0, 1, 2] + ([3] if precision == "fp32" else [])
    sweep = sweeps[int(g.integers(0, len(sweeps)))]
    if flow == "none":
        box = wl.make_box("none", 0.0, n, density=density, pot=pot, t=0.0, seed=9000 + seed)
    else:
        box = wl.make_box(flow, float(g.uniform(0.05, 1.0)), n, density=density, pot=pot,
                          t_frac=float(g.uniform(0.0, 2.0)), seed=9000 + seed)
    return box, variant, precision, sweep


@pytest.mark.parametrize("seed", range(64))
def test_random_box(seed):
    box, variant, precision, sweep = draw_case(seed)
    Lr, _, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    counts = oracle.ds_counts(Lr, box.pot.rc) if variant == "ds" else oracle.do_counts(Lr, box.pot.rc)
    if counts.min() < 1:
        pytest.skip("box thinner than the cut-off at this strain")
    x = oracle_positions(box)
    r = run_oracle(box, x)
    label = f"seed{seed}/{box.flow}/n{len(x)}/{variant}/{precision}/sweep{sweep}"
    # built with pair digests: pair sets (count and digest per particle),
    # forces from the production sweep
    g = run_gpu(box, x, variant, precision, options={SWEEP_OPT: sweep})
    compare(g, r, precision, label=label)
    assert g["stats"]["pairs"] == r.stats[1], label
    # built without digests: forces, energy, virial and the pair count
    g = run_gpu(box, x, variant, precision, debug=False, options={SWEEP_OPT: sweep})
    compare(g, r, precision, check_pairs=False, label=label + "/nodebug")
    assert g["stats"]["pairs"] == r.stats[1], label
