"""GPU parity of the half-list sweep (each pair evaluated once, its force
applied to both particles): exact pair sets (every particle's count and
digest, the neighbour's side included) and forces within 1e-5 of
sum_j |f_ij| against the FP64 oracle; both cell-list variants; tiny boxes
where several images of one partner interact, the uniaxial strain sweep
across its remap, planar shear across Lees-Edwards resets, and boxes whose
workgroups overflow the LDS windows (neighbour forces then go straight to
the FP64 array)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import compare, oracle_positions, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

SWEEP_OPT, DET_OPT, HALF = 3, 4, 3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_3784_amd  # noqa: F401  (fails loudly if the library is missing)


def half(box, x, variant, **kw):
    return run_gpu(box, x, variant, "fp32", options={SWEEP_OPT: HALF}, **kw)


TINY = [(flow, side, tf) for flow in ("planar", "uniaxial", "biaxial", "none")
        for side, tf in ((1.3, 0.3), (2.6, 0.5), (3.7, 0.85), (4.9, 1.45))]


@pytest.mark.parametrize("flow,side,tf", TINY)
@pytest.mark.parametrize("variant", ["ds", "do"])
def test_half_tiny_boxes(flow, side, tf, variant):
    box = wl.make_box(flow, 0.7, 60, side=side * wl.WCA_RC, pot=wl.WCA, t_frac=tf, seed=7)
    Lr, _, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    counts = oracle.ds_counts(Lr, box.pot.rc) if variant == "ds" else oracle.do_counts(Lr, box.pot.rc)
    if counts.min() < 1:
        pytest.skip("box too small at this strain")
    x = oracle_positions(box)
    r = run_oracle(box, x)
    g = half(box, x, variant)
    compare(g, r, "fp32", label=f"half/{flow}/{side}/{tf}/{variant}")
    assert g["stats"]["sweep"] == HALF
    assert g["stats"]["pairs"] == r.stats[1]


@pytest.mark.parametrize("variant", ["ds", "do"])
def test_half_wca_planar_4096(variant):
    """4,096 WCA particles at 1.2 per cell: a workgroup's 256 slots span
    more rows than get windows, so neighbour forces take the direct path."""
    box = wl.wca_planar_4096()
    x = oracle_positions(box)
    r = run_oracle(box, x)
    g = half(box, x, variant)
    compare(g, r, "fp32", label=f"half/wca4096/{variant}")
    assert g["stats"]["pairs"] == r.stats[1]


@pytest.mark.parametrize("k", [0, 21, 31, 32, 33, 63])
@pytest.mark.parametrize("variant", ["ds", "do"])
def test_half_lj_uniaxial_strain_sweep_reduced_n(k, variant):
    """uniaxial LJ, 65,536 particles (13 per cell: windows in use) across
    the remap; the half list checks about half the candidates of the full
    per-particle sweep."""
    box = wl.lj_uniaxial_strain(k=k, n=65536)
    x = oracle_positions(box)
    r = run_oracle(box, x)
    g = half(box, x, variant)
    compare(g, r, "fp32", label=f"half/lj_uniaxial/k{k}/{variant}")
    assert g["stats"]["pairs"] == r.stats[1]
    full = run_gpu(box, x, variant, "fp32", debug=False, options={SWEEP_OPT: 1})
    ratio = g["stats"]["candidates"] / full["stats"]["candidates"]
    assert 0.45 < ratio < 0.56, ratio
    assert abs(g["U"] - full["U"]) <= 1e-7 * np.abs(r.u).sum()


@pytest.mark.parametrize("tf", [0.2, 0.49, 0.51, 1.0, 1.51])
@pytest.mark.parametrize("variant", ["ds", "do"])
def test_half_shear_lees_edwards(tf, variant):
    box = wl.make_box("shear", 1.0, 3000, density=0.8, pot=wl.LJ25, t_frac=tf, seed=31)
    x = oracle_positions(box)
    r = run_oracle(box, x)
    g = half(box, x, variant)
    compare(g, r, "fp32", label=f"half/shear/{tf}/{variant}")


def test_half_grid_jitter_biaxial():
    """the biaxial grid construction (grid + jitter, biaxial, t = T/2) at 32^3."""
    box = wl.lj_biaxial_grid(grid=32)
    x = oracle_positions(box)
    r = run_oracle(box, x)
    for variant in ("ds", "do"):
        g = half(box, x, variant)
        compare(g, r, "fp32", label=f"half/lj_biaxial_grid/{variant}")


def test_half_paper_neighbourhood_rule():
    """dynamic offset with rows grown by a whole cell (the paper's rule)."""
    from paper_1412_3784_amd import nemdcl as n
    box = wl.make_box("biaxial", 0.3, 20000, density=0.8, pot=wl.LJ25, t_frac=0.3, seed=5)
    x = oracle_positions(box)
    r = run_oracle(box, x)
    g = run_gpu(box, x, "do", "fp32", options={SWEEP_OPT: HALF, n.NCL_OPT_DO_TIGHT: 0})
    compare(g, r, "fp32", label="half/paper-rule")


def test_half_repeat_and_autotuner():
    """Two half-list passes agree to rounding (the summation order of the
    atomics varies); with determinism relaxed the autotuner also times the
    half list, and by default it does not."""
    import torch
    from paper_1412_3784_amd import Handle
    box = wl.lj_uniaxial_strain(k=40, n=65536)
    x = oracle_positions(box)
    r = run_oracle(box, x, want_hash=False)
    a = half(box, x, "do", debug=False)
    b = half(box, x, "do", debug=False)
    assert np.abs(a["F"] - b["F"]).max() <= 1e-6 * np.abs(a["F"]).max()
    assert a["U"] == b["U"] and (a["W"] == b["W"]).all()
    for det in (1, 0):
        g = run_gpu(box, x, "do", "fp32", debug=False, options={DET_OPT: det})
        compare(g, r, "fp32", check_pairs=False, label=f"auto/det{det}")
        tm = g["stats"]["tune_ms"]
        if det:
            assert tm[4] == -1.0 and g["stats"]["sweep"] != HALF
        else:
            assert tm[4] > 0.0
    # the half list refuses the precisions it does not implement
    h = Handle(0)
    h.set_potential(box.pot)
    h.set_option(SWEEP_OPT, HALF)
    h.set_lattice(box.L0, box.A, box.t, box.automorphisms)
    xt = torch.from_numpy(x).to("cuda:0")
    h.build_cells("do", xt, "fp64")
    from paper_1412_3784_amd import NclError
    with pytest.raises(NclError):
        h.compute_forces()
    h.close()
