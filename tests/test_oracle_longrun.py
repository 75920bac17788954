"""The long-run neighbourhood volume experiment of Sec. 5.3, geometrically,
with the oracle: a box of initial side ~10 d_cut under uniaxial flow
diag(0.05, -0.025, -0.025), remapped by the generalised KR automorphisms,
d_cut = (3 / 4 pi)^(1/3) so that the cut-off sphere has volume one.

Search efficiency = sphere volume / neighbourhood volume averaged over the
run (Sec. 5: the efficiencies follow from the averaged volumes).  The
neighbourhood volume is 27 V / (c1 c2 c3) for the dynamic-size list
(Sec. 5.1) and avg(l2, l3) V / (l1 l2 l3) with the average cell count
27 + 14/l3 + 6/l2 - 4/(l2 l3) for the dynamic-offset list (Sec. 5.2)."""
import os

import numpy as np
import pytest

import oracle
import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
DCUT = (3.0 / (4.0 * np.pi)) ** (1.0 / 3.0)


def golden(key):
    for line in open(os.path.join(HERE, "golden", "paper_values.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()[:2]
            if k == key:
                return float(v)
    raise KeyError(key)


def long_run(side_cuts, periods=20, samples=10000):
    box = wl.make_box("uniaxial", 0.05, 10, side=side_cuts * DCUT, t=0.0)
    ts = np.linspace(0.0, periods * box.period, samples, endpoint=False)
    vds = np.empty(samples)
    vdo = np.empty(samples)
    for q, t in enumerate(ts):
        L, _, _ = oracle.reduce(box.L0, box.A, t, box.automorphisms)
        V = abs(np.linalg.det(L))
        c = oracle.ds_counts(L, DCUT)
        l = oracle.do_counts(L, DCUT)
        vds[q] = 27.0 * V / np.prod(c)
        avg = 27.0 + 14.0 / l[2] + 6.0 / l[1] - 4.0 / (l[1] * l[2])
        vdo[q] = avg * V / np.prod(l)
    return 1.0 / vds.mean(), 1.0 / vdo.mean(), box


def test_sphere_volume_is_one():
    assert abs(4.0 / 3.0 * np.pi * DCUT ** 3 - 1.0) < 1e-14


def test_long_run_efficiencies_match_the_paper():
    eff_ds, eff_do, box = long_run(10.0)
    assert box.A[0, 0] == pytest.approx(0.05) and box.A[1, 1] == pytest.approx(-0.025)
    assert eff_ds == pytest.approx(golden("ds_long_run_efficiency"), rel=0.015)
    assert eff_do == pytest.approx(golden("do_long_run_efficiency"), rel=0.02)
    # the dynamic-offset list is the more efficient one (Sec. 5.3)
    assert eff_do > 1.6 * eff_ds


def test_do_efficiency_tends_to_equilibrium_for_large_boxes():
    """As the box grows the average count tends to 27 and the efficiency to
    the equilibrium value (4/3) pi / 27 (Sec. 5.3)."""
    _, eff_small, _ = long_run(10.0, periods=4, samples=2000)
    _, eff_large, _ = long_run(200.0, periods=4, samples=2000)
    eq = golden("eq_search_efficiency")
    assert eff_small < eff_large < eq * 1.0001
    assert eff_large == pytest.approx(eq, rel=0.03)
