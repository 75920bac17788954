"""Pins of the oracle's planar-shear (Lees-Edwards) remapping, Sec. 2.2:
A = eps e_x e_y^T, L0 = a I, L_t = (I + tA) L0, reset by the automorphism
M = [[1,-1,0],[0,1,0],[0,0,1]] whenever the box has been sheared by half a
lattice spacing.

* at t* = 1/eps the sheared box is the undeformed lattice again, and the
  reset basis equals L0;
* the deformation angle stays within 90 - atan(2) degrees (printed value
  26.57) and reaches it just before each reset;
* the pair set and forces do not depend on which basis of the lattice is
  used (SL(3;Z) invariance), also in a rotated frame."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))


def golden(key):
    for line in open(os.path.join(HERE, "golden", "paper_values.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()[:2]
            if k == key:
                return float(v)
    raise KeyError(key)


def test_shear_flow_and_basis():
    box = wl.make_box("shear", 0.3, 10, side=4.0, t=0.0)
    assert box.A[0, 1] == 0.3 and np.count_nonzero(box.A) == 1
    assert (box.automorphisms[0] == wl.LE_M).all()
    L = oracle.lattice_at(box.L0, box.A, 1.7)
    assert np.allclose(L, [[4, 4 * 0.3 * 1.7, 0], [0, 4, 0], [0, 0, 4]], rtol=0, atol=1e-14)


def test_reset_at_full_spacing_restores_the_box():
    eps, a = 0.25, 3.0
    box = wl.make_box("shear", eps, 10, side=a, t=0.0)
    Lr, M, c = oracle.reduce(box.L0, box.A, 1.0 / eps, box.automorphisms)
    assert c[0] == 1
    assert (M == wl.LE_M).all()
    assert np.allclose(Lr, box.L0, rtol=0, atol=1e-13)


def test_maximum_angle_is_the_printed_value():
    eps = 0.4
    box = wl.make_box("shear", eps, 10, side=2.5, t=0.0)
    angles, coefs = [], []
    for t in np.linspace(0.0, 6.0 / eps, 6001):
        Lr, M, c = oracle.reduce(box.L0, box.A, t, box.automorphisms)
        assert round(np.linalg.det(M.astype(float))) == 1
        Lt = oracle.lattice_at(box.L0, box.A, t)
        assert np.allclose(Lr, Lt @ M, rtol=0, atol=1e-12 * np.abs(Lt).max())
        # angle between the sheared basis vector and the y axis
        angles.append(math.degrees(math.atan2(abs(Lr[0, 1]), Lr[1, 1])))
        coefs.append(c[0])
    assert max(angles) == pytest.approx(golden("shear_max_angle_deg"), abs=0.01)
    assert max(angles) <= 90.0 - math.degrees(math.atan(2.0)) + 1e-9
    assert sorted(set(coefs)) == list(range(0, 7))


@pytest.mark.parametrize("rotated", [False, True])
def test_pair_set_is_basis_independent(orc, rotated):
    eps = 0.6
    box = wl.make_box("shear", eps, 160, side=4.2, pot=wl.WCA, t=0.0, seed=5)
    L0, A, auts = box.L0, box.A, box.automorphisms
    if rotated:
        R = wl.random_rotation(9)
        L0, A = R @ L0, R @ A @ R.T
    for t in (0.3, 0.8 / eps, 1.4 / eps, 2.5 / eps):
        Lt = oracle.lattice_at(L0, A, t)
        x = box.frac @ Lt.T
        Lr, M, c = oracle.reduce(L0, A, t, auts)
        if rotated:
            assert c[0] == int(math.floor(eps * t + 0.5))
        a = oracle.forces_brute(x, Lt, box.pot)
        b = oracle.forces_brute(x, Lr, box.pot, Mkey=M)
        assert (a.count == b.count).all() and (a.hash == b.hash).all()
        assert np.allclose(a.F, b.F, rtol=0, atol=1e-9 * np.abs(a.F).max())
        assert a.U == pytest.approx(b.U, rel=1e-12)
        # the cell list on the reset basis agrees with brute force
        cl = oracle.forces_cells(x, Lr, box.pot, Mkey=M)
        assert (cl.hash == b.hash).all()


def test_rejects_a_flow_that_is_not_a_shear_of_the_lattice():
    box = wl.make_box("shear", 0.5, 10, side=3.0, t=0.0)
    A = box.A.copy()
    A[1, 0] = 0.1  # no longer nilpotent along N
    with pytest.raises(ValueError):
        oracle.reduce(box.L0, A, 0.7, box.automorphisms)
