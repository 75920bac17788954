"""Pins for the oracle's pair set, forces, energy and virial.

The oracle's brute force is checked against a naive enumeration over a large
fixed image range written here; its cell list (Sec. 4.1) against the brute
force; forces against finite differences of its energy; the virial against
the strain derivative of the energy; and whole configurations against
closed-form symmetry results (Bravais lattices, two-particle geometry,
equilibrium search efficiency of Sec. 5).
"""
import math

import numpy as np
import pytest

import workloads as wl

WCA = wl.WCA
LJ = wl.LJ25


def naive_pairs(x, L, rc, K=3):
    """All (i, j, m) with i < j, or i == j and m > 0, |x_j + L m - x_i| < rc, m in [-K, K]^3."""
    out = []
    n = len(x)
    rng = range(-K, K + 1)
    for i in range(n):
        for j in range(i, n):
            for m0 in rng:
                for m1 in rng:
                    for m2 in rng:
                        m = (m0, m1, m2)
                        if i == j and not (m > (0, 0, 0)):
                            continue
                        d = x[j] - x[i] + L @ np.array(m, dtype=float)
                        if d @ d < rc * rc:
                            out.append((i, j, m0, m1, m2))
    return sorted(out)


def small_box(flow, n, side, pot, t_frac, seed):
    return wl.make_box(flow, 0.7, n, side=side, pot=pot, t_frac=t_frac, seed=seed)


@pytest.mark.parametrize("seed", range(4))
def test_brute_pairs_match_naive_enumeration(orc, seed):
    g = np.random.default_rng(100 + seed)
    # small, strongly skewed boxes where several images of one partner interact
    L = np.diag([2.4, 2.6, 2.9]) + g.uniform(-0.9, 0.9, size=(3, 3)) * (1 - np.eye(3))
    if np.linalg.det(L) < 0:
        L[:, 0] *= -1
    rc = 0.9 * orc.heights(L).min()
    x = g.uniform(-3, 3, size=(7, 3))
    got = sorted(map(tuple, orc.pairs_brute(x, L, rc).tolist()))
    assert got == naive_pairs(x, L, rc)


CASES = [(flow, side, tf, seed)
         for flow in ("planar", "uniaxial", "biaxial", "none")
         for side, tf in ((1.3, 0.3), (2.6, 0.5), (3.7, 0.85), (4.9, 1.45))
         for seed in (1, 2)]


@pytest.mark.parametrize("flow,side,tf,seed", CASES)
def test_cells_equal_brute(orc, flow, side, tf, seed):
    """Sec. 4.1 cell list == brute force on tiny boxes with 1..4 cells per side."""
    pot = WCA
    box = small_box(flow, 60, side * pot.rc * 1.0, pot, tf, seed)
    Lt = orc.lattice_at(box.L0, box.A, box.t)
    Lred, Mtot, _ = orc.reduce(box.L0, box.A, box.t, box.automorphisms)
    if orc.ds_counts(Lred, pot.rc).min() < 1:
        pytest.skip("box too small for this strain")
    x = box.positions(Lt)
    # evaluate in the reduced basis, key images in the unreduced one
    b = orc.forces_brute(x, Lred, pot, Mkey=Mtot)
    c = orc.forces_cells(x, Lred, pot, Mkey=Mtot)
    assert (b.count == c.count).all()
    assert (b.hash == c.hash).all()
    scale = np.abs(b.F).max() + 1.0
    assert np.abs(b.F - c.F).max() <= 1e-12 * scale
    assert abs(b.U - c.U) <= 1e-12 * (abs(b.U) + 1)
    assert np.abs(b.W - c.W).max() <= 1e-12 * (np.abs(b.W).max() + 1)


MEDIUM = [(flow, pot_name, tf) for flow in ("planar", "uniaxial", "biaxial", "shear", "none")
          for pot_name, tf in (("wca", 0.4), ("lj", 0.5))]


@pytest.mark.parametrize("flow,pot_name,tf", MEDIUM)
def test_cells_equal_brute_medium(orc, flow, pot_name, tf):
    """Sec. 4.1 cell list == brute force on medium boxes (at least 5 cells per
    side: 1,500 WCA or 6,000 LJ particles at liquid density), every flow:
    pair sets, forces, energy and virial."""
    if pot_name == "wca":
        pot, n, dens = WCA, 1500, 0.8442
    else:
        pot, n, dens = wl.LJ25, 6000, 0.8
    box = wl.make_box(flow, 0.5, n, density=dens, pot=pot, t_frac=tf, seed=211)
    Lt = orc.lattice_at(box.L0, box.A, box.t)
    Lred, Mtot, _ = orc.reduce(box.L0, box.A, box.t, box.automorphisms)
    assert orc.ds_counts(Lred, pot.rc).min() >= 5
    x = box.positions(Lt)
    b = orc.forces_brute(x, Lred, pot, Mkey=Mtot)
    c = orc.forces_cells(x, Lred, pot, Mkey=Mtot)
    assert b.count.sum() > 2 * n
    assert (b.count == c.count).all()
    assert (b.hash == c.hash).all()
    scale = np.abs(b.F).max() + 1.0
    assert np.abs(b.F - c.F).max() <= 1e-12 * scale
    assert abs(b.U - c.U) <= 1e-12 * (abs(b.U) + 1)
    assert np.abs(b.W - c.W).max() <= 1e-12 * (np.abs(b.W).max() + 1)


def jittered_lattice(n_side, L, sigma, seed):
    g = np.random.default_rng(seed)
    ax = (np.arange(n_side) + 0.5) / n_side
    s = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    return s @ L.T + g.normal(0, sigma, size=s.shape)


def test_newton_third_law(orc):
    box = wl.wca_planar_4096()
    Lred, _, _ = orc.reduce(box.L0, box.A, box.t, box.automorphisms)
    x = jittered_lattice(16, Lred, 0.05, 5)
    r = orc.forces_cells(x, Lred, WCA)
    assert np.abs(r.F.sum(0)).max() <= 1e-12 * np.abs(r.F).sum()


@pytest.mark.parametrize("pot", [WCA, LJ], ids=["wca", "lj"])
def test_force_is_minus_energy_gradient(orc, pot):
    box = wl.make_box("uniaxial", 0.5, 8, side=4 * pot.rc, pot=pot, t_frac=0.3, seed=9)
    Lred, _, _ = orc.reduce(box.L0, box.A, box.t, box.automorphisms)
    x = jittered_lattice(4, Lred, 0.08, 21)
    r = orc.forces_brute(x, Lred, pot)
    h = 1e-6
    g = np.random.default_rng(1)
    for i in g.choice(len(x), 6, replace=False):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            dU = (orc.forces_brute(xp, Lred, pot).U - orc.forces_brute(xm, Lred, pot).U) / (2 * h)
            assert abs(r.F[i, k] + dU) <= 2e-6 * (np.abs(r.F).max() + 1)


@pytest.mark.parametrize("pot", [WCA, LJ], ids=["wca", "lj"])
def test_virial_is_minus_strain_derivative(orc, pot):
    # W_ab = -dU/d(eps_ab) for the affine map x -> (I + eps) x, L -> (I + eps) L
    box = wl.make_box("biaxial", 0.5, 8, side=4 * pot.rc, pot=pot, t_frac=0.6, seed=4)
    Lred, _, _ = orc.reduce(box.L0, box.A, box.t, box.automorphisms)
    x = jittered_lattice(4, Lred, 0.08, 22)
    r = orc.forces_brute(x, Lred, pot)
    h = 1e-7
    for a in range(3):
        for b in range(3):
            E = np.zeros((3, 3))
            E[a, b] = h
            up = orc.forces_brute(x @ (np.eye(3) + E).T, (np.eye(3) + E) @ Lred, pot).U
            dn = orc.forces_brute(x @ (np.eye(3) - E).T, (np.eye(3) - E) @ Lred, pot).U
            assert abs(r.W[a, b] + (up - dn) / (2 * h)) <= 1e-5 * (np.abs(r.W).max() + 1)
    assert np.allclose(r.W, r.W.T, atol=1e-12 * np.abs(r.W).max())


def test_lj_special_distances(orc):
    # phi(sigma) = 0 before the shift; the LJ minimum at 2^(1/6) sigma has
    # phi = -eps and zero force.  Two particles in a big cube.
    L = np.eye(3) * 20.0
    shift = 4 * (2.5 ** -12 - 2.5 ** -6)
    r = orc.forces_brute(np.array([[1.0, 1, 1], [2.0, 1, 1]]), L, LJ)
    assert abs(r.U - (0.0 - shift)) < 1e-14
    r = orc.forces_brute(np.array([[1.0, 1, 1], [1.0, 1 + 2 ** (1 / 6), 1]]), L, LJ)
    assert abs(r.U - (-1.0 - shift)) < 1e-13 and np.abs(r.F).max() < 1e-12
    # WCA: zero energy and force at and beyond the cut-off, +eps at r = sigma
    r = orc.forces_brute(np.array([[1.0, 1, 1], [1.0, 1, 1 + 2 ** (1 / 6)]]), L, WCA)
    assert r.U == 0.0 and np.abs(r.F).max() == 0.0 and r.count.sum() == 0
    r = orc.forces_brute(np.array([[1.0, 1, 1], [1.0, 1, 2.0]]), L, WCA)
    assert abs(r.U - 1.0) < 1e-14


def test_two_particles_across_skewed_face(orc):
    # basis with a strong shear; the nearest image of particle 1 lies across
    # the v1-v2 face shifted by v3 - v1: m = (-1, 0, 1)
    v1, v2, v3 = np.array([5.0, 0, 0]), np.array([1.5, 5.0, 0]), np.array([3.2, 1.1, 5.0])
    L = np.stack([v1, v2, v3], 1)
    x0 = np.array([1.0, 2.0, 4.6])
    target = x0 + np.array([0.3, -0.4, 0.5])            # within WCA? |d| = 0.707 < 1.1225
    x1 = target - (-v1 + v3)                             # so x1 + L(-1,0,1) = target
    pairs = orc.pairs_brute(np.stack([x0, x1]), L, WCA.rc)
    assert pairs.tolist() == [[0, 1, -1, 0, 1]]
    r = orc.forces_brute(np.stack([x0, x1]), L, WCA)
    d = np.array([0.3, -0.4, 0.5])
    # force on 0 points away from the partner image (repulsive), equal and opposite
    assert np.dot(r.F[0], d) < 0 and np.allclose(np.cross(r.F[0], d), 0, atol=1e-9 * np.abs(r.F).max())
    assert np.allclose(r.F[0], -r.F[1])


@pytest.mark.parametrize("flow", ["uniaxial", "planar"])
def test_bravais_lattice_forces_vanish(orc, flow):
    # particles on the sites of a sub-lattice L diag(1/n) Z^3: every force
    # vanishes by inversion symmetry, every particle has the same energy,
    # half the lattice sum of phi over sub-lattice vectors within r_c.
    pot = LJ
    box = wl.make_box(flow, 0.4, 8, side=3.2 * pot.rc, pot=pot, t_frac=0.37, seed=0)
    Lred, _, _ = orc.reduce(box.L0, box.A, box.t, box.automorphisms)
    n = 3
    ax = np.arange(n) / n
    s = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    x = s @ Lred.T
    r = orc.forces_cells(x, Lred, pot)
    fscale = np.abs(orc.forces_cells(x + np.random.default_rng(0).normal(0, .02, x.shape), Lred, pot).F).max()
    assert np.abs(r.F).max() <= 1e-10 * fscale
    assert np.allclose(r.u, r.u[0], rtol=1e-12)
    B = Lred / n
    K = 8
    k = np.arange(-K, K + 1)
    ks = np.stack(np.meshgrid(k, k, k, indexing="ij"), -1).reshape(-1, 3)
    v = ks @ B.T
    rr = np.sqrt((v * v).sum(1))
    rr = rr[(rr > 0) & (rr < pot.rc)]
    assert B.T.shape == (3, 3) and np.linalg.norm(B, axis=0).max() * 1.0 < K * orc.heights(B).min()
    shift = 4 * ((1 / pot.rc) ** 12 - (1 / pot.rc) ** 6)
    phi = 4 * (rr ** -12 - rr ** -6) - shift
    assert abs(r.u[0] - 0.5 * phi.sum()) <= 1e-11 * np.abs(phi).sum()
    assert r.count[0] == len(rr)


def test_invariance_under_unimodular_basis_change(orc):
    # Sec. 2.2: L and L M generate the same lattice, so the interacting set
    # (labelled by images in the L frame) and every force are unchanged.
    box = wl.make_box("biaxial", 0.3, 300, side=5.3 * LJ.rc, pot=LJ, t_frac=0.4, seed=3)
    Lred, _, _ = orc.reduce(box.L0, box.A, box.t, box.automorphisms)
    x = box.positions(Lred)
    ref = orc.forces_brute(x, Lred, LJ)
    for seed in range(4):
        M = wl.random_unimodular(seed, steps=3)
        r = orc.forces_brute(x, Lred @ M, LJ, Mkey=M)   # image m' in L M  ->  M m' in L
        assert (r.count == ref.count).all() and (r.hash == ref.hash).all()
        assert np.allclose(r.F, ref.F, rtol=0, atol=1e-9 * np.abs(ref.F).max())
        assert abs(r.U - ref.U) <= 1e-11 * abs(ref.U)


def test_invariance_rotation_translation_reimaging(orc):
    box = wl.make_box("uniaxial", 0.3, 300, side=5.1 * LJ.rc, pot=LJ, t_frac=0.2, seed=8)
    Lred, _, _ = orc.reduce(box.L0, box.A, box.t, box.automorphisms)
    x = box.positions(Lred)
    ref = orc.forces_cells(x, Lred, LJ)
    fs = np.abs(ref.F).max()
    Q = wl.random_rotation(5)
    r = orc.forces_cells(x @ Q.T, Q @ Lred, LJ)
    assert (r.count == ref.count).all() and (r.hash == ref.hash).all()
    assert np.allclose(r.F, ref.F @ Q.T, atol=1e-9 * fs)
    assert np.allclose(r.W, Q @ ref.W @ Q.T, atol=1e-9 * np.abs(ref.W).max())
    r = orc.forces_cells(x + np.array([3.3, -7.1, 0.4]), Lred, LJ)
    assert (r.count == ref.count).all() and np.allclose(r.F, ref.F, atol=1e-9 * fs)
    n = np.random.default_rng(2).integers(-3, 4, size=(len(x), 3))
    r = orc.forces_cells(x + n @ Lred.T, Lred, LJ)
    assert (r.count == ref.count).all() and np.allclose(r.F, ref.F, atol=1e-9 * fs)
    assert abs(r.U - ref.U) <= 1e-10 * abs(ref.U)


def read_golden():
    import os
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()[:2]
                out[k] = float(v)
    return out


def test_equilibrium_search_efficiency(orc):
    # Sec. 5: with A = 0 and a box side divisible by d_cut the neighbourhood is
    # a cube of side 3 d_cut, so in-range / candidates -> (4/3) pi / 27
    gold = read_golden()["eq_search_efficiency"]
    rc = 1.0
    side = 12 * rc * (1 + 1e-12)
    n = 40000
    g = np.random.default_rng(17)
    x = g.uniform(0, side, size=(n, 3))
    pot = wl.Potential(rc=rc)
    r = orc.forces_cells(x, np.eye(3) * side, pot, want_hash=False)
    cand, inr = r.stats
    eff = inr / cand
    assert abs(eff - (4 / 3) * math.pi / 27) < 0.002
    assert abs(eff - gold) < 0.002
    # O(N): candidates per particle do not grow with N at fixed density (Sec. 3)
    n2 = n // 8
    x2 = g.uniform(0, side / 2, size=(n2, 3))
    r2 = orc.forces_cells(x2, np.eye(3) * side / 2, pot, want_hash=False)
    assert abs(r2.stats[0] / n2 - cand / n) < 0.03 * cand / n
