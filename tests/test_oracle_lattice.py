"""Pins for the oracle's lattice functions (Sec. 2.1-2.2, 4.1, 4.2).

Each check compares the oracle with something other than itself: scipy's
expm, closed forms, integer lattice identities, cross-product heights and
numpy's QR.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore")


def test_expm_diagonal_closed_form(orc):
    A = np.diag([0.3, -0.1, -0.2])
    E = orc.expm(A, 1.7)
    assert np.allclose(E, np.diag(np.exp(1.7 * np.array([0.3, -0.1, -0.2]))), rtol=0, atol=1e-15)


def test_expm_general_matches_scipy(orc):
    g = np.random.default_rng(7)
    for _ in range(20):
        A = g.normal(size=(3, 3))
        t = g.uniform(0.1, 3.0)
        ref = scipy.linalg.expm(t * A)
        got = orc.expm(A, t)
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_expm_shear_is_affine(orc):
    # Sec. 2.2: under planar shear the basis grows linearly, L_t = (I + tA) L0
    A = np.zeros((3, 3))
    A[0, 1] = 0.37
    for t in (0.0, 0.5, 2.0, 10.0):
        E = orc.expm(A, t)
        assert np.allclose(E, np.eye(3) + t * A, rtol=0, atol=1e-13)


def test_kr_period_identity(orc):
    # eq:kr: exp(A t*) L0 = L0 M with M integral, unimodular, independent of the rate
    for rate in (0.1, 0.37, 1.0):
        box = wl.make_box("planar", rate, 64, side=7.0)
        T = math.log(wl.KR_LAMBDA) / rate
        lhs = orc.lattice_at(box.L0, box.A, T)
        rhs = box.L0 @ wl.KR_M
        assert np.allclose(lhs, rhs, rtol=0, atol=1e-12 * 7.0)
        Mt = np.linalg.solve(box.L0, lhs)
        assert np.allclose(Mt, np.round(Mt), atol=1e-10)
        assert round(np.linalg.det(np.round(Mt))) == 1


def test_gkr_automorphisms_commute_and_are_unimodular():
    M1 = wl.GKR_M1.astype(np.int64)
    M2 = wl.GKR_M2.astype(np.int64)
    assert (M1 @ M2 == M2 @ M1).all()
    assert round(np.linalg.det(M1)) == 1 and round(np.linalg.det(M2)) == 1
    w1 = np.linalg.eigvalsh(M1.astype(float))
    w2 = np.linalg.eigvalsh(M2.astype(float))
    # log-eigenvalue vectors (in the common eigenbasis) are independent and sum to 0
    V = np.linalg.eigh(M1.astype(float))[1]
    mu1 = np.log(np.diag(V.T @ M1 @ V))
    mu2 = np.log(np.diag(V.T @ M2 @ V))
    assert abs(mu1.sum()) < 1e-12 and abs(mu2.sum()) < 1e-12
    assert np.linalg.matrix_rank(np.stack([mu1, mu2]), tol=1e-6) == 2
    assert (w1 > 0).all() and (w2 > 0).all()


@pytest.mark.parametrize("flow", ["planar", "uniaxial", "biaxial"])
def test_reduced_basis_generates_same_lattice(orc, flow):
    # Sec. 2.2: L M generates the same lattice as L for M in SL(3;Z).  The
    # unreduced L_t is computed here with scipy, independently of the oracle.
    box = wl.make_box(flow, 0.5, 64, side=9.0)
    for t in np.linspace(0.0, 5.0 * box.period, 41):
        Lt = scipy.linalg.expm(t * box.A) @ box.L0
        Lred, Mtot, _ = orc.reduce(box.L0, box.A, t, box.automorphisms)
        K = np.linalg.solve(Lred, Lt)  # Lt = Lred K  =>  K integral unimodular
        assert np.allclose(K, np.round(K), atol=1e-7), (flow, t)
        K = np.round(K).astype(np.int64)
        assert round(np.linalg.det(K)) == 1
        # and Lred = Lt Mtot
        assert (K @ Mtot.astype(np.int64) == np.eye(3, dtype=np.int64)).all()


def test_kr_remap_count_closed_form(orc):
    # planar KR: the basis returns to L0 after each period, so the number of
    # remaps at time t is the nearest integer to t / T (ties aside)
    box = wl.make_box("planar", 0.2, 64, side=9.0)
    T = box.period
    for t in np.linspace(0.01, 7.3 * T, 57):
        _, _, (p, q) = orc.reduce(box.L0, box.A, t, box.automorphisms)
        assert p == int(math.floor(t / T + 0.5)) and q == 0


@pytest.mark.parametrize("flow", ["uniaxial", "biaxial", "planar"])
def test_stretch_stays_bounded(orc, flow):
    # generalised KR: the reduced basis is a bounded stretch of L0 for all time
    box = wl.make_box(flow, 1.0, 64, side=10.0)
    hmin = np.inf
    for t in np.linspace(0.0, 200.0, 2001):
        Lred, _, _ = orc.reduce(box.L0, box.A, t, box.automorphisms)
        S = Lred @ np.linalg.inv(box.L0)
        assert np.allclose(S, np.diag(np.diag(S)), atol=1e-9)
        eps = np.log(np.diag(S))
        assert abs(eps.sum()) < 1e-9
        assert np.abs(eps).max() < 2.5
        hmin = min(hmin, orc.heights(Lred).min())
    assert hmin > 0.1 * 10.0


def test_heights_cross_product(orc):
    # h_i = V / |v_j x v_k|: the distance between the faces spanned by v_j, v_k
    g = np.random.default_rng(3)
    for _ in range(30):
        L = g.normal(size=(3, 3)) + 3 * np.eye(3)
        V = abs(np.linalg.det(L))
        v = [L[:, 0], L[:, 1], L[:, 2]]
        ref = np.array([V / np.linalg.norm(np.cross(v[1], v[2])),
                        V / np.linalg.norm(np.cross(v[2], v[0])),
                        V / np.linalg.norm(np.cross(v[0], v[1]))])
        assert np.allclose(orc.heights(L), ref, rtol=1e-12)


def test_ds_counts_floor_of_heights(orc):
    L = np.diag([10.0, 20.0, 35.0])
    assert list(orc.ds_counts(L, 2.5)) == [4, 8, 14]
    box = wl.wca_planar_4096()
    # t = 0: a cube of side 16.929 with the WCA cut-off gives 15 cells per side
    assert list(orc.ds_counts(box.L0, wl.WCA_RC)) == [15, 15, 15]


def test_qr_matches_numpy(orc):
    g = np.random.default_rng(11)
    for _ in range(30):
        L = g.normal(size=(3, 3)) + 2 * np.eye(3)
        if np.linalg.det(L) < 0:
            L[:, 0] *= -1
        Q, R = orc.qr(L)
        Qn, Rn = np.linalg.qr(L)
        S = np.diag(np.sign(np.diag(Rn)))
        Qn, Rn = Qn @ S, S @ Rn
        assert np.allclose(R, Rn, atol=1e-12) and np.allclose(Q, Qn, atol=1e-12)
        assert np.allclose(np.tril(R, -1), 0) and (np.diag(R) > 0).all()
        assert np.allclose(Q @ R, L, atol=1e-12)
        assert abs(np.linalg.det(Q) - 1) < 1e-12


def test_reduce_rejects_bad_automorphisms(orc):
    box = wl.make_box("uniaxial", 0.5, 8, side=6.0)
    with pytest.raises(ValueError):
        orc.reduce(box.L0, box.A, 1.0, [2 * np.eye(3, dtype=np.int32)])  # det 8
    with pytest.raises(ValueError):
        orc.reduce(box.L0, box.A, 1.0, [wl.KR_M])  # not diagonalised by L0
    A = box.A.copy()
    A[0, 1] = 0.1
    with pytest.raises(ValueError):
        orc.reduce(box.L0, A, 1.0, box.automorphisms)  # flow not diagonal
