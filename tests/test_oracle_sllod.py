"""Pins of the oracle's SLLOD trajectory (peculiar momenta in the box that
follows the flow, Sec. 2.1-2.2) against facts that do not depend on it:

* one free particle follows the closed-form solution of dq/dt = p/m + A q,
  dp/dt = -A p, and the splitting converges to it at second order;
* the total momentum of an interacting system obeys sum p(t) = e^{-At} sum p(0)
  exactly (pair forces cancel in pairs);
* the symmetric splitting is time-reversible: reversing p and A retraces
  the trajectory;
* the energy balance H(t) - H(0) + int sum_a A_aa (K_aa + W_aa) dt = 0 holds
  to O(h^2);
* remapping the basis (Sec. 2.2) leaves the trajectory unchanged modulo the
  lattice.

A dropped or misplaced exponential, a wrong phi1, a sign error in the force or
the virial, or an asymmetric splitting fails at least one of these."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def lattice_diff(a, b, L):
    """a - b reduced by the lattice L (nearest image; L columns = basis)."""
    d = np.asarray(a) - np.asarray(b)
    n = np.round(np.linalg.solve(L, d.T)).T
    return d - n @ L.T


def wca_box(flow="planar", rate=0.5, grid=6, seed=11):
    return wl.make_box(flow, rate, grid ** 3, density=0.8442, pot=wl.WCA, t=0.0, seed=seed, grid=grid,
                       jitter_sigma=0.02)


@pytest.mark.parametrize("flow", ["planar", "uniaxial", "biaxial"])
def test_free_particle_closed_form(flow):
    box = wl.make_box(flow, 0.5, 1, side=10.0, pot=wl.WCA, t=0.0, seed=3)
    a = np.diag(box.A)
    q0 = np.array([[1.3, -0.7, 2.1]])
    p0 = np.array([[0.8, 1.1, -0.6]])
    m, T = 1.7, 0.8
    errs = []
    for h in (0.02, 0.01):
        ns = int(round(T / h))
        xf, pf, hist = oracle.sllod(q0, p0, box.L0, box.A, 0.0, box.automorphisms, box.pot, h, m, ns)
        # exact: p_a(t) = e^{-a t} p0,  q_a(t) = e^{a t} q0 + p0 sinh(a t) / (a m)
        pe = np.exp(-a * T) * p0
        qe = np.exp(a * T) * q0 + p0 * np.where(a != 0, np.sinh(a * T) / np.where(a != 0, a, 1), T) / m
        assert np.allclose(pf, pe, rtol=1e-13, atol=0)
        Lr, _, _ = oracle.reduce(box.L0, box.A, T, box.automorphisms)
        errs.append(np.abs(lattice_diff(xf, qe, Lr)).max())
        assert hist[:, 1].max() == 0.0 and np.abs(hist[:, 2:5]).max() == 0.0  # no pairs
    assert errs[0] > 1e-9
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


def test_total_momentum_follows_flow_exactly():
    box = wca_box("uniaxial", 0.7)
    x = box.positions(oracle.lattice_at(box.L0, box.A, 0.0))
    p = wl.maxwell_momenta(len(x), 1.0, seed=5) + np.array([0.3, -0.2, 0.1])
    P0 = p.sum(axis=0)
    xf, pf, hist = oracle.sllod(x, p, box.L0, box.A, 0.0, box.automorphisms, box.pot, 0.003, 1.0, 100)
    assert hist[:, 1].min() > 0  # interacting
    want = np.exp(-np.diag(box.A) * 0.3) * P0
    assert np.allclose(pf.sum(axis=0), want, rtol=0, atol=1e-11 * np.abs(p).sum())


@pytest.mark.parametrize("flow", ["planar", "biaxial"])
def test_time_reversible(flow):
    box = wca_box(flow, 0.6)
    x0 = box.positions(oracle.lattice_at(box.L0, box.A, 0.0))
    p0 = wl.maxwell_momenta(len(x0), 1.0, seed=6)
    h, ns = 0.002, 60
    xf, pf, _ = oracle.sllod(x0, p0, box.L0, box.A, 0.0, [], box.pot, h, 1.0, ns)
    # reversed run: A -> -A, starting from the lattice reached, p -> -p
    L1 = oracle.lattice_at(box.L0, box.A, ns * h)
    xb, pb, _ = oracle.sllod(xf, -pf, L1, -box.A, 0.0, [], box.pot, h, 1.0, ns)
    L0 = oracle.lattice_at(box.L0, box.A, 0.0)
    assert np.abs(lattice_diff(xb, x0, L0)).max() < 1e-9
    assert np.abs(pb + p0).max() < 1e-9 * np.abs(p0).max()


@pytest.mark.parametrize("flow", ["planar", "uniaxial"])
def test_energy_balance_second_order(flow):
    box = wca_box(flow, 0.5)
    x = box.positions(oracle.lattice_at(box.L0, box.A, 0.0))
    p = wl.maxwell_momenta(len(x), 1.0, seed=12)
    drift = []
    for h in (0.004, 0.002):
        ns = int(round(0.4 / h))
        _, _, hist = oracle.sllod(x, p, box.L0, box.A, 0.0, box.automorphisms, box.pot, h, 1.0, ns)
        eb = oracle.energy_balance(hist, box.A)
        H0 = 0.5 * hist[0, 5:8].sum() + hist[0, 1]
        work = np.abs(np.cumsum(np.diff(hist[:, 0]) * (np.diag(box.A) * (hist[1:, 5:8] + hist[1:, 2:5])).sum(1)))
        assert work.max() > 1.0  # the flow does real work on the system
        drift.append(np.abs(eb).max())
        assert drift[-1] < 2e-3 * H0
    assert 3.3 < drift[0] / drift[1] < 4.7, drift


def test_remap_leaves_trajectory_unchanged():
    # planar KR: the remap happens at t = T/2 (nearest multiple of the period)
    box = wl.make_box("planar", 0.5, 512, density=0.8442, pot=wl.WCA, t=0.0, seed=13, grid=8, jitter_sigma=0.02)
    T = box.period
    t0, h, ns = 0.5 * T - 0.05, 0.002, 50
    x = box.positions(oracle.lattice_at(box.L0, box.A, t0))
    p = wl.maxwell_momenta(len(x), 1.0, seed=14)
    xa, pa, ha = oracle.sllod(x, p, box.L0, box.A, t0, box.automorphisms, box.pot, h, 1.0, ns)
    xb, pb, hb = oracle.sllod(x, p, box.L0, box.A, t0, [], box.pot, h, 1.0, ns)
    _, _, ca = oracle.reduce(box.L0, box.A, t0 + ns * h, box.automorphisms)
    assert ca[0] != 0  # a remap took place
    L = oracle.lattice_at(box.L0, box.A, t0 + ns * h)
    assert np.abs(lattice_diff(xa, xb, L)).max() < 1e-9
    assert np.abs(pa - pb).max() < 1e-9
    assert np.allclose(ha[:, 1:5], hb[:, 1:5], rtol=1e-9, atol=1e-9)
