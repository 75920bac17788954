"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (per-particle sweep, FP32 offsets), on sampled outputs the
oracle computes one by one: per-particle pair digests (exact) and forces
(1e-5 of sum_j |f_ij|) for a seeded sample of particles, plus properties
that hold at any size (sum of forces, energy and virial where the oracle
can afford the whole box).

Sizes: 1,048,576 LJ particles across the remap of the uniaxial strain
sweep; 16,777,216 LJ particles on a jittered grid (biaxial, t = T/2, Kahan
sums); the 512-replica WCA batch (8.9 M particles, a sample of replicas);
SLLOD steps of the 64-replica LJ batch checked by shadow evaluation."""
import functools

import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import FORCE_FLOOR, TOL_F, TOL_U, oracle_positions

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_3784_amd  # noqa: F401  (fails loudly if the library is missing)


def sample_idx(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(k, n), replace=False))


def gpu_box(box, x, variant, precision, debug):
    import torch
    from paper_1412_3784_amd import Handle
    h = Handle(0)
    h.set_potential(box.pot)
    h.set_lattice(box.L0, box.A, box.t, box.automorphisms)
    xt = torch.from_numpy(x).to("cuda:0")
    h.build_cells(variant, xt, precision, debug=debug)
    F, U, W = h.compute_forces()
    out = {"F": F.cpu().numpy().astype(np.float64), "U": float(U.cpu()[0]), "W": W.cpu().numpy().reshape(3, 3)}
    if debug:
        c, hs = h.debug_pairs()
        out["count"] = c.cpu().numpy()
        out["hash"] = hs.cpu().numpy().view(np.uint64)
    out["stats"] = h.stats()
    h.close()
    del xt
    torch.cuda.empty_cache()
    return out


def check_sample(g, ref, idx, precision, label):
    """per-particle parity on the sampled particles; returns (max, rms) of
    the force error relative to max(sum_j |f_ij|, eps/sigma)"""
    assert (g["count"][idx] == ref.count).all(), f"{label}: pair counts differ"
    bad = np.nonzero(g["hash"][idx] != ref.hash)[0]
    assert len(bad) == 0, f"{label}: pair sets differ at {idx[bad[:10]]}"
    dF = np.linalg.norm(g["F"][idx] - ref.F, axis=1)
    cond = dF / np.maximum(ref.fmag, FORCE_FLOOR)
    worst = int(np.argmax(cond))
    assert cond.max() <= TOL_F[precision], f"{label}: particle {idx[worst]} force error {cond[worst]:.3e}"
    l2 = np.linalg.norm(g["F"][idx] - ref.F) / np.linalg.norm(ref.F)
    assert l2 <= TOL_F[precision], f"{label}: relative L2 force error {l2:.3e}"
    return float(cond.max()), float(np.sqrt(np.mean(cond ** 2)))


@pytest.mark.parametrize("k", [0, 31, 33, 63])
@pytest.mark.parametrize("variant", ["do", "ds"])
def test_lj_1m_strain_sweep(k, variant):
    """1,048,576 LJ particles, uniaxial strain t_k = k T / 64 (the remap lies
    between k = 31 and 33); whole-box energy and virial against the oracle."""
    box = wl.lj_uniaxial_strain(k=k)
    x = oracle_positions(box)
    g = gpu_box(box, x, variant, "fp32", debug=True)
    Lr, Mt, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    idx = sample_idx(len(x), 4096, 17 + k)
    ref = oracle.forces_cells(x, Lr, box.pot, Mkey=Mt, subset=idx)
    mx, rms = check_sample(g, ref, idx, "fp32", f"lj1M/k{k}/{variant}")
    full = oracle.forces_cells(x, Lr, box.pot, Mkey=Mt, want_hash=False)
    assert abs(g["U"] - full.U) <= TOL_U["fp32"] * np.abs(full.u).sum()
    assert np.abs(g["W"] - full.W).max() <= TOL_F["fp32"] * full.fmag.sum()
    assert g["stats"]["pairs"] == full.stats[1]
    print(f"lj1M k={k} {variant}: max {mx:.2e} rms {rms:.2e}")


def test_lj_4m_ten_bit_radix():
    """4,194,304 LJ particles, uniaxial strain t = 40 T / 64, dynamic offset:
    326,040 cells, so the cell keys have 19 bits and the build sorts them in
    two passes of 10-bit digits (the other workloads use 7-, 8- and 9-bit
    digits).  Sampled pair sets and forces against the oracle; every particle
    has a pair count (the permutation misses none)."""
    box = wl.lj_uniaxial_strain(k=40, n=1 << 22)
    x = oracle_positions(box)
    g = gpu_box(box, x, "do", "fp32", debug=True)
    assert (1 << 18) < g["stats"]["ncells"] <= (1 << 20), g["stats"]["ncells"]
    Lr, Mt, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    idx = sample_idx(len(x), 4096, 41)
    ref = oracle.forces_cells(x, Lr, box.pot, Mkey=Mt, subset=idx)
    mx, rms = check_sample(g, ref, idx, "fp32", "lj4M/do")
    assert g["count"].sum() == g["stats"]["pairs"] and g["count"].min() > 0
    print(f"lj4M do: max {mx:.2e} rms {rms:.2e}")


@functools.lru_cache(maxsize=1)
def lj16m_whole_box():
    """the oracle's energy, virial and pair count of the whole 16M box (one
    FP64 evaluation on all host threads, shared by both variants)"""
    box = wl.lj_biaxial_grid()
    x = oracle_positions(box)
    Lr, Mt, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    full = oracle.forces_cells(x, Lr, box.pot, Mkey=Mt, want_hash=False)
    return full.U, full.W.copy(), float(np.abs(full.u).sum()), float(full.fmag.sum()), int(full.stats[1])


@pytest.mark.parametrize("variant", ["do", "ds"])
def test_lj_16m_grid_kahan(variant):
    """16,777,216 LJ particles (grid + jitter, biaxial, t = T/2), FP32 offsets
    with Kahan sums: sampled parity; whole-box energy (1e-7 of sum |u_i|; no
    close pairs here, so every pair takes the FP32 path) and virial against
    the oracle; total force ~ 0 (Newton's third law holds pair by pair in
    exact arithmetic)."""
    box = wl.lj_biaxial_grid()
    x = oracle_positions(box)
    g = gpu_box(box, x, variant, "fp32k", debug=True)
    Lr, Mt, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    idx = sample_idx(len(x), 8192, 23)
    ref = oracle.forces_cells(x, Lr, box.pot, Mkey=Mt, subset=idx)
    mx, rms = check_sample(g, ref, idx, "fp32k", f"lj16M/{variant}")
    Fsum = g["F"].sum(axis=0)
    assert np.abs(Fsum).max() <= 1e-5 * np.abs(g["F"]).sum(axis=0).max()
    assert g["stats"]["pairs"] > 0 and g["stats"]["max_occupancy"] > 0
    U, W, usum, fsum, npairs = lj16m_whole_box()
    assert g["stats"]["pairs"] == npairs
    assert g["stats"]["fp64_pairs"] < 1e-4 * npairs  # the FP32 path carries the energy
    relU = abs(g["U"] - U) / usum
    assert relU <= TOL_U["fp32k"], f"lj16M/{variant}: energy error {relU:.3e}"
    assert np.abs(g["W"] - W).max() <= TOL_F["fp32k"] * fsum
    print(f"lj16M {variant}: max {mx:.2e} rms {rms:.2e}, |sum F| {np.abs(Fsum).max():.3e}, rel U {relU:.2e}")


def test_wca_512_replica_batch():
    """The whole 512-replica batch in one launch; 16 replicas checked in full
    against the oracle (forces, digests, U, W)."""
    import torch
    from paper_1412_3784_amd import Batch
    boxes = wl.wca_replica_batch()
    xs = [oracle_positions(b) for b in boxes]
    bt = Batch([len(v) for v in xs])
    bt.set_potential(boxes[0].pot)
    bt.set_lattices("do", [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    x = torch.from_numpy(np.concatenate(xs)).to("cuda:0")
    bt.build_cells(x, "fp32", debug=True)
    F, U, W = bt.compute_forces()
    c, hs = bt.debug_pairs()
    torch.cuda.synchronize()
    F, U, W = F.cpu().numpy().astype(np.float64), U.cpu().numpy(), W.cpu().numpy().reshape(-1, 3, 3)
    c, hs = c.cpu().numpy(), hs.cpu().numpy().view(np.uint64)
    bt.stats()
    bt.close()
    off = np.concatenate([[0], np.cumsum([len(v) for v in xs])])
    for r in sample_idx(len(boxes), 16, 29):
        b = boxes[r]
        Lr, Mt, _ = oracle.reduce(b.L0, b.A, b.t, b.automorphisms)
        ref = oracle.forces_cells(xs[r], Lr, b.pot, Mkey=Mt)
        sl = slice(off[r], off[r + 1])
        g = {"F": F[sl], "count": c[sl], "hash": hs[sl]}
        check_sample(g, ref, np.arange(len(xs[r])), "fp32", f"batch512/rep{r}")
        assert abs(U[r] - ref.U) <= TOL_U["fp32"] * np.abs(ref.u).sum()
        assert np.abs(W[r] - ref.W).max() <= TOL_F["fp32"] * ref.fmag.sum()


def test_lj_64_replica_sllod_shadow():
    """100 graph-replayed SLLOD steps of the 64-replica LJ batch (53 M
    particles, config 5 at a tenth of its length).  The oracle evaluates
    forces on the GPU's own FP64 states (shadow evaluation) for the four
    smallest replicas: forces per particle, and the pressure tensor
    P = (sum p p^T / m + W) / V.  The smallest replica also runs the oracle's
    own FP64 trajectory: positions and momenta pointwise, the time-averaged
    diagonal pressure, and the energy balance, which the FP64 integrator
    itself holds only to O(h^2)."""
    import torch
    from paper_1412_3784_amd import Batch
    boxes = wl.lj_sllod_batch()
    ns = [len(b.frac) for b in boxes]
    xs = [b.positions(oracle.lattice_at(b.L0, b.A, b.t)) for b in boxes]
    ps = [wl.maxwell_momenta(n, 1.0, seed=5000 + r) for r, n in enumerate(ns)]
    bt = Batch(ns)
    bt.set_potential(boxes[0].pot)
    bt.set_lattices("do", [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    x = torch.from_numpy(np.concatenate(xs)).to("cuda:0")
    p = torch.from_numpy(np.concatenate(ps)).to("cuda:0")
    bt.build_cells(x, "fp32")
    h, nsteps = 0.002, 100
    F, U, W, hist = bt.sllod_run(x, p, h, 1.0, nsteps, use_graph=True, history=True)
    torch.cuda.synchronize()
    bt.stats()
    bt.close()
    off = np.concatenate([[0], np.cumsum(ns)])
    xg, pg, Fg = x.cpu().numpy(), p.cpu().numpy(), F.cpu().numpy().astype(np.float64)
    Wg = W.cpu().numpy().reshape(-1, 3, 3)
    hist = hist.cpu().numpy()                     # (nsteps + 1, R, 8)
    order = np.argsort(ns, kind="stable")
    for r in order[:4]:
        b = boxes[r]
        sl = slice(off[r], off[r + 1])
        t1 = b.t + nsteps * h
        Lr, _, _ = oracle.reduce(b.L0, b.A, t1, b.automorphisms)
        ref = oracle.forces_cells(xg[sl], Lr, b.pot, want_hash=False)
        dF = np.linalg.norm(Fg[sl] - ref.F, axis=1) / np.maximum(ref.fmag, FORCE_FLOOR)
        assert dF.max() <= TOL_F["fp32"], f"shadow rep {r}: {dF.max():.3e}"
        assert np.abs(Wg[r] - ref.W).max() <= TOL_F["fp32"] * ref.fmag.sum(), f"shadow rep {r}: virial"
        V = abs(np.linalg.det(Lr))
        K = pg[sl].T @ pg[sl]
        P_g, P_o = (K + Wg[r]) / V, (K + ref.W) / V
        relP = np.abs(P_g - P_o).max() / np.abs(P_o).max()
        assert relP <= 1e-6, f"shadow rep {r}: pressure tensor {relP:.3e}"
    r = order[0]
    b = boxes[r]
    sl = slice(off[r], off[r + 1])
    xo, po, ho = oracle.sllod(xs[r], ps[r], b.L0, b.A, b.t, b.automorphisms, b.pot, h, 1.0, nsteps)
    L = oracle.lattice_at(b.L0, b.A, b.t + nsteps * h)
    d = xg[sl] - xo
    d -= np.round(np.linalg.solve(L, d.T)).T @ L.T
    assert np.abs(d).max() < 1e-4, np.abs(d).max()
    assert np.abs(pg[sl] - po).max() < 1e-4 * np.abs(po).max()
    V = abs(np.linalg.det(b.L0))
    Pg = ((hist[:, r, 2:5] + hist[:, r, 5:8]) / V).mean(axis=0)
    Po = ((ho[:, 2:5] + ho[:, 5:8]) / V).mean(axis=0)
    assert np.abs(Pg - Po).max() <= 1e-6 * np.abs(Po).max(), (Pg, Po)
    # the energy balance: the GPU run drifts no more than the FP64
    # integrator does on the same start (its O(h^2) splitting error)
    eb_o = np.abs(oracle.energy_balance(ho, b.A)).max()
    eb_g = np.abs(oracle.energy_balance(hist[:, r], b.A)).max()
    assert eb_g <= 1.5 * eb_o, (eb_g, eb_o)
