"""SLLOD of batches with neighbour lists reused between rebuilds (skin > 0):
trajectories against the FP64 oracle (including a replica that crosses a KR
remap during the run, which forces a rebuild), the final forces, energy,
virial and exact pair count against the oracle evaluated on the GPU's final
positions, rebuilds triggered by displacement with a thin skin, the list
capacity error and the state it leaves, and option errors."""
import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import FORCE_FLOOR, TOL_F, oracle_positions

pytestmark = pytest.mark.gpu

SKIN = 5  # NCL_OPT_SKIN


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_3784_amd  # noqa: F401  (fails loudly if the library is missing)


def nemd_batch(t0s=None, seed0=7100, pot=wl.WCA, density=0.8442, grids=(12, 14, 11, 13)):
    flows = ("planar", "uniaxial", "biaxial", "uniaxial")
    rates = (0.5, 0.3, 0.4, 0.1)
    boxes = []
    for r, (g, fl, ra) in enumerate(zip(grids, flows, rates)):
        b = wl.make_box(fl, ra, g ** 3, density=density, pot=pot, t=0.0, seed=seed0 + r, grid=g,
                        jitter_sigma=0.02, name=f"vl{r}")
        if t0s is not None:
            b.t = t0s[r]
        boxes.append(b)
    return boxes


def start_state(boxes):
    xs = [oracle_positions(b) for b in boxes]
    ps = [wl.maxwell_momenta(len(x), 1.0, seed=900 + r) for r, x in enumerate(xs)]
    return xs, ps


def lattice_diff(a, b, L):
    d = np.asarray(a) - np.asarray(b)
    n = np.round(np.linalg.solve(L, d.T)).T
    return d - n @ L.T


def sllod_lists(boxes, xs, ps, h, nsteps, precision, skin, variant="do"):
    import torch
    from paper_1412_3784_amd import Batch
    bt = Batch([len(x) for x in xs])
    bt.set_potential(boxes[0].pot)
    bt.set_option(SKIN, skin)
    bt.set_lattices(variant, [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    x = torch.from_numpy(np.concatenate(xs)).to("cuda:0")
    p = torch.from_numpy(np.concatenate(ps)).to("cuda:0")
    bt.build_cells(x, precision)
    F, U, W, hist = bt.sllod_run(x, p, h, 1.0, nsteps, use_graph=False, history=True)
    torch.cuda.synchronize()
    out = {"x": x.cpu().numpy(), "p": p.cpu().numpy(), "F": F.cpu().numpy().astype(np.float64),
           "U": U.cpu().numpy(), "W": W.cpu().numpy().reshape(-1, 3, 3), "hist": hist.cpu().numpy(),
           "stats": bt.stats(), "Lred": bt.lattices()[0]}
    bt.close()
    return out


@pytest.mark.parametrize("variant", ["do", "ds"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 2e-6)])
def test_lists_match_oracle_trajectory(precision, tol, variant):
    """40 steps with a 0.3 sigma skin against the oracle's FP64 trajectory; the
    first replica crosses a KR remap, which must force a rebuild."""
    T0 = wl.make_box("planar", 0.5, 125, side=6.0).period
    boxes = nemd_batch(t0s=(0.5 * T0 - 0.04, 0.0, 0.1, 0.0))
    xs, ps = start_state(boxes)
    h, ns = 0.002, 40
    g = sllod_lists(boxes, xs, ps, h, ns, precision, 0.3, variant)
    cut = np.cumsum([0] + [len(x) for x in xs])
    for r, b in enumerate(boxes):
        xo, po, ho = oracle.sllod(xs[r], ps[r], b.L0, b.A, b.t, b.automorphisms, b.pot, h, 1.0, ns)
        L = oracle.lattice_at(b.L0, b.A, b.t + ns * h)
        dx = np.abs(lattice_diff(g["x"][cut[r]:cut[r + 1]], xo, L)).max()
        dp = np.abs(g["p"][cut[r]:cut[r + 1]] - po).max() / np.abs(po).max()
        assert dx < tol * np.abs(L).max(), f"rep {r}: position error {dx:.3e}"
        assert dp < 10 * tol, f"rep {r}: momentum error {dp:.3e}"
        hg = g["hist"][:, r, :]
        scale = np.abs(ho[:, 1:]).max(axis=0)
        err = (np.abs(hg[:, 1:] - ho[:, 1:]) / scale).max()
        assert err < 10 * tol, f"rep {r}: observable error {err:.3e}"
    _, _, ca = oracle.reduce(boxes[0].L0, boxes[0].A, boxes[0].t + ns * h, boxes[0].automorphisms)
    _, _, cb = oracle.reduce(boxes[0].L0, boxes[0].A, boxes[0].t, boxes[0].automorphisms)
    assert tuple(ca) != tuple(cb)  # the remap was crossed
    # the initial build, the remap, and a few rebuilds for displacement
    assert 2 <= g["stats"]["list_rebuilds"] <= 12, g["stats"]["list_rebuilds"]
    # positions are back in the reduced box at the end
    for r in range(len(boxes)):
        s = np.linalg.solve(g["Lred"][r], g["x"][cut[r]:cut[r + 1]].T)
        assert s.min() >= -1e-12 and s.max() < 1.0 + 1e-12


@pytest.mark.parametrize("variant", ["do", "ds"])
def test_lists_thin_skin_final_forces(variant):
    """LJ replicas, 120 steps with a 0.06 sigma skin (rebuilds forced by
    displacement); the forces, energy, virial and pair count of the last step
    equal the oracle's on the GPU's own final positions and lattices."""
    boxes = nemd_batch(pot=wl.LJ25, density=0.8, grids=(11, 12, 10, 13), seed0=7300)
    xs, ps = start_state(boxes)
    h, ns = 0.002, 120
    g = sllod_lists(boxes, xs, ps, h, ns, "fp32", 0.06, variant)
    assert 6 <= g["stats"]["list_rebuilds"] < ns
    cut = np.cumsum([0] + [len(x) for x in xs])
    pairs = 0
    for r, b in enumerate(boxes):
        Lr = g["Lred"][r]
        ref = oracle.forces_cells(g["x"][cut[r]:cut[r + 1]], Lr, b.pot, want_hash=False)
        F = g["F"][cut[r]:cut[r + 1]]
        cond = np.linalg.norm(F - ref.F, axis=1) / np.maximum(ref.fmag, FORCE_FLOOR)
        assert cond.max() <= TOL_F["fp32"], f"rep {r}: force error {cond.max():.3e}"
        assert abs(g["U"][r] - ref.U) <= 1e-7 * np.abs(ref.u).sum()
        assert np.abs(g["W"][r] - ref.W).max() <= 1e-5 * ref.fmag.sum()
        pairs += ref.stats[1]
    assert g["stats"]["pairs"] == pairs


def test_lists_capacity_error_and_options():
    """A replica with a dense cluster exceeds the list capacity sized from
    the mean density: NCL_E_CAPACITY, no fault; option misuse is refused."""
    import torch
    from paper_1412_3784_amd import Batch, NclError
    from paper_1412_3784_amd import nemdcl as n
    boxes = nemd_batch(pot=wl.LJ25, density=0.8, grids=(10, 10, 10, 10), seed0=7500)
    xs, ps = start_state(boxes)
    # a quarter of replica 1's particles packed into a ball of radius 2 sigma
    rng = np.random.default_rng(3)
    k = len(xs[1]) // 4
    c = oracle.lattice_at(boxes[1].L0, boxes[1].A, boxes[1].t) @ np.full(3, 0.5)
    v = rng.normal(size=(k, 3))
    xs[1][:k] = c + 2.0 * v / np.linalg.norm(v, axis=1)[:, None] * rng.random((k, 1)) ** (1 / 3)
    bt = Batch([len(x) for x in xs])
    bt.set_potential(boxes[0].pot)
    with pytest.raises(NclError) as e:
        bt.set_option(SKIN, -0.1)
    assert e.value.code == n.NCL_E_ARG
    bt.set_option(SKIN, 0.3)
    bt.set_lattices("do", [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    with pytest.raises(NclError) as e:
        bt.set_option(SKIN, 0.2)
    assert e.value.code == n.NCL_E_STATE
    x = torch.from_numpy(np.concatenate(xs)).to("cuda:0")
    p = torch.from_numpy(np.concatenate(ps)).to("cuda:0")
    bt.build_cells(x, "fp32")
    with pytest.raises(NclError) as e:
        bt.sllod_run(x, p, 0.0005, 1.0, 2, use_graph=False, history=False)
    assert e.value.code == n.NCL_E_CAPACITY
    # after a failed run the batch holds no lattice or cells that could be
    # paired with positions of an unknown step: it refuses until the
    # lattices are set again, and then works
    with pytest.raises(NclError) as e:
        bt.compute_forces()
    assert e.value.code == n.NCL_E_STATE
    with pytest.raises(NclError) as e:
        bt.build_cells(x, "fp32")
    assert e.value.code == n.NCL_E_STATE
    bt.set_lattices("do", [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    bt.build_cells(x, "fp32")
    F, U, W = bt.compute_forces()
    torch.cuda.synchronize()
    assert np.isfinite(U.cpu().numpy()).all()
    bt.close()
