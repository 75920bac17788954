"""GPU parity of the batched form: many independent boxes of uneven size,
each with its own flow, rate and strain time, binned and swept together.
Every replica is checked against the FP64 oracle on its own positions, to the
same bar as the single-box path (exact pair sets, forces within 1e-5 of
sum_j |f_ij|, energy 1e-7).  SLLOD runs of a batch (peculiar momenta, the box
following the flow, Sec. 2.1-2.2) are checked against the oracle's FP64
trajectory, and captured-graph replay against eager stepping, bit for bit."""
import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import compare, oracle_positions, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_3784_amd  # noqa: F401  (fails loudly if the library is missing)


def fits(box, variant):
    Lr, _, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    c = oracle.ds_counts(Lr, box.pot.rc) if variant == "ds" else oracle.do_counts(Lr, box.pot.rc)
    return c.min() >= 1


def small_batch(replicas=24, n_lo=300, n_hi=5000, variant="do"):
    boxes = [b for b in wl.wca_replica_batch(replicas=replicas, n_lo=n_lo, n_hi=n_hi) if fits(b, variant)]
    assert len(boxes) >= replicas // 2
    return boxes


def run_batch(boxes, variant, precision, debug=True, options=None):
    import torch
    from paper_1412_3784_amd import Batch
    xs = [oracle_positions(b) for b in boxes]
    bt = Batch([len(x) for x in xs])
    bt.set_potential(boxes[0].pot)
    for k, v in (options or {}).items():
        bt.set_option(k, v)
    bt.set_lattices(variant, [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    xt = torch.from_numpy(np.concatenate(xs)).to("cuda:0")
    bt.build_cells(xt, precision, debug=debug)
    F, U, W = bt.compute_forces()
    out = {"x": xs}
    if debug:
        c, hs = bt.debug_pairs()
        out["count"] = c.cpu().numpy()
        out["hash"] = hs.cpu().numpy().view(np.uint64)
    torch.cuda.synchronize()
    out["F"] = F.cpu().numpy().astype(np.float64)
    out["U"] = U.cpu().numpy()
    out["W"] = W.cpu().numpy().reshape(-1, 3, 3)
    out["stats"] = bt.stats()
    out["lattices"] = bt.lattices()
    bt.close()
    return out


def check_replicas(boxes, g, precision, label):
    off = 0
    tot_pairs = 0
    for r, b in enumerate(boxes):
        n = len(g["x"][r])
        ref = run_oracle(b, g["x"][r])
        gr = {"F": g["F"][off:off + n], "U": float(g["U"][r]), "W": g["W"][r]}
        if "count" in g:
            gr["count"] = g["count"][off:off + n]
            gr["hash"] = g["hash"][off:off + n]
        compare(gr, ref, precision, check_pairs="count" in g, label=f"{label}/rep{r}({b.name}, n={n})")
        Lr, _, _ = oracle.reduce(b.L0, b.A, b.t, b.automorphisms)
        assert np.allclose(g["lattices"][0][r], Lr, rtol=0, atol=1e-12 * np.abs(Lr).max())
        tot_pairs += int(ref.count.sum())
        off += n
    assert g["stats"]["pairs"] == tot_pairs


@pytest.mark.parametrize("variant", ["ds", "do"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32k"])
def test_batch_matches_oracle_per_replica(variant, precision):
    boxes = small_batch(variant=variant)
    g = run_batch(boxes, variant, precision)
    check_replicas(boxes, g, precision, f"batch/{variant}/{precision}")


@pytest.mark.parametrize("variant", ["ds", "do"])
def test_batch_paper_do_rule_and_nondebug(variant):
    boxes = small_batch(replicas=10, variant=variant)
    g = run_batch(boxes, variant, "fp32", debug=False, options={0: 0.0})  # DO grown by whole cells
    check_replicas(boxes, g, "fp32", f"batch-nodebug/{variant}")


def test_batch_edge_sizes():
    """A one-particle replica, sizes at and around the 256-slot padding, and a
    flow-free replica in one batch."""
    base = wl.wca_replica_batch(replicas=4, n_lo=600, n_hi=900)
    boxes = [
        wl.make_box("planar", 0.3, 1, density=0.05, pot=wl.WCA, t_frac=0.2, seed=91, name="single"),
        wl.make_box("uniaxial", 0.4, 256, density=0.8442, pot=wl.WCA, t_frac=0.7, seed=92, name="n256"),
        wl.make_box("biaxial", 0.9, 257, density=0.8442, pot=wl.WCA, t_frac=0.4, seed=93, name="n257"),
        wl.make_box("none", 0.0, 511, density=0.8442, pot=wl.WCA, t=0.0, seed=94, name="still"),
    ] + base
    boxes = [b for b in boxes if fits(b, "do") and fits(b, "ds")]
    assert len(boxes) >= 6
    for variant in ("ds", "do"):
        for precision in ("fp64", "fp32"):
            g = run_batch(boxes, variant, precision)
            check_replicas(boxes, g, precision, f"edge/{variant}/{precision}")


def test_batch_single_replica_and_determinism():
    boxes = [wl.wca_planar_4096()]
    a = run_batch(boxes, "do", "fp32")
    check_replicas(boxes, a, "fp32", "single")
    b = run_batch(boxes, "do", "fp32")
    assert (a["F"] == b["F"]).all() and (a["U"] == b["U"]).all() and (a["W"] == b["W"]).all()


def test_batch_errors():
    import torch
    from paper_1412_3784_amd import Batch, NclError, nemdcl
    boxes = small_batch(replicas=6)
    xs = [oracle_positions(b) for b in boxes]
    bt = Batch([len(x) for x in xs])
    bt.set_potential(boxes[0].pot)
    with pytest.raises(NclError) as e:
        bt.build_cells(torch.zeros((sum(map(len, xs)), 3), dtype=torch.float64, device="cuda:0"))
    assert e.value.code == nemdcl.NCL_E_STATE
    A = [b.A.copy() for b in boxes]
    A[1][0, 1] = 0.1
    with pytest.raises(NclError) as e:
        bt.set_lattices("do", [b.L0 for b in boxes], A, [b.t for b in boxes], [b.automorphisms for b in boxes])
    assert e.value.code == nemdcl.NCL_E_LATTICE
    bt.set_lattices("do", [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    x = np.concatenate(xs)
    x[len(xs[0]) + 3, 1] = np.nan
    bt.build_cells(torch.from_numpy(x).to("cuda:0"), "fp32")
    bt.compute_forces()
    with pytest.raises(NclError) as e:
        bt.stats()
    assert e.value.code == nemdcl.NCL_E_DEVICE_FLAG
    # the flag is cleared once reported; a clean rebuild succeeds
    bt.build_cells(torch.from_numpy(np.concatenate(xs)).to("cuda:0"), "fp32")
    bt.compute_forces()
    bt.stats()
    bt.close()


def test_batch_box_too_small_is_flagged_and_skipped():
    """A replica whose box is thinner than the cut-off at its time raises
    BOX_TOO_SMALL from the next synchronising call; its forces are zero and the
    other replicas are unaffected."""
    import torch
    from paper_1412_3784_amd import Batch, NclError, nemdcl
    good = small_batch(replicas=4)
    thin = wl.make_box("uniaxial", 0.5, 40, side=2.2, pot=wl.WCA, t=0.0, seed=95, name="thin")
    # strained far enough without remap that a height drops below r_c
    thin.t, thin.automorphisms = 4.5, []
    assert not fits(thin, "do")
    boxes = good + [thin]
    xs = [oracle_positions(b) for b in boxes]
    bt = Batch([len(x) for x in xs])
    bt.set_potential(boxes[0].pot)
    bt.set_lattices("do", [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    bt.build_cells(torch.from_numpy(np.concatenate(xs)).to("cuda:0"), "fp32")
    F, U, W = bt.compute_forces()
    with pytest.raises(NclError) as e:
        bt.stats()
    assert e.value.code == nemdcl.NCL_E_BOX_TOO_SMALL
    Fh = F.cpu().numpy()
    assert (Fh[-len(xs[-1]):] == 0).all()
    off = 0
    for r, b in enumerate(good):
        ref = run_oracle(b, xs[r])
        n = len(xs[r])
        compare({"F": Fh[off:off + n].astype(np.float64), "U": float(U[r]), "W": W.cpu().numpy()[9 * r:9 * r + 9]
                 .reshape(3, 3)}, ref, "fp32", check_pairs=False, label=f"thin-batch/rep{r}")
        off += n
    bt.close()


# ---------------------------------------------------------------------------
# SLLOD
# ---------------------------------------------------------------------------
def nemd_batch(seed0=700, grids=(5, 6, 7, 6), flows=("planar", "uniaxial", "biaxial", "planar"),
               rates=(0.5, 0.3, 0.6, 0.4), t0s=None):
    boxes = []
    for r, (g, fl, ra) in enumerate(zip(grids, flows, rates)):
        b = wl.make_box(fl, ra, g ** 3, density=0.8442, pot=wl.WCA, t=0.0, seed=seed0 + r, grid=g,
                        jitter_sigma=0.02, name=f"nemd{r}")
        if t0s is not None:
            b.t = t0s[r]
        boxes.append(b)
    return boxes


def lattice_diff(a, b, L):
    d = np.asarray(a) - np.asarray(b)
    n = np.round(np.linalg.solve(L, d.T)).T
    return d - n @ L.T


def sllod_gpu(boxes, xs, ps, h, nsteps, precision, use_graph, history=True, bt=None, close=True):
    import torch
    from paper_1412_3784_amd import Batch
    if bt is None:
        bt = Batch([len(x) for x in xs])
        bt.set_potential(boxes[0].pot)
        bt.set_lattices("do", [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                        [b.automorphisms for b in boxes])
    x = torch.from_numpy(np.concatenate(xs)).to("cuda:0")
    p = torch.from_numpy(np.concatenate(ps)).to("cuda:0")
    bt.build_cells(x, precision)  # fixes the precision the run uses
    F, U, W, hist = bt.sllod_run(x, p, h, 1.0, nsteps, use_graph=use_graph, history=history)
    torch.cuda.synchronize()
    out = {"x": x.cpu().numpy(), "p": p.cpu().numpy(), "F": F.cpu().numpy(), "U": U.cpu().numpy(),
           "W": W.cpu().numpy(), "hist": None if hist is None else hist.cpu().numpy()}
    if close:
        bt.close()
        return out
    return out, bt


def start_state(boxes):
    xs = [oracle_positions(b) for b in boxes]
    ps = [wl.maxwell_momenta(len(x), 1.0, seed=900 + r) for r, x in enumerate(xs)]
    return xs, ps


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sllod_graph_equals_eager_bitwise(precision):
    boxes = nemd_batch()
    xs, ps = start_state(boxes)
    e = sllod_gpu(boxes, xs, ps, 0.002, 25, precision, use_graph=False)
    for rep in range(3):  # several replays, with eager work and syncs in between
        g = sllod_gpu(boxes, xs, ps, 0.002, 25, precision, use_graph=True)
        for k in ("x", "p", "F", "U", "W", "hist"):
            assert (g[k] == e[k]).all(), f"replay {rep}: {k} differs"


def test_sllod_continuation_matches_one_run():
    """Two runs of 15 steps on one batch object equal one run of 30 steps."""
    import torch
    boxes = nemd_batch()
    xs, ps = start_state(boxes)
    one = sllod_gpu(boxes, xs, ps, 0.002, 30, "fp64", use_graph=True, history=False)
    half, bt = sllod_gpu(boxes, xs, ps, 0.002, 15, "fp64", use_graph=True, history=False, close=False)
    n = [len(x) for x in xs]
    cut = np.cumsum([0] + n)
    xs2 = [half["x"][cut[r]:cut[r + 1]] for r in range(len(n))]
    ps2 = [half["p"][cut[r]:cut[r + 1]] for r in range(len(n))]
    two = sllod_gpu(boxes, xs2, ps2, 0.002, 15, "fp64", use_graph=False, history=False, bt=bt)
    torch.cuda.synchronize()
    for k in ("x", "p", "U", "W"):
        assert np.allclose(two[k], one[k], rtol=1e-12, atol=1e-12), k


def test_sllod_single_steps_and_zero_steps():
    """Runs of one step (a first step and the last step's second kick, no
    replayed step) chained three times equal one run of three steps; a run
    of zero steps leaves x and p unchanged and returns the starting forces,
    energy and virial."""
    boxes = nemd_batch()
    xs, ps = start_state(boxes)
    one = sllod_gpu(boxes, xs, ps, 0.002, 3, "fp64", use_graph=True, history=False)
    n = [len(x) for x in xs]
    cut = np.cumsum([0] + n)
    cur, bt = sllod_gpu(boxes, xs, ps, 0.002, 1, "fp64", use_graph=True, history=True, close=False)
    assert cur["hist"].shape[0] == 2
    for _ in range(2):
        xs_k = [cur["x"][cut[r]:cut[r + 1]] for r in range(len(n))]
        ps_k = [cur["p"][cut[r]:cut[r + 1]] for r in range(len(n))]
        cur, bt = sllod_gpu(boxes, xs_k, ps_k, 0.002, 1, "fp64", use_graph=True, history=False, bt=bt,
                            close=False)
    bt.close()
    for k in ("x", "p", "U", "W"):
        assert np.allclose(cur[k], one[k], rtol=1e-12, atol=1e-12), k
    zero = sllod_gpu(boxes, xs, ps, 0.002, 0, "fp64", use_graph=True, history=True)
    assert (zero["x"] == np.concatenate(xs)).all() and (zero["p"] == np.concatenate(ps)).all()
    start = sllod_gpu(boxes, xs, ps, 0.002, 1, "fp64", use_graph=False, history=True)
    assert (zero["hist"][0] == start["hist"][0]).all()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 2e-6)])
def test_sllod_matches_oracle_trajectory(precision, tol):
    """40 steps of every replica against the oracle's FP64 trajectory; the
    first replica crosses a KR remap during the run."""
    T0 = wl.make_box("planar", 0.5, 125, side=6.0).period
    boxes = nemd_batch(t0s=(0.5 * T0 - 0.04, 0.0, 0.1, 0.0))
    xs, ps = start_state(boxes)
    h, ns = 0.002, 40
    g = sllod_gpu(boxes, xs, ps, h, ns, precision, use_graph=True)
    cut = np.cumsum([0] + [len(x) for x in xs])
    for r, b in enumerate(boxes):
        xo, po, ho = oracle.sllod(xs[r], ps[r], b.L0, b.A, b.t, b.automorphisms, b.pot, h, 1.0, ns)
        L = oracle.lattice_at(b.L0, b.A, b.t + ns * h)
        dx = np.abs(lattice_diff(g["x"][cut[r]:cut[r + 1]], xo, L)).max()
        dp = np.abs(g["p"][cut[r]:cut[r + 1]] - po).max() / np.abs(po).max()
        assert dx < tol * np.abs(L).max(), f"rep {r}: position error {dx:.3e}"
        assert dp < 10 * tol, f"rep {r}: momentum error {dp:.3e}"
        hg = g["hist"][:, r, :]
        assert np.allclose(hg[:, 0], ho[:, 0], rtol=0, atol=1e-12)
        scale = np.abs(ho[:, 1:]).max(axis=0)
        err = (np.abs(hg[:, 1:] - ho[:, 1:]) / scale).max()
        assert err < 10 * tol, f"rep {r}: observable error {err:.3e}"
    _, _, ca = oracle.reduce(boxes[0].L0, boxes[0].A, boxes[0].t + ns * h, boxes[0].automorphisms)
    _, _, cb = oracle.reduce(boxes[0].L0, boxes[0].A, boxes[0].t, boxes[0].automorphisms)
    assert tuple(ca) != tuple(cb)  # the remap was crossed


def test_sllod_energy_balance():
    """Over 200 steps the energy balance of every replica drifts by no more
    than the oracle's own O(h^2) splitting error (plus FP32 force noise)."""
    boxes = nemd_batch()
    xs, ps = start_state(boxes)
    h, ns = 0.002, 200
    g = sllod_gpu(boxes, xs, ps, h, ns, "fp32", use_graph=True)
    for r, b in enumerate(boxes):
        _, _, ho = oracle.sllod(xs[r], ps[r], b.L0, b.A, b.t, b.automorphisms, b.pot, h, 1.0, ns)
        eo = np.abs(oracle.energy_balance(ho, b.A)).max()
        eg = np.abs(oracle.energy_balance(g["hist"][:, r, :], b.A)).max()
        H0 = 0.5 * ho[0, 5:8].sum() + ho[0, 1]
        assert eg < 2.0 * eo + 1e-5 * H0, f"rep {r}: GPU drift {eg:.3e} vs oracle {eo:.3e}"
