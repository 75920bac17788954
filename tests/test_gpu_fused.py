"""The batched form's fused bin + force launch (NCL_OPT_SWEEP = 4 for
batches): every replica's cell build sorted inside one workgroup, the
sweep blocks waiting on per-replica ready flags.  It must give the staged
schedule's forces, energy and virial bit for bit (the sort is stable and the
sweep code is shared), and match the FP64 oracle per replica.  Replica sizes
cover one particle, the 256-slot padding edges, and a box with more than
2^16 cells (a third radix pass); the batched autotuner picks one of the two
schedules and reports both times."""
import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import compare, oracle_positions, run_oracle

pytestmark = pytest.mark.gpu

SWEEP_OPT = 3  # NCL_OPT_SWEEP


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


def mixed_boxes(variant, big=False):
    boxes = [
        wl.make_box("planar", 0.3, 1, density=0.05, pot=wl.WCA, t_frac=0.2, seed=191, name="single"),
        wl.make_box("uniaxial", 0.4, 256, density=0.8442, pot=wl.WCA, t_frac=0.7, seed=192, name="n256"),
        wl.make_box("biaxial", 0.9, 257, density=0.8442, pot=wl.WCA, t_frac=0.4, seed=193, name="n257"),
        wl.make_box("none", 0.0, 700, density=0.8442, pot=wl.WCA, t=0.0, seed=194, name="still"),
    ] + wl.wca_replica_batch(replicas=20, n_lo=300, n_hi=6000)
    if big:
        # about 1e5 cells: 17-bit keys, three radix passes
        boxes.append(wl.make_box("uniaxial", 0.2, 120000, density=0.8442, pot=wl.WCA, t_frac=0.3, seed=195,
                                 name="big"))
    return [b for b in boxes if fits(b, variant)]


def run(boxes, variant, precision, mode, xs=None):
    import torch
    from paper_1412_3784_amd import Batch
    xs = xs or [oracle_positions(b) for b in boxes]
    bt = Batch([len(x) for x in xs])
    bt.set_potential(boxes[0].pot)
    if mode is not None:
        bt.set_option(SWEEP_OPT, mode)
    bt.set_lattices(variant, [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    xt = torch.from_numpy(np.concatenate(xs)).to("cuda:0")
    bt.build_cells(xt, precision)
    F, U, W = bt.compute_forces()
    torch.cuda.synchronize()
    out = {"x": xs, "F": F.cpu().numpy(), "U": U.cpu().numpy(), "W": W.cpu().numpy().reshape(-1, 3, 3)}
    out["stats"] = bt.stats()
    # a second pass on the same positions (the fused schedule bins again)
    bt.build_cells(xt, precision)
    F2, U2, W2 = bt.compute_forces()
    torch.cuda.synchronize()
    out["repeat_equal"] = bool(np.array_equal(F2.cpu().numpy(), out["F"]) and np.array_equal(U2.cpu().numpy(), out["U"]))
    bt.close()
    return out


@pytest.mark.parametrize("variant", ["ds", "do"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32k"])
def test_fused_equals_staged_and_oracle(variant, precision):
    from paper_1412_3784_amd import nemdcl as n
    boxes = mixed_boxes(variant, big=(precision == "fp32"))
    assert len(boxes) >= 18
    xs = [oracle_positions(b) for b in boxes]
    st = run(boxes, variant, precision, n.NCL_SWEEP_PARTICLE, xs)
    fu = run(boxes, variant, precision, n.NCL_SWEEP_FUSED, xs)
    label = f"fused/{variant}/{precision}"
    assert fu["stats"]["sweep"] == n.NCL_SWEEP_FUSED and st["stats"]["sweep"] == n.NCL_SWEEP_PARTICLE
    assert np.array_equal(fu["F"], st["F"]), f"{label}: forces differ from the staged schedule"
    assert np.array_equal(fu["U"], st["U"]) and np.array_equal(fu["W"], st["W"]), label
    assert fu["stats"]["pairs"] == st["stats"]["pairs"] and fu["stats"]["candidates"] == st["stats"]["candidates"]
    assert fu["stats"]["max_occupancy"] == st["stats"]["max_occupancy"]
    assert fu["repeat_equal"] and st["repeat_equal"]
    off, tot = 0, 0
    for r, b in enumerate(boxes):
        nr = len(xs[r])
        ref = run_oracle(b, xs[r], want_hash=False)
        g = {"F": fu["F"][off:off + nr].astype(np.float64), "U": float(fu["U"][r]), "W": fu["W"][r]}
        compare(g, ref, precision, check_pairs=False, label=f"{label}/rep{r}({b.name}, n={nr})")
        tot += int(ref.stats[1])
        off += nr
    assert fu["stats"]["pairs"] == tot


def test_fused_autotuner_picks_and_reports():
    from paper_1412_3784_amd import nemdcl as n
    boxes = mixed_boxes("do")
    xs = [oracle_positions(b) for b in boxes]
    st = run(boxes, "do", "fp32", n.NCL_SWEEP_PARTICLE, xs)
    au = run(boxes, "do", "fp32", None, xs)  # default: autotuned
    tm = au["stats"]["tune_ms"]
    assert tm[0] > 0 and tm[1] > 0, tm
    assert np.array_equal(au["F"], st["F"]) and np.array_equal(au["U"], st["U"])
    assert au["repeat_equal"]


def test_fused_invalid_replica_isolated():
    """A replica thinner than the cut-off is flagged and gets zero forces;
    the others are unaffected (as in the staged schedule)."""
    import torch
    from paper_1412_3784_amd import Batch, NclError
    from paper_1412_3784_amd import nemdcl as n
    boxes = mixed_boxes("do")[:6]
    thin = wl.make_box("none", 0.0, 50, side=1.0, pot=wl.WCA, t=0.0, seed=7, name="thin")
    allb = boxes + [thin]
    xs = [oracle_positions(b) for b in allb]
    outs = {}
    for mode in (n.NCL_SWEEP_PARTICLE, n.NCL_SWEEP_FUSED):
        bt = Batch([len(x) for x in xs])
        bt.set_potential(boxes[0].pot)
        bt.set_option(SWEEP_OPT, mode)
        bt.set_lattices("do", [b.L0 for b in allb], [b.A for b in allb], [b.t for b in allb],
                        [b.automorphisms for b in allb])
        xt = torch.from_numpy(np.concatenate(xs)).to("cuda:0")
        bt.build_cells(xt, "fp32")
        F, U, W = bt.compute_forces()
        torch.cuda.synchronize()
        with pytest.raises(NclError) as e:
            bt.stats()
        assert e.value.code == n.NCL_E_BOX_TOO_SMALL
        outs[mode] = (F.cpu().numpy(), U.cpu().numpy())
        bt.close()
    Fs, Us = outs[n.NCL_SWEEP_PARTICLE]
    Ff, Uf = outs[n.NCL_SWEEP_FUSED]
    assert np.array_equal(Fs, Ff) and np.array_equal(Us, Uf)
    assert np.all(Ff[-len(xs[-1]):] == 0.0)


@pytest.mark.parametrize("mode", [None, 4])
def test_positions_read_only_at_build(mode):
    """The positions array may be released after ncl_batch_build_cells (the
    fused schedule and the autotuner work from a copy): a temporary tensor
    whose memory is reused by the force outputs still gives the staged
    schedule's results."""
    import torch
    from paper_1412_3784_amd import Batch
    from paper_1412_3784_amd import nemdcl as n
    boxes = mixed_boxes("do")[:8]
    xs = [oracle_positions(b) for b in boxes]
    ref = run(boxes, "do", "fp32", n.NCL_SWEEP_PARTICLE, xs)
    bt = Batch([len(x) for x in xs])
    bt.set_potential(boxes[0].pot)
    if mode is not None:
        bt.set_option(SWEEP_OPT, mode)
    bt.set_lattices("do", [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    bt.build_cells(torch.from_numpy(np.concatenate(xs)).to("cuda:0"), "fp32")  # a temporary
    junk = torch.full((sum(len(x) for x in xs), 3), float("nan"), dtype=torch.float64, device="cuda:0")
    F, U, W = bt.compute_forces()
    torch.cuda.synchronize()
    del junk
    assert np.array_equal(F.cpu().numpy(), ref["F"]) and np.array_equal(U.cpu().numpy(), ref["U"])
    bt.stats()
    bt.close()
