"""The entry point that allocates nothing (ncl_forces_noalloc): called
through the C ABI twice in a row, the second time on a smaller box, and
compared with the handle path it replaces (ncl_set_lattice +
ncl_build_cells + ncl_compute_forces with the per-particle sweep) on the
same inputs: forces, energy and virial identical bit for bit, both cell-list
variants, FP32 and FP64.  Sizes beyond the maximum are refused before any
work is enqueued."""
import numpy as np
import pytest

import workloads as wl
from parity_util import compare, oracle_positions, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_3784_amd  # noqa: F401  (fails loudly if the library is missing)


def handle_path(box, x, variant, precision):
    import torch
    from paper_1412_3784_amd import Handle
    from paper_1412_3784_amd import nemdcl as n
    h = Handle(0)
    h.set_potential(box.pot)
    h.set_option(n.NCL_OPT_SWEEP, n.NCL_SWEEP_PARTICLE)
    h.set_lattice(box.L0, box.A, box.t, box.automorphisms)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    h.build_cells(variant, xt, precision)
    F, U, W = h.compute_forces()
    torch.cuda.synchronize()
    out = F.cpu().numpy(), U.cpu().numpy().copy(), W.cpu().numpy().copy()
    h.close()
    return out


def noalloc_path(box, x, variant, precision):
    import torch
    from paper_1412_3784_amd import nemdcl as n
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    F = torch.full((len(x), 3), float("nan"), device=dev,
                   dtype=torch.float64 if precision == "fp64" else torch.float32)
    U = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    W = torch.full((9,), float("nan"), dtype=torch.float64, device=dev)
    pot = (box.pot.eps, box.pot.sigma, box.pot.rc, 1.0 if box.pot.shift else 0.0)
    n.ncl_forces_noalloc(0, torch.cuda.current_stream(dev).cuda_stream, box.L0, box.A, box.t, box.automorphisms,
                         pot, n.VARIANTS[variant], n.PRECISIONS[precision], xt, len(x), F, U, W)
    return F, U, W


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("variant", ["ds", "do"])
def test_noalloc_matches_handle_path_twice(variant, precision):
    import torch
    big = wl.wca_planar_4096()
    small = wl.make_box("biaxial", 0.4, 1500, density=0.8442, pot=wl.WCA, t_frac=0.6, seed=4242)
    xb, xs = oracle_positions(big), oracle_positions(small)
    rb = handle_path(big, xb, variant, precision)
    rs = handle_path(small, xs, variant, precision)
    # two calls in a row on the shared scratch, the second smaller
    Fb, Ub, Wb = noalloc_path(big, xb, variant, precision)
    torch.cuda.synchronize()
    Fb, Ub, Wb = Fb.cpu().numpy(), Ub.cpu().numpy(), Wb.cpu().numpy()
    Fs, Us, Ws = noalloc_path(small, xs, variant, precision)
    torch.cuda.synchronize()
    Fs, Us, Ws = Fs.cpu().numpy(), Us.cpu().numpy(), Ws.cpu().numpy()
    for (F, U, W), (Fr, Ur, Wr), label in (((Fb, Ub, Wb), rb, "4096"), ((Fs, Us, Ws), rs, "1500")):
        assert np.array_equal(F, Fr), f"{label}/{variant}/{precision}: forces differ"
        assert np.array_equal(U, Ur) and np.array_equal(W, Wr), f"{label}/{variant}/{precision}: U or W differ"
    # and the second call against the oracle
    g = {"F": Fs.astype(np.float64), "U": float(Us[0]), "W": Ws.reshape(3, 3)}
    compare(g, run_oracle(small, xs), precision, check_pairs=False, label=f"noalloc/{variant}/{precision}")


def test_noalloc_refuses_sizes_beyond_maximum():
    import torch
    from paper_1412_3784_amd import NclError
    from paper_1412_3784_amd import nemdcl as n
    dev = torch.device("cuda:0")
    nmax = n.NCL_NOALLOC_MAX_N
    box = wl.make_box("uniaxial", 0.3, nmax + 1, density=0.8, pot=wl.LJ25, t_frac=0.2, seed=9)
    x = torch.zeros((nmax + 1, 3), dtype=torch.float64, device=dev)
    F = torch.zeros((nmax + 1, 3), dtype=torch.float32, device=dev)
    U = torch.zeros(1, dtype=torch.float64, device=dev)
    W = torch.zeros(9, dtype=torch.float64, device=dev)
    pot = (1.0, 1.0, 2.5, 1.0)
    with pytest.raises(NclError) as e:
        n.ncl_forces_noalloc(0, 0, box.L0, box.A, box.t, box.automorphisms, pot, n.NCL_DYNAMIC_OFFSET,
                             n.NCL_PREC_FP32, x, nmax + 1, F, U, W)
    assert e.value.code == n.NCL_E_CAPACITY
    # few particles in a box with more cells than the maximum
    box = wl.make_box("none", 0.0, 1000, side=60.0 * 2.5, pot=wl.LJ25, seed=10)
    xs = torch.from_numpy(oracle_positions(box)).to(dev)
    with pytest.raises(NclError) as e:
        n.ncl_forces_noalloc(0, 0, box.L0, box.A, box.t, box.automorphisms, pot, n.NCL_DYNAMIC_SIZE,
                             n.NCL_PREC_FP32, xs, 1000, F, U, W)
    assert e.value.code == n.NCL_E_CAPACITY
    assert float(U.cpu()[0]) == 0.0  # nothing was enqueued
