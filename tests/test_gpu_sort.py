"""The cell build's radix sort at sizes that reach its edges, checked through
the whole force pass against the FP64 oracle for every particle (pair
digests exactly, forces, energy and virial to the precision's bar):

* a partial last tile (2,048 keys) and a partial last segment of the
  two-level column scan (64 tiles), two 9-bit passes;
* keys in runs of one digit (a jittered grid given in lattice order, so
  that neighbouring inputs share cells), two 7-bit passes;
* three passes (more than 2^20 cells: 1.7 M WCA particles at 1.2 per cell).

The expected pass count is derived from the cell counts and asserted, so a
change of the tile or digit sizes cannot silently drop a case."""
import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import compare, oracle_positions, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

RS_TILE, RS_SEG, RS_MAXLOG = 2048, 64, 10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_3784_amd  # noqa: F401  (fails loudly if the library is missing)


def sort_plan(box, variant):
    """(cells, digit passes, tiles, column-scan segments) of the build"""
    Lr, _, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    c = oracle.ds_counts(Lr, box.pot.rc) if variant == "ds" else oracle.do_counts(Lr, box.pot.rc)
    nc = int(np.prod(c.astype(np.int64)))
    bits = max(1, int(nc - 1).bit_length())
    passes = -(-bits // RS_MAXLOG)
    nt = -(-box.n // RS_TILE)
    return nc, passes, nt, -(-nt // RS_SEG)


CASES = {
    "partial_segment": lambda: wl.make_box("uniaxial", 0.4, 300001, density=0.8442, pot=wl.WCA, t_frac=0.3,
                                           seed=501, name="partial_segment"),
    "digit_runs": lambda: wl.make_box("biaxial", 0.2, 48 ** 3, density=0.8, pot=wl.LJ25, t_frac=0.5, seed=502,
                                      name="digit_runs", grid=48, jitter_sigma=0.05),
    "three_passes": lambda: wl.make_box("planar", 0.3, 1700000, density=0.8442, pot=wl.WCA, t_frac=0.6,
                                        seed=503, name="three_passes"),
}


@pytest.mark.parametrize("variant", ["do", "ds"])
@pytest.mark.parametrize("case", list(CASES))
def test_sorted_build_edges(case, variant):
    box = CASES[case]()
    nc, passes, nt, nseg = sort_plan(box, variant)
    if case == "partial_segment":
        assert box.n % RS_TILE != 0 and nt % RS_SEG != 0 and nseg >= 2 and passes == 2, (nc, passes, nt)
    elif case == "digit_runs":
        assert passes == 2 and box.n / nc > 8, (nc, passes)
    else:
        assert passes == 3, (nc, passes)
    x = oracle_positions(box)
    g = run_gpu(box, x, variant, "fp32")
    assert g["stats"]["ncells"] == nc
    r = run_oracle(box, x)
    compare(g, r, "fp32", label=f"{case}/{variant} ({nc} cells, {passes} passes, {nt} tiles)")
