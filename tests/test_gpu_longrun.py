"""The long-run neighbourhood experiment of Sec. 5.3 with counts measured by
the GPU lists: over 20 remap periods of the uniaxial run the measured search
efficiency (in-range pairs / candidates) of the dynamic-size list and of the
dynamic-offset list with the paper's neighbourhood must equal the geometric
efficiency 1 / <neighbourhood volume> at the same times (uniform particles
make the counts proportional to volumes), and both sit near the paper's
long-run values 0.0688 and 0.123."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_3784_amd  # noqa: F401


def test_measured_long_run_efficiency():
    import bench
    r = bench.longrun_measure(samples=120)
    assert r["ds"] == pytest.approx(r["geometric_ds"], rel=0.01)
    # the paper's case counts assume generic face offsets; aligned offsets
    # need fewer cells, so the measured list is at least as efficient
    assert r["do_paper"] >= r["geometric_do_paper"] * 0.99
    assert r["do_paper"] == pytest.approx(r["geometric_do_paper"], rel=0.03)
    assert r["ds"] == pytest.approx(0.0688, rel=0.03)
    assert r["do_paper"] == pytest.approx(0.123, rel=0.04)
    # growing by d_cut instead of whole cells only removes cells
    assert r["do_tight"] > r["do_paper"]
    print(r)
