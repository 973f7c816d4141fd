"""The histogram entry point that allocates nothing (rt_mu_histogram_noalloc) against
rt_mu_histogram, through the C ABI: identical kernels, so identical results, on two
calls in a row (the second with fewer values and fewer bins, over the scratch the first
left behind), and the bin limit refused on the host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1110_4894_amd import rt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


def _both(mus, n_bins, lo, hi):
    dev = torch.device("cuda")
    m = torch.from_numpy(mus).to(dev)
    out = []
    for fn in (rt.rt_mu_histogram, rt.rt_mu_histogram_noalloc):
        pdf = torch.full((n_bins,), np.nan, dtype=torch.float64, device=dev)
        mom = torch.full((6,), np.nan, dtype=torch.float64, device=dev)
        fn(len(mus), m, n_bins, lo, hi, pdf, mom)
        rt.rt_sync()
        out.append((pdf.cpu().numpy(), mom.cpu().numpy()))
    return out


def test_noalloc_histogram_matches_allocating_one():
    rng = np.random.default_rng(21)
    big = np.concatenate([np.exp(rng.normal(0, 0.08, 40011)), [-1.0, 0.0, 0.3, 7.0]])
    small = np.concatenate([np.exp(rng.normal(0, 0.05, 999)), [-2.0, 50.0]])
    for mus, nb, lo, hi in ((big, 200, -0.1, 0.3), (small, 37, -0.05, 0.1)):
        (p_ref, m_ref), (p, m) = _both(mus, nb, lo, hi)
        assert np.array_equal(p, p_ref)
        assert np.array_equal(m, m_ref)
        assert np.all(np.isfinite(p)) and m[0] > 0


def test_noalloc_histogram_refuses_too_many_bins():
    dev = torch.device("cuda")
    m = torch.ones(10, dtype=torch.float64, device=dev)
    pdf = torch.empty(65537, dtype=torch.float64, device=dev)
    mom = torch.empty(6, dtype=torch.float64, device=dev)
    with pytest.raises(rt.RTError):
        rt.rt_mu_histogram_noalloc(10, m, 65537, -0.1, 0.3, pdf, mom)
