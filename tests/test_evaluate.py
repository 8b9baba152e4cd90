"""Host-side accuracy criteria (Sec. 4.4) and the ER + Poisson generator of
the paper's experiments (Sec. 3.5): no device needed."""
import numpy as np
import pytest
from scipy.stats import wasserstein_distance

import tn_inputs as T
from paper_2307_04890_amd.evaluate import emd_1d, relative_memory


def test_emd_matches_the_library_routine():
    g = T.rng(1)
    for k in range(20):
        a = g.integers(1, 500, size=g.integers(1, 300))
        b = g.integers(1, 500, size=g.integers(1, 300))
        assert emd_1d(a, b) == pytest.approx(wasserstein_distance(a, b), rel=1e-12, abs=1e-12)


def test_emd_closed_forms():
    a = np.array([1, 5, 9, 9, 40])
    assert emd_1d(a, a) == 0.0
    assert emd_1d(a, a + 7) == pytest.approx(7.0)           # a shift moves all mass by 7
    assert emd_1d([0], [3]) == pytest.approx(3.0)
    # equal sizes: the mean gap between the sorted samples
    b = np.array([2, 2, 10, 30, 41])
    assert emd_1d(a, b) == pytest.approx(np.mean(np.abs(np.sort(a) - np.sort(b))))
    with pytest.raises(ValueError):
        emd_1d([], [1])


def test_relative_memory_of_the_paper_setting():
    # n_s = 0.3 n and 5 hashes: about 5 * 0.09 = 0.45 of the exact matrix
    assert relative_memory(10_000, 3_000, 5) == pytest.approx(0.45, abs=0.01)


def test_er_poisson_generator():
    n, m = 2000, 50_000
    s, d, t = T.er_poisson(n, m, 10 * m, seed=3)
    assert s.shape == d.shape == t.shape == (m,)
    assert (np.diff(t) >= 0).all() and (s != d).all()
    links = {(min(a, b), max(a, b)) for a, b in zip(s.tolist(), d.tolist())}
    # G(n, 2/n) has about n - 1 links (Binomial(n(n-1)/2, 2/n))
    assert 0.85 * (n - 1) < len(links) < 1.15 * (n - 1)
    deg = np.bincount(np.array([x for e in links for x in e]), minlength=n)
    assert 1.7 < deg.mean() < 2.3  # Poisson degree distribution of mean 2
