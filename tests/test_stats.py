"""The ensemble statistics (KS, W1, moments) against scipy's implementations."""
import numpy as np
import pytest
from scipy import stats

from paper_2605_00479_amd import stats as st


@pytest.mark.parametrize("shift", [0.0, 0.2, 1.0])
def test_ks_matches_scipy_asymptotic(shift):
    rng = np.random.default_rng(1)
    a = rng.poisson(20, 5000)
    b = rng.poisson(20 + shift, 7000)
    d, p = st.ks_2samp(a, b)
    ref = stats.ks_2samp(a, b, method="asymp")
    assert abs(d - ref.statistic) < 1e-12
    en = a.size * b.size / (a.size + b.size)
    # limiting Kolmogorov law exactly; scipy's finite-n variant to within 10%
    assert abs(p - stats.kstwobign.sf(d * np.sqrt(en))) < 1e-10
    assert abs(p - ref.pvalue) < 1e-6 + 0.1 * ref.pvalue


def test_kolmogorov_sf_matches_scipy():
    for lam in np.linspace(0.05, 4.0, 80):
        assert abs(st.ks_sf(lam) - stats.kstwobign.sf(lam)) < 1e-10


def test_w1_matches_scipy():
    rng = np.random.default_rng(2)
    for _ in range(5):
        a = rng.poisson(30, 3000)
        b = rng.negative_binomial(5, 0.15, 2000)
        assert abs(st.wasserstein1(a, b) - stats.wasserstein_distance(a, b)) < 1e-9
    x = rng.normal(size=1000)
    assert abs(st.wasserstein1(x, x + 0.5) - 0.5) < 1e-12
    assert st.wasserstein1(a, a) == 0.0


def test_moments_and_compare():
    x = np.array([1, 2, 3, 4, 10])
    m, v, f = st.moments(x)
    assert m == 4.0 and v == np.var(x, ddof=1) and f == v / m
    c = st.compare(x, x)
    assert c["ks_D"] == 0 and c["ks_p"] == 1.0 and c["w1"] == 0 and c["mean_rel_err"] == 0
