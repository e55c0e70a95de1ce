"""The product's energy-series statistics (paper_1602_05716_amd.analysis),
the ESS/s figures of the benchmark rest on them: T_c = 1/2 + sum_k C_k of
Sec. 5.2 against the oracle's direct-sum estimator and against closed forms.
"""
import math

import numpy as np
import pytest

from paper_1602_05716_amd import analysis


def _ar1(rho, n, seed):
    from scipy.signal import lfilter
    return lfilter([1.0], [1.0, -rho], np.random.default_rng(seed).normal(size=n))


@pytest.mark.parametrize("rho", [-0.6, -0.3, 0.0, 0.4, 0.8, 0.95])
def test_integrated_time_matches_oracle_and_ar1(oracle, rho):
    """AR(1): C_k = rho^k, T_c = (1 + rho) / (2 (1 - rho)); the FFT
    autocovariance and the oracle's direct sums stop at the same lag."""
    x = _ar1(rho, 100_000 if rho < 0.9 else 400_000, 40 + int(10 * rho))
    t = analysis.integrated_time(x)
    assert t == pytest.approx(oracle.tau_int(x), rel=1e-9)
    assert t == pytest.approx((1 + rho) / (2 * (1 - rho)), rel=0.08, abs=0.012)
    assert analysis.effective_samples(x) == pytest.approx(len(x) / (2 * t), rel=1e-15)


def test_integrated_time_on_short_and_degenerate_series(oracle):
    rng = np.random.default_rng(3)
    for n in (2, 3, 9, 50, 501):
        x = rng.normal(size=n).cumsum()
        assert analysis.integrated_time(x) == pytest.approx(oracle.tau_int(x), rel=1e-9, abs=1e-12)
    assert math.isnan(analysis.integrated_time(np.full(40, 2.5)))
    assert math.isnan(analysis.integrated_time(np.array([1.0])))


def test_autocorrelation_matches_definition():
    """C_k = sum_t (x_t - m)(x_{t+k} - m) / sum_t (x_t - m)^2, by hand."""
    x = np.random.default_rng(4).normal(size=257)
    c = analysis.autocorrelation(x, 20)
    d = x - x.mean()
    want = np.array([np.dot(d[: len(d) - k], d[k:]) for k in range(21)]) / np.dot(d, d)
    assert np.allclose(c, want, rtol=1e-12, atol=1e-14)
