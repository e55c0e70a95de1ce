"""Host-side analysis of chain output: energy autocorrelation and effective
sample size.

Paper: Liang, Xing, Li, arXiv:1602.05716, Sec. 5.2 -- autocorrelation function
C_n of the total energy and the integrated autocorrelation time
T_c = 1/2 + sum_{k>=1} C_k.  The paper does not say where the infinite sum is
cut; here it stops at the first window M >= c T_c(M) (Sokal's automatic
window, c = 5).  The effective sample size of n correlated values is
n / (2 T_c).
"""
from __future__ import annotations

import numpy as np


def autocorrelation(series: np.ndarray, max_lag: int | None = None) -> np.ndarray:
    """Normalised autocovariance C_0..C_max_lag via FFT (C_0 = 1)."""
    x = np.asarray(series, np.float64)
    x = x - x.mean()
    n = len(x)
    if max_lag is None:
        max_lag = n - 1
    size = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(x, size)
    acov = np.fft.irfft(f * np.conj(f), size)[: max_lag + 1] / n
    return acov / acov[0] if acov[0] > 0 else np.zeros(max_lag + 1)


def integrated_time(series: np.ndarray, window_c: float = 5.0) -> float:
    c = autocorrelation(series)
    tau = 0.5
    for m in range(1, len(c)):
        tau += c[m]
        if m >= window_c * tau:
            break
    return max(tau, 0.5)


def effective_samples(series: np.ndarray, window_c: float = 5.0) -> float:
    return len(series) / (2.0 * integrated_time(series, window_c))
