"""Host-side analysis of chain output: energy autocorrelation and effective
sample size.

Paper: Liang, Xing, Li, arXiv:1602.05716, Sec. 5.2 -- autocorrelation function
C_n of the total energy and the integrated autocorrelation time
T_c = 1/2 + sum_{k>=1} C_k.  The paper does not say where the infinite sum is
cut; here it runs over pairs of lags, C_{2m} + C_{2m+1}, up to the first pair
whose sum is not positive (Geyer's initial positive sequence, 1992), which
also converges for negatively correlated series.  The effective sample size
of n correlated values is n / (2 T_c).
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


def integrated_time(series: np.ndarray) -> float:
    """T_c = 1/2 + sum_{k>=1} C_k = -1/2 + sum_{m>=0} (C_{2m} + C_{2m+1}),
    summed over pairs of lags up to the first pair whose sum is not positive.
    NaN for a constant series or fewer than two values."""
    x = np.asarray(series, np.float64)
    if len(x) < 2 or not np.any(x != x[0]):
        return float("nan")
    c = autocorrelation(x)
    npairs = len(c) // 2
    pairs = c[0:2 * npairs:2] + c[1:2 * npairs:2]
    stop = np.flatnonzero(~(pairs > 0.0))
    m = int(stop[0]) if stop.size else npairs
    return float(-0.5 + np.sum(pairs[:m]))


def effective_samples(series: np.ndarray) -> float:
    """n / (2 T_c)."""
    return len(series) / (2.0 * integrated_time(series))


# --------------------------------------------------------------------------- #
# Renormalised (dressed-ion) parameters of a binary electrolyte, Sec. 5.1     #
# --------------------------------------------------------------------------- #
# Reduced units: lengths in ion diameters, energies in kT, charges in e, so
# the solvent permittivity is eps = 1 / (4 pi l_B).  Species 0 is the cation,
# species 1 the anion; g[a, b] is g_ab(r) on the bin centres r (the layout of
# mc_rdf).  Far from a fixed ion of species a the dressed-ion theory gives
#   U_ab(r)   = (eps / eps_R) l_B q_a^R q_b^R exp(-kappa_R r) / r,
#   rho_a(r)  = -kappa_R^2 (eps / eps_R) q_a^R exp(-kappa_R r) / (4 pi r),
# the charge density from Poisson's equation rho = -eps lap(phi) for the mean
# potential phi_a = q_a^R exp(-kappa_R r) / (4 pi eps_R r).


def g_from_counts(counts, centres, n_of_type, sigma_of_type, R: float, rmax: float):
    """g_ab(r_k) = C_ab(k) / (Ncentre_a n_b V_k) from raw counts (the
    normalisation mc_rdf applies; counts and centre counts may be sums over
    several chains of one system): n_b = (N_b - delta_ab) / ((4/3) pi
    (R - sigma_b / 2)^3), V_k the k-th shell.  Returns (bin centres, g)."""
    counts = np.asarray(counts, np.float64)
    centres = np.asarray(centres, np.float64)
    nt, _, bins = counts.shape
    dr = rmax / bins
    edges = np.arange(bins + 1) * dr
    vk = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    g = np.zeros_like(counts)
    for a in range(nt):
        for b in range(nt):
            nb = (n_of_type[b] - (1 if a == b else 0)) / (4.0 / 3.0 * np.pi * (R - 0.5 * sigma_of_type[b]) ** 3)
            if centres[a] > 0:
                g[a, b] = counts[a, b] / (centres[a] * nb * vk)
    return 0.5 * (edges[1:] + edges[:-1]), g


def bare_kappa(lB: float, n, q) -> float:
    """Debye-Hueckel inverse screening length, kappa^2 = 4 pi l_B sum n_a q_a^2."""
    n = np.asarray(n, np.float64)
    q = np.asarray(q, np.float64)
    return float(np.sqrt(4.0 * np.pi * lB * np.sum(n * q * q)))


def tail_plateau(r, g, r_flat: float) -> np.ndarray:
    """g_ab averaged over r >= r_flat: its bulk value.  mc_rdf normalises by
    the mean density over the whole sphere, which differs from the density
    of the bulk the centres sit in by a wall-layer correction; the plateau
    measures that ratio."""
    r = np.asarray(r, np.float64)
    sel = r >= r_flat
    if sel.sum() < 3:
        raise ValueError("fewer than 3 bins beyond r_flat")
    return np.asarray(g, np.float64)[..., sel].mean(axis=-1)


def pmf(g, g_inf) -> np.ndarray:
    """Potential of mean force U_ab = -log(g_ab / g_ab(inf)) in kT (Sec. 5.1)."""
    g = np.asarray(g, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return -np.log(g / np.asarray(g_inf, np.float64)[..., None])


def charge_density(g, n, q, g_inf) -> np.ndarray:
    """rho_a(r) = sum_b n_b q_b (g_ab(r) - g_ab(inf)): the mean charge density
    around a fixed ion of species a (the centre, first index of g), its own
    charge excluded (Eq. rho-g-g), with the bulk value subtracted (zero for a
    neutral bulk)."""
    g = np.asarray(g, np.float64)
    n = np.asarray(n, np.float64)
    q = np.asarray(q, np.float64)
    gi = np.asarray(g_inf, np.float64)
    nt = g.shape[0]
    return np.stack([sum(n[b] * q[b] * (g[a, b] - gi[a, b]) for b in range(nt)) for a in range(nt)])


def _screened_fit(rw, rho, wt, kappa0):
    """Weighted least squares of rho[a] = A_a exp(-k r) / r over the rows a
    with one k: the amplitudes are linear (solved for each k), k is found on a
    log grid over [kappa0 / 10, 10 kappa0] and refined by bounded Brent
    search.  Returns (k, amplitudes)."""
    from scipy.optimize import minimize_scalar

    def amps(k):
        f = np.exp(-k * rw) / rw
        return np.array([np.sum(wt[a] * f * rho[a]) / np.sum(wt[a] * f * f) for a in range(len(rho))]), f

    def chi2(k):
        A, f = amps(k)
        return float(sum(np.sum(wt[a] * (rho[a] - A[a] * f) ** 2) for a in range(len(rho))))

    grid = kappa0 * np.exp(np.linspace(np.log(0.1), np.log(10.0), 241))
    i = int(np.argmin([chi2(k) for k in grid]))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
    k = float(minimize_scalar(chi2, bounds=(lo, hi), method="bounded", options={"xatol": 1e-12 * kappa0}).x)
    return k, amps(k)[0]


def charge_density_error(counts, g, n, q) -> np.ndarray:
    """Standard error of rho_a per bin from Poisson errors of the pair counts
    (sigma_g = g / sqrt(C)); correlations between samples scale every bin
    alike, so the relative weights of a fit are unaffected."""
    C = np.maximum(np.asarray(counts, np.float64), 1.0)
    sg = np.asarray(g, np.float64) / np.sqrt(C)
    n = np.asarray(n, np.float64)
    q = np.asarray(q, np.float64)
    nt = sg.shape[0]
    return np.sqrt(np.stack([sum((n[b] * q[b] * sg[a, b]) ** 2 for b in range(nt)) for a in range(nt)]))


def renormalised_parameters(r, g, n, q, lB: float, fit, r_flat: float | None = None, g_inf=None,
                            rho_err=None) -> dict:
    """Renormalised inverse Debye length, valences and dielectric constant
    from the tails of g_ab (Sec. 5.1), and the dressed-ion relation
    (kappa_R / kappa)^2 = (q_+^R - q_-^R) / (q_+ - q_-) (Eq. RD).

    r, g: bin centres and g[a, b, bins] (species 0 cation, 1 anion); n: the
    densities g is normalised by; q: bare valences; fit = (r_lo, r_hi): the
    far-field window; r_flat: start of the plateau that gives g_ab(inf)
    (default: 0.9 of the last bin), or g_inf given directly.

      * kappa_R: the common slope of log|r rho_a| against r for both centre
        species (Eq. linear-fit; the two lines share it), one least-squares
        fit with an intercept per species; also each species' own slope.
        With rho_err [2, bins] (standard errors of rho) the same model,
        rho_a = A_a exp(-kappa_R r) / r, is fitted to rho itself by weighted
        least squares instead (noise can flip the sign of far bins, which a
        fit of the log cannot take).
      * q_b^R, two ways: q_b^R = -eps kappa_R^2 U_ab / rho_a (Eq. qR-U-rho)
        with centre a = + and a = -, each a least-squares ratio over the
        window.
      * eps_R / eps, two ways: from the intercept of log|r rho_a| at slope
        -kappa_R and q_a^R (Eq. ep_R-phi).
    """
    r = np.asarray(r, np.float64)
    g = np.asarray(g, np.float64)
    n = np.asarray(n, np.float64)
    q = np.asarray(q, np.float64)
    if g.shape[:2] != (2, 2) or len(n) != 2 or len(q) != 2 or not (q[0] > 0 > q[1]):
        raise ValueError("a binary electrolyte (cation, anion) is expected")
    if g_inf is None:
        g_inf = tail_plateau(r, g, r[-1] * 0.9 if r_flat is None else r_flat)
    g_inf = np.asarray(g_inf, np.float64)
    w = (r >= fit[0]) & (r <= fit[1])
    if w.sum() < 5:
        raise ValueError("fewer than 5 bins in the fit window")
    rho = charge_density(g, n, q, g_inf)
    U = pmf(g, g_inf)
    n_bulk = n * np.diag(g_inf)
    kappa = bare_kappa(lB, n_bulk, q)
    # far-field signs: the cloud around a cation is negative, around an anion positive
    sign = np.array([-1.0, 1.0])
    rw = r[w]
    k_a, c_a = np.zeros(2), np.zeros(2)
    if rho_err is None:
        ys, rbar, ybar = [], np.zeros(2), np.zeros(2)
        for a in range(2):
            y = sign[a] * rw * rho[a, w]
            if np.any(y <= 0):
                raise ValueError("rho_%s changes sign inside the fit window" % "+-"[a])
            y = np.log(y)
            rbar[a], ybar[a] = rw.mean(), y.mean()
            k_a[a] = -np.sum((rw - rbar[a]) * (y - ybar[a])) / np.sum((rw - rbar[a]) ** 2)
            ys.append(y)
        kR = float(k_a.mean())  # the common slope on one grid: the mean of the two
        for a in range(2):
            c_a[a] = float(ybar[a] + kR * rbar[a])
    else:
        err = np.asarray(rho_err, np.float64)[:, w]
        wt = 1.0 / err ** 2
        for a in range(2):
            k_a[a] = _screened_fit(rw, rho[a:a + 1, w], wt[a:a + 1], kappa)[0]
        kR, amp = _screened_fit(rw, rho[:, w], wt, kappa)
        for a in range(2):
            if sign[a] * amp[a] <= 0:
                raise ValueError("the fitted amplitude of rho_%s has the wrong sign" % "+-"[a])
            c_a[a] = float(np.log(sign[a] * amp[a]))
    pre = -kR * kR / (4.0 * np.pi * lB)  # -eps kappa_R^2 in reduced units
    qR = np.zeros((2, 2))  # qR[b, a]: valence of species b measured around centre a
    for b in range(2):
        for a in range(2):
            u, p = U[a, b, w], rho[a, w]
            wt = np.ones_like(p) if rho_err is None else 1.0 / np.asarray(rho_err, np.float64)[a, w] ** 2
            qR[b, a] = pre * float(np.sum(wt * u * p) / np.sum(wt * p * p))
    qR_mean = qR.mean(axis=1)
    epsR = np.array([kR * kR * abs(qR_mean[a]) / (4.0 * np.pi * np.exp(c_a[a])) for a in range(2)])
    lhs = (kR / kappa) ** 2
    rhs = (qR_mean[0] - qR_mean[1]) / (q[0] - q[1])
    return {"kappa": kappa, "kappa_R": kR, "kappa_R_by_centre": k_a.tolist(),
            "qR_plus": qR[0].tolist(), "qR_minus": qR[1].tolist(), "qR": qR_mean.tolist(),
            "epsR_over_eps": epsR.tolist(), "rd_lhs": float(lhs), "rd_rhs": float(rhs),
            "g_inf": g_inf.tolist(), "window_bins": int(w.sum()), "rho": rho, "U": U}
