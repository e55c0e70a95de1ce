"""Dilute-limit pins of the oracle chain (many-body statistics).

Paper: Liang, Xing, Li, arXiv:1602.05716, Sec. 5.1 -- Poisson-Boltzmann /
Debye-Hueckel pair potential of mean force with kappa^2 from Eq.
(alpha-kappa_0), and Sec. 5.2 -- PMF = -kT ln g and the charge density around
a fixed ion, Eq. (rho-g-g).
"""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def dilute_run(oracle):
    from paper_1602_05716_amd import inputs
    n, phi, lB, rmax, dr = 2000, 0.001, 0.7, 20.0, 0.5
    s = inputs.electrolyte(n // 2, n // 2, 1.0, -1.0, 1.0, 1.0, phi, lB)
    s.xyz = inputs.random_start(s, 21)
    a = s.R - 0.5
    dens = n / (4.0 / 3.0 * np.pi * a ** 3)
    kappa = oracle.debye_kappa(lB, [dens / 2, dens / 2], [1.0, -1.0])
    c = oracle.Chain(s.xyz, s.q, s.sigma, s.R, lB, 3.0, seed=5)
    c.run(20)
    types, _ = s.types()
    bins = int(rmax / dr)
    C = np.zeros((2, 2, bins), np.uint64)
    Cc = np.zeros(2, np.uint64)
    for _ in range(150):
        c.run(2)
        cc, ce = oracle.rdf_counts(c.x, types, 2, s.R, rmax, bins)
        C += cc
        Cc += ce
    g, r = oracle.rdf_normalise(C, Cc, [n // 2, n // 2], [1.0, 1.0], s.R, rmax, bins)
    return dict(g=g, r=r, kappa=kappa, lB=lB, dens=dens, counts=C, dr=dr)


@pytest.mark.slow
def test_debye_hueckel_limit_of_g(oracle, dilute_run):
    """ln(g_{+-}/g_{++}) -> 2 l_B exp(-kappa (r - sigma)) / (r (1 + kappa sigma)).

    Dilute 1:1 system (phi = 0.001, R kappa = 8.3).  Fits the amplitude A of
    the DH form and the decay rate of r ln(g_{+-}/g_{++}); DH is the leading
    order, so A is allowed a band of O(l_B kappa) plus nonlinear corrections
    near contact.  A sign error gives A < 0, a wrong Bjerrum-length factor
    moves A by ~2x, and stale neighbour positions spoil the screening length.
    """
    g, r, kappa, lB = dilute_run["g"], dilute_run["r"], dilute_run["kappa"], dilute_run["lB"]
    sel = (r > 2.0) & (r < 12.0)
    lr = np.log(g[0, 1][sel] / g[0, 0][sel])
    dh = oracle.dh_log_ratio(r[sel], lB, kappa, 1.0)
    A = float(np.sum(lr * dh) / np.sum(dh * dh))
    assert 0.85 < A < 1.45, A
    sel2 = (r > 2.0) & (r < 9.0)
    y = np.log(r[sel2] * np.log(g[0, 1][sel2] / g[0, 0][sel2]))
    slope = np.polyfit(r[sel2], y, 1)[0]
    assert -slope == pytest.approx(kappa, rel=0.3), (-slope, kappa)


@pytest.mark.slow
def test_like_ion_symmetry_and_hard_core(oracle, dilute_run):
    """1:1 symmetry g_{++} = g_{--} within noise; bins below contact are exactly empty."""
    g, r, C = dilute_run["g"], dilute_run["r"], dilute_run["counts"]
    assert np.all(C[:, :, r + 0.5 * dilute_run["dr"] <= 1.0] == 0)
    sel = (r > 2.0) & (r < 15.0)
    d = g[0, 0][sel] - g[1, 1][sel]
    assert np.sqrt(np.mean(d ** 2)) < 0.03


@pytest.mark.slow
def test_screening_cloud_charge(oracle, dilute_run):
    """Charge of the screening cloud, Q(r) = 4 pi int_0^r s^2 rho^q(s) ds (Eq. (rho-g-g)).

    In the dilute limit the cloud around an ion of charge q follows the DH
    form Q(r) = -q [1 - (1 + kappa r) exp(-kappa (r - sigma)) / (1 + kappa sigma)],
    which tends to -q (electroneutrality).  Checked up to r ~ 1.3 Debye
    lengths, where the r^2 growth of the noise still leaves a sharp test;
    averaged over both centre species.
    """
    g, r, kappa, dens, dr = (dilute_run[k] for k in ("g", "r", "kappa", "dens", "dr"))
    rho_p = 0.5 * dens * (g[0, 0] - g[0, 1])
    rho_m = 0.5 * dens * (g[1, 1] - g[1, 0])
    Q = 0.5 * (np.cumsum(4 * np.pi * r ** 2 * rho_p * dr) + np.cumsum(4 * np.pi * r ** 2 * rho_m * dr))
    for rr in (5.0, 8.0, 10.0):
        k = int(round(rr / dr)) - 1
        edge = r[k] + 0.5 * dr
        dh = -(1.0 - (1 + kappa * edge) * np.exp(-kappa * (edge - 1.0)) / (1 + kappa))
        assert Q[k] == pytest.approx(dh, abs=0.08), (edge, Q[k], dh)
