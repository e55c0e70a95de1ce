"""CPU pins of the renormalised-parameter analysis (Sec. 5.1: kappa_R from
the tails of r rho_a, q^R two ways from U / rho, eps_R two ways, and the
dressed-ion relation (kappa_R / kappa)^2 = (q_+^R - q_-^R) / (q_+ - q_-)).

Pinned against closed forms, not against itself:
  * a synthetic far field in the dressed-ion form with chosen kappa_R, q^R,
    eps_R (kappa_R fixed by the relation, which makes the linear charge
    density consistent), including a bulk-plateau offset of g;
  * the linearised Debye-Hueckel limit with a hard core a, whose dressed-ion
    form is kappa_R = kappa, q^R = q, eps_R / eps = (1 + kappa a) exp(-kappa a)
    (Debye-Hueckel potential q exp(kappa a) exp(-kappa r) / ((1 + kappa a) r)).
"""
import numpy as np
import pytest

from paper_1602_05716_amd import analysis


def _grid(rmax=80.0, bins=1600):
    dr = rmax / bins
    return (np.arange(bins) + 0.5) * dr


def _g_from_u(U, r, core=1.0, plateau=(1.0, 1.0)):
    """g[a, b] (centre a, neighbour b) = c_b exp(-U_ab): the plateau c_b is
    the bulk density of b over the density g is normalised by."""
    g = np.exp(-U) * np.asarray(plateau)[None, :, None]
    g[..., r < core] = 0.0
    return g


def _dressed_case(plateau=(1.02, 1.01)):
    """3:-1 at the paper's bare Debye length (3.8 diameters), its measured
    q^R = 4.125 / -0.884, and an arbitrary eps_R / eps = 1.25."""
    lB = 7.117 / 7.5
    q = np.array([3.0, -1.0])
    n_bulk = np.array([4.83e-4, 1.449e-3])
    qR = np.array([4.125, -0.884])
    epsr = 1.25
    kR = np.sqrt(4 * np.pi * lB * np.sum(n_bulk * q * qR))
    r = _grid()
    U = np.array([[lB / epsr * qR[a] * qR[b] * np.exp(-kR * r) / r for b in range(2)] for a in range(2)])
    g = _g_from_u(U, r, plateau=plateau)
    return r, g, n_bulk / np.asarray(plateau), q, lB, qR, epsr, kR


def test_dressed_ion_far_field_is_recovered():
    r, g, n, q, lB, qR, epsr, kR = _dressed_case()
    res = analysis.renormalised_parameters(r, g, n, q, lB, fit=(22.0, 38.0), r_flat=70.0)
    assert abs(res["kappa"] - analysis.bare_kappa(lB, n * np.array([1.02, 1.01]), q)) < 1e-9
    assert np.allclose(res["g_inf"], [[1.02, 1.01], [1.02, 1.01]], rtol=1e-9)
    assert abs(res["kappa_R"] / kR - 1) < 1e-4
    for k in range(2):  # both centres give the same slope
        assert abs(res["kappa_R_by_centre"][k] / kR - 1) < 1e-4
    for way in range(2):  # q^R two ways
        assert abs(res["qR_plus"][way] / qR[0] - 1) < 1e-3
        assert abs(res["qR_minus"][way] / qR[1] - 1) < 1e-3
    for a in range(2):  # eps_R two ways
        assert abs(res["epsR_over_eps"][a] / epsr - 1) < 1e-3
    assert abs(res["rd_lhs"] - res["rd_rhs"]) < 1e-3 * res["rd_lhs"]
    # the bare / renormalised Debye lengths in Angstrom (diameter 7.5 A)
    assert abs(7.5 / res["kappa"] - 28.53) < 0.05
    assert abs(7.5 / res["kappa_R"] - 7.5 / kR) < 0.05


def test_far_window_converges():
    """The nonlinear part of rho (from exp(-U) - 1 + U) decays as exp(-2
    kappa_R r): the estimate improves as the window moves out."""
    r, g, n, q, lB, qR, epsr, kR = _dressed_case(plateau=(1.0, 1.0))
    errs = []
    for lo in (8.0, 14.0, 22.0):
        res = analysis.renormalised_parameters(r, g, n, q, lB, fit=(lo, lo + 12.0), g_inf=np.ones((2, 2)))
        errs.append(abs(res["qR_plus"][0] / qR[0] - 1))
    assert errs[0] > errs[1] > errs[2]


def test_debye_hueckel_limit():
    lB, a = 0.7, 1.0
    q = np.array([1.0, -1.0])
    n = np.array([1e-3, 1e-3])
    kappa = analysis.bare_kappa(lB, n, q)
    r = _grid(60.0, 1200)
    U = np.array([[lB * q[i] * q[j] * np.exp(kappa * a) / (1 + kappa * a) * np.exp(-kappa * r) / r
                   for j in range(2)] for i in range(2)])
    g = _g_from_u(U, r, core=a)
    res = analysis.renormalised_parameters(r, g, n, q, lB, fit=(12.0, 40.0), g_inf=np.ones((2, 2)))
    # symmetric 1:1: rho_+ = -2 n sinh(U), so only the cubic term U^3 / 6
    # (U < 7e-3 in the window) separates it from the linear form
    assert abs(res["kappa_R"] / kappa - 1) < 1e-4
    assert np.allclose(res["qR_plus"], 1.0, rtol=1e-4) and np.allclose(res["qR_minus"], -1.0, rtol=1e-4)
    assert np.allclose(res["epsR_over_eps"], (1 + kappa * a) * np.exp(-kappa * a), rtol=1e-4)
    assert abs(res["rd_lhs"] - 1) < 1e-4 and abs(res["rd_rhs"] - 1) < 1e-4


def test_noisy_tail_within_statistical_error():
    """Seeded Gaussian noise of 2e-6 on g (a long run's per-bin error): the
    estimates stay within a few per cent."""
    r, g, n, q, lB, qR, epsr, kR = _dressed_case()
    rng = np.random.default_rng(7)
    g = g + rng.normal(0.0, 2e-6, g.shape) * (g > 0)
    res = analysis.renormalised_parameters(r, g, n, q, lB, fit=(14.0, 26.0), r_flat=60.0)
    assert abs(res["kappa_R"] / kR - 1) < 0.02
    assert abs(np.mean(res["qR"][0]) / qR[0] - 1) < 0.05
    assert abs(res["qR"][1] / qR[1] - 1) < 0.05


def test_rejects_bad_windows():
    r, g, n, q, lB, *_ = _dressed_case()
    with pytest.raises(ValueError):
        analysis.renormalised_parameters(r, g, n, q, lB, fit=(30.0, 30.1))
    with pytest.raises(ValueError):
        analysis.renormalised_parameters(r, g, n, q[::-1], lB, fit=(20.0, 30.0))


def test_weighted_fit_recovers_the_noiseless_far_field():
    """The fit of rho itself (used with errors) and the fit of its log agree
    with the dressed-ion values on noiseless data."""
    r, g, n, q, lB, qR, epsr, kR = _dressed_case()
    kw = dict(fit=(22.0, 38.0), r_flat=70.0)
    a = analysis.renormalised_parameters(r, g, n, q, lB, **kw)
    b = analysis.renormalised_parameters(r, g, n, q, lB, rho_err=1e-3 * np.abs(a["rho"]), **kw)
    for res in (a, b):
        assert abs(res["kappa_R"] / kR - 1) < 1e-4
        assert np.allclose(res["kappa_R_by_centre"], kR, rtol=1e-4)
        assert abs(res["qR"][0] / qR[0] - 1) < 1e-3 and abs(res["qR"][1] / qR[1] - 1) < 1e-3
        assert np.allclose(res["epsR_over_eps"], epsr, rtol=1e-3)


def test_weighted_fit_with_counting_noise():
    """Pair counts drawn from Poisson laws around a dressed-ion g (seeded):
    the fit weighted by the counts' errors recovers kappa_R and q^R over a
    window whose far end is noise-dominated."""
    r, g, n, q, lB, qR, epsr, kR = _dressed_case(plateau=(1.0, 1.0))
    dr = r[1] - r[0]
    vk = 4.0 / 3.0 * np.pi * ((r + dr / 2) ** 3 - (r - dr / 2) ** 3)
    centres = np.array([4e7, 1.2e8])
    mean = g * centres[:, None, None] * n[None, :, None] * vk[None, None, :]
    rng = np.random.default_rng(11)
    C = rng.poisson(mean).astype(np.float64)
    gn = C / (centres[:, None, None] * n[None, :, None] * vk[None, None, :])
    err = analysis.charge_density_error(C, gn, n, q)
    # the window starts where the nonlinear part of rho (exp(-U) - 1 + U,
    # about U_++ / 2 of it: 3 % at r = 10) has mostly died out
    fit = (10.0, 30.0)
    wres = analysis.renormalised_parameters(r, gn, n, q, lB, fit=fit, g_inf=np.ones((2, 2)), rho_err=err)
    assert abs(wres["kappa_R"] / kR - 1) < 0.03
    assert abs(wres["qR"][0] / qR[0] - 1) < 0.05 and abs(wres["qR"][1] / qR[1] - 1) < 0.05
    # far bins of rho_- change sign with this much noise: the log fit cannot take the window
    with pytest.raises(ValueError):
        analysis.renormalised_parameters(r, gn, n, q, lB, fit=fit, g_inf=np.ones((2, 2)))
