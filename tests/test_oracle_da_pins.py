"""Pins of the oracle's delayed-acceptance (DA) stage against things other
than itself: hand-built neighbour histograms, closed-form networks, detailed
balance of the two-stage rule, the two-ion stationary density with a
deliberately bad surrogate, the plain chain when DA is off, and central finite
differences of the training gradient.

The two-stage rule (Christen and Fox 2005) is not in the paper; it keeps the
paper's exact chain (Sec. 2) as its second stage.
"""
import math

import numpy as np
import pytest


def _params(rng, scale=0.05):
    from oracle import oracle as O
    return O.bf16(rng.normal(0.0, scale, O.da_nparam()))


def test_features_hand_built(oracle):
    """Ion 0 at the origin (q = +1): like ions at r = 0.5 and 3.99, an unlike
    ion at 1.03, an unlike ion exactly at r = rc (excluded), a neutral ion."""
    x = np.array([[0, 0, 0], [0.5, 0, 0], [0, 1.03, 0], [0, 0, 3.99], [4.0, 0, 0], [0, 0, -2.0]], float)
    q = np.array([1.0, 1.0, -1.0, 1.0, -1.0, 0.0])
    f = oracle.da_features(x, q, 0, x[0], rc=4.0)
    want = np.zeros(128, np.int32)
    want[8] = 1          # r = 0.5:  0.5 / 0.0625 = 8
    want[63] = 1         # r = 3.99: 63.84
    want[64 + 16] = 1    # r = 1.03: 16.48, unlike
    assert np.array_equal(f, want)
    # at p = (0, 0, 1): ion 0 itself never counts; like at 1.118 (bin 17) and
    # 2.99 (bin 47), unlike at 1.4357 (bin 22); r = sqrt(17) > 4 excluded
    g = oracle.da_features(x, q, 0, np.array([0.0, 0.0, 1.0]), rc=4.0)
    want = np.zeros(128, np.int32)
    want[17] = 1
    want[47] = 1
    want[64 + 22] = 1
    assert np.array_equal(g, want)
    # the sign convention follows the moving ion's charge
    h = oracle.da_features(x, -q, 0, x[0], rc=4.0)
    assert np.array_equal(h, f)


def test_bf16_rounding_ties_to_even(oracle):
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 0.75 * 2 ** -7, -2.0 - 2 ** -7])
    want = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.0])
    assert np.array_equal(oracle.bf16(v), want)
    for a, b in zip(v, want):
        assert oracle.lib().orc_bf16_round(float(a)) == b


def test_network_closed_forms(oracle):
    """Identity layers: eps = sum(f) + b3; with b1 = -1 the ReLU cuts each
    count by one (eps = sum(max(f - 1, 0)) + b3)."""
    n = oracle.da_nparam()
    p = np.zeros(n)
    W1, b1, W2, b2, w3, _ = oracle.unpack_params(p)
    p = p.copy()
    o = 0
    p[o:o + 128 * 128] = np.eye(128).ravel(); o += 128 * 128
    o += 128
    p[o:o + 128 * 128] = np.eye(128).ravel(); o += 128 * 128
    o += 128
    p[o:o + 128] = 1.0; o += 128
    p[o] = 0.5
    rng = np.random.default_rng(3)
    f = rng.integers(0, 4, 128).astype(np.int32)
    assert oracle.mlp_eps(p, f) == float(f.sum()) + 0.5
    p[128 * 128:128 * 128 + 128] = -1.0
    assert oracle.mlp_eps(p, f) == float(np.maximum(f - 1, 0).sum()) + 0.5
    p[128 * 128:128 * 128 + 128] = 0.0
    o2 = 2 * 128 * 128 + 128
    p[o2:o2 + 128] = -2.0  # second layer's bias: eps = sum(max(f - 2, 0)) + b3
    assert oracle.mlp_eps(p, f) == float(np.maximum(f - 2, 0).sum()) + 0.5
    # and the vectorised forward agrees with the C network on random weights
    q = _params(rng)
    F = rng.integers(0, 3, (20, 128))
    out, _ = oracle.mlp_forward(q, F)
    for r in range(20):
        assert out[r] == pytest.approx(oracle.mlp_eps(q, F[r].astype(np.int32)), rel=1e-12, abs=1e-12)


def test_two_stage_detailed_balance_enumerated(oracle):
    """pi(x) a1 a2 (x -> y) = pi(y) a1 a2 (y -> x) for single-ion moves with a
    random (bad) surrogate: a1 = min(1, e^-dEh), a2 = min(1, e^-(dE - dEh)),
    dEh = l_B (eps(phi(y_k)) - eps(phi(x_k))) from the other ions' positions."""
    rng = np.random.default_rng(5)
    p = _params(rng, 0.2)
    n, lB = 6, 1.3
    q = np.array([1.0, -1.0, 1.0, -1.0, 2.0, -2.0])
    sig = np.full(n, 0.5)
    checked = 0
    for _ in range(300):
        x = rng.uniform(-2.5, 2.5, (n, 3))
        k = int(rng.integers(n))
        y = x.copy()
        y[k] = x[k] + rng.uniform(-0.8, 0.8, 3)
        dxy, ov1 = oracle.delta_energy(x, q, sig, k, y[k], lB)
        dyx, ov2 = oracle.delta_energy(y, q, sig, k, x[k], lB)
        d0 = np.linalg.norm(x[:, None] - x[None], axis=-1)[np.triu_indices(n, 1)].min()
        if ov1 or ov2 or d0 < 0.5:
            continue
        fx = oracle.da_features(x, q, k, x[k], 3.0)
        fy = oracle.da_features(x, q, k, y[k], 3.0)
        h_xy = lB * (oracle.mlp_eps(p, fy) - oracle.mlp_eps(p, fx))
        gx = oracle.da_features(y, q, k, y[k], 3.0)
        gy = oracle.da_features(y, q, k, x[k], 3.0)
        h_yx = lB * (oracle.mlp_eps(p, gy) - oracle.mlp_eps(p, gx))
        assert h_yx == -h_xy
        a_xy = min(1.0, math.exp(-h_xy)) * min(1.0, math.exp(-(dxy - h_xy)))
        a_yx = min(1.0, math.exp(-h_yx)) * min(1.0, math.exp(-(dyx - h_yx)))
        ex, ey = oracle.total_energy(x, q, lB), oracle.total_energy(y, q, lB)
        assert math.exp(-ex) * a_xy == pytest.approx(math.exp(-ey) * a_yx, rel=1e-11)
        checked += 1
    assert checked > 100


def test_da_off_is_the_plain_chain(oracle):
    """With DA off the DA chain makes exactly the plain chain's decisions."""
    from paper_1602_05716_amd import inputs
    sy = inputs.electrolyte(60, 60, 1.0, -1.0, 1.0, 1.0, 0.05, 0.9)
    sy.xyz = inputs.random_start(sy, 17)
    p = np.zeros(oracle.da_nparam())
    r = oracle.da_run(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, 1.5, 99, 3, 0, 3 * sy.n, p, band=2, da_on=0)
    ref = oracle.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, 1.5, seed=99, chain=3)
    t = ref.run(3, trace=3 * sy.n)
    assert np.array_equal(r["own"], t["acc"])
    assert np.array_equal(r["x"], ref.x)


def test_conflict_rule_hand_built(oracle):
    """Two 64-ion groups, band 1: ion 64 (first of group 1) is a conflict move
    when an ion of group 0 sits within rc; ion 65 also sees ion 64."""
    n = 128
    rng = np.random.default_rng(8)
    x = np.zeros((n, 3))
    # group 0 far away on a shell, group 1 near the origin, well separated
    for i in range(64):
        x[i] = [30.0 + 1.5 * (i % 8), 1.5 * (i // 8), 0.0]
    for i in range(64, n):
        x[i] = [1.5 * ((i - 64) % 8) - 40.0, 1.5 * ((i - 64) // 8), 0.0]
    x[0] = [-40.0, -3.0, 0.0]  # ion 0 within 3.0 of ion 64 at (-40, 0, 0)
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    sig = np.full(n, 1.0)
    p = np.zeros(oracle.da_nparam())
    r = oracle.da_run(x, q, sig, 80.0, 0.7, 0.01, 5, 0, 0, n, p, rc=4.0, band=1, da_on=1)
    conflict = (r["flags"] >> 2) & 1
    assert conflict[64] == 1          # ion 0 (group 0, pending for group 1) is near
    assert conflict[65] == 1          # ion 64 is near ion 65 (own group, lower index)
    r0 = oracle.da_run(x, q, sig, 80.0, 0.7, 0.01, 5, 0, 0, n, p, rc=4.0, band=0, da_on=1)
    c0 = (r0["flags"] >> 2) & 1
    assert c0[64] == 0                # with band 0 group 0 is decided
    assert c0[1] == 0                 # ion 0 is far from ion 1
    assert c0[2] == 1                 # ion 1 is 1.5 from ion 2, same group, lower index


def _two_ion_density(r, a, lB, q1q2):
    f = 3 * r ** 2 / a ** 3 * (1 - 3 * r / (4 * a) + r ** 3 / (16 * a ** 3))
    return f * np.exp(-lB * q1q2 / r)


@pytest.mark.slow
def test_da_chain_two_ion_density_with_bad_surrogate(oracle):
    """Two ions in the sphere under the DA chain with a random network: the
    distance density is still the ball-line-picking density times the
    Boltzmann factor (stage 2 corrects whatever stage 1 does)."""
    from scipy import integrate
    rng = np.random.default_rng(12)
    p = _params(rng, 0.3)
    R, sig, lB, q1q2 = 3.5, 1.0, 2.0, -1.0
    a = R - 0.5 * sig
    q = np.array([1.0, q1q2])
    rs = []
    stage1 = 0
    for sd in range(200, 212):
        x = np.array([[-1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
        x = oracle.da_run(x, q, [sig, sig], R, lB, 2.0, sd, 0, 0, 2 * 50, p, rc=2.0, band=0)["x"]
        for s in range(50, 6050, 3):
            r1 = oracle.da_run(x, q, [sig, sig], R, lB, 2.0, sd, 0, s, 6, p, rc=2.0, band=0)
            x = r1["x"]
            stage1 += int(np.sum((r1["flags"] >> 3) & 1))
            rs.append(np.linalg.norm(x[0] - x[1]))
    assert stage1 > 1000  # the surrogate does reject at stage 1
    r = np.array(rs)
    edges = np.linspace(sig, 2 * a, 13)
    norm = integrate.quad(_two_ion_density, sig, 2 * a, args=(a, lB, q1q2))[0]
    pr = np.array([integrate.quad(_two_ion_density, lo, hi, args=(a, lB, q1q2))[0]
                   for lo, hi in zip(edges[:-1], edges[1:])]) / norm
    h, _ = np.histogram(r, edges)
    expect = pr * len(r)
    chi2 = float(np.sum((h - expect) ** 2 / expect))
    assert chi2 < 45.0, (chi2, h, expect)


def test_backprop_matches_central_differences(oracle):
    """Gradient of the training loss by backpropagation against central
    finite differences (without the bfloat16 rounding of the activations,
    which makes the loss piecewise constant at the scale of its ulp)."""
    rng = np.random.default_rng(21)
    p = rng.normal(0.0, 0.1, oracle.da_nparam())
    Xo = rng.integers(0, 3, (16, 128)).astype(float)
    Xn = rng.integers(0, 3, (16, 128)).astype(float)
    y = rng.normal(0.0, 1.0, 16)
    loss, g = oracle.mlp_loss_grad(p, Xo, Xn, y, rounding=False)
    idx = np.concatenate([rng.choice(128 * 128, 40, replace=False),
                          128 * 128 + np.arange(0, 128, 16),
                          128 * 128 + 128 + rng.choice(128 * 128, 40, replace=False),
                          [len(p) - 1 - k for k in range(0, 129, 8)]])
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (oracle.mlp_loss_grad(pp, Xo, Xn, y, rounding=False)[0] -
              oracle.mlp_loss_grad(pm, Xo, Xn, y, rounding=False)[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-8), k
    assert loss > 0


@pytest.mark.parametrize("band,n,R", [(1, 192, 8.0), (2, 192, 8.0), (3, 256, 8.8)])
def test_conflict_rule_keeps_independent_ions_uniform(oracle, band, n, R):
    """Exactness of the conflict rule at band >= 1, independent of how the
    rule is tiled: point ions (sigma 1e-3) with l_B = 1e-6 are, to 1e-5 in
    the Boltzmann factor, independent and uniform in the ball, so g_ab = 1 at
    every r (the closed form pinned for the estimator above).  The network's
    output layer is scaled by 1/l_B so that stage 1 rejects freely
    (dEh of order 1 kT); a conflict rule that depends on which of the two
    positions {x_i, x~_i} is the current one leaves the chain with a
    different stationary law (measured: g about 0.5 below rc)."""
    rng = np.random.default_rng(5)
    lB, rc, sig = 1e-6, 1.0, 1e-3
    p = _params(rng, 0.3)
    w3 = len(p) - 129
    p[w3:w3 + 128] = oracle.bf16(p[w3:w3 + 128] / lB)
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    types = (np.arange(n) % 2).astype(np.int32)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    x = v * ((R - 0.5 * sig) * rng.uniform(size=n) ** (1.0 / 3.0))[:, None]
    sweeps = 400
    r = oracle.da_run(x, q, np.full(n, sig), R, lB, 2.0, 8, 0, 0, n * sweeps, p, rc=rc, band=band,
                      snapshots=True)
    fl = r["flags"]
    conflict = ((fl >> 2) & 1).mean()
    stage1_rej = ((fl >> 3) & 1).mean()
    assert 0.15 < conflict < 0.85 and stage1_rej * len(fl) > 500, (conflict, stage1_rej)
    bins = 4
    C = np.zeros((2, 2, bins), np.uint64)
    ce = np.zeros(2, np.uint64)
    for s in r["snapshots"][10:]:
        c, cc = oracle.rdf_counts(s, types, 2, R, rc, bins)
        C += c
        ce += cc
    # pooled over the shells r >= rc / 4 (bin 0 holds few pairs)
    Cp = C[:, :, 1:].sum(axis=2).astype(float)
    dr = rc / bins
    vol = 4.0 / 3.0 * np.pi * ((bins * dr) ** 3 - dr ** 3)
    for a in range(2):
        for b in range(2):
            nb = (n // 2 - (1 if a == b else 0)) / (4.0 / 3.0 * np.pi * (R - 0.5 * sig) ** 3)
            g = Cp[a, b] / (float(ce[a]) * nb * vol)
            assert abs(g - 1.0) < 0.12, (band, a, b, g, Cp[a, b])
