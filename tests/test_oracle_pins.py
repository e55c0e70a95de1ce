"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Paper: Liang, Xing, Li, arXiv:1602.05716.  Each test names the passage or the
mathematical fact it pins and the kind of mistake it would catch.
"""
import math
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


# --------------------------------------------------------------------------- #
# Philox4x32-10 against an independent implementation                         #
# --------------------------------------------------------------------------- #

def _torch_philox_ref():
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    src = os.path.join(ROOT, "tests", "helpers", "philox_torch_ref.cpp")
    exe = os.path.join("/tmp", "philox_torch_ref_%d" % os.getpid())
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", inc, "-o", exe, src])
    return exe


def test_philox_matches_torch_engine(oracle):
    """Philox4x32-10 (Salmon et al., SC'11) vs PyTorch's header-only engine.

    Pins every constant, the round structure and the key schedule: a wrong
    multiplier, Weyl constant, word order or round count changes all outputs.
    """
    exe = _torch_philox_ref()
    rng = np.random.default_rng(7)
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 0, 1, 0, 0]]
    rows += rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64).tolist()
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    os.unlink(exe)
    ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()], np.uint64)
    assert ref.shape == (len(rows), 4)
    for r, expect in zip(rows, ref):
        got = oracle.philox(r[:4], r[4:])
        assert got.tolist() == expect.tolist(), r


def test_philox_matches_rocrand_rounds(oracle):
    """The same blocks against a second independent implementation: the ten
    rounds of rocRAND's header-only Philox4x32-10 engine, built for the host
    with hipcc.  Unlike a stream interface it takes any 128-bit counter."""
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not installed")
    src = os.path.join(ROOT, "tests", "helpers", "philox_rocrand_ref.cpp")
    exe = os.path.join("/tmp", "philox_rocrand_ref_%d" % os.getpid())
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-o", exe, src])
    rng = np.random.default_rng(8)
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [0, 0, 0, 0xFFFFFFFF, 1, 0]]
    rows += rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64).tolist()
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    os.unlink(exe)
    ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()], np.uint64)
    assert ref.shape == (len(rows), 4)
    for r, expect in zip(rows, ref):
        assert oracle.philox(r[:4], r[4:]).tolist() == expect.tolist(), r


def test_move_words_counter_layout(oracle):
    """Move (ion i, sweep s, chain c) uses counter (i, s, c, tag), key = seed words."""
    seed = 0x0123456789ABCDEF
    w = oracle.move_words(seed, 5, 17, 42, 0)
    ref = oracle.philox([42, 17, 5, 0], [0x89ABCDEF, 0x01234567])
    assert w.tolist() == ref.tolist()


# --------------------------------------------------------------------------- #
# Energy                                                                      #
# --------------------------------------------------------------------------- #

def _load_golden(name):
    path = os.path.join(GOLDEN, name)
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.rsplit("=", 1)
                vals[k.strip()] = v.strip()
    return vals


def test_two_ion_energy_closed_form(oracle):
    """Bare pair potential U_12 = l_B q1 q2 / r (Sec. 5.1 with kappa -> 0).

    A 3-4-5 triangle makes r exactly 5; the values are fixed in the golden file.
    """
    g = _load_golden("two_ion_energy.txt")
    xyz = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    for lB, q1, q2 in [(0.7, 1.0, -1.0), (7.117, 3.0, -1.0), (2.0, 2.0, 2.0)]:
        key = "E(lB=%g,q1=%g,q2=%g)" % (lB, q1, q2)
        expect = float(g[key])
        got = oracle.total_energy(xyz, [q1, q2], lB)
        assert got == pytest.approx(expect, rel=1e-15, abs=0), key


def test_rocksalt_cube_energy(oracle):
    """Eight alternating charges on the corners of a cube of edge a.

    Closed form: E = (l_B / a) (-12 + 12/sqrt(2) - 4/sqrt(3)) (12 unlike
    edges, 12 like face diagonals, 4 unlike body diagonals).  A dropped or
    double-counted pair, a sign error or a self term fails it.
    """
    g = _load_golden("rocksalt_cube.txt")
    a, lB = float(g["a"]), float(g["lB"])
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float)
    q = np.array([(-1.0) ** (i + j + k) for i, j, k in corners.astype(int)])
    xyz = corners * a + np.array([0.1, -0.2, 0.3])
    assert oracle.total_energy(xyz, q, lB) == pytest.approx(float(g["E"]), rel=1e-13)


def _random_system(n, seed, R=8.0, sig=(1.0, 0.8)):
    from paper_1602_05716_amd import inputs
    nc = n // 3
    s = inputs.electrolyte(nc, n - nc, 2.0, -1.0, sig[0], sig[1], 0.05, 0.9)
    s.R = R
    s.xyz = inputs.random_start(s, seed)
    return s


def test_delta_energy_is_energy_difference(oracle):
    """Eq. (Delta E_ij): the per-move sum equals E(after) - E(before).

    Both sides come from different oracle loops (per-move sum over j != i vs
    the full pair sum), so a wrong index, a missing self-exclusion, a sign or
    a factor of two in either fails.  2:1 charges and two diameters.
    """
    s = _random_system(120, 3)
    rng = np.random.default_rng(11)
    e0 = oracle.total_energy(s.xyz, s.q, s.lB)
    for _ in range(60):
        i = int(rng.integers(s.n))
        xt = s.xyz[i] + rng.uniform(-0.7, 0.7, 3)
        dE, _ = oracle.delta_energy(s.xyz, s.q, s.sigma, i, xt, s.lB)
        y = s.xyz.copy()
        y[i] = xt
        e1 = oracle.total_energy(y, s.q, s.lB)
        assert dE == pytest.approx(e1 - e0, rel=1e-9, abs=1e-11)


def test_overlap_rule_additive_diameters(oracle):
    """Hard core: overlap iff r < (sigma_i + sigma_j)/2; contact is allowed."""
    xyz = np.array([[0.0, 0.0, 0.0], [5.0, 0.0, 0.0]])
    q = np.array([1.0, -1.0])
    sig = np.array([1.0, 0.5])
    contact = 0.75
    _, ov = oracle.delta_energy(xyz, q, sig, 1, [contact, 0.0, 0.0], 0.7)
    assert not ov
    _, ov = oracle.delta_energy(xyz, q, sig, 1, [np.nextafter(contact, 0.0), 0.0, 0.0], 0.7)
    assert ov
    _, ov = oracle.delta_energy(xyz, q, sig, 0, [4.3, 0.0, 0.0], 0.7)
    assert ov


def test_wall_rule(oracle):
    """Hard wall (Sec. 5.2): the ion surface may touch but not cross radius R."""
    R, sig = 10.0, 0.8
    a = R - 0.5 * sig
    assert oracle.lib().orc_outside_wall(np.array([a, 0.0, 0.0]).ctypes.data_as(
        oracle._f64p), R, sig) == 0
    assert oracle.lib().orc_outside_wall(np.array([np.nextafter(a, 20.0), 0.0, 0.0]).ctypes.data_as(
        oracle._f64p), R, sig) == 1


def test_detailed_balance_enumerated(oracle):
    """pi(x) alpha(x->y) = pi(y) alpha(y->x) for single-ion moves (Sec. 2).

    alpha = min(1, exp(-dE)) with dE from the per-move sum and pi = exp(-E)
    from the total energy; checks that the two agree in sign and size.
    """
    s = _random_system(3, 5, R=3.0, sig=(1.0, 1.0))
    rng = np.random.default_rng(2)
    for _ in range(200):
        k = int(rng.integers(3))
        x = s.xyz
        y = x.copy()
        y[k] = x[k] + rng.uniform(-0.5, 0.5, 3)
        dxy, ov1 = oracle.delta_energy(x, s.q, s.sigma, k, y[k], s.lB)
        dyx, ov2 = oracle.delta_energy(y, s.q, s.sigma, k, x[k], s.lB)
        if ov1:
            continue
        ex, ey = oracle.total_energy(x, s.q, s.lB), oracle.total_energy(y, s.q, s.lB)
        lhs = math.exp(-ex) * min(1.0, math.exp(-dxy))
        rhs = math.exp(-ey) * min(1.0, math.exp(-dyx))
        assert lhs == pytest.approx(rhs, rel=1e-12)


# --------------------------------------------------------------------------- #
# The chain: stationary distributions with closed forms                       #
# --------------------------------------------------------------------------- #

def _collect(oracle, xyz, q, sig, R, lB, D, seeds, sweeps, burn, fn):
    out = []
    for sd in seeds:
        c = oracle.Chain(xyz, q, sig, R, lB, D, seed=sd)
        c.run(burn)
        for _ in range(sweeps):
            c.run(1)
            out.append(fn(c.x))
    return np.array(out)


def test_one_ion_uniform_in_ball(oracle):
    """A lone ion samples the ball |x| <= R - sigma/2 uniformly.

    P(|x| <= r) = (r/a)^3.  Pins the wall radius (a, not R), the symmetric
    cube move and the acceptance of dE = 0 moves.
    """
    from scipy import stats
    R, sig = 5.5, 1.0
    a = R - 0.5 * sig
    r = _collect(oracle, [[0.0, 0.0, 0.0]], [0.0], [sig], R, 0.7, 3.0,
                 seeds=range(8), sweeps=4000, burn=50,
                 fn=lambda x: np.linalg.norm(x[0]))[::4]
    u = (r / a) ** 3
    assert u.max() <= 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert np.mean(r ** 2) == pytest.approx(3.0 * a * a / 5.0, rel=0.03)


def _two_ion_density(r, a, lB, q1q2):
    """Distance density of two uniform points in a ball of radius a ("ball line
    picking"), f(r) = 3 r^2/a^3 (1 - 3r/(4a) + r^3/(16 a^3)), times the
    Boltzmann factor of the bare pair potential."""
    f = 3 * r ** 2 / a ** 3 * (1 - 3 * r / (4 * a) + r ** 3 / (16 * a ** 3))
    return f * np.exp(-lB * q1q2 / r)


@pytest.mark.parametrize("q1q2,lB", [(-1.0, 2.0), (1.0, 2.0), (-1.0, 0.0)])
def test_two_ion_distance_distribution(oracle, q1q2, lB):
    """Two ions in the sphere: p(r) ~ ball-line-picking density x exp(-l_B q1 q2 / r)
    on [sigma, 2a].  Pins the energy sign, the Bjerrum-length scaling, the
    hard core and the wall together (chi-square on 12 bins)."""
    from scipy import integrate
    R, sig = 3.5, 1.0
    a = R - 0.5 * sig
    q = [1.0, q1q2]
    xyz = [[-1.0, 0.0, 0.0], [1.0, 0.0, 0.0]]
    r = _collect(oracle, xyz, q, [sig, sig], R, lB, 2.0, seeds=range(100, 112),
                 sweeps=6000, burn=50, fn=lambda x: np.linalg.norm(x[0] - x[1]))[::3]
    edges = np.linspace(sig, 2 * a, 13)
    norm = integrate.quad(_two_ion_density, sig, 2 * a, args=(a, lB, q1q2))[0]
    p = np.array([integrate.quad(_two_ion_density, lo, hi, args=(a, lB, q1q2))[0]
                  for lo, hi in zip(edges[:-1], edges[1:])]) / norm
    h, _ = np.histogram(r, edges)
    assert h.sum() == len(r)
    expect = p * len(r)
    chi2 = float(np.sum((h - expect) ** 2 / expect))
    # 11 dof; thinning leaves mild correlation, so allow a generous bound
    assert chi2 < 45.0, (chi2, h, expect)


def test_three_ion_mean_energy_vs_quadrature(oracle):
    """<E> of a 3-ion system vs a non-Markov estimate.

    The estimate weights i.i.d. uniform configurations in the ball by
    exp(-E) (zero for overlap); the chain must agree within combined
    statistical errors.
    """
    R, sig, lB = 3.0, 1.0, 1.0
    a = R - 0.5 * sig
    q = np.array([2.0, -1.0, -1.0])
    rng = np.random.default_rng(99)
    m = 1_500_000
    v = rng.normal(size=(m, 3, 3))
    v /= np.linalg.norm(v, axis=2)[:, :, None]
    pts = v * (a * rng.random((m, 3)) ** (1 / 3))[:, :, None]
    e = np.zeros(m)
    ok = np.ones(m, bool)
    for i, j in [(0, 1), (0, 2), (1, 2)]:
        r = np.linalg.norm(pts[:, i] - pts[:, j], axis=1)
        ok &= r >= sig
        e += lB * q[i] * q[j] / np.where(r > 0, r, 1.0)
    w = np.where(ok, np.exp(-(e - e[ok].min())), 0.0)
    e_q = float(np.sum(w * e) / np.sum(w))
    # error of the ratio estimator (delta method)
    wn = w / w.sum()
    err_q = float(np.sqrt(np.sum(wn ** 2 * (e - e_q) ** 2)))

    xyz = [[-1.5, 0.0, 0.0], [0.0, 0.0, 0.0], [1.5, 0.0, 0.0]]
    series = []
    for sd in range(16):
        c = oracle.Chain(xyz, q, [sig] * 3, R, lB, 1.6, seed=1000 + sd)
        c.run(100)
        res = c.run(8000, series=True)
        series.append(res["e_series"])
    series = np.array(series)
    means = series.reshape(16 * 8, -1).mean(axis=1)  # batch means
    e_c = float(means.mean())
    err_c = float(means.std(ddof=1) / np.sqrt(len(means)))
    assert abs(e_c - e_q) < 4.0 * math.hypot(err_c, err_q), (e_c, e_q, err_c, err_q)


# --------------------------------------------------------------------------- #
# Bookkeeping invariants                                                      #
# --------------------------------------------------------------------------- #

def test_running_energy_matches_resum(oracle):
    """E_run (sum of accepted dE) equals the FP64 re-sum after 200 sweeps."""
    from paper_1602_05716_amd import inputs
    s = inputs.electrolyte(100, 100, 1.0, -1.0, 1.0, 1.0, 0.05, 1.5)
    s.xyz = inputs.random_start(s, 1)
    c = oracle.Chain(s.xyz, s.q, s.sigma, s.R, s.lB, 1.0, seed=9)
    c.run(200)
    e = oracle.total_energy(c.x, s.q, s.lB)
    assert c.e_run == pytest.approx(e, rel=1e-11, abs=1e-11)


def test_resume_is_bit_exact(oracle):
    """Counter-based random numbers: 20 sweeps == 10 sweeps + 10 sweeps."""
    from paper_1602_05716_amd import inputs
    s = inputs.electrolyte(60, 60, 1.0, -1.0, 1.0, 1.0, 0.03, 0.7)
    s.xyz = inputs.random_start(s, 2)
    a = oracle.Chain(s.xyz, s.q, s.sigma, s.R, s.lB, 1.0, seed=77)
    ra = a.run(20, trace=2400)
    b = oracle.Chain(s.xyz, s.q, s.sigma, s.R, s.lB, 1.0, seed=77)
    rb1 = b.run(10, trace=1200)
    b2 = oracle.Chain(b.x, s.q, s.sigma, s.R, s.lB, 1.0, seed=77, sweep=10)
    b2.e_run = b.e_run
    rb2 = b2.run(10, trace=1200)
    assert np.array_equal(a.x, b2.x)
    assert np.array_equal(ra["acc"], np.concatenate([rb1["acc"], rb2["acc"]]))
    assert a.e_run == b2.e_run


def test_sequential_order_and_move_formula(oracle):
    """One sweep tries ions 0..N-1 in order with x~ = x + D (u - 1/2) (Algorithm 1).

    Rebuilt here move by move from the oracle's single-move primitives; a
    chain that visits ions out of order, reuses counters or mixes Philox
    words fails.
    """
    from paper_1602_05716_amd import inputs
    s = inputs.electrolyte(20, 20, 1.0, -1.0, 1.0, 1.0, 0.05, 0.7)
    s.xyz = inputs.random_start(s, 4)
    D, seed = 1.3, 31
    c = oracle.Chain(s.xyz, s.q, s.sigma, s.R, s.lB, D, seed=seed, chain=3, sweep=5)
    res = c.run(2, trace=80)
    x = s.xyz.copy()
    m = 0
    for sweep in (5, 6):
        for i in range(s.n):
            w = oracle.move_words(seed, 3, sweep, i)
            u = w.astype(np.float64) * 2.0 ** -32
            xt = x[i] + D * (u[:3] - 0.5)
            dE, ov = oracle.delta_energy(x, s.q, s.sigma, i, xt, s.lB)
            wall = np.dot(xt, xt) > (s.R - 0.5 * s.sigma[i]) ** 2
            acc = (not wall) and (not ov) and (dE <= 0 or u[3] < math.exp(-dE))
            assert bool(res["acc"][m]) == acc
            if acc:
                x[i] = xt
            m += 1
    assert np.array_equal(x, c.x)


def test_replay_f32_follows_given_trajectory(oracle):
    """The float-state replay reproduces its own decisions and energy change."""
    from paper_1602_05716_amd import inputs
    s = inputs.electrolyte(50, 50, 1.0, -1.0, 1.0, 1.0, 0.05, 0.7)
    s.xyz = inputs.random_start(s, 6)
    x32 = s.xyz.astype(np.float32)
    r1 = oracle.replay_f32(x32, s.q, s.sigma, s.R, s.lB, 1.0, 5, 0, 0, 300)
    r2 = oracle.replay_f32(x32, s.q, s.sigma, s.R, s.lB, 1.0, 5, 0, 0, 300, acc_given=r1["own"])
    assert r2["mismatches"] == 0 and np.array_equal(r1["xyz"], r2["xyz"])
    e0 = oracle.total_energy(x32.astype(np.float64), s.q, s.lB)
    e1 = oracle.total_energy(r1["xyz"].astype(np.float64), s.q, s.lB)
    assert e1 - e0 == pytest.approx(float(np.sum(r1["dE"][r1["own"] == 1])), rel=1e-9, abs=1e-10)
    flipped = r1["own"].copy()
    flipped[7] ^= 1
    assert oracle.replay_f32(x32, s.q, s.sigma, s.R, s.lB, 1.0, 5, 0, 0, 300,
                             acc_given=flipped)["mismatches"] >= 1


# --------------------------------------------------------------------------- #
# Pair correlation counts                                                     #
# --------------------------------------------------------------------------- #

def test_rdf_counts_brute_force(oracle):
    """Integer g(r) counts vs a pure-Python loop over ordered pairs."""
    rng = np.random.default_rng(3)
    n, R, rmax, bins = 40, 6.0, 3.0, 12
    xyz = rng.uniform(-3.5, 3.5, (n, 3))
    types = rng.integers(0, 2, n).astype(np.int32)
    counts, centres = oracle.rdf_counts(xyz, types, 2, R, rmax, bins)
    ref = np.zeros((2, 2, bins), np.uint64)
    refc = np.zeros(2, np.uint64)
    for i in range(n):
        if math.sqrt(sum(v * v for v in xyz[i])) > R - rmax:
            continue
        refc[types[i]] += 1
        for j in range(n):
            if j != i:
                r = math.dist(xyz[i], xyz[j])
                if r < rmax:
                    ref[types[i], types[j], int(r // (rmax / bins))] += 1
    assert np.array_equal(counts, ref) and np.array_equal(centres, refc)


def test_rdf_pair_symmetry_when_every_ion_is_a_centre(oracle):
    """With all ions as centres, C_ab(k) == C_ba(k) exactly (ordered pairs)."""
    rng = np.random.default_rng(4)
    xyz = rng.uniform(-2, 2, (80, 3))
    types = rng.integers(0, 3, 80).astype(np.int32)
    counts, centres = oracle.rdf_counts(xyz, types, 3, 100.0, 5.0, 25)
    assert centres.sum() == 80
    assert np.array_equal(counts, counts.transpose(1, 0, 2))


# --------------------------------------------------------------------------- #
# Autocorrelation time                                                        #
# --------------------------------------------------------------------------- #

def _ar1(rho, n, seed):
    from scipy.signal import lfilter
    return lfilter([1.0], [1.0, -rho], np.random.default_rng(seed).normal(size=n))


@pytest.mark.parametrize("rho", [-0.6, -0.3, 0.0, 0.5, 0.8])
def test_tau_int_on_ar1(oracle, rho):
    """AR(1) with coefficient rho has C_k = rho^k, so T_c = (1 + rho) / (2 (1 - rho))
    under T_c = 1/2 + sum_k C_k (Sec. 5.2), for negative rho as well."""
    x = _ar1(rho, 200_000, 12)
    expect = (1 + rho) / (2 * (1 - rho))
    assert oracle.tau_int(x) == pytest.approx(expect, rel=0.06, abs=0.01)
    assert oracle.ess(x) == pytest.approx(len(x) / (2 * oracle.tau_int(x)), rel=1e-15)


def test_tau_int_of_a_moving_average(oracle):
    """x_t = e_t + e_{t-1} has C_1 = 1/2 and C_k = 0 beyond, so T_c = 1
    exactly; the estimate must not pick up the noise of the empty lags."""
    e = np.random.default_rng(13).normal(size=400_001)
    x = e[1:] + e[:-1]
    assert oracle.tau_int(x) == pytest.approx(1.0, abs=0.02)
    assert math.isnan(oracle.tau_int(np.full(50, 3.0)))


# --------------------------------------------------------------------------- #
# g(r) normalisation                                                          #
# --------------------------------------------------------------------------- #

def _uniform_ball_counts(n_of_type, a_of_type, R, rmax, bins, samples, seed):
    """Counts of the Sec. 5.2 estimator (centres |x| <= R - rmax, ordered
    pairs) over i.i.d. configurations: every ion of type b uniform in the
    ball of radius a_b, independently of all others (no hard core)."""
    rng = np.random.default_rng(seed)
    types = np.concatenate([np.full(nb, b) for b, nb in enumerate(n_of_type)])
    nt, n = len(n_of_type), len(types)
    radii = np.array([a_of_type[t] for t in types])
    counts = np.zeros((nt, nt, bins), np.int64)
    centres = np.zeros(nt, np.int64)
    chunk = 4000
    for s0 in range(0, samples, chunk):
        m = min(chunk, samples - s0)
        v = rng.normal(size=(m, n, 3))
        v /= np.sqrt(np.einsum("mnk,mnk->mn", v, v))[..., None]
        x = v * (radii * rng.uniform(size=(m, n)) ** (1.0 / 3.0))[..., None]
        cen = np.einsum("mnk,mnk->mn", x, x) <= (R - rmax) ** 2
        d = np.zeros((m, n, n))
        for c in range(3):
            d += (x[:, :, None, c] - x[:, None, :, c]) ** 2
        d = np.sqrt(d)
        k = np.floor(d / (rmax / bins)).astype(np.int64)
        ok = cen[:, :, None] & (d < rmax) & ~np.eye(n, dtype=bool)[None]
        pair_type = (types[:, None] * nt + types[None, :]) * bins
        idx = (pair_type[None] + np.minimum(k, bins - 1))[ok]
        counts += np.bincount(idx, minlength=nt * nt * bins).reshape(nt, nt, bins)
        centres += np.bincount(np.broadcast_to(types, cen.shape)[cen], minlength=nt)
    return counts, centres


def test_rdf_normalise_is_one_for_independent_ions(oracle):
    """Ions placed independently and uniformly, type b in the ball of radius
    R - sigma_b / 2: a neighbour of type b lies in shell k of a centre with
    probability V_k / ((4/3) pi (R - sigma_b/2)^3) for each of the N_b -
    delta_ab other ions, so the pooled estimator g_ab(r_k) has expectation
    1 in every shell that lies inside the neighbours' ball for every centre
    (r_{k+1} <= rmax - sigma_b / 2).  Closed form, no Markov chain; a density
    without the ion radius or a neighbour count that includes the centre is
    off by 5-30 %."""
    n_of_type, sig = [12, 16], [1.0, 0.4]
    R, rmax, bins, samples = 6.0, 2.5, 5, 60_000
    a_of_type = [R - 0.5 * s for s in sig]
    counts, centres = _uniform_ball_counts(n_of_type, a_of_type, R, rmax, bins, samples, 31)
    g, r = oracle.rdf_normalise(counts, centres, n_of_type, sig, R, rmax, bins, n_samples=samples)
    edges = np.arange(bins + 1) * (rmax / bins)
    for a in range(2):
        for b in range(2):
            for k in range(1, bins):
                if edges[k + 1] > rmax - 0.5 * sig[b]:
                    continue
                sd = 1.0 / math.sqrt(counts[a, b, k])
                assert abs(g[a, b, k] - 1.0) < 4.5 * sd + 1e-3, (a, b, k, g[a, b, k], sd)
    assert np.allclose(r, 0.5 * (edges[1:] + edges[:-1]))


def test_openmp_build_runs_the_same_chain(oracle):
    """The oracle's OpenMP build (used only to time the CPU on all host
    threads) sums each move's partners in another order: the same decisions
    and energy changes to 1e-12 on a system large enough to split."""
    from paper_1602_05716_amd import inputs
    s = inputs.electrolyte(2048, 2048, 1.0, -1.0, 1.0, 1.0, 0.05, 0.7)
    s.xyz = inputs.random_start(s, 17)
    a = oracle.Chain(s.xyz, s.q, s.sigma, s.R, s.lB, 2.0, seed=5)
    b = oracle.Chain(s.xyz, s.q, s.sigma, s.R, s.lB, 2.0, seed=5, threaded=True)
    ra, rb = a.run(1, trace=s.n), b.run(1, trace=s.n)
    assert np.array_equal(ra["acc"], rb["acc"])
    assert np.allclose(ra["dE"], rb["dE"], rtol=1e-12, atol=1e-12)
