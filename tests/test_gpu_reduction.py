"""GPU parity of the per-move parallel-reduction scheme (mc_sweep_reduction)
against the CPU oracle, through the C ABI.

Paper: Liang, Xing, Li, arXiv:1602.05716, Sec. 4 -- the GPU comparison code
that moves one particle per kernel launch and sums the N - 1 pair terms by a
parallel reduction.  It runs the same sequential chain as the sweep kernel
(Sec. 2), so the bar is the same: the double path reproduces the oracle's
accept/reject sequence bit for bit, the float path matches the exact double
dE of the same float state within |dE32 - dE64| <= 1e-5 max(|dE64|, 1 kT).
Both schemes work on one chain state, so they may take turns on a chain.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _sys(n_cat, n_an, q=(1.0, -1.0), s=(1.0, 1.0), phi=0.05, lB=0.7, seed=1):
    from paper_1602_05716_amd import inputs
    sy = inputs.electrolyte(n_cat, n_an, q[0], q[1], s[0], s[1], phi, lB)
    sy.xyz = inputs.random_start(sy, seed)
    return sy


def _ragged(n):
    from paper_1602_05716_amd import inputs
    if n == 1:
        sy = inputs.electrolyte(1, 0, 0.0, 0.0, 1.0, 1.0, 0.05, 0.7)
        sy.xyz = np.zeros((1, 3))
        return sy
    sy = _sys(n // 2, n - n // 2, seed=n)
    if n % 2:
        sy.q = sy.q.copy()
        sy.q[-1] = 0.0  # keep neutral with an odd count
    return sy


def _fp64_run(sy, plan, seed, D, **opts):
    """Runs the chain by plan = [(scheme, sweeps), ...] and returns its trace."""
    from paper_1602_05716_amd import mc
    sweeps = sum(k for _, k in plan)
    n_moves = sweeps * sy.n
    _say("reduction fp64 N=%d plan=%s seed=%d D=%g opts=%s" % (sy.n, plan, seed, D, opts))
    with mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, precision="fp64", max_disp=0.5 * D,
                  trace_moves=n_moves, resum_every=0, **opts) as ch:
        for scheme, k in plan:
            (ch.sweep_reduction if scheme == "reduce" else ch.sweep)(k, seed)
        acc, de = ch.trace(n_moves)
        out = dict(acc=acc, de=de, x=ch.positions(), e_run=ch.energy(), st=ch.stats(),
                   es=ch.energy_series(sweeps))
    return out


def _fp64_check(oracle, sy, plan, seed, D, **opts):
    g = _fp64_run(sy, plan, seed, D, **opts)
    sweeps = sum(k for _, k in plan)
    ref = oracle.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, D, seed=seed)
    r = ref.run(sweeps, trace=sweeps * sy.n, series=True)
    bad = np.flatnonzero(g["acc"] != r["acc"])
    assert bad.size == 0, "first mismatching move %d" % bad[0]
    err = np.abs(g["de"] - r["dE"]) / np.maximum(np.abs(r["dE"]), 1.0)
    assert err.max() < 1e-10, err.max()
    assert np.array_equal(g["x"], ref.x)
    assert abs(g["e_run"] - ref.e_run) <= 1e-9 * max(1.0, abs(ref.e_run))
    assert np.allclose(g["es"], r["e_series"], rtol=1e-10, atol=1e-10)
    st = g["st"]
    assert st["moves"] == sweeps * sy.n and st["accepted"] == int(r["acc"].sum())
    assert st["accepted"] + st["rejected_wall"] + st["rejected_overlap"] + st["rejected_metropolis"] == st["moves"]
    return g, r


def test_reduction_fp64_small_config_bit_exact(oracle):
    """1:1, N = 1000, phi = 0.01, l_B = 0.7: 30 sweeps, one launch per move."""
    from paper_1602_05716_amd import inputs
    sy = inputs.small_fp64()
    _fp64_check(oracle, sy, [("reduce", 30)], 0x5EED0001, 1.0)


@pytest.mark.parametrize("n", [1, 2, 63, 65, 255, 257, 700])
def test_reduction_fp64_ragged_sizes(oracle, n):
    """Ragged N: padding lanes, one to three workgroups with a partial last one."""
    _fp64_check(oracle, _ragged(n), [("reduce", 6)], 99 + n, 1.6)


def test_reduction_fp64_asymmetric_2to1(oracle):
    """q = +2/-1, sigma = 1.0/0.8, phi = 0.2: overlaps with per-ion diameters."""
    sy = _sys(200, 400, q=(2.0, -1.0), s=(1.0, 0.8), phi=0.2, seed=5)
    g, r = _fp64_check(oracle, sy, [("reduce", 8)], 3, 0.8)
    assert g["st"]["rejected_overlap"] > 0 and g["st"]["rejected_wall"] >= 0


@pytest.mark.parametrize("plan,band", [([("sweep", 3), ("reduce", 2), ("sweep", 3)], 2),
                                       ([("reduce", 2), ("sweep", 2), ("reduce", 1)], 4)])
def test_reduction_takes_turns_with_the_sweep_kernel(oracle, plan, band):
    """Both schemes on one chain: positions, version tags, group records and
    the energy bookkeeping stay consistent across the switch."""
    sy = _ragged(777)
    _fp64_check(oracle, sy, plan, 21, 1.4, band=band)


def _fp32_check(oracle, sy, sweeps, seed, D, sample_every=1):
    from paper_1602_05716_amd import mc
    n_moves = sweeps * sy.n
    _say("reduction fp32 N=%d sweeps=%d seed=%d D=%g" % (sy.n, sweeps, seed, D))
    with mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, precision="fp32", max_disp=0.5 * D,
                  trace_moves=n_moves, resum_every=0) as ch:
        ch.sweep_reduction(sweeps, seed)
        acc, de = ch.trace(n_moves)
        x = ch.positions()
    mask = np.zeros(n_moves, np.uint8)
    mask[::sample_every] = 1
    rp = oracle.replay_f32(sy.xyz.astype(np.float32), sy.q, sy.sigma, sy.R, sy.lB, np.float32(D),
                           seed, 0, 0, n_moves, acc_given=acc, eval_mask=mask)
    assert np.array_equal(x.astype(np.float32), rp["xyz"])
    ev = mask == 1
    d64, d32 = rp["dE"][ev], de[ev]
    err = np.abs(d32 - d64) / np.maximum(np.abs(d64), 1.0)
    assert err.max() <= TOL32, (err.max(), int(np.argmax(err)))
    own, flags, a = rp["own"][ev], rp["flags"][ev], acc[ev]
    thr = -np.log(np.maximum(rp["u3"][ev], 1e-300))
    dis = np.flatnonzero(a != own)
    for k in dis:
        near = abs(d64[k] - thr[k]) <= TOL32 * max(abs(d64[k]), 1.0)
        assert near or flags[k] != 0, ("decision differs away from threshold", k, d64[k], thr[k])
    return dis.size, int(ev.sum())


def test_reduction_fp32_multi_group(oracle):
    sy = _sys(2048, 2048, phi=0.05, seed=8)
    ndis, nev = _fp32_check(oracle, sy, 2, 77, 1.0)
    assert ndis <= 2


def test_reduction_fp32_large_config_sampled(oracle):
    """1:1, N = 32768, phi = 0.05, l_B = 0.7 at the benchmark's move size
    (max_disp 5.2): one sweep of 32768 launches, every 61st move checked."""
    from paper_1602_05716_amd import inputs
    sy = inputs.large_fp32()
    ndis, nev = _fp32_check(oracle, sy, 1, 0x5EED0003, 10.4, sample_every=61)
    assert nev > 500 and ndis <= 2


def test_reduction_rejects_batches():
    from paper_1602_05716_amd import mc
    systems = [_sys(50, 50, seed=30 + k) for k in range(2)]
    with mc.Batch(systems) as b:
        assert mc.lib().mc_sweep_reduction(b.h, 1, 1) == -1  # MC_E_ARG


def test_reduction_interleaves_resum_and_rdf_like_the_sweep_kernel():
    """Re-sum and g(r) intervals inside mc_sweep_reduction: the same positions,
    re-sum count, g(r) counts and (to rounding) energies as mc_sweep."""
    from paper_1602_05716_amd import mc
    sy = _sys(200, 400, q=(2.0, -1.0), s=(1.0, 0.8), phi=0.08, seed=17)
    kw = dict(precision="fp64", max_disp=0.6, resum_every=3, rdf_every=2, rdf_bins=50, rdf_rmax=5.0)
    out = []
    for scheme in ("sweep", "reduce"):
        _say("reduction intervals scheme=%s" % scheme)
        with mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, **kw) as ch:
            (ch.sweep_reduction if scheme == "reduce" else ch.sweep)(7, 5)
            st = ch.stats()
            out.append(dict(x=ch.positions(), e=ch.energy(exact=True), es=ch.energy_series(7), rdf=ch.rdf(),
                            resums=st["resums"], moves=st["moves"], acc=st["accepted"]))
    a, b = out
    assert np.array_equal(a["x"], b["x"])
    assert a["resums"] == b["resums"] == 2 and a["moves"] == b["moves"] == 7 * sy.n and a["acc"] == b["acc"]
    assert np.allclose(a["es"], b["es"], rtol=1e-10, atol=1e-10)
    assert abs(a["e"][0] - b["e"][0]) <= 1e-9 * max(1.0, abs(a["e"][1])) and a["e"][1] == b["e"][1]
    assert a["rdf"]["samples"] == b["rdf"]["samples"] == 3
    assert np.array_equal(a["rdf"]["counts"], b["rdf"]["counts"])
