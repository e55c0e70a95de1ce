"""Checkpoint and resume through the C ABI (mc_save / mc_load).

The random stream is a function of (seed, sweep, ion, chain), so a chain
saved after k sweeps, loaded and run on must reproduce the uninterrupted
chain bit for bit: decisions, positions, the running energy, the energy
series, the re-sum record, the counters and the g(r) counts.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _sys(n_cat, n_an, q=(1.0, -1.0), s=(1.0, 1.0), phi=0.05, lB=0.7, seed=1):
    from paper_1602_05716_amd import inputs
    sy = inputs.electrolyte(n_cat, n_an, q[0], q[1], s[0], s[1], phi, lB)
    sy.xyz = inputs.random_start(sy, seed)
    return sy


KEYS = ("sweeps", "moves", "accepted", "rejected_wall", "rejected_overlap", "rejected_metropolis", "resums",
        "last_drift", "max_abs_drift")


def _state(ch, sweeps, n):
    acc, de = ch.trace(sweeps * n)
    st = ch.stats()
    r = ch.rdf()
    return dict(x=ch.positions(), e=ch.energy(), es=ch.energy_series(sweeps), acc=acc, de=de,
                st={k: st[k] for k in KEYS}, counts=r["counts"], centres=r["centres"], samples=r["samples"])


@pytest.mark.parametrize("precision,opts", [("fp64", {}), ("fp32", dict(band=4, waves=8)),
                                            ("fp32", dict(band=2))])
def test_resume_is_bit_exact(tmp_path, precision, opts):
    from paper_1602_05716_amd import mc
    sy = _sys(350, 350, q=(1.0, -1.0), seed=21)
    total, cut, seed = 10, 6, 77
    kw = dict(precision=precision, max_disp=0.7, resum_every=4, rdf_every=3, rdf_bins=40, rdf_rmax=4.0,
              trace_moves=total * sy.n, **opts)
    _say("resume %s N=%d opts=%s" % (precision, sy.n, opts))
    with mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, **kw) as a:
        a.sweep(total, seed)
        ref = _state(a, total, sy.n)
    path = str(tmp_path / "chain.ckpt")
    with mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, **kw) as b:
        b.sweep(cut, seed)
        b.save(path)
    with mc.Chain.load(path) as c:  # the saved options
        assert c.stats()["sweeps"] == cut
        c.sweep(total - cut, seed)
        got = _state(c, total, sy.n)
    assert np.array_equal(got["x"], ref["x"])
    assert got["e"] == ref["e"]
    assert np.array_equal(got["es"], ref["es"])
    m = slice(cut * sy.n, total * sy.n)  # traced after the load
    assert np.array_equal(got["acc"][m], ref["acc"][m]) and np.array_equal(got["de"][m], ref["de"][m])
    assert got["st"] == ref["st"]
    assert got["samples"] == ref["samples"] == 3
    assert np.array_equal(got["counts"], ref["counts"]) and np.array_equal(got["centres"], ref["centres"])


def test_batch_resume_and_options(tmp_path):
    from paper_1602_05716_amd import mc
    systems = [_sys(100 + 37 * k, 100 + 37 * k, seed=40 + k) for k in range(3)]
    kw = dict(precision="fp32", resum_every=5)
    _say("batch resume 3 chains")
    with mc.Batch(systems, max_disp=[0.4, 0.6, 0.8], **kw) as a:
        a.sweep(9, 5)
        ref = [a.positions(k) for k in range(3)]
        ea = [a.energy(k) for k in range(3)]
    path = str(tmp_path / "batch.ckpt")
    with mc.Batch(systems, max_disp=[0.4, 0.6, 0.8], **kw) as b:
        b.sweep(4, 5)
        b.save(path)
    # options given on load: same precision and g(r) bins, a different schedule
    with mc.Batch.load(path, precision="fp32", resum_every=5, workgroups=3) as c:
        c.sweep(5, 5)
        for k in range(3):
            assert np.array_equal(c.positions(k), ref[k])
            assert abs(c.energy(k) - ea[k]) <= 1e-9 * max(1.0, abs(ea[k]))
    with pytest.raises(mc.MCError):
        mc.Batch.load(path, precision="fp64")
    with pytest.raises(mc.MCError):  # another g(r) histogram than the saved counts'
        mc.Batch.load(path, precision="fp32", rdf_rmax=5.0)


def test_production_driver_runs_and_pools(tmp_path):
    """The 3:-1 production driver end to end at a small size (no physics
    assertion: a few sweeps carry no far-field signal): counts saved, pooled,
    and the pooled g equal to the library's own for one run."""
    from paper_1602_05716_amd import analysis, dressed
    _say("dressed driver N=4096")
    sy, md, r, st, es, wall, n_of_type, (e_run, e_ex), margin = dressed.run(
        4096, 6, 2, 2, 12.0, 60, 9, chunk=3, debye_A=20.0, trace=True)
    assert r["samples"] == 3 and st["sweeps"] == 8 and len(es) == 6
    # no re-sum in 8 sweeps: the running energy carries the float error of
    # every accepted dE, each within the float path's 1e-5 max(|dE|, 1 kT)
    acc, de = st["trace"]
    bound = 1e-5 * float(np.sum(np.maximum(np.abs(de[acc == 1]), 1.0)))
    _say("running minus re-summed energy %.3e kT, bound %.3e kT, |E| %.1f kT" % (e_run - e_ex, bound, abs(e_ex)))
    assert abs(e_run - e_ex) <= bound
    path = str(tmp_path / "d.npz")
    np.savez(path, counts=r["counts"], centres=r["centres"], samples=r["samples"], g=r["g"], n_of_type=n_of_type,
             R=sy.R, rmax=12.0, bins=60, energy=es, max_disp=md, n=4096, margin=margin)
    rc, g = analysis.g_from_counts(r["counts"], r["centres"], n_of_type, [1.0, 1.0], sy.R, 12.0)
    assert np.allclose(g, r["g"], rtol=1e-12, atol=0)
    with pytest.raises(ValueError):
        dressed.pooled([path, path], (5.0, 5.1))  # too few bins in the window


def test_running_energy_error_is_the_sum_of_move_errors(oracle):
    """Float path, the 3:-1 system with cube moves of side L / 3: the running
    energy is the start's double re-sum plus every accepted float dE, the
    re-sum of the final state the start's plus every accepted exact dE, so
    their difference is the sum of the per-move float errors (each checked
    against the exact double dE of the same float state), up to double
    rounding of the two pair sums."""
    from scipy.spatial.distance import pdist

    from paper_1602_05716_amd import inputs, mc
    sy = inputs.three_to_one(4096, 9, 20.0)
    sweeps, seed, md = 8, 9, sy.R / 3.0
    n_moves = sweeps * sy.n
    _say("running-energy error, 3:-1 N=4096, %d sweeps" % sweeps)
    with mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, precision="fp32", max_disp=md, resum_every=0,
                  trace_moves=n_moves) as ch:
        e0 = ch.energy()
        ch.sweep(sweeps, seed)
        acc, de = ch.trace(n_moves)
        e_run, e_ex = ch.energy(exact=True)
    rp = oracle.replay_f32(sy.xyz.astype(np.float32), sy.q, sy.sigma, sy.R, sy.lB, np.float32(2 * md), seed, 0, 0,
                           n_moves, acc_given=acc)
    a = acc == 1
    err = de - rp["dE"]
    assert np.max(np.abs(err) / np.maximum(np.abs(rp["dE"]), 1.0)) <= 1e-5
    x0 = sy.xyz.astype(np.float32).astype(np.float64)
    x1 = rp["xyz"].astype(np.float64)
    qq = np.abs(np.outer(sy.q, sy.q))[np.triu_indices(sy.n, 1)]
    rounding = 1e-12 * sy.lB * (float(np.sum(qq / pdist(x0))) + float(np.sum(qq / pdist(x1))))
    _say("drift %.3e kT = sum of %d move errors %.3e kT (largest %.2e); |E| %.1f kT" %
         (e_run - e_ex, int(a.sum()), float(np.sum(err[a])), float(np.max(np.abs(err[a]))), abs(e_ex)))
    assert abs((e_run - e_ex) - float(np.sum(err[a]))) <= rounding + 1e-12 * float(np.sum(np.abs(de[a])))
    assert abs((e_ex - e0) - float(np.sum(rp["dE"][a]))) <= rounding + 1e-12 * float(np.sum(np.abs(de[a])))

