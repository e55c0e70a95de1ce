"""Batched chains in one persistent launch, against the CPU oracle (C ABI).

Every chain of a batch is an independent exact Metropolis chain (Sec. 2);
serving many chains from one launch with per-chain workgroups (the
multi-thread-per-particle idea of Sec. 3.7, whose best setting depends on N,
Sec. 4) must not change any chain's trajectory: the double path reproduces
each chain's oracle run bit for bit whatever the schedule, and the float path
matches the exact double dE within the float tolerance.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _chain_sys(n, phi, lB, seed, q=(1.0, -1.0), s=(1.0, 1.0)):
    from paper_1602_05716_amd import inputs
    n_c = n // 2
    sy = inputs.electrolyte(n_c, n - n_c, q[0], q[1], s[0], s[1], phi, lB)
    if n % 2:
        sy.q = sy.q.copy()
        sy.q[-1] = 0.0
    sy.xyz = inputs.random_start(sy, seed)
    return sy


def _mixed_batch():
    # uneven sizes (ragged groups, one ion, one group), concentrations,
    # Bjerrum lengths and move sizes
    spec = [(1, 0.05, 0.7, 1.0), (65, 0.02, 1.5, 1.2), (200, 0.08, 0.5, 0.8), (333, 0.01, 2.0, 2.0),
            (700, 0.05, 0.7, 1.0), (128, 0.1, 1.0, 0.6)]
    systems, D = [], []
    for k, (n, phi, lB, d) in enumerate(spec):
        if n == 1:
            from paper_1602_05716_amd import inputs
            sy = inputs.electrolyte(1, 0, 0.0, 0.0, 1.0, 1.0, phi, lB)
            sy.xyz = np.zeros((1, 3))
        else:
            sy = _chain_sys(n, phi, lB, seed=1000 + k)
        systems.append(sy)
        D.append(d)
    return systems, D


def _oracle_run(oracle, sy, D, seed, chain, sweeps, trace):
    ref = oracle.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, D, seed=seed, chain=chain)
    r = ref.run(sweeps, trace=trace, series=True)
    return ref, r


def test_fp64_batch_bit_exact_per_chain(oracle):
    """Six uneven chains in one launch: each chain's decisions, dE, final
    positions and per-sweep running energies equal its own oracle run."""
    from paper_1602_05716_amd import mc
    systems, D = _mixed_batch()
    sweeps, seed = 6, 0xBA7C4
    cap = max(sy.n for sy in systems) * sweeps
    _say("fp64 batch sizes=%s sweeps=%d" % ([sy.n for sy in systems], sweeps))
    with mc.Batch(systems, max_disp=[0.5 * d for d in D], chain_ids=[7 * k + 3 for k in range(len(systems))],
                  precision="fp64", trace_moves=cap, resum_every=0) as b:
        b.sweep(sweeps, seed)
        for k, sy in enumerate(systems):
            n_moves = sweeps * sy.n
            acc, de = b.trace(k, n_moves)
            ref, r = _oracle_run(oracle, sy, D[k], seed, 7 * k + 3, sweeps, n_moves)
            bad = np.flatnonzero(acc != r["acc"])
            assert bad.size == 0, ("chain", k, "first mismatching move", bad[:1])
            err = np.abs(de - r["dE"]) / np.maximum(np.abs(r["dE"]), 1.0)
            assert err.max() < 1e-10, (k, err.max())
            assert np.array_equal(b.positions(k), ref.x), k
            es = b.energy_series(k, sweeps)
            assert np.allclose(es, r["e_series"], rtol=1e-9, atol=1e-9), k
            st = b.stats(k)
            assert st["moves"] == n_moves and st["accepted"] == int(r["acc"].sum()), k


def test_schedule_does_not_change_trajectories(oracle):
    """The same float batch under the default schedule, one workgroup per
    chain, and the autotuned schedule: identical positions after every call."""
    from paper_1602_05716_amd import mc
    systems = [_chain_sys(n, phi, 0.7 + 0.1 * k, seed=2000 + k)
               for k, (n, phi) in enumerate([(500, 0.02), (1500, 0.05), (3000, 0.08), (900, 0.01)])]
    seed = 0x5C4ED
    _say("schedule independence sizes=%s" % [sy.n for sy in systems])
    runs = []
    for mode in ("default", "ones", "autotune"):
        with mc.Batch(systems, precision="fp32", max_disp=[1.0] * 4, resum_every=0) as b:
            if mode == "ones":
                b.set_schedule(np.ones(len(systems), np.int32))
            if mode == "autotune":
                a, bb = b.autotune(3, seed)
                assert a > 0 and bb > 0
                w, model = b.schedule()
                assert w.min() >= 1 and model == (a, bb)
                b.sweep(2, seed)
            else:
                b.sweep(5, seed)
            runs.append([b.positions(k) for k in range(len(systems))])
            ms = b.launch_ms()
            assert np.all(ms > 0)
    for k in range(len(systems)):
        assert np.array_equal(runs[0][k], runs[1][k]), k
        assert np.array_equal(runs[0][k], runs[2][k]), k


def test_fp64_batch_energy_and_rdf(oracle):
    """Per-chain double re-sum against the oracle's total energy of the same
    positions, and per-chain g(r) counts against the oracle's counts."""
    from paper_1602_05716_amd import mc
    from paper_1602_05716_amd import inputs
    asym = inputs.electrolyte(100, 200, 2.0, -1.0, 1.0, 0.8, 0.1, 1.2)
    asym.xyz = inputs.random_start(asym, 3003)
    systems = [_chain_sys(400, 0.03, 0.7, seed=3001), asym]
    _say("fp64 batch energy/rdf")
    with mc.Batch(systems, precision="fp64", max_disp=[0.6, 0.4], resum_every=3, rdf_bins=50,
                  rdf_rmax=4.0, rdf_every=2) as b:
        b.sweep(6, 11)
        for k, sy in enumerate(systems):
            x = b.positions(k)
            e_run, e_exact = b.energy(k, exact=True)
            e_ref = oracle.total_energy(x, sy.q, sy.lB)
            scale = sy.lB * float(np.sum(np.abs(np.outer(sy.q, sy.q))[np.triu_indices(sy.n, 1)] /
                                         np.maximum(1e-300, _pdist(x))))
            assert abs(e_exact - e_ref) <= 1e-12 * scale, (k, e_exact, e_ref)
            assert abs(e_run - e_ref) <= 1e-9 * scale, (k, e_run, e_ref)
            st = b.stats(k)
            assert st["resums"] == 2
            assert b.rdf(k)["samples"] == 3
        # oracle g(r) counts of the three sampled states (after sweeps 2, 4, 6)
        for k, sy in enumerate(systems):
            ref = oracle.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, [1.2, 0.8][k], seed=11, chain=k)
            types, _ = sy.types()
            nt = int(types.max()) + 1
            tot = None
            cen = None
            for _ in range(3):
                ref.run(2)
                c, ce = oracle.rdf_counts(ref.x, types, nt, sy.R, 4.0, 50)
                tot = c if tot is None else tot + c
                cen = ce if cen is None else cen + ce
            got = b.rdf(k)
            assert np.array_equal(got["counts"], tot), k
            assert np.array_equal(got["centres"], cen), k


def _pdist(x):
    from scipy.spatial.distance import pdist
    return pdist(x)


def test_packed_chains_keep_their_trajectories(oracle):
    """Six chains of very different size on a budget of six workgroups: after
    the autotuner has measured them, the small chains share one workgroup
    (run one after another) and the two large ones get several each.  Every
    chain's positions equal those of one workgroup per chain."""
    from paper_1602_05716_amd import mc
    sizes = [200, 300, 500, 800, 3000, 4000]
    systems = [_chain_sys(n, 0.05, 0.8, seed=3000 + k) for k, n in enumerate(sizes)]
    seed = 0xBA11
    _say("packing sizes=%s" % sizes)
    runs = []
    for mode in ("ones", "packed"):
        with mc.Batch(systems, precision="fp32", max_disp=[1.0] * 6, resum_every=0, workgroups=6) as b:
            if mode == "ones":
                b.set_schedule(np.ones(6, np.int32))
                b.sweep(1, seed)  # the calibration sweep of the other run
            else:
                b.autotune(1, seed)
                w, _ = b.schedule()
                _say("packed schedule", w.tolist())
                assert w.sum() > 6 and w[5] > 1  # the launch holds at most six workgroups
            b.sweep(4, seed)
            runs.append([b.positions(k) for k in range(6)])
    for k in range(6):
        assert np.array_equal(runs[0][k], runs[1][k]), k


def test_ensemble_sampled_chains_fp32(oracle):
    """The batched-ensemble workload (256 chains, N log-uniform in [500, 8000],
    phi in [0.005, 0.1], l_B in [0.5, 2]) in one launch with the autotuned
    schedule; 8 chains stratified by N are checked move by move (every 7th
    move of two sweeps) against the exact double dE of the same float state.
    The launch runs on eight waves per workgroup, the library's choice for
    this many groups."""
    from paper_1602_05716_amd import inputs, mc
    params = inputs.ensemble_params(256)
    systems = [inputs.ensemble_chain(*p) for p in params]
    order = np.argsort([s.n for s in systems])
    picks = [int(order[int(round(q))]) for q in np.linspace(0, 255, 8)]
    seed = 0x5EED0004
    _say("ensemble 256 chains, sum N = %d" % sum(s.n for s in systems))
    sweeps = 2
    # the trace covers the calibration sweep and the checked sweeps
    with mc.Batch(systems, precision="fp32", max_disp=[0.5] * 256,
                  trace_moves=max(s.n for s in systems) * (1 + sweeps), resum_every=0) as b:
        # 11014 groups in all: the eight-wave kernel, whole decided groups per wave
        assert b.stats(0)["waves"] == 8
        a, bb = b.autotune(1, seed)
        _say("autotune model a=%.3f b=%.3f us" % (a, bb))
        w, _ = b.schedule()
        # after the autotuner has measured them, chains that one workgroup
        # serves alone may share a workgroup, so the per-chain counts can add
        # up to more than the launch's workgroups
        assert w.min() >= 1 and all(w[k] <= (systems[k].n + 63) // 64 for k in range(256))
        # positions after the calibration sweep are the starting state of the checked sweeps
        starts = {k: b.positions(k).astype(np.float32) for k in picks}
        b.sweep(sweeps, seed)
        for k in picks:
            sy = systems[k]
            n_moves = sweeps * sy.n
            acc, de = b.trace(k, sy.n * (1 + sweeps))
            acc, de = acc[sy.n:], de[sy.n:]
            mask = np.zeros(n_moves, np.uint8)
            mask[::7] = 1
            rp = oracle.replay_f32(starts[k], sy.q, sy.sigma, sy.R, sy.lB, np.float32(1.0), seed, k, 1,
                                   n_moves, acc_given=acc, eval_mask=mask)
            assert np.array_equal(b.positions(k).astype(np.float32), rp["xyz"]), k
            ev = mask == 1
            err = np.abs(de[ev] - rp["dE"][ev]) / np.maximum(np.abs(rp["dE"][ev]), 1.0)
            assert err.max() <= TOL32, (k, err.max())


def test_autotune_calibration_keeps_the_interval_work(oracle):
    """The autotuner's calibration sweeps run as mc_sweep runs them: a
    calibration that crosses a re-sum boundary takes that re-sum (the
    running energy is reset to the double re-sum there), and the chains
    continue bit-exactly."""
    from paper_1602_05716_amd import mc
    systems, D = _mixed_batch()
    systems, D = systems[1:4], D[1:4]
    seed = 0xA770
    cap = max(sy.n for sy in systems) * 9
    _say("autotune across a re-sum boundary, sizes=%s" % [sy.n for sy in systems])
    with mc.Batch(systems, max_disp=[0.5 * d for d in D], precision="fp64", trace_moves=cap,
                  resum_every=5) as b:
        b.sweep(3, seed)
        b.autotune(4, seed)  # sweeps 3..6: crosses the re-sum at sweep 5
        for k in range(len(systems)):
            assert b.stats(k)["resums"] == 1, k
        b.sweep(2, seed)
        for k, sy in enumerate(systems):
            st = b.stats(k)
            assert st["sweeps"] == 9 and st["resums"] == 1, (k, st)
            acc, de = b.trace(k, 9 * sy.n)
            ref, r = _oracle_run(oracle, sy, D[k], seed, k, 9, 9 * sy.n)  # chain id k
            assert np.array_equal(acc, r["acc"]), k
            assert np.array_equal(b.positions(k), ref.x), k
            e_run, e_ex = b.energy(k, exact=True)
            assert abs(e_run - e_ex) <= 1e-9 * max(1.0, abs(e_ex)), k
