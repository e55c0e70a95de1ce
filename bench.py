"""Benchmark: exact-energy sequential Metropolis MC of the 1:1 primitive model
at N = 32768 on one MI355X.

One step = mc_sweep of --sweeps-per-step sweeps (default 100) of the whole
hot path: the persistent sweep kernel (trial draw, exact dE over all N-1
partners with the hard-core test, sequential accept/reject, in-place update)
followed by the double-precision energy re-sum that closes the interval.

Workload: 16384 cations (+1) and 16384 anions (-1), sigma = 1, l_B = 0.7,
hard-wall sphere at volume fraction 0.05, seeded random start (synthetic),
float positions and pair terms with double per-move and running-energy sums;
the trial cube is tuned to about 40 % acceptance during warm-up and then
frozen.  Prints one JSON line (see the repository's design notes for the
roofline and CPU-baseline definitions).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MC moves/s + pair terms/s at N=32768; ESS/s plain vs batched vs surrogate-DA"
CUS, CLOCK_HZ = 256, 2.4e9
# ALU roofline of one pair term (float path).  Algorithmic work per term:
# two squared distances (3 sub + 3 mul/fma each), the difference of the two
# inverse distances and its charge-weighted accumulation (2), the contact
# test (1): 15 vector ALU lane-ops, plus 2 reciprocal square roots.
# Chip rates: the published FP32 vector peak, 157.3 TFLOP/s = 128 FMA lanes
# per clock per CU; transcendentals at a quarter of that, 32 lanes per clock
# per CU (the valu_peak probe measures both on the device).
VALU_PER_PAIR, RSQ_PER_PAIR = 15, 2
VALU_LANES_PER_CLK_CU, RSQ_LANES_PER_CLK_CU = 128.0, 32.0
PAIR_PEAK_PER_S = CUS * CLOCK_HZ / (VALU_PER_PAIR / VALU_LANES_PER_CLK_CU + RSQ_PER_PAIR / RSQ_LANES_PER_CLK_CU)


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "sweep_kernel_n32768_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1602_05716_amd", "csrc", f)
                  for f in ("mc_sweep_kernel.hpp", "mc_device.hpp")]


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch(sweeps_per_launch):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, calibrated on a copy kernel); None when the summary is absent
    or was taken on a different version of the sweep kernel."""
    try:
        kv = {}
        with open(TRAFFIC_SUMMARY) as fh:
            for line in fh:
                if line.startswith("- ") and ": " in line:
                    k, v = line[2:].split(": ", 1)
                    kv[k.strip()] = v.strip().strip("`")
        if kv.get("kernel_source_digest") != kernel_source_digest():
            return None
        return float(kv["hbm_bytes_per_launch_fixed"]) + float(kv["hbm_bytes_per_sweep"]) * sweeps_per_launch
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def tune_max_disp(chain, max_disp, target=0.40, rounds=8, sweeps=4, seed=0xD15C):
    """Warm-up only: D <- D * clamp(acc / target, 1/2, 2) after each round."""
    md = max_disp
    for r in range(rounds):
        chain.set_max_disp(md)
        st0 = chain.stats()
        chain.sweep(sweeps, seed + r)
        st1 = chain.stats()
        acc = (st1["accepted"] - st0["accepted"]) / max(1, st1["moves"] - st0["moves"])
        log("tune round %d: max_disp %.4f acceptance %.4f" % (r, md, acc))
        md *= min(2.0, max(0.5, acc / target))
    chain.set_max_disp(md)
    return md


def cpu_baseline(system, D, seed, sweeps=1):
    """The FP64 oracle, serial, on the same system and start (bounded sample)."""
    from oracle import oracle
    ch = oracle.Chain(system.xyz, system.q, system.sigma, system.R, system.lB, D, seed=seed)
    t0 = time.perf_counter()
    ch.run(sweeps)
    dt = time.perf_counter() - t0
    n = system.n
    return {"value": sweeps * n / dt, "unit": "moves/s", "cores": 1, "kind": "oracle",
            "pair_terms_per_s": sweeps * n * (n - 1) / dt,
            "sample": "%d sweep(s) = %d moves of the same N=%d system and start, FP64 oracle, "
                      "1 thread, %.1f s" % (sweeps, sweeps * n, n, dt)}


def run_valu_probe():
    exe = os.path.join(ROOT, "paper_1602_05716_amd", "valu_peak")
    if not os.path.exists(exe):
        return None
    try:
        out = subprocess.run([exe], capture_output=True, text=True, timeout=60, check=True).stdout
        return json.loads(out.strip().splitlines()[-1])
    except Exception as e:  # the probe is informational
        log("valu probe failed:", e)
        return None


def batched_leg(args, log_fn=None):
    """Batched ensemble: 256 independent 1:1 chains (N log-uniform in [500,
    8000], phi uniform in [0.005, 0.1], l_B uniform in [0.5, 2]) in one
    persistent launch with the autotuned schedule, against the same chains
    run one after another with the single-chain path.

    A chain's trajectory does not depend on the schedule (tested), so both
    modes give every chain the same energy series and the same ESS; only the
    wall time differs.  The one-after-another time of each chain is measured
    alone on ``seq_sweeps`` sweeps of the same stretch and scaled to the
    batched sweep count."""
    import torch
    from paper_1602_05716_amd import analysis, inputs, mc
    params = inputs.ensemble_params(256)
    systems = [inputs.ensemble_chain(*p) for p in params]
    nsum = sum(s.n for s in systems)
    pairs = sum(s.n * (s.n - 1) for s in systems)
    S, seed = args.batch_sweeps, 0x5EED0004
    stream = torch.cuda.Stream()
    b = mc.Batch(systems, precision="fp32", max_disp=[0.5] * len(systems), resum_every=100,
                 hip_stream=stream.cuda_stream, record_timing=1)
    # warm-up: per-chain move-size tuning, then the autotuner, then equilibration
    md = np.full(len(systems), 0.5)
    for r in range(8):
        st0 = [b.stats(k) for k in range(len(systems))]
        b.sweep(4, 0xD15C + r)
        for k in range(len(systems)):
            st1 = b.stats(k)
            acc = (st1["accepted"] - st0[k]["accepted"]) / max(1, st1["moves"] - st0[k]["moves"])
            md[k] *= min(2.0, max(0.5, acc / 0.40))
            b.set_max_disp(k, md[k])
    model = b.autotune(2, seed)
    b.sweep(66, seed)  # equilibration up to a multiple of the re-sum interval
    s0 = b.stats(0)["sweeps"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.sweep(S, seed)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ess = []
    for k in range(len(systems)):
        e = b.energy_series(k, s0 + S)[s0:]
        ess.append(analysis.effective_samples(e))
    w, _ = b.schedule()
    b.close()
    # the same chains, one at a time, same state and parameters at the start of the timed stretch
    t_seq = 0.0
    for k, sy in enumerate(systems):
        ch = mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, precision="fp32", max_disp=float(md[k]),
                      chain_id=k, resum_every=100, hip_stream=stream.cuda_stream)
        ch.sweep(2, 0)  # the cost of a sweep does not depend on which sweep it is
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ch.sweep(args.seq_sweeps, seed)
        torch.cuda.synchronize()
        t_seq += (time.perf_counter() - t1) * S / args.seq_sweeps
        ch.close()
    ess_tot = float(np.nansum(ess))
    return {"workload": "256 independent 1:1 chains, N log-uniform [500, 8000] (sum %d), phi U[0.005, 0.1], "
                        "l_B U[0.5, 2], move size tuned per chain to ~40%% acceptance" % nsum,
            "chains": len(systems), "sum_n": nsum, "sweeps": S,
            "wall_s": t_batch, "moves_per_s": S * nsum / t_batch, "pair_terms_per_s": S * pairs / t_batch,
            "ess_total": ess_tot, "ess_per_s": ess_tot / t_batch,
            "workgroups_total": int(w.sum()), "cost_model_us": {"a": model[0], "b": model[1]},
            "one_after_another": {"wall_s": t_seq, "ess_per_s": ess_tot / t_seq,
                                  "measured_sweeps_per_chain": args.seq_sweeps},
            "batched_over_sequential": t_seq / t_batch}


def reduction_leg(chain, args, sweep_rate):
    """The paper's GPU comparison code (Sec. 4): the same chain continued by
    the per-move parallel-reduction scheme, one launch per trial move, after
    the timed region (it does not touch the measured sweeps)."""
    import torch
    n = chain.n
    chain.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chain.sweep_reduction(args.reduction_sweeps, args.seed + 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _, ms, _ = chain.timing()
    moves = args.reduction_sweeps * n
    return {"kernel": "reduce_move_kernel<float>", "sweeps": args.reduction_sweeps, "launches": moves,
            "wall_s": wall, "event_s": ms * 1e-3, "moves_per_s": moves / wall, "us_per_move": 1e6 * wall / moves,
            "sweep_kernel_over_reduction": sweep_rate / (moves / wall)}


def _gr_sample_run(chain, sweeps, seed, every):
    """Runs `sweeps` sweeps with a g(r) sample every `every` sweeps; returns
    (wall seconds, energy series, g(r) of the first and second halves)."""
    import torch
    s0 = chain.stats()["sweeps"]
    chain.rdf_reset()
    halves = []
    t = 0.0
    for half in range(2):
        for _ in range(sweeps // 2 // every):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            chain.sweep(every, seed)
            chain.rdf_sample()
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
        halves.append(chain.rdf())
        chain.rdf_reset()
    e = chain.energy_series(chain.stats()["sweeps"])[s0:]
    return t, e, halves


def da_leg(args, md):
    """Surrogate delayed acceptance on the N=32768 system: log moves of a
    plain run, train the network on the GPU, then run the two-stage chain and
    the plain chain from the same state for the same number of sweeps."""
    import torch
    from paper_1602_05716_amd import analysis, inputs, mc
    system = inputs.large_fp32()
    n = system.n
    stream = torch.cuda.Stream()
    sweeps_log = max(1, -(-args.da_log_moves // n))
    n_log = sweeps_log * n
    seed = 0x5EED0005
    with mc.Chain(system.xyz, system.q, system.sigma, system.R, system.lB, precision="fp32", max_disp=md,
                  resum_every=100, waves=4, log_moves=n_log, hip_stream=stream.cuda_stream,
                  band=args.da_band) as lg_chain:
        lg_chain.sweep(sweeps_log, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = lg_chain.train_surrogate(n_log, epochs=args.da_epochs, batch=4096, lr=2e-3, seed=7)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        x0 = lg_chain.positions()
    out = {"workload": "1:1 N=32768 phi=0.05 l_B=0.7 (the plain benchmark's system), %d logged moves, "
                       "network 128-128-128-1 bfloat16" % n_log,
           "train_s": t_train, "train_loss": [float(v) for v in tr["loss"]], "val_loss": tr["val_loss"],
           "ref_stage2_reject": tr["ref_stage2_reject"], "sweeps": args.da_sweeps}
    runs = {}
    for mode in ("plain", "da"):
        kw = dict(precision="fp32", max_disp=md, resum_every=100, hip_stream=stream.cuda_stream, rdf_bins=200,
                  rdf_rmax=10.0)
        if mode == "da":
            kw["waves"] = 4
            kw["band"] = args.da_band
        with mc.Chain(x0, system.q, system.sigma, system.R, system.lB, **kw) as c:
            if mode == "da":
                c.set_surrogate(tr["params"], tr["ref_stage2_reject"], True)
            # first launch out of the timed region; one drift-monitor window
            # (10 sweeps), so that every timed call below is a single launch
            c.sweep(10, seed + 1)
            t, e, halves = _gr_sample_run(c, args.da_sweeps, seed + 2, 10)
            st = c.stats()
            ess = analysis.effective_samples(e)
            g = 0.5 * (halves[0]["g"] + halves[1]["g"])
            runs[mode] = {"wall_s": t, "ess": ess, "ess_per_s": ess / t, "moves_per_s": args.da_sweeps * n / t,
                          "acceptance": st["accepted"] / max(1, st["moves"]), "g": g, "halves": halves,
                          "stats": st}
    # g(r) accuracy: RMS difference between the two runs against the plain
    # run's own half-to-half RMS difference (the statistical noise scale)
    r = (np.arange(200) + 0.5) * 0.05
    sel = r >= 1.0
    def rms(a, b):
        return float(np.sqrt(np.mean((a[..., sel] - b[..., sel]) ** 2)))
    ph = runs["plain"]["halves"]
    out["plain"] = {k: v for k, v in runs["plain"].items() if k in ("wall_s", "ess", "ess_per_s", "moves_per_s", "acceptance")}
    out["da"] = {k: v for k, v in runs["da"].items() if k in ("wall_s", "ess", "ess_per_s", "moves_per_s", "acceptance")}
    sd = runs["da"]["stats"]
    out["da"].update({"stage1_rejected": sd["da_stage1_rejected"], "stage1_passed": sd["da_stage1_passed"],
                      "stage2_rejected": sd["da_stage2_rejected"], "conflict_moves": sd["da_conflicts"],
                      "two_stage_moves": sd["da_moves"], "fallback_sweep": sd["da_fallback_sweep"],
                      "active_at_end": sd["da_active"]})
    out["g_rms_da_vs_plain"] = rms(runs["da"]["g"], runs["plain"]["g"])
    out["g_rms_plain_half_vs_half"] = rms(ph[0]["g"], ph[1]["g"])
    out["ess_per_s_da_over_plain"] = out["da"]["ess_per_s"] / out["plain"]["ess_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps-per-step", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0x5EED0002)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=1)
    ap.add_argument("--no-probe", action="store_true", help="skip the VALU issue-rate probe")
    ap.add_argument("--band", type=int, default=-1)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--batch-sweeps", type=int, default=1000)
    ap.add_argument("--seq-sweeps", type=int, default=20)
    ap.add_argument("--no-da", action="store_true", help="skip the surrogate delayed-acceptance leg")
    ap.add_argument("--da-log-moves", type=int, default=1000000)
    ap.add_argument("--da-epochs", type=int, default=6)
    ap.add_argument("--da-sweeps", type=int, default=400)
    ap.add_argument("--no-reduction", action="store_true",
                    help="skip the per-move parallel-reduction comparison leg")
    ap.add_argument("--reduction-sweeps", type=int, default=1)
    ap.add_argument("--da-band", type=int, default=-1,
                    help="band of the logging and surrogate chains (-1: the library's default)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: a single chain does not shard across GPUs "
              "(independent chains would, see the design notes); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1602_05716_amd import analysis, inputs, mc

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.init()
    stream = torch.cuda.Stream()  # default priority; the chain enqueues all its work here

    log("building the N=32768 start")
    system = inputs.large_fp32()
    n = system.n
    chain = mc.Chain(system.xyz, system.q, system.sigma, system.R, system.lB, precision="fp32",
                     max_disp=0.5, resum_every=args.sweeps_per_step, record_timing=1,
                     hip_stream=stream.cuda_stream, band=args.band, waves=args.waves)
    md = tune_max_disp(chain, 0.5)
    log("frozen max_disp %.4f" % md)
    for _ in range(args.warmup):
        chain.sweep(args.sweeps_per_step, args.seed)
    chain.energy()
    st0 = chain.stats()
    chain.timing_reset()
    sweeps0 = st0["sweeps"]

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        chain.sweep(args.sweeps_per_step, args.seed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0

    st1 = chain.stats()
    launches, kernel_ms, kernel_sweeps = chain.timing()
    series = chain.energy_series(st1["sweeps"])[sweeps0:]
    e_run, e_exact = chain.energy(exact=True)
    sweeps = args.steps * args.sweeps_per_step
    moves = sweeps * n
    pairs = sweeps * n * (n - 1)
    acc = (st1["accepted"] - st0["accepted"]) / max(1, st1["moves"] - st0["moves"])
    ess = analysis.effective_samples(series) if len(series) > 8 else float("nan")
    tau = analysis.integrated_time(series) if len(series) > 8 else float("nan")

    # dominant kernel: the persistent sweep kernel, timed by HIP events on its stream
    avg_launch_s = kernel_ms * 1e-3 / max(1, launches)
    per_launch_pairs = (kernel_sweeps / max(1, launches)) * n * (n - 1)
    achieved = per_launch_pairs / avg_launch_s / 1e12
    peak = PAIR_PEAK_PER_S / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tpairterm/s",
                "frac": achieved / peak, "traffic": traffic_per_launch(kernel_sweeps / max(1, launches)),
                "per_unit": "pair term = %d VALU + %d rsq lane-ops" % (VALU_PER_PAIR, RSQ_PER_PAIR),
                "rsq_only_frac": achieved * RSQ_PER_PAIR / (CUS * CLOCK_HZ * RSQ_LANES_PER_CLK_CU / 1e12),
                "kernel": "sweep_kernel<float,%d>" % st1["waves"],
                "avg_launch_ms": avg_launch_s * 1e3, "launches": launches,
                "sweeps_per_launch": kernel_sweeps / max(1, launches)}
    reduction = None
    if not args.no_reduction:
        log("per-move parallel-reduction leg (%d sweep(s))" % args.reduction_sweeps)
        reduction = reduction_leg(chain, args, moves / elapsed)
    probe = None if args.no_probe else run_valu_probe()
    if probe:
        roofline["probe"] = probe

    batched = None
    if not args.no_batched:
        log("batched ensemble leg")
        batched = batched_leg(args)

    da = None
    if not args.no_da:
        log("surrogate delayed-acceptance leg")
        da = da_leg(args, md)

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle (%d sweep(s))" % args.cpu_sweeps)
        cpu = cpu_baseline(system, 2.0 * md, args.seed, args.cpu_sweeps)
        cpu["cores_available"] = os.cpu_count()
        cpu["gpu_over_cpu"] = (moves / elapsed) / cpu["value"]

    out = {
        "metric": METRIC, "value": moves / elapsed, "unit": "moves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1:1 primitive model, N=32768 (16384 +1 / 16384 -1), sigma=1, "
                               "l_B=0.7, hard-wall sphere phi=0.05, seeded random start",
                   "n_ions": n, "sweeps_per_step": args.sweeps_per_step,
                   "precision": "f32 pair terms, f64 per-move and running sums",
                   "max_disp": md, "acceptance": acc, "band": st1["band"], "waves": st1["waves"],
                   "workgroups": st1["workgroups"]},
        "pair_terms_per_s": pairs / elapsed,
        "ess_per_s": {"plain": ess / elapsed,
                      "batched": batched["ess_per_s"] if batched else None,
                      "batched_one_after_another": batched["one_after_another"]["ess_per_s"] if batched else None,
                      "surrogate_da": da["da"]["ess_per_s"] if da else None,
                      "plain_same_run_as_da": da["plain"]["ess_per_s"] if da else None},
        "batched": batched,
        "surrogate_da": da,
        "reduction_scheme": reduction,
        "energy": {"tau_int_sweeps": tau, "e_running": e_run, "e_resum": e_exact,
                   "max_abs_drift_per_resum": st1["max_abs_drift"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "context": "paper: 440x over a serial CPU code on a Tesla K20 (quoted, not a target)",
    }
    chain.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
