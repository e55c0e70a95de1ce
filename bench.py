"""Benchmark: exact-energy sequential Metropolis MC of the 1:1 primitive model
at N = 32768 on one MI355X.

One step = mc_sweep of --sweeps-per-step sweeps (default 500) of the whole
hot path: the persistent sweep kernel (trial draw, exact dE over all N-1
partners with the hard-core test, sequential accept/reject, in-place update)
with the double-precision energy re-sum every 100 sweeps (five per step; 20
steps are the 10^4 sweeps of the workload).

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
# Roofline of the sweep kernel: the reciprocal square roots.  One pair term
# (float path) is two inverse distances, 2 v_rsq_f32, plus 15 vector ALU
# lane-ops (two squared distances, 3 sub + 3 mul/fma each; the difference of
# the inverse distances and its charge-weighted accumulation, 2; the contact
# test, 1).  frac = 2 x pair terms/s over the v_rsq_f32 rate the valu_peak
# probe measures on the device (nominal: a quarter of the 128 FMA lanes per
# clock per CU of the published 157.3 TFLOP/s FP32 peak, 32 lanes).
VALU_PER_PAIR, RSQ_PER_PAIR = 15, 2
VALU_LANES_PER_CLK_CU, RSQ_LANES_PER_CLK_CU = 128.0, 32.0
RSQ_PEAK_NOMINAL = CUS * CLOCK_HZ * RSQ_LANES_PER_CLK_CU
# the same pair term with the rsq and the other VALU ops issued one after the
# other (they do not co-issue; packed FP32 is off): the instruction-mix ceiling
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


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(system, D, seed, sweeps=1, omp_sweeps=2):
    """The FP64 oracle on the same system and start (bounded samples): serial
    on one core (the paper's serial-CPU baseline), and its OpenMP build with
    the partner sum split over all host threads."""
    from oracle import oracle
    n = system.n
    ch = oracle.Chain(system.xyz, system.q, system.sigma, system.R, system.lB, D, seed=seed)
    t0 = time.perf_counter()
    ch.run(sweeps)
    dt = time.perf_counter() - t0
    out = {"value": sweeps * n / dt, "unit": "moves/s", "cores": 1, "kind": "oracle",
           "pair_terms_per_s": sweeps * n * (n - 1) / dt, "cpu_model": cpu_model(),
           "sample": "%d sweep(s) = %d moves of the same N=%d system and start, FP64 oracle, "
                     "1 thread, %.1f s" % (sweeps, sweeps * n, n, dt)}
    if omp_sweeps > 0:
        cm = oracle.Chain(system.xyz, system.q, system.sigma, system.R, system.lB, D, seed=seed, threaded=True)
        t0 = time.perf_counter()
        cm.run(omp_sweeps)
        dm = time.perf_counter() - t0
        out["all_cores"] = {"value": omp_sweeps * n / dm, "unit": "moves/s", "threads": cm.threads,
                            "pair_terms_per_s": omp_sweeps * n * (n - 1) / dm,
                            "sample": "%d sweep(s), OpenMP build of the oracle (partner sum over %d threads), "
                                      "%.1f s" % (omp_sweeps, cm.threads, dm)}
    return out


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


def asymmetric_leg(args, rsq_peak):
    """The size- and charge-asymmetric 2:1 system: N = 98304 (32768 at +2
    with sigma 1.0, 65536 at -1 with sigma 0.8), l_B 0.7, phi 0.1, float pair
    terms with double sums, trial cube side 1 (max displacement 0.5); the
    sweep kernel for per-ion diameters, all three g_ab(r) sampled every 10
    sweeps.  Timed with HIP events on the chain's stream."""
    import torch
    from paper_1602_05716_amd import inputs, mc
    system = inputs.asymmetric_2to1()
    n = system.n
    stream = torch.cuda.Stream()
    with mc.Chain(system.xyz, system.q, system.sigma, system.R, system.lB, precision="fp32", max_disp=0.5,
                  resum_every=100, rdf_every=10, rdf_bins=200, rdf_rmax=10.0, record_timing=1,
                  hip_stream=stream.cuda_stream) as c:
        c.sweep(args.asym_sweeps // 4, args.seed)  # warm-up launch
        c.energy()
        c.timing_reset()
        st0 = c.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.sweep(args.asym_sweeps, args.seed)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        launches, kernel_ms, kernel_sweeps = c.timing()
        st = c.stats()
        r = c.rdf()
    pairs = args.asym_sweeps * n * (n - 1)
    pair_rate = kernel_sweeps * n * (n - 1) / (kernel_ms * 1e-3)
    return {"workload": "2:1, N=98304 (32768 at +2, sigma 1.0; 65536 at -1, sigma 0.8), l_B 0.7, phi 0.1, "
                        "seeded random start, max displacement 0.5",
            "kernel": "sweep_kernel<float,%d> (per-ion diameters)" % st["waves"],
            "sweeps": args.asym_sweeps, "wall_s": wall, "ms_per_sweep": 1e3 * wall / args.asym_sweeps,
            "moves_per_s": args.asym_sweeps * n / wall, "pair_terms_per_s": pairs / wall,
            "kernel_pair_terms_per_s": pair_rate,
            "rsq_frac": 2.0 * pair_rate / rsq_peak, "band": st["band"], "workgroups": st["workgroups"],
            "acceptance": (st["accepted"] - st0["accepted"]) / max(1, st["moves"] - st0["moves"]),
            "rdf_samples": r["samples"], "g_pairs": int(r["g"].shape[0] * r["g"].shape[1])}


def large_n_leg(args, rsq_peak):
    """The same 1:1 electrolyte at N = 131072, where the launch is bound by
    the pair terms rather than by the decision chain (the library picks
    eight waves per workgroup there): move size tuned to about 40 %
    acceptance, about 2e11 pair terms timed with HIP events."""
    from paper_1602_05716_amd import compare
    r = compare.measure(args.large_n, reduction_sweeps=0)
    sk = r["sweep_kernel"]
    n = r["n"]
    rate = n * (n - 1.0) / (sk["event_ms_per_sweep"] * 1e-3)
    return {"workload": "1:1 N=%d phi=0.05 l_B=0.7, seeded random start, move size tuned to ~40%% acceptance" % n,
            "kernel": "sweep_kernel<float,%d>" % r["waves"], "band": r["band"], "sweeps": sk["sweeps"],
            "max_disp": r["max_disp"], "acceptance": sk["acceptance"], "ms_per_sweep": sk["ms_per_sweep"],
            "event_ms_per_sweep": sk["event_ms_per_sweep"], "kernel_pair_terms_per_s": rate,
            "rsq_frac": 2.0 * rate / rsq_peak}


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
    """Surrogate delayed acceptance on the N=32768 system (or the same
    electrolyte at --da-n ions): log moves of a plain run, train the network
    on the GPU, then run the two-stage chain and the plain chain from the
    same state for the same number of sweeps."""
    import torch
    from paper_1602_05716_amd import analysis, inputs, mc, surrogate
    if args.da_n == 32768:
        system = inputs.large_fp32()
    else:
        system = inputs.electrolyte(args.da_n // 2, args.da_n - args.da_n // 2, 1.0, -1.0, 1.0, 1.0, 0.05, 0.7)
        system.xyz = inputs.random_start(system, 0x5EED0002)
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
        # the same held-out moves scored with the non-learned first stage (a
        # pass with a vanishing learning rate leaves its weights as they are)
        coul = lg_chain.train_surrogate(n_log, epochs=1, batch=4096, lr=1e-12, seed=7,
                                        params_in=surrogate.truncated_coulomb_params(4.0))
        x0 = lg_chain.positions()
    out = {"workload": "1:1 N=%d phi=0.05 l_B=0.7, %d logged moves, network 128-128-128-1 bfloat16" % (n, n_log),
           "train_s": t_train, "train_loss": [float(v) for v in tr["loss"]], "val_loss": tr["val_loss"],
           "ref_stage2_reject": tr["ref_stage2_reject"],
           "coulomb_ref_stage2_reject": coul["ref_stage2_reject"], "coulomb_val_loss": coul["val_loss"],
           "sweeps": args.da_sweeps}
    runs = {}
    nets = {"da": (tr["params"], tr["ref_stage2_reject"]), "da_coulomb": (coul["params"], coul["ref_stage2_reject"])}
    for mode in ("plain", "da", "da_coulomb"):
        kw = dict(precision="fp32", max_disp=md, resum_every=100, hip_stream=stream.cuda_stream, rdf_bins=200,
                  rdf_rmax=10.0)
        if mode != "plain":
            kw["waves"] = 4
            kw["band"] = args.da_band
        with mc.Chain(x0, system.q, system.sigma, system.R, system.lB, **kw) as c:
            if mode != "plain":
                c.set_surrogate(nets[mode][0], nets[mode][1], True)
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
    keys = ("wall_s", "ess", "ess_per_s", "moves_per_s", "acceptance")
    sp = runs["plain"]["stats"]
    moves = max(1, sp["moves"])
    out["plain"] = {k: v for k, v in runs["plain"].items() if k in keys}
    out["plain"].update({"rejected_wall": sp["rejected_wall"], "rejected_overlap": sp["rejected_overlap"]})
    for mode in ("da", "da_coulomb"):
        out[mode] = {k: v for k, v in runs[mode].items() if k in keys}
        sd = runs[mode]["stats"]
        out[mode].update({"stage1_rejected": sd["da_stage1_rejected"], "stage1_passed": sd["da_stage1_passed"],
                          "stage2_rejected": sd["da_stage2_rejected"], "conflict_moves": sd["da_conflicts"],
                          "two_stage_moves": sd["da_moves"], "fallback_sweep": sd["da_fallback_sweep"],
                          "active_at_end": sd["da_active"], "rejected_wall": sd["rejected_wall"],
                          "rejected_overlap": sd["rejected_overlap"],
                          "stage2_reject_rate": sd["da_stage2_rejected"] / max(1, sd["da_stage1_passed"]),
                          "g_rms_vs_plain": rms(runs[mode]["g"], runs["plain"]["g"])})
    out["g_rms_da_vs_plain"] = out["da"]["g_rms_vs_plain"]
    out["g_rms_plain_half_vs_half"] = rms(ph[0]["g"], ph[1]["g"])
    out["ess_per_s_da_over_plain"] = out["da"]["ess_per_s"] / out["plain"]["ess_per_s"]
    out["ess_per_s_coulomb_over_plain"] = out["da_coulomb"]["ess_per_s"] / out["plain"]["ess_per_s"]
    # What a kernel that skipped the exact work of moves rejected early (with
    # survivor compaction, which this kernel does not do) could gain at most:
    # the fraction of moves that would still need the exact pair sum.  Wall
    # rejections are known from the trial position alone; overlap rejections
    # by an exact cell-list test (non-learned); stage-1 rejections of moves
    # without a conflict by the learned first stage.
    sd = runs["da"]["stats"]
    wall_f = sp["rejected_wall"] / moves
    ov_f = sp["rejected_overlap"] / moves
    s1_f = sd["da_stage1_rejected"] / max(1, sd["moves"])
    out["exact_work_bound"] = {
        "plain": 1.0,
        "wall_prerejection": 1.0 - wall_f,
        "wall_and_overlap_prerejection": 1.0 - wall_f - ov_f,
        "learned_stage1_and_prerejection_at_least": 1.0 - wall_f - ov_f - s1_f,
        "note": "fractions of moves needing the exact O(N) sum; ideal speed-up = 1 / fraction, before the cost "
                "of compaction and of the lower acceptance of the two-stage chain"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps-per-step", type=int, default=500)
    ap.add_argument("--seed", type=int, default=0x5EED0002)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=1)
    ap.add_argument("--cpu-omp-sweeps", type=int, default=2,
                    help="sweeps of the oracle's OpenMP build on all host threads (0: skip)")
    ap.add_argument("--no-probe", action="store_true", help="skip the VALU issue-rate probe")
    ap.add_argument("--band", type=int, default=-1)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--no-asym", action="store_true", help="skip the 2:1 N=98304 leg")
    ap.add_argument("--asym-sweeps", type=int, default=40)
    ap.add_argument("--large-n", type=int, default=131072,
                    help="ions of the pair-term-bound 1:1 leg (0: skip it)")
    ap.add_argument("--batch-sweeps", type=int, default=1000)
    ap.add_argument("--seq-sweeps", type=int, default=20)
    ap.add_argument("--no-da", action="store_true", help="skip the surrogate delayed-acceptance leg")
    ap.add_argument("--da-log-moves", type=int, default=1000000)
    ap.add_argument("--da-epochs", type=int, default=6)
    ap.add_argument("--da-sweeps", type=int, default=1500)
    ap.add_argument("--da-n", type=int, default=32768, help="ions of the surrogate leg's 1:1 system")
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
                     max_disp=0.5, resum_every=100, record_timing=1,
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
    pair_rate = per_launch_pairs / avg_launch_s
    probe = None if args.no_probe else run_valu_probe()
    rsq_peak = probe["rsq_per_s"] if probe else RSQ_PEAK_NOMINAL
    achieved = RSQ_PER_PAIR * pair_rate / 1e12
    peak = rsq_peak / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "T v_rsq_f32/s",
                "frac": achieved / peak, "traffic": traffic_per_launch(kernel_sweeps / max(1, launches)),
                "per_unit": "pair term = %d v_rsq_f32 (+ %d other VALU lane-ops)" % (RSQ_PER_PAIR, VALU_PER_PAIR),
                "peak_source": "v_rsq_f32 rate measured by the valu_peak probe" if probe else
                               "nominal 32 rsq lanes per clock per CU at 2.4 GHz",
                "pair_terms_per_s": pair_rate,
                "kernel": "sweep_kernel<float,%d>" % st1["waves"],
                "avg_launch_ms": avg_launch_s * 1e3, "launches": launches,
                "sweeps_per_launch": kernel_sweeps / max(1, launches)}
    # the instruction-mix ceiling: rsq and the other VALU ops issued one after
    # the other, at the nominal and at the probe's measured lane rates
    mix = {"pair_peak_nominal": PAIR_PEAK_PER_S / 1e12, "frac_nominal": pair_rate / PAIR_PEAK_PER_S,
           "rsq_frac_attainable_nominal": RSQ_PER_PAIR * PAIR_PEAK_PER_S / RSQ_PEAK_NOMINAL, "unit": "Tpairterm/s"}
    if probe:
        clk_per_pair = (VALU_PER_PAIR / probe["fma_lanes_per_clk_cu"] +
                        RSQ_PER_PAIR / probe["rsq_lanes_per_clk_cu"])
        pair_peak_probe = CUS * CLOCK_HZ / clk_per_pair
        mix.update({"pair_peak_probe": pair_peak_probe / 1e12, "frac_probe": pair_rate / pair_peak_probe,
                    "rsq_frac_attainable_probe": RSQ_PER_PAIR * pair_peak_probe / rsq_peak})
        roofline["probe"] = probe
    roofline["instruction_mix_ceiling"] = mix
    reduction = None
    if not args.no_reduction:
        log("per-move parallel-reduction leg (%d sweep(s))" % args.reduction_sweeps)
        reduction = reduction_leg(chain, args, moves / elapsed)

    asym = None
    if not args.no_asym:
        log("2:1 N=98304 leg (%d sweeps)" % args.asym_sweeps)
        asym = asymmetric_leg(args, rsq_peak)

    large = None
    if args.large_n > 0:
        log("1:1 N=%d leg" % args.large_n)
        large = large_n_leg(args, rsq_peak)

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
        cpu = cpu_baseline(system, 2.0 * md, args.seed, args.cpu_sweeps, args.cpu_omp_sweeps)
        cpu["cores_available"] = os.cpu_count()
        cpu["gpu_over_cpu"] = (moves / elapsed) / cpu["value"]
        if "all_cores" in cpu:
            cpu["all_cores"]["gpu_over_cpu"] = (moves / elapsed) / cpu["all_cores"]["value"]

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
        "asymmetric_2to1": asym,
        "large_n": large,
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
