"""Sequential-sweep kernel against the per-move parallel-reduction scheme over
system size: the shape of the paper's GPU comparison (Liang, Xing, Li,
arXiv:1602.05716, Sec. 4: execution time per Monte Carlo cycle of both GPU
codes, and their ratio).

For each N: a 1:1 system (sigma = 1, l_B = 0.7, phi = 0.05, seeded random
start), its move size tuned to about 40 % acceptance on the sweep kernel,
then the same chain timed by both schemes -- ``sweeps`` sweeps of mc_sweep
and ``reduction_sweeps`` of mc_sweep_reduction (one launch per move) --
with HIP events around each stretch and the wall clock.  One JSON line per N.

    python -m paper_1602_05716_amd.compare --ns 8192 16384 32768 65536 131072

With --waves and --band lists (and --reduction-sweeps 0) it times the sweep
kernel alone over its launch shapes: the counterpart of the paper's search
for the best threads per particle (Sec. 4, Table Para).
"""
from __future__ import annotations

import argparse
import json
import time


def _tune(ch, md, rounds=6, sweeps=2, target=0.40, seed=0xD15C):
    for r in range(rounds):
        ch.set_max_disp(md)
        a = ch.stats()
        ch.sweep(sweeps, seed + r)
        b = ch.stats()
        acc = (b["accepted"] - a["accepted"]) / max(1, b["moves"] - a["moves"])
        md *= min(2.0, max(0.5, acc / target))
    ch.set_max_disp(md)
    return md


def _timed(ch, fn, sweeps, seed):
    ch.timing_reset()
    ch.energy()  # synchronises the chain's stream
    t0 = time.perf_counter()
    fn(sweeps, seed)
    ch.energy()  # synchronises the chain's stream
    wall = time.perf_counter() - t0
    _, ms, sw = ch.timing()
    return wall, ms * 1e-3


def measure(n: int, sweeps: int = 0, reduction_sweeps: int = 1, seed: int = 0x5EED0006, waves: int = 0,
            band: int = -1) -> dict:
    from . import inputs, mc
    sy = inputs.electrolyte(n // 2, n - n // 2, 1.0, -1.0, 1.0, 1.0, 0.05, 0.7)
    sy.xyz = inputs.random_start(sy, seed)
    if sweeps <= 0:  # about 2e11 pair terms, at least 2 sweeps
        sweeps = max(2, int(2e11 / (n * (n - 1.0))))
    with mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, precision="fp32", max_disp=0.5, resum_every=0,
                  record_timing=1, waves=waves, band=band) as ch:  # the handle's own stream
        md = _tune(ch, 0.5)
        st0 = ch.stats()
        w_s, k_s = _timed(ch, ch.sweep, sweeps, seed)
        st1 = ch.stats()
        if reduction_sweeps > 0:
            w_r, k_r = _timed(ch, ch.sweep_reduction, reduction_sweeps, seed)
        st2 = ch.stats()
    pairs = n * (n - 1.0)
    acc_s = (st1["accepted"] - st0["accepted"]) / max(1, st1["moves"] - st0["moves"])
    out = {"n": n, "max_disp": md, "waves": st1["waves"], "band": st1["band"],
           "sweep_kernel": {"sweeps": sweeps, "ms_per_sweep": 1e3 * w_s / sweeps,
                            "event_ms_per_sweep": 1e3 * k_s / sweeps, "acceptance": acc_s,
                            "pair_terms_per_s": sweeps * pairs / w_s}}
    if reduction_sweeps > 0:
        acc_r = (st2["accepted"] - st1["accepted"]) / max(1, st2["moves"] - st1["moves"])
        out["reduction"] = {"sweeps": reduction_sweeps, "ms_per_sweep": 1e3 * w_r / reduction_sweeps,
                            "event_ms_per_sweep": 1e3 * k_r / reduction_sweeps, "acceptance": acc_r,
                            "us_per_move": 1e6 * w_r / (reduction_sweeps * n),
                            "pair_terms_per_s": reduction_sweeps * pairs / w_r}
        out["sweep_kernel_speedup"] = (w_r / reduction_sweeps) / (w_s / sweeps)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--ns", type=int, nargs="+", default=[8192, 16384, 32768, 65536, 131072])
    ap.add_argument("--sweeps", type=int, default=0, help="sweep-kernel sweeps (0: about 2e11 pair terms)")
    ap.add_argument("--reduction-sweeps", type=int, default=1, help="0: the sweep kernel only")
    ap.add_argument("--waves", type=int, nargs="+", default=[0], help="waves per workgroup (0: automatic)")
    ap.add_argument("--band", type=int, nargs="+", default=[-1], help="look-ahead band (-1: automatic)")
    a = ap.parse_args()
    for n in a.ns:
        for w in a.waves:
            for b in a.band:
                print(json.dumps(measure(n, a.sweeps, a.reduction_sweeps, waves=w, band=b)), flush=True)


if __name__ == "__main__":
    main()
