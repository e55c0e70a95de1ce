"""Per-group latency breakdown of the decision chain (diagnostic build).

``build()`` compiles ``libmc_timeline.so`` with ``-DMC_TIMELINE``: the float
sweep kernel then writes device wall-clock stamps (100 MHz) into the dE trace
buffer instead of dE values, 32 64-bit words per group g:

====  ========================================================================
slot  stamp (chain wave unless noted)
====  ========================================================================
0     chain step entered (after the wave's own share and hand-off)
1     every wave's hand-off complete
2     accept mask of group g-1 seen
3     group g published
4     g-1's masked row added
5     last evaluation done (speculative path)
6     wait for g-1's mask begun (speculative path)
7     evaluations after g-1's mask (a count, not a stamp)
8     partial sums combined
9     helper's sums received (speculative path; after the early check otherwise)
10    first solve done (speculative path)
11    target's work begun (wave 0)
12    decided partner tiles done (wave 0)
13    older band groups folded (wave 0); 21-23: waves 1-3
14    last decided tile seen (wave 0); 25-27: waves 1-3
16-19 hand-off counted, waves 0-3
28    helper wave done
====  ========================================================================

``run()`` sweeps the N = 32768 benchmark system with the diagnostic library
(after untimed warm-up sweeps) and returns percentiles (10, 50, 90, 99) of
the stages in microseconds, over the timed sweeps after their first.  The
stamps cost time themselves: the diagnostic build runs about a quarter
slower than the plain one.

    python -m paper_1602_05716_amd.timeline --build --max-disp 5.2 --band 4
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess

import numpy as np

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmc_timeline.so")
SLOTS = 32


def build(verbose: bool = False) -> str:
    cmd = [_build.HIPCC] + _build.FLAGS + ["-DMC_TIMELINE", "-I", os.path.join(HERE, "..", "include"),
                                           "-o", LIB] + [os.path.join(_build.CSRC, s) for s in _build.SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return LIB


def _pct(a):
    a = np.asarray(a, dtype=np.float64)
    if a.size == 0:
        return None
    return [round(float(np.percentile(a, q)), 3) for q in (10, 50, 90, 99)]


def run(max_disp: float = 5.2, band: int = -1, sweeps: int = 6, warmup: int = 2) -> dict:
    from . import inputs, mc
    mc._lib = mc.load(LIB)
    sy = inputs.large_fp32()
    nb = (sy.n + 63) // 64
    total = warmup + sweeps
    cap = SLOTS * nb * total
    with mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, precision="fp32", max_disp=max_disp, resum_every=0,
                  trace_moves=cap, record_timing=1, band=band) as ch:
        ch.sweep(warmup, 1)  # the process's first launch is slower: untimed
        ch.timing_reset()
        ch.sweep(sweeps, 2)
        _, de = ch.trace(min(cap, total * sy.n))
        _, ms, sw = ch.timing()
        st = ch.stats()
    tl = de.view(np.uint64).reshape(-1, SLOTS).astype(np.int64)[(warmup + 1) * nb: total * nb]
    us = 1e-2  # 100 MHz ticks -> microseconds
    t0, t1, t2, t3 = tl[:, 0], tl[:, 1], tl[:, 2], tl[:, 3]
    t4, t5, t6 = tl[:, 4], tl[:, 5], tl[:, 6]
    t11, t12, t13, t14 = tl[:, 11], tl[:, 12], tl[:, 13], tl[:, 14]
    spec = t5 > 0
    late = t6[1:] > t3[:-1]
    kl = st["band"] + 1
    return {
        "max_disp": max_disp, "band": st["band"], "ms_per_sweep": ms / sw,
        "early_fraction": st["early_groups"] / (st["moves"] / 64),
        "hop_us": _pct(np.diff(t3) * us),
        "handoff_after_predecessor_us": _pct((t1[1:] - t3[:-1]) * us),
        "chain_prework_us": _pct(((t6 - t1) * us)[spec]),
        "wait_begins_after_predecessor_fraction": float(np.mean(late[spec[1:]])) if spec[1:].any() else None,
        "mask_detection_us": _pct(((t2[1:] - np.maximum(t3[:-1], t6[1:])) * us)[spec[1:]]),
        "post_mask_us": _pct(((t3 - t2) * us)[spec]),
        "masked_row_us": _pct(((t4 - t2) * us)[spec]),
        "evaluations_after_mask": _pct(tl[:, 7][spec]),
        # the last decided partner tile of target g is group g - band - 1
        "last_tile_seen_after_publication_us": _pct(((t14[kl:] - t3[:-kl]) * us)[t14[kl:] > 0]),
        "last_tile_compute_us": _pct(((t12 - t14) * us)[t14 > 0]),
        "tiles_phase_us": _pct(((t12 - t11) * us)[t11 > 0]),
        "fold_to_handoff_us": _pct(((t1 - t13) * us)[t13 > 0]),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--build", action="store_true", help="compile the diagnostic library first")
    ap.add_argument("--max-disp", type=float, default=5.2)
    ap.add_argument("--band", type=int, default=-1)
    ap.add_argument("--sweeps", type=int, default=6)
    a = ap.parse_args()
    if a.build:
        build(verbose=True)
    print(json.dumps(run(a.max_disp, a.band, a.sweeps)), flush=True)


if __name__ == "__main__":
    main()
