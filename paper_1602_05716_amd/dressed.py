"""The paper's production measurement (Liang, Xing, Li, arXiv:1602.05716,
Sec. 5): a 3:-1 primitive-model electrolyte at the bare Debye length
28.53 A, its pair correlation functions sampled far from the wall, and the
renormalised parameters of the dressed-ion theory from their tails (Sec. 5.1).

The chain runs on the GPU (FP32 pair terms, FP64 sums); trial moves are cubes
of side about L / 3 (L = 2 R, the domain size), as in the paper.  g(r) is
sampled every ``every`` sweeps after ``equil`` equilibration sweeps, with
centres at least ``rmax`` + ten bare Debye lengths inside the wall, so that
every neighbour counted lies in the bulk (the paper leaves ions within ten
Debye lengths of the wall out of the data).  The
raw counts, centre counts and the energy series go to ``--out`` (npz); the
analysis is printed as one JSON line, lengths also in Angstrom (diameter
7.5 A) beside the paper's values for context.

    python -m paper_1602_05716_amd.dressed --n 262144 --sweeps 1000 --out dressed.npz
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import analysis, inputs

# the paper's measured values (Sec. 5.1, Figs. logrrho and rhoU), for context
PAPER_KAPPA_R_INV_A = 25.57
PAPER_QR = (4.125, -0.884)
PAPER_TAU_INT = 2.3


def _log(*a):
    print("[dressed]", *a, file=sys.stderr, flush=True)


def run(n: int, sweeps: int, equil: int, every: int, rmax: float, bins: int, seed: int, chunk: int = 100,
        margin: float | None = None, debye_A: float = inputs.PAPER_DEBYE_A, trace: bool = False,
        save: str = "", resume: str = ""):
    """With `resume`, the chain continues from a checkpoint written by an
    earlier run's `save` (same system, seed and sampling options): no
    equilibration, and the g(r) counts go on accumulating from the saved ones."""
    from . import mc
    t0 = time.perf_counter()
    sy = inputs.three_to_one(n, seed, debye_A, start=not resume)
    _log("system built: N=%d R=%.2f (%.1f s)" % (n, sy.R, time.perf_counter() - t0))
    md = sy.R / 3.0  # cube side 2 md = L / 3
    if margin is None:  # every neighbour counted at least ten bare Debye lengths inside the wall
        margin = 10.0 * sy.meta["kappa_inv"]
    # the handle's own stream: nothing here needs another GPU runtime
    if resume:
        chain = mc.Chain.load(resume)
        o = chain.opt
        if (chain.n != n or o.rdf_every != every or o.rdf_bins != bins or o.rdf_rmax != rmax
                or abs(o.rdf_margin - margin) > 1e-12 * max(1.0, margin)):
            chain.close()
            raise ValueError("the checkpoint was written for another system or g(r) sampling")
    else:
        chain = mc.Chain(sy.xyz, sy.q, sy.sigma, sy.R, sy.lB, precision="fp32", max_disp=md, resum_every=100,
                         rdf_every=every, rdf_bins=bins, rdf_rmax=rmax, rdf_margin=margin,
                         trace_moves=(equil + sweeps) * n if trace else 0)
    with chain as ch:
        if not resume:
            done = 0
            while done < equil:
                k = min(chunk, equil - done)
                ch.sweep(k, seed)
                ch.energy()
                done += k
                _log("equilibration %d / %d sweeps" % (done, equil))
            ch.rdf_reset()
        s0 = ch.stats()["sweeps"]
        t1 = time.perf_counter()
        done = 0
        while done < sweeps:
            k = min(chunk, sweeps - done)
            ch.sweep(k, seed)
            ch.energy()
            done += k
            _log("production %d / %d sweeps (%.1f s)" % (done, sweeps, time.perf_counter() - t1))
        wall = time.perf_counter() - t1
        r = ch.rdf()
        st = ch.stats()
        es = ch.energy_series(st["sweeps"])[s0:]
        e_run, e_ex = ch.energy(exact=True)
        if trace:
            st["trace"] = ch.trace((equil + sweeps) * n)
        if save:
            ch.save(save)
            _log("checkpoint written: %s (sweep %d)" % (save, st["sweeps"]))
    types, keys = sy.types()
    n_of_type = np.bincount(types, minlength=len(keys))
    return sy, md, r, st, es, wall, n_of_type, (e_run, e_ex), margin


def analyse(r_c, g, n_of_type, R, fit, r_flat=None, counts=None):
    """Dressed-ion parameters of one run (or of pooled counts); with the raw
    counts the fit is weighted by their Poisson errors."""
    vb = 4.0 / 3.0 * np.pi * (R - 0.5) ** 3
    n = n_of_type / vb
    q = [3.0, -1.0]
    err = None if counts is None else analysis.charge_density_error(counts, g, n, q)
    res = analysis.renormalised_parameters(r_c, g, n, q, inputs.PAPER_BJERRUM_A / inputs.PAPER_DIAMETER_A,
                                           fit=fit, r_flat=r_flat, rho_err=err)
    d = inputs.PAPER_DIAMETER_A
    out = {k: v for k, v in res.items() if k not in ("rho", "U")}
    out.update({"fit_window_sigma": list(fit), "kappa_inv_A": d / res["kappa"], "kappa_R_inv_A": d / res["kappa_R"],
                "paper": {"kappa_R_inv_A": PAPER_KAPPA_R_INV_A, "kappa_inv_A": inputs.PAPER_DEBYE_A,
                          "qR": list(PAPER_QR)}})
    return out


def pooled(paths, fit, r_flat=None) -> dict:
    """Analysis of the summed counts of several saved runs of one system
    (independent chains: the ensemble and time average of the paper)."""
    runs = [np.load(p) for p in paths]
    ref = runs[0]
    for d in runs[1:]:
        if (int(d["n"]) != int(ref["n"]) or float(d["rmax"]) != float(ref["rmax"])
                or int(d["bins"]) != int(ref["bins"]) or float(d.get("margin", 0.0)) != float(ref.get("margin", 0.0))):
            raise ValueError("runs of different systems or histograms")
    counts = sum(d["counts"].astype(np.float64) for d in runs)
    centres = sum(d["centres"].astype(np.float64) for d in runs)
    R, rmax = float(ref["R"]), float(ref["rmax"])
    r_c, g = analysis.g_from_counts(counts, centres, ref["n_of_type"], [1.0, 1.0], R, rmax)
    out = analyse(r_c, g, ref["n_of_type"], R, fit, r_flat, counts=counts)
    out.update({"runs": len(runs), "samples": int(sum(int(d["samples"]) for d in runs)),
                "tau_int_sweeps": [analysis.integrated_time(d["energy"]) for d in runs]})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=1 << 18)
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--equil", type=int, default=100)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--debye-A", type=float, default=inputs.PAPER_DEBYE_A,
                    help="bare Debye length in Angstrom (sets the density)")
    ap.add_argument("--rmax", type=float, default=0.0,
                    help="g(r) range in diameters (0: 10.5 bare Debye lengths)")
    ap.add_argument("--bins", type=int, default=400)
    ap.add_argument("--seed", type=int, default=0x5EED0007)
    ap.add_argument("--chunk", type=int, default=100, help="sweeps per call (progress lines)")
    ap.add_argument("--fit", type=float, nargs=2, default=[0.0, 0.0],
                    help="far-field window in diameters (0 0: 4.2 to 7.9 bare Debye lengths)")
    ap.add_argument("--out", default="")
    ap.add_argument("--save", default="", help="write a checkpoint of the chain at the end")
    ap.add_argument("--resume", default="",
                    help="continue the chain of this checkpoint (same system and sampling options)")
    ap.add_argument("--pool", nargs="+", default=None,
                    help="analysis only (no GPU): pool the counts of these saved runs of one system")
    a = ap.parse_args()
    lam = a.debye_A / inputs.PAPER_DIAMETER_A  # bare Debye length in diameters
    if a.rmax <= 0:
        a.rmax = round(10.5 * lam, 1)
    if a.fit[1] <= 0:
        a.fit = [round(4.2 * lam, 1), round(7.9 * lam, 1)]
    if a.pool:
        print(json.dumps(pooled(a.pool, tuple(a.fit))), flush=True)
        return
    sy, md, r, st, es, wall, n_of_type, (e_run, e_ex), margin = run(a.n, a.sweeps, a.equil, a.every, a.rmax, a.bins, a.seed,
                                                             a.chunk, debye_A=a.debye_A, save=a.save,
                                                             resume=a.resume)
    dr = a.rmax / a.bins
    r_c = (np.arange(a.bins) + 0.5) * dr
    if a.out:
        np.savez(a.out, counts=r["counts"], centres=r["centres"], samples=r["samples"], g=r["g"],
                 n_of_type=n_of_type, R=sy.R, rmax=a.rmax, bins=a.bins, energy=es, max_disp=md, n=a.n,
                 margin=margin, debye_A=a.debye_A)
    tau = analysis.integrated_time(es) if len(es) > 8 else float("nan")
    out = {"n": a.n, "debye_A": a.debye_A, "R": sy.R, "max_disp": md, "rdf_margin": margin, "rmax": a.rmax,
           "sweeps": a.sweeps, "equil": 0 if a.resume else a.equil, "every": a.every,
           "resumed_at_sweep": (st["sweeps"] - a.sweeps) if a.resume else None, "total_sweeps": st["sweeps"],
           "samples": r["samples"], "wall_s": wall, "ms_per_sweep": 1e3 * wall / max(1, a.sweeps),
           "acceptance": st["accepted"] / max(1, st["moves"]), "tau_int_sweeps": tau,
           "paper_tau_int": PAPER_TAU_INT, "e_running": e_run, "e_resum": e_ex,
           "rejected_wall": st["rejected_wall"], "rejected_overlap": st["rejected_overlap"]}
    try:
        out["dressed"] = analyse(r_c, r["g"], n_of_type, sy.R, tuple(a.fit), counts=r["counts"])
    except ValueError as e:  # a noisy window: the raw counts are saved for another fit
        out["dressed_error"] = str(e)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
