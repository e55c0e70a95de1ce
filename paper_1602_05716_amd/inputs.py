"""Seeded synthetic inputs: primitive-model electrolytes in a hard-wall sphere.

This module builds initial states only (charges, diameters, wall radius and a
non-overlapping random start); it contains none of the Monte Carlo method's
arithmetic and is shared by the library's users, the tests and the benchmark.

Paper: Liang, Xing, Li, arXiv:1602.05716, Sec. 5.2 -- charged hard spheres in
a spherical domain with a hard wall, started from a uniform random placement
without hard-core overlap.  The paper's own runs use 2^20 ions in physical
units; the systems here are the reduced-unit workloads (diameter 1) of the
benchmark configurations, with the wall radius fixed by the ion volume
fraction phi = sum_i sigma_i^3 / (8 R^3).

Ion order: all cations first, then all anions (the sequential updating scheme
tries ions in index order; positions are independent of the index).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class System:
    """An electrolyte: per-ion charge/diameter, wall radius, Bjerrum length."""

    q: np.ndarray
    sigma: np.ndarray
    R: float
    lB: float
    xyz: np.ndarray | None = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.q)

    def types(self):
        """Species index per ion (distinct (q, sigma) pairs, cations first)."""
        keys = sorted({(float(a), float(b)) for a, b in zip(self.q, self.sigma)},
                      key=lambda t: (-t[0], t[1]))
        lut = {k: i for i, k in enumerate(keys)}
        t = np.array([lut[(float(a), float(b))] for a, b in zip(self.q, self.sigma)], np.int32)
        return t, keys


def radius_for_fraction(sigma, phi: float) -> float:
    """R such that sum sigma^3 / (8 R^3) = phi."""
    return float((np.sum(np.asarray(sigma, np.float64) ** 3) / (8.0 * phi)) ** (1.0 / 3.0))


def electrolyte(n_cation: int, n_anion: int, q_cation: float, q_anion: float,
                sigma_cation: float, sigma_anion: float, phi: float, lB: float,
                name: str = "") -> System:
    q = np.concatenate([np.full(n_cation, q_cation), np.full(n_anion, q_anion)]).astype(np.float64)
    s = np.concatenate([np.full(n_cation, sigma_cation),
                        np.full(n_anion, sigma_anion)]).astype(np.float64)
    return System(q=q, sigma=s, R=radius_for_fraction(s, phi), lB=float(lB), name=name,
                  meta={"phi": phi})


def random_start(system: System, seed: int, batch: int = 4096, max_rounds: int = 100000) -> np.ndarray:
    """Random sequential addition inside the wall, no hard-core overlap.

    Ions of one species are interchangeable, so each species block (in index
    order) is filled by a stream of candidate centres, uniform in the ball of
    radius R - sigma/2; a candidate is kept when it overlaps no ion kept
    before it (contact allowed).  Candidates are drawn in batches and screened
    with k-d trees, which keeps exactly the candidates one-at-a-time addition
    would keep from the same stream.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    n = system.n
    sig = system.sigma
    smax = float(sig.max()) if n else 1.0
    xyz = np.zeros((n, 3), np.float64)
    placed = 0
    # kept ions are indexed by two k-d trees: one over xyz[:big_n], rebuilt
    # only when the other, over the ions kept since, has grown to a quarter
    # of it (the candidates tested are the same as with one tree)
    trees = []
    big_n = 0
    rounds = 0
    while placed < n:
        rounds += 1
        if rounds > max_rounds:
            raise RuntimeError("random_start: packing too dense for random sequential addition")
        s_here = sig[placed]
        end = placed
        while end < n and sig[end] == s_here:
            end += 1
        need = end - placed
        m = min(batch, 2 * need + 16)
        a = system.R - 0.5 * s_here
        v = rng.normal(size=(m, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        rad = a * rng.random(m) ** (1.0 / 3.0)
        cand = v * rad[:, None]
        ok = np.ones(m, bool)
        for tree, base in trees:
            hits = tree.query_ball_point(cand, r=smax)
            for k in np.flatnonzero(np.fromiter(map(len, hits), np.int64, m)):
                if not ok[k]:
                    continue
                for j in hits[k]:
                    j += base
                    d = np.sqrt(np.sum((cand[k] - xyz[j]) ** 2))
                    if d < 0.5 * (s_here + sig[j]):
                        ok[k] = False
                        break
        # within a batch an earlier kept candidate wins over a later one; the
        # pairs come sorted by first index, so ok[k1] is final when tested
        btree = cKDTree(cand)
        for k1, k2 in sorted(btree.query_pairs(r=s_here)):
            if ok[k1] and ok[k2]:
                d = np.sqrt(np.sum((cand[k1] - cand[k2]) ** 2))
                if d < s_here:
                    ok[k2] = False
        kept = cand[ok][:need]
        xyz[placed:placed + len(kept)] = kept
        placed += len(kept)
        if placed - big_n > max(batch, big_n // 4):
            big_n = placed
            trees = [(cKDTree(xyz[:placed]), 0)]
        else:
            trees = trees[:1] if big_n else []
            trees.append((cKDTree(xyz[big_n:placed]), big_n))
    return xyz


# --------------------------------------------------------------------------- #
# Named workloads                                                             #
# --------------------------------------------------------------------------- #

def small_fp64(seed: int = 0x5EED0001) -> System:
    """1:1, N = 1000, sigma = 1, l_B = 0.7, phi = 0.01 (double precision workload)."""
    s = electrolyte(500, 500, 1.0, -1.0, 1.0, 1.0, 0.01, 0.7, name="1:1 N=1000 phi=0.01 lB=0.7")
    s.xyz = random_start(s, seed)
    s.meta.update(max_disp=0.5, sweeps=200, rdf_bins=200, rdf_rmax=10.0, seed=seed)
    return s


def large_fp32(seed: int = 0x5EED0002) -> System:
    """1:1, N = 32768, sigma = 1, l_B = 0.7, phi = 0.05 (FP32 pair terms, FP64 sums)."""
    s = electrolyte(16384, 16384, 1.0, -1.0, 1.0, 1.0, 0.05, 0.7,
                    name="1:1 N=32768 phi=0.05 lB=0.7")
    s.xyz = random_start(s, seed)
    s.meta.update(sweeps=10000, target_acceptance=0.40, seed=seed)
    return s


def asymmetric_2to1(seed: int = 0x5EED0003) -> System:
    """2:1, N = 98304 (32768 at +2 with sigma 1.0, 65536 at -1 with sigma 0.8), l_B = 0.7, phi = 0.1."""
    s = electrolyte(32768, 65536, 2.0, -1.0, 1.0, 0.8, 0.1, 0.7,
                    name="2:1 N=98304 phi=0.1 lB=0.7")
    s.xyz = random_start(s, seed)
    s.meta.update(sweeps=2000, rdf_bins=200, rdf_rmax=10.0, seed=seed)
    return s


def ensemble_params(n_chains: int = 256, seed: int = 0x5EED0004):
    """Per-chain (N, phi, l_B, seed) of the batched ensemble.

    N is log-uniform on [500, 8000] rounded to an even number (1:1, neutral),
    phi uniform on [0.005, 0.1], l_B uniform on [0.5, 2.0].
    """
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n_chains):
        n = int(2 * round(0.5 * np.exp(rng.uniform(np.log(500.0), np.log(8000.0)))))
        phi = float(rng.uniform(0.005, 0.1))
        lB = float(rng.uniform(0.5, 2.0))
        out.append((n, phi, lB, seed + 1 + c))
    return out


def ensemble_chain(n: int, phi: float, lB: float, seed: int) -> System:
    s = electrolyte(n // 2, n // 2, 1.0, -1.0, 1.0, 1.0, phi, lB,
                    name=f"1:1 N={n} phi={phi:.4f} lB={lB:.3f}")
    s.xyz = random_start(s, seed)
    s.meta.update(seed=seed)
    return s


# The paper's production electrolyte (Sec. 5.2): 3:-1, ion diameter 7.5 A
# (radius 3.75 A), Bjerrum length 7.117 A, bare Debye length 28.53 A.  In
# units of the diameter: l_B = 7.117 / 7.5; the cation density follows from
# kappa^2 = 4 pi l_B (n_+ 9 + n_- 1) with n_- = 3 n_+.
PAPER_DIAMETER_A = 7.5
PAPER_BJERRUM_A = 7.117
PAPER_DEBYE_A = 28.53


def three_to_one_density(debye_A: float = PAPER_DEBYE_A) -> tuple[float, float]:
    """(n_+, n_-) in ions per diameter^3 of the paper's 3:-1 electrolyte at the
    bare Debye length debye_A (Angstrom; 28.53 is the paper's system)."""
    lB = PAPER_BJERRUM_A / PAPER_DIAMETER_A
    kappa = PAPER_DIAMETER_A / debye_A
    n_plus = kappa * kappa / (4.0 * np.pi * lB * (9.0 + 3.0))
    return n_plus, 3.0 * n_plus


def three_to_one(n: int = 1 << 20, seed: int = 0x5EED0007, debye_A: float = PAPER_DEBYE_A,
                 start: bool = True) -> System:
    """The paper's 3:-1 system with n ions (n / 4 at +3, 3 n / 4 at -1, all
    of diameter 1 = 7.5 A), at the density of bare Debye length debye_A
    (the paper's 28.53 A: phi = (n_+ + n_-) pi / 6, about 1.0e-3), in a
    hard-wall sphere; uniform random start without overlap (none with
    start=False, for a chain resumed from a checkpoint)."""
    if n % 4:
        raise ValueError("n must be a multiple of 4")
    n_plus, n_minus = three_to_one_density(debye_A)
    phi = (n_plus + n_minus) * np.pi / 6.0
    s = electrolyte(n // 4, 3 * n // 4, 3.0, -1.0, 1.0, 1.0, phi, PAPER_BJERRUM_A / PAPER_DIAMETER_A,
                    name=f"3:-1 N={n}, bare Debye length {debye_A} A (diameter 7.5 A)")
    if start:
        s.xyz = random_start(s, seed)
    s.meta.update(seed=seed, kappa_inv=debye_A / PAPER_DIAMETER_A, phi=phi, debye_A=debye_A)
    return s
