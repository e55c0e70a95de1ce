"""ctypes front end of the C oracle plus the oracle's host-side analysis.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the library.  The GPU path shares
no code with it.

Paper: Liang, Xing, Li, arXiv:1602.05716.  The C part (mc_oracle.c) holds the
Markov chain itself; this module adds
  * g_ab(r) normalisation of the integer pair counts (Sec. 5.2, pair
    correlation functions),
  * the integrated autocorrelation time T_c = 1/2 + sum_k C_k of the energy
    series (Sec. 5.2, definitions of C_n and T_c), the sum stopped at the
    first non-positive sum of a pair of lags (the paper does not say where
    to stop it),
  * Debye-Hueckel closed forms (Sec. 5.1, Eq. (alpha-kappa_0) and the PB pair
    potential) used by the dilute-limit test.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mc_oracle.c")
_LIB = os.path.join(_HERE, "libmc_oracle.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)


_LIB_OMP = os.path.join(_HERE, "libmc_oracle_omp.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fused multiply-add), and its
    OpenMP build, which only the CPU timing uses."""
    for lib_path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(_SRC):
            tmp = lib_path + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                                   "-std=c99", "-fPIC", "-shared"] + extra + ["-o", tmp, _SRC, "-lm"])
            os.replace(tmp, lib_path)
    return _LIB


_lib = None
_lib_omp = None


def lib_omp():
    """The OpenMP build (CPU timing only)."""
    global _lib_omp
    if _lib_omp is None:
        build()
        _lib_omp = _declare(ctypes.CDLL(_LIB_OMP))
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _declare(L):
    """Argument and result types of the oracle's exported functions."""
    L.orc_philox.argtypes = [_u32p, _u32p, _u32p]
    L.orc_philox.restype = None
    L.orc_move_words.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_uint32, _u32p]
    L.orc_move_words.restype = None
    L.orc_total_energy.argtypes = [ctypes.c_int32, _f64p, _f64p, ctypes.c_double]
    L.orc_total_energy.restype = ctypes.c_double
    L.orc_delta_energy.argtypes = [ctypes.c_int32, _f64p, _f64p, _f64p, ctypes.c_int32,
                                   _f64p, ctypes.c_double, _i32p]
    L.orc_delta_energy.restype = ctypes.c_double
    L.orc_outside_wall.argtypes = [_f64p, ctypes.c_double, ctypes.c_double]
    L.orc_outside_wall.restype = ctypes.c_int32
    L.orc_trial_f64.argtypes = [_f64p, _u32p, ctypes.c_double, _f64p]
    L.orc_trial_f64.restype = None
    L.orc_sweeps_f64.argtypes = [ctypes.c_int32, _f64p, _f64p, _f64p, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                 ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int32, _f64p,
                                 _u8p, _f64p, _u8p, ctypes.c_int64, _f64p]
    L.orc_sweeps_f64.restype = ctypes.c_int64
    L.orc_replay_f32.argtypes = [ctypes.c_int32, _f32p, _f64p, _f64p, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_float, ctypes.c_uint64,
                                 ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64, _u8p,
                                 _u8p, _f64p, _f64p, _u8p, _u8p, _f64p]
    L.orc_replay_f32.restype = ctypes.c_int64
    L.orc_rdf_counts.argtypes = [ctypes.c_int32, _f64p, _i32p, ctypes.c_int32,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int32, _u64p,
                                 _u64p]
    L.orc_rdf_counts.restype = None
    L.orc_da_nparam.argtypes = []
    L.orc_da_nparam.restype = ctypes.c_int32
    L.orc_bf16_round.argtypes = [ctypes.c_double]
    L.orc_bf16_round.restype = ctypes.c_double
    L.orc_da_features.argtypes = [ctypes.c_int32, _f64p, _f64p, ctypes.c_int32, _f64p,
                                  ctypes.c_double, _i32p]
    L.orc_da_features.restype = None
    L.orc_mlp_eps.argtypes = [_f64p, _i32p]
    L.orc_mlp_eps.restype = ctypes.c_double
    L.orc_da_run.argtypes = [ctypes.c_int32, _f64p, _f64p, _f64p, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                             ctypes.c_uint32, ctypes.c_int64, ctypes.c_int32, _f64p,
                             ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _u8p, _u8p,
                             ctypes.c_int64, _f64p, _f64p, _u8p, _u8p, _i32p, _f64p, _f64p,
                             _f64p, _f64p, _f64p]
    L.orc_da_run.restype = ctypes.c_int64
    L.orc_threads.argtypes = []
    L.orc_threads.restype = ctypes.c_int32
    return L


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


# --------------------------------------------------------------------------- #
# Random numbers                                                              #
# --------------------------------------------------------------------------- #

def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(_p(c, _u32p), _p(k, _u32p), _p(out, _u32p))
    return out


def move_words(seed: int, chain: int, sweep: int, i: int, tag: int = 0) -> np.ndarray:
    """The four Philox words of trial move (ion i, sweep) of a chain."""
    out = np.zeros(4, np.uint32)
    lib().orc_move_words(seed, chain, sweep, i, tag, _p(out, _u32p))
    return out


# --------------------------------------------------------------------------- #
# Energies and the chain                                                      #
# --------------------------------------------------------------------------- #

def total_energy(xyz, q, lB) -> float:
    """E = l_B sum_{i<j} q_i q_j / r_ij in kT (bare Coulomb, Sec. 5.1)."""
    x = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
    qq = np.ascontiguousarray(q, np.float64)
    return lib().orc_total_energy(len(qq), _p(x, _f64p), _p(qq, _f64p), lB)


def delta_energy(xyz, q, sigma, i, xt, lB):
    """(dE, overlap) for moving ion i to xt; Eq. (Delta E_ij) summed over j."""
    x = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
    qq = np.ascontiguousarray(q, np.float64)
    ss = np.ascontiguousarray(sigma, np.float64)
    t = np.ascontiguousarray(xt, np.float64)
    ov = ctypes.c_int32(0)
    dE = lib().orc_delta_energy(len(qq), _p(x, _f64p), _p(qq, _f64p), _p(ss, _f64p), int(i),
                                _p(t, _f64p), lB, ctypes.byref(ov))
    return dE, bool(ov.value)


class Chain:
    """Sequential-update Metropolis chain in double precision (Sec. 2).

    ``run(n)`` performs n sweeps; each sweep tries ions 0..N-1 once, in order.
    """

    def __init__(self, xyz, q, sigma, R, lB, D, seed, chain=0, sweep=0, threaded=False):
        # threaded: run on the OpenMP build (all host threads, another
        # summation order); for timing the CPU baseline only
        self._L = lib_omp() if threaded else lib()
        self.threads = int(self._L.orc_threads())
        self.x = np.array(xyz, np.float64).reshape(-1, 3).copy()
        self.q = np.ascontiguousarray(q, np.float64)
        self.sigma = np.ascontiguousarray(sigma, np.float64)
        self.n = len(self.q)
        self.R, self.lB, self.D = float(R), float(lB), float(D)
        self.seed, self.chain, self.sweep = int(seed), int(chain), int(sweep)
        self.e_run = total_energy(self.x, self.q, self.lB)
        self.accepted = 0

    def run(self, n_sweeps, trace=0, series=False):
        cap = int(trace)
        acc = np.zeros(max(cap, 1), np.uint8)
        de = np.zeros(max(cap, 1), np.float64)
        fl = np.zeros(max(cap, 1), np.uint8)
        es = np.zeros(max(n_sweeps, 1), np.float64) if series else None
        e = ctypes.c_double(self.e_run)
        nacc = self._L.orc_sweeps_f64(self.n, _p(self.x, _f64p), _p(self.q, _f64p),
                                    _p(self.sigma, _f64p), self.R, self.lB, self.D,
                                    self.seed, self.chain, self.sweep, int(n_sweeps),
                                    ctypes.byref(e), _p(acc, _u8p), _p(de, _f64p),
                                    _p(fl, _u8p), cap, _p(es, _f64p))
        self.e_run = e.value
        self.sweep += int(n_sweeps)
        self.accepted += int(nacc)
        out = {"accepted": int(nacc)}
        if cap:
            out.update(acc=acc[:cap], dE=de[:cap], flags=fl[:cap])
        if series:
            out["e_series"] = es[:n_sweeps]
        return out


def replay_f32(xyz_f32, q, sigma, R, lB, D, seed, chain, sweep0, n_moves, acc_given=None,
               eval_mask=None):
    """Exact double dE of each move along a float-state trajectory.

    The trajectory follows ``acc_given`` (e.g. another implementation's
    decisions); with ``eval_mask`` only the marked moves are evaluated.
    Returns a dict with dE, u3, flags (bit0 wall, bit1 overlap), the contact
    margin min_j r~_ij / sigma_ij - 1 of each evaluated trial, the oracle's
    own decision per move, the final float state and the number of moves
    whose given decision differs from the oracle's.
    """
    x = np.array(xyz_f32, np.float32).reshape(-1, 3).copy()
    qq = np.ascontiguousarray(q, np.float64)
    ss = np.ascontiguousarray(sigma, np.float64)
    n = len(qq)
    de = np.zeros(n_moves, np.float64)
    u3 = np.zeros(n_moves, np.float64)
    fl = np.zeros(n_moves, np.uint8)
    own = np.zeros(n_moves, np.uint8)
    margin = np.full(n_moves, np.inf)
    ag = None if acc_given is None else np.ascontiguousarray(acc_given, np.uint8)
    em = None if eval_mask is None else np.ascontiguousarray(eval_mask, np.uint8)
    mism = lib().orc_replay_f32(n, _p(x, _f32p), _p(qq, _f64p), _p(ss, _f64p), R, lB,
                                np.float32(D), seed, chain, sweep0, int(n_moves),
                                _p(ag, _u8p), _p(em, _u8p), _p(de, _f64p), _p(u3, _f64p),
                                _p(fl, _u8p), _p(own, _u8p), _p(margin, _f64p))
    return {"dE": de, "u3": u3, "flags": fl, "own": own, "xyz": x, "mismatches": int(mism),
            "margin": margin}


# --------------------------------------------------------------------------- #
# Pair correlation functions                                                  #
# --------------------------------------------------------------------------- #

def rdf_counts(xyz, types, ntypes, R, rmax, bins):
    """Integer pair counts C[a, b, k] and centre counts (Sec. 5.2 estimator)."""
    x = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(types, np.int32)
    counts = np.zeros((ntypes, ntypes, bins), np.uint64)
    centres = np.zeros(ntypes, np.uint64)
    lib().orc_rdf_counts(len(t), _p(x, _f64p), _p(t, _i32p), ntypes, R, rmax, bins,
                         _p(counts, _u64p), _p(centres, _u64p))
    return counts, centres


def rdf_normalise(counts, centres, n_of_type, sigma_of_type, R, rmax, bins, n_samples=1):
    """g_ab(r_k) = C_ab(k) / (Ncentre_a n_b V_k).

    n_b = (N_b - delta_ab) / ((4/3) pi (R - sigma_b/2)^3) is the density of
    possible neighbours of type b in the region their centres can reach and
    V_k the shell volume.  Centre counts and pair counts are totals over
    ``n_samples`` samples (the centre counts already include every sample).
    """
    counts = np.asarray(counts, np.float64)
    centres = np.asarray(centres, np.float64)
    nt = counts.shape[0]
    dr = rmax / bins
    edges = np.arange(bins + 1) * dr
    vk = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    g = np.zeros_like(counts)
    for a in range(nt):
        for b in range(nt):
            vb = 4.0 / 3.0 * np.pi * (R - 0.5 * sigma_of_type[b]) ** 3
            nb = (n_of_type[b] - (1 if a == b else 0)) / vb
            if centres[a] > 0:
                g[a, b] = counts[a, b] / (centres[a] * nb * vk)
    return g, 0.5 * (edges[1:] + edges[:-1])


# --------------------------------------------------------------------------- #
# Autocorrelation / effective sample size                                     #
# --------------------------------------------------------------------------- #

def autocorr(series, max_lag=None):
    """C_n of Sec. 5.2: normalised autocovariance of the series at lag n."""
    e = np.asarray(series, np.float64)
    e = e - e.mean()
    n = len(e)
    max_lag = n - 1 if max_lag is None else min(max_lag, n - 1)
    var = np.dot(e, e) / n
    if var == 0.0:
        return np.zeros(max_lag + 1)
    c = np.array([np.dot(e[: n - k], e[k:]) / n for k in range(max_lag + 1)])
    return c / var


def tau_int(series):
    """T_c = 1/2 + sum_{k>=1} C_k (Sec. 5.2).

    The paper does not say where the infinite sum stops.  Written as
    T_c = -1/2 + sum_{m>=0} (C_{2m} + C_{2m+1}), the sum runs over the pairs
    of lags up to, not including, the first pair whose sum is not positive
    (Geyer's initial positive sequence, Stat. Sci. 7, 1992).  Unlike a window
    in units of T_c it also converges for negatively correlated series.
    NaN for a constant series (C_n undefined).
    """
    e = np.asarray(series, np.float64)
    n = len(e)
    d = e - e.mean()
    var = np.dot(d, d) / n
    if n < 2 or var == 0.0:
        return float("nan")

    def c(k):  # C_k, the normalised autocovariance at lag k
        return np.dot(d[: n - k], d[k:]) / n / var

    tau = -0.5
    for m in range(n // 2):
        pair = c(2 * m) + c(2 * m + 1)
        if not pair > 0.0:
            break
        tau += pair
    return tau


def ess(series):
    """Effective sample size n / (2 T_c)."""
    return len(series) / (2.0 * tau_int(series))


# --------------------------------------------------------------------------- #
# Debye-Hueckel closed forms (Sec. 5.1)                                       #
# --------------------------------------------------------------------------- #

def debye_kappa(lB, densities, charges):
    """kappa^2 = 4 pi l_B sum_a n_a q_a^2 (Eq. (alpha-kappa_0) with beta e^2/eps = 4 pi l_B)."""
    return float(np.sqrt(4.0 * np.pi * lB * np.sum(np.asarray(densities) * np.asarray(charges) ** 2)))


def dh_log_ratio(r, lB, kappa, sigma):
    """ln(g_{+-}/g_{++}) for a symmetric 1:1 electrolyte in the linearised DH limit.

    The PB pair potential of mean force beta U = q1 q2 l_B exp(-kappa r)/r
    (Sec. 5.1) with the finite-size (extended DH) factor
    exp(kappa sigma)/(1 + kappa sigma); -ln g = beta U gives the ratio
    2 l_B exp(-kappa (r - sigma)) / (r (1 + kappa sigma)).
    """
    r = np.asarray(r, np.float64)
    return 2.0 * lB * np.exp(-kappa * (r - sigma)) / (r * (1.0 + kappa * sigma))


# --------------------------------------------------------------------------- #
# Delayed acceptance with a learned first stage (two-stage Metropolis of      #
# Christen and Fox 2005; not in the paper).  See mc_oracle.c for the          #
# definitions of the features, the network and the conflict rule.            #
# --------------------------------------------------------------------------- #

DA_BINS, DA_IN, DA_HID = 64, 128, 128


def da_nparam() -> int:
    return int(lib().orc_da_nparam())


def bf16(a):
    """Round to the nearest bfloat16 value (ties to even), elementwise."""
    a = np.asarray(a, np.float64)
    f = a.astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack_params(params):
    """Views (W1, b1, W2, b2, w3, b3) of the flat parameter vector."""
    p = np.asarray(params, np.float64)
    o = 0
    W1 = p[o:o + DA_IN * DA_HID].reshape(DA_IN, DA_HID); o += DA_IN * DA_HID
    b1 = p[o:o + DA_HID]; o += DA_HID
    W2 = p[o:o + DA_HID * DA_HID].reshape(DA_HID, DA_HID); o += DA_HID * DA_HID
    b2 = p[o:o + DA_HID]; o += DA_HID
    w3 = p[o:o + DA_HID]; o += DA_HID
    return W1, b1, W2, b2, w3, p[o]


def da_features(xyz, q, i, p, rc=4.0) -> np.ndarray:
    x = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
    qq = np.ascontiguousarray(q, np.float64)
    pp = np.ascontiguousarray(p, np.float64)
    out = np.zeros(DA_IN, np.int32)
    lib().orc_da_features(len(qq), _p(x, _f64p), _p(qq, _f64p), int(i), _p(pp, _f64p), rc, _p(out, _i32p))
    return out


def mlp_eps(params, feat) -> float:
    pp = np.ascontiguousarray(params, np.float64)
    f = np.ascontiguousarray(feat, np.int32)
    return float(lib().orc_mlp_eps(_p(pp, _f64p), _p(f, _i32p)))


def da_run(xyz, q, sigma, R, lB, D, seed, chain, sweep0, n_moves, params, rc=4.0, band=0, da_on=1,
           f32=False, acc_given=None, eval_mask=None, features=False, snapshots=False):
    """DA chain (own decisions) or replay (``acc_given``); returns a dict with
    the final state ``x`` and per-move dE, dEh, flags, own, u3, u2 (and
    features [n_moves, 256], and the positions after every completed sweep
    [sweeps, n, 3] as ``snapshots``, if asked) and the contact margin
    min_j r~_ij / sigma_ij - 1 of each evaluated trial."""
    x = np.array(xyz, np.float64).reshape(-1, 3).copy()
    if f32:
        x = x.astype(np.float32).astype(np.float64)
    qq = np.ascontiguousarray(q, np.float64)
    ss = np.ascontiguousarray(sigma, np.float64)
    pp = np.ascontiguousarray(params, np.float64)
    m = int(n_moves)
    de = np.zeros(m); deh = np.zeros(m); u3 = np.zeros(m); u2 = np.zeros(m)
    fl = np.zeros(m, np.uint8); own = np.zeros(m, np.uint8)
    feat = np.zeros((m, 2 * DA_IN), np.int32) if features else None
    ag = None if acc_given is None else np.ascontiguousarray(acc_given, np.uint8)
    em = None if eval_mask is None else np.ascontiguousarray(eval_mask, np.uint8)
    snap = np.zeros((m // len(qq), len(qq), 3)) if snapshots else None
    margin = np.full(m, np.inf)
    e = ctypes.c_double(0.0)
    mism = lib().orc_da_run(len(qq), _p(x, _f64p), _p(qq, _f64p), _p(ss, _f64p), R, lB, D, seed, chain,
                            sweep0, m, 1 if f32 else 0, _p(pp, _f64p), rc, band, da_on, _p(ag, _u8p),
                            _p(em, _u8p), m, _p(de, _f64p), _p(deh, _f64p), _p(fl, _u8p), _p(own, _u8p),
                            _p(feat, _i32p), _p(u3, _f64p), _p(u2, _f64p), ctypes.byref(e),
                            _p(snap, _f64p), _p(margin, _f64p))
    if mism < 0:
        raise ValueError("orc_da_run failed (%d)" % mism)
    return {"x": x, "dE": de, "dEh": deh, "flags": fl, "own": own, "u3": u3, "u2": u2,
            "features": feat, "mismatches": int(mism), "e_change": e.value, "snapshots": snap,
            "margin": margin}


def mlp_forward(params, X, rounding=True):
    """eps over the rows of X [rows, 128] in double, hidden activations
    rounded to bfloat16 as in orc_mlp_eps (rounding=False: not rounded);
    returns (out, cache)."""
    W1, b1, W2, b2, w3, b3 = unpack_params(params)
    X = np.asarray(X, np.float64)
    rnd = bf16 if rounding else (lambda a: a)
    Z1 = X @ W1 + b1
    H1 = rnd(np.maximum(Z1, 0.0))
    Z2 = H1 @ W2 + b2
    H2 = rnd(np.maximum(Z2, 0.0))
    out = H2 @ w3 + b3
    return out, (X, Z1, H1, Z2, H2)


def mlp_loss_grad(params, Xo, Xn, y, rounding=True):
    """Loss L = mean((eps(Xn) - eps(Xo) - y)^2) over the batch and its
    gradient with respect to the flat parameters, by backpropagation in
    double (the bfloat16 rounding of the activations is passed through
    unchanged by the derivative)."""
    W1, b1, W2, b2, w3, b3 = unpack_params(params)
    on, cn = mlp_forward(params, Xn, rounding)
    oo, co = mlp_forward(params, Xo, rounding)
    r = on - oo - np.asarray(y, np.float64)
    B = len(r)
    loss = float(np.mean(r * r))
    d = 2.0 * r / B
    g = np.zeros(len(params))
    gW1 = np.zeros_like(W1); gb1 = np.zeros_like(b1); gW2 = np.zeros_like(W2); gb2 = np.zeros_like(b2)
    gw3 = np.zeros_like(w3); gb3 = 0.0
    for sign, (X, Z1, H1, Z2, H2) in ((1.0, cn), (-1.0, co)):
        dout = sign * d
        gw3 += H2.T @ dout
        gb3 += float(np.sum(dout))
        dZ2 = np.outer(dout, w3) * (Z2 > 0)
        gW2 += H1.T @ dZ2
        gb2 += dZ2.sum(0)
        dZ1 = (dZ2 @ W2.T) * (Z1 > 0)
        gW1 += X.T @ dZ1
        gb1 += dZ1.sum(0)
    g[:] = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return loss, g
