"""Thin ctypes binding of the C ABI in include/mc.h (libmc.so, HIP, gfx950).

Argument marshalling only: every step of the Monte Carlo path runs in the
library's kernels.  Importing this module loads the library and raises
``MCLibraryError`` if it is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmc.so")

MC_OK = 0
STATUS = {0: "MC_OK", -1: "MC_E_ARG", -2: "MC_E_OVERLAP", -3: "MC_E_WALL", -4: "MC_E_NOT_NEUTRAL",
          -5: "MC_E_DEVICE", -6: "MC_E_OOM", -7: "MC_E_TIMEOUT", -8: "MC_E_STATE"}
MC_FP64 = 0
MC_FP32_ACC64 = 1


class MCLibraryError(RuntimeError):
    pass


class MCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_disp", ctypes.c_double),
                ("resum_every", ctypes.c_int32), ("rdf_every", ctypes.c_int32),
                ("rdf_bins", ctypes.c_int32), ("rdf_rmax", ctypes.c_double),
                ("chain_id", ctypes.c_uint32), ("hip_stream", ctypes.c_void_p),
                ("band", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("workgroups", ctypes.c_int32), ("trace_moves", ctypes.c_int64),
                ("wait_timeout_s", ctypes.c_double), ("record_timing", ctypes.c_int32),
                ("da_rcut", ctypes.c_double), ("da_window", ctypes.c_int32), ("da_delta", ctypes.c_double),
                ("log_moves", ctypes.c_int64), ("rdf_margin", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("moves", ctypes.c_int64), ("accepted", ctypes.c_int64),
                ("rejected_wall", ctypes.c_int64), ("rejected_overlap", ctypes.c_int64),
                ("rejected_metropolis", ctypes.c_int64), ("fixpoint_iterations", ctypes.c_int64),
                ("early_groups", ctypes.c_int64),
                ("resums", ctypes.c_int64), ("last_drift", ctypes.c_double),
                ("max_abs_drift", ctypes.c_double), ("band", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("da_active", ctypes.c_int32), ("da_moves", ctypes.c_int64), ("da_conflicts", ctypes.c_int64),
                ("da_stage1_rejected", ctypes.c_int64), ("da_stage1_passed", ctypes.c_int64),
                ("da_stage2_rejected", ctypes.c_int64), ("da_fallback_sweep", ctypes.c_int64),
                ("da_last_rate", ctypes.c_double), ("da_kernel", ctypes.c_int32), ("reserved0", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ChainSpec(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("charges", ctypes.POINTER(ctypes.c_double)),
                ("diameters", ctypes.POINTER(ctypes.c_double)),
                ("positions", ctypes.POINTER(ctypes.c_double)),
                ("radius", ctypes.c_double), ("l_B", ctypes.c_double), ("max_disp", ctypes.c_double),
                ("chain_id", ctypes.c_uint32), ("reserved1", ctypes.c_int32)]


# Every symbol include/mc.h declares.
SYMBOLS = ["mc_options_init", "mc_create", "mc_sweep", "mc_sweep_reduction", "mc_energy", "mc_rdf", "mc_rdf_sample",
           "mc_rdf_reset", "mc_save", "mc_load", "mc_species", "mc_get_positions", "mc_trace", "mc_energy_series",
           "mc_get_stats", "mc_timing", "mc_timing_reset", "mc_set_max_disp",
           "mc_create_batch", "mc_chain_count", "mc_chain_energy", "mc_chain_rdf", "mc_chain_species",
           "mc_chain_positions", "mc_chain_trace", "mc_chain_energy_series", "mc_chain_stats",
           "mc_chain_set_max_disp", "mc_get_schedule", "mc_set_schedule", "mc_chain_launch_ms",
           "mc_autotune", "mc_plan_schedule", "mc_set_surrogate", "mc_get_log", "mc_mlp_grad", "mc_mlp_grad_noalloc",
           "mc_train_surrogate",
           "mc_destroy", "mc_last_error"]

DA_NPARAM = 33153

_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_hp = ctypes.c_void_p


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise MCLibraryError("HIP library %s is not built (run __graft_entry__.build())" % path)
    L = ctypes.CDLL(path)
    sig = {
        "mc_options_init": ([ctypes.POINTER(Options)], ctypes.c_int),
        "mc_create": ([ctypes.c_int32, _f64p, _f64p, _f64p, ctypes.c_double, ctypes.c_double,
                       ctypes.POINTER(Options), ctypes.POINTER(_hp)], ctypes.c_int),
        "mc_sweep": ([_hp, ctypes.c_int64, ctypes.c_uint64], ctypes.c_int),
        "mc_sweep_reduction": ([_hp, ctypes.c_int64, ctypes.c_uint64], ctypes.c_int),
        "mc_energy": ([_hp, _f64p, _f64p], ctypes.c_int),
        "mc_rdf": ([_hp, ctypes.c_int32, _f64p, _u64p, _u64p, _i64p], ctypes.c_int),
        "mc_rdf_sample": ([_hp], ctypes.c_int),
        "mc_rdf_reset": ([_hp], ctypes.c_int),
        "mc_save": ([_hp, ctypes.c_char_p], ctypes.c_int),
        "mc_load": ([ctypes.c_char_p, ctypes.POINTER(Options), ctypes.POINTER(_hp)], ctypes.c_int),
        "mc_species": ([_hp, _i32p, _f64p, _f64p], ctypes.c_int),
        "mc_get_positions": ([_hp, _f64p], ctypes.c_int),
        "mc_trace": ([_hp, ctypes.c_int64, _u8p, _f64p], ctypes.c_int),
        "mc_energy_series": ([_hp, ctypes.c_int64, _f64p], ctypes.c_int),
        "mc_get_stats": ([_hp, ctypes.POINTER(Stats)], ctypes.c_int),
        "mc_timing": ([_hp, _i64p, _f64p, _i64p], ctypes.c_int),
        "mc_timing_reset": ([_hp], ctypes.c_int),
        "mc_set_max_disp": ([_hp, ctypes.c_double], ctypes.c_int),
        "mc_create_batch": ([ctypes.c_int32, ctypes.POINTER(ChainSpec), ctypes.POINTER(Options),
                             ctypes.POINTER(_hp)], ctypes.c_int),
        "mc_chain_count": ([_hp, _i32p], ctypes.c_int),
        "mc_chain_energy": ([_hp, ctypes.c_int32, _f64p, _f64p], ctypes.c_int),
        "mc_chain_rdf": ([_hp, ctypes.c_int32, ctypes.c_int32, _f64p, _u64p, _u64p, _i64p], ctypes.c_int),
        "mc_chain_species": ([_hp, ctypes.c_int32, _i32p, _f64p, _f64p], ctypes.c_int),
        "mc_chain_positions": ([_hp, ctypes.c_int32, _f64p], ctypes.c_int),
        "mc_chain_trace": ([_hp, ctypes.c_int32, ctypes.c_int64, _u8p, _f64p], ctypes.c_int),
        "mc_chain_energy_series": ([_hp, ctypes.c_int32, ctypes.c_int64, _f64p], ctypes.c_int),
        "mc_chain_stats": ([_hp, ctypes.c_int32, ctypes.POINTER(Stats)], ctypes.c_int),
        "mc_chain_set_max_disp": ([_hp, ctypes.c_int32, ctypes.c_double], ctypes.c_int),
        "mc_get_schedule": ([_hp, _i32p, _f64p], ctypes.c_int),
        "mc_set_schedule": ([_hp, _i32p], ctypes.c_int),
        "mc_chain_launch_ms": ([_hp, _f64p], ctypes.c_int),
        "mc_autotune": ([_hp, ctypes.c_int32, ctypes.c_uint64, _f64p], ctypes.c_int),
        "mc_plan_schedule": ([ctypes.c_int32, _i32p, _f64p, _u8p, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                              _i32p, _i32p, _i32p, _i32p, _i32p, ctypes.c_int32], ctypes.c_int),
        "mc_set_surrogate": ([_hp, ctypes.c_int32, _f64p, ctypes.c_double, ctypes.c_int32], ctypes.c_int),
        "mc_get_log": ([_hp, ctypes.c_int32, ctypes.c_int64, _u8p, _f64p, _f64p, _u8p], ctypes.c_int),
        "mc_mlp_grad": ([ctypes.c_int32, _u8p, _f64p, _f64p, _f64p, _f64p], ctypes.c_int),
        "mc_mlp_grad_noalloc": ([ctypes.c_int32, _u8p, _f64p, _f64p, _f64p, _f64p], ctypes.c_int),
        "mc_train_surrogate": ([_hp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                ctypes.c_uint64, _f64p, _f64p, _f64p, _f64p, _f64p], ctypes.c_int),
        "mc_destroy": ([_hp], None),
        "mc_last_error": ([_hp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


_lib = None
# handles still open: destroyed (their streams synchronised, their device
# memory freed) before the interpreter's own teardown, so that no HIP object
# of the library outlives the runtime's exit handlers
_live = weakref.WeakSet()


def _close_live():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def lib():
    global _lib
    if _lib is None:
        _lib = load()
        atexit.register(_close_live)
    return _lib


def options(**kw) -> Options:
    o = Options()
    lib().mc_options_init(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": MC_FP64, "fp32": MC_FP32_ACC64}[v]
        setattr(o, k, v)
    return o


def _p(a, t):
    return a.ctypes.data_as(t)


RING = 1024  # group records kept per chain (accept masks in a checkpoint)


def _checkpoint_header(path):
    """(saved options, ion count per chain) from a checkpoint written by mc_save."""
    with open(path, "rb") as f:
        head = f.read(8 + 16 + 16 + ctypes.sizeof(Options))
        if len(head) < 40 + ctypes.sizeof(Options) or head[:8] != b"MCCKPT01":
            raise MCError(-1, "%s is not a checkpoint" % path)
        hdr = np.frombuffer(head[8:24], np.int32)  # version, chains, sizeof(options), counters
        n_chains, n_counters = int(hdr[1]), int(hdr[3])
        saved = Options.from_buffer_copy(head[40:])
        ns = []
        for _ in range(n_chains):
            ci = np.frombuffer(f.read(16), np.int32)
            ns.append(int(ci[0]))
            nt, bins = int(ci[1]), int(ci[2])
            f.read(32 + 32 + 8 * n_counters)  # R, l_B, max_disp, energy; re-sum record; counters
            f.seek(8 * (8 * ns[-1] + RING + nt * nt * bins + nt), 1)
            m = int(np.frombuffer(f.read(8), np.int64)[0])
            f.seek(8 * m, 1)
    return saved, ns


class Chain:
    """One Markov chain living on the GPU (a handle of the C ABI)."""

    def __init__(self, xyz, q, sigma, R, lB, **opts):
        self._L = lib()
        self.q = np.ascontiguousarray(q, np.float64)
        self.sigma = np.ascontiguousarray(sigma, np.float64)
        x = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
        self.n = len(self.q)
        self.R, self.lB = float(R), float(lB)
        self.opt = options(**opts)
        h = _hp()
        rc = self._L.mc_create(self.n, _p(self.q, _f64p), _p(self.sigma, _f64p), _p(x, _f64p),
                               self.R, self.lB, ctypes.byref(self.opt), ctypes.byref(h))
        if rc != MC_OK:
            raise MCError(rc, self._L.mc_last_error(None).decode())
        self.h = h
        _live.add(self)

    def _check(self, rc):
        if rc != MC_OK:
            raise MCError(rc, self._L.mc_last_error(self.h).decode())

    def sweep(self, n_sweeps, seed):
        self._check(self._L.mc_sweep(self.h, int(n_sweeps), int(seed)))

    def sweep_reduction(self, n_sweeps, seed):
        """The same sweeps by the per-move parallel-reduction scheme (mc_sweep_reduction)."""
        self._check(self._L.mc_sweep_reduction(self.h, int(n_sweeps), int(seed)))

    def save(self, path):
        """Checkpoint of the chain (mc_save)."""
        self._check(self._L.mc_save(self.h, os.fsencode(path)))

    @classmethod
    def load(cls, path, **opts):
        """A chain resumed from a checkpoint (mc_load); no options: the saved ones."""
        saved, ns = _checkpoint_header(path)
        if len(ns) != 1:
            raise MCError(-1, "the checkpoint holds %d chains (use Batch.load)" % len(ns))
        self = cls.__new__(cls)
        self._L = lib()
        self.opt = options(**opts) if opts else saved
        self.n = ns[0]
        h = _hp()
        rc = self._L.mc_load(os.fsencode(path), ctypes.byref(self.opt) if opts else None, ctypes.byref(h))
        if rc != MC_OK:
            raise MCError(rc, self._L.mc_last_error(None).decode())
        self.h = h
        _live.add(self)
        return self

    def energy(self, exact=False):
        er = ctypes.c_double()
        ee = ctypes.c_double()
        self._check(self._L.mc_energy(self.h, ctypes.byref(er), ctypes.byref(ee) if exact else None))
        return (er.value, ee.value) if exact else er.value

    def positions(self):
        out = np.zeros((self.n, 3), np.float64)
        self._check(self._L.mc_get_positions(self.h, _p(out, _f64p)))
        return out

    def trace(self, n_moves):
        acc = np.zeros(n_moves, np.uint8)
        de = np.zeros(n_moves, np.float64)
        self._check(self._L.mc_trace(self.h, int(n_moves), _p(acc, _u8p), _p(de, _f64p)))
        return acc, de

    def energy_series(self, n):
        e = np.zeros(n, np.float64)
        self._check(self._L.mc_energy_series(self.h, int(n), _p(e, _f64p)))
        return e

    def species(self):
        nt = ctypes.c_int32()
        self._check(self._L.mc_species(self.h, ctypes.byref(nt), None, None))
        q = np.zeros(nt.value)
        s = np.zeros(nt.value)
        self._check(self._L.mc_species(self.h, None, _p(q, _f64p), _p(s, _f64p)))
        return q, s

    def rdf_sample(self):
        self._check(self._L.mc_rdf_sample(self.h))

    def rdf_reset(self):
        self._check(self._L.mc_rdf_reset(self.h))

    def rdf(self):
        q, _ = self.species()
        nt = len(q)
        bins = self.opt.rdf_bins
        g = np.zeros((nt, nt, bins))
        c = np.zeros((nt, nt, bins), np.uint64)
        ce = np.zeros(nt, np.uint64)
        ns = ctypes.c_int64()
        self._check(self._L.mc_rdf(self.h, bins, _p(g, _f64p), _p(c, _u64p), _p(ce, _u64p),
                                   ctypes.byref(ns)))
        return {"g": g, "counts": c, "centres": ce, "samples": ns.value}

    def stats(self):
        st = Stats()
        self._check(self._L.mc_get_stats(self.h, ctypes.byref(st)))
        return st.as_dict()

    def timing(self):
        """(launches, summed sweep-kernel ms, sweeps covered) from HIP events."""
        la = ctypes.c_int64()
        ms = ctypes.c_double()
        sw = ctypes.c_int64()
        self._check(self._L.mc_timing(self.h, ctypes.byref(la), ctypes.byref(ms), ctypes.byref(sw)))
        return la.value, ms.value, sw.value

    def timing_reset(self):
        self._check(self._L.mc_timing_reset(self.h))

    def set_max_disp(self, v):
        self._check(self._L.mc_set_max_disp(self.h, float(v)))

    def close(self):
        if getattr(self, "h", None):
            self._L.mc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Independent chains served by one persistent launch (mc_create_batch).

    ``systems`` is a sequence of (xyz, q, sigma, R, lB) or of objects with
    those attributes (``inputs.System``); ``max_disp`` and ``chain_ids`` are
    optional per-chain sequences.  Methods taking ``c`` address one chain.
    """

    def __init__(self, systems, max_disp=None, chain_ids=None, **opts):
        self._L = lib()
        self.opt = options(**opts)
        self._keep = []
        specs = (ChainSpec * len(systems))()
        self.n = []
        for k, sy in enumerate(systems):
            if isinstance(sy, tuple):
                xyz, q, sigma, R, lB = sy
            else:
                xyz, q, sigma, R, lB = sy.xyz, sy.q, sy.sigma, sy.R, sy.lB
            q = np.ascontiguousarray(q, np.float64)
            sg = np.ascontiguousarray(sigma, np.float64)
            x = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
            self._keep += [q, sg, x]
            specs[k].n = len(q)
            specs[k].charges = _p(q, _f64p)
            specs[k].diameters = _p(sg, _f64p)
            specs[k].positions = _p(x, _f64p)
            specs[k].radius = float(R)
            specs[k].l_B = float(lB)
            specs[k].max_disp = 0.0 if max_disp is None else float(max_disp[k])
            specs[k].chain_id = k if chain_ids is None else int(chain_ids[k])
            self.n.append(len(q))
        h = _hp()
        rc = self._L.mc_create_batch(len(systems), specs, ctypes.byref(self.opt), ctypes.byref(h))
        self._keep = []
        if rc != MC_OK:
            raise MCError(rc, self._L.mc_last_error(None).decode())
        self.h = h
        _live.add(self)
        self.count = len(systems)

    def _check(self, rc):
        if rc != MC_OK:
            raise MCError(rc, self._L.mc_last_error(self.h).decode())

    def sweep(self, n_sweeps, seed):
        self._check(self._L.mc_sweep(self.h, int(n_sweeps), int(seed)))

    def energy(self, c, exact=False):
        er = ctypes.c_double()
        ee = ctypes.c_double()
        self._check(self._L.mc_chain_energy(self.h, int(c), ctypes.byref(er), ctypes.byref(ee) if exact else None))
        return (er.value, ee.value) if exact else er.value

    def positions(self, c):
        out = np.zeros((self.n[c], 3), np.float64)
        self._check(self._L.mc_chain_positions(self.h, int(c), _p(out, _f64p)))
        return out

    def trace(self, c, n_moves):
        acc = np.zeros(n_moves, np.uint8)
        de = np.zeros(n_moves, np.float64)
        self._check(self._L.mc_chain_trace(self.h, int(c), int(n_moves), _p(acc, _u8p), _p(de, _f64p)))
        return acc, de

    def energy_series(self, c, n):
        e = np.zeros(n, np.float64)
        self._check(self._L.mc_chain_energy_series(self.h, int(c), int(n), _p(e, _f64p)))
        return e

    def species(self, c):
        nt = ctypes.c_int32()
        self._check(self._L.mc_chain_species(self.h, int(c), ctypes.byref(nt), None, None))
        q = np.zeros(nt.value)
        s = np.zeros(nt.value)
        self._check(self._L.mc_chain_species(self.h, int(c), None, _p(q, _f64p), _p(s, _f64p)))
        return q, s

    def rdf_sample(self):
        self._check(self._L.mc_rdf_sample(self.h))

    def rdf_reset(self):
        self._check(self._L.mc_rdf_reset(self.h))

    def rdf(self, c):
        q, _ = self.species(c)
        nt = len(q)
        bins = self.opt.rdf_bins
        g = np.zeros((nt, nt, bins))
        cnt = np.zeros((nt, nt, bins), np.uint64)
        ce = np.zeros(nt, np.uint64)
        ns = ctypes.c_int64()
        self._check(self._L.mc_chain_rdf(self.h, int(c), bins, _p(g, _f64p), _p(cnt, _u64p), _p(ce, _u64p),
                                         ctypes.byref(ns)))
        return {"g": g, "counts": cnt, "centres": ce, "samples": ns.value}

    def stats(self, c):
        st = Stats()
        self._check(self._L.mc_chain_stats(self.h, int(c), ctypes.byref(st)))
        return st.as_dict()

    def save(self, path):
        """Checkpoint of every chain (mc_save)."""
        self._check(self._L.mc_save(self.h, os.fsencode(path)))

    @classmethod
    def load(cls, path, **opts):
        """A batch resumed from a checkpoint (mc_load); no options: the saved ones."""
        saved, ns = _checkpoint_header(path)
        self = cls.__new__(cls)
        self._L = lib()
        self._keep = []
        self.opt = options(**opts) if opts else saved
        self.n = ns
        h = _hp()
        rc = self._L.mc_load(os.fsencode(path), ctypes.byref(self.opt) if opts else None, ctypes.byref(h))
        if rc != MC_OK:
            raise MCError(rc, self._L.mc_last_error(None).decode())
        self.h = h
        _live.add(self)
        return self

    def set_max_disp(self, c, v):
        self._check(self._L.mc_chain_set_max_disp(self.h, int(c), float(v)))

    def schedule(self):
        """(workgroups per chain, cost model (a, b) in microseconds)."""
        w = np.zeros(self.count, np.int32)
        m = np.zeros(2, np.float64)
        self._check(self._L.mc_get_schedule(self.h, _p(w, _i32p), _p(m, _f64p)))
        return w, (float(m[0]), float(m[1]))

    def set_schedule(self, workgroups):
        w = np.ascontiguousarray(workgroups, np.int32)
        self._check(self._L.mc_set_schedule(self.h, _p(w, _i32p)))

    def launch_ms(self):
        ms = np.zeros(self.count, np.float64)
        self._check(self._L.mc_chain_launch_ms(self.h, _p(ms, _f64p)))
        return ms

    def autotune(self, calib_sweeps, seed):
        m = np.zeros(2, np.float64)
        self._check(self._L.mc_autotune(self.h, int(calib_sweeps), int(seed), _p(m, _f64p)))
        return float(m[0]), float(m[1])

    def timing(self):
        la = ctypes.c_int64()
        ms = ctypes.c_double()
        sw = ctypes.c_int64()
        self._check(self._L.mc_timing(self.h, ctypes.byref(la), ctypes.byref(ms), ctypes.byref(sw)))
        return la.value, ms.value, sw.value

    def timing_reset(self):
        self._check(self._L.mc_timing_reset(self.h))

    def close(self):
        if getattr(self, "h", None):
            self._L.mc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _set_surrogate(self, params, ref_stage2_reject=-1.0, active=True, chain=-1):
    p = np.ascontiguousarray(params, np.float64)
    if p.size != DA_NPARAM:
        raise ValueError("expected %d network parameters" % DA_NPARAM)
    self._check(self._L.mc_set_surrogate(self.h, int(chain), _p(p, _f64p), float(ref_stage2_reject),
                                         1 if active else 0))


def _get_log(self, n, chain=0):
    """Logged moves: dict of feats [n, 256] uint8, dE, dEh, flags."""
    f = np.zeros((n, 256), np.uint8)
    de = np.zeros(n)
    deh = np.zeros(n)
    fl = np.zeros(n, np.uint8)
    self._check(self._L.mc_get_log(self.h, int(chain), int(n), _p(f, _u8p), _p(de, _f64p), _p(deh, _f64p),
                                   _p(fl, _u8p)))
    return {"feats": f, "dE": de, "dEh": deh, "flags": fl}


Chain.set_surrogate = _set_surrogate
Chain.get_log = _get_log
Batch.set_surrogate = _set_surrogate
Batch.get_log = _get_log


def plan_schedule(nb, scale=None, measured=None, a=1.2, b=1.3, budget=512):
    """The batch planner alone (mc_plan_schedule, host only): returns
    (workgroups per chain, launch items as rows (chain, index, launch workgroup))."""
    nb = np.ascontiguousarray(nb, np.int32)
    n = len(nb)
    sc = None if scale is None else np.ascontiguousarray(scale, np.float64)
    me = None if measured is None else np.ascontiguousarray(measured, np.uint8)
    wg = np.zeros(n, np.int32)
    nl = ctypes.c_int32()
    cap = max(int(budget), 1) + n
    items = np.zeros((3, cap), np.int32)
    rc = lib().mc_plan_schedule(n, _p(nb, _i32p), None if sc is None else _p(sc, _f64p),
                                None if me is None else _p(me, _u8p), a, b, budget, _p(wg, _i32p), ctypes.byref(nl),
                                _p(items[0], _i32p), _p(items[1], _i32p), _p(items[2], _i32p), cap)
    if rc != MC_OK:
        raise MCError(rc, "mc_plan_schedule failed")
    k = int(wg.sum())
    return wg, items[:, :k].T.copy(), int(nl.value)


def mlp_grad(feats, target, params):
    """(loss, grad) of the network on the GPU (mc_mlp_grad)."""
    f = np.ascontiguousarray(feats, np.uint8).reshape(-1, 256)
    t = np.ascontiguousarray(target, np.float64)
    p = np.ascontiguousarray(params, np.float64)
    loss = ctypes.c_double()
    g = np.zeros(DA_NPARAM)
    rc = lib().mc_mlp_grad(len(f), _p(f, _u8p), _p(t, _f64p), _p(p, _f64p), ctypes.byref(loss), _p(g, _f64p))
    if rc != MC_OK:
        raise MCError(rc, "mc_mlp_grad failed")
    return loss.value, g


def mlp_grad_noalloc(feats, target, params):
    """(loss, grad) as mlp_grad, from the library's fixed device workspace
    (mc_mlp_grad_noalloc: no device allocation; batch <= MC_NOALLOC_MAX_BATCH)."""
    f = np.ascontiguousarray(feats, np.uint8).reshape(-1, 256)
    t = np.ascontiguousarray(target, np.float64)
    p = np.ascontiguousarray(params, np.float64)
    loss = ctypes.c_double()
    g = np.zeros(DA_NPARAM)
    rc = lib().mc_mlp_grad_noalloc(len(f), _p(f, _u8p), _p(t, _f64p), _p(p, _f64p), ctypes.byref(loss),
                                   _p(g, _f64p))
    if rc != MC_OK:
        raise MCError(rc, lib().mc_last_error(None).decode())
    return loss.value, g


def _train_surrogate(self, n_moves, epochs=10, batch=1024, lr=1e-3, seed=1, params_in=None, chain=0):
    """Trains the surrogate on the chain's log; returns a dict with params,
    per-epoch losses, held-out loss and the stage-2 rejection reference."""
    out = np.zeros(DA_NPARAM)
    losses = np.zeros(epochs)
    vl = ctypes.c_double()
    ref = ctypes.c_double()
    pin = None if params_in is None else np.ascontiguousarray(params_in, np.float64)
    self._check(self._L.mc_train_surrogate(self.h, int(chain), int(n_moves), int(epochs), int(batch), float(lr),
                                           int(seed), _p(pin, _f64p) if pin is not None else None, _p(out, _f64p),
                                           _p(losses, _f64p), ctypes.byref(vl), ctypes.byref(ref)))
    return {"params": out, "loss": losses, "val_loss": vl.value, "ref_stage2_reject": ref.value}


Chain.train_surrogate = _train_surrogate
Batch.train_surrogate = _train_surrogate
