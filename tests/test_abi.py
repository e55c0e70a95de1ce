"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/mc.h declares, and rejects bad input in mc_create before any device
work (host validation only; no compute call is made without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "mc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mc_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    from paper_1602_05716_amd import mc
    L = mc.load()
    names = _declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert sorted(mc.SYMBOLS) == names


def test_null_handles_are_rejected():
    from paper_1602_05716_amd import mc
    L = mc.lib()
    assert L.mc_sweep(None, 1, 1) == -1
    assert L.mc_sweep_reduction(None, 1, 1) == -1


def test_checkpoint_entry_points_reject_bad_input(tmp_path):
    """Host-side checks of mc_save / mc_load (no device work)."""
    from paper_1602_05716_amd import mc
    L = mc.lib()
    h = ctypes.c_void_p()
    assert L.mc_save(None, b"x") == -1
    assert L.mc_load(None, None, ctypes.byref(h)) == -1 and not h.value
    assert L.mc_load(str(tmp_path / "missing").encode(), None, ctypes.byref(h)) == -1 and not h.value
    junk = tmp_path / "junk.ckpt"
    junk.write_bytes(b"MCCKPT01" + b"\x00" * 64)
    assert L.mc_load(str(junk).encode(), None, ctypes.byref(h)) == -1 and not h.value
    assert "checkpoint" in L.mc_last_error(None).decode()


def test_options_defaults():
    from paper_1602_05716_amd import mc
    o = mc.options()
    assert o.precision == mc.MC_FP32_ACC64 and o.max_disp == 0.5 and o.resum_every == 100
    assert o.rdf_bins == 200 and o.rdf_rmax == 10.0 and o.band == -1 and o.rdf_margin == 0.0
    assert mc.lib().mc_options_init(None) == -1


def _create(n, q, s, x, R=10.0, lB=0.7, **kw):
    from paper_1602_05716_amd import mc
    L = mc.lib()
    h = ctypes.c_void_p()
    q = np.ascontiguousarray(q, np.float64)
    s = np.ascontiguousarray(s, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    o = mc.options(**kw)
    rc = L.mc_create(n, q.ctypes.data_as(mc._f64p), s.ctypes.data_as(mc._f64p),
                     x.ctypes.data_as(mc._f64p), R, lB, ctypes.byref(o), ctypes.byref(h))
    msg = L.mc_last_error(None).decode()
    if rc == 0:
        L.mc_destroy(h)
    assert not (rc != 0 and h.value), "handle leaked on error"
    return rc, msg


def test_create_rejects_non_neutral():
    rc, msg = _create(2, [1.0, 1.0], [1.0, 1.0], [[0, 0, 0], [3, 0, 0]])
    assert rc == -4, msg


def test_create_rejects_wall_crossing():
    # surface of ion 1 crosses R = 10 (centre at 9.6, radius 0.5)
    rc, msg = _create(2, [1.0, -1.0], [1.0, 1.0], [[0, 0, 0], [9.6, 0, 0]])
    assert rc == -3, msg
    rc, _ = _create(2, [1.0, -1.0], [1.0, 1.0], [[0, 0, 0], [9.5, 0, 0]])
    assert rc != -3


def test_create_rejects_bad_rdf_margin():
    rc, msg = _create(2, [1.0, -1.0], [1.0, 1.0], [[0, 0, 0], [3, 0, 0]], rdf_margin=-1.0)
    assert rc == -1 and "rdf_margin" in msg, msg


def test_create_rejects_overlap():
    rc, msg = _create(3, [1.0, -1.0, 0.0], [1.0, 0.5, 1.0], [[0, 0, 0], [0.74, 0, 0], [5, 0, 0]])
    assert rc == -2, msg
    rc, _ = _create(3, [1.0, -1.0, 0.0], [1.0, 0.5, 1.0], [[0, 0, 0], [0.75, 0, 0], [5, 0, 0]])
    assert rc != -2


@pytest.mark.parametrize("kw", [dict(max_disp=0.0), dict(rdf_bins=0), dict(band=9), dict(waves=3),
                                dict(precision=7), dict(wait_timeout_s=-1.0)])
def test_create_rejects_bad_options(kw):
    rc, msg = _create(2, [1.0, -1.0], [1.0, 1.0], [[0, 0, 0], [3, 0, 0]], **kw)
    assert rc == -1, (kw, msg)


def test_create_rejects_bad_arrays():
    rc, _ = _create(2, [1.0, np.nan], [1.0, 1.0], [[0, 0, 0], [3, 0, 0]])
    assert rc == -1
    rc, _ = _create(2, [1.0, -1.0], [1.0, -1.0], [[0, 0, 0], [3, 0, 0]])
    assert rc == -1
    rc, _ = _create(2, [1.0, -1.0], [1.0, 1.0], [[0, 0, 0], [3, np.inf, 0]])
    assert rc == -1
    rc, _ = _create(0, [], [], np.zeros((0, 3)))
    assert rc == -1


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1602_05716_amd import mc
    with pytest.raises(mc.MCLibraryError):
        mc.load(str(tmp_path / "missing.so"))


def _create_batch(specs, **kw):
    """specs: list of (q, sigma, xyz, R, lB); returns (rc, message)."""
    from paper_1602_05716_amd import mc
    L = mc.lib()
    arr = (mc.ChainSpec * len(specs))()
    keep = []
    for k, (q, s, x, R, lB) in enumerate(specs):
        q = np.ascontiguousarray(q, np.float64)
        s = np.ascontiguousarray(s, np.float64)
        x = np.ascontiguousarray(x, np.float64)
        keep += [q, s, x]
        arr[k].n = len(q)
        arr[k].charges = q.ctypes.data_as(mc._f64p)
        arr[k].diameters = s.ctypes.data_as(mc._f64p)
        arr[k].positions = x.ctypes.data_as(mc._f64p)
        arr[k].radius = R
        arr[k].l_B = lB
        arr[k].chain_id = k
    h = ctypes.c_void_p()
    o = mc.options(**kw)
    rc = L.mc_create_batch(len(specs), arr, ctypes.byref(o), ctypes.byref(h))
    msg = L.mc_last_error(None).decode()
    if rc == 0:
        L.mc_destroy(h)
    assert not (rc != 0 and h.value), "handle leaked on error"
    return rc, msg


def test_create_batch_validates_every_chain():
    good = ([1.0, -1.0], [1.0, 1.0], [[0, 0, 0], [3, 0, 0]], 10.0, 0.7)
    bad_neutral = ([1.0, 1.0], [1.0, 1.0], [[0, 0, 0], [3, 0, 0]], 10.0, 0.7)
    bad_wall = ([1.0, -1.0], [1.0, 1.0], [[0, 0, 0], [9.6, 0, 0]], 10.0, 0.7)
    bad_overlap = ([1.0, -1.0], [1.0, 1.0], [[0, 0, 0], [0.9, 0, 0]], 10.0, 0.7)
    rc, msg = _create_batch([good, bad_neutral])
    assert rc == -4 and msg.startswith("chain 1:"), msg
    rc, msg = _create_batch([bad_wall, good])
    assert rc == -3 and msg.startswith("chain 0:"), msg
    rc, msg = _create_batch([good, good, bad_overlap])
    assert rc == -2 and msg.startswith("chain 2:"), msg
    rc, msg = _create_batch([good], max_disp=-1.0)
    assert rc == -1, msg


def test_create_batch_rejects_empty_and_null():
    from paper_1602_05716_amd import mc
    L = mc.lib()
    h = ctypes.c_void_p()
    assert L.mc_create_batch(0, None, None, ctypes.byref(h)) == -1 and not h.value
    assert L.mc_create_batch(1, None, None, ctypes.byref(h)) == -1 and not h.value


def test_chain_calls_reject_null_handle():
    from paper_1602_05716_amd import mc
    L = mc.lib()
    n = ctypes.c_int32()
    assert L.mc_chain_count(None, ctypes.byref(n)) == -1
    assert L.mc_get_schedule(None, None, None) == -1
    assert L.mc_set_schedule(None, None) == -1
    assert L.mc_autotune(None, 1, 0, None) == -1
    assert L.mc_chain_launch_ms(None, None) == -1
