"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/dare.h declares, and its host-only helpers validate
their arguments and agree with the oracle's readings."""
from __future__ import annotations

import ctypes as ct
import os
import re

import numpy as np
import pytest

import synth
from oracle import geometry as og

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(dare_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_function():
    import paper_2605_26325_amd as dare
    names = declared_functions()
    assert "dare_reconstruct_frames" in names and "dare_reslice" in names and "dare_reslice_batch" in names
    raw = ct.CDLL(dare.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing


def test_default_params_are_the_papers():
    import paper_2605_26325_amd as dare
    p = dare.default_params()
    assert (p.k_normal, p.k_inplane, p.thr_normal_deg, p.thr_inplane_deg) == (10.0, 5.0, 25.0, 15.0)
    assert p.radius_vox == 1.0 and p.normal_axis == 2 and p.max_bins == 64


def test_status_strings():
    import paper_2605_26325_amd as dare
    assert dare.status_str(dare.OK) == "ok"
    assert "budget" in dare.status_str(dare.ERR_BUDGET)
    assert dare.status_str(99) == "unknown status"


def test_arena_bytes_grow_with_bricks_and_reject_bad_input():
    import paper_2605_26325_amd as dare
    g = dare.make_geometry([0, 0, 0], 0.5, [64, 64, 64], np.eye(4))
    p = dare.default_params()
    a0 = dare.dare_volume_arena_bytes(g, p, dare.F32, 0)
    a1 = dare.dare_volume_arena_bytes(g, p, dare.F32, 1000)
    b1 = dare.dare_volume_arena_bytes(g, p, dare.BF16, 1000)
    f1 = dare.dare_volume_arena_bytes(g, p, dare.FP8, 1000)
    assert 0 < a0 < a1 and f1 < b1 < a1
    # per brick: 4 KiB of exact accumulators plus 512 stored pairs (8 / 4 / 2 bytes)
    assert a1 - a0 >= 1000 * (4096 + 512 * 8)
    bad = dare.default_params(radius_vox=1.5)
    assert dare.dare_volume_arena_bytes(g, bad, dare.F32, 10) == 0
    g_bad = dare.make_geometry([0, 0, 0], -1.0, [64, 64, 64], np.eye(4))
    assert dare.dare_volume_arena_bytes(g_bad, p, dare.F32, 10) == 0


def test_bounds_from_frames_matches_oracle_reading():
    import paper_2605_26325_amd as dare
    wl = synth.config1()
    g = dare.dare_bounds_from_frames(wl.sweep.probe_poses, wl.sweep.width, wl.sweep.height, wl.sweep.pitch,
                                     wl.calib, 0.5)
    o, dims = og.bounds_from_frames(wl.sweep.probe_poses, wl.sweep.width, wl.sweep.height, wl.sweep.pitch,
                                    wl.calib, 0.5)
    assert list(g.origin_mm) == list(o)
    assert tuple(g.dims) == tuple(dims)
    assert g.spacing_mm == 0.5 and np.array_equal(np.array(g.calib), wl.calib.reshape(16))


def test_bounds_rejects_non_rigid_pose():
    import paper_2605_26325_amd as dare
    P = np.eye(4, dtype=np.float32)[None].copy()
    P[0, 0, 0] = 1.01
    with pytest.raises(dare.DareError) as e:
        dare.dare_bounds_from_frames(P, 4, 4, (1, 1), np.eye(4), 1.0)
    assert e.value.status == dare.ERR_BAD_POSE
    with pytest.raises(dare.DareError) as e:
        dare.dare_bounds_from_frames(np.eye(4, dtype=np.float32)[None], 0, 4, (1, 1), np.eye(4), 1.0)
    assert e.value.status == dare.ERR_INVALID_ARG


# ----------------------------------------------------------------- saved volumes (host checks)

def _saved_buffer(dare, table, K, used, rep=None):
    """A buffer in the library's save format: header, brick table, then the used slots'
    accumulators (4 KiB), FP32 pairs (4 KiB) and FP8 scales (8 B)."""
    class Header(ct.Structure):
        _fields_ = [("magic", ct.c_char * 8), ("version", ct.c_uint32), ("header_bytes", ct.c_uint32),
                    ("g", dare.Geometry), ("p", dare.Params), ("dtype", ct.c_int32), ("K", ct.c_int32),
                    ("saturated", ct.c_int32), ("used", ct.c_uint32), ("rep_n", ct.c_double * 192),
                    ("rep_x", ct.c_double * 192), ("table_bytes", ct.c_uint64), ("acc_bytes", ct.c_uint64),
                    ("data_bytes", ct.c_uint64), ("scales_bytes", ct.c_uint64)]
    h = Header()
    h.magic = b"DAREVOL1"
    h.version, h.header_bytes = 1, ct.sizeof(Header)
    h.g = dare.make_geometry([0, 0, 0], 0.5, [16, 16, 16], np.eye(4))
    h.p = dare.default_params(max_bins=4)
    h.dtype, h.K, h.saturated, h.used = dare.F32, K, 0, used
    rep = np.tile([0.0, 0.0, 1.0], 64) if rep is None else rep
    for k in range(192):
        h.rep_n[k] = rep[k]
        h.rep_x[k] = [1.0, 0.0, 0.0][k % 3]
    table = np.asarray(table, np.int32)
    h.table_bytes = table.nbytes
    h.acc_bytes, h.data_bytes, h.scales_bytes = used * 4096, used * 4096, used * 8
    body = np.zeros(h.acc_bytes + h.data_bytes + h.scales_bytes, np.uint8)
    return np.concatenate([np.frombuffer(bytes(h), np.uint8), table.ravel().view(np.uint8), body])


def _device_visible():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.mark.skipif(_device_visible(), reason="passes a placeholder arena address: host-only test")
def test_volume_load_refuses_a_tampered_brick_table():
    """A damaged table is refused on the host, before any device call.  The arena argument is a
    placeholder address that no call may touch: with no device present, a buffer that passes
    the host checks fails at the first device call (DARE_ERR_HIP) instead."""
    import paper_2605_26325_amd as dare
    lib = dare.lib
    good = np.full((4, 8), -1, np.int32)          # 4 bins x 8 bricks of a 16^3 grid
    good[0, 0], good[0, 5], good[1, 2] = 0, 1, 2

    def load(buf):
        h = ct.c_void_p()
        return lib.dare_volume_load(buf.ctypes.data_as(ct.c_void_p), buf.nbytes, ct.c_void_p(1 << 32),
                                    1 << 26, ct.byref(h))

    assert load(_saved_buffer(dare, good, 2, 3)) == dare.ERR_HIP

    cases = {}
    t = good.copy(); t[0, 1] = 3; cases["slot beyond the used count"] = (t, 2, 3)
    t = good.copy(); t[0, 1] = -2; cases["negative slot"] = (t, 2, 3)
    t = good.copy(); t[1, 3] = 0; cases["slot owned twice"] = (t, 2, 3)
    t = good.copy(); t[2, 0] = 2; t[1, 2] = -1; cases["entry in a bin beyond the codebook"] = (t, 2, 3)
    t = good.copy(); t[1, 2] = -1; cases["slot owned by no entry"] = (t, 2, 3)
    for what, (tab, K, used) in cases.items():
        assert load(_saved_buffer(dare, tab, K, used)) == dare.ERR_INVALID_ARG, what
    rep = np.tile([0.0, 0.0, 1.0], 64)
    rep[4] = np.nan
    assert load(_saved_buffer(dare, good, 2, 3, rep)) == dare.ERR_INVALID_ARG
    bad = _saved_buffer(dare, good, 2, 3)
    bad[:8] = np.frombuffer(b"DAREVOL2", np.uint8)
    assert load(bad) == dare.ERR_INVALID_ARG
