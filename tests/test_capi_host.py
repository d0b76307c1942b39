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
