"""Volume persistence through the C ABI: a saved and reloaded volume reslices bit for bit like
the original, holds the same sums, codebook and bricks, and keeps compounding incrementally to the
same state as the original; damaged buffers and small arenas are refused."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from gpu_helpers import make_volume, note
from oracle.reslice import Params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dare():
    import paper_2605_26325_amd as d
    return d


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    wl = synth.config1()
    frames = wl.render("cuda")
    poses = torch.from_numpy(np.asarray(wl.sweep.probe_poses, np.float32)).cuda()
    return torch, wl, frames, poses


def _same(torch, a, b):
    return torch.equal(torch.nan_to_num(a, nan=-1.0), torch.nan_to_num(b, nan=-1.0))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_save_load_roundtrip_and_incremental(dare, setup, dtype):
    torch, wl, frames, poses = setup
    note(f"persistence round trip, {dtype}")
    first = list(range(0, 70)) + list(range(100, 170))
    rest = list(range(70, 100)) + list(range(170, 200))
    vol = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(), dtype=dtype)
    vol.reconstruct(frames[first].contiguous(), poses[first].contiguous(), wl.sweep.pitch)
    buf = vol.save()
    loaded = dare.Volume.load(buf, vol.arena.numel())
    assert loaded.dtype == vol.dtype and tuple(loaded.geometry.dims) == tuple(vol.geometry.dims)
    a, b = vol.info(), loaded.info()
    assert (a.bins, a.bricks_used, a.saturated) == (b.bins, b.bricks_used, b.saturated)
    rn0, rx0 = vol.codebook()
    rn1, rx1 = loaded.codebook()
    assert np.array_equal(rn0, rn1) and np.array_equal(rx0, rx1)
    for k in range(4):
        P = wl.slices.probe_poses[k]
        assert _same(torch, vol.reslice(P, 128, 128, (0.25, 0.25)), loaded.reslice(P, 128, 128, (0.25, 0.25))), k
    # both keep compounding: the same later frames give the same state
    for v in (vol, loaded):
        v.reconstruct(frames[rest].contiguous(), poses[rest].contiguous(), wl.sweep.pitch)
    torch.cuda.synchronize()
    S0, C0 = vol.download_sums()
    S1, C1 = loaded.download_sums()
    assert torch.equal(S0, S1) and torch.equal(C0, C1)
    for k in range(4, 8):
        P = wl.slices.probe_poses[k]
        assert _same(torch, vol.reslice(P, 128, 128, (0.25, 0.25)), loaded.reslice(P, 128, 128, (0.25, 0.25))), k


def test_damaged_buffers_and_small_arenas_refused(dare, setup):
    torch, wl, frames, poses = setup
    note("persistence: damaged buffer, truncated buffer, small arena")
    vol = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params())
    vol.reconstruct(frames, poses, wl.sweep.pitch)
    buf = vol.save()
    bad = buf.copy()
    bad[0] ^= 0xFF
    with pytest.raises(dare.DareError) as e:
        dare.Volume.load(bad, vol.arena.numel())
    assert e.value.status == dare.ERR_INVALID_ARG
    with pytest.raises(dare.DareError) as e:
        dare.Volume.load(buf[:-1], vol.arena.numel())
    assert e.value.status == dare.ERR_INVALID_ARG
    used = vol.info().bricks_used
    small = dare.dare_volume_arena_bytes(vol.geometry, vol.params, vol.dtype, used // 2)
    with pytest.raises(dare.DareError) as e:
        dare.Volume.load(buf, small)
    assert e.value.status == dare.ERR_BUDGET
    torch.cuda.synchronize()
