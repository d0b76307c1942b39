"""GPU test of dare_reslice_batch_noalloc, the batch entry point that allocates nothing (for
callers that cannot allocate device memory): through the C ABI, its results equal those of
dare_reslice_batch with a caller workspace, bit for bit, on two calls in a row (the second with a
smaller input, over the library's shared per-device workspace), at radius 1 (device-built units)
and radius 2 (host-built units); a batch beyond the workspace is refused before anything runs.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from gpu_helpers import make_volume, note, oracle_grid, upload_grid
from oracle.reslice import Params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2605_26325_amd as dare
    wl = synth.config1()
    wl.render("cpu")
    g = oracle_grid(wl, wl.frames.numpy(), Params())
    vols = {}
    for dt, R in (("bf16", 1), ("f32", 1), ("fp8", 1), ("f32", 2)):
        v = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(radius_vox=R), dtype=dt)
        upload_grid(v, g.S, g.C, *g.codebook.arrays())
        vols[(dt, R)] = v
    return dare, torch, wl, vols


def _centred(wl, P, W, H, pitch):
    """Pose P moved so that a W x H slice at `pitch` is centred on the middle of P's frame."""
    T = np.asarray(P, np.float64) @ wl.calib
    fw = np.asarray(wl.sweep.pitch, np.float64) * np.array([wl.sweep.width - 1, wl.sweep.height - 1])
    mid = T[:3, 3] + 0.5 * fw[0] * T[:3, 0] + 0.5 * fw[1] * T[:3, 1]
    T[:3, 3] = mid - 0.5 * (W - 1) * pitch[0] * T[:3, 0] - 0.5 * (H - 1) * pitch[1] * T[:3, 1]
    return T @ np.linalg.inv(wl.calib)


def _requests(dare, wl, vols, keys, n, seed, sizes):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        W, H, pitch = sizes[k % len(sizes)]
        P = _centred(wl, wl.slices.probe_poses[int(rng.integers(len(wl.slices.probe_poses)))], W, H, pitch)
        if k % 4 == 3:
            P[:3, 3] += rng.normal(0.0, 5.0, 3)
        reqs.append((vols[keys[k % len(keys)]], dare.make_spec(P, W, H, pitch)))
    return reqs


def _both(dare, torch, reqs):
    vs, ss = [v for v, _ in reqs], [s for _, s in reqs]
    ref = [torch.full((s.height, s.width), -7.0, device="cuda") for s in ss]
    ws = torch.empty(dare.dare_reslice_batch_workspace_bytes(vs, ss), dtype=torch.uint8, device="cuda")
    dare.dare_reslice_batch(vs, ss, ref, ws)
    got = [torch.full((s.height, s.width), -5.0, device="cuda") for s in ss]
    dare.dare_reslice_batch_noalloc(vs, ss, got)
    torch.cuda.synchronize()
    for k in range(len(reqs)):
        a, b = got[k].cpu().numpy(), ref[k].cpu().numpy()
        assert not (b == -7.0).any() and not (a == -5.0).any(), k
        assert np.array_equal(a, b, equal_nan=True), k
    return sum(int(np.isfinite(r.cpu().numpy()).sum()) for r in ref)


def test_noalloc_equals_workspace_call_twice(env):
    dare, torch, wl, vols = env
    keys = [("bf16", 1), ("f32", 1), ("fp8", 1), ("f32", 2)]
    big = [(128, 128, (0.25, 0.25)), (61, 47, (0.45, 0.55)), (24, 20, (2.0, 2.0)), (200, 90, (0.16, 0.3))]
    note("no-alloc batch: first call, 24 mixed requests")
    first = _both(dare, torch, _requests(dare, wl, vols, keys, 24, 11, big))
    note("no-alloc batch: second call, 5 smaller requests on the same shared workspace")
    small = [(16, 9, (0.5, 0.5)), (3, 2, (0.6, 8.0)), (33, 17, (0.3, 0.3))]
    second = _both(dare, torch, _requests(dare, wl, vols, keys[:2], 5, 12, small))
    assert first > 20000 and second > 100


def test_noalloc_refuses_beyond_its_workspace(env):
    dare, torch, wl, vols = env
    note("no-alloc batch beyond the workspace is refused")
    v = vols[("bf16", 1)]
    specs = [dare.make_spec(wl.slices.probe_poses[0], 2048, 2048, (0.01, 0.01)) for _ in range(16)]
    assert dare.dare_reslice_batch_workspace_bytes([v] * 16, specs) > dare.NOALLOC_WORKSPACE_BYTES
    outs = [torch.empty(1, device="cuda") for _ in specs]     # never written: the call is refused first
    with pytest.raises(dare.DareError) as e:
        dare.dare_reslice_batch_noalloc([v] * 16, specs, outs)
    assert e.value.status == dare.ERR_BUDGET
