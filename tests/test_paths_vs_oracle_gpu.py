"""GPU parity of every reslice path directly against the FP64 oracle.

Each path is compared element by element with the oracle on the same stored grid (FP32, or the
dequantised BF16 / FP16 / FP8 grid the oracle emulates bit for bit): |d| <= 1e-5 max(|ref|, 1)
and identical NaN masks.  Covered here:
  * radius 1 at output pitches from 1/4 voxel (32 x 32 staged tiles in a batch) through about
    one voxel (16 x 16 staged tiles) to 2, 4 and 8 voxels (per-pixel gathers), alone and batched;
  * batched requests of several sizes with ragged tiles, every storage form;
  * BF16 and FP8 at radius 2 and 4, alone and batched;
  * served results (the continuous-batching server) against the oracle;
  * the server's volume budget: admission, refusal, removal and admission after removal.
The slice setup (pose composition, Eq. 1 gates, Eq. 2 weights) runs on the device in every path,
so each comparison also checks it.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from gpu_helpers import assert_parity, make_volume, note, oracle_grid, upload_grid
from helpers import random_grid, random_unit, rodrigues
from oracle import quant, reslice
from oracle.reslice import Params

pytestmark = pytest.mark.gpu

FORMS = {"f32": "fp32", "bf16": "bf16", "f16": "fp16", "fp8": "fp8"}


@pytest.fixture(scope="module")
def dare():
    import paper_2605_26325_amd as d
    return d


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def cfg1():
    wl = synth.config1()
    wl.render("cpu")
    return wl


@pytest.fixture(scope="module")
def cfg1_grid(cfg1):
    return oracle_grid(cfg1, cfg1.frames.numpy(), Params())


def _volume(cfg1, cfg1_grid, dtype, prm=None):
    prm = prm or Params()
    v = make_volume(cfg1.origin, cfg1.spacing, cfg1.dims, cfg1.calib, prm, dtype=dtype)
    upload_grid(v, cfg1_grid.S, cfg1_grid.C, *cfg1_grid.codebook.arrays())
    return v


def _oracle(cfg1, g, P, W, H, pitch, dtype, prm=None):
    return reslice.reslice_grid(g, cfg1.calib, P, W, H, pitch, prm or Params(), form=FORMS[dtype])


def _centred(cfg1, P, W, H, pitch):
    """The pose P moved so that a W x H slice at `pitch` is centred where P's frame is."""
    T = np.asarray(P, np.float64) @ cfg1.calib
    fw = np.asarray(cfg1.sweep.pitch, np.float64) * np.array([cfg1.sweep.width - 1, cfg1.sweep.height - 1])
    mid = T[:3, 3] + 0.5 * fw[0] * T[:3, 0] + 0.5 * fw[1] * T[:3, 1]
    T2 = T.copy()
    T2[:3, 3] = mid - 0.5 * (W - 1) * pitch[0] * T[:3, 0] - 0.5 * (H - 1) * pitch[1] * T[:3, 1]
    return T2 @ np.linalg.inv(cfg1.calib)


# radius-1 slices from fine to coarse pitch (config-1 voxel h = 0.5 mm): 1/4 voxel, about one
# voxel, then 2, 4 and 8 voxels, where a 16 x 16 tile's box exceeds the LDS budget
R1_CASES = [(96, 80, (0.125, 0.125)), (61, 47, (0.45, 0.55)), (40, 33, (1.0, 1.0)), (24, 20, (2.0, 2.0)),
            (9, 7, (4.0, 4.0)), (3, 2, (0.6, 8.0))]


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_radius1_all_pitches_alone_and_batched(dare, torch_cuda, cfg1, cfg1_grid, dtype):
    torch = torch_cuda
    note(f"radius 1 {dtype}: fine to coarse pitch, alone and batched, against the oracle")
    vol = _volume(cfg1, cfg1_grid, dtype)
    sl = cfg1.slices
    specs, refs, poses = [], [], []
    for k, (W, H, pitch) in enumerate(R1_CASES * 2):
        P = _centred(cfg1, sl.probe_poses[k % len(sl.probe_poses)], W, H, pitch)
        poses.append(P)
        specs.append(dare.make_spec(P, W, H, pitch))
        refs.append(_oracle(cfg1, cfg1_grid, P, W, H, pitch, dtype))
    assigned = 0
    for k, (s, ref) in enumerate(zip(specs, refs)):
        out = torch.full((s.height, s.width), -3.0, device="cuda")
        dare.dare_reslice(vol, s, out)
        torch.cuda.synchronize()
        assigned += assert_parity(out.cpu().numpy(), ref, what=f"alone case {k}")
    outs = [torch.full((s.height, s.width), -7.0, device="cuda") for s in specs]
    ws = torch.empty(dare.dare_reslice_batch_workspace_bytes([vol] * len(specs), specs), dtype=torch.uint8,
                     device="cuda")
    dare.dare_reslice_batch([vol] * len(specs), specs, outs, ws)
    torch.cuda.synchronize()
    for k, (o, ref) in enumerate(zip(outs, refs)):
        assert_parity(o.cpu().numpy(), ref, what=f"batched case {k}")
    assert assigned > 5000


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16", "fp8"])
def test_batched_sizes_vs_oracle(dare, torch_cuda, cfg1, cfg1_grid, dtype):
    """Ragged sizes (tiles cut by the slice edge), near-acquired and random poses, one call."""
    torch = torch_cuda
    note(f"batched radius-1 {dtype}: ragged sizes against the oracle")
    vol = _volume(cfg1, cfg1_grid, dtype)
    rng = np.random.default_rng(31)
    sizes = [(128, 128, (0.25, 0.25)), (33, 65, (0.3, 0.2)), (1, 1, (1.0, 1.0)), (100, 3, (0.1, 0.4)),
             (47, 95, (0.5, 0.5)), (64, 64, (0.125, 0.25))]
    specs, refs = [], []
    for k in range(12):
        W, H, pitch = sizes[k % len(sizes)]
        P = np.array(cfg1.slices.probe_poses[int(rng.integers(len(cfg1.slices.probe_poses)))])
        if k % 4 == 3:
            P[:3, 3] += rng.normal(0.0, 6.0, 3)
        specs.append(dare.make_spec(P, W, H, pitch))
        refs.append(_oracle(cfg1, cfg1_grid, P, W, H, pitch, dtype))
    outs = [torch.full((s.height, s.width), -7.0, device="cuda") for s in specs]
    ws = torch.empty(dare.dare_reslice_batch_workspace_bytes([vol] * len(specs), specs), dtype=torch.uint8,
                     device="cuda")
    dare.dare_reslice_batch([vol] * len(specs), specs, outs, ws)
    torch.cuda.synchronize()
    checked = 0
    for k, (o, ref) in enumerate(zip(outs, refs)):
        checked += assert_parity(o.cpu().numpy(), ref, what=f"request {k}")
    assert checked > 20000


def _random_case(seed, K, dims, p_empty):
    rng = np.random.default_rng(seed)
    S, C = random_grid(rng, K, dims, p_empty=p_empty)
    origin = np.array([-850.0, 310.0, -1620.0]) + rng.uniform(-1, 1, 3)
    n0 = random_unit(rng)
    x0 = random_unit(rng)
    x0 = x0 - (x0 @ n0) * n0
    x0 /= np.linalg.norm(x0)
    rn, rx = [], []
    for _ in range(K):
        R = rodrigues(random_unit(rng), math.radians(rng.uniform(0, 35)))
        rn.append(R @ n0)
        rx.append(R @ x0)
    return rng, S, C, origin, np.array(rn), np.array(rx), n0, x0


def _slice_pose(rng, origin, h, dims, n0, x0, W, H, pitch, calib, spread_deg=12.0):
    R = rodrigues(random_unit(rng), math.radians(rng.uniform(0, spread_deg)))
    n, x = R @ n0, R @ x0
    beam = np.cross(n, x)
    centre = origin + h * (np.array(dims) - 1) / 2 + rng.normal(0, 2.0, 3)
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2] = x, beam, n
    T[:3, 3] = centre - x * (W - 1) * pitch[0] / 2 - beam * (H - 1) * pitch[1] / 2
    return T @ np.linalg.inv(calib)


@pytest.mark.parametrize("R", [2, 4])
@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_precision_forms_larger_radius_vs_oracle(dare, torch_cuda, dtype, R):
    torch = torch_cuda
    note(f"radius {R} {dtype}: alone and batched against the oracle on the dequantised grid")
    dims = (21, 17, 19)
    rng, S, C, origin, rn, rx, n0, x0 = _random_case(200 + R, K=3, dims=dims, p_empty=0.5)
    calib = synth.make_calibration(16, 0.5)
    h = 0.5
    prm = Params(radius_vox=R)
    vol = make_volume(origin, h, dims, calib, prm, dtype=dtype)
    upload_grid(vol, S, C, rn, rx)
    a, c = quant.storage(S, C, FORMS[dtype])
    specs, refs = [], []
    for (W, H, pitch) in ((29, 19, (0.3, 0.33)), (8, 8, (0.9, 0.9)), (40, 36, (0.15, 0.2))):
        P = _slice_pose(rng, origin, h, dims, n0, x0, W, H, pitch, calib)
        specs.append(dare.make_spec(P, W, H, pitch))
        refs.append(reslice.reslice(a, c, origin, h, rn, rx, calib, P, W, H, pitch, prm))
    for k, (s, ref) in enumerate(zip(specs, refs)):
        out = torch.full((s.height, s.width), -3.0, device="cuda")
        dare.dare_reslice(vol, s, out)
        torch.cuda.synchronize()
        assert_parity(out.cpu().numpy(), ref, what=f"R={R} {dtype} alone {k}")
    outs = [torch.full((s.height, s.width), -7.0, device="cuda") for s in specs]
    ws = torch.empty(dare.dare_reslice_batch_workspace_bytes([vol] * len(specs), specs), dtype=torch.uint8,
                     device="cuda")
    dare.dare_reslice_batch([vol] * len(specs), specs, outs, ws)
    torch.cuda.synchronize()
    for k, (o, ref) in enumerate(zip(outs, refs)):
        assert_parity(o.cpu().numpy(), ref, what=f"R={R} {dtype} batched {k}")


def test_served_results_vs_oracle(dare, torch_cuda, cfg1, cfg1_grid):
    torch = torch_cuda
    note("served BF16 results against the oracle on the dequantised grid")
    vol = _volume(cfg1, cfg1_grid, "bf16")
    srv = dare.Server(64 << 20, n_streams=2, max_tick_requests=8)
    vid = srv.add_volume(vol)
    rng = np.random.default_rng(77)
    sizes = [(128, 128, (0.25, 0.25)), (37, 23, (0.6, 0.7)), (64, 65, (0.5, 0.5)), (24, 20, (2.0, 2.0))]
    reqs, outs, tickets = [], [], []
    for k in range(24):
        W, H, pitch = sizes[k % len(sizes)]
        P = cfg1.slices.probe_poses[int(rng.integers(len(cfg1.slices.probe_poses)))]
        o = torch.full((H, W), -5.0, dtype=torch.float32, pin_memory=True)
        t = None
        while t is None:
            t = srv.submit(vid, P, W, H, pitch, o)
        reqs.append((P, W, H, pitch))
        outs.append(o)
        tickets.append(t)
    srv.drain()
    assert all(srv.poll(t) is not None for t in tickets)
    srv.close()
    for k, ((P, W, H, pitch), o) in enumerate(zip(reqs, outs)):
        assert_parity(o.numpy(), _oracle(cfg1, cfg1_grid, P, W, H, pitch, "bf16"), what=f"served {k}")


def test_server_volume_budget(dare, torch_cuda, cfg1, cfg1_grid):
    torch = torch_cuda
    note("server volume budget: admit, refuse, remove, admit again")
    vols = [_volume(cfg1, cfg1_grid, "bf16") for _ in range(3)]
    each = int(vols[0].arena.numel())
    srv = dare.Server(64 << 20, n_streams=2, max_tick_requests=8, volume_budget_bytes=2 * each + each // 2)
    a = srv.add_volume(vols[0])
    b = srv.add_volume(vols[1])
    assert srv.volume_bytes() == (2 * each, 2)
    with pytest.raises(dare.DareError) as e:
        srv.add_volume(vols[2])
    assert e.value.status == dare.ERR_BUDGET
    assert srv.volume_bytes() == (2 * each, 2)
    P = cfg1.slices.probe_poses[0]
    o = torch.full((64, 64), -5.0, dtype=torch.float32, pin_memory=True)
    t = srv.submit(a, P, 64, 64, (0.5, 0.5), o)
    srv.remove_volume(a, wait_seconds=30.0)          # waits for the queued request
    assert srv.poll(t) is not None and not (o.numpy() == -5.0).any()
    assert srv.volume_bytes() == (each, 1)
    with pytest.raises(dare.DareError) as e:         # removed: its id takes no more requests
        srv.submit(a, P, 64, 64, (0.5, 0.5), o)
    assert e.value.status == dare.ERR_INVALID_ARG
    c = srv.add_volume(vols[2])                      # fits again
    assert c not in (a, b) and srv.volume_bytes() == (2 * each, 2)
    o2 = torch.full((64, 64), -5.0, dtype=torch.float32, pin_memory=True)
    t2 = srv.submit(c, P, 64, 64, (0.5, 0.5), o2)
    srv.drain()
    assert srv.poll(t2) is not None
    srv.close()
    assert np.array_equal(o.numpy(), o2.numpy(), equal_nan=True)   # same grid, same request


def test_server_radius5_full_size_request(dare, torch_cuda, cfg1, cfg1_grid):
    """A radius-5 server sizes its unit table for 64 lanes per pixel: a 512 x 512 request is
    admitted and served equal to the same request alone."""
    torch = torch_cuda
    note("radius-5 server with a 512^2 request")
    prm = Params(radius_vox=5)
    vol = _volume(cfg1, cfg1_grid, "bf16", prm)
    P = _centred(cfg1, cfg1.slices.probe_poses[2], 512, 512, (0.0625, 0.0625))
    ref = torch.full((512, 512), -3.0, device="cuda")
    dare.dare_reslice(vol, dare.make_spec(P, 512, 512, (0.0625, 0.0625)), ref)
    srv = dare.Server(64 << 20, n_streams=1, max_tick_requests=4)
    vid = srv.add_volume(vol)
    o = torch.full((512, 512), -5.0, dtype=torch.float32, pin_memory=True)
    t = srv.submit(vid, P, 512, 512, (0.0625, 0.0625), o)
    srv.drain()
    assert srv.poll(t) is not None
    srv.close()
    torch.cuda.synchronize()
    assert np.array_equal(o.numpy(), ref.cpu().numpy(), equal_nan=True)
    assert np.isfinite(o.numpy()).mean() > 0.5
