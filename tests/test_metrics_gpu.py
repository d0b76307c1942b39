"""GPU image similarity (Sec. 3's NCC and SSIM of a reslice against the acquired frame) against
the FP64 oracle in `oracle.metrics`: random images with unassigned blobs at ragged and square
sizes, all-assigned and almost-empty images, and a config-1 reslice at a held-out frame's pose.
Both sides are FP64; the bar is 1e-9 absolute on NCC and SSIM and exact pixel and window counts.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from gpu_helpers import make_volume, note
from oracle import metrics
from oracle.reslice import Params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dare():
    import paper_2605_26325_amd as d
    return d


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _pair(rng, H, W, p_hole):
    frame = rng.integers(0, 256, (H, W), dtype=np.uint8)
    img = np.clip(frame.astype(np.float64) * rng.uniform(0.5, 1.2) + rng.normal(0, 30, (H, W)), 0, 255)
    holes = np.zeros((H, W), bool)
    for _ in range(int(p_hole * 40)):             # unassigned blobs, as reslices leave them
        cy, cx, r = rng.integers(0, H), rng.integers(0, W), rng.integers(1, 9)
        yy, xx = np.ogrid[:H, :W]
        holes |= (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
    img[holes] = np.nan
    return img.astype(np.float32), frame


def _check(dare, torch, img, frame, what):
    got = dare.compare_to_frame(torch.from_numpy(img).cuda(), torch.from_numpy(frame).cuda())
    ref_ncc, n = metrics.ncc(img, frame)
    ref_ssim, m = metrics.ssim(img, frame)
    assert got[2] == n and got[3] == m, (what, got, n, m)
    for g, r in ((got[0], ref_ncc), (got[1], ref_ssim)):
        assert np.isnan(g) == np.isnan(r), (what, got, ref_ncc, ref_ssim)
        if not np.isnan(r):
            assert abs(g - r) <= 1e-9, (what, got, ref_ncc, ref_ssim)


@pytest.mark.parametrize("shape,p_hole", [((23, 37), 0.3), ((64, 64), 0.5), ((200, 131), 0.8), ((256, 256), 0.0)])
def test_random_images_against_oracle(dare, torch_cuda, shape, p_hole):
    note(f"image similarity, random {shape} with holes {p_hole}")
    rng = np.random.default_rng(shape[0] * 1000 + shape[1])
    img, frame = _pair(rng, *shape, p_hole)
    _check(dare, torch_cuda, img, frame, f"{shape}")


def test_degenerate_images(dare, torch_cuda):
    note("image similarity: identical, all unassigned, too small for a window")
    torch = torch_cuda
    rng = np.random.default_rng(3)
    frame = rng.integers(0, 256, (40, 30), dtype=np.uint8)
    got = dare.compare_to_frame(torch.from_numpy(frame.astype(np.float32)).cuda(), torch.from_numpy(frame).cuda())
    assert abs(got[0] - 1.0) <= 1e-12 and abs(got[1] - 1.0) <= 1e-12
    empty = np.full((40, 30), np.nan, np.float32)
    got = dare.compare_to_frame(torch.from_numpy(empty).cuda(), torch.from_numpy(frame).cuda())
    assert np.isnan(got[0]) and np.isnan(got[1]) and got[2] == 0 and got[3] == 0
    small = rng.uniform(0, 255, (7, 9)).astype(np.float32)
    _check(dare, torch, small, rng.integers(0, 256, (7, 9), dtype=np.uint8), "7x9")


def test_held_out_frame_of_config1(dare, torch_cuda):
    """The evaluation protocol on config 1: a frame left out of the reconstruction, resliced at
    its own pose from the other frames, compared with the frame itself."""
    torch = torch_cuda
    wl = synth.config1()
    frames = wl.render("cpu")
    keep = [f for f in range(frames.shape[0]) if f % 10 != 5]
    fr = frames[keep].cuda()
    poses = torch.from_numpy(np.asarray(wl.sweep.probe_poses, np.float32)[keep]).cuda()
    note("image similarity: config 1 held-out frames")
    vol = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params())
    vol.reconstruct(fr, poses, wl.sweep.pitch)
    torch.cuda.synchronize()
    F, H, W = frames.shape
    for f in (5, 105):
        img = vol.reslice(wl.sweep.probe_poses[f], W, H, wl.sweep.pitch).cpu().numpy()
        _check(dare, torch, img, frames[f].numpy(), f"held-out frame {f}")
        assert np.isfinite(img).mean() > 0.5
