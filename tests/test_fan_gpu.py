"""GPU parity of fan-probe compounding (curvilinear and phased arrays, binning per column sector)
against ``oracle.fan``: sums, counts and codebook bit-exact; reslices of the fan-built volume
within 1e-5 of the FP64 oracle's with identical NaN masks; the hand-worked example; batches split
at 4096 / sectors frames; incremental calls; argument checks."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from gpu_helpers import assert_parity, make_volume, note
from oracle import compound, fan, reslice
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


def _sums(torch, vol):
    S, C = vol.download_sums()
    torch.cuda.synchronize()
    return S.cpu().numpy().view(np.uint32).astype(np.int64), C.cpu().numpy().view(np.uint32).astype(np.int64)


def _oracle(wl, frames_np, poses, sectors, prm=Params(), apex=None, r0=None):
    f = fan.Fan(apex=apex or wl.fan["apex"], r0=wl.fan["r0"] if r0 is None else r0, dr=wl.fan["dr"],
                sectors=sectors)
    g = compound.empty_grid(wl.origin, wl.spacing, wl.dims, prm.bin_tol_deg, prm.max_bins)
    fan.compound_fan(g, frames_np, poses, wl.calib, f, wl.beams)
    return f, g


def _gpu(torch, wl, frames, poses, f, prm=Params(), dtype="f32", calls=((0, None),)):
    vol = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, prm, dtype=dtype)
    P = torch.from_numpy(np.ascontiguousarray(poses, np.float32)).cuda()
    B = torch.from_numpy(np.ascontiguousarray(wl.beams, np.float64)).cuda()
    fr = frames.cuda()
    for a, b in calls:
        vol.reconstruct_fan(fr[a:b].contiguous(), P[a:b].contiguous(), f.apex, f.r0, f.dr, f.sectors, B)
    return vol


def _same_codebook(vol, g):
    rn, rx = vol.codebook()
    return (rn.shape[0] == g.K and np.array_equal(rn, np.array(g.codebook.rep_n).reshape(-1, 3))
            and np.array_equal(rx, np.array(g.codebook.rep_x).reshape(-1, 3)))


@pytest.fixture(scope="module")
def fan8():
    wl = synth.fan_config(sectors=8)
    fr = wl.render("cpu")
    f, g = _oracle(wl, fr.numpy(), wl.sweep.probe_poses, 8)
    return wl, fr, f, g


def test_fan_compound_bit_exact(dare, torch_cuda, fan8):
    torch = torch_cuda
    wl, fr, f, g = fan8
    note("fan compounding, curvilinear 96x128, 8 sectors, 200 frames")
    vol = _gpu(torch, wl, fr, wl.sweep.probe_poses, f)
    S, C = _sums(torch, vol)
    assert np.array_equal(C, g.C) and np.array_equal(S, g.S)
    assert _same_codebook(vol, g) and g.K > 8


def test_fan_incremental_equals_single_call(dare, torch_cuda, fan8):
    torch = torch_cuda
    wl, fr, f, g = fan8
    note("fan compounding in three calls")
    vol = _gpu(torch, wl, fr, wl.sweep.probe_poses, f, calls=((0, 37), (37, 150), (150, None)))
    S, C = _sums(torch, vol)
    assert np.array_equal(C, g.C) and np.array_equal(S, g.S) and _same_codebook(vol, g)


def test_fan_reslice_parity(dare, torch_cuda, fan8):
    torch = torch_cuda
    wl, fr, f, g = fan8
    note("fan volume reslices against the oracle")
    prm = Params()
    for dtype, form in (("f32", "fp32"), ("bf16", "bf16")):
        vol = _gpu(torch, wl, fr, wl.sweep.probe_poses, f, dtype=dtype)
        for k in range(6):
            P = wl.slices.probe_poses[k]
            got = vol.reslice(P, 128, 128, (0.25, 0.25)).cpu().numpy()
            ref = reslice.reslice_grid(g, wl.calib, P, 128, 128, (0.25, 0.25), prm, form=form)
            assert_parity(got, ref, what=f"fan {dtype} slice {k}")


@pytest.mark.parametrize("sectors,phased", [(1, False), (64, False), (8, True)])
def test_fan_variants(dare, torch_cuda, sectors, phased):
    """One sector (the whole fan one bin per frame), 64 sectors (batches of 64 frames, so 200
    frames take four), and a phased array (r0 = 0, apex on the face)."""
    torch = torch_cuda
    note(f"fan compounding variant sectors={sectors} phased={phased}")
    wl = synth.fan_config(sectors=sectors)
    fr = wl.render("cpu")
    apex = (wl.fan["apex"][0], 1.0) if phased else None
    r0 = 0.0 if phased else None
    f, g = _oracle(wl, fr.numpy(), wl.sweep.probe_poses, sectors, apex=apex, r0=r0)
    vol = _gpu(torch, wl, fr, wl.sweep.probe_poses, f)
    S, C = _sums(torch, vol)
    assert np.array_equal(C, g.C) and np.array_equal(S, g.S) and _same_codebook(vol, g)
    assert vol.info().saturated == int(g.codebook.saturated)


def test_fan_worked_example_on_gpu(dare, torch_cuda):
    """The hand-worked three-beam case of the oracle pins, through the C ABI."""
    torch = torch_cuda
    note("fan compounding, hand-worked three-beam example")
    b = np.array([[-0.6, 0.8], [0.0, 1.0], [0.6, 0.8]])
    frame = torch.tensor([[[1 + 10 * i + j for i in range(3)] for j in range(3)]], dtype=torch.uint8)
    g = dare.make_geometry((0.0, 0.0, 0.0), 1.0, (12, 6, 1), np.eye(4))
    for tol, bins in ((5.0, [0, 1, 2]), (40.0, [0, 0, 1])):
        vol = dare.Volume(g, dare.default_params(bin_tol_deg=tol))
        vol.reconstruct_fan(frame.cuda(), torch.eye(4).reshape(1, 4, 4).cuda(), (8.0, 0.0), 2.0, 1.0, 3,
                            torch.from_numpy(b).cuda())
        S, C = _sums(torch, vol)
        hand = {0: [(7, 2), (6, 2), (6, 3)], 1: [(8, 2), (8, 3), (8, 4)], 2: [(9, 2), (10, 2), (10, 3)]}
        Se = np.zeros((max(bins) + 1, 1, 6, 12), np.int64)
        Ce = np.zeros_like(Se)
        for i, cells in hand.items():
            for j, (vx, vy) in enumerate(cells):
                Se[bins[i], 0, vy, vx] += 1 + 10 * i + j
                Ce[bins[i], 0, vy, vx] += 1
        assert np.array_equal(S, Se) and np.array_equal(C, Ce), tol


def test_fan_argument_checks(dare, torch_cuda, fan8):
    torch = torch_cuda
    wl, fr, f, g = fan8
    note("fan compounding argument checks")
    vol = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params())
    P = torch.from_numpy(np.ascontiguousarray(wl.sweep.probe_poses[:2], np.float32)).cuda()
    B = torch.from_numpy(np.ascontiguousarray(wl.beams, np.float64)).cuda()
    x = fr[:2].cuda()
    for apex, r0, dr, G in ((f.apex, f.r0, f.dr, 0), (f.apex, f.r0, f.dr, 97), (f.apex, f.r0, f.dr, 65),
                            (f.apex, f.r0, 0.0, 8), (f.apex, -1.0, f.dr, 8), ((np.nan, 0.0), f.r0, f.dr, 8)):
        with pytest.raises(dare.DareError) as e:
            vol.reconstruct_fan(x, P, apex, r0, dr, G, B)
        assert e.value.status == dare.ERR_INVALID_ARG
    assert vol.info().bins == 0 and vol.info().bricks_used == 0
    v1 = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(normal_axis=1))
    with pytest.raises(dare.DareError) as e:
        v1.reconstruct_fan(x, P, f.apex, f.r0, f.dr, 8, B)
    assert e.value.status == dare.ERR_INVALID_ARG
