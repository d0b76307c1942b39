"""Out-of-core bricks through the C ABI (bricks moved to host memory and back, Sec. 4's data sets
beyond GPU memory).  Bars, all bit-exact: a volume whose bricks went to host memory and came back
equals one that never moved them (sums, counts, stored pairs, reslices), also when compounding
re-created held bricks in between, and equals the oracle's compounding; a volume compounded with
spilling in an arena a third of its footprint holds, restored one slab of bricks at a time, the
oracle's sums in every slab."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from gpu_helpers import make_volume, note, oracle_grid
from oracle.reslice import Params

pytestmark = pytest.mark.gpu

BRICK = 8


@pytest.fixture(scope="module")
def dare():
    import paper_2605_26325_amd as d
    return d


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    wl = synth.config1()
    frames = wl.render("cpu")
    grid = oracle_grid(wl, frames.numpy(), Params())
    poses = torch.from_numpy(np.asarray(wl.sweep.probe_poses, np.float32)).cuda()
    return torch, wl, frames.cuda(), poses, grid


def _sums(torch, vol):
    S, C = vol.download_sums()
    torch.cuda.synchronize()
    return S.cpu().numpy().view(np.uint32).astype(np.int64), C.cpu().numpy().view(np.uint32).astype(np.int64)


def _same(torch, a, b):
    return torch.equal(torch.nan_to_num(a, nan=-1.0), torch.nan_to_num(b, nan=-1.0))


def _whole(wl):
    return (0, 0, 0), tuple(int(d) - 1 for d in wl.dims)


def _brick_mask(dims, lo, hi):
    """(nz, ny, nx) mask of the voxels whose brick meets the voxel box lo..hi (x, y, z order)."""
    axes = []
    for a in range(3):
        b = np.arange(dims[a]) // BRICK
        axes.append((b * BRICK <= hi[a]) & (b * BRICK + BRICK - 1 >= lo[a]))
    return axes[2][:, None, None] & axes[1][None, :, None] & axes[0][None, None, :]


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_evict_and_restore_is_exact(dare, setup, dtype):
    torch, wl, frames, poses, grid = setup
    note(f"out-of-core: evict outside a box and restore, {dtype}")
    ref = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(), dtype=dtype)
    ref.reconstruct(frames, poses, wl.sweep.pitch)
    vol = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(), dtype=dtype)
    vol.reconstruct(frames, poses, wl.sweep.pitch)
    total = ref.info().bricks_used
    nz = int(wl.dims[2])
    lo, hi = (0, 0, nz // 3), (int(wl.dims[0]) - 1, int(wl.dims[1]) - 1, 2 * nz // 3)
    vol.evict_outside(lo, hi)
    n_held, nbytes = vol.held()
    assert n_held > 0 and nbytes == n_held * 512 * 8
    assert vol.info().bricks_used + n_held == total
    # the resident part is the bricks meeting the box, unchanged; the rest reads as empty
    S0, C0 = _sums(torch, ref)
    S1, C1 = _sums(torch, vol)
    m = _brick_mask(wl.dims, lo, hi)
    assert np.array_equal(S1[:, m], S0[:, m]) and np.array_equal(C1[:, m], C0[:, m])
    assert not C1[:, ~m].any() and C0[:, ~m].any()
    with pytest.raises(dare.DareError) as e:   # a save would lose the held bricks
        vol.save()
    assert e.value.status == dare.ERR_INVALID_ARG
    vol.restore_box(*_whole(wl))
    assert vol.held() == (0, 0) and vol.info().bricks_used == total
    S1, C1 = _sums(torch, vol)
    assert np.array_equal(S1, grid.S) and np.array_equal(C1, grid.C)
    A0, N0 = ref.download_storage()
    A1, N1 = vol.download_storage()
    assert torch.equal(A0, A1) and torch.equal(N0, N1)
    for k in range(6):
        P = wl.slices.probe_poses[k]
        assert _same(torch, ref.reslice(P, 128, 128, (0.25, 0.25)), vol.reslice(P, 128, 128, (0.25, 0.25))), k


def test_compounding_into_held_bricks_merges_exactly(dare, setup):
    """Even frames, then every brick to host memory, then odd frames (which re-create most of the
    held bricks in HBM), then everything back: the held and the new sums add up exactly."""
    torch, wl, frames, poses, grid = setup
    note("out-of-core: compounding into held bricks, then restore")
    even, odd = list(range(0, frames.shape[0], 2)), list(range(1, frames.shape[0], 2))
    vol = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params())
    vol.reconstruct(frames[even].contiguous(), poses[even].contiguous(), wl.sweep.pitch)
    vol.evict_outside((1, 1, 1), (0, 0, 0))          # an empty box: every brick leaves
    assert vol.info().bricks_used == 0 and vol.held()[0] > 0
    S, C = _sums(torch, vol)
    assert not C.any()
    vol.reconstruct(frames[odd].contiguous(), poses[odd].contiguous(), wl.sweep.pitch)
    assert vol.info().bricks_used > 0
    # a box restore merges only what meets the box; then the rest
    nz = int(wl.dims[2])
    vol.restore_box((0, 0, 0), (int(wl.dims[0]) - 1, int(wl.dims[1]) - 1, nz // 2))
    vol.restore_box(*_whole(wl))
    assert vol.held() == (0, 0)
    S, C = _sums(torch, vol)
    assert np.array_equal(S, grid.S) and np.array_equal(C, grid.C)
    ref = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params())
    ref.reconstruct(frames, poses, wl.sweep.pitch)
    assert vol.info().bricks_used == ref.info().bricks_used
    for k in range(4):
        P = wl.slices.probe_poses[k]
        assert _same(torch, ref.reslice(P, 128, 128, (0.25, 0.25)), vol.reslice(P, 128, 128, (0.25, 0.25))), k


def test_spill_in_a_small_arena(dare, setup):
    """Compounding with spilling on in an arena of a third of the volume's bricks, ten frames per
    call: no batch fails, and every z slab of bricks, brought back alone, holds the oracle's
    sums.  Restoring everything at once is refused for room, with nothing changed."""
    torch, wl, frames, poses, grid = setup
    note("out-of-core: spill mode in an arena of a third of the bricks")
    occupied = grid.C.reshape(grid.C.shape[0], -1)
    nb = [(int(d) + BRICK - 1) // BRICK for d in wl.dims]
    Cb = np.zeros((grid.C.shape[0], nb[2] * BRICK, nb[1] * BRICK, nb[0] * BRICK), np.int64)
    Cb[:, :grid.C.shape[1], :grid.C.shape[2], :grid.C.shape[3]] = grid.C
    per_brick = Cb.reshape(Cb.shape[0], nb[2], BRICK, nb[1], BRICK, nb[0], BRICK).sum(axis=(2, 4, 6)) > 0
    total = int(per_brick.sum())
    assert occupied.any() and total > 30
    cap_bricks = total // 3
    slab_need = per_brick.sum(axis=(0, 2, 3))          # bricks per z layer of bricks
    assert slab_need.max() <= cap_bricks, (slab_need, cap_bricks)
    vol = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(), bricks=cap_bricks)
    cap = vol.info().bricks_capacity
    with pytest.raises(dare.DareError) as e:           # without spilling the arena is too small
        vol.reconstruct(frames, poses, wl.sweep.pitch)
    assert e.value.status == dare.ERR_BUDGET
    vol.set_spill(True)
    F = frames.shape[0]
    for a in range(0, F, 10):
        vol.reconstruct(frames[a:a + 10].contiguous(), poses[a:a + 10].contiguous(), wl.sweep.pitch)
    inf = vol.info()
    n_held = vol.held()[0]
    assert inf.bricks_used <= cap and n_held > 0 and inf.bricks_used + n_held >= total
    used0 = inf.bricks_used
    with pytest.raises(dare.DareError) as e:
        vol.restore_box(*_whole(wl))
    assert e.value.status == dare.ERR_BUDGET
    assert vol.held()[0] == n_held and vol.info().bricks_used == used0
    vol.set_spill(False)
    nx, ny, nz = (int(d) for d in wl.dims)
    for bz in range(nb[2]):
        lo, hi = (0, 0, bz * BRICK), (nx - 1, ny - 1, bz * BRICK + BRICK - 1)
        vol.evict_outside(lo, hi)
        vol.restore_box(lo, hi)
        assert vol.info().bricks_used == int(slab_need[bz]), bz
        S, C = _sums(torch, vol)
        z = slice(bz * BRICK, min(nz, bz * BRICK + BRICK))
        assert np.array_equal(S[:, z], grid.S[:, z]) and np.array_equal(C[:, z], grid.C[:, z]), bz
        rest = np.ones(nz, bool)
        rest[z] = False
        assert not C[:, rest].any(), bz


def test_spill_with_fan_frames(dare, setup):
    """Spilling composes with fan-probe compounding (the same batch admission): curvilinear frames
    compounded 20 per call into an arena of 60 % of their bricks; each z half of the grid, brought
    back alone, holds the fan oracle's sums."""
    from oracle import compound, fan
    torch = setup[0]
    note("out-of-core: spill mode with fan frames")
    wl = synth.fan_config(sectors=4)
    fr = wl.render("cpu")
    f = fan.Fan(apex=wl.fan["apex"], r0=wl.fan["r0"], dr=wl.fan["dr"], sectors=4)
    g = compound.empty_grid(wl.origin, wl.spacing, wl.dims, Params().bin_tol_deg, Params().max_bins)
    fan.compound_fan(g, fr.numpy(), wl.sweep.probe_poses, wl.calib, f, wl.beams)
    ref = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params())
    P = torch.from_numpy(np.ascontiguousarray(wl.sweep.probe_poses, np.float32)).cuda()
    B = torch.from_numpy(np.ascontiguousarray(wl.beams, np.float64)).cuda()
    frc = fr.cuda()
    ref.reconstruct_fan(frc, P, f.apex, f.r0, f.dr, 4, B)
    total = ref.info().bricks_used
    vol = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(), bricks=int(total * 0.6))
    vol.set_spill(True)
    for a in range(0, frc.shape[0], 20):
        vol.reconstruct_fan(frc[a:a + 20].contiguous(), P[a:a + 20].contiguous(), f.apex, f.r0, f.dr, 4, B)
    assert vol.held()[0] > 0
    nx, ny, nz = (int(d) for d in wl.dims)
    half = (nz // 2 // BRICK) * BRICK
    for lo, hi, z in (((0, 0, 0), (nx - 1, ny - 1, half - 1), slice(0, half)),
                      ((0, 0, half), (nx - 1, ny - 1, nz - 1), slice(half, nz))):
        vol.evict_outside(lo, hi)
        vol.restore_box(lo, hi)
        S, C = _sums(torch, vol)
        assert np.array_equal(S[:, z], g.S[:, z]) and np.array_equal(C[:, z], g.C[:, z]), z
