"""Pins of the FP64 oracle against what the paper and mathematics fix (CPU only).

Each test checks the oracle against something other than itself: closed forms
of Eq. 2 at chosen angles, hand-worked clustering, library routines
(numpy matmul, scipy's order-1 ``map_coordinates``, torch's dtype casts),
brute force on tiny inputs, and invariants (constant, affine, translation,
rotation, intensity equivariance), plus a second, separately written
per-sample formulation.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

import synth
from helpers import (GOLDEN, pose_from_axes, random_grid, random_reps, read_golden_rows, rodrigues,
                     random_unit)
from oracle import bins, compound, geometry, literal, quant, reslice
from oracle.reslice import Params




# ----------------------------------------------------------------------------- helpers

def homogeneous_coords(P, C, width, height, pitch, origin, h):
    """Voxel coordinates of pixel centres via a plain library matmul (independent of geometry)."""
    T = np.asarray(P, np.float64) @ np.asarray(C, np.float64)
    jj, ii = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    u = np.stack([ii * pitch[0], jj * pitch[1], np.zeros_like(ii, dtype=float),
                  np.ones_like(ii, dtype=float)], axis=-1)
    p = u @ T.T
    return (p[..., :3] - origin) / h


def trilinear_lib(field, cc):
    """scipy order-1 interpolation of field (nz, ny, nx) at voxel coords cc (..., 3) [x, y, z]."""
    coords = np.stack([cc[..., 2].ravel(), cc[..., 1].ravel(), cc[..., 0].ravel()])
    return ndi.map_coordinates(field, coords, order=1, mode="grid-constant", cval=0.0).reshape(cc.shape[:-1])


def interior(cc, dims):
    nx, ny, nz = dims
    return ((cc[..., 0] >= 0) & (cc[..., 0] <= nx - 1) & (cc[..., 1] >= 0) & (cc[..., 1] <= ny - 1)
            & (cc[..., 2] >= 0) & (cc[..., 2] <= nz - 1))


def all_corners_valid(valid, cc):
    """True where every voxel of the trilinear cell (with non-zero weight) is valid."""
    nz, ny, nx = valid.shape
    b = np.floor(cc).astype(np.int64)
    ok = np.ones(cc.shape[:-1], bool)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                v = b + np.array([dx, dy, dz])
                frac_zero = np.zeros(cc.shape[:-1], bool)
                for a, d in enumerate((dx, dy, dz)):
                    if d == 1:
                        frac_zero |= (cc[..., a] == b[..., a])
                inside = ((v[..., 0] >= 0) & (v[..., 0] < nx) & (v[..., 1] >= 0) & (v[..., 1] < ny)
                          & (v[..., 2] >= 0) & (v[..., 2] < nz))
                vv = valid[np.clip(v[..., 2], 0, nz - 1), np.clip(v[..., 1], 0, ny - 1),
                           np.clip(v[..., 0], 0, nx - 1)]
                ok &= frac_zero | (inside & vv)
    return ok


@pytest.fixture(scope="module")
def cfg1():
    wl = synth.config1()
    wl.render("cpu")
    return wl


@pytest.fixture(scope="module")
def cfg1_grid(cfg1):
    prm = Params()
    g = compound.empty_grid(cfg1.origin, cfg1.spacing, cfg1.dims, prm.bin_tol_deg, prm.max_bins)
    compound.compound(g, cfg1.frames.numpy(), cfg1.sweep.probe_poses, cfg1.calib, cfg1.sweep.pitch)
    return g


# ----------------------------------------------------------------------------- P1: Eq. 2

def test_eq2_closed_forms():
    rows = read_golden_rows("eq2_weights.txt")
    prm = Params()
    rng = np.random.default_rng(11)
    C = synth.make_calibration(16, 0.5)
    for A, B, expected in rows:
        n_b = random_unit(rng)
        x_b = random_unit(rng)
        x_b = x_b - (x_b @ n_b) * n_b
        x_b /= np.linalg.norm(x_b)
        n_r = rodrigues(x_b, math.radians(A)) @ n_b
        x_r = rodrigues(n_r, math.radians(B)) @ x_b
        T = pose_from_axes(x_r, n_r, synth.WORLD_OFFSET_MM + rng.uniform(0, 30, 3))
        P = T @ np.linalg.inv(C)
        w = reslice.slice_weights(np.array([n_b]), np.array([x_b]), P, C, prm)
        assert w[0] == pytest.approx(expected, rel=1e-9, abs=1e-12), (A, B)


def test_eq2_weight_range_and_order():
    """Every surviving bin has w in [w(25,15), 1]: no underflow; the normal term is the steeper."""
    prm = Params()
    rng = np.random.default_rng(3)
    rn, rx = random_reps(rng, 4000)
    nr, xr = rn[0], rx[0]
    w = reslice.angular_weights(rn, rx, nr, xr, prm)
    live = w[w > 0]
    assert live.min() >= 0.3304 and live.max() <= 1.0 + 1e-12
    assert w[0] == pytest.approx(1.0)


# ----------------------------------------------------------------------------- geometry

def test_compose_matches_library_matmul():
    rng = np.random.default_rng(1)
    P = rng.standard_normal((20, 4, 4)).astype(np.float32)
    C = rng.standard_normal((4, 4))
    T = geometry.compose(P, C)
    np.testing.assert_allclose(T, P.astype(np.float64) @ C, rtol=1e-13, atol=1e-13)


def test_pixel_positions_match_homogeneous_transform():
    rng = np.random.default_rng(2)
    C = synth.make_calibration(9, 0.3)
    T = pose_from_axes(random_unit(rng), random_unit(rng), synth.WORLD_OFFSET_MM)
    P = (T @ np.linalg.inv(C)).astype(np.float32)
    p = geometry.pixel_positions(geometry.compose(P, C), 9, 7, (0.3, 0.2))
    cc = homogeneous_coords(P, C, 9, 7, (0.3, 0.2), np.zeros(3), 1.0)
    np.testing.assert_allclose(p, cc, rtol=0, atol=1e-9)


def test_bounds_brute_force():
    wl = synth.tiny_workload(4)
    o, dims = geometry.bounds_from_frames(wl.sweep.probe_poses, wl.sweep.width, wl.sweep.height,
                                          wl.sweep.pitch, wl.calib, 0.5)
    T = wl.sweep.probe_poses.astype(np.float64) @ wl.calib
    pts = []
    for f in range(len(T)):
        for i in range(wl.sweep.width):
            for j in range(wl.sweep.height):
                pts.append((T[f] @ np.array([i * wl.sweep.pitch[0], j * wl.sweep.pitch[1], 0, 1]))[:3])
    pts = np.array(pts)
    np.testing.assert_allclose(o, pts.min(0), atol=1e-9)
    for a in range(3):
        # the box holds every pixel centre and is at most one voxel larger than needed
        assert (dims[a] - 1) * 0.5 >= pts[:, a].max() - o[a] - 1e-9
        assert (dims[a] - 2) * 0.5 < pts[:, a].max() - o[a]


# ----------------------------------------------------------------------------- bins

def test_leader_clustering_hand_worked():
    rows = read_golden_rows("bins_leader.txt")
    angles, exp64, exp2 = rows
    x = np.array([1.0, 0.0, 0.0])
    n0 = np.array([0.0, 0.0, 1.0])
    nh = np.array([rodrigues(x, math.radians(a)) @ n0 for a in angles])
    xh = np.repeat(x[None], len(angles), 0)
    cb = bins.Codebook(3.0, 64)
    assert list(cb.assign(nh, xh)) == [int(v) for v in exp64]
    assert not cb.saturated
    cb2 = bins.Codebook(3.0, 2)
    assert list(cb2.assign(nh, xh)) == [int(v) for v in exp2]
    assert cb2.saturated


def test_zero_tolerance_gives_distinct_orientations():
    rng = np.random.default_rng(5)
    rn, rx = random_reps(rng, 7)
    idx = [0, 1, 0, 2, 3, 1, 4, 5, 6, 6]
    cb = bins.Codebook(0.0, 64)
    got = cb.assign(rn[idx], rx[idx])
    # identical orientations may or may not merge (dot of a unit vector with itself can round
    # below 1), but distinct ones never share a bin, and every bin's representative is exactly
    # the orientation of all its frames
    rep_n, rep_x = cb.arrays()
    for f, b in enumerate(got):
        np.testing.assert_array_equal(rep_n[b], rn[idx[f]])
        np.testing.assert_array_equal(rep_x[b], rx[idx[f]])


# ----------------------------------------------------------------------------- P10: compounding

def test_compound_brute_force_nearest_voxel_and_conservation():
    wl = synth.tiny_workload(7, N=6, n_frames=4, w=5)
    frames = wl.render("cpu").numpy()
    prm = Params()
    g = compound.empty_grid(wl.origin, wl.spacing, wl.dims, prm.bin_tol_deg, prm.max_bins)
    fb = compound.compound(g, frames, wl.sweep.probe_poses, wl.calib, wl.sweep.pitch)
    nx, ny, nz = wl.dims
    centres = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"),
                       -1).reshape(-1, 3) * wl.spacing + wl.origin
    S = np.zeros_like(g.S)
    Cn = np.zeros_like(g.C)
    n_in, s_in = 0, 0
    T = wl.sweep.probe_poses.astype(np.float64) @ wl.calib
    for f in range(len(frames)):
        for j in range(frames.shape[1]):
            for i in range(frames.shape[2]):
                p = (T[f] @ np.array([i * wl.sweep.pitch[0], j * wl.sweep.pitch[1], 0.0, 1.0]))[:3]
                d = np.abs(centres - p).max(axis=1)        # Chebyshev distance to every centre
                k = int(np.argmin(d))
                if d[k] <= wl.spacing / 2:                  # inside the grid's voxel cells
                    ix, iy, iz = np.unravel_index(k, (nx, ny, nz))
                    S[fb[f], iz, iy, ix] += frames[f, j, i]
                    Cn[fb[f], iz, iy, ix] += 1
                    n_in += 1
                    s_in += int(frames[f, j, i])
    np.testing.assert_array_equal(g.C, Cn)
    np.testing.assert_array_equal(g.S, S)
    assert g.C.sum() == n_in and g.S.sum() == s_in


# ----------------------------------------------------------------------------- P2 / P3 / P4

def test_single_bin_cancels_to_trilinear(cfg1):
    prm = Params()
    g = compound.empty_grid(cfg1.origin, cfg1.spacing, cfg1.dims, prm.bin_tol_deg, prm.max_bins)
    sel = cfg1.sweep.sweep_id == 0
    compound.compound(g, cfg1.frames.numpy()[sel], cfg1.sweep.probe_poses[sel], cfg1.calib,
                      cfg1.sweep.pitch)
    assert g.K == 1
    a, c = g.mean_count()
    sl = synth.slice_poses(77, synth.sweeps.Sweep(cfg1.sweep.probe_poses[sel], cfg1.sweep.image_poses[sel],
                                                  cfg1.sweep.centers[sel], cfg1.sweep.sweep_id[sel], 128, 128,
                                                  cfg1.sweep.pitch),
                           3, 3, 40, 40, (0.7, 0.7), 64, 0.5, cfg1.calib, max_rot_deg=5.0, trans_sigma_mm=1.0)
    checked = 0
    for P in sl.probe_poses:
        out = reslice.reslice_grid(g, cfg1.calib, P, 40, 40, (0.7, 0.7), prm)
        cc = homogeneous_coords(P, cfg1.calib, 40, 40, (0.7, 0.7), cfg1.origin, cfg1.spacing)
        ok = interior(cc, cfg1.dims) & all_corners_valid(c[0] > 0, cc)
        ref = trilinear_lib(a[0], cc)
        np.testing.assert_allclose(out[ok], ref[ok], rtol=0, atol=1e-9)
        checked += ok.sum()
    assert checked > 1000
    # a plane in the other sweep's orientation (40 deg in-plane away) discards the only bin
    Pother = cfg1.sweep.probe_poses[cfg1.sweep.sweep_id == 1][50]
    assert np.isnan(reslice.reslice_grid(g, cfg1.calib, Pother, 32, 32, (0.5, 0.5), prm)).all()


def test_directionality_off_is_plain_mean_compounding(cfg1, cfg1_grid):
    g = cfg1_grid
    assert g.K == 2
    prm = Params(k_normal=0.0, k_inplane=0.0, thr_normal_deg=90.0, thr_inplane_deg=90.0)
    pooled = g.S.sum(0).astype(np.float64)
    cnt = g.C.sum(0).astype(np.float64)
    mean = np.divide(pooled, cnt, out=np.zeros_like(cnt), where=cnt > 0)
    checked = 0
    for P in cfg1.slices.probe_poses[:6]:
        out = reslice.reslice_grid(g, cfg1.calib, P, 64, 64, (0.5, 0.5), prm)
        cc = homogeneous_coords(P, cfg1.calib, 64, 64, (0.5, 0.5), cfg1.origin, cfg1.spacing)
        ok = interior(cc, cfg1.dims) & all_corners_valid(cnt > 0, cc)
        np.testing.assert_allclose(out[ok], trilinear_lib(mean, cc)[ok], rtol=0, atol=1e-9)
        checked += ok.sum()
    assert checked > 5000


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_isotropic_grid_is_renormalised_trilinear(seed):
    rng = np.random.default_rng(seed)
    dims = (12, 10, 9)
    K = 4
    _, Cn = random_grid(rng, K, dims, p_empty=0.5)
    f = rng.integers(0, 256, size=(dims[2], dims[1], dims[0])).astype(np.float64)
    a = np.where(Cn > 0, f[None], 0.0)
    rn, rx = random_reps(rng, K)
    # the plane is aligned with bin 0; bins 1.. are random (mostly discarded)
    origin = np.array([3.0, -2.0, 7.0])
    T = pose_from_axes(rx[0], rn[0], origin + np.array([4.0, 3.0, 2.0]) + rng.uniform(-1, 1, 3))
    C = np.eye(4)
    prm = Params()
    w = reslice.slice_weights(rn, rx, T, C, prm)
    assert w[0] == pytest.approx(1.0)
    out = reslice.reslice(a, Cn.astype(float), origin, 1.0, rn, rx, C, T, 20, 20, (0.37, 0.41), prm)
    valid = ((Cn > 0) & (w[:, None, None, None] > 0)).any(0).astype(np.float64)
    cc = homogeneous_coords(T, C, 20, 20, (0.37, 0.41), origin, 1.0)
    num = trilinear_lib(f * valid, cc)
    den = trilinear_lib(valid, cc)
    ok = interior(cc, dims)
    ref = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.nan)
    np.testing.assert_array_equal(np.isnan(out[ok]), np.isnan(ref[ok]))
    m = ok & ~np.isnan(ref)
    assert m.sum() > 50
    np.testing.assert_allclose(out[m], ref[m], rtol=0, atol=1e-9)


def test_isotropic_pipeline_reslices_as_trilinear(cfg1):
    """Frames rendered from a voxel-constant field: every bin mean equals the field."""
    rng = np.random.default_rng(9)
    nx, ny, nz = cfg1.dims
    f = rng.integers(0, 256, size=(nz, ny, nx))
    T = cfg1.sweep.probe_poses.astype(np.float64) @ cfg1.calib
    w_, h_ = cfg1.sweep.width, cfg1.sweep.height
    frames = np.zeros((len(T), h_, w_), np.uint8)
    for k in range(len(T)):
        cc = homogeneous_coords(cfg1.sweep.probe_poses[k], cfg1.calib, w_, h_, cfg1.sweep.pitch,
                                cfg1.origin, cfg1.spacing)
        v = np.floor(cc + 0.5).astype(int)
        ins = ((v >= 0) & (v < np.array([nx, ny, nz]))).all(-1)
        vc = np.clip(v, 0, np.array([nx, ny, nz]) - 1)
        frames[k] = np.where(ins, f[vc[..., 2], vc[..., 1], vc[..., 0]], 0)
    prm = Params()
    g = compound.empty_grid(cfg1.origin, cfg1.spacing, cfg1.dims, prm.bin_tol_deg, prm.max_bins)
    compound.compound(g, frames, cfg1.sweep.probe_poses, cfg1.calib, cfg1.sweep.pitch)
    a, c = g.mean_count()
    assert np.all(a[c > 0] == np.broadcast_to(f, a.shape)[c > 0])
    for P in cfg1.slices.probe_poses[:4]:
        out = reslice.reslice_grid(g, cfg1.calib, P, 48, 48, (0.6, 0.6), prm)
        wts = reslice.slice_weights(*g.codebook.arrays(), P, cfg1.calib, prm)
        valid = ((c > 0) & (wts[:, None, None, None] > 0)).any(0).astype(float)
        cc = homogeneous_coords(P, cfg1.calib, 48, 48, (0.6, 0.6), cfg1.origin, cfg1.spacing)
        num, den = trilinear_lib(f * valid, cc), trilinear_lib(valid, cc)
        ok = interior(cc, cfg1.dims) & (den > 1e-6)
        np.testing.assert_allclose(out[ok], (num / np.where(den > 0, den, 1))[ok], rtol=0, atol=1e-8)


# ----------------------------------------------------------------------------- P5 / P6 / P13

def test_constant_volume_constant_image():
    rng = np.random.default_rng(4)
    dims = (10, 11, 12)
    K = 3
    _, Cn = random_grid(rng, K, dims, p_empty=0.4)
    a = np.where(Cn > 0, 173.0, 0.0)
    rn, rx = random_reps(rng, K)
    rn[1], rx[1] = rn[0], rx[0]
    T = pose_from_axes(rx[0], rn[0], np.array([5.0, 5.0, 5.0]))
    out = reslice.reslice(a, Cn.astype(float), np.zeros(3), 1.0, rn, rx, np.eye(4), T, 30, 30,
                          (0.3, 0.3), Params())
    m = ~np.isnan(out)
    assert m.sum() > 100
    np.testing.assert_allclose(out[m], 173.0, rtol=1e-13)


@pytest.mark.parametrize("R", [1, 2, 4])
def test_affine_field_reproduced(R):
    rng = np.random.default_rng(10 + R)
    dims = (14, 13, 15)
    K = 2
    _, Cn = random_grid(rng, K, dims, p_empty=0.0)
    alpha, beta = np.array([1.7, -2.3, 0.9]), 41.0
    zz, yy, xx = np.meshgrid(np.arange(dims[2]), np.arange(dims[1]), np.arange(dims[0]), indexing="ij")
    g = alpha[0] * xx + alpha[1] * yy + alpha[2] * zz + beta
    a = np.broadcast_to(g, (K,) + g.shape).astype(float)
    rn, rx = random_reps(rng, K)
    rn[1], rx[1] = rn[0], rx[0]
    origin = np.array([-850.0, 310.0, -1620.0])
    T = pose_from_axes(rx[0], rn[0], origin + 0.5 * (np.array(dims) - 1) / 2 + np.array([0.1, -0.2, 0.05]))
    T[:3, 3] -= 11.5 * 0.11 * T[:3, 0] + 11.5 * 0.13 * T[:3, 1]
    out = reslice.reslice(a, Cn.astype(float), origin, 0.5, rn, rx, np.eye(4), T, 24, 24, (0.11, 0.13),
                          Params(radius_vox=R))
    cc = homogeneous_coords(T, np.eye(4), 24, 24, (0.11, 0.13), origin, 0.5)
    ok = np.ones(cc.shape[:-1], bool)
    for ax in range(3):
        ok &= (cc[..., ax] >= R - 1) & (cc[..., ax] <= dims[ax] - R)
    assert ok.sum() > 100
    np.testing.assert_allclose(out[ok], (cc @ alpha + beta)[ok], rtol=0, atol=1e-8)


@pytest.mark.parametrize("R", [1, 2])
def test_face_pixels_take_the_last_layer(R):
    """Pixels 1e-9 below the grid's upper x face: their cells reach past the grid, so only the
    last layer (and, at R = 2, the one before it with a weight of about 1e-9) holds valid voxels.
    The tent weights renormalised over the valid voxels (Fig. 2 caption; Sec. 2.1: unassigned only
    when nothing in reach holds a sample) give the affine field's value on the last layer,
    whatever the size of the surviving weights."""
    rng = np.random.default_rng(30 + R)
    dims = (14, 13, 15)
    K = 2
    _, Cn = random_grid(rng, K, dims, p_empty=0.0)
    alpha, beta = np.array([1.7, -2.3, 0.9]), 41.0
    zz, yy, xx = np.meshgrid(np.arange(dims[2]), np.arange(dims[1]), np.arange(dims[0]), indexing="ij")
    g = alpha[0] * xx + alpha[1] * yy + alpha[2] * zz + beta
    a = np.broadcast_to(g, (K,) + g.shape).astype(float)
    rn = np.tile([0.0, 0.0, 1.0], (K, 1))
    rx = np.tile([1.0, 0.0, 0.0], (K, 1))
    origin, h = np.array([-850.0, 310.0, -1620.0]), 0.5
    W, H, i_face = 8, 8, 7
    T = np.eye(4)
    T[:3, 3] = origin + h * np.array([(dims[0] - 1e-9) - i_face * 0.5, 2.3, 4.4])
    out = reslice.reslice(a, Cn.astype(float), origin, h, rn, rx, np.eye(4), T, W, H, (0.25, 0.25),
                          Params(radius_vox=R))
    cc = homogeneous_coords(T, np.eye(4), W, H, (0.25, 0.25), origin, h)
    assert np.all(cc[:, i_face, 0] < dims[0]) and np.all(cc[:, i_face, 0] > dims[0] - 1e-8)
    face = out[:, i_face]
    assert not np.isnan(face).any()
    expect = alpha[0] * (dims[0] - 1) + alpha[1] * cc[:, i_face, 1] + alpha[2] * cc[:, i_face, 2] + beta
    np.testing.assert_allclose(face, expect, rtol=0, atol=1e-6)


def test_intensity_equivariance(cfg1, cfg1_grid):
    prm = Params()
    a, c = cfg1_grid.mean_count()
    rn, rx = cfg1_grid.codebook.arrays()
    P = cfg1.slices.probe_poses[2]
    out = reslice.reslice(a, c, cfg1.origin, cfg1.spacing, rn, rx, cfg1.calib, P, 50, 50, (0.6, 0.6), prm)
    out2 = reslice.reslice(-0.37 * a + 12.5, c, cfg1.origin, cfg1.spacing, rn, rx, cfg1.calib, P, 50, 50,
                           (0.6, 0.6), prm)
    m = ~np.isnan(out)
    assert m.sum() > 500
    np.testing.assert_array_equal(m, ~np.isnan(out2))
    np.testing.assert_allclose(out2[m], -0.37 * out[m] + 12.5, rtol=0, atol=1e-10)


# ----------------------------------------------------------------------------- P7: frame reproduction

def test_single_axis_aligned_frame_reproduced_exactly():
    rng = np.random.default_rng(12)
    h = 0.5
    origin = np.array([-850.0, 310.0, -1620.0])
    dims = (20, 8, 18)
    frame = rng.integers(0, 256, size=(1, 15, 17)).astype(np.uint8)
    T = np.eye(4)
    T[:3, 0] = (1.0, 0.0, 0.0)
    T[:3, 1] = (0.0, 0.0, 1.0)
    T[:3, 2] = (0.0, -1.0, 0.0)
    T[:3, 3] = origin + h * np.array([2.0, 5.0, 1.0])
    prm = Params()
    g = compound.empty_grid(origin, h, dims, prm.bin_tol_deg, prm.max_bins)
    compound.compound(g, frame, T[None].astype(np.float32), np.eye(4), (h, h))
    out = reslice.reslice_grid(g, np.eye(4), T, 17, 15, (h, h), prm)
    assert np.array_equal(out, frame[0].astype(np.float64))


def test_linear_ramp_reproduced_within_interpolation_error(cfg1):
    """Isotropic ramp phantom: at acquired poses |error| <= |grad| (sqrt(3)/2) h + 1 grey level."""
    alpha = np.array([2.1, -1.3, 3.2])          # grey levels per mm
    T = cfg1.sweep.probe_poses.astype(np.float64) @ cfg1.calib
    w_, h_ = cfg1.sweep.width, cfg1.sweep.height
    frames = np.zeros((len(T), h_, w_), np.uint8)
    for k in range(len(T)):
        cc = homogeneous_coords(cfg1.sweep.probe_poses[k], cfg1.calib, w_, h_, cfg1.sweep.pitch,
                                cfg1.origin, cfg1.spacing)
        frames[k] = np.clip(np.round(60.0 + (cc * cfg1.spacing) @ alpha), 0, 255)
    prm = Params()
    g = compound.empty_grid(cfg1.origin, cfg1.spacing, cfg1.dims, prm.bin_tol_deg, prm.max_bins)
    compound.compound(g, frames, cfg1.sweep.probe_poses, cfg1.calib, cfg1.sweep.pitch)
    bound = np.linalg.norm(alpha) * math.sqrt(3) / 2 * cfg1.spacing + 1.0
    for k in (10, 60, 130, 170):
        out = reslice.reslice_grid(g, cfg1.calib, cfg1.sweep.probe_poses[k], w_, h_, cfg1.sweep.pitch, prm)
        ref = frames[k].astype(float)
        unclipped = (ref > 0) & (ref < 255) & ~np.isnan(out)
        assert unclipped.sum() > 2000
        assert np.abs(out - ref)[unclipped].max() <= bound


# ----------------------------------------------------------------------------- P8: binned == literal

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_zero_tolerance_binned_equals_literal(seed):
    wl = synth.tiny_workload(seed)
    frames = wl.render("cpu").numpy()
    prm = Params(bin_tol_deg=0.0)
    g = compound.empty_grid(wl.origin, wl.spacing, wl.dims, 0.0, 64)
    compound.compound(g, frames, wl.sweep.probe_poses, wl.calib, wl.sweep.pitch)
    store = literal.SampleStore(wl.origin, wl.spacing, wl.dims)
    store.add_frames(frames, wl.sweep.probe_poses, wl.calib, wl.sweep.pitch)
    a, c = g.mean_count()
    rn, rx = g.codebook.arrays()
    sl = wl.slices
    n_assigned = 0
    for k, P in enumerate(sl.probe_poses):
        for spatial, norm, R in (("tent", "two_stage", 1), ("tent", "sample", 1), ("tent", "two_stage", 2),
                                 ("box", "two_stage", 1), ("box", "sample", 1)):
            prmR = Params(bin_tol_deg=0.0, radius_vox=R, thr_normal_deg=40.0, thr_inplane_deg=40.0)
            got = reslice.reslice(a, c, g.origin, g.spacing, rn, rx, wl.calib, P, sl.width, sl.height,
                                  sl.pitch, prmR, spatial=spatial, norm=norm)
            ref = literal.reslice(store, wl.calib, P, sl.width, sl.height, sl.pitch, prmR,
                                  spatial=spatial, norm=norm)
            np.testing.assert_array_equal(np.isnan(got), np.isnan(ref))
            m = ~np.isnan(ref)
            n_assigned += m.sum()
            np.testing.assert_allclose(got[m], ref[m], rtol=1e-12, atol=1e-10)
    assert n_assigned > 20


# ----------------------------------------------------------------------------- P11 / P12

def test_translation_invariance_fp64(cfg1):
    prm = Params()
    sel = slice(0, 200, 4)
    frames = cfg1.frames.numpy()[sel]
    P = cfg1.sweep.probe_poses[sel].astype(np.float64)
    D = np.array([1234.0, -777.0, 2048.0])
    outs = []
    for shift in (np.zeros(3), D):
        Ps = P.copy()
        Ps[:, :3, 3] += shift
        g = compound.empty_grid(cfg1.origin + shift, cfg1.spacing, cfg1.dims, prm.bin_tol_deg, prm.max_bins)
        compound.compound(g, frames, Ps, cfg1.calib, cfg1.sweep.pitch)
        Pr = cfg1.slices.probe_poses[1].copy()
        Pr[:3, 3] += shift
        outs.append(reslice.reslice_grid(g, cfg1.calib, Pr, 64, 64, (0.5, 0.5), prm))
    np.testing.assert_array_equal(np.isnan(outs[0]), np.isnan(outs[1]))
    m = ~np.isnan(outs[0])
    assert m.sum() > 1000
    np.testing.assert_allclose(outs[0][m], outs[1][m], rtol=0, atol=1e-9)


def test_half_turn_about_slice_normal(cfg1, cfg1_grid):
    prm = Params()
    W, H, pitch = 40, 30, (0.55, 0.45)
    P = cfg1.slices.probe_poses[3]
    T = P @ cfg1.calib
    T2 = T.copy()
    T2[:3, 0] = -T[:3, 0]
    T2[:3, 1] = -T[:3, 1]
    T2[:3, 3] = T[:3, 3] + (W - 1) * pitch[0] * T[:3, 0] + (H - 1) * pitch[1] * T[:3, 1]
    P2 = T2 @ np.linalg.inv(cfg1.calib)
    out = reslice.reslice_grid(cfg1_grid, cfg1.calib, P, W, H, pitch, prm)
    out2 = reslice.reslice_grid(cfg1_grid, cfg1.calib, P2, W, H, pitch, prm)
    rot = out[::-1, ::-1]
    np.testing.assert_array_equal(np.isnan(rot), np.isnan(out2))
    m = ~np.isnan(rot)
    assert m.sum() > 300
    np.testing.assert_allclose(out2[m], rot[m], rtol=0, atol=1e-8)


# ----------------------------------------------------------------------------- storage forms

def _cast_lib(x, dt):
    return torch.from_numpy(np.asarray(x, np.float32)).to(dt).to(torch.float64).numpy()


@pytest.mark.parametrize("fmt,dt,vmax", [("bf16", torch.bfloat16, 3.0e38), ("fp16", torch.float16, 65504.0),
                                         ("e4m3", torch.float8_e4m3fn, 448.0)])
def test_round_to_nearest_even_matches_library_casts(fmt, dt, vmax):
    rng = np.random.default_rng(6)
    x = np.concatenate([
        rng.standard_normal(20000) * 3, rng.uniform(-1, 1, 20000) * min(vmax, 1e4),
        rng.uniform(-1e-3, 1e-3, 5000), rng.uniform(-0.02, 0.02, 5000),
        np.arange(-300, 300) / 4.0, np.arange(0, 2048) * 0.5 + 0.25,
    ]).astype(np.float32)
    x = x[np.abs(x) <= vmax]
    # exact ties between neighbouring representable values, built from the library's own grid
    grid = np.unique(_cast_lib(rng.uniform(-min(vmax, 400), min(vmax, 400), 4000), dt))
    mids = ((grid[:-1] + grid[1:]) / 2).astype(np.float32)
    x = np.concatenate([x, mids[(mids.astype(np.float64) == (grid[:-1] + grid[1:]) / 2)]])
    np.testing.assert_array_equal(quant.rne(x, fmt), _cast_lib(x, dt))


def test_storage_forms_error_bounds():
    rng = np.random.default_rng(8)
    S, Cn = random_grid(rng, 2, (16, 16, 16), p_empty=0.2, max_count=300)
    a64 = np.divide(S, Cn, out=np.zeros(S.shape), where=Cn > 0)
    has = Cn > 0
    bounds = {"fp32": 1e-4, "fp16": 2.0 ** -11 * 127.5 + 1e-4, "bf16": 2.0 ** -8 * 127.5 + 1e-4}
    for form, bnd in bounds.items():
        a, c = quant.storage(S, Cn, form)
        assert np.abs(a[has] - a64[has]).max() <= bnd, form
        assert np.all(c[has] > 0) and np.all(c[~has] == 0)
    a, c = quant.storage(S, Cn, "fp8")
    s_val, _ = quant.fp8_scales(S, Cn)
    sv = quant.brick_expand(s_val, S.shape)
    assert np.all(np.abs(a[has] - a64[has]) <= 16.0 * sv[has] + 1e-3)
    assert np.all(c[has] > 0)
    # counts: exact in fp16 up to 2048, in bf16 up to 256
    a16, c16 = quant.storage(S, Cn, "fp16")
    small = has & (Cn <= 256)
    np.testing.assert_array_equal(c16[small], Cn[small])


# FP8 storage form: codes and per-(bin, brick) scales, pinned independently of the oracle's
# own scale computation (hand-worked brick, and properties of the construction).

def _fp8_golden():
    rows = read_golden_rows("fp8_brick.txt")
    scales = {}
    with open(os.path.join(GOLDEN, "fp8_brick.txt")) as fh:
        for line in fh:
            if line.startswith("#S"):
                b, sv, sc = line.split()[1:]
                scales[int(b)] = (float(sv), float(sc))
    return rows, scales


def _fp8_pin_failures(encode):
    """Names of the fp8 pins that ``encode(S, C) -> (qv, qc, s_val, s_cnt)`` breaks."""
    bad = []
    rows, scales = _fp8_golden()
    S = np.zeros((2, 8, 8, 8), np.int64)
    C = np.zeros_like(S)
    for b, x, y, z, s_, c_, _, _ in rows:
        S[int(b), int(z), int(y), int(x)] = int(s_)
        C[int(b), int(z), int(y), int(x)] = int(c_)
    qv, qc, sv, sc = encode(S, C)
    for b, x, y, z, _, _, q_val, q_cnt in rows:
        at = (int(b), int(z), int(y), int(x))
        if qv[at] != q_val or qc[at] != q_cnt:
            bad.append("hand-worked codes")
            break
    for b, (s_val, s_cnt) in scales.items():
        if abs(float(sv[b, 0, 0, 0]) / s_val - 1) > 1e-7 or abs(float(sc[b, 0, 0, 0]) / s_cnt - 1) > 1e-7:
            bad.append("hand-worked scales")
            break
    # random grids whose values stay near mid-grey (so an empty voxel, read as 0, would be the
    # farthest from 127.5) and whose counts vary per brick
    rng = np.random.default_rng(81)
    K, n = 3, 24
    C = rng.integers(1, 40, size=(K, n, n, n)) * (rng.random((K, n, n, n)) > 0.4)
    C[:, :8, :8, :8] = 0                        # whole empty bricks
    a = rng.uniform(100.0, 160.0, C.shape)
    S = np.where(C > 0, np.floor(a * C), 0).astype(np.int64)
    qv, qc, sv, sc = encode(S, C)
    has = C > 0
    if np.any(qv[~has] != 0) or np.any(qc[~has] != 0):
        bad.append("empty voxels encode to 0")
    for b in range(K):
        for bz in range(0, n, 8):
            for by in range(0, n, 8):
                for bx in range(0, n, 8):
                    sl = (b, slice(bz, bz + 8), slice(by, by + 8), slice(bx, bx + 8))
                    occ = has[sl]
                    if not occ.any():
                        continue
                    # brute force, from the voxels' own means
                    amean = np.float32(S[sl][occ]) / np.float32(C[sl][occ])
                    dev = np.abs(amean.astype(np.float64) - 127.5)
                    if dev.max() > 1e-3 and np.abs(qv[sl][occ]).max() != 448.0:
                        bad.append("farthest voxel encodes to 448")
                        return bad
                    if qc[sl][occ].max() != 448.0 or qc[sl][occ][np.argmax(C[sl][occ])] != 448.0:
                        bad.append("largest count encodes to 448")
                        return bad
                    if np.any(qc[sl][occ] <= 0) or np.any(np.abs(qv[sl][occ]) > 448):
                        bad.append("code range")
                        return bad
                    # 3 mantissa bits: relative half-quantum 2^-4 of the value's distance from 127.5
                    dec = qv[sl][occ] * float(sv[b, bz // 8, by // 8, bx // 8]) + 127.5
                    err = np.abs(dec - amean)
                    if np.any(err > dev * 2.0 ** -4 + 1e-4):
                        bad.append("value error within e4m3 precision")
                        return bad
    return bad


def _fp8_mutant(value_div=448.0, scale_over_empty=False, count_div=448.0):
    """The fp8 encoding with one planted mistake (used only to show that the pins catch it)."""
    def enc(S, C):
        has = np.asarray(C) > 0
        a32 = quant.mean32(S, C)
        dev = np.abs((a32 - np.float32(127.5)).astype(np.float32)).astype(np.float64)
        if not scale_over_empty:
            dev = np.where(has, dev, -np.inf)
        m = quant.brick_reduce_max(dev)
        m = np.where(np.isfinite(m), m, 0.0).astype(np.float32)
        s_val = np.maximum((m / np.float32(value_div)).astype(np.float32), np.float32(2.0 ** -20))
        cm = quant.brick_reduce_max(np.where(has, np.asarray(C, np.float64), -np.inf))
        cm = np.where(np.isfinite(cm), cm, 448.0).astype(np.float32)
        s_cnt = (cm / np.float32(count_div)).astype(np.float32)
        sv = quant.brick_expand(s_val, S.shape)
        sc = quant.brick_expand(s_cnt, S.shape)
        x = ((a32 - np.float32(127.5)).astype(np.float32) / sv).astype(np.float32)
        qv = np.where(has, quant.rne(x, "e4m3"), 0.0)
        qc = np.where(has, quant.rne((np.asarray(C, np.float32) / sc).astype(np.float32), "e4m3"), 0.0)
        return qv, qc, s_val, s_cnt
    return enc


def test_fp8_codes_and_scales_pinned():
    assert _fp8_pin_failures(quant.fp8_encode) == []
    # the same construction written again with no mistake passes, each planted mistake fails
    assert _fp8_pin_failures(_fp8_mutant()) == []
    for kw in ({"value_div": 224.0}, {"scale_over_empty": True}, {"count_div": 224.0}, {"count_div": 512.0}):
        assert _fp8_pin_failures(_fp8_mutant(**kw)), kw


def test_fp8_storage_decodes_the_codes():
    rng = np.random.default_rng(82)
    S, Cn = random_grid(rng, 2, (16, 16, 16), p_empty=0.3, max_count=60)
    qv, qc, sv, sc = quant.fp8_encode(S, Cn)
    a, c = quant.storage(S, Cn, "fp8")
    has = Cn > 0
    svx, scx = quant.brick_expand(sv, S.shape), quant.brick_expand(sc, S.shape)
    np.testing.assert_array_equal(a[has], ((qv * svx).astype(np.float32) + np.float32(127.5))[has])
    np.testing.assert_array_equal(c[has], (qc * scx).astype(np.float32)[has])


# ---------------------------------------------------------------- evaluation metrics (Sec. 3)

from oracle import metrics  # noqa: E402


def test_ncc_pins():
    rng = np.random.default_rng(31)
    a = rng.uniform(0, 255, (23, 17))
    assert metrics.ncc(a, a)[0] == pytest.approx(1.0, abs=1e-12)
    assert metrics.ncc(a, 3.0 * a + 7.0)[0] == pytest.approx(1.0, abs=1e-12)
    assert metrics.ncc(a, 100.0 - 2.0 * a)[0] == pytest.approx(-1.0, abs=1e-12)
    b = rng.uniform(0, 255, a.shape)
    holes = a.copy()
    holes[rng.random(a.shape) < 0.3] = np.nan
    m = np.isfinite(holes)
    got, n = metrics.ncc(holes, b)
    assert n == int(m.sum())
    assert got == pytest.approx(float(np.corrcoef(a[m], b[m])[0, 1]), abs=1e-12)


def test_ssim_pins():
    rng = np.random.default_rng(32)
    g = metrics.gaussian_window()
    assert g.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(g, g.T) and np.allclose(g, g[::-1, ::-1])
    a = rng.uniform(0, 255, (26, 21))
    b = np.clip(a + rng.normal(0, 25, a.shape), 0, 255)
    assert metrics.ssim(a, a)[0] == pytest.approx(1.0, abs=1e-12)
    s_ab, n = metrics.ssim(a, b)
    assert n == (26 - 10) * (21 - 10)
    assert s_ab == pytest.approx(metrics.ssim(b, a)[0], abs=1e-12)
    # the same index from separable Gaussian filtering (radius 5 = truncate 5 / 1.5)
    f = lambda x: ndi.gaussian_filter(x, 1.5, truncate=5.0 / 1.5, mode="constant")  # noqa: E731
    ma, mb = f(a), f(b)
    va, vb, cab = f(a * a) - ma * ma, f(b * b) - mb * mb, f(a * b) - ma * mb
    c1, c2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    smap = ((2 * ma * mb + c1) * (2 * cab + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2))
    assert s_ab == pytest.approx(float(smap[5:-5, 5:-5].mean()), abs=1e-9)
    assert s_ab < 0.99
    # an unassigned pixel removes exactly the windows that contain it
    holes = a.copy()
    holes[9, 12] = np.nan
    got, n2 = metrics.ssim(holes, b)
    inside = [(j, i) for j in range(5, 21) for i in range(5, 16) if abs(j - 9) <= 5 and abs(i - 12) <= 5]
    assert n2 == n - len(inside)
    keep = np.ones_like(smap, bool)
    for j, i in inside:
        keep[j, i] = False
    keep[:5], keep[-5:], keep[:, :5], keep[:, -5:] = False, False, False, False
    assert got == pytest.approx(float(smap[keep].mean()), abs=1e-9)
