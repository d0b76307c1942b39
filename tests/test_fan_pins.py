"""Pins of the fan-probe oracle (``oracle.fan``) against facts fixed outside it: closed forms of
the fan geometry, a compounding worked by hand, the reduction of a one-column fan to the pinned
linear-array compounding, and the per-sector axes' orthogonality and binning.  CPU only."""
from __future__ import annotations

import math

import numpy as np

from oracle import compound, fan, geometry


def _beams(deg):
    t = np.deg2rad(np.asarray(deg, np.float64))
    return np.stack([np.sin(t), np.cos(t)], axis=1)


def _pose(rng):
    a, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(a) < 0:
        a[:, 0] = -a[:, 0]
    T = np.eye(4)
    T[:3, :3] = a
    T[:3, 3] = rng.normal(0.0, 5.0, 3)
    return T


def test_fan_geometry_closed_forms():
    """Every pixel lies on its column's beam at r0 + j dr from the apex, in image millimetres and
    in the world (p - (t + a0 e0 + a1 e1) = r (b0 e0 + b1 e1))."""
    rng = np.random.default_rng(5)
    W, H = 37, 23
    b = _beams(np.sort(rng.uniform(-40.0, 40.0, W)))
    f = fan.Fan(apex=(3.25, -7.5), r0=11.0, dr=0.3, sectors=5)
    u, v = fan.pixel_uv(f, b, W, H)
    r = 11.0 + 0.3 * np.arange(H)
    du, dv = u - 3.25, v + 7.5
    np.testing.assert_allclose(np.hypot(du, dv), np.broadcast_to(r[:, None], (H, W)), rtol=1e-13)
    np.testing.assert_allclose(du * b[None, :, 1] - dv * b[None, :, 0], 0.0, atol=1e-12)    # on the beam
    assert (du * b[None, :, 0] + dv * b[None, :, 1] > 0).all()                               # past the apex
    T = _pose(rng)
    p = fan.pixel_positions(T, f, b, W, H)
    e0, e1, t = T[:3, 0], T[:3, 1], T[:3, 3]
    ref = (t + 3.25 * e0 - 7.5 * e1)[None, None, :] + r[:, None, None] * (
        b[None, :, 0, None] * e0[None, None, :] + b[None, :, 1, None] * e1[None, None, :])
    np.testing.assert_allclose(p, ref, atol=1e-11)


def test_sector_partition_and_axes():
    """Sectors split the columns into contiguous runs whose sizes differ by at most one, each
    middle column inside its sector; the sector axis is a unit vector in the image plane across
    its middle beam, and a sector whose middle beam is axial takes the frame's x axis."""
    rng = np.random.default_rng(8)
    for W, G in ((96, 8), (97, 8), (10, 10), (13, 1), (64, 7)):
        sec = fan.sector_of_columns(W, G)
        assert sec[0] == 0 and sec[-1] == G - 1 and (np.diff(sec) >= 0).all() and (np.diff(sec) <= 1).all()
        sizes = np.bincount(sec, minlength=G)
        assert sizes.min() >= 1 and sizes.max() - sizes.min() <= 1
        mid = fan.sector_middle_columns(W, G)
        assert np.array_equal(sec[mid], np.arange(G))
    W, G = 45, 9                     # odd sector count, symmetric fan: the middle sector is axial
    b = _beams((np.arange(W) - (W - 1) / 2.0) * 0.9)
    T = np.stack([_pose(rng) for _ in range(3)])
    n, x = fan.sector_axes(T, b, W, G)
    _, _, _, xhat, nhat = geometry.axes(T)
    yhat = T[:, :3, 1] / np.linalg.norm(T[:, :3, 1], axis=1)[:, None]
    bm = b[fan.sector_middle_columns(W, G)]
    beam_world = bm[None, :, 0, None] * xhat[:, None, :] + bm[None, :, 1, None] * yhat[:, None, :]
    np.testing.assert_allclose(np.linalg.norm(x, axis=-1), 1.0, atol=1e-13)
    np.testing.assert_allclose((x * beam_world).sum(-1), 0.0, atol=1e-13)
    np.testing.assert_allclose((x * nhat[:, None, :]).sum(-1), 0.0, atol=1e-13)
    assert np.array_equal(x[:, G // 2], xhat) and np.array_equal(n[:, 0], nhat)
    # the angle between sector axes equals the angle between their beams
    ang = np.degrees(np.arccos(np.clip((x[:, 0] * x[:, -1]).sum(-1), -1, 1)))
    beam_ang = np.degrees(np.arccos(bm[0] @ bm[-1]))
    np.testing.assert_allclose(ang, beam_ang, atol=1e-9)


def test_fan_compound_worked_by_hand():
    """Identity pose and calibration (image mm = world mm), 1 mm voxels from the origin; apex (8, 0),
    first row at 2 mm, 1 mm rows, three beams along (-0.6, 0.8), (0, 1) and (0.6, 0.8), one column
    per sector.  Pixel centres and voxels worked out by hand:
      column 0: (6.8, 1.6) -> (7, 2), (6.2, 2.4) -> (6, 2), (5.6, 3.2) -> (6, 3)
      column 1: (8, 2), (8, 3), (8, 4)
      column 2: (9.2, 1.6) -> (9, 2), (9.8, 2.4) -> (10, 2), (10.4, 3.2) -> (10, 3).
    Sector axes 0.8 x + 0.6 y, x, 0.8 x - 0.6 y: at 5 degrees three bins; at 40 degrees
    (cos = 0.766 < 0.8) the axial sector joins the first, and the third (|0.28| < 0.766) opens a
    second bin."""
    b = np.array([[-0.6, 0.8], [0.0, 1.0], [0.6, 0.8]])
    f = fan.Fan(apex=(8.0, 0.0), r0=2.0, dr=1.0, sectors=3)
    frame = np.array([[[1 + 10 * i + j for i in range(3)] for j in range(3)]], np.uint8)   # (1, H=3, W=3)
    P = np.eye(4, dtype=np.float32)[None]
    hand = {0: [(7, 2), (6, 2), (6, 3)], 1: [(8, 2), (8, 3), (8, 4)], 2: [(9, 2), (10, 2), (10, 3)]}
    for tol, expect_bins in ((5.0, [0, 1, 2]), (40.0, [0, 0, 1])):
        g = compound.empty_grid((0.0, 0.0, 0.0), 1.0, (12, 6, 1), tol, 64)
        got = fan.compound_fan(g, frame, P, np.eye(4), f, b)
        assert got.tolist() == [expect_bins], (tol, got)
        S = np.zeros_like(g.S)
        C = np.zeros_like(g.C)
        for i, cells in hand.items():
            for j, (vx, vy) in enumerate(cells):
                S[expect_bins[i], 0, vy, vx] += 1 + 10 * i + j
                C[expect_bins[i], 0, vy, vx] += 1
        assert np.array_equal(g.S, S) and np.array_equal(g.C, C), tol
    n = np.array(g.codebook.rep_x)
    np.testing.assert_allclose(n, [[0.8, 0.6, 0.0], [0.8, -0.6, 0.0]], atol=1e-15)


def test_one_column_fan_is_a_linear_frame():
    """A fan of one axial beam from the origin with r0 = 0 and dr = sy places row j at image mm
    (0, j sy), as a one-column linear frame: compounding, bins and codebook are bit-identical to
    the linear oracle's (itself pinned by brute force)."""
    rng = np.random.default_rng(21)
    F, H, sy = 7, 40, 0.37
    T = np.stack([_pose(rng) for _ in range(F)])
    T[:, :3, 3] = rng.uniform(4.0, 8.0, (F, 3))
    P = T.astype(np.float32)
    frames = rng.integers(0, 256, (F, H, 1), dtype=np.uint8)
    ga = compound.empty_grid((0.0, 0.0, 0.0), 0.5, (40, 40, 40), 5.0, 64)
    gb = compound.empty_grid((0.0, 0.0, 0.0), 0.5, (40, 40, 40), 5.0, 64)
    ba = fan.compound_fan(ga, frames, P, np.eye(4), fan.Fan(apex=(0.0, 0.0), r0=0.0, dr=sy, sectors=1),
                          np.array([[0.0, 1.0]]))
    bb = compound.compound(gb, frames, P, np.eye(4), (1.0, sy))
    assert np.array_equal(ba[:, 0], bb)
    assert np.array_equal(ga.S, gb.S) and np.array_equal(ga.C, gb.C) and ga.C.sum() > 0
    assert np.array_equal(np.array(ga.codebook.rep_x), np.array(gb.codebook.rep_x))


def test_fan_conservation_and_sector_bins():
    """On the curvilinear workload, every in-grid pixel is counted once, and each bin's samples
    come from the (frame, sector) entries assigned to it."""
    import synth
    wl = synth.fan_config(sectors=4)
    wl.sweep.probe_poses = wl.sweep.probe_poses[::20]
    fr = wl.render("cpu").numpy()
    f = fan.Fan(apex=wl.fan["apex"], r0=wl.fan["r0"], dr=wl.fan["dr"], sectors=4)
    g = compound.empty_grid(wl.origin, wl.spacing, wl.dims, 5.0, 64)
    bins_fg = fan.compound_fan(g, fr, wl.sweep.probe_poses, wl.calib, f, wl.beams)
    T = geometry.compose(wl.sweep.probe_poses, wl.calib)
    sec = fan.sector_of_columns(fr.shape[2], 4)
    counts = np.zeros(g.K, np.int64)
    for k in range(fr.shape[0]):
        p = fan.pixel_positions(T[k], f, wl.beams, fr.shape[2], fr.shape[1])
        c = np.floor((p - wl.origin) / wl.spacing + 0.5)
        inside = ((c >= 0) & (c < np.asarray(wl.dims))).all(-1)
        np.add.at(counts, bins_fg[k][sec][None, :].repeat(fr.shape[1], 0)[inside], 1)
    assert np.array_equal(g.C.reshape(g.K, -1).sum(1), counts)
    assert math.isclose(float(g.C.sum()), float(counts.sum()))
