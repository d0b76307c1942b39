"""Compounding frames of a curvilinear or phased-array probe (FP64 / exact integers).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper acquires with a linear array (Sec. 2.2), whose pixels sit on a rectangular grid in the
image plane and whose samples all share the frame's in-plane direction.  Eq. 1 compares each
sample's acquisition normal and in-plane direction (x-axis) with the reslice plane's.  A fan
probe's beams leave one apex at different angles, so the in-plane direction varies across the
columns.  Readings:

  * Column i's beam has unit direction b_i = (b_i0, b_i1) in image millimetres (lateral, axial),
    given as an input table, so both sides take the same values and no trigonometry enters.
    Pixel (i, j) sits on that beam at r_j = r0 + j dr from the apex a = (a0, a1):
        u = a0 + r_j b_i0,   v = a1 + r_j b_i1   (image mm, evaluated in that order),
    and in the world at p = (t + u e0) + v e1, exactly as a linear-array pixel at (u, v).
    A phased array is the case r0 = 0 (the beams leave one point on the face).
  * A sample's in-plane direction is the image-plane direction across its beam,
    x = b1 xhat - b0 yhat, with xhat = e0 / |e0| and yhat = e1 / |e1| (a beam along the axial
    axis, b = (0, 1), gives xhat, the linear array's direction).  The acquisition normal is the
    frame's image-plane normal, as for a linear array (normal_axis 2 only).
  * Binning per column fan: the columns are split into G sectors, column i in sector
    floor(i G / W).  Sector g's samples share the in-plane direction of its middle column
    m_g = floor((first_g + last_g) / 2), first_g = ceil(g W / G), last_g = ceil((g + 1) W / G) - 1.
    The (frame, sector) orientations enter the leader clustering of ``oracle.bins`` in
    frame-major order, sectors in order: each is one entry of the codebook's frame list.
Positions, nearest voxel and accumulation are then those of ``oracle.compound``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import geometry
from .compound import DirGrid


@dataclass
class Fan:
    apex: tuple               # (a0, a1) image mm
    r0: float                 # radius of the first row from the apex, mm
    dr: float                 # radial step per row, mm
    sectors: int              # G


def pixel_uv(fan: Fan, beams, width: int, height: int):
    """Image-mm (u, v) of every pixel, each (height, width)."""
    b = np.asarray(beams, np.float64).reshape(width, 2)
    r = float(fan.r0) + np.arange(height, dtype=np.float64) * float(fan.dr)
    u = float(fan.apex[0]) + r[:, None] * b[None, :, 0]
    v = float(fan.apex[1]) + r[:, None] * b[None, :, 1]
    return u, v


def sector_of_columns(width: int, sectors: int) -> np.ndarray:
    return (np.arange(width, dtype=np.int64) * sectors) // width


def sector_middle_columns(width: int, sectors: int) -> np.ndarray:
    g = np.arange(sectors, dtype=np.int64)
    first = (g * width + sectors - 1) // sectors
    last = ((g + 1) * width + sectors - 1) // sectors - 1
    return (first + last) // 2


def sector_axes(T, beams, width: int, sectors: int):
    """(nhat, x) per (frame, sector), each (F, G, 3): the frames' image-plane normals and the
    sectors' in-plane directions."""
    T = np.asarray(T, np.float64)
    _, e0, e1, xhat, nhat = geometry.axes(T, 2)
    yhat = geometry._unit(e1)
    b = np.asarray(beams, np.float64).reshape(width, 2)[sector_middle_columns(width, sectors)]   # (G, 2)
    x = b[None, :, 1, None] * xhat[:, None, :] - b[None, :, 0, None] * yhat[:, None, :]
    n = np.broadcast_to(nhat[:, None, :], x.shape)
    return n, x


def pixel_positions(T, fan: Fan, beams, width: int, height: int) -> np.ndarray:
    """World positions (height, width, 3) of one fan frame's pixels."""
    t, e0, e1, _, _ = geometry.axes(T)
    u, v = pixel_uv(fan, beams, width, height)
    p = t[None, None, :] + u[..., None] * e0[None, None, :]
    return p + v[..., None] * e1[None, None, :]


def compound_fan(grid: DirGrid, frames, probe_poses, calib, fan: Fan, beams) -> np.ndarray:
    """Add fan frames (F, H, W) uint8 with probe poses (F, 4, 4) to ``grid`` in place.
    Returns the bin of every (frame, sector), (F, G)."""
    frames = np.asarray(frames)
    F, H, W = frames.shape
    G = int(fan.sectors)
    T = geometry.compose(np.asarray(probe_poses), np.asarray(calib))
    n, x = sector_axes(T, beams, W, G)
    bins = grid.codebook.assign(n.reshape(-1, 3), x.reshape(-1, 3)).reshape(F, G)
    K = grid.codebook.K
    nx, ny, nz = grid.dims
    if grid.S.shape[0] < K:
        pad = K - grid.S.shape[0]
        grid.S = np.concatenate([grid.S, np.zeros((pad, nz, ny, nx), np.int64)])
        grid.C = np.concatenate([grid.C, np.zeros((pad, nz, ny, nx), np.int64)])
    flatS = grid.S.reshape(-1)
    flatC = grid.C.reshape(-1)
    nvox = nx * ny * nz
    col_bin = np.empty((F, W), np.int64)
    sec = sector_of_columns(W, G)
    for f in range(F):
        col_bin[f] = bins[f][sec]
        p = pixel_positions(T[f], fan, beams, W, H)
        v = geometry.nearest_voxel(geometry.voxel_coords(p, grid.origin, grid.spacing))
        inside = ((v[..., 0] >= 0) & (v[..., 0] < nx) & (v[..., 1] >= 0) & (v[..., 1] < ny)
                  & (v[..., 2] >= 0) & (v[..., 2] < nz))
        b = np.broadcast_to(col_bin[f][None, :], (H, W))[inside]
        vi = v[inside]
        lin = b * nvox + (vi[:, 2] * ny + vi[:, 1]) * nx + vi[:, 0]
        np.add.at(flatS, lin, frames[f][inside].astype(np.int64))
        np.add.at(flatC, lin, 1)
    return bins
