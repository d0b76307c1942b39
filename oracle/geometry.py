"""Pose composition, frame axes and pixel positions (FP64).

Sec. 2.1 "Volume reconstruction": each image is transformed to its pose
relative to the tracking setup; a bounding box is computed from the collected
transducer positions.  The paper gives no formulas; the readings are:

  * The tracker reports the probe pose P (probe -> world, float32 promoted
    exactly to FP64); the calibration C maps image millimetres to the probe.
    The image pose is T = P . C, each entry summed left to right,
    T[r][c] = ((P[r][0] C[0][c] + P[r][1] C[1][c]) + P[r][2] C[2][c]) + P[r][3] C[3][c],
    with no fused multiply-add, so that voxel decisions are reproducible.
  * Pixel (i, j) (column i lateral, row j depth) sits at image millimetres
    (i sx, j sy, 0), i.e. at world p = (t + (i sx) e0) + (j sy) e1 where e0, e1
    are columns 0 and 1 of T and t its translation, evaluated in that order.
  * Directions: the in-plane (x) axis is e0 / |e0|; the acquisition normal is
    the image-plane normal e2 / |e2| (normal_axis = 2), or the beam axis
    e1 / |e1| (normal_axis = 1).  |v| = sqrt((v0 v0 + v1 v1) + v2 v2).
  * Voxel coordinates: c = (p - o) * (1 / h), 1 / h computed once.
"""
from __future__ import annotations

import math

import numpy as np


def compose(P, C) -> np.ndarray:
    """T = P . C for one pose or a stack (..., 4, 4); fixed summation order."""
    P = np.asarray(P).astype(np.float64)
    C = np.asarray(C, dtype=np.float64)
    T = np.empty(np.broadcast_shapes(P.shape, C.shape))
    for r in range(4):
        for c in range(4):
            acc = P[..., r, 0] * C[..., 0, c]
            acc = acc + P[..., r, 1] * C[..., 1, c]
            acc = acc + P[..., r, 2] * C[..., 2, c]
            acc = acc + P[..., r, 3] * C[..., 3, c]
            T[..., r, c] = acc
    return T


def _unit(v: np.ndarray) -> np.ndarray:
    n = np.sqrt((v[..., 0] * v[..., 0] + v[..., 1] * v[..., 1]) + v[..., 2] * v[..., 2])
    return v / n[..., None]


def axes(T: np.ndarray, normal_axis: int = 2):
    """(t, e0, e1, xhat, nhat) of image pose(s) T."""
    T = np.asarray(T, dtype=np.float64)
    t = T[..., :3, 3]
    e0 = T[..., :3, 0]
    e1 = T[..., :3, 1]
    xhat = _unit(e0)
    nhat = _unit(T[..., :3, normal_axis])
    return t, e0, e1, xhat, nhat


def pixel_positions(T: np.ndarray, width: int, height: int, pitch) -> np.ndarray:
    """World positions (height, width, 3) of a frame's or slice's pixel centres."""
    t, e0, e1, _, _ = axes(T)
    i = np.arange(width, dtype=np.float64) * float(pitch[0])      # i * sx
    j = np.arange(height, dtype=np.float64) * float(pitch[1])     # j * sy
    p = t[None, None, :] + i[None, :, None] * e0[None, None, :]
    p = p + j[:, None, None] * e1[None, None, :]
    return p


def voxel_coords(p: np.ndarray, origin, spacing: float) -> np.ndarray:
    """Continuous voxel coordinates c = (p - o) * (1/h)."""
    inv_h = 1.0 / float(spacing)
    return (p - np.asarray(origin, dtype=np.float64)) * inv_h


def nearest_voxel(c: np.ndarray) -> np.ndarray:
    """Nearest voxel index, ties rounded up: floor(c + 0.5)."""
    return np.floor(c + 0.5).astype(np.int64)


def bounds_from_frames(probe_poses, width: int, height: int, pitch, calib, spacing: float):
    """Axis-aligned box of all frames' corner pixel centres.

    Returns (origin, dims): origin is the minimum corner, dims[a] =
    ceil((max_a - min_a) / h) + 1 so that both extreme corners have a voxel.
    """
    T = compose(np.asarray(probe_poses), np.asarray(calib))
    corners = []
    for (i, j) in ((0, 0), (width - 1, 0), (0, height - 1), (width - 1, height - 1)):
        t, e0, e1, _, _ = axes(T)
        p = (t + (i * float(pitch[0])) * e0) + (j * float(pitch[1])) * e1
        corners.append(p.reshape(-1, 3))
    allp = np.concatenate(corners)
    lo, hi = allp.min(axis=0), allp.max(axis=0)
    dims = [int(math.ceil((hi[a] - lo[a]) / spacing)) + 1 for a in range(3)]
    return lo, tuple(dims)
