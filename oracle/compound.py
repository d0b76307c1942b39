"""Voxelization of tracked frames into the directional grid (FP64 / exact integers).

Sec. 2.1 "Volume reconstruction": images are transformed to their poses and
voxelized into a 3D grid whose locations keep the intensities together with
their acquisition orientations.  Readings:

  * every pixel goes to its nearest voxel, v = floor(c + 0.5) per axis, with c
    from ``geometry.voxel_coords``; pixels with any v_a outside [0, dims_a) are
    dropped; every pixel counts, intensity 0 included;
  * per (bin, voxel) the grid keeps the exact integer sum S of intensities and
    the sample count C; the mean intensity is a = S / C where C > 0.

The grid is stored densely here, S and C of shape (K, nz, ny, nx), x fastest.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import geometry
from .bins import Codebook


@dataclass
class DirGrid:
    origin: np.ndarray        # world mm of voxel (0,0,0)'s centre
    spacing: float            # h, mm
    dims: tuple               # (nx, ny, nz)
    codebook: Codebook
    S: np.ndarray             # (K, nz, ny, nx) int64 intensity sums
    C: np.ndarray             # (K, nz, ny, nx) int64 sample counts

    @property
    def K(self) -> int:
        return self.S.shape[0]

    def mean_count(self):
        """FP64 mean intensity a = S / C (0 where C = 0) and count C as float64."""
        C = self.C.astype(np.float64)
        a = np.divide(self.S.astype(np.float64), C, out=np.zeros_like(C), where=C > 0)
        return a, C


def empty_grid(origin, spacing, dims, tol_deg, max_bins) -> DirGrid:
    nx, ny, nz = dims
    return DirGrid(np.asarray(origin, np.float64), float(spacing), tuple(dims),
                   Codebook(tol_deg, max_bins),
                   np.zeros((0, nz, ny, nx), np.int64), np.zeros((0, nz, ny, nx), np.int64))


def compound(grid: DirGrid, frames, probe_poses, calib, pitch, normal_axis: int = 2) -> np.ndarray:
    """Add frames (F, H, W) uint8 with probe poses (F, 4, 4) to ``grid`` in place.

    Returns the bin index assigned to each frame.
    """
    frames = np.asarray(frames)
    F, H, W = frames.shape
    T = geometry.compose(np.asarray(probe_poses), np.asarray(calib))
    _, _, _, xhat, nhat = geometry.axes(T, normal_axis)
    bins = grid.codebook.assign(nhat, xhat)
    K = grid.codebook.K
    nx, ny, nz = grid.dims
    if grid.S.shape[0] < K:
        pad = K - grid.S.shape[0]
        grid.S = np.concatenate([grid.S, np.zeros((pad, nz, ny, nx), np.int64)])
        grid.C = np.concatenate([grid.C, np.zeros((pad, nz, ny, nx), np.int64)])
    flatS = grid.S.reshape(-1)
    flatC = grid.C.reshape(-1)
    nvox = nx * ny * nz
    for f in range(F):
        p = geometry.pixel_positions(T[f], W, H, pitch)
        v = geometry.nearest_voxel(geometry.voxel_coords(p, grid.origin, grid.spacing))
        inside = ((v[..., 0] >= 0) & (v[..., 0] < nx) & (v[..., 1] >= 0) & (v[..., 1] < ny)
                  & (v[..., 2] >= 0) & (v[..., 2] < nz))
        vi = v[inside]
        lin = bins[f] * nvox + (vi[:, 2] * ny + vi[:, 1]) * nx + vi[:, 0]
        np.add.at(flatS, lin, frames[f][inside].astype(np.int64))
        np.add.at(flatC, lin, 1)
    return bins
