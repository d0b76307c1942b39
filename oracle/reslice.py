"""Directionality-aware reslice of the binned grid (FP64).

Sec. 2.1 "Reslicing" and Fig. 2:
  * a virtual image plane is posed and sampled at its pixel positions;
  * candidates come from a cubic neighbourhood of fixed interpolation distance;
  * Eq. 1: d_normal = n_s . n_r (signed), d_inplane = |x_s . x_r|;
  * samples misaligned beyond the thresholds (25 deg normal, 15 deg in-plane)
    are discarded -- equality is kept, compared as d >= cos(threshold);
  * Eq. 2: w = exp(k_normal (d_normal - 1) + k_inplane (d_inplane - 1)),
    k_normal = 10, k_inplane = 5;
  * the pixel is the weighted average of what survives, or unassigned (NaN)
    when nothing does; Fig. 2 adds weighting by distance.

Readings taken where the paper is silent:
  * a bin's samples share its representative orientation (n_b, x_b), so the
    angular weight is one number per bin per slice;
  * distance weighting is the separable tent t_v = prod_a (1 - |c_a - v_a| / R)
    over voxels with |c_a - v_a| < R on every axis, R = radius / h in voxels
    (R = 1 is trilinear interpolation);
  * two-stage normalisation: each voxel is first blended over directions,
    V_v = sum_b w_b c_vb a_vb / sum_b w_b c_vb (valid iff the denominator is
    > 0), then out = sum_valid t_v V_v / sum_valid t_v;
  * variants for fidelity studies: ``norm="sample"`` gives
    sum_v t_v A_v / sum_v t_v B_v (the single weighted average read
    literally), ``spatial="box"`` gives weight 1 over the (2R+1)^3 cube around
    the nearest voxel.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import geometry
from .bins import dot3


@dataclass
class Params:
    k_normal: float = 10.0
    k_inplane: float = 5.0
    thr_normal_deg: float = 25.0
    thr_inplane_deg: float = 15.0
    radius_vox: float = 1.0
    bin_tol_deg: float = 5.0
    max_bins: int = 64
    normal_axis: int = 2

    @classmethod
    def from_dict(cls, d):
        return cls(**{k: d[k] for k in cls.__dataclass_fields__ if k in d})


def alignment(rep_n, rep_x, nhat_r, xhat_r):
    """Eq. 1 per bin: (d_normal, d_inplane)."""
    dn = np.array([dot3(rep_n[b], nhat_r) for b in range(len(rep_n))])
    di = np.array([abs(dot3(rep_x[b], xhat_r)) for b in range(len(rep_x))])
    return dn, di


def angular_weights(rep_n, rep_x, nhat_r, xhat_r, prm: Params) -> np.ndarray:
    """Eq. 2 weight per bin, 0 for bins beyond either threshold."""
    cos_n = math.cos(math.radians(prm.thr_normal_deg))
    cos_i = math.cos(math.radians(prm.thr_inplane_deg))
    dn, di = alignment(rep_n, rep_x, nhat_r, xhat_r)
    w = np.zeros(len(dn))
    for b in range(len(dn)):
        if dn[b] >= cos_n and di[b] >= cos_i:
            w[b] = math.exp(prm.k_normal * (dn[b] - 1.0) + prm.k_inplane * (di[b] - 1.0))
    return w


def slice_weights(rep_n, rep_x, probe_pose, calib, prm: Params) -> np.ndarray:
    T = geometry.compose(np.asarray(probe_pose, np.float64), calib)
    _, _, _, xr, nr = geometry.axes(T, prm.normal_axis)
    return angular_weights(rep_n, rep_x, nr, xr, prm)


def reslice(a, c, origin, spacing, rep_n, rep_x, calib, probe_pose, width, height, pitch,
            prm: Params, spatial: str = "tent", norm: str = "two_stage", weights=None):
    """Reslice one plane.  a, c: (K, nz, ny, nx) mean intensity and count per
    (bin, voxel).  Returns (height, width) float64 with NaN where unassigned."""
    a = np.asarray(a, np.float64)
    c = np.asarray(c, np.float64)
    K, nz, ny, nx = a.shape
    T = geometry.compose(np.asarray(probe_pose, np.float64), calib)
    w = slice_weights(rep_n, rep_x, probe_pose, calib, prm) if weights is None else weights
    active = [b for b in range(K) if w[b] > 0.0]
    cc = geometry.voxel_coords(geometry.pixel_positions(T, width, height, pitch), origin, spacing)
    R = float(prm.radius_vox)
    num = np.zeros((height, width))
    den = np.zeros((height, width))
    if spatial == "tent":
        base = np.floor(cc).astype(np.int64)
        m = int(math.ceil(R))
        offsets = range(-m + 1, m + 1)
    elif spatial == "box":
        base = geometry.nearest_voxel(cc)
        m = int(round(R))
        offsets = range(-m, m + 1)
    else:
        raise ValueError(spatial)
    dimsxyz = (nx, ny, nz)
    for dz in offsets:
        for dy in offsets:
            for dx in offsets:
                v = base + np.array([dx, dy, dz])
                if spatial == "tent":
                    t = np.ones((height, width))
                    for ax in range(3):
                        t = t * np.maximum(0.0, 1.0 - np.abs(cc[..., ax] - v[..., ax]) / R)
                else:
                    t = np.ones((height, width))
                inside = np.ones((height, width), bool)
                for ax in range(3):
                    inside &= (v[..., ax] >= 0) & (v[..., ax] < dimsxyz[ax])
                take = inside & (t > 0.0)
                vx = np.clip(v[..., 0], 0, nx - 1)
                vy = np.clip(v[..., 1], 0, ny - 1)
                vz = np.clip(v[..., 2], 0, nz - 1)
                A = np.zeros((height, width))
                B = np.zeros((height, width))
                for b in active:
                    cb = np.where(take, c[b, vz, vy, vx], 0.0)
                    ab = np.where(take, a[b, vz, vy, vx], 0.0)
                    A += w[b] * cb * ab
                    B += w[b] * cb
                if norm == "two_stage":
                    valid = take & (B > 0.0)
                    V = np.divide(A, B, out=np.zeros_like(A), where=valid)
                    num += np.where(valid, t * V, 0.0)
                    den += np.where(valid, t, 0.0)
                elif norm == "sample":
                    num += np.where(take, t * A, 0.0)
                    den += np.where(take, t * B, 0.0)
                else:
                    raise ValueError(norm)
    out = np.full((height, width), np.nan)
    np.divide(num, den, out=out, where=den > 0.0)
    return out


def reslice_grid(grid, calib, probe_pose, width, height, pitch, prm: Params, form: str = "fp64",
                 **kw):
    """Reslice a ``compound.DirGrid`` with its values in storage ``form``
    ("fp64" for the exact means, else a form of ``quant.storage``)."""
    from . import quant
    if form == "fp64":
        a, c = grid.mean_count()
    else:
        a, c = quant.storage(grid.S, grid.C, form)
    rep_n, rep_x = grid.codebook.arrays()
    return reslice(a, c, grid.origin, grid.spacing, rep_n, rep_x, calib, probe_pose, width, height,
                   pitch, prm, **kw)
