"""Per-sample reference: the paper's flat storage taken literally (tiny inputs only).

Sec. 2.1: each grid location points into a flat store of the samples that
landed there, each with its own acquisition orientation; reslicing weighs each
sample by Eq. 1 and Eq. 2 with its own orientation.  This module is written
separately from ``bins``/``compound``/``reslice`` with explicit scalar loops,
so that agreement between the two formulations (with bin tolerance 0) checks
both.  The position arithmetic follows the same readings as ``geometry``:
T = P . C summed left to right, p = (t + (i sx) e0) + (j sy) e1, nearest voxel
floor(c + 0.5), neighbourhood |c_a - v_a| < R with tent weights.
"""
from __future__ import annotations

import math

import numpy as np


def _matmul4(P, C):
    T = [[0.0] * 4 for _ in range(4)]
    for r in range(4):
        for k in range(4):
            s = float(P[r][0]) * float(C[0][k])
            for m in range(1, 4):
                s = s + float(P[r][m]) * float(C[m][k])
            T[r][k] = s
    return T


def _col(T, k):
    return [T[0][k], T[1][k], T[2][k]]


def _normalize(v):
    n = math.sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2])
    return [v[0] / n, v[1] / n, v[2] / n]


def _dot(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def _pos(T, i, j, sx, sy):
    t, e0, e1 = _col(T, 3), _col(T, 0), _col(T, 1)
    return [(t[a] + (i * sx) * e0[a]) + (j * sy) * e1[a] for a in range(3)]


class SampleStore:
    """voxel (ix, iy, iz) -> list of (intensity, frame index); plus frame orientations."""

    def __init__(self, origin, spacing, dims, normal_axis=2):
        self.origin = [float(v) for v in origin]
        self.h = float(spacing)
        self.dims = tuple(int(d) for d in dims)
        self.normal_axis = normal_axis
        self.samples = {}
        self.frame_n = []
        self.frame_x = []

    def add_frames(self, frames, probe_poses, calib, pitch):
        inv_h = 1.0 / self.h
        sx, sy = float(pitch[0]), float(pitch[1])
        for f in range(len(frames)):
            T = _matmul4(np.asarray(probe_poses[f]).astype(np.float64).tolist(),
                         np.asarray(calib, np.float64).tolist())
            fid = len(self.frame_n)
            self.frame_x.append(_normalize(_col(T, 0)))
            self.frame_n.append(_normalize(_col(T, self.normal_axis)))
            img = np.asarray(frames[f])
            for j in range(img.shape[0]):
                for i in range(img.shape[1]):
                    p = _pos(T, i, j, sx, sy)
                    v = tuple(int(math.floor((p[a] - self.origin[a]) * inv_h + 0.5)) for a in range(3))
                    if all(0 <= v[a] < self.dims[a] for a in range(3)):
                        self.samples.setdefault(v, []).append((int(img[j, i]), fid))


def sample_weight(store: SampleStore, fid: int, n_r, x_r, prm) -> float:
    dn = _dot(store.frame_n[fid], n_r)
    di = abs(_dot(store.frame_x[fid], x_r))
    if dn < math.cos(math.radians(prm.thr_normal_deg)) or di < math.cos(math.radians(prm.thr_inplane_deg)):
        return 0.0
    return math.exp(prm.k_normal * (dn - 1.0) + prm.k_inplane * (di - 1.0))


def reslice(store: SampleStore, calib, probe_pose, width, height, pitch, prm,
            spatial: str = "tent", norm: str = "two_stage"):
    T = _matmul4(np.asarray(probe_pose, np.float64).tolist(), np.asarray(calib, np.float64).tolist())
    x_r = _normalize(_col(T, 0))
    n_r = _normalize(_col(T, prm.normal_axis))
    sx, sy = float(pitch[0]), float(pitch[1])
    inv_h = 1.0 / store.h
    R = float(prm.radius_vox)
    out = np.full((height, width), np.nan)
    for j in range(height):
        for i in range(width):
            p = _pos(T, i, j, sx, sy)
            c = [(p[a] - store.origin[a]) * inv_h for a in range(3)]
            if spatial == "tent":
                lo = [math.floor(c[a] - R) + 1 for a in range(3)]
                hi = [math.ceil(c[a] + R) - 1 for a in range(3)]
            else:
                ctr = [math.floor(c[a] + 0.5) for a in range(3)]
                r = int(round(R))
                lo = [ctr[a] - r for a in range(3)]
                hi = [ctr[a] + r for a in range(3)]
            num = den = 0.0
            for vz in range(lo[2], hi[2] + 1):
                for vy in range(lo[1], hi[1] + 1):
                    for vx in range(lo[0], hi[0] + 1):
                        v = (vx, vy, vz)
                        if spatial == "tent":
                            t = 1.0
                            for a in range(3):
                                t *= max(0.0, 1.0 - abs(c[a] - v[a]) / R)
                        else:
                            t = 1.0
                        if t <= 0.0 or v not in store.samples:
                            continue
                        sw = swi = 0.0
                        for (inten, fid) in store.samples[v]:
                            wi = sample_weight(store, fid, n_r, x_r, prm)
                            sw += wi
                            swi += wi * inten
                        if norm == "two_stage":
                            if sw > 0.0:
                                num += t * (swi / sw)
                                den += t
                        else:
                            num += t * swi
                            den += t * sw
            if den > 0.0:
                out[j, i] = num / den
    return out
