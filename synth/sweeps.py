"""Tracked sweeps and reslice pose sets.

All positions are grid-local millimetres plus ``WORLD_OFFSET_MM``.  The beam of
an unrotated probe points along +z (depth), its lateral axis along +x and the
sweep advances along the elevation axis.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .poses import (WORLD_OFFSET_MM, image_pose, probe_pose_from_image_pose, random_rotation,
                    rot_y, rot_z, rotvec_to_matrix)


@dataclass
class Sweep:
    probe_poses: np.ndarray     # (F,4,4) float32, what the tracker reports
    image_poses: np.ndarray     # (F,4,4) float64, the intended image poses
    centers: np.ndarray         # (F,3) world mm of each frame's central pixel
    sweep_id: np.ndarray        # (F,) int
    width: int
    height: int
    pitch: tuple


def _concat(parts, width, height, pitch) -> Sweep:
    return Sweep(probe_poses=np.concatenate([p[0] for p in parts]),
                 image_poses=np.concatenate([p[1] for p in parts]),
                 centers=np.concatenate([p[2] for p in parts]),
                 sweep_id=np.concatenate([np.full(len(p[0]), k) for k, p in enumerate(parts)]),
                 width=width, height=height, pitch=tuple(pitch))


def linear_tilted_sweeps(N: int, h: float, n_frames: int, width: int, height: int, pitch,
                         tilts_deg, calib: np.ndarray) -> Sweep:
    """Parallel linear sweeps along elevation, each tilted in-plane (about elevation)."""
    mid = (N - 1) * h / 2.0
    ys = np.linspace(0.0, (N - 1) * h, n_frames)
    parts = []
    for tilt in tilts_deg:
        R = rot_y(np.deg2rad(tilt))
        lat, beam = R @ np.array([1.0, 0.0, 0.0]), R @ np.array([0.0, 0.0, 1.0])
        Ps, Ts, Cs = [], [], []
        for y in ys:
            c = WORLD_OFFSET_MM + np.array([mid, y, mid])
            T = image_pose(c, lat, beam, width, height, pitch)
            Ps.append(probe_pose_from_image_pose(T, calib))
            Ts.append(T)
            Cs.append(c)
        parts.append((np.stack(Ps), np.stack(Ts), np.stack(Cs)))
    return _concat(parts, width, height, pitch)


def azimuth_sweeps(N: int, h: float, n_frames: int, width: int, height: int, pitch,
                   azimuths_deg, jitter_mm: float, jitter_deg: float, seed: int,
                   calib: np.ndarray) -> Sweep:
    """Linear sweeps through the grid centre at several azimuths about the vertical,
    with independent Gaussian position and rotation-vector jitter per frame."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mid = (N - 1) * h / 2.0
    ss = np.linspace(-mid, mid, n_frames)
    parts = []
    for az in azimuths_deg:
        Rz = rot_z(np.deg2rad(az))
        lat0, elev = Rz @ np.array([1.0, 0.0, 0.0]), Rz @ np.array([0.0, 1.0, 0.0])
        beam0 = np.array([0.0, 0.0, 1.0])
        Ps, Ts, Cs = [], [], []
        for s in ss:
            Rj = rotvec_to_matrix(np.deg2rad(rng.normal(0.0, jitter_deg, 3)))
            c = WORLD_OFFSET_MM + np.array([mid, mid, mid]) + s * elev + rng.normal(0.0, jitter_mm, 3)
            T = image_pose(c, Rj @ lat0, Rj @ beam0, width, height, pitch)
            Ps.append(probe_pose_from_image_pose(T, calib))
            Ts.append(T)
            Cs.append(c)
        parts.append((np.stack(Ps), np.stack(Ts), np.stack(Cs)))
    return _concat(parts, width, height, pitch)


def random_walk_sweep(N: int, h: float, n_frames: int, width: int, height: int, pitch, rate_hz: float,
                      seed: int, calib: np.ndarray, speed_mm_s: float = 5.0, turn_deg_s: float = 20.0,
                      tau_s: float = 1.0) -> Sweep:
    """A freehand probe stream: frames at ``rate_hz`` along a smooth random walk (Ornstein-
    Uhlenbeck velocity and angular velocity with time constant ``tau_s`` and scales
    ``speed_mm_s`` / ``turn_deg_s``), starting at the grid centre with the beam along +z and
    reflected at the grid's inner 70 %."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = (N - 1) * h
    lo = WORLD_OFFSET_MM + 0.15 * L
    hi = WORLD_OFFSET_MM + 0.85 * L
    c = WORLD_OFFSET_MM + 0.5 * L
    R = np.eye(3)                      # columns: lateral, elevation, beam
    v = np.zeros(3)
    w = np.zeros(3)
    dt = 1.0 / rate_hz
    a = np.exp(-dt / tau_s)
    b = np.sqrt(max(0.0, 1.0 - a * a))
    sw_rad = np.deg2rad(turn_deg_s)
    Ps, Ts, Cs = [], [], []
    for _ in range(n_frames):
        T = image_pose(c, R[:, 0], R[:, 2], width, height, pitch)
        Ps.append(probe_pose_from_image_pose(T, calib))
        Ts.append(T)
        Cs.append(c.copy())
        v = a * v + b * speed_mm_s * rng.standard_normal(3)
        w = a * w + b * sw_rad * rng.standard_normal(3)
        c = c + v * dt
        for k in range(3):
            if c[k] < lo[k]:
                c[k] = 2 * lo[k] - c[k]
                v[k] = -v[k]
            if c[k] > hi[k]:
                c[k] = 2 * hi[k] - c[k]
                v[k] = -v[k]
        R = rotvec_to_matrix(w * dt) @ R
    return _concat([(np.stack(Ps), np.stack(Ts), np.stack(Cs))], width, height, pitch)


@dataclass
class SliceSet:
    probe_poses: np.ndarray     # (n,4,4) float64
    width: int
    height: int
    pitch: tuple
    near: np.ndarray            # (n,) bool: perturbed acquired pose (else random)


def slice_poses(seed: int, sweep: Sweep, n: int, n_near: int, width: int, height: int, pitch,
                N: int, h: float, calib: np.ndarray, max_rot_deg: float = 10.0,
                trans_sigma_mm: float = 2.0) -> SliceSet:
    """``n_near`` slices near acquired poses (random rotation of U(0, max_rot_deg) about a
    uniform axis, Gaussian translation), then ``n - n_near`` uniformly oriented slices
    centred in the middle half of the grid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ps, near = [], []
    L = (N - 1) * h
    for k in range(n):
        if k < n_near:
            f = int(rng.integers(len(sweep.probe_poses)))
            Tf = sweep.image_poses[f]
            ax = rng.standard_normal(3)
            ax /= np.linalg.norm(ax)
            R = rotvec_to_matrix(ax * np.deg2rad(rng.uniform(0.0, max_rot_deg)))
            c = sweep.centers[f] + rng.normal(0.0, trans_sigma_mm, 3)
            T = image_pose(c, R @ Tf[:3, 0], R @ Tf[:3, 1], width, height, pitch)
            near.append(True)
        else:
            R = random_rotation(rng)
            c = WORLD_OFFSET_MM + rng.uniform(0.25 * L, 0.75 * L, 3)
            T = image_pose(c, R[:, 0], R[:, 2], width, height, pitch)
            near.append(False)
        Ps.append(probe_pose_from_image_pose(T, calib, dtype=np.float64))
    return SliceSet(probe_poses=np.stack(Ps), width=width, height=height, pitch=tuple(pitch),
                    near=np.array(near))
