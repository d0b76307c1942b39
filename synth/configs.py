"""The synthetic workloads, shaped like the paper's experiments.

* ``config1``: 64^3 grid at 0.5 mm, 12 spheres + 4 planes, two linear sweeps of
  100 frames (128^2 uint8 at 0.25 mm) tilted +-20 deg in-plane, 16 slices of 128^2.
* ``config2``: 256^3 grid at 0.125 mm (the paper's voxel size), 30 spheres + 10
  planes, three azimuth sweeps (0/120/240 deg) of 600 frames of 256^2 at
  0.125 mm with 1 mm / 2 deg jitter, 1000 slices of 512^2 at 0.0625 mm
  (80 % near acquired poses, 20 % uniformly random).
* ``config3_slices``: 1000 slices of 512^2 at 0.0625 mm through the config-1 volume.
* ``serving_volume``: N^3 volumes at 0.125 mm built from three azimuth sweeps of
  N^2 frames.
* ``tiny_workload``: a few small frames on a small grid, for brute-force checks.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .phantom import Phantom, make_phantom
from .poses import WORLD_OFFSET_MM, make_calibration, rotvec_to_matrix
from .render import render_frames
from .sweeps import SliceSet, Sweep, azimuth_sweeps, linear_tilted_sweeps, random_walk_sweep, slice_poses


@dataclass
class Workload:
    name: str
    dims: tuple                   # (nx, ny, nz)
    spacing: float                # voxel size h, mm
    origin: np.ndarray            # world mm of voxel (0,0,0)'s centre
    calib: np.ndarray             # (4,4) float64 image-mm -> probe
    phantom: Phantom
    sweep: Sweep
    slices: SliceSet
    frame_seed: int
    frames: object = None         # torch uint8 (F,H,W), filled by ``render``
    fan: dict = None              # fan probes: apex (a0, a1), r0, dr, sectors, width, height
    beams: np.ndarray = None      # fan probes: (width, 2) unit beam direction per column

    def render(self, device="cpu"):
        if self.fan is None:
            self.frames = render_frames(self.phantom, self.sweep.probe_poses, self.calib,
                                        self.sweep.width, self.sweep.height, self.sweep.pitch,
                                        seed=self.frame_seed, device=device)
        else:
            W, H = self.fan["width"], self.fan["height"]
            r = self.fan["r0"] + self.fan["dr"] * np.arange(H, dtype=np.float64)
            uv = (self.fan["apex"][0] + r[:, None] * self.beams[None, :, 0],
                  self.fan["apex"][1] + r[:, None] * self.beams[None, :, 1])
            self.frames = render_frames(self.phantom, self.sweep.probe_poses, self.calib, W, H, self.sweep.pitch,
                                        seed=self.frame_seed, device=device, fan_uv=uv, fan_beams=self.beams)
        return self.frames




def config1(n_slices: int = 16, n_near: int = 12) -> Workload:
    N, h, w, pitch = 64, 0.5, 128, (0.25, 0.25)
    C = make_calibration(w, pitch[0])
    ph = make_phantom(seed=1, L=N * h, n_sph=12, n_pl=4, shell_mm=h)
    sw = linear_tilted_sweeps(N, h, 100, w, w, pitch, (20.0, -20.0), C)
    sl = slice_poses(101, sw, n_slices, n_near, 128, 128, (0.25, 0.25), N, h, C)
    return Workload("config1: 64^3 @0.5mm, 2x100 frames 128^2, 16 slices 128^2", (N, N, N), h,
                    WORLD_OFFSET_MM.copy(), C, ph, sw, sl, frame_seed=1)


def fan_beams(width: int, step_deg: float) -> np.ndarray:
    """(width, 2) unit beam directions (lateral, axial) of a fan whose columns are step_deg apart,
    symmetric about the axial direction."""
    th = np.deg2rad((np.arange(width, dtype=np.float64) - (width - 1) / 2.0) * step_deg)
    return np.stack([np.sin(th), np.cos(th)], axis=1)


def fan_config(sectors: int = 8, n_slices: int = 16, n_near: int = 12) -> Workload:
    """Config 1's grid, phantom and two tilted sweeps, imaged by a curvilinear probe: 96 beams
    0.5 deg apart (a 47.5 deg fan) from an apex 8 mm above the first row, 128 rows 0.2 mm apart,
    the columns binned in ``sectors`` sectors."""
    N, h, w, pitch = 64, 0.5, 128, (0.25, 0.25)
    C = make_calibration(w, pitch[0])
    ph = make_phantom(seed=1, L=N * h, n_sph=12, n_pl=4, shell_mm=h)
    sw = linear_tilted_sweeps(N, h, 100, w, w, pitch, (20.0, -20.0), C)
    sl = slice_poses(101, sw, n_slices, n_near, 128, 128, (0.25, 0.25), N, h, C)
    fan = dict(apex=((w - 1) * pitch[0] / 2.0, -6.0), r0=8.0, dr=0.2, sectors=int(sectors), width=96, height=128)
    return Workload(f"fan: 64^3 @0.5mm, 2x100 curvilinear frames 96x128, {sectors} sectors", (N, N, N), h,
                    WORLD_OFFSET_MM.copy(), C, ph, sw, sl, frame_seed=11, fan=fan,
                    beams=fan_beams(96, 0.5))


def fan_config2(sectors: int = 8, n_slices: int = 100, n_near: int = 80) -> Workload:
    """Config 2's grid, phantom and three azimuth sweeps of 600 frames, imaged by a curvilinear
    probe: 192 beams 0.25 deg apart (a 47.75 deg fan) from an apex 4 mm above the first row,
    256 rows 0.1 mm apart, the columns binned in ``sectors`` sectors; 512^2 slices."""
    N, h, w, pitch = 256, 0.125, 256, (0.125, 0.125)
    C = make_calibration(w, pitch[0])
    ph = make_phantom(seed=2, L=N * h, n_sph=30, n_pl=10, shell_mm=h)
    sw = azimuth_sweeps(N, h, 600, w, w, pitch, (0.0, 120.0, 240.0), 1.0, 2.0, seed=202, calib=C)
    sl = slice_poses(203, sw, n_slices, n_near, 512, 512, (0.0625, 0.0625), N, h, C)
    fan = dict(apex=((w - 1) * pitch[0] / 2.0, -3.0), r0=4.0, dr=0.1, sectors=int(sectors), width=192, height=256)
    return Workload(f"fan config2: 256^3 @0.125mm, 3x600 curvilinear frames 192x256, {sectors} sectors", (N, N, N),
                    h, WORLD_OFFSET_MM.copy(), C, ph, sw, sl, frame_seed=12, fan=fan,
                    beams=fan_beams(192, 0.25))


def config2(n_slices: int = 1000, n_near: int = 800) -> Workload:
    N, h, w, pitch = 256, 0.125, 256, (0.125, 0.125)
    C = make_calibration(w, pitch[0])
    ph = make_phantom(seed=2, L=N * h, n_sph=30, n_pl=10, shell_mm=h)
    sw = azimuth_sweeps(N, h, 600, w, w, pitch, (0.0, 120.0, 240.0), 1.0, 2.0, seed=202, calib=C)
    sl = slice_poses(203, sw, n_slices, n_near, 512, 512, (0.0625, 0.0625), N, h, C)
    return Workload("config2: 256^3 @0.125mm, 3x600 frames 256^2, 1000 slices 512^2", (N, N, N), h,
                    WORLD_OFFSET_MM.copy(), C, ph, sw, sl, frame_seed=2)


def config3_slices(wl1: Workload, n_slices: int = 1000, n_near: int = 800) -> SliceSet:
    N = wl1.dims[0]
    return slice_poses(3, wl1.sweep, n_slices, n_near, 512, 512, (0.0625, 0.0625), N,
                       wl1.spacing, wl1.calib)


def serving_volume(N: int, seed: int, n_frames: int = 600, n_slices: int = 64) -> Workload:
    h, pitch = 0.125, (0.125, 0.125)
    C = make_calibration(N, pitch[0])
    ph = make_phantom(seed=seed, L=N * h, n_sph=30, n_pl=10, shell_mm=h)
    sw = azimuth_sweeps(N, h, n_frames, N, N, pitch, (0.0, 120.0, 240.0), 1.0, 2.0,
                        seed=seed * 100 + 1, calib=C)
    sl = slice_poses(seed * 100 + 2, sw, n_slices, int(0.8 * n_slices), 512, 512,
                     (N * h / 512, N * h / 512), N, h, C)
    return Workload(f"serving volume {N}^3 @0.125mm", (N, N, N), h, WORLD_OFFSET_MM.copy(), C, ph,
                    sw, sl, frame_seed=seed)


def config5(seconds: float = 6.0, rate_hz: float = 30.0, N: int = 512) -> Workload:
    """The streaming case: an N^3 grid at 0.125 mm filled from a 512^2 probe stream at rate_hz on
    a random-walk trajectory (5 mm/s, 20 deg/s); consoles reslice 512^2 slices meanwhile."""
    h, w = 0.125, 512
    pitch = (N * h / w, N * h / w)
    C = make_calibration(w, pitch[0])
    ph = make_phantom(seed=5, L=N * h, n_sph=30, n_pl=10, shell_mm=h)
    sw = random_walk_sweep(N, h, int(round(seconds * rate_hz)), w, w, pitch, rate_hz, seed=501, calib=C)
    sl = slice_poses(502, sw, 64, 51, 512, 512, pitch, N, h, C)
    return Workload(f"config5: {N}^3 @0.125mm streamed from {w}^2 frames at {rate_hz:g} Hz", (N, N, N), h,
                    WORLD_OFFSET_MM.copy(), C, ph, sw, sl, frame_seed=5)


def tiny_workload(seed: int, N: int = 8, n_frames: int = 6, w: int = 6, n_slices: int = 4,
                  slice_w: int = 7, slice_h: int = 5, jitter_deg: float = 12.0,
                  exponent: float = 4.0, speckle: float = 0.3) -> Workload:
    """A handful of jittered frames on a small grid: for brute-force and literal checks."""
    h = 1.0
    pitch = (N * h / w, N * h / w)
    C = make_calibration(w, pitch[0])
    ph = make_phantom(seed=seed, L=N * h, n_sph=3, n_pl=2, shell_mm=2 * h, exponent=exponent,
                      speckle_sigma=speckle)
    sw = azimuth_sweeps(N, h, n_frames // 2, w, w, pitch, (0.0, 30.0), 0.5, jitter_deg,
                        seed=seed * 7 + 3, calib=C)
    sl = slice_poses(seed * 7 + 5, sw, n_slices, max(1, n_slices - 1), slice_w, slice_h,
                     (N * h / slice_w, N * h / slice_h), N, h, C, max_rot_deg=20.0)
    return Workload(f"tiny {N}^3 seed {seed}", (N, N, N), h, WORLD_OFFSET_MM.copy(), C, ph, sw, sl,
                    frame_seed=seed)


# ---- evaluation protocol: an initial sweep set for reconstruction and a secondary, different
# sweep for reslicing and ground truth, each sweep tracked with a rigid misregistration of its own

@dataclass
class EvalPair:
    initial: Workload            # frames rendered at true poses; reconstruct with `initial_tracked`
    initial_tracked: np.ndarray  # (F,4,4) float32 tracked probe poses of the initial frames
    secondary: Workload          # its frames are the ground truth
    secondary_tracked: np.ndarray  # (G,4,4) float32 tracked poses: the reslice poses
    offsets_mm_deg: list         # per sweep (initial sweeps, then the secondary): |t| mm, angle deg


def tracking_offsets(seed: int, n: int, centre, trans_mm: float, rot_deg: float) -> list:
    """n rigid world transforms (4x4): a rotation about ``centre`` by a rotation vector with
    N(0, rot_deg) components, then a translation with N(0, trans_mm) components."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    c = np.asarray(centre, np.float64)
    for _ in range(n):
        R = rotvec_to_matrix(np.deg2rad(rng.normal(0.0, rot_deg, 3)))
        t = rng.normal(0.0, trans_mm, 3)
        M = np.eye(4)
        M[:3, :3] = R
        M[:3, 3] = c - R @ c + t
        out.append(M)
    return out


def tracked(sweep: Sweep, offsets: list) -> np.ndarray:
    """What the tracker reports: sweep k's true probe poses moved by offsets[k]."""
    P = np.asarray(sweep.probe_poses, np.float64)
    out = np.empty_like(P)
    for f in range(len(P)):
        out[f] = offsets[int(sweep.sweep_id[f])] @ P[f]
        out[f, 3, :] = (0.0, 0.0, 0.0, 1.0)
    return out.astype(np.float32)


def _offset_size(M: np.ndarray, centre) -> tuple:
    """(displacement of the volume centre in mm, rotation angle in degrees)."""
    c = np.asarray(centre, np.float64)
    ang = float(np.degrees(np.arccos(np.clip((np.trace(M[:3, :3]) - 1.0) / 2.0, -1.0, 1.0))))
    return (round(float(np.linalg.norm(M[:3, :3] @ c + M[:3, 3] - c)), 3), round(ang, 3))


def eval_pair(config: int, trans_vox: float = 0.5, rot_lever_vox: float = 0.5) -> EvalPair:
    """The two-sweep protocol on config 1 or 2.  Config 1: the two +-20 degree tilted sweeps,
    then a secondary sweep of 40 frames tilted +10 degrees (10 degrees from one initial sweep,
    30 from the other).  Config 2: the three azimuth sweeps, then a secondary sweep of 60 frames
    at azimuth 10 degrees with the same jitter.  Secondary frames use speckle of their own.
    Tracking offsets per sweep: translation components N(0, trans_vox voxels), rotation-vector
    components N(0, r) with r the angle that moves a point half the grid away by rot_lever_vox
    voxels, so that misregistration is of the order of a voxel at every grid size."""
    if config == 1:
        wl = config1()
        N, h = wl.dims[0], wl.spacing
        sec = linear_tilted_sweeps(N, h, 40, wl.sweep.width, wl.sweep.height, wl.sweep.pitch, (10.0,), wl.calib)
        seed = 11
    elif config == 2:
        wl = config2(n_slices=1, n_near=1)
        N, h = wl.dims[0], wl.spacing
        sec = azimuth_sweeps(N, h, 60, wl.sweep.width, wl.sweep.height, wl.sweep.pitch, (10.0,), 1.0, 2.0,
                             seed=224, calib=wl.calib)
        seed = 22
    else:
        raise ValueError(config)
    centre = WORLD_OFFSET_MM + 0.5 * (N - 1) * h
    n0 = int(wl.sweep.sweep_id.max()) + 1
    rot_deg = float(np.degrees(rot_lever_vox / (0.5 * N)))
    offs = tracking_offsets(seed, n0 + 1, centre, trans_vox * h, rot_deg)
    sw = Workload(wl.name + " secondary sweep", wl.dims, h, wl.origin, wl.calib, wl.phantom, sec, wl.slices,
                  frame_seed=wl.frame_seed + 1000)
    return EvalPair(initial=wl, initial_tracked=tracked(wl.sweep, offs[:n0]), secondary=sw,
                    secondary_tracked=tracked(sec, [offs[n0]]), offsets_mm_deg=[_offset_size(M, centre) for M in offs])
