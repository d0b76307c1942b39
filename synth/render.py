"""B-mode frame renderer for the synthetic phantom (torch, any device).

Pixel (i, j) of a frame (column i lateral, row j depth) lies at image
millimetres (i*sx, j*sy, 0).  The renderer maps it to world coordinates with
the frame's probe pose and the calibration, evaluates the phantom's echo with
the frame's beam direction, adds Rayleigh speckle and rounds to uint8 (round
half to even).  This is a physics stand-in only: it knows nothing of voxels,
bins or reslicing.
"""
from __future__ import annotations

import numpy as np
import torch

from .phantom import Phantom
from .poses import WORLD_OFFSET_MM


def _frame_seed(seed: int, f: int) -> int:
    return (int(seed) * 1_000_003 + 7919 * int(f) + 12345) & 0x7FFF_FFFF_FFFF


@torch.no_grad()
def render_frames(ph: Phantom, probe_poses: np.ndarray, calib: np.ndarray, width: int,
                  height: int, pitch, seed: int, device="cpu", chunk: int = 32,
                  world_offset=WORLD_OFFSET_MM, fan_uv=None, fan_beams=None) -> torch.Tensor:
    """Render ``len(probe_poses)`` frames; returns uint8 (F, height, width) on ``device``.

    A fan probe passes ``fan_uv`` = (u, v), the image-mm position of every pixel (each
    (height, width)), and ``fan_beams`` (width, 2), every column's unit beam direction in image
    mm (lateral, axial); the echo then takes each column's own beam."""
    dev = torch.device(device)
    P = torch.as_tensor(np.asarray(probe_poses, dtype=np.float32), device=dev).to(torch.float64)
    C = torch.as_tensor(np.asarray(calib, dtype=np.float64), device=dev)
    W0 = torch.as_tensor(np.asarray(world_offset, dtype=np.float64), device=dev)
    F = P.shape[0]
    out = torch.empty((F, height, width), dtype=torch.uint8, device=dev)
    ii = torch.arange(width, device=dev, dtype=torch.float64) * float(pitch[0])
    jj = torch.arange(height, device=dev, dtype=torch.float64) * float(pitch[1])
    sph_c = torch.as_tensor(ph.sph_c, device=dev)
    pl_n = torch.as_tensor(ph.pl_n, device=dev)
    pl_q = torch.as_tensor(ph.pl_q, device=dev)
    shell = float(ph.shell_mm)
    for f0 in range(0, F, chunk):
        f1 = min(F, f0 + chunk)
        T = P[f0:f1] @ C                                     # (B,4,4)
        e0, e1, t = T[:, :3, 0], T[:, :3, 1], T[:, :3, 3]
        if fan_uv is None:
            loc = (t - W0)[:, None, None, :] \
                + jj[None, :, None, None] * e1[:, None, None, :] \
                + ii[None, None, :, None] * e0[:, None, None, :]   # (B,H,W,3) local mm
            beam = (e1 / e1.norm(dim=1, keepdim=True))[:, None, None, :]
        else:
            uu = torch.as_tensor(np.asarray(fan_uv[0], np.float64), device=dev)
            vv = torch.as_tensor(np.asarray(fan_uv[1], np.float64), device=dev)
            bb = torch.as_tensor(np.asarray(fan_beams, np.float64), device=dev)
            loc = (t - W0)[:, None, None, :] + vv[None, :, :, None] * e1[:, None, None, :] \
                + uu[None, :, :, None] * e0[:, None, None, :]
            x0 = e0 / e0.norm(dim=1, keepdim=True)
            y0 = e1 / e1.norm(dim=1, keepdim=True)
            beam = (bb[None, :, 0, None] * x0[:, None, :] + bb[None, :, 1, None] * y0[:, None, :])[:, None, :, :]
        E = torch.zeros(loc.shape[:3], dtype=torch.float64, device=dev)
        for s in range(sph_c.shape[0]):
            d = loc - sph_c[s]
            rr = d.norm(dim=-1)
            dist = rr - float(ph.sph_r[s])
            shellw = (1.0 - dist.abs() / shell).clamp_min(0.0)
            if ph.exponent != 0.0:
                cosv = ((d * beam).sum(-1) / rr.clamp_min(1e-12)).abs()
                shellw = shellw * cosv.pow(ph.exponent)
            E += float(ph.sph_i[s]) * shellw
        for q in range(pl_n.shape[0]):
            dist = ((loc - pl_q[q]) * pl_n[q]).sum(-1)
            shellw = (1.0 - dist.abs() / shell).clamp_min(0.0)
            if ph.exponent != 0.0:
                cosv = (beam * pl_n[q]).sum(-1).abs()
                shellw = shellw * cosv.pow(ph.exponent)
            E += float(ph.pl_i[q]) * shellw
        if ph.speckle_sigma > 0.0:
            sp = torch.empty_like(E)
            for k, f in enumerate(range(f0, f1)):
                g = torch.Generator(device=dev)
                g.manual_seed(_frame_seed(seed, f))
                u = torch.rand((height, width), generator=g, device=dev, dtype=torch.float64)
                sp[k] = float(ph.speckle_sigma) * torch.sqrt(-2.0 * torch.log1p(-u))
            E = E + sp
        out[f0:f1] = torch.round(255.0 * E.clamp(0.0, 1.0)).to(torch.uint8)
    return out
