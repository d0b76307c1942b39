"""Helpers for the GPU parity tests: move oracle-side inputs to the device and
compare results to the parity bar."""
from __future__ import annotations

import sys

import numpy as np

from oracle import compound, reslice
from oracle.reslice import Params


def note(msg: str):
    """Name the case about to run on the GPU (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def oracle_params(p) -> Params:
    return Params(k_normal=p.k_normal, k_inplane=p.k_inplane, thr_normal_deg=p.thr_normal_deg,
                  thr_inplane_deg=p.thr_inplane_deg, radius_vox=p.radius_vox, bin_tol_deg=p.bin_tol_deg,
                  max_bins=p.max_bins, normal_axis=p.normal_axis)


def lib_params(prm: Params):
    import paper_2605_26325_amd as dare
    return dare.default_params(k_normal=prm.k_normal, k_inplane=prm.k_inplane, thr_normal_deg=prm.thr_normal_deg,
                               thr_inplane_deg=prm.thr_inplane_deg, radius_vox=prm.radius_vox,
                               bin_tol_deg=prm.bin_tol_deg, max_bins=prm.max_bins, normal_axis=prm.normal_axis)


def make_volume(origin, spacing, dims, calib, prm: Params, dtype="f32", bricks=None):
    import paper_2605_26325_amd as dare
    g = dare.make_geometry(origin, spacing, dims, calib)
    return dare.Volume(g, lib_params(prm), dtype=dtype, bricks=bricks)


def upload_grid(vol, S, C, rep_n, rep_x):
    import torch
    St = torch.from_numpy(np.ascontiguousarray(S.astype(np.uint32)).view(np.int32)).cuda()
    Ct = torch.from_numpy(np.ascontiguousarray(C.astype(np.uint32)).view(np.int32)).cuda()
    vol.upload_sums(rep_n, rep_x, St, Ct)
    torch.cuda.synchronize()


def oracle_grid(wl, frames_np, prm: Params):
    g = compound.empty_grid(wl.origin, wl.spacing, wl.dims, prm.bin_tol_deg, prm.max_bins)
    compound.compound(g, frames_np, wl.sweep.probe_poses, wl.calib, wl.sweep.pitch, prm.normal_axis)
    return g


def assert_parity(got, ref, rel=1e-5, what=""):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    gn, rn = np.isnan(got), np.isnan(ref)
    mism = int((gn != rn).sum())
    assert mism == 0, f"{what}: NaN masks differ at {mism} pixels"
    m = ~rn
    if m.any():
        err = np.abs(got[m] - ref[m])
        tol = rel * np.maximum(np.abs(ref[m]), 1.0)
        bad = int((err > tol).sum())
        assert bad == 0, f"{what}: {bad} pixels beyond {rel} relative; max abs err {err.max():.3g}"
    return int(m.sum())


def oracle_reslice_storage(a, c, origin, spacing, rep_n, rep_x, calib, P, W, H, pitch, prm):
    return reslice.reslice(a, c, origin, spacing, rep_n, rep_x, calib, P, W, H, pitch, prm)
