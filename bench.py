#!/usr/bin/env python3
"""Benchmark of the directionality-aware reslice on one MI355X.

Workload (synthetic, shaped like the paper's timing experiment): a 256^3 grid
of 0.125 mm voxels compounded from three azimuth sweeps of 600 frames of
256^2 uint8 pixels (1 mm / 2 deg pose jitter), then 1000 slices of 512^2
pixels at 0.0625 mm, 80 % near acquired poses and 20 % uniformly oriented,
resliced with an interpolation radius of one voxel.

A step is one pass over the 1000-slice batch with one dare_reslice launch per
slice (FP32 storage, FP64 positions, FP32 blending), inputs resident in HBM.
The same run also measures: the reconstruction (compounding) of the frames,
BF16/FP16/FP8 storage and the batched entry point on the same slices,
unloaded submit-to-host latency, the reslice kernel's average launch time
with HIP events against its algorithmic bytes (the HBM roofline), the
per-sample store, the evaluation protocol, compounding from a curvilinear probe,
compounding with bricks spilled to host memory, serving and streaming, and the
FP64 CPU oracle on a bounded sample of the same workload.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import dataclasses
import ctypes as ct
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles, 2.4 GHz
VALU_PEAK_WAVE_INSTR_S = 256 * 4 * 2.4e9 / 4
PAIR_BYTES = {"f32": 8, "bf16": 4, "f16": 4, "fp8": 2}
# sources of the radius-1 reslice kernels and of the compounding kernels: stored counter figures
# are used only while these are unchanged
RESLICE_SOURCES = ("dare_tiles.hip", "dare_batch.hip", "dare_batch.h", "dare_reslice_dev.h", "dare_codec.h",
                   "dare_internal.h")
COMPOUND_SOURCES = ("dare_compound.hip", "dare_internal.h")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2605_26325_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_counters(path):
    """Per-kernel counter figures of the committed profile (bytes scaled by the copy kernel's
    calibration, wave instructions), keeping only the kernels whose sources are unchanged."""
    try:
        with open(path) as fh:
            doc = json.load(fh)
    except (OSError, ValueError):
        return {}
    ok = {"reslice": doc.get("reslice_hash") == source_hash(RESLICE_SOURCES),
          "compound": doc.get("compound_hash") == source_hash(COMPOUND_SOURCES)}
    return {k: v for k, v in doc.get("kernels", {}).items() if ok.get(v.get("group"), False)}


def valu_roofline(insts, seconds, what):
    """VALU-issue bound: wave64 VALU instructions per launch over the launch's duration."""
    if insts is None or seconds <= 0:
        return None
    ach = insts / seconds
    return {"bound": "valu", "achieved": round(ach / 1e9, 1), "peak": round(VALU_PEAK_WAVE_INSTR_S / 1e9, 1),
            "unit": "G wave-instr/s", "frac": round(ach / VALU_PEAK_WAVE_INSTR_S, 4),
            "valu_insts_per_launch": round(insts), "basis": what}


def footprint_voxels(torch, P, calib, origin, h, dims, W, H, pitch):
    """Distinct in-grid voxels with non-zero trilinear weight over one slice (untimed)."""
    dev = "cuda"
    T = torch.tensor(P, dtype=torch.float64, device=dev) @ torch.tensor(calib, dtype=torch.float64, device=dev)
    i = torch.arange(W, device=dev, dtype=torch.float64) * pitch[0]
    j = torch.arange(H, device=dev, dtype=torch.float64) * pitch[1]
    p = T[:3, 3] + i[None, :, None] * T[:3, 0] + j[:, None, None] * T[:3, 1]
    c = (p - torch.tensor(origin, dtype=torch.float64, device=dev)) / h
    b = torch.floor(c)
    f = c - b
    b = b.to(torch.int64)
    n = torch.tensor(dims, device=dev)
    keys = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                d = torch.tensor([dx, dy, dz], device=dev)
                v = b + d
                ok = ((v >= 0) & (v < n)).all(-1)
                nz = torch.ones_like(ok)
                for a, da in enumerate((dx, dy, dz)):
                    if da == 1:
                        nz &= f[..., a] > 0
                ok &= nz
                vv = v[ok]
                keys.append((vv[:, 2] * n[1] + vv[:, 1]) * n[0] + vv[:, 0])
    return int(torch.unique(torch.cat(keys)).numel())


def voxel_sample_counts(torch, frames_shape, poses, calib, origin, h, dims, pitch):
    """Samples per voxel of the per-sample store (every in-grid frame pixel at its nearest voxel),
    recomputed in torch for the untimed algorithmic-byte count."""
    dev = poses.device
    F, Hf, Wf = frames_shape
    n = torch.tensor(dims, device=dev)
    counts = torch.zeros(int(dims[0]) * int(dims[1]) * int(dims[2]), dtype=torch.int64, device=dev)
    C = torch.tensor(calib, dtype=torch.float64, device=dev)
    i = torch.arange(Wf, device=dev, dtype=torch.float64) * pitch[0]
    j = torch.arange(Hf, device=dev, dtype=torch.float64) * pitch[1]
    o = torch.tensor(origin, dtype=torch.float64, device=dev)
    for f0 in range(0, F, 64):
        T = poses[f0:f0 + 64].to(torch.float64) @ C
        p = T[:, None, None, :3, 3] + i[None, None, :, None] * T[:, None, None, :3, 0] \
            + j[None, :, None, None] * T[:, None, None, :3, 1]
        v = torch.floor((p - o) / h + 0.5).to(torch.int64).reshape(-1, 3)
        ok = ((v >= 0) & (v < n)).all(-1)
        v = v[ok]
        counts += torch.bincount((v[:, 2] * n[1] + v[:, 1]) * n[0] + v[:, 0], minlength=counts.numel())
    return counts


def box_reading_bytes(torch, counts, P, calib, origin, h, dims, W, H, pitch, R=1):
    """Algorithmic bytes of one box-reading reslice: the samples (4 B) and CSR offsets (8 B) of the
    distinct voxels within R of some pixel's nearest voxel, plus 4 B of output per pixel."""
    dev = counts.device
    T = torch.tensor(P, dtype=torch.float64, device=dev) @ torch.tensor(calib, dtype=torch.float64, device=dev)
    i = torch.arange(W, device=dev, dtype=torch.float64) * pitch[0]
    j = torch.arange(H, device=dev, dtype=torch.float64) * pitch[1]
    p = T[:3, 3] + i[None, :, None] * T[:3, 0] + j[:, None, None] * T[:3, 1]
    ctr = torch.floor((p - torch.tensor(origin, dtype=torch.float64, device=dev)) / h + 0.5).to(torch.int64)
    ctr = torch.unique(ctr.reshape(-1, 3), dim=0)
    n = torch.tensor(dims, device=dev)
    keys = []
    for dz in range(-R, R + 1):
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                v = ctr + torch.tensor([dx, dy, dz], device=dev)
                v = v[((v >= 0) & (v < n)).all(-1)]
                keys.append((v[:, 2] * n[1] + v[:, 1]) * n[0] + v[:, 0])
    u = torch.unique(torch.cat(keys))
    return int(4 * counts[u].sum().item() + 8 * u.numel() + 4 * W * H)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else float("nan")


class Console:
    """A simulated expert console: a probe pose following a smooth random walk
    (Ornstein-Uhlenbeck velocity and angular velocity, tau = 1 s, 5 mm/s and
    20 deg/s scales), starting at an acquired pose, kept inside the volume and
    within MAX_TILT_DEG of the starting orientation (both reflected at the
    bound): an unbounded orientation walk drifts, within a minute, to planes
    that no acquisition direction passes the angular gates for, and those
    reslice to all-NaN images."""

    MAX_TILT_DEG = 10.0

    def __init__(self, rng, wl, vol_id, sizes):
        self.rng = rng
        self.vol_id = vol_id
        self.wl = wl
        f = int(rng.integers(len(wl.sweep.image_poses)))
        self.R = wl.sweep.image_poses[f][:3, :3].copy()
        self.R0 = self.R.copy()
        self.c = wl.sweep.centers[f].copy()
        self.v = np.zeros(3)
        self.w = np.zeros(3)
        self.sizes = sizes
        self.lo = wl.origin + 0.15 * (np.array(wl.dims) - 1) * wl.spacing
        self.hi = wl.origin + 0.85 * (np.array(wl.dims) - 1) * wl.spacing

    def step(self, dt, synth):
        tau, sv, sw = 1.0, 5.0, np.deg2rad(20.0)
        a = np.exp(-dt / tau)
        b = np.sqrt(max(0.0, 1.0 - a * a))
        self.v = a * self.v + b * sv * self.rng.standard_normal(3)
        self.w = a * self.w + b * sw * self.rng.standard_normal(3)
        self.c = self.c + self.v * dt
        for k in range(3):                     # reflect at the volume's inner bounds
            if self.c[k] < self.lo[k]:
                self.c[k] = 2 * self.lo[k] - self.c[k]
                self.v[k] = -self.v[k]
            if self.c[k] > self.hi[k]:
                self.c[k] = 2 * self.hi[k] - self.c[k]
                self.v[k] = -self.v[k]
        R = synth.rotvec_to_matrix(self.w * dt) @ self.R
        cos_t = (np.trace(R @ self.R0.T) - 1.0) / 2.0
        if cos_t < np.cos(np.deg2rad(self.MAX_TILT_DEG)):
            self.w = -self.w                   # reflect at the orientation bound
        else:
            self.R = R
        n = int(self.sizes[int(self.rng.integers(len(self.sizes)))])
        L = self.wl.dims[0] * self.wl.spacing
        pitch = (L / n, L / n)
        T = synth.image_pose(self.c, self.R[:, 0], self.R[:, 1], n, n, pitch)
        return synth.probe_pose_from_image_pose(T, self.wl.calib, dtype=np.float64), n, pitch


def run_closed(srv, consoles, bufs, ring, sizes, duration, synth, depth=2, seq_len=48):
    """Closed loop: every console keeps `depth` requests in flight, resubmitting as soon as one
    completes.  Poses are precomputed (30 Hz walk) so that the driver costs two grouped calls
    per iteration, not Python work per request.  Also returns the request mix (every console's
    pose sequence and how many times each entry was served) for the algorithmic-byte count."""
    import paper_2605_26325_amd as dare
    nc = len(consoles)
    seqs, npx, steps_all = [], [], []
    for c in consoles:
        steps = [c.step(1.0 / 30.0, synth) for _ in range(seq_len)]
        steps_all.append(steps)
        seqs.append(dare.spec_array([P for P, _, _ in steps], [n for _, n, _ in steps], [n for _, n, _ in steps],
                                    [pt for _, _, pt in steps]))
        npx.append(np.array([n * n for _, n, _ in steps], np.int64))
    vol_of = np.array([c.vol_id for c in consoles], np.int32)
    cursor = np.zeros(nc, np.int64)
    served = np.zeros((nc, seq_len), np.int64)
    owner = {}                       # ticket -> (console, pixels, sequence entry)
    lat = {n: [] for n in sizes}
    dev_lat = []
    px = 0
    st0 = srv.stats()

    def submit(ks):
        nonlocal cursor
        if not ks:
            return
        ks = np.asarray(ks)
        idx = cursor[ks] % seq_len
        specs = np.concatenate([seqs[k][i:i + 1] for k, i in zip(ks, idx)])
        outs = [bufs[k][int(cursor[k]) % ring].data_ptr() for k in ks]
        tickets, _ = srv.submit_many(vol_of[ks], specs, outs)
        for j, t in enumerate(tickets):
            k = int(ks[j])
            owner[int(t)] = (k, int(npx[k][idx[j]]), int(idx[j]))
            cursor[k] += 1
        return len(tickets)

    def done(k, p, i, t_host, t_dev, t_sub):
        nonlocal px
        lat[int(round(p ** 0.5))].append(1e3 * (t_host - t_sub))
        if t_dev > 0.0:
            dev_lat.append(1e3 * (t_dev - t_sub))
        px += p
        served[k, i] += 1

    t_start = time.perf_counter()
    submit([k for k in range(nc) for _ in range(depth)])
    while time.perf_counter() - t_start < duration:
        tk = np.fromiter(owner.keys(), np.uint64, len(owner))
        states, times = srv.poll_many(tk, wait_seconds=0.005)
        again = []
        for j in np.nonzero(states != dare.ERR_NOT_READY)[0]:
            k, p, i = owner.pop(int(tk[j]))
            if states[j] != dare.OK:
                raise dare.DareError(int(states[j]), "served request")
            done(k, p, i, times["t_host_done"][j], times["t_device_done"][j], times["t_submit"][j])
            again.append(k)
        submit(again)
    srv.drain()
    tk = np.fromiter(owner.keys(), np.uint64, len(owner))
    states, times = srv.poll_many(tk)
    for j in range(len(tk)):
        k, p, i = owner.pop(int(tk[j]))
        done(k, p, i, times["t_host_done"][j], times["t_device_done"][j], times["t_submit"][j])
    el = time.perf_counter() - t_start
    st1 = srv.stats()
    alll = [x for v in lat.values() for x in v]
    dev_busy = st1.device_busy_seconds - st0.device_busy_seconds
    res = {"seconds": round(el, 2), "requests": len(alll), "Mpx_s": round(px / el / 1e6, 1),
           "latency_ms": {"p50": round(percentile(alll, 50), 3), "p99": round(percentile(alll, 99), 3),
                          "p99_512": round(percentile(lat[512], 99), 3),
                          "p50_512": round(percentile(lat[512], 50), 3),
                          "p99_1024": round(percentile(lat[1024], 99), 3),
                          "device_p99": round(percentile(dev_lat, 99), 3)},
           "ticks": int(st1.ticks - st0.ticks),
           "mean_requests_per_tick": round(len(alll) / max(1, st1.ticks - st0.ticks), 2),
           "busy_fraction": round((st1.busy_seconds - st0.busy_seconds) / el, 3),
           "device_busy_fraction": round(dev_busy / el, 3),
           "device_Mpx_s": round(px / max(dev_busy, 1e-9) / 1e6, 1),
           "mean_tick_kernel_ms": round(1e3 * (st1.kernel_seconds - st0.kernel_seconds)
                                        / max(1, st1.ticks - st0.ticks), 4),
           "untimed_ticks": int(st1.untimed_ticks - st0.untimed_ticks)}
    mix = {"steps": steps_all, "served": served, "device_busy_seconds": dev_busy, "pixels": px}
    return res, mix


def run_streaming(dare, torch, synth, seconds, log):
    """Streaming form: a 512^3 FP16 volume filled through the server from a 30 Hz probe stream
    of 512^2 frames on a random walk, while 32 consoles request 512^2 slices at 30 Hz each."""
    dev = torch.device("cuda:0")
    rate = 30.0
    wl = synth.config5(seconds=seconds, rate_hz=rate)
    t0 = time.perf_counter()
    frames = wl.render(dev)
    poses = torch.from_numpy(np.ascontiguousarray(wl.sweep.probe_poses, np.float32)).to(dev)
    torch.cuda.synchronize()
    F, Hf, Wf = frames.shape
    log(f"streaming: rendered {F} frames {Wf}x{Hf} in {time.perf_counter() - t0:.1f} s")
    geom = dare.make_geometry(wl.origin, wl.spacing, wl.dims, wl.calib)
    vol = dare.Volume(geom, dare.default_params(), dtype="f16", bricks=2_000_000)
    srv = dare.Server(4 << 30, n_streams=3, max_tick_requests=64, max_tick_pixels=16 << 20, max_queue=8192)
    vid = srv.add_volume(vol)
    rng = np.random.default_rng(55)
    consoles = [Console(rng, wl, vid, (512,)) for _ in range(32)]
    ring = 6
    bufs = [[torch.empty((512 * 512,), dtype=torch.float32, pin_memory=True) for _ in range(ring)]
            for _ in range(32)]
    fr_views = [(frames[f:f + 1], poses[f:f + 1]) for f in range(F)]
    pending, fpend = {}, {}
    lat, flat = [], []
    slot = [0] * 32
    st0 = srv.stats()
    t_start = time.perf_counter()
    next_t = [t_start + rng.exponential(1.0 / rate) for _ in range(32)]
    last = [t_start] * 32
    nf = 0
    while nf < F or pending or fpend:
        now = time.perf_counter()
        if nf < F and now >= t_start + nf / rate:
            t = srv.submit_frames(vid, fr_views[nf][0], fr_views[nf][1], wl.sweep.pitch)
            if t is not None:
                fpend[t] = nf
                nf += 1
        if nf < F:
            for k in range(32):
                if now < next_t[k]:
                    continue
                c = consoles[k]
                P, n, pitch = c.step(max(1e-3, now - last[k]), synth)
                last[k] = now
                buf = bufs[k][slot[k] % ring]
                slot[k] += 1
                t = srv.submit(vid, P, n, n, pitch, buf)
                if t is not None:
                    pending[t] = k
                next_t[k] += rng.exponential(1.0 / rate)
        if pending:
            tk = np.fromiter(pending.keys(), np.uint64, len(pending))
            states, times = srv.poll_many(tk)
            for j in np.nonzero(states != dare.ERR_NOT_READY)[0]:
                pending.pop(int(tk[j]))
                if states[j] != dare.OK:
                    raise dare.DareError(int(states[j]), "streamed reslice")
                lat.append(1e3 * (times["t_host_done"][j] - times["t_submit"][j]))
        for t in list(fpend):
            r = srv.poll_frames(t)
            if r is not None:
                st, tm = r
                if st not in (dare.OK, dare.WARN_BINS_SATURATED):
                    raise dare.DareError(int(st), "streamed frames")
                fpend.pop(t)
                flat.append(1e3 * (tm.t_host_done - tm.t_submit))
    el = time.perf_counter() - t_start
    st1 = srv.stats()
    nfr = int(st1.frames - st0.frames)
    comp_s = float(st1.compound_seconds - st0.compound_seconds)
    info = vol.info()
    # flat out: the same stream again into a fresh volume, one job of 30 frames at a time, no consoles
    vol2 = dare.Volume(geom, dare.default_params(), dtype="f16", bricks=2_000_000)
    vid2 = srv.add_volume(vol2)
    t1 = time.perf_counter()
    jobs = [srv.submit_frames(vid2, frames[a:a + 30].contiguous(), poses[a:a + 30].contiguous(), wl.sweep.pitch)
            for a in range(0, F, 30)]
    srv.drain()
    for t in jobs:
        srv.poll_frames(t)
    el2 = time.perf_counter() - t1
    srv.close()
    # algorithmic bytes of compounding per input pixel when the pixel pitch equals the voxel size
    # (FP16 storage): 1 B read, 16 B accumulator read-modify-write, finalize 8 B read + 4 B pair
    bpp = 1 + 16 + 8 + 4
    res = {"grid": list(wl.dims), "dtype": "f16", "frame_px": [Wf, Hf], "rate_hz": rate, "seconds": round(el, 2),
           "frames": nfr, "frames_per_s": round(nfr / el, 1), "bins": int(info.bins),
           "bricks_used": int(info.bricks_used), "consoles": 32,
           "reslice_latency_ms": {"p50": round(percentile(lat, 50), 3), "p99": round(percentile(lat, 99), 3),
                                  "requests": len(lat)},
           "frame_latency_ms": {"p50": round(percentile(flat, 50), 3), "p99": round(percentile(flat, 99), 3)},
           "compound_ms_per_frame": round(1e3 * comp_s / max(nfr, 1), 3),
           "flat_out_frames_per_s": round(F / el2, 1),
           "compound_algorithmic_GBps": round(F * Wf * Hf * bpp / el2 / 1e9, 1)}
    del frames, poses, vol, vol2
    torch.cuda.empty_cache()
    return res


def served_mix_bytes(torch, dare, vols, wls, consoles, mix, sample, rng):
    """Algorithmic bytes of the saturation run's served mix: for a seeded sample of its (console,
    sequence entry) requests, the exact footprint voxels x surviving bins x BF16 pair bytes + 4 B
    of output per pixel (the per-pixel figure of the reslice); bytes per pixel averaged per output
    size, times the pixels served at that size."""
    steps, served = mix["steps"], mix["served"]
    nc, seq_len = served.shape
    picks = rng.choice(nc * seq_len, size=min(sample, nc * seq_len), replace=False)
    per_size = {}
    for q in picks:
        k, i = divmod(int(q), seq_len)
        P, n, pitch = steps[k][i]
        vi = consoles[k].vol_index
        wl = wls[vi]
        kact = len(vols[vi].active_bins(P, n, n, pitch)[0])
        nvox = footprint_voxels(torch, P, wl.calib, wl.origin, wl.spacing, wl.dims, n, n, pitch)
        per_size.setdefault(n, []).append((4 * n * n + nvox * kact * PAIR_BYTES["bf16"]) / (n * n))
    total, px = 0.0, 0
    for k in range(nc):
        for i in range(seq_len):
            n = steps[k][i][1]
            cnt = int(served[k, i])
            if cnt and n in per_size:
                total += cnt * n * n * float(np.mean(per_size[n]))
                px += cnt * n * n
    return total, px, {int(n): round(float(np.mean(v)), 3) for n, v in sorted(per_size.items())}, len(picks)


def run_serving(dare, torch, synth, seconds, sat_seconds, budget_seconds, log, sample_cap=200):
    """Serving form: 4 resident BF16 volumes admitted against a volume budget, 64 consoles,
    Poisson arrivals at 30 Hz each.  (a) the offered load, with a seeded 1 % sample of the
    requests to the 128^3 and 256^3 volumes (at most sample_cap) kept for the oracle;
    (b) saturation: closed loop, with the device time of the ticks' kernels and the served mix's
    algorithmic bytes (the served path's HBM roofline); (c) a small budget: a volume budget that
    refuses the fourth volume until one is removed, and an arena and queue that make requests
    wait for result slots and refuse them when the queue is full."""
    dev = torch.device("cuda:0")
    vols, wls, host_frames = [], [], []
    t0 = time.perf_counter()
    for N, seed in ((128, 41), (256, 42), (256, 43), (384, 44)):
        wl = synth.serving_volume(N, seed)
        fr = wl.render(dev)
        poses = torch.from_numpy(np.ascontiguousarray(wl.sweep.probe_poses, np.float32)).to(dev)
        geom = dare.make_geometry(wl.origin, wl.spacing, wl.dims, wl.calib)
        nb = ((N + 7) // 8) ** 3
        v = dare.Volume(geom, dare.default_params(), dtype="bf16", bricks=nb * 40)
        v.reconstruct(fr, poses, wl.sweep.pitch)
        host_frames.append(fr.cpu().numpy() if N <= 256 else None)   # the oracle checks volumes 0..2
        del fr, poses
        vols.append(v)
        wls.append(wl)
    torch.cuda.synchronize()
    vol_bytes = [int(v.arena.numel()) for v in vols]
    log(f"serving: built 4 BF16 volumes in {time.perf_counter() - t0:.1f} s: "
        + ", ".join(f"{w.dims[0]}^3 {v.info().bins} bins {b / 1e6:.0f} MB" for w, v, b in zip(wls, vols, vol_bytes)))
    sizes = (256, 512, 768, 1024)
    srv = dare.Server(2 << 30, n_streams=3, max_tick_requests=64, max_tick_pixels=16 << 20, max_queue=8192,
                      volume_budget_bytes=sum(vol_bytes))
    ids = [srv.add_volume(v) for v in vols]
    rng = np.random.default_rng(2024)
    consoles = [Console(rng, wls[k // 16], ids[k // 16], sizes) for k in range(64)]
    for k, c in enumerate(consoles):
        c.vol_index = k // 16
    ring = 6
    bufs = [[torch.empty((1024 * 1024,), dtype=torch.float32, pin_memory=True) for _ in range(ring)]
            for _ in range(64)]
    for vi in range(4):                         # warm up every size once per volume
        for n in sizes:
            L = wls[vi].dims[0] * wls[vi].spacing
            t = srv.submit(ids[vi], consoles[vi * 16].step(0.0, synth)[0], n, n, (L / n, L / n), bufs[0][0])
            srv.drain()
            srv.poll(t)

    sample_rng = np.random.default_rng(7)
    served_sample = []                          # (volume index, pose, n, pitch, result)

    def run(server, cons, duration, rate=30.0, keep_sample=False):
        """Open loop: each console submits at Poisson arrivals of `rate` per second."""
        nc = len(cons)
        next_t = [time.perf_counter() + rng.exponential(1.0 / rate) for _ in range(nc)]
        last = [time.perf_counter()] * nc
        slot = [0] * nc
        pending = {}
        sampled = {}
        lat = {n: [] for n in sizes}
        dev_lat, wait = [], []
        px = 0
        refused = 0
        t_start = time.perf_counter()
        st0 = server.stats()

        def reap(tk, states, times):
            nonlocal px
            for j in np.nonzero(states != dare.ERR_NOT_READY)[0]:
                k, n = pending.pop(int(tk[j]))
                if states[j] != dare.OK:
                    raise dare.DareError(int(states[j]), "served request")
                if int(tk[j]) in sampled:
                    vi, P_s, pitch_s, buf_s = sampled.pop(int(tk[j]))
                    served_sample.append((vi, P_s, n, pitch_s, buf_s[:n * n].numpy().reshape(n, n).copy()))
                lat[n].append(1e3 * (times["t_host_done"][j] - times["t_submit"][j]))
                dev_lat.append(1e3 * (times["t_device_done"][j] - times["t_submit"][j]))
                wait.append(1e3 * (times["t_admit"][j] - times["t_submit"][j]))
                px += n * n

        while True:
            now = time.perf_counter()
            if now - t_start > duration:
                break
            for k in range(nc):
                if now < next_t[k]:
                    continue
                c = cons[k]
                P, n, pitch = c.step(max(1e-3, now - last[k]), synth)
                last[k] = now
                buf = bufs[k][slot[k] % ring]
                slot[k] += 1
                t = server.submit(c.vol_id, P, n, n, pitch, buf)
                if t is not None:
                    pending[t] = (k, n)
                    if (keep_sample and c.vol_index < 3 and len(served_sample) + len(sampled) < sample_cap
                            and sample_rng.random() < 0.01):
                        sampled[t] = (c.vol_index, P, pitch, buf)
                else:
                    refused += 1
                next_t[k] += rng.exponential(1.0 / rate)
            if pending:
                tk = np.fromiter(pending.keys(), np.uint64, len(pending))
                reap(tk, *server.poll_many(tk))
        server.drain()
        if pending:
            tk = np.fromiter(pending.keys(), np.uint64, len(pending))
            reap(tk, *server.poll_many(tk))
        el = time.perf_counter() - t_start
        st1 = server.stats()
        alll = [x for v in lat.values() for x in v]
        return {"seconds": round(el, 2), "requests": len(alll), "refused_queue_full": refused,
                "Mpx_s": round(px / el / 1e6, 1),
                "latency_ms": {"p50": round(percentile(alll, 50), 3), "p99": round(percentile(alll, 99), 3),
                               "p99_512": round(percentile(lat[512], 99), 3),
                               "p50_512": round(percentile(lat[512], 50), 3),
                               "p99_1024": round(percentile(lat[1024], 99), 3),
                               "device_p99": round(percentile(dev_lat, 99), 3),
                               "queue_wait_p99": round(percentile(wait, 99), 3)},
                "ticks": int(st1.ticks - st0.ticks),
                "mean_requests_per_tick": round(len(alll) / max(1, st1.ticks - st0.ticks), 2),
                "busy_fraction": round((st1.busy_seconds - st0.busy_seconds) / el, 3),
                "device_busy_fraction": round((st1.device_busy_seconds - st0.device_busy_seconds) / el, 4)}

    offered = run(srv, consoles, seconds, keep_sample=True)
    log(f"serving at 64 x 30 Hz: {offered}")
    sat, mix = run_closed(srv, consoles, bufs, ring, sizes, sat_seconds, synth)
    log(f"serving saturated (closed loop, 2 in flight per console, grouped submit/poll): {sat}")
    # (d) the same closed loop delivering into device buffers: no transfer over the host link
    dbufs = [[torch.empty((1024 * 1024,), dtype=torch.float32, device=dev) for _ in range(ring)] for _ in range(64)]
    sat_dev, _ = run_closed(srv, consoles, dbufs, ring, sizes, 0.5 * sat_seconds, synth)
    log(f"serving saturated, results delivered to device buffers: {sat_dev}")
    del dbufs
    srv.close()

    # the served path's roofline: the saturation run's algorithmic bytes over the union of its
    # ticks' kernel spans (device time)
    algo, px_m, bpp, nsamp = served_mix_bytes(torch, dare, vols, wls, consoles, mix, 256, np.random.default_rng(5))
    dev_s = mix["device_busy_seconds"]
    ach = algo / max(dev_s, 1e-9) / 1e9
    roofline_served = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                       "kernels": "k_tiles_setup + k_tiles + k_tiles_direct, one graph per tick",
                       "run": "saturation", "device_busy_seconds": round(dev_s, 4),
                       "device_Mpx_s": sat["device_Mpx_s"], "mean_tick_kernel_ms": sat["mean_tick_kernel_ms"],
                       "algo_bytes": round(algo), "algo_bytes_per_px_by_size": bpp,
                       "bytes_basis": f"BF16 pairs of the exact footprint x surviving bins + 4 B/px output, per "
                                      f"output size from a seeded sample of {nsamp} of the run's requests"}
    log(f"served roofline: {roofline_served}")

    # (c) small budget: a volume budget of the three largest volumes' bytes (volumes 0..2 are
    # admitted, the fourth refused until volume 0 is removed); an arena with room for one 1024^2
    # result beside the streams' workspaces and a 32-deep queue, under four times the load
    budget = sum(vol_bytes[1:])
    cfg_c = dict(n_streams=3, max_tick_requests=64, max_tick_pixels=16 << 20, max_queue=32, volume_budget_bytes=budget)
    lo, hi = 1 << 20, 1 << 31                  # smallest arena that takes the first volume
    while lo < hi:
        mid = (lo + hi) // 2
        s_try = dare.Server(mid, **cfg_c)
        try:
            s_try.add_volume(vols[0])
            hi = mid
        except dare.DareError:
            lo = mid + 1
        s_try.close()
    arena_c = lo + (4 << 20) + 4096
    srv_c = dare.Server(arena_c, **cfg_c)
    ids_c = [srv_c.add_volume(v) for v in vols[:3]]
    admission = {"budget_bytes": budget, "arena_bytes": arena_c, "result_slots_1024": 1, "max_queue": 32}
    try:
        srv_c.add_volume(vols[3])
        admission["fourth_volume"] = "admitted"
    except dare.DareError as e:
        admission["fourth_volume"] = "refused" if e.status == dare.ERR_BUDGET else f"error {e.status}"
    cons_c = [Console(rng, wls[k // 16], ids_c[k // 16], sizes) for k in range(48)]
    for k, c in enumerate(cons_c):
        c.vol_index = k // 16
    small = run(srv_c, cons_c, budget_seconds, rate=120.0)
    srv_c.remove_volume(ids_c[0])
    try:
        srv_c.add_volume(vols[3])
        admission["fourth_volume_after_removing_one"] = "admitted"
    except dare.DareError as e:
        admission["fourth_volume_after_removing_one"] = f"refused ({e.status})"
    small["admission"] = admission
    small["consoles"] = 48
    small["rate_hz_per_console"] = 120
    srv_c.close()
    log(f"serving under a small budget: {small}")

    res = {"volumes": [list(w.dims) for w in wls], "volume_MB": [round(b / 1e6, 1) for b in vol_bytes],
           "dtype": "bf16", "consoles": 64, "rate_hz_per_console": 30, "sizes": list(sizes), "offered": offered,
           "saturation": sat, "saturation_device_delivery": sat_dev, "small_budget": small}
    sample = {"workloads": wls[:3], "frames": host_frames[:3], "items": served_sample}
    return res, roofline_served, sample


def run_fan(dare, torch, synth, dev, bricks, log):
    """Curvilinear-probe compounding at config-2 scale: the three azimuth sweeps of 600 frames
    imaged by a 192-beam fan (256 rows), binned per column sector, timed as the linear
    reconstruction is (median of three builds after a warm-up build); then 100 slices of 512^2
    resliced from the fan-built volume, one launch each."""
    wl = synth.fan_config2()
    fr = wl.render(dev)
    po = torch.from_numpy(np.ascontiguousarray(wl.sweep.probe_poses, np.float32)).to(dev)
    beams = torch.from_numpy(np.ascontiguousarray(wl.beams, np.float64)).to(dev)
    geom = dare.make_geometry(wl.origin, wl.spacing, wl.dims, wl.calib)
    prm = dare.default_params()
    fz = wl.fan
    times, vol = [], None
    for k in range(4):
        vol = dare.Volume(geom, prm, dtype="f32", bricks=bricks)
        torch.cuda.synchronize()
        t = time.perf_counter()
        vol.reconstruct_fan(fr, po, fz["apex"], fz["r0"], fz["dr"], fz["sectors"], beams)
        torch.cuda.synchronize()
        if k:
            times.append(time.perf_counter() - t)
    F, H, W = fr.shape
    info = vol.info()
    sl = wl.slices
    specs = [dare.make_spec(P, sl.width, sl.height, sl.pitch) for P in sl.probe_poses]
    out = torch.empty((len(specs), sl.height, sl.width), dtype=torch.float32, device=dev)
    sh = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    for k, sp in enumerate(specs):
        dare.lib.dare_reslice(vol.handle, ct.byref(sp), ct.c_void_p(out[k].data_ptr()), sh)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k, sp in enumerate(specs):
        dare.lib.dare_reslice(vol.handle, ct.byref(sp), ct.c_void_p(out[k].data_ptr()), sh)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / len(specs)
    med = float(np.median(times))
    res = {"workload": wl.name, "frames": int(F), "frame_px": [W, H], "sectors": int(fz["sectors"]),
           "bins": int(info.bins), "bricks_used": int(info.bricks_used),
           "reconstruct_ms": round(1e3 * med, 3), "frames_per_s": round(F / med, 1),
           "input_Mpx_s": round(F * W * H / med / 1e6, 1),
           "reslice_ms_per_slice": round(ms, 4), "reslice_Mpx_s": round(sl.width * sl.height / (ms * 1e-3) / 1e6, 1),
           "unassigned_fraction": round(float(torch.isnan(out).float().mean()), 4)}
    log(f"curvilinear: {res}")
    del vol, fr, out
    torch.cuda.synchronize()
    return res


def run_out_of_core(dare, torch, geom, prm, frames, poses, pitch, total_bricks, in_core_ms, log):
    """Out-of-core bricks on config 2: the 1800 frames compounded 100 per call with spilling on,
    in an arena of a third of the bricks the volume needs; then every brick moved to host memory
    and one z quarter of the grid brought back (PCIe rates from the bytes moved)."""
    cap = max(1, total_bricks // 3)
    vol = dare.Volume(geom, prm, dtype="f32", bricks=cap)
    vol.set_spill(True)
    F = frames.shape[0]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for a in range(0, F, 100):
        vol.reconstruct(frames[a:a + 100], poses[a:a + 100], pitch)
    torch.cuda.synchronize()
    t_spill = time.perf_counter() - t
    held, held_bytes = vol.held()
    resident = vol.info().bricks_used
    acc_bytes = 512 * 8
    t = time.perf_counter()
    vol.evict_outside((1, 1, 1), (0, 0, 0))
    t_evict = time.perf_counter() - t
    nz = int(geom.dims[2])
    lo, hi = (0, 0, 0), (int(geom.dims[0]) - 1, int(geom.dims[1]) - 1, nz // 4 - 1)
    n_before = vol.held()[0]
    t = time.perf_counter()
    try:
        vol.restore_box(lo, hi)
        restored = n_before - vol.held()[0]
    except dare.DareError:
        restored = 0
    t_restore = time.perf_counter() - t
    res = {"arena_bricks": int(vol.info().bricks_capacity), "volume_bricks": int(total_bricks),
           "spill_reconstruct_ms": round(1e3 * t_spill, 2), "in_core_reconstruct_ms": round(in_core_ms, 2),
           "calls": (F + 99) // 100, "held_after_reconstruct": int(held), "held_MB": round(held_bytes / 1e6, 1),
           "resident_after_reconstruct": int(resident),
           "evict_bricks": int(resident), "evict_ms": round(1e3 * t_evict, 2),
           "evict_GBps": round(resident * acc_bytes / max(t_evict, 1e-9) / 1e9, 2),
           "restore_bricks": int(restored), "restore_ms": round(1e3 * t_restore, 2),
           "restore_GBps": round(restored * acc_bytes / max(t_restore, 1e-9) / 1e9, 2)}
    log(f"out-of-core: {res}")
    del vol
    torch.cuda.synchronize()
    return res


def run_evaluation(dare, torch, synth, config, bricks, log):
    """The evaluation protocol of Sec. 2.2 and Sec. 3 on config 1 or 2: reconstruct from the
    initial sweep set at its tracked poses (each sweep misregistered by a seeded rigid offset),
    reslice at the tracked poses of a secondary, different sweep, and score every reslice with
    NCC and SSIM against that sweep's acquired frame and against the same view rendered without
    speckle (speckle is drawn per frame, so no reconstruction can predict it); DARE against plain
    mean compounding (thresholds at 180 degrees, k = 0: every sample weighs 1)."""
    dev = torch.device("cuda:0")
    pair = synth.eval_pair(config)
    wl, sw = pair.initial, pair.secondary
    frames = wl.render(dev)
    sec = sw.render(dev)
    poses = torch.from_numpy(np.ascontiguousarray(pair.initial_tracked)).to(dev)
    geom = dare.make_geometry(wl.origin, wl.spacing, wl.dims, wl.calib)
    G, Hf, Wf = sec.shape
    pitch = sw.sweep.pitch
    echo = synth.render.render_frames(dataclasses.replace(wl.phantom, speckle_sigma=0.0), sw.sweep.probe_poses,
                                      wl.calib, Wf, Hf, pitch, seed=0, device=dev)
    ws_c = torch.empty(int(dare.lib.dare_compare_workspace_bytes()), dtype=torch.uint8, device=dev)
    img = torch.empty((Hf, Wf), dtype=torch.float32, device=dev)
    out = {"initial_frames": int(frames.shape[0]), "secondary_frames": int(G), "frame_px": [Wf, Hf],
           "tracking_offsets_mm_deg": pair.offsets_mm_deg,
           "protocol": "reconstruct from the initial sweeps at their tracked poses; reslice at the secondary "
                       "sweep's tracked poses; score against its frames (rendered at its true poses)"}
    q = lambda xs: [round(float(np.nanpercentile(xs, p_)), 4) for p_ in (25, 50, 75)]  # noqa: E731
    for name, prm_e in (("dare", dare.default_params()),
                        ("plain_mean", dare.default_params(k_normal=0.0, k_inplane=0.0, thr_normal_deg=180.0,
                                                           thr_inplane_deg=180.0))):
        v_e = dare.Volume(geom, prm_e, dtype="f32", bricks=bricks)
        v_e.reconstruct(frames, poses, wl.sweep.pitch)
        res = {"vs_frame": ([], []), "vs_echo": ([], [])}
        fracs = []
        t_cmp = 0.0
        for k in range(G):
            v_e.reslice(pair.secondary_tracked[k], Wf, Hf, pitch, out=img)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c = dare.compare_to_frame(img, sec[k], ws_c)
            t_cmp += time.perf_counter() - t0
            ce = dare.compare_to_frame(img, echo[k], ws_c)
            for key, cc in (("vs_frame", c), ("vs_echo", ce)):
                res[key][0].append(cc[0])
                res[key][1].append(cc[1])
            fracs.append(c[2] / (Wf * Hf))
        out[name] = {}
        for key, (ncc, ssim) in res.items():
            qn, qs = q(ncc), q(ssim)
            out[name][key] = {"ncc_q25_median_q75": qn, "ncc_iqr": round(qn[2] - qn[0], 4),
                              "ssim_q25_median_q75": qs, "ssim_iqr": round(qs[2] - qs[0], 4)}
        out[name]["assigned_fraction_mean"] = round(float(np.mean(fracs)), 4)
        out[name]["compare_ms_per_image"] = round(1e3 * t_cmp / G, 3)
        log(f"evaluation config {config} {name}: {out[name]}")
        del v_e
    del frames, sec, echo, poses
    torch.cuda.synchronize()
    return out


# ---- the FP64 oracle on the host cores, in a child process that never touches the GPU ----------
#
# The parent sends the inputs (frames, poses, slice poses) and the GPU's results as raw arrays
# over a pipe; the child compounds with the oracle, reslices over a pool of forked workers (which
# share the oracle's grids copy-on-write) and returns timings and error statistics as one JSON
# line.  Nothing in the child imports torch or the library.

def cpu_share():
    """(CPUs in this process's affinity mask, CPU quota of its cgroup or None, pool workers)."""
    aff = len(os.sched_getaffinity(0))
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            q, per = fh.read().split()[:2]
        if q != "max":
            quota = max(1, int(math.ceil(int(q) / int(per))))
    except (OSError, ValueError):
        pass
    return aff, quota, (min(aff, quota) if quota else aff)


def send_arrays(fh, meta, arrays):
    """One JSON header line (meta, then name/dtype/shape of every array), then the raw bytes."""
    hdr = {"meta": meta, "arrays": [{"name": k, "dtype": str(a.dtype), "shape": list(a.shape)}
                                    for k, a in arrays.items()]}
    fh.write((json.dumps(hdr) + "\n").encode())
    for a in arrays.values():
        fh.write(memoryview(np.ascontiguousarray(a)).cast("B"))
    fh.flush()


def recv_arrays(fh):
    hdr = json.loads(fh.readline())
    arrays = {}
    for d in hdr["arrays"]:
        a = np.empty(d["shape"], np.dtype(d["dtype"]))
        mv = memoryview(a).cast("B")
        got = 0
        while got < mv.nbytes:
            n = fh.readinto(mv[got:])
            if not n:
                raise EOFError(f"input ended inside array {d['name']}")
            got += n
        arrays[d["name"]] = a
    return hdr["meta"], arrays


def _err_partial(got, ref):
    """(max |got - ref|, sum, pixels, NaN masks equal, pixels whose NaN status differs), the
    differences over the pixels both assign."""
    gn, rn = np.isnan(got), np.isnan(ref)
    mism = int(np.count_nonzero(gn != rn))
    m = ~gn & ~rn
    if not m.any():
        return 0.0, 0.0, 0, mism == 0, mism
    d = np.abs(got[m].astype(np.float64) - ref[m])
    return float(d.max()), float(d.sum()), int(m.sum()), mism == 0, mism


def _err_merge(parts):
    worst = max((p[0] for p in parts), default=0.0)
    tot = sum(p[1] for p in parts)
    cnt = sum(p[2] for p in parts)
    return {"max_abs_grey": round(worst, 6), "mean_abs_grey": round(tot / max(cnt, 1), 7),
            "nan_mask_equal": all(p[3] for p in parts), "nan_mask_mismatch_pixels": sum(p[4] for p in parts),
            "pixels": cnt}


_OJ = {}      # the child's job state, set before its pool forks


def _oracle_job(k):
    """Worker: reslice item k of the current job with the oracle and compare the GPU results."""
    from oracle import reslice as oreslice
    j = _OJ
    if j["kind"] == "served":
        P, n, pitch = j["P"][k], int(j["n"][k]), tuple(j["pitch"][k])
        W = H = n
        got = {"bf16": j["res"][int(j["off"][k]):int(j["off"][k]) + n * n].reshape(n, n)}
    else:
        P, W, H, pitch = j["P"][k], j["W"], j["H"], j["pitch"]
        got = {name: arr[k] for name, arr in j["gpu"].items()}
    t = time.perf_counter()
    ref = oreslice.reslice(j["a"], j["c"], j["origin"], j["spacing"], j["rep_n"], j["rep_x"], j["calib"], P, W, H,
                           pitch, j["prm"])
    dt = time.perf_counter() - t
    return k, dt, {name: _err_partial(g, ref) for name, g in got.items()}


def oracle_child():
    """Entry of the child process (bench.py --oracle-child): read the inputs from stdin, print
    one JSON line of results on stdout, progress on stderr."""
    import multiprocessing as mp

    from oracle import compound
    from oracle.reslice import Params as OParams

    def clog(msg):
        print(f"[bench:oracle] {msg}", file=sys.stderr, flush=True)

    meta, arrs = recv_arrays(sys.stdin.buffer)
    workers = int(meta["workers"])
    prm = OParams()
    ctx = mp.get_context("fork")
    out = {"workers": workers}

    def build(g):
        t = time.perf_counter()
        grid = compound.empty_grid(g["origin"], g["spacing"], g["dims"], prm.bin_tol_deg, prm.max_bins)
        compound.compound(grid, arrs[g["frames"]], arrs[g["poses"]], np.asarray(g["calib"]).reshape(4, 4),
                          tuple(g["pitch"]))
        t_c = time.perf_counter() - t
        a, c = grid.mean_count()
        rep_n, rep_x = grid.codebook.arrays()
        touched = int(np.count_nonzero(grid.C))
        K = grid.K
        del grid
        return {"a": a, "c": c, "rep_n": rep_n, "rep_x": rep_x, "origin": np.asarray(g["origin"], np.float64),
                "spacing": float(g["spacing"]), "calib": np.asarray(g["calib"], np.float64).reshape(4, 4),
                "prm": prm}, t_c, touched, K

    def pool_run(n, nw):
        t = time.perf_counter()
        with ctx.Pool(nw) as pool:
            res = pool.map(_oracle_job, range(n), chunksize=1)
        return time.perf_counter() - t, res

    # config 2: compounding of every frame, one slice on one core, then the 16 slices on the pool
    if "config2" in meta:
        g = meta["config2"]
        state, t_c, touched, K = build(g)
        clog(f"config 2: compounded {arrs[g['frames']].shape[0]} frames in {t_c:.1f} s, {K} bins")
        _OJ.clear()
        _OJ.update(state, kind="slices", P=arrs[g["slices"]], W=g["W"], H=g["H"], pitch=tuple(g["slice_pitch"]),
                   gpu={name: arrs[a] for name, a in g["gpu"].items()})
        n = arrs[g["slices"]].shape[0]
        _, t_one, _ = _oracle_job(0)
        nw = min(workers, n)
        t_pool, res = pool_run(n, nw)
        out["config2"] = {"compound_seconds": round(t_c, 2), "bins": K, "touched_bin_voxels": touched,
                          "single_core_seconds_per_slice": round(t_one, 3), "slices": n, "pool_workers": nw,
                          "pool_seconds": round(t_pool, 2),
                          "pool_Mpx_s": round(n * g["W"] * g["H"] / t_pool / 1e6, 4),
                          "single_core_Mpx_s": round(g["W"] * g["H"] / t_one / 1e6, 4),
                          "errors": {name: _err_merge([r[2][name] for r in res]) for name in g["gpu"]}}
        clog(f"config 2: {out['config2']}")
        _OJ.clear()
        del state

    # config 1 in full (compounding and its 16 slices), then config 3's slices on the same grid
    if "config1" in meta:
        g = meta["config1"]
        state, t_c, touched, K = build(g)
        _OJ.clear()
        _OJ.update(state, kind="slices", P=arrs[g["slices"]], W=g["W"], H=g["H"], pitch=tuple(g["slice_pitch"]),
                   gpu={name: arrs[a] for name, a in g["gpu"].items()})
        n = arrs[g["slices"]].shape[0]
        t_pool, res = pool_run(n, min(workers, n))
        out["config1"] = {"compound_seconds": round(t_c, 3), "bins": K, "slices": n, "pool_seconds": round(t_pool, 2),
                          "errors": {name: _err_merge([r[2][name] for r in res]) for name in g["gpu"]}}
        clog(f"config 1: {out['config1']}")
        g3 = meta.get("config3")
        if g3:
            _OJ.update(P=arrs[g3["slices"]], W=g3["W"], H=g3["H"], pitch=tuple(g3["slice_pitch"]),
                       gpu={name: arrs[a] for name, a in g3["gpu"].items()})
            n3 = arrs[g3["slices"]].shape[0]
            t3, res3 = pool_run(n3, min(workers, n3))
            out["config3"] = {"slices": n3, "pool_seconds": round(t3, 1),
                              "errors": {name: _err_merge([r[2][name] for r in res3]) for name in g3["gpu"]}}
            clog(f"config 3: {out['config3']}")
        _OJ.clear()
        del state

    # served results: every sampled volume compounded in turn, its sampled requests on the pool
    if "served" in meta:
        parts, nreq, t_tot = [], [], 0.0
        for g in meta["served"]:
            state, t_c, _, _ = build(g)
            _OJ.clear()
            _OJ.update(state, kind="served", P=arrs[g["req_P"]], n=arrs[g["req_n"]], pitch=arrs[g["req_pitch"]],
                       off=arrs[g["req_off"]], res=arrs[g["results"]])
            n = arrs[g["req_n"]].shape[0]
            if n:
                t_p, res = pool_run(n, min(workers, n))
                parts += [r[2]["bf16"] for r in res]
                t_tot += t_p
            nreq.append(int(n))
            clog(f"served: volume {g['dims']} compounded in {t_c:.1f} s, {n} requests checked")
            _OJ.clear()
            del state
        out["served"] = dict(_err_merge(parts), requests_per_volume=nreq, pool_seconds=round(t_tot, 1))
    print(json.dumps(out), flush=True)


def run_oracle_child(meta, arrays, log):
    """Run the oracle child on these inputs; returns its JSON result, or None (logged) on failure."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-child"]
    try:
        proc = subprocess.Popen(cmd, stdin=subprocess.PIPE, stdout=subprocess.PIPE, cwd=ROOT)
    except OSError as e:
        log(f"oracle child could not start: {e}")
        return None
    try:
        send_arrays(proc.stdin, meta, arrays)
        proc.stdin.close()
    except (BrokenPipeError, OSError) as e:
        log(f"oracle child closed its input: {e}")
    out = proc.stdout.read()
    rc = proc.wait()
    if rc != 0:
        log(f"oracle child exited with status {rc}")
        return None
    try:
        return json.loads(out.decode().strip().splitlines()[-1])
    except (ValueError, IndexError):
        log("oracle child printed no result")
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--slices", type=int, default=1000)
    ap.add_argument("--cpu-slices", type=int, default=16)
    ap.add_argument("--config3-slices", type=int, default=1000)
    ap.add_argument("--served-sample", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--latency-sample", type=int, default=200)
    ap.add_argument("--counters", default=os.path.join(ROOT, "profiles", "reslice_counters.json"))
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-seconds", type=float, default=60.0)
    ap.add_argument("--saturation-seconds", type=float, default=20.0)
    ap.add_argument("--budget-seconds", type=float, default=15.0)
    ap.add_argument("--no-streaming", action="store_true")
    ap.add_argument("--no-literal", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--streaming-seconds", type=float, default=60.0)
    ap.add_argument("--oracle-child", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_child:
        oracle_child()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: it measures one GPU's share of the work (--gpus 1); "
              "sharding over several GPUs is designed, not implemented or measured.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2605_26325_amd as dare
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sh = ct.c_void_p(stream.cuda_stream)

    wl = synth.config2(n_slices=args.slices, n_near=int(round(0.8 * args.slices)))
    log(f"workload: {wl.name}")
    t0 = time.perf_counter()
    frames = wl.render(dev)
    torch.cuda.synchronize()
    log(f"rendered {tuple(frames.shape)} frames on the GPU in {time.perf_counter() - t0:.1f} s")
    poses = torch.from_numpy(np.ascontiguousarray(wl.sweep.probe_poses, np.float32)).to(dev)
    geom = dare.make_geometry(wl.origin, wl.spacing, wl.dims, wl.calib)
    prm = dare.default_params()
    nb = 1
    for d in wl.dims:
        nb *= (d + 7) // 8
    pitch_f = wl.sweep.pitch
    F, Hf, Wf = frames.shape

    def build_volume(dtype):
        vol = dare.Volume(geom, prm, dtype=dtype, bricks=nb * 40)
        torch.cuda.synchronize()
        t = time.perf_counter()
        vol.reconstruct(frames, poses, pitch_f)
        torch.cuda.synchronize()
        return vol, time.perf_counter() - t

    vol, _ = build_volume("f32")          # first build warms up the kernels
    recon_times = []
    for _ in range(3):
        v2, dt = build_volume("f32")
        recon_times.append(dt)
        del v2
    info = vol.info()
    log(f"volume: {info.bins} bins, {info.bricks_used} bricks of 8^3 used; reconstruct median "
        f"{1e3 * np.median(recon_times):.2f} ms")
    # input pixels that land in the grid (each one read-modify-writes one voxel's sum and count)
    in_grid_px = int(voxel_sample_counts(torch, tuple(frames.shape), poses, wl.calib, wl.origin, wl.spacing,
                                         wl.dims, pitch_f).sum().item())

    sl = wl.slices
    W, H, pitch = sl.width, sl.height, sl.pitch
    specs = [dare.make_spec(P, W, H, pitch) for P in sl.probe_poses]
    spec_refs = [ct.byref(s) for s in specs]
    outs = torch.empty((len(specs), H, W), dtype=torch.float32, device=dev)
    out_ptrs = [ct.c_void_p(outs[k].data_ptr()) for k in range(len(specs))]
    reslice = dare.lib.dare_reslice

    def step(v):
        h = v.handle
        for k in range(len(specs)):
            st = reslice(h, spec_refs[k], out_ptrs[k], sh)
            if st != 0:
                raise dare.DareError(st, "dare_reslice")

    for _ in range(args.warmup):
        step(vol)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step(vol)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    px_per_step = len(specs) * W * H
    value = px_per_step / (ms_per_step / 1e3) / 1e6
    log(f"fp32 one launch per slice: {ms_per_step:.2f} ms/step ({ev0.elapsed_time(ev1) / args.steps:.2f} ms "
        f"device), {value:.0f} Mpixel/s")
    nan_frac = float(torch.isnan(outs).float().mean().item())

    # ---- the same launches spread over two streams (slices are independent): one kernel's tail
    # and the next one's dispatch and setup overlap; results must not change
    concurrent = None
    if not args.no_forms:
        ref_outs = outs.clone()
        s2 = torch.cuda.Stream()
        hs = [sh, ct.c_void_p(s2.cuda_stream)]

        def step2(v):
            h = v.handle
            for k in range(len(specs)):
                st = reslice(h, spec_refs[k], out_ptrs[k], hs[k & 1])
                if st != 0:
                    raise dare.DareError(st, "dare_reslice")

        def timed2(n):
            c0, c1, c2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            torch.cuda.synchronize()
            c0.record(stream)
            s2.wait_event(c0)
            for _ in range(n):
                step2(vol)
            c2.record(s2)
            stream.wait_event(c2)
            c1.record(stream)
            torch.cuda.synchronize()
            return c0.elapsed_time(c1) / n

        timed2(max(1, args.warmup))
        ms2 = timed2(args.steps)
        same2 = bool(torch.equal(torch.nan_to_num(outs, nan=-1.0), torch.nan_to_num(ref_outs, nan=-1.0)))
        concurrent = {"streams": 2, "ms_per_step": round(ms2, 3),
                      "Mpx_s": round(px_per_step / (ms2 * 1e-3) / 1e6, 1), "equal_to_one_stream": same2}
        log(f"fp32 one launch per slice over 2 streams: {ms2:.2f} ms/step, {concurrent['Mpx_s']:.0f} Mpixel/s, "
            f"same results: {same2}")
        del ref_outs

    # ---- roofline of the reslice kernel over the timed launches: their average duration is the
    # event-timed device span of the timed steps divided by the launches in it (back to back on
    # one stream), and the algorithmic bytes are counted per slice by an untimed pass
    dev_s = ev0.elapsed_time(ev1) * 1e-3
    launches = args.steps * len(specs)
    avg_launch = dev_s / launches
    algo = []
    kacts = []
    nvoxs = []
    for k in range(len(specs)):
        kact = len(vol.active_bins(sl.probe_poses[k], W, H, pitch)[0])
        nvox = footprint_voxels(torch, sl.probe_poses[k], wl.calib, wl.origin, wl.spacing, wl.dims, W, H, pitch)
        algo.append(4 * W * H + nvox * kact * PAIR_BYTES["f32"])
        kacts.append(kact)
        nvoxs.append(nvox)
    algo = np.array(algo, dtype=np.float64)
    achieved = float(algo.mean() / avg_launch / 1e9)
    counters = stored_counters(args.counters)
    head = counters.get("k_reslice_tile<fp32>", {})
    traffic = head.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_reslice_tile<fp32>", "avg_launch_us": round(1e6 * avg_launch, 2),
                "algo_bytes_per_launch": round(float(algo.mean())), "launches": launches,
                "mean_active_bins": round(float(np.mean(kacts)), 2),
                "bytes_per_px": round(float(algo.mean()) / (W * H), 2),
                "valu": valu_roofline(head.get("valu_insts_per_launch"), avg_launch,
                                      "SQ_INSTS_VALU per launch of the committed profile over the event-timed "
                                      "average launch")}
    log(f"roofline: {achieved:.0f} GB/s algorithmic over {launches} launches, mean {1e6 * avg_launch:.1f} us, "
        f"{algo.mean() / 1e6:.2f} MB/launch, active bins {np.mean(kacts):.2f}")

    # ---- copy bandwidth on this machine (calibrates the roofline and the byte counters)
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dare.dare_copy_probe(src, dst, nbytes)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        dare.dare_copy_probe(src, dst, nbytes)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    roofline["copy_probe_GBps"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(achieved / copy_gbs, 4)

    # ---- unloaded latency: submit -> result in pinned host memory, one request at a time
    lat_out = torch.empty((H, W), dtype=torch.float32, device=dev)
    lat_ptr = ct.c_void_p(lat_out.data_ptr())

    def latencies(v, n):
        if n <= 0:
            return None
        host = torch.empty((H, W), dtype=torch.float32, pin_memory=True)
        lat, dlat = [], []
        for k in range(n):
            e_a, e_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t = time.perf_counter()
            e_a.record(stream)
            reslice(v.handle, spec_refs[k % len(specs)], lat_ptr, sh)
            e_b.record(stream)
            host.copy_(lat_out, non_blocking=True)
            stream.synchronize()
            lat.append(1e3 * (time.perf_counter() - t))
            dlat.append(e_a.elapsed_time(e_b))
        return {"p50": round(percentile(lat, 50), 4), "p99": round(percentile(lat, 99), 4),
                "device_p50": round(percentile(dlat, 50), 4), "device_p99": round(percentile(dlat, 99), 4)}

    lat32 = latencies(vol, args.latency_sample)
    if lat32:
        log(f"fp32 latency submit->host p50 {lat32['p50']:.3f} ms p99 {lat32['p99']:.3f} ms")

    # ---- precision forms and the batched entry point on the same slices
    forms = {}
    form_vols = {}
    roofline_batched = {}
    if not args.no_forms:
        for dt in ("bf16", "f16", "fp8"):
            v, dtr = build_volume(dt)
            form_vols[dt] = v
            outs_f = torch.empty_like(outs)
            ptrs_f = [ct.c_void_p(outs_f[k].data_ptr()) for k in range(len(specs))]
            for _ in range(max(1, args.warmup)):
                for k in range(len(specs)):
                    reslice(v.handle, spec_refs[k], ptrs_f[k], sh)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for k in range(len(specs)):
                reslice(v.handle, spec_refs[k], ptrs_f[k], sh)
            torch.cuda.synchronize()
            mpx = px_per_step / (time.perf_counter() - t) / 1e6
            m = ~torch.isnan(outs)
            diff = (outs_f - outs)[m].abs()
            forms[dt] = {"one_launch_per_slice_Mpx_s": round(mpx, 1),
                         "max_abs_diff_vs_fp32": round(float(diff.max().item()), 4),
                         "mean_abs_diff_vs_fp32": round(float(diff.mean().item()), 5),
                         "reconstruct_ms": round(1e3 * dtr, 2)}
            if dt == "bf16":
                forms[dt]["latency_ms"] = latencies(v, args.latency_sample)
            log(f"{dt}: {mpx:.0f} Mpixel/s, max |diff| vs fp32 {forms[dt]['max_abs_diff_vs_fp32']}")
            del outs_f
        # batched: groups of 64 slices per dare_reslice_batch call
        for dt, v in (("f32", vol), ("bf16", form_vols["bf16"])):
            G = 64
            groups = [list(range(a, min(a + G, len(specs)))) for a in range(0, len(specs), G)]
            ws_bytes = max(dare.dare_reslice_batch_workspace_bytes([v] * len(g), [specs[k] for k in g])
                           for g in groups)
            wss = [torch.empty(ws_bytes, dtype=torch.uint8, device=dev) for _ in groups]
            outs_b = torch.empty_like(outs)
            # argument arrays built once, as for the one-launch step: the timed loop calls the library
            bargs = []
            for gi, g in enumerate(groups):
                n = len(g)
                bargs.append(((ct.c_void_p * n)(*([v.handle] * n)), (dare.SliceSpec * n)(*[specs[k] for k in g]),
                              (ct.c_void_p * n)(*[outs_b[k].data_ptr() for k in g]), n,
                              ct.c_void_p(wss[gi].data_ptr()), ct.c_uint64(ws_bytes)))
            batch_call = dare.lib.dare_reslice_batch

            def run_batches():
                for a in bargs:
                    st = batch_call(*a, sh)
                    if st != 0:
                        raise dare.DareError(st, "dare_reslice_batch")

            run_batches()
            torch.cuda.synchronize()
            eb0, eb1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t = time.perf_counter()
            eb0.record(stream)
            for _ in range(args.steps):
                run_batches()
            eb1.record(stream)
            torch.cuda.synchronize()
            mpx = args.steps * px_per_step / (time.perf_counter() - t) / 1e6
            key = "fp32" if dt == "f32" else dt
            forms.setdefault(key, {})["batched64_Mpx_s"] = round(mpx, 1)
            # algorithmic bytes of the same slices at this storage's pair size, over the device span
            dev_b = eb0.elapsed_time(eb1) * 1e-3
            algo_b = float(sum(4 * W * H + nv * ka * PAIR_BYTES[dt] for nv, ka in zip(nvoxs, kacts)))
            ach_b = algo_b * args.steps / dev_b / 1e9
            calls = args.steps * len(groups)
            names = ["k_tiles_setup", f"k_tiles<{key}>", f"k_tiles_direct<{key}>"]
            kc = [counters.get(n) for n in names]
            b_traffic = None
            if kc[1] is not None:
                b_traffic = round(sum(c.get("hbm_bytes_per_launch", 0.0) for c in kc if c) * len(groups))
            b_valu = None
            if all(c is not None for c in kc):
                b_valu = valu_roofline(sum(c["valu_insts_per_launch"] for c in kc), dev_b / calls,
                                       "SQ_INSTS_VALU of the three kernels per call (committed profile) over "
                                       "the event-timed device time per call")
            roofline_batched[key] = {"bound": "hbm", "achieved": round(ach_b, 1), "peak": HBM_PEAK_GBS,
                                     "unit": "GB/s", "frac": round(ach_b / HBM_PEAK_GBS, 4),
                                     "traffic": b_traffic,
                                     "kernels": "k_tiles_setup + k_tiles + k_tiles_direct, 64 slices per call",
                                     "algo_bytes_per_step": round(algo_b),
                                     "device_ms_per_step": round(1e3 * dev_b / args.steps, 3),
                                     "valu": b_valu}
            if dt == "f32":
                same = bool(torch.equal(torch.nan_to_num(outs_b, nan=-1.0), torch.nan_to_num(outs, nan=-1.0)))
                forms[key]["batched_equals_alone"] = same
            log(f"{dt} batched x64: {mpx:.0f} Mpixel/s")
            del outs_b, wss

    # ---- radius sweep: one launch per slice at R = 1, 2, 4 voxels (0.125, 0.25, 0.5 mm), first 100 slices
    radius = None
    if not args.no_forms:
        radius = {}
        nr = min(100, len(specs))
        rad_out = torch.empty((H, W), dtype=torch.float32, device=dev)    # the sweep's own output
        rad_ptr = ct.c_void_p(rad_out.data_ptr())
        for R in (1, 2, 4):
            vR = dare.Volume(geom, dare.default_params(radius_vox=float(R)), dtype="f32", bricks=nb * 40)
            vR.reconstruct(frames, poses, pitch_f)
            for k in range(nr):
                reslice(vR.handle, spec_refs[k], rad_ptr, sh)
            torch.cuda.synchronize()
            e_a, e_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e_a.record(stream)
            for k in range(nr):
                reslice(vR.handle, spec_refs[k], rad_ptr, sh)
            e_b.record(stream)
            torch.cuda.synchronize()
            ms = e_a.elapsed_time(e_b) / nr
            radius[f"R{R}"] = {"radius_mm": R * wl.spacing, "neighbourhood_voxels": (2 * R) ** 3,
                               "ms_per_slice": round(ms, 4), "Mpx_s": round(W * H / (ms * 1e-3) / 1e6, 1)}
            log(f"radius {R} ({R * wl.spacing} mm): {ms * 1e3:.1f} us per 512^2 slice")
            del vR
        torch.cuda.synchronize()
        del rad_out

    # ---- per-sample store (Sec. 2.1's flat per-sample storage read literally): built from the same
    # frames; the first 100 slices resliced one launch each in both readings; the tent reading
    # compared with the binned FP32 volume above (the binning approximation at its tolerance)
    literal_res = None
    if not args.no_forms and not args.no_literal:
        nl = min(100, len(specs))
        store = dare.SampleStore(geom, int(F) * Wf * Hf, int(F))
        builds = []
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n_samples = store.build(frames, poses, pitch_f)
            torch.cuda.synchronize()
            builds.append(time.perf_counter() - t0)
        prm_l = dare.default_params()
        lit_fn = dare.lib.dare_samples_reslice
        lit_out = torch.empty((nl, H, W), dtype=torch.float32, device=dev)
        lit_ptrs = [ct.c_void_p(lit_out[k].data_ptr()) for k in range(nl)]
        literal_res = {"samples": int(n_samples), "build_ms": round(1e3 * min(builds), 2),
                       "store_MB": round(store.arena.numel() / 1e6, 1), "slices": nl}
        for mode_name, mode in (("box", 0), ("tent", 1)):
            for k in range(nl):
                lit_fn(store.handle, ct.byref(prm_l), spec_refs[k], mode, lit_ptrs[k], sh)
            torch.cuda.synchronize()
            e_a, e_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e_a.record(stream)
            for k in range(nl):
                st_l = lit_fn(store.handle, ct.byref(prm_l), spec_refs[k], mode, lit_ptrs[k], sh)
                if st_l != 0:
                    raise dare.DareError(st_l, "dare_samples_reslice")
            e_b.record(stream)
            torch.cuda.synchronize()
            ms = e_a.elapsed_time(e_b) / nl
            literal_res[mode_name] = {"ms_per_slice": round(ms, 4), "Mpx_s": round(W * H / (ms * 1e-3) / 1e6, 1)}
            if mode_name == "box":
                counts = voxel_sample_counts(torch, tuple(frames.shape), poses, wl.calib, wl.origin, wl.spacing,
                                             wl.dims, pitch_f)
                nb_l = min(10, nl)
                byt = float(np.mean([box_reading_bytes(torch, counts, sl.probe_poses[k], wl.calib, wl.origin,
                                                       wl.spacing, wl.dims, W, H, pitch) for k in range(nb_l)]))
                ach = byt / (ms * 1e-3) / 1e9
                literal_res["box"]["roofline"] = {
                    "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "algo_bytes_per_launch": round(byt),
                    "bytes_basis": f"first {nb_l} slices: samples (4 B) and CSR offsets (8 B) of the distinct "
                                   "voxels in reach, 4 B output per pixel"}
                del counts
            if mode_name == "tent":
                a, b = lit_out.double(), outs[:nl].double()
                both = torch.isfinite(a) & torch.isfinite(b)
                d = (a - b).abs()[both]
                literal_res["tent_vs_binned_fp32"] = {
                    "bin_tol_deg": float(dare.default_params().bin_tol_deg), "pixels": int(both.sum().item()),
                    "max_abs_grey": round(float(d.max().item()) if d.numel() else 0.0, 4),
                    "mean_abs_grey": round(float(d.mean().item()) if d.numel() else 0.0, 5),
                    "nan_mask_mismatch": int((torch.isfinite(a) != torch.isfinite(b)).sum().item())}
                # the binning tolerance: the same comparison with the grid binned at smaller delta,
                # and the largest delta at which the worst pixel differs by less than one grey level
                sweep_d = []
                tmp = torch.empty((H, W), dtype=torch.float32, device=dev)
                for tol in (5.0, 3.0, 2.0, 1.0, 0.5):
                    v_d = dare.Volume(geom, dare.default_params(bin_tol_deg=tol), dtype="f32", bricks=nb * 64)
                    st_d = v_d.reconstruct(frames, poses, pitch_f)
                    worst, tot, cnt, mism = 0.0, 0.0, 0, 0
                    for k in range(nl):
                        v_d.reslice(sl.probe_poses[k], W, H, pitch, out=tmp)
                        a_k, b_k = lit_out[k].double(), tmp.double()
                        both_k = torch.isfinite(a_k) & torch.isfinite(b_k)
                        d_k = (a_k - b_k).abs()[both_k]
                        if d_k.numel():
                            worst = max(worst, float(d_k.max().item()))
                            tot += float(d_k.sum().item())
                            cnt += int(d_k.numel())
                        mism += int((torch.isfinite(a_k) != torch.isfinite(b_k)).sum().item())
                    inf_d = v_d.info()
                    sweep_d.append({"bin_tol_deg": tol, "bins": int(inf_d.bins), "saturated": bool(inf_d.saturated),
                                    "max_abs_grey": round(worst, 4), "mean_abs_grey": round(tot / max(cnt, 1), 5),
                                    "nan_mask_mismatch": mism})
                    del v_d, st_d
                below = [e["bin_tol_deg"] for e in sweep_d if e["max_abs_grey"] < 1.0]
                literal_res["tent_vs_binned_by_bin_tol"] = sweep_d
                literal_res["largest_bin_tol_below_one_grey"] = max(below) if below else None
                del tmp
            log(f"per-sample store {mode_name}: {ms * 1e3:.1f} us per 512^2 slice ({n_samples} samples)")
        log(f"per-sample store: {literal_res}")
        del store, lit_out
        torch.cuda.synchronize()

    # ---- evaluation protocol (Sec. 2.2, Sec. 3): NCC and SSIM of reslices at a secondary sweep's
    # poses against its frames, the volume built from a different, misregistered sweep set; config 1
    # (two sweeps tilted +-20 deg, secondary at +10 deg) and config 2 (three azimuths, secondary at
    # 10 deg azimuth)
    evaluation = None
    if not args.no_forms and not args.no_literal:
        evaluation = {"config1": run_evaluation(dare, torch, synth, 1, None, log),
                      "config2": run_evaluation(dare, torch, synth, 2, nb * 40, log)}

    # ---- curvilinear probes (binning per column sector) and out-of-core bricks
    curvilinear, out_of_core = None, None
    if not args.no_forms and not args.no_extras:
        curvilinear = run_fan(dare, torch, synth, dev, nb * 40, log)
        out_of_core = run_out_of_core(dare, torch, geom, prm, frames, poses, pitch_f, int(info.bricks_used),
                                      1e3 * float(np.median(recon_times)), log)

    # GPU results on the oracle's sample (the first cpu_slices slices in every storage form), kept
    # before the serving form frees the volumes
    ncs = min(args.cpu_slices, len(specs))
    oracle_in, oracle_meta = {}, {}
    if not args.no_cpu_baseline:
        c2_gpu = {"fp32": outs[:ncs].cpu().numpy()}
        for name, v in form_vols.items():
            o = torch.empty((ncs, H, W), dtype=torch.float32, device=dev)
            for k in range(ncs):
                reslice(v.handle, spec_refs[k], ct.c_void_p(o[k].data_ptr()), sh)
            torch.cuda.synchronize()
            c2_gpu[name] = o.cpu().numpy()
        oracle_in.update(c2_frames=frames.cpu().numpy(), c2_poses=np.ascontiguousarray(wl.sweep.probe_poses),
                         c2_slices=np.ascontiguousarray(np.asarray(sl.probe_poses[:ncs])))
        for name, a in c2_gpu.items():
            oracle_in[f"c2_gpu_{name}"] = a
        oracle_meta["config2"] = {
            "frames": "c2_frames", "poses": "c2_poses", "slices": "c2_slices",
            "calib": np.asarray(wl.calib, np.float64).ravel().tolist(), "origin": [float(x) for x in wl.origin],
            "spacing": float(wl.spacing), "dims": [int(x) for x in wl.dims], "pitch": [float(x) for x in pitch_f],
            "W": W, "H": H, "slice_pitch": [float(x) for x in pitch], "gpu": {n_: f"c2_gpu_{n_}" for n_ in c2_gpu}}
        del c2_gpu

    # ---- serving form: continuous batching under console load
    serving, roofline_served, served_sample = None, None, None
    if not args.no_serving:
        form_vols.clear()
        del outs
        torch.cuda.empty_cache()
        serving, roofline_served, served_sample = run_serving(
            dare, torch, synth, args.serving_seconds, args.saturation_seconds, args.budget_seconds, log,
            sample_cap=args.served_sample)

    # ---- streaming form: compounding through the server while consoles reslice
    streaming = None
    if not args.no_streaming:
        streaming = run_streaming(dare, torch, synth, args.streaming_seconds, log)
        log(f"streaming: {streaming}")

    # ---- the FP64 oracle on the host cores (a child process with a pool of workers): config 2's
    # compounding and first slices (the timed baseline), config 1 in full, config 3's slices on the
    # config-1 grid in every storage form, and the sample of served results
    cpu_baseline, precision = None, None
    if not args.no_cpu_baseline:
        wl1 = synth.config1()
        fr1 = wl1.render(dev)
        poses1 = torch.from_numpy(np.ascontiguousarray(wl1.sweep.probe_poses, np.float32)).to(dev)
        geom1 = dare.make_geometry(wl1.origin, wl1.spacing, wl1.dims, wl1.calib)
        nb1 = 1
        for d in wl1.dims:
            nb1 *= (d + 7) // 8
        sl1 = wl1.slices
        n3 = max(1, args.config3_slices)
        sl3 = synth.config3_slices(wl1, n_slices=n3, n_near=int(round(0.8 * n3)))
        c3_keys = []
        for dt in ("f32", "bf16", "f16", "fp8"):
            key = "fp32" if dt == "f32" else dt
            v1 = dare.Volume(geom1, dare.default_params(), dtype=dt, bricks=nb1 * 8)
            v1.reconstruct(fr1, poses1, wl1.sweep.pitch)
            if dt == "f32":
                oracle_in["c1_gpu_fp32"] = np.stack(
                    [v1.reslice(P, sl1.width, sl1.height, sl1.pitch).cpu().numpy() for P in sl1.probe_poses])
            o3 = torch.empty((n3, sl3.height, sl3.width), dtype=torch.float32, device=dev)
            for k in range(n3):
                v1.reslice(sl3.probe_poses[k], sl3.width, sl3.height, sl3.pitch, out=o3[k])
            torch.cuda.synchronize()
            oracle_in[f"c3_gpu_{key}"] = o3.cpu().numpy()
            c3_keys.append(key)
            del v1, o3
        oracle_in.update(c1_frames=fr1.cpu().numpy(), c1_poses=np.ascontiguousarray(wl1.sweep.probe_poses),
                         c1_slices=np.ascontiguousarray(np.asarray(sl1.probe_poses)),
                         c3_slices=np.ascontiguousarray(np.asarray(sl3.probe_poses)))
        oracle_meta["config1"] = {
            "frames": "c1_frames", "poses": "c1_poses", "slices": "c1_slices",
            "calib": np.asarray(wl1.calib, np.float64).ravel().tolist(), "origin": [float(x) for x in wl1.origin],
            "spacing": float(wl1.spacing), "dims": [int(x) for x in wl1.dims],
            "pitch": [float(x) for x in wl1.sweep.pitch], "W": sl1.width, "H": sl1.height,
            "slice_pitch": [float(x) for x in sl1.pitch], "gpu": {"fp32": "c1_gpu_fp32"}}
        oracle_meta["config3"] = {"slices": "c3_slices", "W": sl3.width, "H": sl3.height,
                                  "slice_pitch": [float(x) for x in sl3.pitch],
                                  "gpu": {k: f"c3_gpu_{k}" for k in c3_keys}}
        del fr1, poses1
        if served_sample and served_sample["items"]:
            oracle_meta["served"] = []
            for vi, (ws_, fr_s) in enumerate(zip(served_sample["workloads"], served_sample["frames"])):
                items = [it for it in served_sample["items"] if it[0] == vi]
                offs = np.cumsum([0] + [it[2] * it[2] for it in items])[:-1].astype(np.int64)
                pre = f"s{vi}_"
                oracle_in.update({
                    pre + "frames": fr_s, pre + "poses": np.ascontiguousarray(ws_.sweep.probe_poses),
                    pre + "P": np.asarray([np.asarray(it[1], np.float64) for it in items], np.float64).reshape(-1, 4, 4),
                    pre + "n": np.asarray([it[2] for it in items], np.int64),
                    pre + "pitch": np.asarray([it[3] for it in items], np.float64).reshape(-1, 2),
                    pre + "off": offs,
                    pre + "res": (np.concatenate([it[4].ravel() for it in items]) if items
                                  else np.zeros(0, np.float32)).astype(np.float32)})
                oracle_meta["served"].append({
                    "frames": pre + "frames", "poses": pre + "poses",
                    "calib": np.asarray(ws_.calib, np.float64).ravel().tolist(),
                    "origin": [float(x) for x in ws_.origin], "spacing": float(ws_.spacing),
                    "dims": [int(x) for x in ws_.dims], "pitch": [float(x) for x in ws_.sweep.pitch],
                    "req_P": pre + "P", "req_n": pre + "n", "req_pitch": pre + "pitch", "req_off": pre + "off",
                    "results": pre + "res"})
        aff, quota, workers = cpu_share()
        oracle_meta["workers"] = workers
        log(f"oracle child: {workers} workers (affinity {aff} CPUs, cgroup quota {quota}), "
            f"{sum(a.nbytes for a in oracle_in.values()) / 1e9:.2f} GB of inputs")
        t_child = time.perf_counter()
        ores = run_oracle_child(oracle_meta, oracle_in, log)
        oracle_in.clear()
        log(f"oracle child finished in {time.perf_counter() - t_child:.1f} s")
        if ores and "config2" in ores:
            c2 = ores["config2"]
            cpu_baseline = {
                "value": c2["pool_Mpx_s"], "unit": "Mpixel/s", "cores": c2["pool_workers"], "kind": "oracle",
                "sample": f"FP64 NumPy oracle reslicing the first {c2['slices']} of the {len(specs)} 512x512 "
                          f"config-2 slices over a pool of {c2['pool_workers']} worker processes "
                          f"({c2['pool_seconds']} s) on its own grid, compounded from all {F} frames in "
                          f"{c2['compound_seconds']} s on one core (not in the rate)",
                "single_core": {"Mpx_s": c2["single_core_Mpx_s"],
                                "seconds_per_slice": c2["single_core_seconds_per_slice"]},
                "host_cpus": {"affinity": aff, "cgroup_quota": quota, "pool_workers": workers},
                "compound_seconds": c2["compound_seconds"],
                "gpu_error_vs_fp64_on_sample": c2["errors"],
                "config1": ores.get("config1")}
            recon_touched = c2.get("touched_bin_voxels")
        else:
            recon_touched = None
        if ores and "config3" in ores:
            precision = dict(ores["config3"], slice_px=[sl3.width, sl3.height], pitch_mm=list(sl3.pitch),
                             grid="config-1 volume, 64^3 @0.5 mm")
        if ores and "served" in ores and serving is not None:
            serving["oracle_sample"] = dict(ores["served"], basis=(
                f"a seeded 1% of the offered run's requests to the 128^3 and 256^3 volumes "
                f"(at most {args.served_sample}), each compared in full with the FP64 oracle on the FP64 grid"))
    else:
        recon_touched = None

    # ---- reconstruction roofline: 1 B read per input pixel, a read-modify-write of the 4 B sum and
    # 4 B count per in-grid pixel (16 B), and per touched (bin, voxel) the 8 B read of the
    # accumulators and the FP32 pair written once
    recon_med = float(np.median(recon_times))
    recon_roof = None
    if recon_touched is not None:
        algo_r = F * Wf * Hf + 16 * in_grid_px + recon_touched * (8 + PAIR_BYTES["f32"])
        ach_r = algo_r / recon_med / 1e9
        kacc = counters.get("k_accumulate")
        recon_roof = {"bound": "hbm", "achieved": round(ach_r, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(ach_r / HBM_PEAK_GBS, 4), "algo_bytes": int(algo_r),
                      "in_grid_px": int(in_grid_px), "touched_bin_voxels": int(recon_touched),
                      "traffic": kacc.get("hbm_bytes_per_launch") if kacc else None,
                      "basis": "whole dare_reconstruct_frames call (host-timed median) against the compulsory "
                               "bytes; touched (bin, voxel) count from the oracle's grid"}

    result = {
        "metric": "reslice Mpixel/s + p50/p99 latency, served BF16 vs plain FP32; % HBM roofline",
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "config2: 256^3 grid @0.125 mm from 3x600 frames 256^2 (1 mm/2 deg jitter); "
                               f"{len(specs)} slices 512^2 @0.0625 mm, one dare_reslice launch per slice, radius 1",
                   "grid": list(wl.dims), "voxel_mm": wl.spacing, "frames": int(F), "slices": len(specs),
                   "slice_px": [W, H], "storage": "fp32", "positions": "f64", "bins": int(info.bins),
                   "bricks_used": int(info.bricks_used), "unassigned_fraction": round(nan_frac, 4)},
        "roofline": roofline,
        "roofline_batched": roofline_batched or None,
        "two_streams": concurrent,
        "latency_ms": {"fp32": lat32, **({"bf16": forms["bf16"]["latency_ms"]} if "bf16" in forms else {})},
        "roofline_served": roofline_served,
        "reconstruct": {"frames": int(F), "frame_px": [Wf, Hf], "median_ms": round(1e3 * recon_med, 3),
                        "frames_per_s": round(F / recon_med, 1),
                        "input_Mpx_s": round(F * Wf * Hf / recon_med / 1e6, 1),
                        "roofline": recon_roof},
        "precision_config3": precision,
        "forms": forms,
        "radius_sweep": radius,
        "per_sample_store": literal_res,
        "evaluation": evaluation,
        "curvilinear": curvilinear,
        "out_of_core": out_of_core,
        "serving": serving,
        "streaming": streaming,
        "cpu_baseline": cpu_baseline,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
