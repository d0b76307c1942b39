"""GPU tests of the serving form: continuous batching through the C ABI.

Every request served inside a mix of requests (other consoles, sizes, poses,
volumes) must equal the same request resliced alone with dare_reslice, bit for
bit; a small result budget forces admission queueing without losing or
duplicating requests.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from gpu_helpers import make_volume, note, oracle_grid, upload_grid
from oracle.reslice import Params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2605_26325_amd as dare
    wl = synth.config1()
    wl.render("cpu")
    g = oracle_grid(wl, wl.frames.numpy(), Params())
    vols = []
    for dt in ("bf16", "bf16"):
        v = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(), dtype=dt)
        upload_grid(v, g.S, g.C, *g.codebook.arrays())
        vols.append(v)
    return dare, torch, wl, vols


def _requests(wl, n, seed):
    rng = np.random.default_rng(seed)
    sizes = [(128, 128, (0.25, 0.25)), (37, 23, (0.6, 0.7)), (200, 90, (0.16, 0.3)), (64, 65, (0.5, 0.5)),
             (16, 16, (1.0, 1.0)), (96, 160, (0.3, 0.2))]
    out = []
    for k in range(n):
        W, H, pitch = sizes[int(rng.integers(len(sizes)))]
        P = wl.slices.probe_poses[int(rng.integers(len(wl.slices.probe_poses)))]
        out.append((int(rng.integers(2)), P, W, H, pitch))
    return out


def _alone(dare, torch, vols, reqs):
    res = []
    for vi, P, W, H, pitch in reqs:
        o = torch.full((H, W), -3.0, device="cuda")
        dare.dare_reslice(vols[vi], dare.make_spec(P, W, H, pitch), o)
        res.append(o)
    torch.cuda.synchronize()
    return [r.cpu().numpy() for r in res]


def _serve(dare, torch, vols, reqs, arena_bytes, **cfg):
    srv = dare.Server(arena_bytes, **cfg)
    ids = [srv.add_volume(v) for v in vols]
    outs = [torch.full((H, W), -5.0, dtype=torch.float32, pin_memory=True) for (_, _, W, H, _) in reqs]
    tickets = []
    for (vi, P, W, H, pitch), o in zip(reqs, outs):
        t = None
        while t is None:                 # queue full: wait for the scheduler to admit some
            t = srv.submit(ids[vi], P, W, H, pitch, o)
        tickets.append(t)
    srv.drain()
    times = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    return [o.numpy() for o in outs], times, st


@pytest.mark.parametrize("graphs,streams", [(1, 3), (0, 2), (1, 1)])
def test_served_equals_alone(env, graphs, streams):
    dare, torch, wl, vols = env
    note(f"server graphs={graphs} streams={streams}")
    reqs = _requests(wl, 48, seed=streams + 10 * graphs)
    ref = _alone(dare, torch, vols, reqs)
    got, times, st = _serve(dare, torch, vols, reqs, 64 << 20, use_graphs=graphs, n_streams=streams,
                            max_tick_requests=8)
    for k in range(len(reqs)):
        assert np.array_equal(got[k], ref[k], equal_nan=True), k
    assert all(t is not None for t in times)
    for t in times:
        assert t.t_submit <= t.t_admit <= t.t_launch <= t.t_host_done
    assert st.completed == len(reqs) and st.submitted == len(reqs) and st.ticks >= len(reqs) // 8


def test_small_budget_queues_and_completes(env):
    dare, torch, wl, vols = env
    note("server with room for about two results at a time")
    reqs = _requests(wl, 30, seed=99)
    ref = _alone(dare, torch, vols, reqs)
    cfg = dict(n_streams=2, max_tick_requests=4, max_tick_pixels=1 << 16, max_queue=64)
    largest = max(W * H for (_, _, W, H, _) in reqs) * 4
    arena = _table_bytes(dare, cfg, vols[0]) + 2 * largest + 4096
    got, times, st = _serve(dare, torch, vols, reqs, arena, **cfg)
    for k in range(len(reqs)):
        assert np.array_equal(got[k], ref[k], equal_nan=True), k
    total = sum(W * H * 4 for (_, _, W, H, _) in reqs)
    n_done, n_ticks = int(st.completed), int(st.ticks)
    assert n_done == len(reqs)
    # no more than the result budget can be in flight: at least total / budget ticks
    assert n_ticks >= total // (2 * largest + 4096), (n_ticks, total, largest)


def _table_bytes(dare, cfg, vol):
    """Smallest arena in which a server takes its first volume (the streams' workspaces are laid
    out then), found by bisection."""
    lo, hi = 1 << 10, 1 << 28
    while lo < hi:
        mid = (lo + hi) // 2
        try:
            s = dare.Server(mid, **cfg)
            try:
                s.add_volume(vol)
                hi = mid
            except dare.DareError:
                lo = mid + 1
            s.close()
        except dare.DareError:
            lo = mid + 1
    return lo


def test_submit_rejects_what_can_never_fit(env):
    dare, torch, wl, vols = env
    note("server rejects oversized requests")
    cfg = dict(n_streams=1, max_tick_requests=2, max_tick_pixels=4096)
    srv = dare.Server(_table_bytes(dare, cfg, vols[0]) + 64 * 64 * 4 + 1024, **cfg)
    vid = srv.add_volume(vols[0])
    big = torch.empty((128, 128), dtype=torch.float32, pin_memory=True)
    with pytest.raises(dare.DareError) as e:
        srv.submit(vid, wl.slices.probe_poses[0], 128, 128, (0.25, 0.25), big)
    assert e.value.status == dare.ERR_INVALID_ARG
    ok = torch.empty((32, 32), dtype=torch.float32, pin_memory=True)
    t = srv.submit(vid, wl.slices.probe_poses[0], 32, 32, (1.0, 1.0), ok)
    srv.drain()
    assert srv.poll(t) is not None
    # a second volume with another storage dtype cannot join this server
    other = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(), dtype="f32")
    with pytest.raises(dare.DareError):
        srv.add_volume(other)
    srv.close()


def test_grouped_submit_and_poll(env):
    dare, torch, wl, vols = env
    note("server grouped submit_many / poll_many with waiting")
    reqs = _requests(wl, 40, seed=7)
    ref = _alone(dare, torch, vols, reqs)
    srv = dare.Server(64 << 20, n_streams=2, max_tick_requests=16, max_queue=24)
    ids = [srv.add_volume(v) for v in vols]
    outs = [torch.full((H, W), -5.0, dtype=torch.float32, pin_memory=True) for (_, _, W, H, _) in reqs]
    specs = dare.spec_array([P for (_, P, _, _, _) in reqs], [W for (_, _, W, _, _) in reqs],
                            [H for (_, _, _, H, _) in reqs], [p for (_, _, _, _, p) in reqs])
    vid = np.array([ids[vi] for (vi, _, _, _, _) in reqs], np.int32)
    ptrs = np.array([o.data_ptr() for o in outs], np.uint64)
    tickets, k = [], 0
    while k < len(reqs):               # max_queue 24 < 40: some groups come back partly accepted
        t, st = srv.submit_many(vid[k:], specs[k:], ptrs[k:])
        assert st in (dare.OK, dare.ERR_QUEUE_FULL)
        tickets.extend(int(x) for x in t)
        k += len(t)
    assert len(tickets) == len(reqs) and len(set(tickets)) == len(reqs)
    left = np.array(tickets, np.uint64)
    seen = 0
    while len(left):
        states, times = srv.poll_many(left, wait_seconds=5.0)
        done = states != dare.ERR_NOT_READY
        assert done.any()              # the wait returns only once something finished
        assert (states[done] == dare.OK).all()
        assert (times["t_submit"][done] <= times["t_host_done"][done]).all()
        seen += int(done.sum())
        left = left[~done]
    assert seen == len(reqs)
    # retired tickets are unknown afterwards
    states, _ = srv.poll_many(np.array(tickets[:3], np.uint64))
    assert (states == dare.ERR_INVALID_ARG).all()
    srv.close()
    for k in range(len(reqs)):
        assert np.array_equal(outs[k].numpy(), ref[k], equal_nan=True), k


def test_frames_compounded_in_request_order(env):
    """Frames submitted to the server are compounded between the requests around them: every
    request equals the same request resliced alone on a volume compounded with exactly the
    frame batches submitted before it."""
    dare, torch, wl, _ = env
    note("server compounding frame batches between requests")
    frames = wl.frames.to("cuda").contiguous()
    poses = torch.from_numpy(np.ascontiguousarray(wl.sweep.probe_poses, np.float32)).to("cuda")
    nb = 4
    edges = np.linspace(0, frames.shape[0], nb + 1).astype(int)
    batches = [(frames[a:b].contiguous(), poses[a:b].contiguous()) for a, b in zip(edges[:-1], edges[1:])]
    groups = [_requests(wl, 6, seed=50 + k) for k in range(nb + 1)]
    served = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(), dtype="bf16")
    srv = dare.Server(64 << 20, n_streams=2, max_tick_requests=4)
    vid = srv.add_volume(served)
    outs, tickets, ftickets = [], [], []
    for k in range(nb + 1):
        row = []
        for (_, P, W, H, pitch) in groups[k]:
            o = torch.full((H, W), -5.0, dtype=torch.float32, pin_memory=True)
            t = srv.submit(vid, P, W, H, pitch, o)
            assert t is not None
            row.append(o)
            tickets.append(t)
        outs.append(row)
        if k < nb:
            ft = srv.submit_frames(vid, batches[k][0], batches[k][1], wl.sweep.pitch)
            assert ft is not None
            ftickets.append(ft)
    srv.drain()
    for ft in ftickets:
        st, tm = srv.poll_frames(ft)
        assert st == dare.OK and tm.t_submit <= tm.t_admit <= tm.t_host_done
    assert all(srv.poll(t) is not None for t in tickets)
    stats = srv.stats()
    assert stats.frames == frames.shape[0]
    srv.close()
    ref_vol = make_volume(wl.origin, wl.spacing, wl.dims, wl.calib, Params(), dtype="bf16")
    for k in range(nb + 1):
        if k > 0:
            ref_vol.reconstruct(batches[k - 1][0], batches[k - 1][1], wl.sweep.pitch)
        for (_, P, W, H, pitch), o in zip(groups[k], outs[k]):
            ref = torch.full((H, W), -9.0, device="cuda")
            dare.dare_reslice(ref_vol, dare.make_spec(P, W, H, pitch), ref)
            torch.cuda.synchronize()
            assert np.array_equal(o.numpy(), ref.cpu().numpy(), equal_nan=True), k
    # before any frame every result is unassigned
    assert all(np.isnan(o.numpy()).all() for o in outs[0])


def test_served_into_device_buffers_equals_alone(env):
    """Results delivered to device buffers (no host transfer) equal the requests resliced alone."""
    dare, torch, wl, vols = env
    note("server delivering into device buffers")
    reqs = _requests(wl, 24, seed=77)
    ref = _alone(dare, torch, vols, reqs)
    srv = dare.Server(64 << 20, n_streams=2, max_tick_requests=8)
    ids = [srv.add_volume(v) for v in vols]
    outs = [torch.full((H, W), -5.0, dtype=torch.float32, device="cuda") for (_, _, W, H, _) in reqs]
    tickets = []
    for (vi, P, W, H, pitch), o in zip(reqs, outs):
        t = None
        while t is None:
            t = srv.submit(ids[vi], P, W, H, pitch, o)
        tickets.append(t)
    srv.drain()
    assert all(srv.poll(t) is not None for t in tickets)
    srv.close()
    torch.cuda.synchronize()
    for k in range(len(reqs)):
        assert np.array_equal(outs[k].cpu().numpy(), ref[k], equal_nan=True), k
