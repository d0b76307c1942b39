"""Host checks of the evaluation protocol's synthetic inputs: per-sweep tracking offsets are
rigid, applied sweep by sweep, and the secondary sweep is a different acquisition."""
import numpy as np

import synth


def _rigid(M):
    R = M[:3, :3]
    return np.allclose(R.T @ R, np.eye(3), atol=1e-12) and abs(np.linalg.det(R) - 1.0) < 1e-12


def test_tracking_offsets_are_rigid_and_seeded():
    c = np.array([10.0, 20.0, 30.0])
    a = synth.tracking_offsets(5, 3, c, 0.5, 1.0)
    b = synth.tracking_offsets(5, 3, c, 0.5, 1.0)
    assert all(_rigid(M) for M in a)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    # zero offsets are the identity
    z = synth.tracking_offsets(5, 2, c, 0.0, 0.0)
    assert all(np.allclose(M, np.eye(4)) for M in z)


def test_tracked_poses_move_each_sweep_by_its_own_offset():
    p = synth.eval_pair(1)
    sw = p.initial.sweep
    P = np.asarray(sw.probe_poses, np.float64)
    T = p.initial_tracked.astype(np.float64)
    for k in range(int(sw.sweep_id.max()) + 1):
        f = np.nonzero(sw.sweep_id == k)[0]
        # one rigid transform per sweep: T_f P_f^-1 is the same for every frame of sweep k
        M = T[f[0]] @ np.linalg.inv(P[f[0]])
        for g in f[1:]:
            assert np.allclose(T[g] @ np.linalg.inv(P[g]), M, atol=1e-4)
        assert not np.allclose(M, np.eye(4), atol=1e-3)
    assert len(p.offsets_mm_deg) == int(sw.sweep_id.max()) + 2


def test_secondary_sweep_is_a_different_acquisition():
    for cfg, tilt in ((1, 10.0), (2, None)):
        p = synth.eval_pair(cfg)
        assert p.secondary.frame_seed != p.initial.frame_seed
        sec = np.asarray(p.secondary.sweep.image_poses)
        ini = np.asarray(p.initial.sweep.image_poses)
        # the secondary's in-plane axis differs from every initial sweep's
        lat_s = sec[:, :3, 0].mean(0)
        for k in range(int(p.initial.sweep.sweep_id.max()) + 1):
            lat_k = ini[p.initial.sweep.sweep_id == k][:, :3, 0].mean(0)
            cos = abs(lat_s @ lat_k) / (np.linalg.norm(lat_s) * np.linalg.norm(lat_k))
            assert cos < 0.9999
        if tilt is not None:
            # config 1: +10 deg, between the +20 and -20 deg sweeps (10 and 30 deg away)
            ang = sorted(np.degrees(np.arccos(np.clip(
                [abs(lat_s @ ini[p.initial.sweep.sweep_id == k][:, :3, 0].mean(0))
                 / (np.linalg.norm(lat_s) * np.linalg.norm(ini[p.initial.sweep.sweep_id == k][:, :3, 0].mean(0)))
                 for k in (0, 1)], -1, 1))))
            assert abs(ang[0] - 10.0) < 0.5 and abs(ang[1] - 30.0) < 0.5
