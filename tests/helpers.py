"""Shared test helpers: pose builders, random grids, fixtures on disk."""
from __future__ import annotations

import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return rows


def rodrigues(axis, ang_rad):
    k = np.asarray(axis, np.float64)
    k = k / np.linalg.norm(k)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]], np.float64)
    return np.eye(3) + math.sin(ang_rad) * K + (1 - math.cos(ang_rad)) * (K @ K)


def pose_from_axes(x_axis, normal, origin):
    """4x4 image pose with lateral ``x_axis``, plane normal ``normal`` (beam = normal x lateral)."""
    x = np.asarray(x_axis, np.float64)
    n = np.asarray(normal, np.float64)
    x = x / np.linalg.norm(x)
    n = n - (n @ x) * x
    n = n / np.linalg.norm(n)
    beam = np.cross(n, x)            # so that x cross beam = n
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = x, beam, n, origin
    return T


def random_grid(rng, K, dims, p_empty=0.3, max_count=5):
    """Random integer sums/counts per (bin, voxel), with empty voxels."""
    nx, ny, nz = dims
    C = rng.integers(1, max_count + 1, size=(K, nz, ny, nx))
    C = np.where(rng.random((K, nz, ny, nx)) < p_empty, 0, C)
    S = np.where(C > 0, rng.integers(0, 256, size=C.shape) * C + rng.integers(0, 1, size=C.shape), 0)
    # sums need not be multiples of the count: add a random remainder below the count
    S = S + np.where(C > 0, rng.integers(0, 1 << 30, size=C.shape) % np.maximum(C, 1), 0)
    return S.astype(np.int64), C.astype(np.int64)


def random_unit(rng):
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def random_reps(rng, K):
    """K random orthonormal (normal, x) pairs as representative orientations."""
    rn, rx = [], []
    for _ in range(K):
        n = random_unit(rng)
        x = random_unit(rng)
        x = x - (x @ n) * n
        x /= np.linalg.norm(x)
        rn.append(n)
        rx.append(x)
    return np.array(rn), np.array(rx)
