"""Rigid poses for the simulated tracker, probe calibration and slice requests.

Conventions (shared with the library's header):
  * An *image pose* T maps image millimetres (u, v, 0) to world millimetres;
    column 0 is the lateral axis, column 1 the depth (beam) axis, column 2 the
    elevation normal (column 0 x column 1), column 3 the position of pixel (0, 0).
  * A *probe pose* P maps probe coordinates to world (the tracker's output).
  * The calibration C maps image millimetres to probe coordinates, so that
    T = P . C.

Poses are 4x4 row-major float64 here; the tracker hands frames' probe poses
over as float32 (see ``probe_pose_from_image_pose``).
"""
from __future__ import annotations

import math

import numpy as np

# A tracker-scale world translation of the volume (about 2 m from the tracker
# origin).  All components are integers, hence exact in float32 and float64.
WORLD_OFFSET_MM = np.array([-850.0, 310.0, -1620.0])


def rot_x(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rot_y(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rot_z(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rotvec_to_matrix(rv) -> np.ndarray:
    """Rotation matrix of a rotation vector (axis * angle in radians)."""
    rv = np.asarray(rv, dtype=np.float64)
    ang = float(np.linalg.norm(rv))
    if ang == 0.0:
        return np.eye(3)
    k = rv / ang
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + math.sin(ang) * K + (1.0 - math.cos(ang)) * (K @ K)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation (normalised Gaussian quaternion)."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def make_calibration(width: int, pitch_x: float) -> np.ndarray:
    """Image-mm -> probe calibration of a linear array.

    The transducer is centred laterally (the middle pixel column sits on the
    probe axis); a small rotation and offset stand in for what a phantom-based
    calibration returns, so that composing with it is never the identity.
    """
    R = rotvec_to_matrix(np.deg2rad([0.35, -0.6, 0.9]))
    C = np.eye(4)
    C[:3, :3] = R
    C[:3, 3] = R @ np.array([-(width - 1) * pitch_x / 2.0, 0.0, 0.0]) + np.array([0.21, 1.3, -0.4])
    return C


def image_pose(center, lateral, beam, width: int, height: int, pitch) -> np.ndarray:
    """Image pose whose central pixel sits at ``center`` with the given axes."""
    a = np.asarray(lateral, np.float64)
    b = np.asarray(beam, np.float64)
    a = a / np.linalg.norm(a)
    b = b - (b @ a) * a
    b = b / np.linalg.norm(b)
    n = np.cross(a, b)
    T = np.eye(4)
    T[:3, 0] = a
    T[:3, 1] = b
    T[:3, 2] = n
    T[:3, 3] = (np.asarray(center, np.float64)
                - a * (width - 1) * pitch[0] / 2.0
                - b * (height - 1) * pitch[1] / 2.0)
    return T


def probe_pose_from_image_pose(T: np.ndarray, C: np.ndarray, dtype=np.float32) -> np.ndarray:
    """Probe pose P with P . C = T, rounded to the tracker's precision."""
    P = T @ np.linalg.inv(C)
    P[3, :] = (0.0, 0.0, 0.0, 1.0)
    return P.astype(dtype)
