"""Seeded phantom of spheres and planes in a cube of side L.

Structures live in grid-local millimetres (voxel (0,0,0) centre at the local
origin); the world frame adds ``WORLD_OFFSET_MM``.  Each surface echoes with
intensity I * |cos(theta)|^e, theta being the angle between the beam and the
surface normal, inside a shell of half-thickness ``shell_mm`` around it.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Phantom:
    L: float                      # cube side in mm
    shell_mm: float               # echo shell half-thickness (one voxel)
    sph_c: np.ndarray             # (S,3) sphere centres, local mm
    sph_r: np.ndarray             # (S,) radii
    sph_i: np.ndarray             # (S,) intensities in [0.6, 1]
    pl_n: np.ndarray              # (Q,3) unit plane normals
    pl_q: np.ndarray              # (Q,3) a point on each plane, local mm
    pl_i: np.ndarray              # (Q,) intensities
    exponent: float = 4.0         # |cos|^exponent directivity (0 = isotropic)
    speckle_sigma: float = 0.3    # Rayleigh sigma of the additive speckle (0 = none)
    meta: dict = field(default_factory=dict)


def make_phantom(seed: int, L: float, n_sph: int, n_pl: int, shell_mm: float,
                 exponent: float = 4.0, speckle_sigma: float = 0.3) -> Phantom:
    rng = np.random.Generator(np.random.PCG64(seed))
    sph_c = rng.uniform(0.15 * L, 0.85 * L, size=(n_sph, 3))
    sph_r = rng.uniform(0.04 * L, 0.15 * L, size=n_sph)
    sph_i = rng.uniform(0.6, 1.0, size=n_sph)
    nrm = rng.standard_normal((n_pl, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    pl_q = rng.uniform(0.3 * L, 0.7 * L, size=(n_pl, 3))
    pl_i = rng.uniform(0.6, 1.0, size=n_pl)
    return Phantom(L=L, shell_mm=shell_mm, sph_c=sph_c, sph_r=sph_r, sph_i=sph_i,
                   pl_n=nrm, pl_q=pl_q, pl_i=pl_i, exponent=exponent,
                   speckle_sigma=speckle_sigma, meta={"seed": seed})
