"""Codebook of acquisition orientations (direction bins), FP64.

Sec. 2.1 "Volume reconstruction" (and Fig. 1): each grid location keeps its
intensities together with their acquisition orientations.  A linear array
images a whole frame from one orientation, so the orientation is a property of
the frame.  Reading: frames are grouped, in the order given, by leader
clustering with tolerance delta:

  * frame f joins bin b iff n_f . n_b >= cos(delta) and |x_f . x_b| >= cos(delta);
    among qualifying bins it takes the one maximising n_f . n_b + |x_f . x_b|,
    ties to the lowest index;
  * if none qualifies and fewer than K_max bins exist, a new bin is created
    whose representative is the frame's own (n_f, x_f);
  * otherwise the frame goes to the maximiser over all bins and the codebook is
    reported saturated.

Representatives never change.  With delta = 0 every distinct orientation has
its own bin, and binned reslicing equals the per-sample form.  Dot products
are summed left to right, (a0 b0 + a1 b1) + a2 b2.
"""
from __future__ import annotations

import math

import numpy as np


def dot3(a, b) -> float:
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


class Codebook:
    def __init__(self, tol_deg: float, max_bins: int):
        self.cos_tol = math.cos(math.radians(tol_deg))
        self.max_bins = int(max_bins)
        self.rep_n: list = []
        self.rep_x: list = []
        self.saturated = False

    @property
    def K(self) -> int:
        return len(self.rep_n)

    def assign(self, nhat: np.ndarray, xhat: np.ndarray) -> np.ndarray:
        """Assign frames (F,3)+(F,3) in order; returns bin index per frame."""
        out = np.empty(len(nhat), dtype=np.int64)
        for f in range(len(nhat)):
            n_f = [float(v) for v in nhat[f]]
            x_f = [float(v) for v in xhat[f]]
            best, best_s = -1, -math.inf
            any_best, any_s = -1, -math.inf
            for b in range(self.K):
                dn = dot3(n_f, self.rep_n[b])
                di = abs(dot3(x_f, self.rep_x[b]))
                s = dn + di
                if s > any_s:
                    any_best, any_s = b, s
                if dn >= self.cos_tol and di >= self.cos_tol and s > best_s:
                    best, best_s = b, s
            if best < 0:
                if self.K < self.max_bins:
                    self.rep_n.append(n_f)
                    self.rep_x.append(x_f)
                    best = self.K - 1
                else:
                    best = any_best
                    self.saturated = True
            out[f] = best
        return out

    def arrays(self):
        return np.array(self.rep_n, dtype=np.float64).reshape(-1, 3), \
            np.array(self.rep_x, dtype=np.float64).reshape(-1, 3)
