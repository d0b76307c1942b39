"""FP64 CPU oracle for directionality-aware reconstruction and reslicing (DARE).

TEST INFRASTRUCTURE ONLY.  Nothing in the library path imports, links or runs
this package; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the GPU path.

What it computes, and where the paper defines it:
  geometry  -- pose composition and pixel positions (Sec. 2.1, "Volume
               reconstruction": images are transformed to their poses);
               bounding box of the collected frames (same passage).
  bins      -- the per-volume codebook of acquisition orientations that stands
               in for the per-sample quaternion list (same passage, Fig. 1).
  compound  -- nearest-voxel voxelization into per-(bin, voxel) sums and counts
               (same passage: images "voxelized into a 3D grid").
  quant     -- the reduced-precision storage forms of the directional data.
  reslice   -- the reslice of Sec. 2.1 "Reslicing": Eq. 1 (alignment dot
               products), the angular thresholds and Eq. 2 (exponential
               weights, k_normal = 10, k_inplane = 5, 25 and 15 degrees), the
               cubic neighbourhood of a fixed interpolation distance with
               weighting by distance (Fig. 2 caption), the weighted average and
               the "unassigned" rule.
  literal   -- the same reslice over every individual sample with its own
               acquisition orientation, written separately with explicit loops
               for tiny inputs (the paper's flat per-sample storage).
  metrics   -- the evaluation's image similarity of a reslice against the
               acquired frame at its pose (Sec. 3: NCC and SSIM).

Every floating-point step is FP64 unless a storage form fixes another
precision.  Where the paper is silent the readings are stated in each module.
"""

from . import geometry, bins, compound, quant, reslice, literal, metrics  # noqa: F401
