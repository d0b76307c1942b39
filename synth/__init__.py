"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package simulates an acquisition: a phantom of spheres and planes with a
beam-angle dependent echo, tracked sweeps of a linear array (or of a curvilinear
probe, ``fan_config``), their 2D uint8 frames,
and reslice poses.  It holds none of the reconstruction or reslicing
arithmetic; both the FP64 oracle and the GPU path receive what it produces as
plain arrays.

Random parameters (structures, poses, jitter) come from NumPy's PCG64 seeded
per configuration; per-pixel speckle comes from a torch generator on the device
the frames are rendered on.
"""

from .poses import (  # noqa: F401
    rot_x, rot_y, rot_z, rotvec_to_matrix, random_rotation, make_calibration,
    image_pose, probe_pose_from_image_pose, WORLD_OFFSET_MM,
)
from .phantom import Phantom, make_phantom  # noqa: F401
from .sweeps import (  # noqa: F401
    Sweep, linear_tilted_sweeps, azimuth_sweeps, random_walk_sweep, slice_poses, SliceSet,
)
from .render import render_frames  # noqa: F401
from .configs import (  # noqa: F401
    Workload, config1, config2, config3_slices, config5, serving_volume, tiny_workload, fan_beams, fan_config, fan_config2,
    EvalPair, eval_pair, tracking_offsets, tracked,
)
