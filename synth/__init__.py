"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This package only *produces* scenes, views and targets (leaf sets, corner
tables, SH coefficients, tracks, cameras).  It holds none of the renderer's
arithmetic: no ray casting through voxels, no activation, no compositing and
no SH evaluation.  Every draw is seeded with ``numpy.random.default_rng``.

Data model (plain dicts of numpy arrays, consumed by both sides):

octree
    ``root_min`` f64[3], ``root_size`` f64 (cube side), ``max_level`` int,
    ``level`` u8[N], ``ijk`` i32[3,N] (integer cell at that level),
    ``corner_idx`` i32[8,N] (corner m = mx + 2*my + 4*mz),
    ``corner_density`` f32[Nc] (raw densities), ``sh_degree`` int,
    ``sh`` f32[S,3,N] with S = (degree+1)^2,
    ``box_min``/``box_max`` f64[3] (actors only: the local interval box).
track
    ``t`` f64[K] keyframe times, ``yaw`` f64[K] (rad, about world +z),
    ``trans`` f64[K,3]; the pose is linear in t between keyframes.
view
    ``fx fy cx cy`` (pixels), ``W H`` (image), ``x0 y0 w h`` (rendered
    window), ``c2w`` f64[3,4] camera-to-world (OpenCV axes), ``t`` (s).
scene
    ``octrees`` (index 0 = static background), ``tracks`` (None for 0).
"""
from .octree import (make_octree, dedup_corners, random_subdivide,
                     leaves_from_grid)
from .configs import make_config, make_view, look_at_c2w

__all__ = ["make_octree", "dedup_corners", "random_subdivide",
           "leaves_from_grid", "make_config", "make_view", "look_at_c2w"]
