"""FP64 CPU oracle for the compositional multi-octree voxel renderer.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It is a plain, slow,
brute-force statement of what the renderer computes, written from the paper
(DrivingVoxels, arXiv 2606.23031):

* scene = one static world-frame octree plus one local-frame octree per rigid
  actor posed at the view's timestamp (Sec. 3.1-3.2);
* every ray is intersected with every leaf of every octree; actor boxes split
  the ray into background and asset segments (Sec. 3.4, App. A, Alg. 1);
* each clipped piece is integrated with trilinear raw density, exp-linear
  activation and alpha compositing, carrying (C, D, N, T) front to back
  (Sec. 3.4), then composited over the background colour (Eq. 2);
* the adjoint is the hand-derived reverse pass of the same sum.

Readings of passages the paper leaves open (integration rule, activation
constant, SH convention, depth/normal definitions, ownership of overlapping
boxes, camera model, ordering and binning contracts) are listed in the
design notes; each function names the reading it implements.

It shares no code with the HIP path and imports nothing from it.
"""
from . import geometry, sh, field, render, adjoint, binning, prior, features

__all__ = ["geometry", "sh", "field", "render", "adjoint", "binning",
           "prior", "features"]
