"""FP64 CPU oracle for the batched differentiable RGB-D-N Gaussian rasterizer
of CityGS-X (arXiv 2503.23044, Sec. 3.1-3.3, Eqs. 1 and 4-8).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.
It shares no code with the GPU library and imports nothing from it; the
GPU path never calls it.

It is a plain, slow restatement of what the rasterizer computes, in float64
NumPy, in the order the method defines it:

  anchors.py   a0 active-anchor selection (LoD by observation distance,
               Sec. 3.1; visible-voxel search, Sec. 3.3), a1 anchor decode
               (Sec. 3.2, Eq. 4) and its adjoint a10
  project.py   a2 EWA projection, SH colour, normal and plane distance
               (Eqs. 6-7 inputs) and its adjoint a9
  sh.py        real spherical-harmonic basis up to degree 3
  raster.py    a3-a5 tile binning and the (tile | depth) sort, a6
               front-to-back compositing of RGB / D / N / alpha and the
               unbiased depth (Eqs. 1, 5, 6, 7), a7 the L1 seed (Eq. 8),
               a8 the reverse-order compositing adjoint
  pipeline.py  the whole chain for explicit Gaussians and for voxel anchors
  bf16.py      bfloat16 rounding emulation of the decoder's feature input

Every discrete decision that gates membership (LoD, frustum, near plane,
depth key, pixel box) is taken in float64 with a fixed operation order that
the GPU path reproduces exactly.  Decisions that depend on continuous
values the GPU computes in float32 (radius ceiling, alpha >= 1/255,
transmittance cut-off, normal orientation, the 0.99 clamp, ReLU) are flagged
as fragile when the float64 margin is below a stated bound, and the tests
exclude (and count) outputs that such a decision touches.

Parity status: every function is pinned by closed forms, brute force,
library routines or finite differences in tests/test_oracle_*.py.  The
absolute constants that the paper leaves unstated (near plane, dilation,
guard band, alpha thresholds, SH convention) are fixed here by definition;
against the paper itself they are parity unpinned.
"""
from . import bf16, sh, anchors, project, raster, pipeline  # noqa: F401
