"""CPU oracle for the dense RGB-D-inertial tracking step (TEST INFRASTRUCTURE).

This package is a plain, slow, obviously-correct implementation of what the
tracking step computes, written from the paper (Laidlow et al., "Dense
RGB-D-Inertial SLAM with Map Deformations", Section IV).  It exists only to
check the GPU library: only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import it.  The product path never calls it
and shares no code with it.

Two layers:

* a **mask layer** (``pyramid``, ``association``) that reproduces, in NumPy
  float32 with one rounding per operation and no fused multiply-adds, the
  exact FP32 operation sequence that decides pyramid values, pixel validity and
  projective data association, so that association masks and inlier counts
  can be compared bit for bit;
* a **value layer** in float64 (``residuals``, ``imu``, ``solve``, ``track``)
  that evaluates residuals with per-pixel 12-parameter Jacobians in the world
  frame, preintegrates the IMU by the exact zero-order-hold recursion, takes
  IMU-factor Jacobians and noise propagation by finite differences, and runs
  the Gauss-Newton solve and Schur-complement marginalisation with library
  linear algebra.

Every function cites the passage of the paper it follows, or the reading of
the paper it implements where the paper is silent.
"""
from . import lie, pyramid, association, residuals, imu, solve, track  # noqa: F401
