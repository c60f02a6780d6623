// Device-side data layout shared by the kernels and the host library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/dslam.h"

namespace dslam {

// One pyramid level: float32 planes of width W, height H, pitch W.
// vertex V (x, y, z = depth), normal N (0 where invalid), intensity I and,
// for the model view, the central-difference intensity gradient G.
struct LevelPtrs {
  float* V[3];
  float* N[3];
  float* I;
  float* G[2];
  int W, H;
  float fx, fy, cx, cy;  // level intrinsics, float32
};

// Per-session estimator state resident in device memory.
struct SessionDev {
  dslam_frame_state x0, x1;
  double qIW[4];
  dslam_prior prior;
  dslam_preint pre;
  float xf[24];        // Ra-I (9) ta (3) Rb-I (9) tb (3) for the next residual pass
  double sys[58];      // reduced sums of the last residual pass
  dslam_track_result result;
  int32_t status;      // first error of the current frame
  int32_t frame_index;
  int32_t pad[2];
};

// Arguments of one residual pass.
struct ResidualArgs {
  const float *cV0, *cV1, *cV2, *cN0, *cN1, *cN2, *cI;                  // current level
  const float *mV0, *mV1, *mV2, *mN0, *mN1, *mN2, *mI, *mG0, *mG1;     // model level
  int W, H, npix;
  float fx, fy, cx, cy;
  float dist2, cosmin, depth_k, sigma_I, huber_k;
  const float* xf;   // device, 24 floats: Ra-I, ta, Rb-I, tb
  float* partials;   // device, [gridDim.x][64] block sums
  uint8_t* mask;     // device, optional
};

enum { RES_THREADS = 256, PARTIAL_STRIDE = 64, SOLVE_THREADS = 256 };

}  // namespace dslam
