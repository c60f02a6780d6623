// Device-side data layout shared by the kernels and the host library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/dslam.h"

namespace dslam {

// One pyramid level: planes of width W, height H, pitch W.
//   V: vertex (x, y, z = depth), 3 float32 planes;
//   N: normal (3 float32 planes, 0 where invalid);
//   I: intensity in fixed point, I * 64 as uint16 (exact: level l holds
//      multiples of 4^-l <= 255 and l <= 3);
//   G: model view only, the central-difference gradient * 128 as int16
//      (exact for the same reason: multiples of 2^-(2l+1), |G| <= 127.5).
struct LevelPtrs {
  float* V[3];
  float* N[3];
  uint16_t* I;
  int16_t* G[2];
  int W, H;
  float fx, fy, cx, cy;  // level intrinsics, float32
};

constexpr float kIntensityScale = 64.0f, kGradientScale = 128.0f;

// Per-session estimator state resident in device memory.
struct SessionDev {
  dslam_frame_state x0, x1;
  double qIW[4];
  dslam_prior prior;
  dslam_preint pre;
  double Linv[81];     // L^-1 of pre.Sigma = L L^T (row-major, lower triangular)
  float xf[24];        // Ra-I (9) ta (3) Rb-I (9) tb (3) for the next residual pass
  double sys[58];      // reduced sums of the last residual pass
  dslam_track_result result;
  double cost_first;   // visual cost at the first iteration of the frame's finest level (health check)
  // the frame's start (inertial-only fallback): x0, the IMU prediction of x1, q_IW and the prior
  dslam_frame_state x0_frame, x1_pred;
  double qIW_frame[4];
  dslam_prior prior_frame;
  int32_t status;      // first error of the current frame
  int32_t frame_index;
};

// Arguments of one residual pass.
struct ResidualArgs {
  const float *cV0, *cV1, *cV2, *cN0, *cN1, *cN2;   // current level
  const uint16_t* cI;
  const float *mV0, *mV1, *mV2, *mN0, *mN1, *mN2;   // model level
  const uint16_t* mI;
  const int16_t *mG0, *mG1;
  int W, H, npix;
  float fx, fy, cx, cy;
  float dist2, cosmin, depth_k, sigma_I, huber_k;
  const float* xf;   // device, 24 floats: Ra-I, ta, Rb-I, tb
  float* partials;   // device, [gridDim.x][64] block sums
  uint8_t* mask;     // device, optional
  int32_t jac;       // DSLAM_JAC_*: how the per-pixel terms are reduced
  float col_scale[2];  // precision form: power-of-two scale of the ICP / photometric row entries
  int32_t banded;      // tile order of the launch (tile_of)
};

// Tile processed by workgroup bid of an n-workgroup launch.  Workgroups are
// dealt to the 8 XCDs round-robin (workgroup bid runs on XCD bid % 8); with
// banded != 0 XCD x takes the contiguous tiles [x q + min(x, r), ...) of its
// share (q = n / 8, r = n % 8), so that neighbouring tiles, which read the
// same rows of the model view, share that XCD's L2.  A bijection of [0, n):
// each tile's partial sums land in the same place either way.
__device__ __forceinline__ int tile_of(int bid, int n, int banded) {
  if (!banded) return bid;
  const int x = bid & 7, i = bid >> 3, q = n >> 3, r = n & 7;
  return x * q + (x < r ? x : r) + i;
}

enum { RES_THREADS = 256, PARTIAL_STRIDE = 64, SOLVE_THREADS = 512 };

// ---- batched steps: several sessions share every launch ---------------------
enum { MAX_BATCH = 256, MAX_CLASSES = 16 };

// One session's visual inputs for a batched step (device copy of host staging).
struct SlotVis {
  ResidualArgs res[DSLAM_MAX_LEVELS];  // xf = the session's transforms, partials = its buffer
  LevelPtrs cur[DSLAM_MAX_LEVELS], model[DSLAM_MAX_LEVELS];
  const float* depth;                  // current frame, device
  const uint8_t* inten;
  const float* mdepth;                 // model view, device
  const uint8_t* minten;
  int32_t pitch, mpitch;
  int32_t ppt[DSLAM_MAX_LEVELS];       // pixels per thread of each level's residual pass
  int32_t cur_normals;                 // 1: the step writes the current pyramid's normal planes
};

// Work split of one batched launch.  The slots are ordered so that slots with
// the same number of workgroups are contiguous; class c covers workgroups
// [first_block[c], first_block[c+1]) and slots first_slot[c] onwards, each
// slot taking blocks_per_slot[c] consecutive workgroups.
struct BatchGrid {
  int32_t nclass;
  int32_t first_block[MAX_CLASSES + 1];
  int32_t blocks_per_slot[MAX_CLASSES];
  int32_t first_slot[MAX_CLASSES];
};

// Workgroup -> (slot, workgroup within the slot); uniform across the workgroup.
// With banded != 0 the tile order (tile_of) is applied within each class: the
// class's workgroups that share an XCD (same local index mod 8) take one
// contiguous band of its tiles, so every XCD gets an equal share of every
// class (tiles of different classes differ in cost) and neighbouring tiles of
// one session share an L2.
__device__ __forceinline__ void batch_locate(const BatchGrid& g, int blk, int* slot, int* b, int banded = 0) {
  int c = 0;
  for (int k = 1; k < g.nclass; ++k) c = blk >= g.first_block[k] ? k : c;
  const int off = tile_of(blk - g.first_block[c], g.first_block[c + 1] - g.first_block[c], banded);
  const int q = off / g.blocks_per_slot[c];
  *slot = g.first_slot[c] + q;
  *b = off - q * g.blocks_per_slot[c];
}

}  // namespace dslam
