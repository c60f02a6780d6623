// Arguments of the per-frame device kernels (frame initialisation, solve) and
// the launch wrappers of every kernel, shared by the kernel sources and the
// host library.
#pragma once
#include <hip/hip_runtime.h>
#include "device.h"
#include "pyramid.h"
#include "solve_core.h"

namespace dslam {

// The frame's IMU samples, by value (they reach the device inside kernel
// arguments or a batch's staging copy).
struct ImuBatch {
  int32_t n;
  double t0, t1;
  dslam_imu_sample s[DSLAM_MAX_IMU_SAMPLES];
};

struct FrameArgs {
  ImuParamsD imu;
  double sigma_g, sigma_a;
  double R_WM[9], t_WM[3];
  int32_t mode;
  int32_t imu_fallback;  // keep the frame's start for the inertial-only fallback
};

struct SolveArgs {
  SolveParams sp;
  int32_t level;
  int32_t flags;     // STEP_* flags
  int32_t nblocks;
};

// One session's share of a batched step, frame-initialisation and solve part.
struct SlotSolve {
  SessionDev* sd;
  const float* partials;
  ImuBatch imu;
  FrameArgs fa;
  SolveParams sp;
  int32_t nblocks[DSLAM_MAX_LEVELS];
};

// Flags of a visual solve: the first iteration of the frame's finest level
// (records the cost the health check compares with) and the frame's last
// iteration (solves the 33-d system, marginalises, publishes the result).
// STEP_INERTIAL: the inertial-only re-estimate of a lost frame (runs after the
// frame's last step; returns at once unless the frame was lost).
enum { STEP_FIRST = 1, STEP_LAST = 2, STEP_INERTIAL = 4 };

// pyramid.hip
hipError_t launch_pyramid(const PyrArgs& a, hipStream_t st);
// every level of every session's current and model-view pyramids; g maps the
// workgroups (2 x PyrTileBatch::tiles per session: current frame first)
hipError_t launch_pyramid_batch(const SlotVis* slots, int levels, const BatchGrid& g, hipStream_t st);
hipError_t launch_normals(const LevelPtrs& L, hipStream_t st);

// kernels.hip
int residual_blocks(int npix, int ppt);
hipError_t launch_residual(const ResidualArgs& a, int ppt, hipStream_t st);
hipError_t launch_tune_scene(float* depth, uint8_t* inten, int W, int H, hipStream_t st);
hipError_t launch_residual_batch(const SlotVis* slots, const BatchGrid& g, int level, int max_ppt, int jac,
                                 int banded, hipStream_t st);

// solve.hip
// the frame initialisation, the current frame's pyramid and (model != nullptr)
// the model view's pyramid in one launch; the frame's solve parameters are
// stored at sp_out, where the step kernels read them
hipError_t launch_frame_init_pyramid(SessionDev* sd, const ImuBatch& b, const FrameArgs& fa, const SolveParams& sp,
                                     const PyrArgs& cur, const PyrArgs* model, SolveParams* sp_out, hipStream_t st);
// one Gauss-Newton step of one session after its residual pass (STEP_* flags)
hipError_t launch_solve(SessionDev* sd, const float* partials, const SolveArgs& a, hipStream_t st);
// the same step with the solve parameters read from device memory
hipError_t launch_solve_graph(SessionDev* sd, const float* partials, const SolveParams* sp, int level, int flags,
                              int nblocks, hipStream_t st);
hipError_t launch_reduce(const float* partials, int nblocks, double* out, hipStream_t st);
hipError_t launch_frame_init_batch(const SlotSolve* slots, int n, hipStream_t st);
hipError_t launch_solve_batch(const SlotSolve* slots, int n, int level, int flags, hipStream_t st);
hipError_t launch_gather_results(const SlotSolve* slots, int n, dslam_track_result* out, hipStream_t st);

}  // namespace dslam
