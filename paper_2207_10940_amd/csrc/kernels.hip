// Kernels of the dense residual pass (the pass itself is in residual.h): one
// session's pass, the batched pass over many sessions, and their launch
// wrappers.  Compiled with -ffp-contract=off and correctly rounded float32
// division and square root.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "residual.h"

namespace dslam {

template <int PPT>
__global__ __launch_bounds__(RES_THREADS) void residual_kernel(ResidualArgs a) {
  residual_block<PPT>(a, tile_of(blockIdx.x, gridDim.x, a.banded), PPT);
}

template <int PPT, int FMT>
__global__ __launch_bounds__(RES_THREADS) void residual_mfma_kernel(ResidualArgs a) {
  residual_block_mfma<PPT, FMT>(a, tile_of(blockIdx.x, gridDim.x, a.banded), PPT);
}

// Batched: one launch runs one residual pass of every session of the batch.
template <int PMAX>
__global__ __launch_bounds__(RES_THREADS) void residual_batch_kernel(const SlotVis* slots, BatchGrid g, int level,
                                                                     int banded) {
  int slot, b;
  batch_locate(g, blockIdx.x, &slot, &b, banded);
  const SlotVis* sv = slots + slot;
  const ResidualArgs a = sv->res[level];
  residual_block<PMAX>(a, b, sv->ppt[level]);
}

template <int PMAX, int FMT>
__global__ __launch_bounds__(RES_THREADS) void residual_batch_mfma_kernel(const SlotVis* slots, BatchGrid g,
                                                                          int level, int banded) {
  int slot, b;
  batch_locate(g, blockIdx.x, &slot, &b, banded);
  const SlotVis* sv = slots + slot;
  const ResidualArgs a = sv->res[level];
  residual_block_mfma<PMAX, FMT>(a, b, sv->ppt[level]);
}

}  // namespace dslam

// ---------------------------------------------------------------------------
// launch wrappers (host)
// ---------------------------------------------------------------------------
namespace dslam {

template <int FMT>
hipError_t launch_residual_batch_fmt(const SlotVis* slots, const BatchGrid& g, int level, int max_ppt,
                                     int banded, hipStream_t st) {
  const dim3 grid(g.first_block[g.nclass]), blk(RES_THREADS);
  constexpr int M = FMT == DSLAM_JAC_FP32 ? DSLAM_JAC_FP32_MFMA : FMT;  // (the plain kernel takes no format)
  auto k1 = FMT == DSLAM_JAC_FP32 ? residual_batch_kernel<1> : residual_batch_mfma_kernel<1, M>;
  auto k2 = FMT == DSLAM_JAC_FP32 ? residual_batch_kernel<2> : residual_batch_mfma_kernel<2, M>;
  auto k4 = FMT == DSLAM_JAC_FP32 ? residual_batch_kernel<4> : residual_batch_mfma_kernel<4, M>;
  switch (max_ppt) {
    case 1: hipLaunchKernelGGL(k1, grid, blk, 0, st, slots, g, level, banded); break;
    case 2: hipLaunchKernelGGL(k2, grid, blk, 0, st, slots, g, level, banded); break;
    case 4: hipLaunchKernelGGL(k4, grid, blk, 0, st, slots, g, level, banded); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_residual_batch(const SlotVis* slots, const BatchGrid& g, int level, int max_ppt, int jac,
                                 int banded, hipStream_t st) {
  switch (jac) {
    case DSLAM_JAC_FP32: return launch_residual_batch_fmt<DSLAM_JAC_FP32>(slots, g, level, max_ppt, banded, st);
    case DSLAM_JAC_FP32_MFMA:
      return launch_residual_batch_fmt<DSLAM_JAC_FP32_MFMA>(slots, g, level, max_ppt, banded, st);
    case DSLAM_JAC_FP16: return launch_residual_batch_fmt<DSLAM_JAC_FP16>(slots, g, level, max_ppt, banded, st);
    case DSLAM_JAC_BF16: return launch_residual_batch_fmt<DSLAM_JAC_BF16>(slots, g, level, max_ppt, banded, st);
    default: return hipErrorInvalidValue;
  }
}

// Synthetic scene for the autotuner: a slanted plane 1.2-2.8 m away with a
// smooth periodic texture, so that every pixel associates and is textured.
__global__ void tune_scene_kernel(float* depth, uint8_t* inten, int W, int H) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= W || j >= H) return;
  const float u = (float)i / (float)W, v = (float)j / (float)H;
  depth[(size_t)j * W + i] = 1.2f + 1.0f * u + 0.6f * v;
  const float t = 128.0f + 60.0f * __sinf(0.21f * (float)i) + 50.0f * __cosf(0.17f * (float)j);
  inten[(size_t)j * W + i] = (uint8_t)t;
}

hipError_t launch_tune_scene(float* depth, uint8_t* inten, int W, int H, hipStream_t st) {
  hipLaunchKernelGGL(tune_scene_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, depth, inten, W, H);
  return hipGetLastError();
}

int residual_blocks(int npix, int ppt) { return (npix + RES_THREADS * ppt - 1) / (RES_THREADS * ppt); }

hipError_t launch_residual(const ResidualArgs& a, int ppt, hipStream_t st) {
  int nb = residual_blocks(a.npix, ppt);
  if (a.jac == DSLAM_JAC_FP16 || a.jac == DSLAM_JAC_BF16 || a.jac == DSLAM_JAC_FP32_MFMA) {
    const int f = a.jac;
    auto pick = [f](auto k16, auto kb16, auto k32) { return f == DSLAM_JAC_FP16 ? k16 : (f == DSLAM_JAC_BF16 ? kb16 : k32); };
    auto k1 = pick(residual_mfma_kernel<1, DSLAM_JAC_FP16>, residual_mfma_kernel<1, DSLAM_JAC_BF16>,
                   residual_mfma_kernel<1, DSLAM_JAC_FP32_MFMA>);
    auto k2 = pick(residual_mfma_kernel<2, DSLAM_JAC_FP16>, residual_mfma_kernel<2, DSLAM_JAC_BF16>,
                   residual_mfma_kernel<2, DSLAM_JAC_FP32_MFMA>);
    auto k4 = pick(residual_mfma_kernel<4, DSLAM_JAC_FP16>, residual_mfma_kernel<4, DSLAM_JAC_BF16>,
                   residual_mfma_kernel<4, DSLAM_JAC_FP32_MFMA>);
    switch (ppt) {
      case 1: hipLaunchKernelGGL(k1, dim3(nb), dim3(RES_THREADS), 0, st, a); break;
      case 2: hipLaunchKernelGGL(k2, dim3(nb), dim3(RES_THREADS), 0, st, a); break;
      case 4: hipLaunchKernelGGL(k4, dim3(nb), dim3(RES_THREADS), 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (a.jac != DSLAM_JAC_FP32) return hipErrorInvalidValue;
  switch (ppt) {
    case 1: hipLaunchKernelGGL(residual_kernel<1>, dim3(nb), dim3(RES_THREADS), 0, st, a); break;
    case 2: hipLaunchKernelGGL(residual_kernel<2>, dim3(nb), dim3(RES_THREADS), 0, st, a); break;
    case 4: hipLaunchKernelGGL(residual_kernel<4>, dim3(nb), dim3(RES_THREADS), 0, st, a); break;
    case 8: hipLaunchKernelGGL(residual_kernel<8>, dim3(nb), dim3(RES_THREADS), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dslam
