// Pyramid launches (gfx950): every level of one image, or of every session's
// two images in a batched step, in one launch.  The tile code and the
// operations that define each value are in pyramid.h; this translation unit
// is compiled with -ffp-contract=off and correctly rounded float32 division
// and square root.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "step.h"

namespace dslam {

// Pyramid (Section IV-D): every level of one image in one launch, one
// workgroup per 64 x 8 tile of level 0 (the tile code and the operations that
// define each value are in pyramid.h).
__global__ __launch_bounds__(256) void pyramid_kernel(PyrArgs a) {
  __shared__ PyrTileStd::Lds s;
  pyramid_tile<256, 64, 8>(a.src, a.L, a.levels, a.with_grad, blockIdx.x, s, threadIdx.x);
}

// Batched: both pyramids of every session of the batch in one launch, per
// session 2 x PyrTileBatch::tiles workgroups (current frame first), located
// through g.
__global__ __launch_bounds__(PYR_BATCH_THREADS) void pyramid_batch_kernel(const SlotVis* slots, int levels,
                                                                          BatchGrid g) {
  int slot, b;
  batch_locate(g, blockIdx.x, &slot, &b);
  const SlotVis* sv = slots + slot;
  const int per = PyrTileBatch::tiles(sv->cur[0].W, sv->cur[0].H);
  const int which = b >= per ? 1 : 0;
  const PyrSrc src{which ? sv->mdepth : sv->depth, which ? sv->minten : sv->inten, which ? sv->mpitch : sv->pitch};
  __shared__ PyrTileBatch::Lds s;
  pyramid_tile<PYR_BATCH_THREADS, PyrTileBatch::W, PyrTileBatch::H>(src, which ? sv->model : sv->cur, levels, which,
                                                                    b - which * per, s, threadIdx.x,
                                                                    which ? 1 : sv->cur_normals);
}

// The normal planes of one level built without them (pyr_normals_at), one
// thread per pixel.
__global__ __launch_bounds__(256) void normals_kernel(LevelPtrs L) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= L.W * L.H) return;
  const int j = p / L.W, i = p - j * L.W;
  pyr_normals_at(L, i, j);
}

// ---------------------------------------------------------------------------
hipError_t launch_pyramid_batch(const SlotVis* slots, int levels, const BatchGrid& g, hipStream_t st) {
  hipLaunchKernelGGL(pyramid_batch_kernel, dim3(g.first_block[g.nclass]), dim3(PYR_BATCH_THREADS), 0, st, slots,
                     levels, g);
  return hipGetLastError();
}

hipError_t launch_normals(const LevelPtrs& L, hipStream_t st) {
  hipLaunchKernelGGL(normals_kernel, dim3((L.W * L.H + 255) / 256), dim3(256), 0, st, L);
  return hipGetLastError();
}

hipError_t launch_pyramid(const PyrArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(pyramid_kernel, dim3(PyrTileStd::tiles(a.L[0].W, a.L[0].H)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace dslam
