// Pyramid construction (Section IV-D: three-level coarse-to-fine scheme), all
// levels of one image in one launch.
//   level 0: depth cleaned (finite and > 0, else 0), intensity = float(uint8);
//   level l+1: depth = mean of the valid depths of the 2x2 block summed in the
//   order (2x,2y), (2x+1,2y), (2x,2y+1), (2x+1,2y+1); intensity =
//   ((a + b) + (c + d)) * 0.25 of the stored (fixed-point) level-l values;
//   vertex = rho(u, d) = (((i - cx) d) / fx, ((j - cy) d) / fy, d);
//   normal = (a x b) / |a x b| with a = V(i+1,j) - V(i,j), b = V(i,j+1) - V(i,j);
//   gradient (model view) = central differences * 0.5, zero on the border.
//
// A workgroup owns a TW x TH tile of level 0 and the (TW/2^l) x (TH/2^l) tile
// above it at every level l.  Each level's depth and intensity are kept in LDS
// over the tile plus a margin of 2^(c-l) pixels (c = coarsest level): one
// pixel for the coarsest level's normals and gradients, and at every finer
// level the 2x2 parents of the next level's margin.  The margin is recomputed
// by the neighbouring tiles too, with the same operations, so every value is
// the one a level-by-level construction produces.  The functions below contract
// no multiply-add (whatever the translation unit's setting); include only in
// translation units built with correctly rounded float32 division and square
// root.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "device.h"

namespace dslam {

// Tile shapes: the standalone pyramid launch uses 64 x 8 tiles (two level-0
// pixels per thread of 256); the launch shared with the frame initialisation
// and the batched launch use 64 x 16 tiles with 512 threads (less margin
// recomputed per tile).  Rows of 64 pixels keep the 16-bit planes' stores in
// whole 128-byte lines.
template <int TW, int TH>
struct PyrTile {
  static_assert((TW >> (DSLAM_MAX_LEVELS - 1)) >= 1 && (TH >> (DSLAM_MAX_LEVELS - 1)) >= 1,
                "tile too small for the deepest pyramid");
  static constexpr int W = TW, H = TH;
  // sides of level l's region in LDS when the coarsest level is c
  __host__ __device__ static constexpr int ew(int l, int c) { return (TW >> l) + 2 * (1 << (c - l)); }
  __host__ __device__ static constexpr int eh(int l, int c) { return (TH >> l) + 2 * (1 << (c - l)); }
  __host__ __device__ static constexpr int entries(int c) {
    int n = 0;
    for (int l = 0; l <= c; ++l) n += ew(l, c) * eh(l, c);
    return n;
  }
  static constexpr int LDS = entries(DSLAM_MAX_LEVELS - 1);
  __host__ __device__ static int tiles(int W, int H) { return ((W + TW - 1) / TW) * ((H + TH - 1) / TH); }
  struct Lds {
    float d[LDS];  // depth of every level's region, level after level
    float i[LDS];  // intensity (float, before the fixed-point store)
  };
};
using PyrTileStd = PyrTile<64, 8>;
using PyrTileBig = PyrTile<64, 16>;
// the batched pyramids' tile and workgroup
using PyrTileBatch = PyrTileBig;
enum { PYR_BATCH_THREADS = 512 };

// The level-0 images of one pyramid (device, row pitch in elements).
struct PyrSrc {
  const float* depth;
  const uint8_t* inten;
  int pitch;
};

// One pyramid launch: its source images and its levels' planes.
struct PyrArgs {
  PyrSrc src;
  LevelPtrs L[DSLAM_MAX_LEVELS];
  int32_t levels, with_grad;
};

__device__ __forceinline__ float clean_depth(float d) { return (__builtin_isfinite(d) && d > 0.0f) ? d : 0.0f; }

// Global-memory loads and stores through the global address space: a generic
// pointer might alias LDS, which would order every LDS access behind them.
template <class T>
__device__ __forceinline__ T pyr_ld(const T* base, size_t idx) {
  typedef const __attribute__((address_space(1))) T GT;
  return ((GT*)base)[idx];
}
template <class T>
__device__ __forceinline__ void pyr_st(T* base, size_t idx, T v) {
  typedef __attribute__((address_space(1))) T GT;
  ((GT*)base)[idx] = v;
}

// Normal of pixel (i, j) of a level from its depth d, its right and lower
// neighbours' depths dr and dd, and its vertex (vx, vy, d): the normalised
// cross product of the forward differences, zero on the last row and column
// and where a depth is missing.
__device__ __forceinline__ void pyr_normal(const LevelPtrs& L, int i, int j, float d, float dr, float dd, float vx,
                                           float vy, float* n) {
#pragma clang fp contract(off)
  const float fi = (float)i, fj = (float)j;
  float nx = 0.0f, ny = 0.0f, nz = 0.0f;
  if (i < L.W - 1 && j < L.H - 1) {
    const float ax = (((fi + 1.0f) - L.cx) * dr) / L.fx - vx;
    const float ay = ((fj - L.cy) * dr) / L.fy - vy;
    const float az = dr - d;
    const float bx = ((fi - L.cx) * dd) / L.fx - vx;
    const float by = (((fj + 1.0f) - L.cy) * dd) / L.fy - vy;
    const float bz = dd - d;
    const float cx = ay * bz - az * by;
    const float cy = az * bx - ax * bz;
    const float cz = ax * by - ay * bx;
    const float len = __builtin_sqrtf((cx * cx + cy * cy) + cz * cz);
    if (d > 0.0f && dr > 0.0f && dd > 0.0f && len > 0.0f) {
      nx = cx / len;
      ny = cy / len;
      nz = cz / len;
    }
  }
  n[0] = nx;
  n[1] = ny;
  n[2] = nz;
}

// Level outputs of pixel (i, j), whose depth and intensity sit at (a, b) of a
// region of width E in LDS (all four neighbours are inside the region).
// Without with_normals the normal planes are left unwritten (pyr_normals_at
// fills them later from the stored depths, with the same operations).
__device__ __forceinline__ void pyr_out(const LevelPtrs& L, const float* D, const float* In, int E, int a, int b,
                                        int i, int j, int with_grad, int with_normals) {
#pragma clang fp contract(off)
  const int q = b * E + a;
  // every LDS read first
  const float d = D[q], dr = D[q + 1], dd = D[q + E];
  const float ic = In[q];
  float il = 0.0f, ir = 0.0f, iu = 0.0f, idn = 0.0f;
  if (with_grad) {
    il = In[q - 1];
    ir = In[q + 1];
    iu = In[q - E];
    idn = In[q + E];
  }
  const size_t p = (size_t)j * L.W + i;
  const float fi = (float)i, fj = (float)j;
  const float vx = ((fi - L.cx) * d) / L.fx;
  const float vy = ((fj - L.cy) * d) / L.fy;
  pyr_st(L.V[0], p, vx);
  pyr_st(L.V[1], p, vy);
  pyr_st(L.V[2], p, d);
  pyr_st(L.I, p, (uint16_t)(ic * kIntensityScale));
  if (with_normals) {
    float n[3];
    pyr_normal(L, i, j, d, dr, dd, vx, vy, n);
    pyr_st(L.N[0], p, n[0]);
    pyr_st(L.N[1], p, n[1]);
    pyr_st(L.N[2], p, n[2]);
  }
  if (with_grad) {
    float gx = 0.0f, gy = 0.0f;
    if (i > 0 && i < L.W - 1 && j > 0 && j < L.H - 1) {
      gx = (ir - il) * 0.5f;
      gy = (idn - iu) * 0.5f;
    }
    pyr_st(L.G[0], p, (int16_t)(gx * kGradientScale));
    pyr_st(L.G[1], p, (int16_t)(gy * kGradientScale));
  }
}

// All levels of tile `tile` (row-major over the level-0 tiles of L[0]) with NT
// threads; tid is the thread's index in the workgroup.  L[l] for l < levels.
template <int NT, int TW, int TH>
__device__ __forceinline__ void pyramid_tile(const PyrSrc& src, const LevelPtrs* L, int levels, int with_grad,
                                             int tile, typename PyrTile<TW, TH>::Lds& s, int tid,
                                             int with_normals = 1) {
#pragma clang fp contract(off)
  using P = PyrTile<TW, TH>;
  const int c = levels - 1;
  const int tiles_x = (L[0].W + TW - 1) / TW;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  {  // level 0 region from the caller's images (zero outside the image): all
     // loads in flight (a pixel outside reads pixel 0), then the LDS stores
    constexpr int IT = (P::ew(0, DSLAM_MAX_LEVELS - 1) * P::eh(0, DSLAM_MAX_LEVELS - 1) + NT - 1) / NT;
    const int m = 1 << c, Ew = P::ew(0, c), n = Ew * P::eh(0, c);
    const int ox = tx * TW - m, oy = ty * TH - m;
    const int W = L[0].W, H = L[0].H;
    float dv[IT], iv[IT];
    bool inside[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const int k = tid + r * NT;
      const int b = k / Ew, a = k - b * Ew;
      const int i = ox + a, j = oy + b;
      inside[r] = k < n && i >= 0 && i < W && j >= 0 && j < H;
      const size_t g = inside[r] ? (size_t)j * src.pitch + i : 0;
      dv[r] = pyr_ld(src.depth, g);
      iv[r] = (float)pyr_ld(src.inten, g);
    }
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const int k = tid + r * NT;
      if (k < n) {
        s.d[k] = inside[r] ? clean_depth(dv[r]) : 0.0f;
        s.i[k] = inside[r] ? iv[r] : 0.0f;
      }
    }
  }
  __syncthreads();
  int off = 0;
  for (int l = 0; l < levels; ++l) {
    const int Tw = TW >> l, Th = TH >> l, m = 1 << (c - l), Ew = Tw + 2 * m;
    const float* D = s.d + off;
    const float* In = s.i + off;
    const LevelPtrs& Ll = L[l];
    for (int k = tid; k < Tw * Th; k += NT) {
      const int b = k / Tw, a = k - b * Tw;
      const int i = tx * Tw + a, j = ty * Th + b;
      if (i < Ll.W && j < Ll.H) pyr_out(Ll, D, In, Ew, a + m, b + m, i, j, with_grad, with_normals);
    }
    if (l + 1 < levels) {  // the next level's region from this one
      const int m1 = m >> 1, E1w = (Tw >> 1) + 2 * m1, E1h = (Th >> 1) + 2 * m1;
      float* D1 = s.d + off + Ew * (Th + 2 * m);
      float* I1 = s.i + off + Ew * (Th + 2 * m);
      const int ox = tx * (Tw >> 1) - m1, oy = ty * (Th >> 1) - m1;
      const int W1 = L[l + 1].W, H1 = L[l + 1].H;
      const float qs = 1.0f / kIntensityScale;
      for (int k = tid; k < E1w * E1h; k += NT) {
        const int b = k / E1w, a = k - b * E1w;
        const int i = ox + a, j = oy + b;
        float d = 0.0f, in = 0.0f;
        if (i >= 0 && i < W1 && j >= 0 && j < H1) {
          const int q = 2 * b * Ew + 2 * a;  // parents (2a, 2b) .. (2a+1, 2b+1) of this level's region
          const float t[4] = {D[q], D[q + 1], D[q + Ew], D[q + Ew + 1]};
          const float u[4] = {In[q], In[q + 1], In[q + Ew], In[q + Ew + 1]};
          float sum = 0.0f, cnt = 0.0f;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (t[v] > 0.0f) {
              sum = sum + t[v];
              cnt = cnt + 1.0f;
            }
          d = cnt > 0.0f ? sum / cnt : 0.0f;
          const float r00 = (float)(uint16_t)(u[0] * kIntensityScale);
          const float r01 = (float)(uint16_t)(u[1] * kIntensityScale);
          const float r10 = (float)(uint16_t)(u[2] * kIntensityScale);
          const float r11 = (float)(uint16_t)(u[3] * kIntensityScale);
          in = ((r00 * qs + r01 * qs) + (r10 * qs + r11 * qs)) * 0.25f;
        }
        D1[k] = d;
        I1[k] = in;
      }
      off += Ew * (Th + 2 * m);
    }
    __syncthreads();
  }
}

// The normal planes of pixel (i, j) of a level whose vertex planes are written
// (a pyramid built without normals): the same operations on the stored depths
// as pyr_out, so the values are those a pyramid with normals holds.
__device__ __forceinline__ void pyr_normals_at(const LevelPtrs& L, int i, int j) {
#pragma clang fp contract(off)
  const size_t p = (size_t)j * L.W + i;
  const float d = pyr_ld(L.V[2], p);
  const float dr = i < L.W - 1 ? pyr_ld(L.V[2], p + 1) : 0.0f;
  const float dd = j < L.H - 1 ? pyr_ld(L.V[2], p + L.W) : 0.0f;
  const float vx = ((((float)i) - L.cx) * d) / L.fx;
  const float vy = ((((float)j) - L.cy) * d) / L.fy;
  float n[3];
  pyr_normal(L, i, j, d, dr, dd, vx, vy, n);
  pyr_st(L.N[0], p, n[0]);
  pyr_st(L.N[1], p, n[1]);
  pyr_st(L.N[2], p, n[2]);
}

}  // namespace dslam
