// Surfel map (gfx950): fusion of tracked frames and prediction of the model
// view the tracker aligns to (the mapping step the paper keeps from its dense
// RGB-D base system, Sections III and V).  Readings:
//   * a surfel holds a world position p, a unit world normal n, an intensity,
//     a radius and a confidence (structure of arrays on the device);
//   * transforms are float32 (D = R - I, t) rounded once from float64, and a
//     point maps as q = p + (((D00 x + D01 y) + D02 z) + t0) per component;
//     projection as in the tracker: inv = 1/q_z, u = ((fx q_x) inv) + cx,
//     rounded half-even;
//   * fusion: every surfel in front of the camera marks the pixel of its
//     projected centre with the key (bits(q_z) << 32) | index, the smallest
//     key wins; the frame's measurement at a pixel is its level-0 vertex with
//     the normal of its parent pixel at level 1 (level 0 for a one-level
//     pyramid: raw full-resolution normals are dominated by depth noise); a
//     valid pixel of the frame updates the surfel of its cell when
//     |z_s - z| <= dist and n_s . n_m >= cos_min, with the confidence-weighted
//     averages c' = c + alpha, p' = ((c p) + (alpha p_m)) / c', n' the
//     normalised (c n) + (alpha n_m), I' likewise, r' = min(r, r_m),
//     alpha = 1 / (1 + g2), g2 = ((i - cx)^2 + (j - cy)^2) / (cx^2 + cy^2),
//     r_m = (z sqrt2) / (fx max(|N_z|, 0.5)); every other valid pixel becomes
//     a new surfel unless one of its 8 neighbouring cells holds a surfel
//     within dist of its depth (the surface is mapped there already: a moving
//     camera leaves cells between projected centres empty), appended in pixel
//     order while the capacity lasts (each surfel marks one cell, so at most
//     one pixel updates it, and the neighbour test reads only the index map:
//     no races);
//   * prediction: each surfel covers the pixels within
//     h = min(ceil((r fx) / q_z), 4) of its rounded centre whose ray meets
//     its disk (depth t = (n_c . q) / (n_c . d), |t d - q|^2 <= r^2); of the
//     surfels covering a pixel, those within `band` of the nearest depth form
//     its front surface and the one whose projected centre is closest to the
//     pixel wins (then the lowest index), so that of several noisy
//     observations of one surface the most central is shown, not the nearest;
//     the model view's depth is the winner's t, its intensity the winner's,
//     rounded half-even and clamped, and its level-0 normals the winners'
//     camera-frame normals (averaged over the fused frames, instead of
//     forward differences of the rendered depth, which keep the depth noise
//     of the frames the surfels came from).
// Every float32 operation is one IEEE operation in the order written (built
// with -ffp-contract=off, correctly rounded division and square root), so the
// map and the rendered view are reproducible bit for bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "host.h"

namespace dslam {

constexpr uint64_t MAP_EMPTY = ~0ull;
constexpr int MAP_HMAX = 4;
constexpr int MAP_SCAN = 1024;  // pixels per scan block of the append (256 threads x 4)
constexpr float MAP_SQRT2 = 1.41421356f;
enum { MAP_PX = 0, MAP_PY, MAP_PZ, MAP_NX, MAP_NY, MAP_NZ, MAP_I, MAP_R, MAP_C, MAP_FIELDS };

struct XformF {
  float D[9];  // R - I
  float t[3];
};

struct MapDev {
  float* f[MAP_FIELDS];  // surfel fields, capacity each
  int32_t* count;        // device: surfels in the map
  int32_t* base;         // device: count before the last append
  int32_t* dropped;      // device: new surfels refused for lack of capacity (cumulative)
  int32_t capacity;
};

struct MapCam {
  float fx, fy, cx, cy;
  int W, H;
};

__device__ __forceinline__ void map_xform(const XformF& T, float x, float y, float z, float* q) {
  q[0] = x + (((T.D[0] * x + T.D[1] * y) + T.D[2] * z) + T.t[0]);
  q[1] = y + (((T.D[3] * x + T.D[4] * y) + T.D[5] * z) + T.t[1]);
  q[2] = z + (((T.D[6] * x + T.D[7] * y) + T.D[8] * z) + T.t[2]);
}

__device__ __forceinline__ void map_rotate(const XformF& T, float x, float y, float z, float* n) {
  n[0] = x + ((T.D[0] * x + T.D[1] * y) + T.D[2] * z);
  n[1] = y + ((T.D[3] * x + T.D[4] * y) + T.D[5] * z);
  n[2] = z + ((T.D[6] * x + T.D[7] * y) + T.D[8] * z);
}

__device__ __forceinline__ uint64_t map_key(float z, uint32_t s) {
  return ((uint64_t)__float_as_uint(z) << 32) | (uint64_t)s;
}

__global__ __launch_bounds__(256) void map_fill_kernel(uint64_t* keys, int n) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < n) keys[p] = MAP_EMPTY;
}

__global__ __launch_bounds__(64) void map_zero_kernel(int32_t* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// Index map: every surfel marks the cell of its projected centre.
__global__ __launch_bounds__(256) void map_index_kernel(MapDev m, XformF cw, MapCam cam, uint64_t* keys) {
  const int n = *m.count;
  for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256) {
    float q[3];
    map_xform(cw, m.f[MAP_PX][s], m.f[MAP_PY][s], m.f[MAP_PZ][s], q);
    const float inv = 1.0f / q[2];
    const float u = rintf(((cam.fx * q[0]) * inv) + cam.cx);
    const float v = rintf(((cam.fy * q[1]) * inv) + cam.cy);
    if (q[2] > 0.0f && u >= 0.0f && u <= (float)(cam.W - 1) && v >= 0.0f && v <= (float)(cam.H - 1))
      atomicMin((unsigned long long*)&keys[(int)v * cam.W + (int)u], (unsigned long long)map_key(q[2], (uint32_t)s));
  }
}

// The frame's measurement at pixel p (level-0 planes of the session's
// current pyramid).
struct MapMeas {
  float p[3], n[3], I, r, alpha;
  bool valid;
};

// The frame's level 0 (vertices, intensity) and the level its normals come
// from (parent pixel (i >> sh, j >> sh)).
struct MapFrame {
  LevelPtrs L0, Ln;
  int sh;
};

__device__ __forceinline__ MapMeas map_measure(const MapFrame& fr, const XformF& wc, const MapCam& cam, int p) {
  MapMeas o;
  const LevelPtrs& L = fr.L0;
  const int j = p / cam.W, i = p - j * cam.W;
  const int pn = (j >> fr.sh) * fr.Ln.W + (i >> fr.sh);
  const float vx = L.V[0][p], vy = L.V[1][p], vz = L.V[2][p];
  const float nx = fr.Ln.N[0][pn], ny = fr.Ln.N[1][pn], nz = fr.Ln.N[2][pn];
  o.valid = vz > 0.0f && (nx != 0.0f || ny != 0.0f || nz != 0.0f);
  map_xform(wc, vx, vy, vz, o.p);
  map_rotate(wc, nx, ny, nz, o.n);
  o.I = (float)L.I[p] * (1.0f / 64.0f);
  const float dx = (float)i - cam.cx, dy = (float)j - cam.cy;
  const float g2 = (dx * dx + dy * dy) / (cam.cx * cam.cx + cam.cy * cam.cy);
  o.alpha = 1.0f / (1.0f + g2);
  o.r = (vz * MAP_SQRT2) / (cam.fx * fmaxf(fabsf(nz), 0.5f));
  return o;
}

// Exclusive prefix of flag over the 256 threads of the block in thread order;
// *total receives the block's sum.  lds: 4 ints.
__device__ __forceinline__ int map_block_scan(int flag, int* lds, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long b = __ballot(flag);
  const int in_wave = __popcll(b & ((1ull << lane) - 1ull));
  if (lane == 0) lds[wave] = __popcll(b);
  __syncthreads();
  int before = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    before += w < wave ? lds[w] : 0;
    sum += lds[w];
  }
  __syncthreads();
  *total = sum;
  return before + in_wave;
}

// Fusion: updates the associated surfels, flags the new pixels and counts them
// per scan block (pixel b*1024 + k*256 + t on thread t, k = 0..3).
__global__ __launch_bounds__(256) void map_fuse_kernel(MapDev m, MapFrame fr, XformF wc, MapCam cam, float dist,
                                                       float cos_min, const uint64_t* keys, uint8_t* flags,
                                                       int32_t* block_new) {
  __shared__ int lds[4];
  const int npx = cam.W * cam.H;
  int block_total = 0;
  for (int k = 0; k < 4; ++k) {
    const int p = blockIdx.x * MAP_SCAN + k * 256 + (int)threadIdx.x;
    int isnew = 0;
    if (p < npx) {
      const MapMeas a = map_measure(fr, wc, cam, p);
      const uint64_t key = keys[p];
      bool assoc = false;
      if (a.valid && key != MAP_EMPTY) {
        const int s = (int)(uint32_t)(key & 0xFFFFFFFFull);
        const float zs = __uint_as_float((uint32_t)(key >> 32));
        // every read of the surfel before any write
        float P[3] = {m.f[MAP_PX][s], m.f[MAP_PY][s], m.f[MAP_PZ][s]};
        float Nn[3] = {m.f[MAP_NX][s], m.f[MAP_NY][s], m.f[MAP_NZ][s]};
        const float Is = m.f[MAP_I][s], rs = m.f[MAP_R][s], c = m.f[MAP_C][s];
        const float ndot = (Nn[0] * a.n[0] + Nn[1] * a.n[1]) + Nn[2] * a.n[2];
        assoc = fabsf(zs - fr.L0.V[2][p]) <= dist && ndot >= cos_min;
        if (assoc) {
          const float c1 = c + a.alpha;
          m.f[MAP_PX][s] = ((c * P[0]) + (a.alpha * a.p[0])) / c1;
          m.f[MAP_PY][s] = ((c * P[1]) + (a.alpha * a.p[1])) / c1;
          m.f[MAP_PZ][s] = ((c * P[2]) + (a.alpha * a.p[2])) / c1;
          m.f[MAP_I][s] = ((c * Is) + (a.alpha * a.I)) / c1;
          const float n0 = (c * Nn[0]) + (a.alpha * a.n[0]);
          const float n1 = (c * Nn[1]) + (a.alpha * a.n[1]);
          const float n2 = (c * Nn[2]) + (a.alpha * a.n[2]);
          const float ln = __builtin_sqrtf((n0 * n0 + n1 * n1) + n2 * n2);
          if (ln > 0.0f) {
            m.f[MAP_NX][s] = n0 / ln;
            m.f[MAP_NY][s] = n1 / ln;
            m.f[MAP_NZ][s] = n2 / ln;
          }
          m.f[MAP_R][s] = fminf(rs, a.r);
          m.f[MAP_C][s] = c1;
        }
      }
      bool covered = false;
      if (a.valid && !assoc) {  // a mapped neighbour cell at this depth
        const int j = p / cam.W, i = p - j * cam.W;
        const float z = fr.L0.V[2][p];
        for (int dj = -1; dj <= 1; ++dj)
          for (int di = -1; di <= 1; ++di) {
            const int i2 = i + di, j2 = j + dj;
            if ((di == 0 && dj == 0) || i2 < 0 || i2 >= cam.W || j2 < 0 || j2 >= cam.H) continue;
            const uint64_t k2 = keys[j2 * cam.W + i2];
            if (k2 != MAP_EMPTY && fabsf(__uint_as_float((uint32_t)(k2 >> 32)) - z) <= dist) covered = true;
          }
      }
      isnew = (a.valid && !assoc && !covered) ? 1 : 0;
      flags[p] = (uint8_t)isnew;
    }
    int t;
    map_block_scan(isnew, lds, &t);
    block_total += t;
  }
  if (threadIdx.x == 0) block_new[blockIdx.x] = block_total;
}

// Exclusive scan of the per-block new counts (one workgroup of 1024), the
// append base and the map's new count.
__global__ __launch_bounds__(1024) void map_scan_kernel(MapDev m, const int32_t* block_new, int nb,
                                                        int32_t* block_off) {
  __shared__ int sums[1024];
  const int t = threadIdx.x, per = (nb + 1023) / 1024;
  int s = 0;
  for (int i = t * per; i < min(nb, (t + 1) * per); ++i) s += block_new[i];
  sums[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan
    const int v = t >= d ? sums[t - d] : 0;
    __syncthreads();
    sums[t] += v;
    __syncthreads();
  }
  int run = t > 0 ? sums[t - 1] : 0;
  for (int i = t * per; i < min(nb, (t + 1) * per); ++i) {
    block_off[i] = run;
    run += block_new[i];
  }
  if (t == 0) {
    const int total = sums[1023], base = *m.count, room = m.capacity - base;
    const int added = total < room ? total : room;
    *m.base = base;
    *m.count = base + added;
    *m.dropped += total - added;
  }
}

// Appends the flagged pixels as new surfels in pixel order.
__global__ __launch_bounds__(256) void map_append_kernel(MapDev m, MapFrame fr, XformF wc, MapCam cam,
                                                         const uint8_t* flags, const int32_t* block_off) {
  __shared__ int lds[4];
  const int npx = cam.W * cam.H, base = *m.base;
  int run = block_off[blockIdx.x];
  for (int k = 0; k < 4; ++k) {
    const int p = blockIdx.x * MAP_SCAN + k * 256 + (int)threadIdx.x;
    const int isnew = p < npx ? (int)flags[p] : 0;
    int total;
    const int rank = run + map_block_scan(isnew, lds, &total);
    run += total;
    const int idx = base + rank;
    if (isnew && idx < m.capacity) {
      const MapMeas a = map_measure(fr, wc, cam, p);
      m.f[MAP_PX][idx] = a.p[0];
      m.f[MAP_PY][idx] = a.p[1];
      m.f[MAP_PZ][idx] = a.p[2];
      m.f[MAP_NX][idx] = a.n[0];
      m.f[MAP_NY][idx] = a.n[1];
      m.f[MAP_NZ][idx] = a.n[2];
      m.f[MAP_I][idx] = a.I;
      m.f[MAP_R][idx] = a.r;
      m.f[MAP_C][idx] = a.alpha;
    }
  }
}

// Splat rendering, in two passes over the surfels' footprints: the nearest
// depth of each pixel, then the most central surfel of its front surface.
// splat_visit calls fn(pixel, t, d2c) for every pixel surfel s covers.
template <class Fn>
__device__ __forceinline__ void splat_visit(const MapDev& m, int s, const XformF& cw, const MapCam& cam, Fn fn) {
  float q[3], nc[3];
  map_xform(cw, m.f[MAP_PX][s], m.f[MAP_PY][s], m.f[MAP_PZ][s], q);
  map_rotate(cw, m.f[MAP_NX][s], m.f[MAP_NY][s], m.f[MAP_NZ][s], nc);
  const float r = m.f[MAP_R][s];
  if (!(q[2] > 0.0f)) return;
  const float inv = 1.0f / q[2];
  const float u = ((cam.fx * q[0]) * inv) + cam.cx, v = ((cam.fy * q[1]) * inv) + cam.cy;
  const float u0 = rintf(u), v0 = rintf(v);
  const float h = fminf(ceilf((r * cam.fx) / q[2]), (float)MAP_HMAX);
  if (!(u0 >= (float)-MAP_HMAX && u0 <= (float)(cam.W - 1 + MAP_HMAX) && v0 >= (float)-MAP_HMAX &&
        v0 <= (float)(cam.H - 1 + MAP_HMAX)))
    return;
  const int ui = (int)u0, vi = (int)v0, hi = (int)h;
  const float r2 = r * r;
  const float num = (nc[0] * q[0] + nc[1] * q[1]) + nc[2] * q[2];
  for (int dv = -hi; dv <= hi; ++dv) {
    const int j = vi + dv;
    if (j < 0 || j >= cam.H) continue;
    const float fj = (float)j;
    const float dyr = (fj - cam.cy) / cam.fy;
    for (int du = -hi; du <= hi; ++du) {
      const int i = ui + du;
      if (i < 0 || i >= cam.W) continue;
      const float fi = (float)i;
      const float dxr = (fi - cam.cx) / cam.fx;
      const float den = (nc[0] * dxr + nc[1] * dyr) + nc[2];
      const float t = num / den;
      const float ex = (t * dxr) - q[0], ey = (t * dyr) - q[1], ez = t - q[2];
      const float d2 = (ex * ex + ey * ey) + ez * ez;
      if (fabsf(den) > 1e-6f && t > 0.0f && d2 <= r2) {
        const float eu = fi - u, ev = fj - v;
        fn(j * cam.W + i, t, eu * eu + ev * ev);
      }
    }
  }
}

__global__ __launch_bounds__(256) void map_fill_u32_kernel(uint32_t* z, int n, uint32_t value) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < n) z[p] = value;
}

__global__ __launch_bounds__(256) void map_splat_depth_kernel(MapDev m, XformF cw, MapCam cam, uint32_t* zmin) {
  const int n = *m.count;
  for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256)
    splat_visit(m, s, cw, cam, [&](int pix, float t, float) { atomicMin(&zmin[pix], __float_as_uint(t)); });
}

__global__ __launch_bounds__(256) void map_splat_front_kernel(MapDev m, XformF cw, MapCam cam, float band,
                                                              const uint32_t* zmin, uint64_t* keys) {
  const int n = *m.count;
  for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256)
    splat_visit(m, s, cw, cam, [&](int pix, float t, float d2c) {
      if (t <= __uint_as_float(zmin[pix]) + band)
        atomicMin((unsigned long long*)&keys[pix], (unsigned long long)map_key(d2c, (uint32_t)s));
    });
}

// The winner's depth at its pixel, by the same operations as splat_visit.
__device__ __forceinline__ float splat_depth_at(const MapDev& m, int s, const XformF& cw, const MapCam& cam, int i,
                                                int j) {
  float q[3], nc[3];
  map_xform(cw, m.f[MAP_PX][s], m.f[MAP_PY][s], m.f[MAP_PZ][s], q);
  map_rotate(cw, m.f[MAP_NX][s], m.f[MAP_NY][s], m.f[MAP_NZ][s], nc);
  const float num = (nc[0] * q[0] + nc[1] * q[1]) + nc[2] * q[2];
  const float dyr = ((float)j - cam.cy) / cam.fy;
  const float dxr = ((float)i - cam.cx) / cam.fx;
  const float den = (nc[0] * dxr + nc[1] * dyr) + nc[2];
  return num / den;
}

__global__ __launch_bounds__(256) void map_resolve_kernel(MapDev m, XformF cw, MapCam cam, const uint64_t* keys,
                                                          float* depth, uint8_t* inten, float* nx, float* ny,
                                                          float* nz) {
  const int npx = cam.W * cam.H;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= npx) return;
  const uint64_t key = keys[p];
  float d = 0.0f, n[3] = {0.0f, 0.0f, 0.0f};
  uint8_t I = 0;
  if (key != MAP_EMPTY) {
    const int s = (int)(uint32_t)(key & 0xFFFFFFFFull);
    const int j = p / cam.W, i = p - j * cam.W;
    d = splat_depth_at(m, s, cw, cam, i, j);
    const float v = rintf(m.f[MAP_I][s]);
    I = (uint8_t)fminf(fmaxf(v, 0.0f), 255.0f);
    map_rotate(cw, m.f[MAP_NX][s], m.f[MAP_NY][s], m.f[MAP_NZ][s], n);
  }
  depth[p] = d;
  inten[p] = I;
  if (nx) {
    nx[p] = n[0];
    ny[p] = n[1];
    nz[p] = n[2];
  }
}

// The model view's level-0 normals: the rendered surfel normals.
__global__ __launch_bounds__(256) void map_set_normals_kernel(LevelPtrs L, const float* nx, const float* ny,
                                                              const float* nz) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= L.W * L.H) return;
  L.N[0][p] = nx[p];
  L.N[1][p] = ny[p];
  L.N[2][p] = nz[p];
}

// Deformation of the map by a solved deformation graph: each surfel moves to
// phi(p) = sum_k w_k (A_k (p - g_k) + g_k + t_k) over its 4 nearest nodes
// (ties by index; w_k = (1 - d_k / d_5)^2 normalised, equal if all vanish)
// and its normal to the normalised sum_k w_k A_k n, in float64, rounded once.
// node: 3 positions then 12 parameters (A row-major, t) per node.
constexpr int MAP_DEF_K = 4, MAP_DEF_MAX_NODES = 256;

__global__ __launch_bounds__(256) void map_deform_kernel(MapDev m, const double* node, int N) {
  const int n = *m.count;
  for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256) {
    const double v[3] = {m.f[MAP_PX][s], m.f[MAP_PY][s], m.f[MAP_PZ][s]};
    // the five nearest nodes by (distance, index), by insertion
    double bd[MAP_DEF_K + 1];
    int bi[MAP_DEF_K + 1];
    for (int k = 0; k <= MAP_DEF_K; ++k) {
      bd[k] = 1e300;
      bi[k] = N;
    }
    for (int l = 0; l < N; ++l) {
      const double* g = node + 15 * l;
      const double dx = v[0] - g[0], dy = v[1] - g[1], dz = v[2] - g[2];
      const double d = sqrt(dx * dx + dy * dy + dz * dz);
      if (!(d < bd[MAP_DEF_K] || (d == bd[MAP_DEF_K] && l < bi[MAP_DEF_K]))) continue;
      int k = MAP_DEF_K;
      while (k > 0 && (d < bd[k - 1] || (d == bd[k - 1] && l < bi[k - 1]))) {
        bd[k] = bd[k - 1];
        bi[k] = bi[k - 1];
        --k;
      }
      bd[k] = d;
      bi[k] = l;
    }
    if (bi[MAP_DEF_K] >= N) continue;  // (non-finite position: left as it is)
    double w[MAP_DEF_K], sw = 0.0;
    for (int k = 0; k < MAP_DEF_K; ++k) {
      const double a = 1.0 - bd[k] / bd[MAP_DEF_K];
      w[k] = a * a;
      sw += w[k];
    }
    const double nv[3] = {m.f[MAP_NX][s], m.f[MAP_NY][s], m.f[MAP_NZ][s]};
    double P[3] = {0.0, 0.0, 0.0}, Q[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < MAP_DEF_K; ++k) {
      const double wk = sw > 0.0 ? w[k] / sw : 1.0 / MAP_DEF_K;
      const double* g = node + 15 * bi[k];
      const double* A = g + 3;
      const double dv[3] = {v[0] - g[0], v[1] - g[1], v[2] - g[2]};
      for (int a = 0; a < 3; ++a) {
        P[a] += wk * (A[3 * a] * dv[0] + A[3 * a + 1] * dv[1] + A[3 * a + 2] * dv[2] + g[a] + A[9 + a]);
        Q[a] += wk * (A[3 * a] * nv[0] + A[3 * a + 1] * nv[1] + A[3 * a + 2] * nv[2]);
      }
    }
    const double ln = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]);
    m.f[MAP_PX][s] = (float)P[0];
    m.f[MAP_PY][s] = (float)P[1];
    m.f[MAP_PZ][s] = (float)P[2];
    if (ln > 0.0) {
      m.f[MAP_NX][s] = (float)(Q[0] / ln);
      m.f[MAP_NY][s] = (float)(Q[1] / ln);
      m.f[MAP_NZ][s] = (float)(Q[2] / ln);
    }
  }
}

}  // namespace dslam

// ---------------------------------------------------------------------------
// C ABI (include/dslam.h)
// ---------------------------------------------------------------------------
using namespace dslam;

struct dslam_map {
  dslam_context* ctx;
  dslam_camera cam;
  dslam_map_params prm;
  MapCam mc;
  uint64_t bytes;
  void* arena;
  MapDev dev;
  uint64_t* keys;        // W x H
  uint32_t* zmin;        // W x H (prediction: nearest depth, float bits)
  uint8_t* flags;        // W x H
  int32_t* block_new;    // scan blocks
  int32_t* block_off;
  float* depth;          // rendered model view, W x H
  uint8_t* inten;
  float* nrm[3];         // its camera-frame normals, W x H each
  double* def_nodes;     // deformation nodes: position and parameters, 15 doubles each
  int nb;
  hipEvent_t done;
  std::mutex mu;
};

#define MAP_HIP(expr)                                \
  do {                                               \
    if ((expr) != hipSuccess) return DSLAM_ERR_DEVICE; \
  } while (0)

static size_t map_align(size_t n) { return (n + 255) & ~size_t(255); }

static bool map_pose_ok(const double* T) {
  if (!T) return false;
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(T[i])) return false;
  return true;
}

// Camera-to-world (wc) and world-to-camera (cw) float32 transforms of the
// float64 pose T_WC (row-major 4x4), each entry rounded once.
static void map_transforms(const double* T, XformF* wc, XformF* cw) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      wc->D[3 * r + c] = (float)(T[4 * r + c] - (r == c ? 1.0 : 0.0));
      cw->D[3 * r + c] = (float)(T[4 * c + r] - (r == c ? 1.0 : 0.0));
    }
  for (int i = 0; i < 3; ++i) {
    wc->t[i] = (float)T[4 * i + 3];
    cw->t[i] = (float)(-((T[4 * 0 + i] * T[3] + T[4 * 1 + i] * T[7]) + T[4 * 2 + i] * T[11]));
  }
}

static int map_grid(int capacity) {
  const int b = (capacity + 255) / 256;
  return b < 4096 ? (b > 0 ? b : 1) : 4096;
}

extern "C" {

dslam_status dslam_map_create(dslam_context* ctx, const dslam_camera* cam, const dslam_map_params* p,
                              dslam_map** out) {
  if (!ctx || !cam || !p || !out || p->capacity < 1 || cam->width < 2 || cam->height < 2) return DSLAM_ERR_INVALID;
  if (!(p->assoc_dist > 0.0f) || !(p->assoc_cos >= -1.0f && p->assoc_cos <= 1.0f) || !(p->render_band >= 0.0f))
    return DSLAM_ERR_INVALID;
  if ((uint64_t)cam->width * cam->height > (1u << 28)) return DSLAM_ERR_INVALID;
  const size_t npx = (size_t)cam->width * cam->height;
  const int nb = (int)((npx + MAP_SCAN - 1) / MAP_SCAN);
  const size_t field = map_align((size_t)p->capacity * sizeof(float));
  const uint64_t bytes = MAP_FIELDS * field + map_align(3 * sizeof(int32_t)) + map_align(npx * 8) +
                         map_align(npx * 4) + map_align(npx) + 2 * map_align((size_t)nb * 4) + 4 * map_align(npx * 4) +
                         map_align(npx) + map_align(MAP_DEF_MAX_NODES * 15 * sizeof(double));
  const uint64_t prev = ctx->used.fetch_add(bytes);
  if (ctx->budget && prev + bytes > ctx->budget) {
    ctx->used.fetch_sub(bytes);
    return DSLAM_ERR_NO_CAPACITY;
  }
  dslam_map* m = new (std::nothrow) dslam_map;
  if (!m) {
    ctx->used.fetch_sub(bytes);
    return DSLAM_ERR_NO_CAPACITY;
  }
  m->ctx = ctx;
  m->cam = *cam;
  m->prm = *p;
  m->mc = MapCam{(float)cam->fx, (float)cam->fy, (float)cam->cx, (float)cam->cy, cam->width, cam->height};
  m->bytes = bytes;
  m->nb = nb;
  if (hipSetDevice(ctx->device) != hipSuccess || hipMalloc(&m->arena, bytes) != hipSuccess) {
    ctx->used.fetch_sub(bytes);
    delete m;
    return DSLAM_ERR_NO_CAPACITY;
  }
  char* q = (char*)m->arena;
  for (int k = 0; k < MAP_FIELDS; ++k) { m->dev.f[k] = (float*)q; q += field; }
  int32_t* ints = (int32_t*)q; q += map_align(3 * sizeof(int32_t));
  m->dev.count = ints;
  m->dev.base = ints + 1;
  m->dev.dropped = ints + 2;
  m->dev.capacity = p->capacity;
  m->keys = (uint64_t*)q; q += map_align(npx * 8);
  m->zmin = (uint32_t*)q; q += map_align(npx * 4);
  m->flags = (uint8_t*)q; q += map_align(npx);
  m->block_new = (int32_t*)q; q += map_align((size_t)nb * 4);
  m->block_off = (int32_t*)q; q += map_align((size_t)nb * 4);
  m->depth = (float*)q; q += map_align(npx * 4);
  for (int k = 0; k < 3; ++k) { m->nrm[k] = (float*)q; q += map_align(npx * 4); }
  m->inten = (uint8_t*)q; q += map_align(npx);
  m->def_nodes = (double*)q;
  if (hipMemsetAsync(ints, 0, 3 * sizeof(int32_t), nullptr) != hipSuccess ||
      hipEventCreateWithFlags(&m->done, hipEventDisableTiming) != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) {
    (void)hipFree(m->arena);
    ctx->used.fetch_sub(bytes);
    delete m;
    return DSLAM_ERR_DEVICE;
  }
  *out = m;
  return DSLAM_OK;
}

dslam_status dslam_map_destroy(dslam_map* m) {
  if (!m) return DSLAM_ERR_INVALID;
  (void)hipSetDevice(m->ctx->device);
  (void)hipEventSynchronize(m->done);  // the map's last enqueued work (not the whole device)
  (void)hipEventDestroy(m->done);
  (void)hipFree(m->arena);
  m->ctx->used.fetch_sub(m->bytes);
  delete m;
  return DSLAM_OK;
}

static bool map_matches(const dslam_map* m, const dslam_session* s) {
  return s->cam.width == m->cam.width && s->cam.height == m->cam.height && s->cam.fx == m->cam.fx &&
         s->cam.fy == m->cam.fy && s->cam.cx == m->cam.cx && s->cam.cy == m->cam.cy && s->ctx == m->ctx;
}

dslam_status dslam_map_fuse(dslam_map* m, dslam_session* s, const double T_WC[16], void* stream) {
  if (!m || !s || !map_pose_ok(T_WC) || !map_matches(m, s)) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(m->mu);
  MAP_HIP(hipSetDevice(m->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  XformF wc, cw;
  map_transforms(T_WC, &wc, &cw);
  const int npx = m->mc.W * m->mc.H;
  if (!s->cur_normals_ok) {  // a batched step left the frame's normals out
    MAP_HIP(order_after_session(s, st));
    MAP_HIP(ensure_cur_normals(s, st));
    MAP_HIP(mark_session(s, st));
  }
  MapFrame fr;
  fr.L0 = s->cur[0];
  fr.Ln = s->levels > 1 ? s->cur[1] : s->cur[0];
  fr.sh = s->levels > 1 ? 1 : 0;
  hipLaunchKernelGGL(map_fill_kernel, dim3((npx + 255) / 256), dim3(256), 0, st, m->keys, npx);
  hipLaunchKernelGGL(map_index_kernel, dim3(map_grid(m->dev.capacity)), dim3(256), 0, st, m->dev, cw, m->mc, m->keys);
  hipLaunchKernelGGL(map_fuse_kernel, dim3(m->nb), dim3(256), 0, st, m->dev, fr, wc, m->mc, m->prm.assoc_dist,
                     m->prm.assoc_cos, (const uint64_t*)m->keys, m->flags, m->block_new);
  hipLaunchKernelGGL(map_scan_kernel, dim3(1), dim3(1024), 0, st, m->dev, (const int32_t*)m->block_new, m->nb,
                     m->block_off);
  hipLaunchKernelGGL(map_append_kernel, dim3(m->nb), dim3(256), 0, st, m->dev, fr, wc, m->mc,
                     (const uint8_t*)m->flags, (const int32_t*)m->block_off);
  MAP_HIP(hipGetLastError());
  MAP_HIP(hipEventRecord(m->done, st));
  return DSLAM_OK;
}

static dslam_status map_render_into(dslam_map* m, const double* T_WM, float* depth, uint8_t* inten, float* const* nrm,
                                    hipStream_t st) {
  XformF wc, cw;
  map_transforms(T_WM, &wc, &cw);
  const int npx = m->mc.W * m->mc.H, g = map_grid(m->dev.capacity);
  hipLaunchKernelGGL(map_fill_u32_kernel, dim3((npx + 255) / 256), dim3(256), 0, st, m->zmin, npx, 0x7F800000u);
  hipLaunchKernelGGL(map_fill_kernel, dim3((npx + 255) / 256), dim3(256), 0, st, m->keys, npx);
  hipLaunchKernelGGL(map_splat_depth_kernel, dim3(g), dim3(256), 0, st, m->dev, cw, m->mc, m->zmin);
  hipLaunchKernelGGL(map_splat_front_kernel, dim3(g), dim3(256), 0, st, m->dev, cw, m->mc, m->prm.render_band,
                     (const uint32_t*)m->zmin, m->keys);
  hipLaunchKernelGGL(map_resolve_kernel, dim3((npx + 255) / 256), dim3(256), 0, st, m->dev, cw, m->mc,
                     (const uint64_t*)m->keys, depth, inten, nrm ? nrm[0] : nullptr, nrm ? nrm[1] : nullptr,
                     nrm ? nrm[2] : nullptr);
  MAP_HIP(hipGetLastError());
  return DSLAM_OK;
}

dslam_status dslam_map_render(dslam_map* m, const double T_WM[16], float* depth_dev, uint8_t* intensity_dev,
                              void* stream) {
  if (!m || !map_pose_ok(T_WM) || !depth_dev || !intensity_dev) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(m->mu);
  MAP_HIP(hipSetDevice(m->ctx->device));
  dslam_status r = map_render_into(m, T_WM, depth_dev, intensity_dev, nullptr, (hipStream_t)stream);
  if (r != DSLAM_OK) return r;
  MAP_HIP(hipEventRecord(m->done, (hipStream_t)stream));
  return DSLAM_OK;
}

dslam_status dslam_map_predict(dslam_map* m, dslam_session* s, const double T_WM[16], void* stream) {
  if (!m || !s || !map_pose_ok(T_WM) || !map_matches(m, s)) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(m->mu);
  MAP_HIP(hipSetDevice(m->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  dslam_status r = map_render_into(m, T_WM, m->depth, m->inten, m->nrm, st);
  if (r != DSLAM_OK) return r;
  r = dslam_build_pyramid(s, DSLAM_PYR_MODEL, m->depth, m->inten, m->mc.W, T_WM, stream);
  if (r != DSLAM_OK) return r;
  const int npx = m->mc.W * m->mc.H;
  hipLaunchKernelGGL(map_set_normals_kernel, dim3((npx + 255) / 256), dim3(256), 0, st, s->model[0],
                     (const float*)m->nrm[0], (const float*)m->nrm[1], (const float*)m->nrm[2]);
  MAP_HIP(hipGetLastError());
  MAP_HIP(hipEventRecord(m->done, st));
  return DSLAM_OK;
}

dslam_status dslam_map_deform(dslam_map* m, int32_t n_nodes, const double* nodes, const double* params,
                              void* stream) {
  if (!m || !nodes || !params || n_nodes < MAP_DEF_K + 1 || n_nodes > MAP_DEF_MAX_NODES) return DSLAM_ERR_INVALID;
  for (int i = 0; i < 3 * n_nodes; ++i)
    if (!std::isfinite(nodes[i])) return DSLAM_ERR_INVALID;
  for (int i = 0; i < 12 * n_nodes; ++i)
    if (!std::isfinite(params[i])) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(m->mu);
  MAP_HIP(hipSetDevice(m->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> buf(15 * (size_t)n_nodes);
  for (int l = 0; l < n_nodes; ++l) {
    for (int i = 0; i < 3; ++i) buf[15 * l + i] = nodes[3 * l + i];
    for (int i = 0; i < 12; ++i) buf[15 * l + 3 + i] = params[12 * l + i];
  }
  MAP_HIP(hipMemcpyAsync(m->def_nodes, buf.data(), sizeof(double) * buf.size(), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(map_deform_kernel, dim3(map_grid(m->dev.capacity)), dim3(256), 0, st, m->dev,
                     (const double*)m->def_nodes, n_nodes);
  MAP_HIP(hipGetLastError());
  MAP_HIP(hipEventRecord(m->done, st));
  MAP_HIP(hipStreamSynchronize(st));  // the staging buffer is the caller's stack
  return DSLAM_OK;
}

dslam_status dslam_map_reset(dslam_map* m, void* stream) {
  if (!m) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(m->mu);
  MAP_HIP(hipSetDevice(m->ctx->device));
  hipLaunchKernelGGL(map_zero_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, m->dev.count, 3);
  MAP_HIP(hipGetLastError());
  MAP_HIP(hipEventRecord(m->done, (hipStream_t)stream));
  return DSLAM_OK;
}

dslam_status dslam_map_count(dslam_map* m, int32_t* count, int32_t* dropped) {
  if (!m || !count) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(m->mu);
  MAP_HIP(hipSetDevice(m->ctx->device));
  MAP_HIP(hipEventSynchronize(m->done));
  int32_t v[3];
  MAP_HIP(hipMemcpy(v, m->dev.count, sizeof(v), hipMemcpyDeviceToHost));
  *count = v[0];
  if (dropped) *dropped = v[2];
  return DSLAM_OK;
}

dslam_status dslam_map_copy(dslam_map* m, int32_t field, float* host_out, int32_t max_surfels) {
  if (!m || !host_out || field < 0 || field >= MAP_FIELDS || max_surfels < 0) return DSLAM_ERR_INVALID;
  int32_t n = 0;
  dslam_status r = dslam_map_count(m, &n, nullptr);
  if (r != DSLAM_OK) return r;
  if (n > max_surfels) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(m->mu);
  if (n > 0) MAP_HIP(hipMemcpy(host_out, m->dev.f[field], (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
  return DSLAM_OK;
}

}  // extern "C"
