// The dense residual pass (gfx950): association, residuals, Jacobians,
// weights and the block reduction of the per-term normal equations (Section
// IV-B/D).  Included by the translation units whose kernels run the pass
// (the plain and batched kernels, and the tracking step's kernel that runs it
// beside the state linearisation).
//
// Every operation that decides a validity bit or an association is one IEEE
// float32 operation in the order written (correctly rounded division and
// square root come from the build options of every including unit);
// multiply-adds are contracted only where written with fmaf(), whatever the
// including unit's contraction setting: the functions with mixed products and
// sums switch contraction off for their bodies, so every kernel that runs the
// pass gets the same bits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "step.h"

namespace dslam {

// ---------------------------------------------------------------------------
// Residual pass: association, residuals, Jacobians, weights and the block
// reduction of the per-term normal equations (Section IV-B/D).
// ---------------------------------------------------------------------------

// j = [k, a x k]; accumulates w j j^T (upper triangle, 21), w j e (6), w e^2
// and the inlier count.  A term that is not an inlier arrives as j = 0, e = 0,
// w = 0 and adds exact zeros, so the sums equal those over the inliers alone.
__device__ __forceinline__ void accumulate(float* acc, const float* jv, float e, float w, bool inlier) {
#pragma clang fp contract(off)
  float wj[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) wj[a] = w * jv[a];
  int k = 0;
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = a; b < 6; ++b) {
      acc[k] = fmaf(wj[a], jv[b], acc[k]);
      ++k;
    }
#pragma unroll
  for (int a = 0; a < 6; ++a) acc[21 + a] = fmaf(wj[a], e, acc[21 + a]);
  acc[27] = fmaf(w * e, e, acc[27]);
  acc[28] = acc[28] + (inlier ? 1.0f : 0.0f);
}

// Value-layer reciprocal: hardware estimate (1 ulp).  No validity bit or
// association depends on it (weights and Jacobian scalings only).
__device__ __forceinline__ float rcp_v(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float huber(float s, float k) { return ((k > 0.0f) & (s > k)) ? k * rcp_v(s) : 1.0f; }

// Per-pixel sinks of the two residual terms: the plain form accumulates the
// 2 x 29 sums per thread; the precision form keeps the pixel's 16-entry row
// [sqrt(w) j_icp (6), sqrt(w) e_icp, sqrt(w) j_rgb (6), sqrt(w) e_rgb, 0, 0].
// Both receive every pixel's two terms, zeroed where the term is not an inlier.
struct SumSink {
  float* acc;
  __device__ __forceinline__ void icp(const float* jv, float e, float w, bool in) { accumulate(acc, jv, e, w, in); }
  __device__ __forceinline__ void rgb(const float* jv, float e, float w, bool in) {
    accumulate(acc + 29, jv, e, w, in);
  }
};

struct RowSink {
  float r[16];
  __device__ __forceinline__ void put(int o, const float* jv, float e, float w) {
#pragma clang fp contract(off)
    const float s = __builtin_amdgcn_sqrtf(w);  // value layer: hardware square root
#pragma unroll
    for (int c = 0; c < 6; ++c) r[o + c] = s * jv[c];
    r[o + 6] = s * e;
  }
  __device__ __forceinline__ void icp(const float* jv, float e, float w, bool) { put(0, jv, e, w); }
  __device__ __forceinline__ void rgb(const float* jv, float e, float w, bool) {
    put(7, jv, e, w);
    r[14] = 0.0f;
    r[15] = 0.0f;
  }
};

// Plane loads at a 32-bit byte offset from a uniform base (one address
// operation per pixel instead of one 64-bit add per plane).  The planes are
// device memory: the cast to the global address space lets the batched kernels,
// which read their plane pointers from memory, use global instead of flat loads.
template <class T>
__device__ __forceinline__ T ld(const T* base, unsigned byte_off) {
  typedef const __attribute__((address_space(1))) T GT;
  typedef const __attribute__((address_space(1))) char GC;
  return *(GT*)((GC*)base + byte_off);
}

// The two pass transforms (24 floats, written by the previous solve) are
// uniform: read them through the constant address space so that they arrive by
// scalar loads into scalar registers, also where the pointer itself was read
// from memory (batched launches).
__device__ __forceinline__ void load_transforms(const float* xf, float* T) {
  typedef const __attribute__((address_space(4))) float CF;
  const CF* c = (const CF*)xf;
#pragma unroll
  for (int k = 0; k < 24; ++k) T[k] = c[k];
}

// Keeps a term's value-layer outputs where it is an inlier and zeros them
// elsewhere (a select, so that NaN or infinity from a pixel that failed an
// earlier test never reaches the sums).
__device__ __forceinline__ void keep_if(bool in, float* jv, float* e, float* w) {
#pragma unroll
  for (int c = 0; c < 6; ++c) jv[c] = in ? jv[c] : 0.0f;
  *e = in ? *e : 0.0f;
  *w = in ? *w : 0.0f;
}

// Association, residuals and Jacobians.
//
// The code is straight-line: every test of the mask layer is evaluated on all
// lanes (the same IEEE operations in the same order as when nested) and the
// tests are combined with non-short-circuit '&' (so the compiler neither
// branches on them nor widens a gather offset that a branch produced), the
// model-view gathers are issued once the projections are known, and a lane
// whose projection fails a test gathers at pixel 0 instead and has that term
// zeroed (j = 0, e = 0, w = 0) before it reaches a sink.  A thread past the end
// of the image (valid = false) evaluates pixel 0 and contributes zeros.

struct Term {
  float j[6], e, w;
  bool in;  // the term is an inlier of this pixel
};

// The current pixel's vertex; zok = the pixel exists and has depth.
struct Cur {
  float x, y, z;
  unsigned o4, o2;  // byte offsets of the pixel in a float / 16-bit plane
  bool valid, zok;
};

__device__ __forceinline__ Cur load_cur(const ResidualArgs& a, int p, bool valid) {
  Cur c;
  const unsigned pv = valid ? (unsigned)p : 0u;
  c.o4 = pv * 4u;
  c.o2 = pv * 2u;
  c.x = ld(a.cV0, c.o4);
  c.y = ld(a.cV1, c.o4);
  c.z = ld(a.cV2, c.o4);
  c.valid = valid;
  c.zok = valid & (c.z > 0.0f);
  return c;
}

// ICP term (eq. (4)): projective association in the model-view camera, the
// distance and optional normal tests, e = n0 . (q - v0), j = [n0, a' x n0].
// Transforms arrive as D = R - I: q = p + (D p + t).
__device__ __forceinline__ Term icp_term(const ResidualArgs& a, const float* T, const Cur& c) {
#pragma clang fp contract(off)
  const float x = c.x, y = c.y, z = c.z;
  const float qx = x + (((T[0] * x + T[1] * y) + T[2] * z) + T[9]);
  const float qy = y + (((T[3] * x + T[4] * y) + T[5] * z) + T[10]);
  const float qz = z + (((T[6] * x + T[7] * y) + T[8] * z) + T[11]);
  const float inv = 1.0f / qz;
  const float u = ((a.fx * qx) * inv) + a.cx;
  const float v = ((a.fy * qy) * inv) + a.cy;
  const float ui = __builtin_rintf(u), vi = __builtin_rintf(v);
  const bool in = c.zok & (qz > 0.0f) & (ui >= 0.0f) & (ui <= (float)(a.W - 1)) & (vi >= 0.0f) & (vi <= (float)(a.H - 1));
  // pixel 0 where the projection failed, selected on the rounded coordinates so
  // that the offset is one unconditional 32-bit expression
  const float us = in ? ui : 0.0f, vs = in ? vi : 0.0f;
  const unsigned m4 = ((unsigned)vs * (unsigned)a.W + (unsigned)us) * 4u;
  const float v0x = ld(a.mV0, m4), v0y = ld(a.mV1, m4), v0z = ld(a.mV2, m4);
  const float n0x = ld(a.mN0, m4), n0y = ld(a.mN1, m4), n0z = ld(a.mN2, m4);
  const bool n0ok = (n0x != 0.0f) | (n0y != 0.0f) | (n0z != 0.0f);
  const float ex = qx - v0x, ey = qy - v0y, ez = qz - v0z;
  const float dist2 = (ex * ex + ey * ey) + ez * ez;
  bool ok = in & (v0z > 0.0f) & n0ok & (dist2 <= a.dist2);
  if (a.cosmin >= -1.0f) {  // optional normal-compatibility gate
    const float n1x = ld(a.cN0, c.o4), n1y = ld(a.cN1, c.o4), n1z = ld(a.cN2, c.o4);
    const bool n1ok = (n1x != 0.0f) | (n1y != 0.0f) | (n1z != 0.0f);
    const float nrx = n1x + ((T[0] * n1x + T[1] * n1y) + T[2] * n1z);
    const float nry = n1y + ((T[3] * n1x + T[4] * n1y) + T[5] * n1z);
    const float nrz = n1z + ((T[6] * n1x + T[7] * n1y) + T[8] * n1z);
    const float cosang = (nrx * n0x + nry * n0y) + nrz * n0z;
    ok = ok & n1ok & (cosang >= a.cosmin);
  }
  Term t;
  t.e = fmaf(n0x, ex, fmaf(n0y, ey, n0z * ez));
  const float px = qx - T[9], py = qy - T[10], pz = qz - T[11];
  t.j[0] = n0x;
  t.j[1] = n0y;
  t.j[2] = n0z;
  t.j[3] = fmaf(py, n0z, -pz * n0y);
  t.j[4] = fmaf(pz, n0x, -px * n0z);
  t.j[5] = fmaf(px, n0y, -py * n0x);
  const float isg = rcp_v(a.depth_k * z * z);
  const float s = fabsf(t.e) * isg;
  t.w = isg * isg * huber(s, a.huber_k);
  keep_if(ok, t.j, &t.e, &t.w);
  t.in = ok;
  return t;
}

// Photometric term (eq. (3)): warp into the reference camera, bilinear I0 and
// gradient at (u, v) from the 16-bit fixed-point planes.
__device__ __forceinline__ Term rgb_term(const ResidualArgs& a, const float* T, const Cur& c) {
#pragma clang fp contract(off)
  const float x = c.x, y = c.y, z = c.z;
  const float rx = x + (((T[12] * x + T[13] * y) + T[14] * z) + T[21]);
  const float ry = y + (((T[15] * x + T[16] * y) + T[17] * z) + T[22]);
  const float rz = z + (((T[18] * x + T[19] * y) + T[20] * z) + T[23]);
  const float inv = 1.0f / rz;
  const float u = ((a.fx * rx) * inv) + a.cx;
  const float v = ((a.fy * ry) * inv) + a.cy;
  const bool in = c.zok & (rz > 0.0f) & (u >= 1.0f) & (u < (float)(a.W - 2)) & (v >= 1.0f) & (v < (float)(a.H - 2));
  const float fu = floorf(u), fv = floorf(v);
  const unsigned m2 = in ? ((unsigned)fv * (unsigned)a.W + (unsigned)fu) * 2u : 0u, r2 = (unsigned)a.W * 2u;
  const unsigned q[4] = {m2, m2 + 2u, m2 + r2, m2 + r2 + 2u};
  float ti[4], tx[4], ty[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ti[k] = (float)ld(a.mI, q[k]);
    tx[k] = (float)ld(a.mG0, q[k]);
    ty[k] = (float)ld(a.mG1, q[k]);
  }
  const float ic = (float)ld(a.cI, c.o2);
  const float au = u - fu, av = v - fv;
  const float w00 = (1.0f - au) * (1.0f - av), w10 = au * (1.0f - av), w01 = (1.0f - au) * av, w11 = au * av;
  // taps in fixed point; the power-of-two unscaling commutes with every
  // rounding of the sum, so it is applied once to the interpolated values
  float I0 = fmaf(w00, ti[0], fmaf(w10, ti[1], fmaf(w01, ti[2], w11 * ti[3])));
  float gx = fmaf(w00, tx[0], fmaf(w10, tx[1], fmaf(w01, tx[2], w11 * tx[3])));
  float gy = fmaf(w00, ty[0], fmaf(w10, ty[1], fmaf(w01, ty[2], w11 * ty[3])));
  I0 *= 1.0f / kIntensityScale;
  gx *= 1.0f / kGradientScale;
  gy *= 1.0f / kGradientScale;
  Term t;
  t.e = I0 - ic * (1.0f / kIntensityScale);
  const float gfx = gx * a.fx * inv, gfy = gy * a.fy * inv;
  const float g2 = -fmaf(gfx, rx, gfy * ry) * inv;
  const float px = rx - T[21], py = ry - T[22], pz = rz - T[23];
  t.j[0] = gfx;
  t.j[1] = gfy;
  t.j[2] = g2;
  t.j[3] = fmaf(py, g2, -pz * gfy);
  t.j[4] = fmaf(pz, gfx, -px * g2);
  t.j[5] = fmaf(px, gfy, -py * gfx);
  const float isI = rcp_v(a.sigma_I);
  const float s = fabsf(t.e) * isI;
  t.w = huber(s, a.huber_k) * (isI * isI);
  keep_if(in, t.j, &t.e, &t.w);
  t.in = in;
  return t;
}

// Both terms of pixel p into the sink; returns the inlier bits (1 = ICP,
// 2 = photometric) and writes them to the mask when one is requested.
template <class Sink>
__device__ __forceinline__ unsigned pixel(const ResidualArgs& a, const float* T, int p, bool valid, Sink& sink) {
  const Cur c = load_cur(a, p, valid);
  const Term ti = icp_term(a, T, c);
  const Term tr = rgb_term(a, T, c);
  sink.icp(ti.j, ti.e, ti.w, ti.in);
  sink.rgb(tr.j, tr.e, tr.w, tr.in);
  const unsigned bits = (ti.in ? 1u : 0u) | (tr.in ? 2u : 0u);
  if (a.mask && valid) a.mask[p] = (uint8_t)bits;
  return bits;
}

// ---- wavefront reduction ---------------------------------------------------
// Sums N <= 32 per-lane values over the 64 lanes of a wavefront and returns
// them transposed: lanes 2q and 2q + 1 both receive the total of value q (0 for
// q >= N).  Five exchange stages each pair up the live values and halve their
// number, a sixth adds the last pair of neighbours:
//   stage 1: v_permlane32_swap of values i and i + 16 (lanes 0-31 keep value i
//            summed over l, l^32; lanes 32-63 value i + 16)
//   stage 2: v_permlane16_swap of values i and i + 8 (partner l^16)
//   stages 3-5: DPP row_mirror, row_half_mirror and quad_perm [3,2,1,0]; each
//            partner differs from the lane in bit 3, 2 or 1 (and lower bits),
//            and the lane keeps the value that its own bit selects
//   stage 6: quad_perm [1,0,3,2] adds lanes l and l^1 (both keep the total).
// After stage k a register holds, in lane l, the value whose index agrees with
// l >> 1 in the bits already exchanged; the pairing masks {32, 16, 15, 7, 3,
// 1} span all 64 lanes, so every total covers each lane once.  About 70 VALU
// instructions with no LDS round trip; the summation order is fixed.
__device__ __forceinline__ float f_of(unsigned u) { return __builtin_bit_cast(float, u); }
__device__ __forceinline__ unsigned u_of(float f) { return __builtin_bit_cast(unsigned, f); }

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

template <int H, int CTRL>
__device__ __forceinline__ void in_row_stage(const float* in, float* out, bool hi) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float keep = hi ? in[i + H] : in[i];
    const float send = hi ? in[i] : in[i + H];
    out[i] = keep + dpp<CTRL>(send);
  }
}

template <int N>
__device__ __forceinline__ float wave_transpose_sum(const float (&v)[N], int lane) {
  static_assert(N > 16 && N <= 32, "needs 17..32 values");
  float s[16], t[8], u[4], w[2], x[1];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const float b = (i + 16 < N) ? v[i + 16] : 0.0f;
    const auto r = __builtin_amdgcn_permlane32_swap(u_of(v[i]), u_of(b), false, false);
    s[i] = f_of(r[0]) + f_of(r[1]);  // lanes 0-31: value i, lanes 32-63: value i+16
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(u_of(s[i]), u_of(s[i + 8]), false, false);
    t[i] = f_of(r[0]) + f_of(r[1]);  // value i + 8 * (lane / 16)
  }
  in_row_stage<4, 0x140>(t, u, lane & 8);  // row_mirror
  in_row_stage<2, 0x141>(u, w, lane & 4);  // row_half_mirror
  in_row_stage<1, 0x1B>(w, x, lane & 2);   // quad_perm [3,2,1,0]
  return x[0] + dpp<0xB1>(x[0]);           // quad_perm [1,0,3,2]
}

// Workgroup blk of a residual pass covers pixels blk*B*ppt .. +B*ppt-1
// (B = RES_THREADS).  The plain form splits its waves by term: the first half
// accumulates the ICP sums, the second half the photometric sums, each thread
// over the 2 ppt pixels blk*B*ppt + t + (B/2) k, k = 0..2ppt-1, t = thread
// index within its half, in that order (so the sums of a session do not depend
// on whether it runs alone or in a batch).  A thread holds 29 running sums
// instead of 58, which keeps enough waves resident to cover the gathers'
// latency.
template <int PMAX>
__device__ __forceinline__ void residual_block(const ResidualArgs& a, int blk, int ppt) {
  constexpr int HALF = RES_THREADS / 2;
  __shared__ float red[RES_THREADS / 64][29];
  __shared__ uint8_t inl[2][RES_THREADS * PMAX];  // inlier bits per term (masks only)
  float T[24];
  load_transforms(a.xf, T);
  float acc[29];
#pragma unroll
  for (int k = 0; k < 29; ++k) acc[k] = 0.0f;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool rgb = threadIdx.x >= HALF;  // uniform per wavefront
  const int t = threadIdx.x - (rgb ? HALF : 0);
  const int first = blk * RES_THREADS * ppt;
#pragma unroll
  for (int k = 0; k < 2 * PMAX; ++k) {
    if (k < 2 * ppt) {  // uniform across the workgroup
      const int p = first + t + k * HALF;
      const Cur c = load_cur(a, p, p < a.npix);
      const Term tm = rgb ? rgb_term(a, T, c) : icp_term(a, T, c);
      accumulate(acc, tm.j, tm.e, tm.w, tm.in);
      if (a.mask) inl[rgb][t + k * HALF] = tm.in;
    }
  }
  const float tot = wave_transpose_sum(acc, lane);
  if ((lane & 1) == 0 && lane < 58) red[wave][lane >> 1] = tot;
  __syncthreads();
  if (threadIdx.x < 58) {
    const int term = threadIdx.x / 29, q = threadIdx.x - 29 * term, w0 = term * (HALF / 64);
    float s = red[w0][q];
#pragma unroll
    for (int w = 1; w < HALF / 64; ++w) s += red[w0 + w][q];
    a.partials[(size_t)blk * PARTIAL_STRIDE + threadIdx.x] = s;
  }
  if (a.mask) {  // uniform
    for (int i = threadIdx.x; i < RES_THREADS * ppt; i += RES_THREADS)
      if (first + i < a.npix) a.mask[first + i] = (uint8_t)(inl[0][i] | (inl[1][i] << 1));
  }
}

// ---- precision form: Jacobian rows in FP16 / BF16, J^T J on MFMA ----------
// Every pixel yields the 16-entry row q = [sqrt(w) j_icp, sqrt(w) e_icp,
// sqrt(w) j_rgb, sqrt(w) e_rgb, 0, 0] (zero for a term that is not an inlier),
// scaled per term by a power of two and rounded to 16 bits.  The Gram matrix
// G = sum q q^T holds both terms' sums in its two 7x7 diagonal blocks:
// G[a][b] = sum w j_a j_b, G[a][6] = sum w j_a e, G[6][6] = sum w e^2.
// v_mfma_f32_16x16x32_{f16,bf16} computes D = A B + C with lane l holding
// A[l % 16][8 (l / 16) + 0..7] and B[8 (l / 16) + 0..7][l % 16]; with
// A = Q^T (16 x 32 pixels) and B = Q the two operands of a lane are the same
// eight values (entry l % 16 of eight pixels), and D = Q^T Q accumulates in
// float32, lane l holding D[4 (l / 16) + r][l % 16], r = 0..3.  Rows reach
// the operand layout through a per-wave transpose in LDS.  Inlier counts come
// from ballots, so they are exact.
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// LDS staging of the rows, per wave one column of 64 pixels per row entry;
// the padding spreads the transposed reads over the LDS banks.
template <int FMT> struct Stage {
  using T = uint16_t;
  static constexpr int pitch = 64 + 8;
};
template <> struct Stage<DSLAM_JAC_FP32_MFMA> {
  using T = float;
  static constexpr int pitch = 64 + 4;
};

template <int FMT>
__device__ __forceinline__ uint16_t to16(float x) {
  if (FMT == DSLAM_JAC_FP16) {
    // saturate instead of overflowing to infinity (entries are scaled to stay far below)
    x = __builtin_fminf(__builtin_fmaxf(x, -65504.0f), 65504.0f);
    return __builtin_bit_cast(uint16_t, (_Float16)x);
  }
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}

template <int FMT>
__device__ __forceinline__ f32x4_t mfma_gram(uint4 v, f32x4_t c) {
  if (FMT == DSLAM_JAC_FP16) {
    const half8_t h = __builtin_bit_cast(half8_t, v);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(h, h, c, 0, 0, 0);
  }
  const bf16x8_t h = __builtin_bit_cast(bf16x8_t, v);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, h, c, 0, 0, 0);
}

// Contracts one wave's 64 staged rows into the Gram accumulator.
template <int FMT>
__device__ __forceinline__ f32x4_t gram_round(const typename Stage<FMT>::T* st, int lane, f32x4_t acc) {
  constexpr int P = Stage<FMT>::pitch;
  if constexpr (FMT == DSLAM_JAC_FP32_MFMA) {
    // v_mfma_f32_16x16x4_f32: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
    // MFMA m takes pixels m, 16 + m, 32 + m, 48 + m, so lane l needs entry l % 16
    // of pixels 16 (l / 16) + 0..15: four 16-byte reads
    const float* src = st + (lane & 15) * P + 16 * (lane >> 4);
    float v[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = *reinterpret_cast<const float4*>(src + 4 * q);
      v[4 * q] = t.x;
      v[4 * q + 1] = t.y;
      v[4 * q + 2] = t.z;
      v[4 * q + 3] = t.w;
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v[m], v[m], acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const uint4 v = *reinterpret_cast<const uint4*>(st + (lane & 15) * P + 32 * m + 8 * (lane >> 4));
      acc = mfma_gram<FMT>(v, acc);
    }
  }
  return acc;
}

template <int FMT>
__device__ __forceinline__ typename Stage<FMT>::T stage_entry(float x) {
  if constexpr (FMT == DSLAM_JAC_FP32_MFMA) return x;
  else return to16<FMT>(x);
}

template <int PMAX, int FMT>
__device__ __forceinline__ void residual_block_mfma(const ResidualArgs& a, int blk, int ppt) {
  using ST = typename Stage<FMT>::T;
  constexpr int P = Stage<FMT>::pitch;
  __shared__ __attribute__((aligned(16))) ST stage[RES_THREADS / 64][16 * P];
  __shared__ float gram[RES_THREADS / 64][16][17];
  __shared__ int counts[RES_THREADS / 64][2];
  float T[24];
  load_transforms(a.xf, T);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  ST* st = stage[wave];
  const float s_icp = a.col_scale[0], s_rgb = a.col_scale[1];
  f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
  int n_icp = 0, n_rgb = 0;
  const int base = blk * RES_THREADS * ppt + threadIdx.x;
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    if (k < ppt) {  // uniform across the workgroup
      const int p = base + k * RES_THREADS;
      RowSink row;
      const unsigned bits = pixel(a, T, p, p < a.npix, row);
      n_icp += __builtin_popcountll(__ballot(bits & 1));
      n_rgb += __builtin_popcountll(__ballot(bits & 2));
#pragma unroll
      for (int c = 0; c < 16; ++c) st[c * P + lane] = stage_entry<FMT>(row.r[c] * (c < 7 ? s_icp : s_rgb));
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      acc = gram_round<FMT>(st, lane, acc);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) gram[wave][4 * (lane >> 4) + r][lane & 15] = acc[r];
  if (lane == 0) {
    counts[wave][0] = n_icp;
    counts[wave][1] = n_rgb;
  }
  __syncthreads();
  if (threadIdx.x < 58) {
    const int term = threadIdx.x / 29, q = threadIdx.x % 29, o = 7 * term;
    int i = o + 6, j = o + 6;  // q == 27: sum w e^2
    if (q < 21) {              // upper triangle of the 6x6 block, row-major
      int r = 0, rem = q;
      while (rem >= 6 - r) {
        rem -= 6 - r;
        ++r;
      }
      i = o + r;
      j = o + r + rem;
    } else if (q < 27) {
      i = o + (q - 21);
    }
    float v;
    if (q == 28) {
      int n = 0;
#pragma unroll
      for (int w = 0; w < RES_THREADS / 64; ++w) n += counts[w][term];
      v = (float)n;
    } else {
      v = gram[0][i][j];
#pragma unroll
      for (int w = 1; w < RES_THREADS / 64; ++w) v += gram[w][i][j];
      const float inv = 1.0f / (term ? s_rgb : s_icp);  // exact: powers of two
      v = v * inv * inv;
    }
    a.partials[(size_t)blk * PARTIAL_STRIDE + threadIdx.x] = v;
  }
}

}  // namespace dslam
