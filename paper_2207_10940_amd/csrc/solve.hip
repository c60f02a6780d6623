// Device-side frame initialisation (IMU preintegration and prediction), the
// fixed-order float64 cross-block reduction and the float64 Gauss-Newton
// solve, so that the whole coarse-to-fine iteration stays on the GPU
// (Section IV-C/D/E).  One workgroup runs each of these small kernels.
#include <hip/hip_runtime.h>
#include "step.h"
#include "solve_wave.h"

namespace dslam {

// Fixed-order float64 sum of the block partials ([nblocks][64] floats, 58
// used): thread t < REDUCE_THREADS sums the float4 column group t % 16 over
// blocks t/16, t/16 + 16, ... (RowSums, in that order; the caller may split
// the blocks into parts run between other work, the running sums staying in
// registers), stores the row sums into red (16 x 64 doubles), and after a
// barrier reduce_cols adds the 16 row sums of each column in row order.  Same
// order whatever the launch.
enum { REDUCE_THREADS = 256 };

struct RowSums {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
};

// Blocks of part `part` (0 or 1 of `parts`): this thread's u-range
// [n part / parts, n (part + 1) / parts) of its n blocks r + 16 u.
template <int CHUNK = 20>  // loads in flight at once (one round trip for up to 16 CHUNK blocks per part)
__device__ __forceinline__ void reduce_rows_part(const float* partials, int nblocks, int part, int parts,
                                                 RowSums& rs) {
  const int g = threadIdx.x & 15, r = threadIdx.x >> 4;
  const float* base = partials + 4 * g;
  const int n = nblocks > r ? (nblocks - r + 15) / 16 : 0;  // this thread sums blocks r + 16 u, u < n
  const int lo = n * part / parts, hi = n * (part + 1) / parts;
  for (int u0 = lo; u0 < hi; u0 += CHUNK) {
    float4 v[CHUNK];
#pragma unroll
    for (int u = 0; u < CHUNK; ++u) {
      const int b = r + 16 * min(u0 + u, hi - 1);  // clamped: always a valid block
      v[u] = *reinterpret_cast<const float4*>(base + (size_t)b * PARTIAL_STRIDE);
    }
#pragma unroll
    for (int u = 0; u < CHUNK; ++u) {
      if (u0 + u < hi) {
        rs.s0 += (double)v[u].x;
        rs.s1 += (double)v[u].y;
        rs.s2 += (double)v[u].z;
        rs.s3 += (double)v[u].w;
      }
    }
  }
}

// One of the two halves of the step's reduction with every load of a thread
// in flight at once up to 16 x 2 x 32 blocks: 20 loads per round trip when
// that covers the half (up to 640 blocks; fewer clamped duplicate loads), 32
// for larger images (a 1280x720 level 0 at 4 pixels per thread has 900
// blocks, which took two round trips per half at 20).
__device__ __forceinline__ void reduce_rows_half(const float* partials, int nblocks, int part, RowSums& rs) {
  if (nblocks <= 16 * 2 * 20) reduce_rows_part<20>(partials, nblocks, part, 2, rs);
  else reduce_rows_part<32>(partials, nblocks, part, 2, rs);
}

__device__ __forceinline__ void reduce_rows_store(const RowSums& rs, double* red) {
  const int g = threadIdx.x & 15, r = threadIdx.x >> 4;
  red[r * 64 + 4 * g + 0] = rs.s0;
  red[r * 64 + 4 * g + 1] = rs.s1;
  red[r * 64 + 4 * g + 2] = rs.s2;
  red[r * 64 + 4 * g + 3] = rs.s3;
}

template <int CHUNK = 20>
__device__ __forceinline__ void reduce_rows(const float* partials, int nblocks, double* red) {
  RowSums rs;
  reduce_rows_part<CHUNK>(partials, nblocks, 0, 1, rs);
  reduce_rows_store(rs, red);
}

__device__ __forceinline__ void reduce_cols(const double* red, double* out) {
  if (threadIdx.x < 58) {
    double acc = 0.0;
    for (int k = 0; k < 16; ++k) acc += red[k * 64 + threadIdx.x];
    out[threadIdx.x] = acc;
  }
}

__global__ __launch_bounds__(REDUCE_THREADS) void reduce_kernel(const float* partials, int nblocks, double* out) {
  __shared__ double red[16 * 64];
  reduce_rows(partials, nblocks, red);
  __syncthreads();
  reduce_cols(red, out);
}


// Preintegrates the frame's IMU samples at x0's bias estimate and predicts x1
// (Section IV-C); resets the frame's status and inlier counts.
__device__ __forceinline__ void frame_init_body(SessionDev* sd, const ImuBatch& batch, const FrameArgs& fa) {
  __shared__ PreintWork pw;
  __shared__ dslam_preint pre;
  __shared__ dslam_frame_state x0, x1, xp;
  __shared__ double qIW[4];
  Par par{(int)threadIdx.x, SOLVE_THREADS};
  SERIAL {
    x0 = sd->x0;
    for (int i = 0; i < 4; ++i) qIW[i] = sd->qIW[i];
    sd->status = DSLAM_OK;
  }
  DSLAM_SYNC();
  int st = DSLAM_OK;
  if (fa.mode != DSLAM_MODE_RGBD)
    st = preintegrate(par, batch.s, batch.n, batch.t0, batch.t1, x0.bg, x0.ba, fa.sigma_g, fa.sigma_a, &pw, &pre);
  if (fa.mode != DSLAM_MODE_RGBD && st == DSLAM_OK) {  // uniform
    // L^-1 of the preintegration covariance for the IMU whitening of every
    // step of this frame (wave 0), and meanwhile the prediction of x1 from
    // the measurement (first lane of wave 1; kept only if the factorisation
    // succeeds)
    __shared__ __attribute__((aligned(16))) double col[128];
    __shared__ double linv[81];
    __shared__ int lbad;
    if (threadIdx.x < 64) {
      const bool ok = chol_inv_lower9_wave(pre.Sigma, linv, (int)threadIdx.x, col);
      if (threadIdx.x == 0) lbad = ok ? 0 : 1;
    } else if (threadIdx.x == 64) {
      dslam_frame_state p = x0;
      if (fa.mode == DSLAM_MODE_GYRO) imu_predict_gyro(x0, pre, fa.imu, &p);
      else imu_predict(x0, qIW, pre, fa.imu, &p);
      xp = p;
    }
    DSLAM_SYNC();
    if (threadIdx.x < 81) sd->Linv[threadIdx.x] = linv[threadIdx.x];
    if (lbad) st = DSLAM_ERR_SINGULAR;
  }
  // all lanes publish the measurement
  if (fa.mode != DSLAM_MODE_RGBD && st == DSLAM_OK) {  // uniform
    const double* src = reinterpret_cast<const double*>(&pre);
    double* dst = reinterpret_cast<double*>(&sd->pre);
    for (int i = threadIdx.x; i < (int)(sizeof(dslam_preint) / 8); i += SOLVE_THREADS) dst[i] = src[i];
  }
  SERIAL {
    if (st != DSLAM_OK) sd->status = st;
    x1 = (fa.mode != DSLAM_MODE_RGBD && st == DSLAM_OK) ? xp : x0;
  }
  DSLAM_SYNC();
  // the first pass's transforms on 24 lanes, the state and the record's reset
  // by the first lane of wave 1
  if (threadIdx.x < 24) sd->xf[threadIdx.x] = next_transform_entry(x0, x1, fa.R_WM, fa.t_WM, (int)threadIdx.x);
  TASK(1) {
    const dslam_frame_state p = x1;
    sd->x1 = p;
    for (int l = 0; l < DSLAM_MAX_LEVELS; ++l) {
      sd->result.n_icp[l] = 0;
      sd->result.n_rgb[l] = 0;
    }
  }
  if (fa.imu_fallback) {  // uniform: the frame's start for the inertial-only fallback, one double per lane
    const int t = (int)threadIdx.x;
    if (t < 16) reinterpret_cast<double*>(&sd->x0_frame)[t] = reinterpret_cast<const double*>(&x0)[t];
    else if (t < 32) reinterpret_cast<double*>(&sd->x1_pred)[t - 16] = reinterpret_cast<const double*>(&x1)[t - 16];
    else if (t < 36) sd->qIW_frame[t - 32] = qIW[t - 32];
    const double* src = reinterpret_cast<const double*>(&sd->prior);
    double* dst = reinterpret_cast<double*>(&sd->prior_frame);
    for (int i = t; i < (int)(sizeof(dslam_prior) / 8); i += SOLVE_THREADS) dst[i] = src[i];
  }
}

// Workgroup 0 initialises the frame and stores the frame's solve parameters
// at sp_out for the step kernels; the others build the current frame's
// pyramid (cur) and, if model_tiles > 0, the model view's (model), one tile
// each, while it runs (the three touch disjoint memory).
__global__ __launch_bounds__(SOLVE_THREADS) void frame_init_pyramid_kernel(SessionDev* sd, ImuBatch batch,
                                                                           FrameArgs fa, SolveParams sp, PyrArgs cur,
                                                                           PyrArgs model, int cur_tiles,
                                                                           SolveParams* sp_out) {
  if (blockIdx.x == 0) {
    frame_init_body(sd, batch, fa);
    // one double per lane (a one-lane struct copy is lowered through scratch memory)
    static_assert(sizeof(SolveParams) % 8 == 0, "solve parameters in whole doubles");
    if (threadIdx.x < sizeof(SolveParams) / 8)
      reinterpret_cast<double*>(sp_out)[threadIdx.x] = reinterpret_cast<const double*>(&sp)[threadIdx.x];
    return;
  }
  const int t = (int)blockIdx.x - 1;
  __shared__ PyrTileBig::Lds lds;
  // (two calls rather than a select between the argument structs, which would
  // copy them to scratch memory)
  if (t < cur_tiles)
    pyramid_tile<SOLVE_THREADS, 64, 16>(cur.src, cur.L, cur.levels, cur.with_grad, t, lds, (int)threadIdx.x);
  else
    pyramid_tile<SOLVE_THREADS, 64, 16>(model.src, model.L, model.levels, model.with_grad, t - cur_tiles, lds,
                                        (int)threadIdx.x);
}
static_assert(sizeof(SessionDev*) + sizeof(ImuBatch) + sizeof(FrameArgs) + sizeof(SolveParams) + 2 * sizeof(PyrArgs) +
                  24 <= 4096,
              "frame-init arguments exceed the kernel-argument segment");

// Batched: one workgroup per session of the batch.  (The batched pyramids run
// in a launch of their own: sharing this kernel's register and LDS allocation
// would leave them a quarter of the occupancy they need at batch scale.)
__global__ __launch_bounds__(SOLVE_THREADS) void frame_init_batch_kernel(const SlotSolve* slots) {
  const SlotSolve* s = slots + blockIdx.x;
  frame_init_body(s->sd, s->imu, s->fa);
}

// One Gauss-Newton step of one session: reduce the block partials, solve,
// update the states (and on the frame's last step marginalise and publish).
// Word k (0..35) of the state triple (x0: 16 doubles, x1: 16, q_IW: 4).
static_assert(sizeof(dslam_frame_state) == 16 * sizeof(double), "state of 16 doubles");
template <class S, class D>
__device__ __forceinline__ D& state_word(S& x0, S& x1, D* q, int k) {
  D* a = reinterpret_cast<D*>(&x0);
  D* b = reinterpret_cast<D*>(&x1);
  return k < 16 ? a[k] : (k < 32 ? b[k - 16] : q[k - 32]);
}

// sp is read where it lies (the kernel argument, or the batch slot in device
// memory): a private copy of it is not promoted to registers reliably and
// then lives in scratch memory.  The marginalisation of the frame's last step
// is selected by `last` (sp.marginalise is ignored here).  With STEP_INERTIAL
// (after the frame's last step, with STEP_LAST) the step re-estimates a lost
// frame without its visual terms: from the frame's start state, its IMU
// prediction and the frame's prior, with zero visual sums; it returns at once
// unless the frame ended with tracking lost and the fallback is enabled.
__device__ __forceinline__ void solve_body(SessionDev* sd, const float* partials, const SolveParams& sp, int level,
                                           int flags, int nblocks) {
  const int last = (flags & STEP_LAST) != 0;
  const bool inertial = (flags & STEP_INERTIAL) != 0;
  if (inertial) nblocks = 0;  // no visual sums
  __shared__ SolveWork w;
  __shared__ double raw[58];
  __shared__ dslam_frame_state x0, x1;
  __shared__ double qIW[4];
  __shared__ dslam_prior marg;
  __shared__ dslam_prior prior;
  __shared__ dslam_preint pre;
  __shared__ double red[16 * 64];
  Par par{(int)threadIdx.x, SOLVE_THREADS};
  // the session's status words, read by every thread (uniform)
  const int status0 = sd->status, lost0 = sd->result.tracking_lost, health0 = sd->result.health;
  // stage the prior, the preintegrated measurement, L^-1 and the states in
  // shared memory so the serial parts never wait on global loads: one flat
  // index over the six regions (636 doubles, at most two per thread), every
  // load issued before the first store, so the whole copy is one memory
  // round trip for every wave
  {
    constexpr int NP = sizeof(dslam_prior) / 8, NQ = sizeof(dslam_preint) / 8, NL = 81, NS = 16, NG = 4;
    constexpr int NT = NP + NQ + NL + 2 * NS + NG;
    static_assert(NT <= 2 * SOLVE_THREADS, "two staged doubles per thread");
    const double* s0 = reinterpret_cast<const double*>(inertial ? &sd->prior_frame : &sd->prior);
    const double* s1 = reinterpret_cast<const double*>(&sd->pre);
    const double* s2 = sd->Linv;
    const double* s3 = reinterpret_cast<const double*>(inertial ? &sd->x0_frame : &sd->x0);
    const double* s4 = reinterpret_cast<const double*>(inertial ? &sd->x1_pred : &sd->x1);
    const double* s5 = inertial ? sd->qIW_frame : sd->qIW;
    double* d0 = reinterpret_cast<double*>(&prior);
    double* d1 = reinterpret_cast<double*>(&pre);
    double* d2 = w.Linv;
    double* d3 = reinterpret_cast<double*>(&x0);
    double* d4 = reinterpret_cast<double*>(&x1);
    double* d5 = qIW;
    auto locate = [&](int i, const double*& src, double*& dst) {
      if (i < NP) { src = s0 + i; dst = d0 + i; return; }
      i -= NP;
      if (i < NQ) { src = s1 + i; dst = d1 + i; return; }
      i -= NQ;
      if (i < NL) { src = s2 + i; dst = d2 + i; return; }
      i -= NL;
      if (i < NS) { src = s3 + i; dst = d3 + i; return; }
      i -= NS;
      if (i < NS) { src = s4 + i; dst = d4 + i; return; }
      i -= NS;
      src = s5 + i;
      dst = d5 + i;
    };
    const int i0 = (int)threadIdx.x, i1 = i0 + SOLVE_THREADS;
    const double *a0, *a1 = nullptr;
    double *b0, *b1 = nullptr;
    locate(i0, a0, b0);
    if (i1 < NT) locate(i1, a1, b1);
    const double v0 = *a0;
    const double v1 = i1 < NT ? *a1 : 0.0;
    *b0 = v0;
    if (i1 < NT) *b1 = v1;
  }
  // 2: nothing to do (an inertial re-estimate of a frame that was tracked, or
  // with the fallback off)
  int skip = status0 != DSLAM_OK;
  if (inertial)
    skip = (!skip && sp.imu_fallback && sp.mode == DSLAM_MODE_RGBDI && lost0 &&
            !(health0 & DSLAM_HEALTH_SINGULAR)) ? 0 : 2;
  DSLAM_SYNC();
  if (skip == 2) return;
  if (skip) {
    if (last) {
      if (threadIdx.x < 36) state_word(sd->result.x0, sd->result.x1, sd->result.q_IW, (int)threadIdx.x) =
          state_word(x0, x1, qIW, (int)threadIdx.x);
      SERIAL {
        sd->result.status = sd->status;
        sd->result.frame_index = sd->frame_index;
        sd->result.health = DSLAM_HEALTH_SINGULAR;
        sd->result.tracking_lost = 1;
      }
    }
    return;
  }
  const bool full = sp.mode != DSLAM_MODE_RGBD;
  // The first four waves reduce the block partials (their loads split over
  // the first two stages, the running sums in registers) while the operands
  // of the IMU factor, the prior offset and the visual lift, which depend on
  // the states only, are computed on the others (three stages, one barrier
  // sequence for both).  Wave w runs on SIMD w % 4: each stage puts its
  // longest serial task on a SIMD whose other wave has little to do.
  //   stage 0: first half of the reduction (waves 0-3); IMU rotations, operand
  //            copies and bias-corrected preintegration (waves 4-6); system
  //            matrix start (waves 4, 5); the visual lift (wave 7: sources on
  //            lane 0, then all entries)
  //   stage 1: second half of the reduction (waves 0-3); IMU residual (wave
  //            7); prior offset and the IMU operands of the stage-0 rotations
  //            (waves 4-6)
  //   stage 2: column sums, then the unpacked sums (wave 0); IMU operands of
  //            the residual (waves 4, 5, 7); right-hand side start (waves 1, 2)
  static_assert(SOLVE_THREADS == 512 && REDUCE_THREADS == 256, "stage plan assumes 8 waves");
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  RowSums rs;
  if (wave < 4) reduce_rows_half(partials, nblocks, 0, rs);
  if (full) imu_stage0(par, 4, x0, x1, qIW, pre, &w.ic, &w.is);
  if (wave == 4 || wave == 5) init_system_H(Par{lane + (wave == 5 ? 64 : 0), 128}, &w, sp, &pre, &prior);
  if (wave == 7) {
    lift_sources(lane, &w, sp, q2R(x0.q), x0, x1);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    lift_fill(lane, 64, &w);
  }
  DSLAM_SYNC();
  if (wave < 4) {
    reduce_rows_half(partials, nblocks, 1, rs);
    reduce_rows_store(rs, red);
  }
  if (full) {
    imu_stage1(par, 7, x0, x1, pre, sp.imu, w.e, &w.is);
    TASK(5) {
      prior_delta_state(&w, &prior, x0);
      imu_rotation_operands(pre, sp.imu, &w.ic, &w.is);
    }
    TASK(6) {
      prior_delta_gravity(&w, &prior, qIW);
      imu_noise_inverse_factors(pre, sp.imu, &w.is);
    }
    TASK(4) imu_krot_operands(pre, sp.imu, &w.ic, &w.is);
  }
  DSLAM_SYNC();
  if (wave == 0) {
    // the column sums and their unpacking: lane t < 58 writes and then reads
    // raw[t] only, so no barrier is needed between them
    reduce_cols(red, raw);
    if (threadIdx.x < 58) sd->sys[threadIdx.x] = raw[threadIdx.x];
    unpack_sums(lane, &w, raw);
  }
  if (full) imu_stage2(par, 4, 7, pre, sp.imu, &w.ic, &w.is, []() {});
  if (wave == 1 || wave == 2) init_system_b(Par{lane + (wave == 2 ? 64 : 0), 128}, &w, sp, &pre, &prior);
  DSLAM_SYNC();
  int st = solve_back(par, &w, sp, &pre, &prior, &x0, &x1, qIW, last ? &marg : nullptr);
  // the next pass's transforms on 24 lanes of wave 0, the states and the
  // step's record by the first lanes of waves 1 and 2
  if (st == DSLAM_OK && threadIdx.x < 24)
    sd->xf[threadIdx.x] = next_transform_entry(x0, x1, sp.R_WM, sp.t_WM, (int)threadIdx.x);
  // the states x0, x1, q_IW (16 + 16 + 4 doubles), one double per lane of
  // wave 1 (a one-lane struct copy is lowered through scratch memory)
  if (wave == 1 && lane < 36) {
    if (st == DSLAM_OK) state_word(sd->x0, sd->x1, sd->qIW, lane) = state_word(x0, x1, qIW, lane);
    else if (lane == 0) sd->status = st;
  }
  TASK(2) {
    if (!inertial) {  // the inertial re-estimate keeps the frame's visual figures
      sd->result.n_icp[level] = (int64_t)raw[28];
      sd->result.n_rgb[level] = (int64_t)raw[57];
      sd->result.cost_icp = w.cost[0];
      sd->result.cost_rgb = w.cost[1];
    }
    sd->result.cost_imu = w.cost[2];
    double nrm = 0.0;
    int n = sp.mode != DSLAM_MODE_RGBD ? NZ : 6;
    for (int i = 0; i < n; ++i) nrm += w.dz[i] * w.dz[i];
    sd->result.last_step_norm = sqrt(nrm);
    if ((flags & STEP_FIRST) && !inertial) sd->cost_first = w.cost[0] + w.cost[1];
  }
  if (last) {
    DSLAM_SYNC();
    const bool ok = st == DSLAM_OK;
    if (ok && sp.mode != DSLAM_MODE_RGBD) {  // publish the marginal prior (parallel copy)
      const double* src = reinterpret_cast<const double*>(&marg);
      double* d1 = reinterpret_cast<double*>(&sd->prior);
      double* d2 = reinterpret_cast<double*>(&sd->result.prior);
      for (int i = threadIdx.x; i < (int)(sizeof(dslam_prior) / 8); i += SOLVE_THREADS) {
        d1[i] = src[i];
        d2[i] = src[i];
      }
    }
    dslam_track_result& r = sd->result;
    // (a failed inertial re-estimate leaves the frame's joint estimate published)
    if (wave == 1 && lane < 36 && (ok || !inertial))
      state_word(r.x0, r.x1, r.q_IW, lane) = state_word(x0, x1, qIW, lane);
    // the current state becomes the previous one of the next frame
    if (ok && wave == 2 && lane < 16) reinterpret_cast<double*>(&sd->x0)[lane] = reinterpret_cast<const double*>(&x1)[lane];
    if (inertial) {
      SERIAL {
        r.health |= ok ? DSLAM_HEALTH_IMU_ONLY : DSLAM_HEALTH_SINGULAR;
        r.tracking_lost = 1;
        if (!ok) sd->status = DSLAM_OK;  // the joint estimate stands; the next frame starts normally
      }
      return;
    }
    SERIAL {
      // health of the frame (dslam_track_result.health)
      int h = ok ? 0 : DSLAM_HEALTH_SINGULAR;
      if (ok) {
        const double n_in = raw[28] + raw[57];
        if (sp.min_inliers > 0.0 && n_in < sp.min_inliers) h |= DSLAM_HEALTH_LOW_INLIERS;
        const double cv = w.cost[0] + w.cost[1];
        bool fin = isfinite(cv + w.cost[2]) && isfinite(qIW[0] + qIW[1] + qIW[2] + qIW[3]);
        const double* a = reinterpret_cast<const double*>(&x0);
        const double* b = reinterpret_cast<const double*>(&x1);
        for (int i = 0; i < 16; ++i) fin = fin && isfinite(a[i]) && isfinite(b[i]);
        if (!fin) h |= DSLAM_HEALTH_NONFINITE;
        if (sp.max_cost_rise > 0.0 && cv > (1.0 + sp.max_cost_rise) * sd->cost_first) h |= DSLAM_HEALTH_COST_UP;
      }
      r.health = h;
      r.tracking_lost = h != 0 ? 1 : 0;
      r.status = sd->status;
      if (ok) sd->frame_index += 1;
      r.frame_index = sd->frame_index;
    }
  }
}

__global__ __launch_bounds__(SOLVE_THREADS) void solve_kernel(SessionDev* sd, const float* partials, SolveArgs a) {
  solve_body(sd, partials, a.sp, a.level, a.flags, a.nblocks);
}

// The same step with the solve parameters in device memory (stored by the
// frame's first launch), so that a frame's launches after the first are the
// same at every frame and can be replayed from a captured graph.
__global__ __launch_bounds__(SOLVE_THREADS) void solve_graph_kernel(SessionDev* sd, const float* partials,
                                                                    const SolveParams* sp, int level, int flags,
                                                                    int nblocks) {
  solve_body(sd, partials, *sp, level, flags, nblocks);
}

__global__ __launch_bounds__(SOLVE_THREADS) void solve_batch_kernel(const SlotSolve* slots, int level, int flags) {
  const SlotSolve* s = slots + blockIdx.x;
  solve_body(s->sd, s->partials, s->sp, level, flags, s->nblocks[level]);
}

// Copies each session's result record into the batch's contiguous result array.
__global__ __launch_bounds__(SOLVE_THREADS) void gather_results_kernel(const SlotSolve* slots,
                                                                         dslam_track_result* out) {
  const double* src = reinterpret_cast<const double*>(&slots[blockIdx.x].sd->result);
  double* dst = reinterpret_cast<double*>(out + blockIdx.x);
  for (int i = threadIdx.x; i < (int)(sizeof(dslam_track_result) / 8); i += SOLVE_THREADS) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
hipError_t launch_solve(SessionDev* sd, const float* partials, const SolveArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(solve_kernel, dim3(1), dim3(SOLVE_THREADS), 0, st, sd, partials, a);
  return hipGetLastError();
}

hipError_t launch_solve_graph(SessionDev* sd, const float* partials, const SolveParams* sp, int level, int flags,
                              int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(solve_graph_kernel, dim3(1), dim3(SOLVE_THREADS), 0, st, sd, partials, sp, level, flags, nblocks);
  return hipGetLastError();
}

hipError_t launch_reduce(const float* partials, int nblocks, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(REDUCE_THREADS), 0, st, partials, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_frame_init_pyramid(SessionDev* sd, const ImuBatch& b, const FrameArgs& fa, const SolveParams& sp,
                                     const PyrArgs& cur, const PyrArgs* model, SolveParams* sp_out, hipStream_t st) {
  const int ct = PyrTileBig::tiles(cur.L[0].W, cur.L[0].H);
  const int mt = model ? PyrTileBig::tiles(model->L[0].W, model->L[0].H) : 0;
  hipLaunchKernelGGL(frame_init_pyramid_kernel, dim3(1 + ct + mt), dim3(SOLVE_THREADS), 0, st, sd, b, fa, sp, cur,
                     model ? *model : cur, ct, sp_out);
  return hipGetLastError();
}

hipError_t launch_frame_init_batch(const SlotSolve* slots, int n, hipStream_t st) {
  hipLaunchKernelGGL(frame_init_batch_kernel, dim3(n), dim3(SOLVE_THREADS), 0, st, slots);
  return hipGetLastError();
}

hipError_t launch_solve_batch(const SlotSolve* slots, int n, int level, int flags, hipStream_t st) {
  hipLaunchKernelGGL(solve_batch_kernel, dim3(n), dim3(SOLVE_THREADS), 0, st, slots, level, flags);
  return hipGetLastError();
}

hipError_t launch_gather_results(const SlotSolve* slots, int n, dslam_track_result* out, hipStream_t st) {
  hipLaunchKernelGGL(gather_results_kernel, dim3(n), dim3(SOLVE_THREADS), 0, st, slots, out);
  return hipGetLastError();
}

}  // namespace dslam
