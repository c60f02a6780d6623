// The float64 Gauss-Newton step of the tracking problem (Section IV-D/E,
// eqs. (6)-(9)), shared by the host entry point dslam_solve_step and the
// device solve kernel.
//
// Unknowns z = [dx0 (15), dx1 (15), dg (3)]; H dz = b with b = -sum J^T W e.
//
// Visual terms arrive as the residual pass's own sums over 6-vectors
// j = [k, a' x k] (k = model normal for ICP in the model-view camera, the
// projected image gradient for RGB in the reference camera; a' = the rotated
// current point).  Their world-frame Jacobians are linear images of j:
//   ICP on x1's pose:   J = P_M j,  P_M = blockdiag(R_WM, R_WM);
//   RGB on (x0, x1):    J = [P_0 M j ; P_0 j],  P_0 = blockdiag(R0, R0),
//                       M = -[[I, 0], [[t_b]x, I]],  t_b = R0^T (r1 - r0),
// which follows from the Jacobians of eq. (3) under the left perturbations of
// Section IV-A.  So H_vis = L (sum w j j^T) L^T and b_vis = -L (sum w j e).
//
// The IMU term is whitened by the Cholesky factor of its covariance (the
// inverse of W_IMU); the prior adds H* and b* - H* ((x0, q_IW) [-] xbar)
// (eq. (6) with the first-order correction of eq. (9)); the system is solved
// by Cholesky; marginalisation re-expresses b at the updated point
// (b' = b - H dz) and takes the Schur complement of the x0 block (eq. (8)).
#pragma once
#include "imu_core.h"

namespace dslam {

enum { NZ = 33 };



struct SolveParams {
  double R_WM[9], t_WM[3];
  ImuParamsD imu;
  int mode;
  int marginalise;
  int imu_fallback;      // 1: a lost RGB-D-inertial frame is re-estimated without its visual terms
  double min_inliers;    // health: level-0 inliers (both terms) below this flag LOW_INLIERS (0: off)
  double max_cost_rise;  // health: finest-level visual cost rise above this fraction flags COST_UP (0: off)
};

struct SolveWork {
  double H[NZ * NZ];   // assembled system (full symmetric)
  double L[(NZ + 1) * NZ];  // Cholesky factor (lower) with the right-hand side as row NZ; Schur workspace
  double b[NZ], y[NZ], dz[NZ];
  double J9[9 * NZ];   // IMU Jacobian rows
  double Linv[81];     // L^-1 of the preintegration covariance Sigma = L L^T
  double M9[81];       // whitening of the IMU error rows: W = M9^T M9
  double e[15];
  double Hm[2][36], gm[2][6];
  double Lr[12 * 6], LH[12 * 6], Li[12 * 6], LHi[12 * 6];
  double Y[18 * 19 > 9 * NZ ? 18 * 19 : 9 * NZ];  // scratch: whitened J9 rows, H00^-1 [H0k, b0], Schur complement
  double prior_d[18];
  double lift_src[27];  // R_WM, R0, R0 [t_b]x for the parallel lift
  double cost[4];
  ImuCommon ic;
  ImuStage is;
  int status;
};

// Unpack the 29-value sums of one term into a symmetric 6x6 and a 6-vector.
DX void unpack_term(const double* raw, double* Hm, double* gm) {
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      Hm[6 * i + j] = raw[k];
      Hm[6 * j + i] = raw[k];
      ++k;
    }
  for (int i = 0; i < 6; ++i) gm[i] = raw[21 + i];
}

// In-place Cholesky factorisation A = L L^T of the leading n x n block of A
// (leading dimension ld) into its lower triangle.  Rows n .. n+nrhs-1 hold
// right-hand sides b^T: they are carried through the elimination, so on
// return they hold (L^-1 b)^T (forward substitution for free).  Each row is
// owned by one lane; two phase barriers per column.  Returns 1 if a pivot
// was not positive and finite (the factor is then meaningless), else 0.
DX int cholesky(Par par, double* A, int n, int ld, int nrhs, int* flag) {
  SERIAL *flag = 0;
  DSLAM_SYNC();
  const int rows = n + nrhs;
  for (int k = 0; k < n; ++k) {
    double p = A[k * ld + k];
    bool good = (p > 0.0) && (p < 1e300);
    double d = good ? sqrt(p) : 1.0;
    PFOR(i, rows - k - 1) A[(k + 1 + i) * ld + k] /= d;
    SERIAL if (!good) *flag = 1;
    DSLAM_SYNC();
    SERIAL A[k * ld + k] = d;  // nobody reads the pivot in this phase
    PFOR(i, rows - k - 1) {
      int r = k + 1 + i;
      double lrk = A[r * ld + k];
      int jend = r < n ? r : n - 1;
      for (int j = k + 1; j <= jend; ++j) A[r * ld + j] -= lrk * A[j * ld + k];
    }
    DSLAM_SYNC();
  }
  return *flag;
}

// Back substitution L^T x = y for one right-hand side, y in y[] (overwritten),
// x written to x[]; one barrier per row.
DX void chol_back(Par par, const double* Lm, int n, int ld, double* y, double* x) {
  for (int k = n - 1; k >= 0; --k) {
    double xk = y[k] / Lm[k * ld + k];
    PFOR(i, k) y[i] -= Lm[k * ld + i] * xk;
    SERIAL x[k] = xk;
    DSLAM_SYNC();
  }
}

// Solve L L^T x = rhs for `nr` right-hand sides stored as columns of X (ld ldx),
// one lane per right-hand side.
DX void chol_solve_cols(Par par, const double* Lm, int n, int ld, double* X, int ldx, int nr) {
  PFOR(c, nr) {
    for (int i = 0; i < n; ++i) {
      double s = X[i * ldx + c];
      for (int k = 0; k < i; ++k) s -= Lm[i * ld + k] * X[k * ldx + c];
      X[i * ldx + c] = s / Lm[i * ld + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = X[i * ldx + c];
      for (int k = i + 1; k < n; ++k) s -= Lm[k * ld + i] * X[k * ldx + c];
      X[i * ldx + c] = s / Lm[i * ld + i];
    }
  }
  DSLAM_SYNC();
}

// Float32 transforms for the next residual pass: (R_a, t_a) = T_WM^-1 T_WC1
// and (R_b, t_b) = T_WC0^-1 T_WC1, rotations stored as R - I, each entry
// formed in float64 and rounded once to float32.
DX void next_transforms(const dslam_frame_state& x0, const dslam_frame_state& x1, const double* R_WM,
                        const double* t_WM, float* xf) {
  M3 RWM = load33(R_WM);
  M3 R0 = q2R(x0.q), R1 = q2R(x1.q);
  M3 Ra = tr(RWM) * R1;
  V3 ta = tr(RWM) * (load3(x1.r) - load3(t_WM));
  M3 Rb = tr(R0) * R1;
  V3 tb = tr(R0) * (load3(x1.r) - load3(x0.r));
  for (int i = 0; i < 9; ++i) {
    double id = (i % 4 == 0) ? 1.0 : 0.0;
    xf[i] = (float)(Ra.m[i] - id);
    xf[12 + i] = (float)(Rb.m[i] - id);
  }
  for (int i = 0; i < 3; ++i) {
    xf[9 + i] = (float)ta[i];
    xf[21 + i] = (float)tb[i];
  }
}

// Entry e (0..23) of next_transforms' output, computed on its own (the same
// operations as next_transforms performs for that entry), so 24 lanes can
// produce the transforms together.
DX float next_transform_entry(const dslam_frame_state& x0, const dslam_frame_state& x1, const double* R_WM,
                              const double* t_WM, int e) {
  const bool second = e >= 12;  // Rb, tb (reference camera) else Ra, ta (model view)
  const int q = second ? e - 12 : e;
  // the transform is L^T [R1 | r1 - o]; L and o chosen entry by entry (a choice
  // between whole private objects would put them in scratch memory)
  const M3 Lq = q2R(x0.q), Lm = load33(R_WM);
  M3 L;
  for (int k = 0; k < 9; ++k) L.m[k] = second ? Lq.m[k] : Lm.m[k];
  const M3 R1 = q2R(x1.q);
  V3 o;
  o.x = second ? x0.r[0] : t_WM[0];
  o.y = second ? x0.r[1] : t_WM[1];
  o.z = second ? x0.r[2] : t_WM[2];
  const V3 d = load3(x1.r) - o;
  // every entry with fixed indices, then a select (private arrays indexed at
  // run time would live in scratch memory)
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int i = k / 3, j = k % 3;
    const double r = L(0, i) * R1(0, j) + L(1, i) * R1(1, j) + L(2, i) * R1(2, j);
    v = (q == k) ? r - ((i == j) ? 1.0 : 0.0) : v;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) v = (q == 9 + i) ? L(0, i) * d.x + L(1, i) * d.y + L(2, i) * d.z : v;
  return (float)v;
}

// The serial tasks below read all their shared-memory operands into registers
// before their first store: the compiler cannot tell that the stores do not
// alias the later reads and would otherwise wait a round trip per statement.
DX void state_boxplus(dslam_frame_state* x, const double* d) {
  dslam_frame_state y = *x;
  double dd[15];
  for (int i = 0; i < 15; ++i) dd[i] = d[i];
  for (int i = 0; i < 3; ++i) {
    y.r[i] += dd[i];
    y.v[i] += dd[6 + i];
    y.bg[i] += dd[9 + i];
    y.ba[i] += dd[12 + i];
  }
  qboxplus(y.q, v3(dd[3], dd[4], dd[5]));
  *x = y;
}

DX void state_boxminus(const dslam_frame_state& xs, const dslam_frame_state& ys, double* d) {
  const dslam_frame_state x = xs, y = ys;  // read before the first store
  V3 a = qboxminus(x.q, y.q);
  for (int i = 0; i < 3; ++i) {
    d[i] = x.r[i] - y.r[i];
    d[3 + i] = a[i];
    d[6 + i] = x.v[i] - y.v[i];
    d[9 + i] = x.bg[i] - y.bg[i];
    d[12 + i] = x.ba[i] - y.ba[i];
  }
}

// Rows of the 12-d world Jacobian over [dr0, da0, dr1, da1] as combinations
// of the pass's 6-vector j: Li for ICP (x1 rows = P_M), Lr for RGB
// (x0 rows = P_0 M, x1 rows = P_0).  Both 12x6 row-major.
DX void build_lift(const double* R_WM, const dslam_frame_state& x0, const dslam_frame_state& x1, double* Li,
                   double* Lr) {
  M3 RWM = load33(R_WM), R0 = q2R(x0.q);
  V3 tb = tr(R0) * (load3(x1.r) - load3(x0.r));
  M3 R0Tb = R0 * hat(tb);
  for (int i = 0; i < 72; ++i) { Lr[i] = 0.0; Li[i] = 0.0; }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Li[6 * (6 + i) + j] = RWM(i, j);
      Li[6 * (9 + i) + 3 + j] = RWM(i, j);
      Lr[6 * (6 + i) + j] = R0(i, j);
      Lr[6 * (9 + i) + 3 + j] = R0(i, j);
      Lr[6 * i + j] = -R0(i, j);
      Lr[6 * (3 + i) + 3 + j] = -R0(i, j);
      Lr[6 * (3 + i) + j] = -R0Tb(i, j);
    }
}

// Host-side lift of one pass's sums to world-frame 12x12 systems per term
// (b = -L sum w j e).  Serial.
DX void lift_visual(const double* raw, const double* R_WM, const dslam_frame_state& x0, const dslam_frame_state& x1,
                    double* H_icp, double* b_icp, double* H_rgb, double* b_rgb) {
  double Li[72], Lr[72], Hm[36], gm[6];
  build_lift(R_WM, x0, x1, Li, Lr);
  for (int t = 0; t < 2; ++t) {
    unpack_term(raw + 29 * t, Hm, gm);
    const double* L = t == 0 ? Li : Lr;
    double* H = t == 0 ? H_icp : H_rgb;
    double* b = t == 0 ? b_icp : b_rgb;
    for (int i = 0; i < 12; ++i) {
      double a = 0.0;
      for (int k = 0; k < 6; ++k) a -= L[6 * i + k] * gm[k];
      b[i] = a;
      for (int j = 0; j < 12; ++j) {
        double s = 0.0;
        for (int k = 0; k < 6; ++k)
          for (int l = 0; l < 6; ++l) s += L[6 * i + k] * Hm[6 * k + l] * L[6 * j + l];
        H[12 * i + j] = s;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Dense SPD back ends.  Host: textbook Cholesky on one thread.  Device: a
// register-resident Gauss-Jordan elimination on one wavefront (solve_wave.h),
// declared here and defined by the device translation unit.
// ---------------------------------------------------------------------------
#ifdef __HIP_DEVICE_COMPILE__
__device__ int spd_solve_dev(const double* H, const double* b, int n, double* dz, double* schur);
#endif

// Linv = L^-1 for the 9x9 SPD S = L L^T (row-major; L lower triangular):
// textbook Cholesky, then forward substitution.  Returns 0, or 1 if S is not
// positive definite.  Host; the device computes it on a wavefront
// (chol_inv_lower9_wave) once per frame.
DX int chol_inv_lower9(const double* S, double* Linv) {
  double L[81] = {0.0};
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j <= i; ++j) {
      double a = S[9 * i + j];
      for (int k = 0; k < j; ++k) a -= L[9 * i + k] * L[9 * j + k];
      if (i == j) {
        if (!(a > 0.0) || !(a < 1e300)) return 1;
        L[9 * i + i] = sqrt(a);
      } else {
        L[9 * i + j] = a / L[9 * j + j];
      }
    }
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      double a = (i == j) ? 1.0 : 0.0;
      if (j > i) {
        Linv[9 * i + j] = 0.0;
        continue;
      }
      for (int k = j; k < i; ++k) a -= L[9 * i + k] * Linv[9 * k + j];
      Linv[9 * i + j] = a / L[9 * i + i];
    }
  return 0;
}

// dz = H^-1 b for the leading n x n block of H (leading dimension NZ).  If
// schur != nullptr (n == NZ), also the Schur complement of the leading 15x15
// block of [H | b]: schur (18 x 19, row-major) = [H_kk - H_k0 H_00^-1 H_0k |
// b_k - H_k0 H_00^-1 b_0].  Returns 0, or 1 if H is not SPD.
DX int spd_solve(Par par, SolveWork* w, const double* H, const double* b, int n, double* dz, double* schur) {
#ifdef __HIP_DEVICE_COMPILE__
  (void)par;
  (void)w;
  return spd_solve_dev(H, b, n, dz, schur);
#else
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) w->L[i * NZ + j] = H[i * NZ + j];
    w->L[n * NZ + i] = b[i];
  }
  if (cholesky(par, w->L, n, NZ, 1, &w->status)) return 1;
  chol_back(par, w->L, n, NZ, w->L + n * NZ, dz);
  for (int i = 0; i < n; ++i)
    if (!(dz[i] == dz[i]) || !(fabs(dz[i]) < 1e30)) return 1;
  if (schur) {
    for (int i = 0; i < 15; ++i)
      for (int j = 0; j < 15; ++j) w->L[i * NZ + j] = H[i * NZ + j];
    if (cholesky(par, w->L, 15, NZ, 0, &w->status)) return 1;
    double Z[15 * 19];  // H00^-1 [H0k, b0]
    for (int i = 0; i < 15; ++i)
      for (int c = 0; c < 19; ++c) Z[i * 19 + c] = c < 18 ? H[i * NZ + 15 + c] : b[i];
    chol_solve_cols(par, w->L, 15, NZ, Z, 19, 19);
    for (int i = 0; i < 18; ++i)
      for (int c = 0; c < 19; ++c) {
        double a = c < 18 ? H[(15 + i) * NZ + 15 + c] : b[15 + i];
        for (int k = 0; k < 15; ++k) a -= H[(15 + i) * NZ + k] * Z[k * 19 + c];
        schur[i * 19 + c] = a;
      }
  }
  return 0;
#endif
}

// One Gauss-Newton step.  raw: the 58 sums of the residual pass (ICP then RGB),
// taken at (x0, x1).  Updates x0, x1, qIW in place on success, writes the
// marginal prior if sp.marginalise.  Returns a dslam_status.
// Gyro-only mode (no accelerometer residuals): the z entries only the dropped
// rows constrain, held fixed -- x0 and x1 velocity (6-8, 21-23) and
// accelerometer bias (12-14, 27-29), and the gravity direction (30-32).
DX bool gyro_fixed(int z) {
  const int q = z < 15 ? z : z - 15;
  return z >= 30 || (q >= 6 && q < 9) || (q >= 12 && q < 15);
}

// The visual sums of one pass and the lift operators at the current states.
DX void visual_front(SolveWork* w, const double* raw, const SolveParams& sp, const dslam_frame_state& x0,
                     const dslam_frame_state& x1) {
  unpack_term(raw, w->Hm[0], w->gm[0]);
  unpack_term(raw + 29, w->Hm[1], w->gm[1]);
  w->cost[0] = raw[27];
  w->cost[1] = raw[29 + 27];
  w->cost[2] = 0.0;
  w->cost[3] = 0.0;
  build_lift(sp.R_WM, x0, x1, w->Li, w->Lr);
}

// visual_front split for the device workgroup, in three parts that run on
// different wavefronts and stages.  The lift operators depend on the states
// only, so they are built before the visual sums are reduced:
//   lift_sources: lane 0 writes the three 3x3 sources of the lift entries
//     (R_WM, R0 and R0 hat(R0^T (r1 - r0)), R0 = x0's rotation, passed in)
//     to shared memory (indexed by entry below; private arrays indexed at run
//     time would live in scratch memory);
//   lift_fill: lanes 0..nl-1 fill the 144 entries of Li and Lr from them;
//   unpack_sums: lanes 0..57 unpack the 58 sums.
DX void lift_sources(int lane, SolveWork* w, const SolveParams& sp, const M3& R0, const dslam_frame_state& x0,
                     const dslam_frame_state& x1) {
  const M3 RWM = load33(sp.R_WM);
  const V3 tb = tr(R0) * (load3(x1.r) - load3(x0.r));
  const M3 R0Tb = R0 * hat(tb);
  // one lane stores all 27 (constant offsets; a store per lane would make
  // the lanes take nine divergent branches in turn)
  double* src = w->lift_src;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      src[k] = RWM.m[k];
      src[9 + k] = R0.m[k];
      src[18 + k] = R0Tb.m[k];
    }
  }
}

// Every entry of Li and Lr is zero, a source entry or its negation; a lane
// first finds its entries' source index and sign (selects, no branches), then
// issues all of its reads, then writes.
DX void lift_fill(int lane, int nl, SolveWork* w) {
  const double* src = w->lift_src;
  constexpr int NE = 144, U = 3;
  for (int base = lane; base < NE; base += U * nl) {
    int at[U];
    bool neg[U];
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * nl;
      const int m = (idx % NE) / 72, r = (idx % 72) / 6, c = idx % 6;  // m 0: Li (ICP), 1: Lr (photometric)
      int k = -1;
      k = (r >= 6 && r < 9 && c < 3) ? 9 * m + 3 * (r - 6) + c : k;
      k = (r >= 9 && c >= 3) ? 9 * m + 3 * (r - 9) + c - 3 : k;
      const bool n1 = m == 1 && r < 3 && c < 3, n2 = m == 1 && r >= 3 && r < 6 && c >= 3,
                 n3 = m == 1 && r >= 3 && r < 6 && c < 3;
      k = n1 ? 9 + 3 * r + c : k;
      k = n2 ? 9 + 3 * (r - 3) + c - 3 : k;
      k = n3 ? 18 + 3 * (r - 3) + c : k;
      at[u] = k;
      neg[u] = n1 || n2 || n3;
      x[u] = src[k >= 0 ? k : 0];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * nl;
      if (idx < NE) {
        const int m = idx / 72, r = (idx % 72) / 6, c = idx % 6;
        const double v = at[u] < 0 ? 0.0 : (neg[u] ? -x[u] : x[u]);
        (m == 0 ? w->Li : w->Lr)[6 * r + c] = v;
      }
    }
  }
}

DX void unpack_sums(int lane, SolveWork* w, const double* raw) {
  if (lane < 58) {
    const int t = lane / 29, q = lane % 29;
    if (q < 21) {
      int r = 0, rem = q;
      while (rem >= 6 - r) {
        rem -= 6 - r;
        ++r;
      }
      w->Hm[t][6 * r + r + rem] = raw[lane];
      w->Hm[t][6 * (r + rem) + r] = raw[lane];
    } else if (q < 27) {
      w->gm[t][q - 21] = raw[lane];
    } else if (q == 27) {
      w->cost[t] = raw[lane];
    }
  }
  if (lane == 0) {
    w->cost[2] = 0.0;
    w->cost[3] = 0.0;
  }
}

// The prior's linearisation offset (x0, q_IW) [-] xbar, in two independent
// parts (the state's 15 entries, the gravity direction's 3).
DX void prior_delta_state(SolveWork* w, const dslam_prior* prior, const dslam_frame_state& x0) {
  state_boxminus(x0, prior->xbar, w->prior_d);
}
DX void prior_delta_gravity(SolveWork* w, const dslam_prior* prior, const double* qIW) {
  V3 dg = qboxminus(qIW, prior->q_IW_bar);
  w->prior_d[15] = dg.x;
  w->prior_d[16] = dg.y;
  w->prior_d[17] = dg.z;
}
DX void prior_delta(SolveWork* w, const dslam_prior* prior, const dslam_frame_state& x0, const double* qIW) {
  prior_delta_state(w, prior, x0);
  prior_delta_gravity(w, prior, qIW);
}

// Start values of the system: the prior on (x0, q_IW) with its first-order
// correction, H* and b* - H* d (eqs. (6), (9)), and the IMU bias random-walk
// rows e = b0 - b1 with J = [I at x0, -I at x1] and weight 1/(sigma_rw^2 dt)
// (RGB-D mode: zero); the visual and IMU terms are added to them.  In two
// parts: init_system_H (the matrix; also zeroes the IMU Jacobian rows) needs
// nothing of the current step, init_system_b (the right-hand
// side) needs the IMU residual e and the prior offset.
struct InitWeights {
  double wbg, wba;
  DX int pidx(int z) const { return z < 15 ? z : (z >= 30 ? z - 15 : -1); }  // z -> prior index, or -1
  DX double rw(int z) const {  // random-walk weight of a bias entry of x0 or x1, else 0
    const int q = z < 15 ? z : z - 15;
    return (z < 30 && q >= 9) ? (q < 12 ? wbg : wba) : 0.0;
  }
};

DX InitWeights init_weights(const SolveParams& sp, const dslam_preint* pre) {
  const bool full = sp.mode != DSLAM_MODE_RGBD;
  const double T = pre->dt;
  InitWeights iw;
  iw.wbg = full ? 1.0 / (sp.imu.sigma_bg_rw * sp.imu.sigma_bg_rw * T) : 0.0;
  iw.wba = (full && sp.mode != DSLAM_MODE_GYRO) ? 1.0 / (sp.imu.sigma_ba_rw * sp.imu.sigma_ba_rw * T) : 0.0;
  return iw;
}

DX void init_system_H(Par par, SolveWork* w, const SolveParams& sp, const dslam_preint* pre,
                      const dslam_prior* prior) {
  const bool full = sp.mode != DSLAM_MODE_RGBD;
  const InitWeights iw = init_weights(sp, pre);
  // U entries per lane and round: all of a lane's prior reads are issued before
  // its stores (one shared-memory round trip instead of one per entry)
  constexpr int U = 9;
  for (int base = par.lane; base < NZ * NZ; base += U * par.nl) {
    double pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * par.nl, i = idx / NZ, j = idx % NZ, pi = iw.pidx(i), pj = iw.pidx(j);
      const bool in_prior = full && idx < NZ * NZ && pi >= 0 && pj >= 0;
      const double h = prior->H[in_prior ? 18 * pi + pj : 0];
      pv[u] = in_prior ? h : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * par.nl, i = idx / NZ, j = idx % NZ;
      if (idx < NZ * NZ) {
        double a = pv[u];
        if (i == j) a += iw.rw(i);
        else if (j == i + 15 || i == j + 15) a -= iw.rw(i);  // x0 bias <-> the same x1 bias
        w->H[idx] = a;
      }
    }
  }
  PFOR(i, 9 * NZ) w->J9[i] = 0.0;
}

DX void init_system_b(Par par, SolveWork* w, const SolveParams& sp, const dslam_preint* pre,
                      const dslam_prior* prior) {
  const bool full = sp.mode != DSLAM_MODE_RGBD;
  const InitWeights iw = init_weights(sp, pre);
  PFOR(i, NZ) {
    const int pi = iw.pidx(i);
    double a = 0.0;
    if (full && pi >= 0) a = prior->b[pi] - dotN<18>(prior->H + 18 * pi, 1, w->prior_d, 1);
    if (full && iw.rw(i) != 0.0) {
      const double eb = w->e[i < 15 ? i : i - 15];  // b0 - b1 for this bias entry
      a += (i < 15 ? -iw.rw(i) : iw.rw(i)) * eb;
    }
    w->b[i] = a;
  }
}

DX void init_system(Par par, SolveWork* w, const SolveParams& sp, const dslam_preint* pre, const dslam_prior* prior) {
  init_system_H(par, w, sp, pre, prior);
  init_system_b(par, w, sp, pre, prior);
}

// Everything of one step after the visual sums are unpacked, the IMU factor's
// operands (imu_common) are computed and the system is initialised
// (init_system): assembly, solve, update and marginalisation.
DX int solve_back(Par par, SolveWork* w, const SolveParams& sp, const dslam_preint* pre, const dslam_prior* prior,
                  dslam_frame_state* x0, dslam_frame_state* x1, double* qIW, dslam_prior* marg_out);

DX int solve_step(Par par, SolveWork* w, const double* raw, const SolveParams& sp, const dslam_preint* pre,
                  const dslam_prior* prior, dslam_frame_state* x0, dslam_frame_state* x1, double* qIW,
                  dslam_prior* marg_out) {
  // ---- independent serial set-up, spread over the first lanes of the wavefronts
  if (sp.mode != DSLAM_MODE_RGBD && chol_inv_lower9(pre->Sigma, w->Linv)) return DSLAM_ERR_SINGULAR;
  TASK(3) visual_front(w, raw, sp, *x0, *x1);
  if (sp.mode != DSLAM_MODE_RGBD)
    imu_common_par(par, *x0, *x1, qIW, *pre, sp.imu, w->e, &w->ic, &w->is, [&]() { prior_delta(w, prior, *x0, qIW); });
  else
    DSLAM_SYNC();
  init_system(par, w, sp, pre, prior);
  DSLAM_SYNC();
  return solve_back(par, w, sp, pre, prior, x0, x1, qIW, marg_out);
}

// IMU term into the system: with the whitened rows M9 J9 in Y and M9 e in y,
// H += (M9 J9)^T (M9 J9), b -= (M9 J9)^T (M9 e), and the IMU cost |M9 e|^2
// plus the random-walk rows into cost[2].  Gyro-only mode holds the entries
// no remaining term constrains fixed.
DX void imu_accumulate(Par par, SolveWork* w, const SolveParams& sp, const dslam_preint* pre) {
  const bool gyro = sp.mode == DSLAM_MODE_GYRO;
  // H += (M9 J9)^T (M9 J9), b -= (M9 J9)^T (M9 e); the IMU cost |M9 e|^2 plus
  // the random-walk rows
  TASK(1) {
    double c = dotN<9>(w->y, 1, w->y, 1);
    const double T = pre->dt;
    const double wbg = 1.0 / (sp.imu.sigma_bg_rw * sp.imu.sigma_bg_rw * T);
    const double wba = gyro ? 0.0 : 1.0 / (sp.imu.sigma_ba_rw * sp.imu.sigma_ba_rw * T);
    for (int i = 0; i < 3; ++i) c += wbg * w->e[9 + i] * w->e[9 + i] + wba * w->e[12 + i] * w->e[12 + i];
    w->cost[2] = c;
  }
  // (M9 J9)^T (M9 J9) is symmetric bit for bit (entry (j, i) has the same
  // products in the same order as (i, j)), so each unordered pair is formed
  // once and added to both entries.  Items: the 33 x 17 pairs (i, i + c mod
  // 33), c = 0..16 (33 is odd: every pair i != j has one circular distance
  // of at most 16 in one direction), then the 33 right-hand-side entries; a
  // lane forms its two items' dot products together (all reads in flight)
  // before any update.
  constexpr int NPAIR = NZ * 17, NITEM = NPAIR + NZ;
  for (int base = par.lane; base < NITEM; base += 2 * par.nl) {
    int ii[2], jj[2];
    double xa[2][9], xb[2][9];
    for (int u = 0; u < 2; ++u) {
      const int it = base + u * par.nl;
      const int q = it < NITEM ? it : 0;  // a past-the-end item reads item 0 and is not applied
      const bool pair = q < NPAIR;
      const int i = pair ? q % NZ : q - NPAIR, c = pair ? q / NZ : 0;
      const int j = pair ? (i + c < NZ ? i + c : i + c - NZ) : -1;
      ii[u] = i;
      jj[u] = j;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        xa[u][k] = w->Y[k * NZ + i];
        xb[u][k] = pair ? w->Y[k * NZ + j] : w->y[k];
      }
    }
#ifdef __HIP_DEVICE_COMPILE__
    __builtin_amdgcn_sched_barrier(0);
#endif
    for (int u = 0; u < 2; ++u) {
      if (base + u * par.nl >= NITEM) continue;
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) a += xa[u][k] * xb[u][k];
      const int i = ii[u], j = jj[u];
      if (j >= 0) {
        // gyro-only: the entries no remaining term constrains are held fixed
        // (identity rows and columns, zero right-hand side)
        if (gyro && (gyro_fixed(i) || gyro_fixed(j))) {
          w->H[i * NZ + j] = (i == j) ? 1.0 : 0.0;
          w->H[j * NZ + i] = (i == j) ? 1.0 : 0.0;
        } else {
          w->H[i * NZ + j] += a;
          if (j != i) w->H[j * NZ + i] += a;
        }
      } else {
        if (gyro && gyro_fixed(i)) w->b[i] = 0.0;
        else w->b[i] -= a;
      }
    }
  }
}

DX int solve_back(Par par, SolveWork* w, const SolveParams& sp, const dslam_preint* pre, const dslam_prior* prior,
                  dslam_frame_state* x0, dslam_frame_state* x1, double* qIW, dslam_prior* marg_out) {
  const bool full = sp.mode != DSLAM_MODE_RGBD;
  const bool gyro = sp.mode == DSLAM_MODE_GYRO;
  const int n = full ? NZ : 6;
  const bool marg = full && sp.marginalise && marg_out != nullptr;
  // ---- LH = L Hm (12x6) per term; IMU Jacobian blocks and the noise map's
  // inverse operands, one entry per lane
  PFOR(idx, 72 + IMU_BLOCK_ENTRIES + 18) {
    if (idx < 72) {
      int i = idx / 6, j = idx % 6;
      w->LH[idx] = dotN<6>(w->Lr + 6 * i, 1, w->Hm[1] + j, 6);
      w->LHi[idx] = dotN<6>(w->Li + 6 * i, 1, w->Hm[0] + j, 6);
    } else if (full && idx < 72 + IMU_BLOCK_ENTRIES) {
      imu_block_entry(w->ic, idx - 72, w->J9);
    } else if (full) {
      imu_noise_inverse_entry(w->is, idx - 72 - IMU_BLOCK_ENTRIES, &w->ic);
    }
  }
  DSLAM_SYNC();
  // ---- visual 12x12 block into z indices {0..5, 15..20} (RGBD mode: only the
  // x1 pose block); the IMU whitening M9 (W = M9^T M9, see imu_whitening;
  // gyro-only: the rotation rows alone, weighted by the inverse of their
  // marginal covariance, whose Cholesky factor is the leading 3x3 block of L)
  PFOR(idx, 144 + 12 + 81) {
    if (idx < 144) {
      int i = idx / 12, j = idx % 12;
      const double a = dot2N<6>(w->LH + 6 * i, w->Lr + 6 * j, w->LHi + 6 * i, w->Li + 6 * j);
      if (full) w->H[(i < 6 ? i : 9 + i) * NZ + (j < 6 ? j : 9 + j)] += a;
      else if (i >= 6 && j >= 6) w->H[(i - 6) * NZ + (j - 6)] += a;
    } else if (idx < 156) {
      int i = idx - 144;
      double a = 0.0;
      for (int k = 0; k < 6; ++k) a -= w->Lr[6 * i + k] * w->gm[1][k] + w->Li[6 * i + k] * w->gm[0][k];
      if (full) w->b[i < 6 ? i : 9 + i] += a;
      else if (i >= 6) w->b[i - 6] += a;
    } else if (full) {
      const int q = idx - 156, i = q / 9, c = q % 9;
      w->M9[q] = (gyro && (i >= 3 || c < 3 || c >= 6)) ? 0.0 : imu_whitening(w->ic, w->Linv, i, c);
    }
  }
  DSLAM_SYNC();
  if (full) {
    // ---- IMU term: whitened rows M9 J9 (9 x 33, into Y) and M9 e (into y)
    PFOR(idx, 9 * NZ + 9) {
      if (idx < 9 * NZ) {
        const int i = idx / NZ, c = idx % NZ;
        w->Y[idx] = dotN<9>(w->M9 + 9 * i, 1, w->J9 + c, NZ);
      } else {
        const int r = idx - 9 * NZ;
        w->y[r] = dotN<9>(w->M9 + 9 * r, 1, w->e, 1);
      }
    }
    DSLAM_SYNC();
    imu_accumulate(par, w, sp, pre);
    DSLAM_SYNC();
  }
  // ---- solve H dz = b (and, on the last iteration, the Schur complement of x0)
  if (spd_solve(par, w, w->H, w->b, n, w->dz, marg ? w->Y : nullptr)) {
    SERIAL w->status = DSLAM_ERR_SINGULAR;
    DSLAM_SYNC();
    return DSLAM_ERR_SINGULAR;
  }
  // ---- box-plus updates (Section IV-D)
  if (full) {
    TASK(0) state_boxplus(x0, w->dz);
    TASK(1) state_boxplus(x1, w->dz + 15);
    TASK(2) qboxplus(qIW, v3(w->dz[30], w->dz[31], w->dz[32]));
  } else {
    SERIAL {
      double d15[15] = {w->dz[0], w->dz[1], w->dz[2], w->dz[3], w->dz[4], w->dz[5], 0, 0, 0, 0, 0, 0, 0, 0, 0};
      state_boxplus(x1, d15);
    }
  }
  // ---- marginalisation (eq. (8)) at the updated point: with b' = b - H dz,
  // S(b') = S(b) - H* dz_k, so b* = S(b) - H* dz_k
  if (marg) {
    PFOR(idx, 18 * 18 + 18) {
      if (idx < 324) {
        int i = idx / 18, j = idx % 18;
        marg_out->H[idx] = 0.5 * (w->Y[i * 19 + j] + w->Y[j * 19 + i]);
      } else {
        int i = idx - 324;
        double a = w->Y[i * 19 + 18];
        for (int k = 0; k < 18; ++k) a -= w->Y[i * 19 + k] * w->dz[15 + k];
        marg_out->b[i] = a;
      }
    }
  }
  DSLAM_SYNC();
  if (marg) {
    SERIAL {
      marg_out->xbar = *x1;
      for (int i = 0; i < 4; ++i) marg_out->q_IW_bar[i] = qIW[i];
    }
    DSLAM_SYNC();
  }
  return DSLAM_OK;
}

}  // namespace dslam
