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
};

struct SolveWork {
  double H[NZ * NZ];   // assembled system (full symmetric)
  double L[NZ * NZ];   // Cholesky factor (lower), also Schur workspace
  double b[NZ], y[NZ], dz[NZ];
  double J9[9 * NZ];   // IMU Jacobian rows (then whitened)
  double A9[81], S9[81];
  double e[15];
  double Hm[2][36], gm[2][6];
  double Lr[12 * 6], LH[12 * 6], Li[12 * 6], LHi[12 * 6];
  double Y[15 * 19];   // H00^-1 [H0k, b'0] during marginalisation
  double prior_d[18];
  double cost[4];
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

// In-place Cholesky of the n x n SPD matrix A (leading dim ld) into its lower
// triangle, on the lanes of `par`.  Returns 0, or 1 if a pivot was not positive.
DX int cholesky(Par par, double* A, int n, int ld, int* flag) {
  SERIAL *flag = 0;
  DSLAM_SYNC();
  for (int k = 0; k < n; ++k) {
    SERIAL {
      double p = A[k * ld + k];
      if (!(p > 0.0) || !(p < 1e300)) {
        *flag = 1;
        A[k * ld + k] = 1.0;
      } else {
        A[k * ld + k] = sqrt(p);
      }
    }
    DSLAM_SYNC();
    double d = A[k * ld + k];
    PFOR(i, n - k - 1) A[(k + 1 + i) * ld + k] /= d;
    DSLAM_SYNC();
    int m = n - k - 1;
    PFOR(idx, m * m) {
      int i = idx / m, j = idx % m;
      if (j <= i) A[(k + 1 + i) * ld + (k + 1 + j)] -= A[(k + 1 + i) * ld + k] * A[(k + 1 + j) * ld + k];
    }
    DSLAM_SYNC();
  }
  return *flag;
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

DX void state_boxplus(dslam_frame_state* x, const double* d) {
  for (int i = 0; i < 3; ++i) {
    x->r[i] += d[i];
    x->v[i] += d[6 + i];
    x->bg[i] += d[9 + i];
    x->ba[i] += d[12 + i];
  }
  qboxplus(x->q, v3(d[3], d[4], d[5]));
}

DX void state_boxminus(const dslam_frame_state& x, const dslam_frame_state& y, double* d) {
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

// One Gauss-Newton step.  raw: the 58 sums of the residual pass (ICP then RGB),
// taken at (x0, x1).  Updates x0, x1, qIW in place on success (lane 0 writes),
// writes the marginal prior if sp.marginalise.  Returns a dslam_status.
DX int solve_step(Par par, SolveWork* w, const double* raw, const SolveParams& sp, const dslam_preint* pre,
                  const dslam_prior* prior, dslam_frame_state* x0, dslam_frame_state* x1, double* qIW,
                  dslam_prior* marg_out) {
  const bool full = sp.mode != DSLAM_MODE_RGBD;
  const int n = full ? NZ : 6;
  SERIAL {
    unpack_term(raw, w->Hm[0], w->gm[0]);
    unpack_term(raw + 29, w->Hm[1], w->gm[1]);
    w->cost[0] = raw[27];
    w->cost[1] = raw[29 + 27];
    w->cost[2] = 0.0;
    w->cost[3] = 0.0;
    build_lift(sp.R_WM, *x0, *x1, w->Li, w->Lr);
  }
  PFOR(i, NZ * NZ) w->H[i] = 0.0;
  PFOR(i, NZ) w->b[i] = 0.0;
  DSLAM_SYNC();
  // LH = L Hm (12x6)
  PFOR(idx, 72) {
    int i = idx / 6, j = idx % 6;
    double a = 0.0, c = 0.0;
    for (int k = 0; k < 6; ++k) {
      a += w->Lr[6 * i + k] * w->Hm[1][6 * k + j];
      c += w->Li[6 * i + k] * w->Hm[0][6 * k + j];
    }
    w->LH[idx] = a;
    w->LHi[idx] = c;
  }
  DSLAM_SYNC();
  // visual 12x12 block into z indices {0..5, 15..20}; in RGBD mode only the x1 pose block
  PFOR(idx, 144) {
    int i = idx / 12, j = idx % 12;
    double a = 0.0;
    for (int k = 0; k < 6; ++k) a += w->LH[6 * i + k] * w->Lr[6 * j + k] + w->LHi[6 * i + k] * w->Li[6 * j + k];
    if (full) {
      int zi = i < 6 ? i : 9 + i, zj = j < 6 ? j : 9 + j;
      w->H[zi * NZ + zj] = a;
    } else if (i >= 6 && j >= 6) {
      w->H[(i - 6) * NZ + (j - 6)] = a;
    }
  }
  PFOR(i, 12) {
    double a = 0.0;
    for (int k = 0; k < 6; ++k) a -= w->Lr[6 * i + k] * w->gm[1][k] + w->Li[6 * i + k] * w->gm[0][k];
    if (full) w->b[i < 6 ? i : 9 + i] = a;
    else if (i >= 6) w->b[i - 6] = a;
  }
  DSLAM_SYNC();
  if (full) {
    // IMU factor: residual, Jacobian rows and noise map (serial), covariance (parallel)
    SERIAL imu_factor(*x0, *x1, qIW, *pre, sp.imu, w->e, w->J9, w->A9);
    DSLAM_SYNC();
    PFOR(idx, 81) {  // Y = A9 Sigma (in L as scratch)
      int i = idx / 9, j = idx % 9;
      double a = 0.0;
      for (int k = 0; k < 9; ++k) a += w->A9[9 * i + k] * pre->Sigma[9 * k + j];
      w->L[idx] = a;
    }
    DSLAM_SYNC();
    PFOR(idx, 81) {
      int i = idx / 9, j = idx % 9;
      double a = 0.0;
      for (int k = 0; k < 9; ++k) a += w->L[9 * i + k] * w->A9[9 * j + k];
      w->S9[idx] = a;
    }
    DSLAM_SYNC();
    int bad = cholesky(par, w->S9, 9, 9, &w->status);
    if (bad) {
      SERIAL w->status = DSLAM_ERR_SINGULAR;
      DSLAM_SYNC();
      return DSLAM_ERR_SINGULAR;
    }
    // whiten: J9 <- S^-1 J9, e9 <- S^-1 e9 (forward substitution per column)
    PFOR(c, NZ + 1) {
      for (int i = 0; i < 9; ++i) {
        double s = c < NZ ? w->J9[i * NZ + c] : w->e[i];
        for (int k = 0; k < i; ++k) s -= w->S9[9 * i + k] * (c < NZ ? w->J9[k * NZ + c] : w->e[k]);
        s /= w->S9[9 * i + i];
        if (c < NZ) w->J9[i * NZ + c] = s;
        else w->e[i] = s;
      }
    }
    DSLAM_SYNC();
    double T = pre->dt;
    double wbg = 1.0 / (sp.imu.sigma_bg_rw * sp.imu.sigma_bg_rw * T);
    double wba = 1.0 / (sp.imu.sigma_ba_rw * sp.imu.sigma_ba_rw * T);
    PFOR(idx, NZ * NZ) {
      int i = idx / NZ, j = idx % NZ;
      double a = 0.0;
      for (int k = 0; k < 9; ++k) a += w->J9[k * NZ + i] * w->J9[k * NZ + j];
      w->H[idx] += a;
    }
    PFOR(i, NZ) {
      double a = 0.0;
      for (int k = 0; k < 9; ++k) a += w->J9[k * NZ + i] * w->e[k];
      w->b[i] -= a;
    }
    DSLAM_SYNC();
    // bias random-walk rows: e = b0 - b1 with J = [I at x0, -I at x1]
    SERIAL {
      double c = 0.0;
      for (int k = 0; k < 9; ++k) c += w->e[k] * w->e[k];
      for (int i = 0; i < 3; ++i) {
        double eg = w->e[9 + i], ea = w->e[12 + i];
        int g0 = 9 + i, g1 = 24 + i, a0 = 12 + i, a1 = 27 + i;
        w->H[g0 * NZ + g0] += wbg; w->H[g1 * NZ + g1] += wbg;
        w->H[g0 * NZ + g1] -= wbg; w->H[g1 * NZ + g0] -= wbg;
        w->H[a0 * NZ + a0] += wba; w->H[a1 * NZ + a1] += wba;
        w->H[a0 * NZ + a1] -= wba; w->H[a1 * NZ + a0] -= wba;
        w->b[g0] -= wbg * eg; w->b[g1] += wbg * eg;
        w->b[a0] -= wba * ea; w->b[a1] += wba * ea;
        c += wbg * eg * eg + wba * ea * ea;
      }
      w->cost[2] = c;
      // prior: d = (x0, q_IW) [-] xbar
      state_boxminus(*x0, prior->xbar, w->prior_d);
      V3 dg = qboxminus(qIW, prior->q_IW_bar);
      w->prior_d[15] = dg.x; w->prior_d[16] = dg.y; w->prior_d[17] = dg.z;
    }
    DSLAM_SYNC();
    PFOR(idx, 18 * 18) {
      int i = idx / 18, j = idx % 18;
      int zi = i < 15 ? i : 15 + i, zj = j < 15 ? j : 15 + j;
      w->H[zi * NZ + zj] += prior->H[idx];
    }
    PFOR(i, 18) {
      double a = prior->b[i];
      for (int k = 0; k < 18; ++k) a -= prior->H[18 * i + k] * w->prior_d[k];
      w->b[i < 15 ? i : 15 + i] += a;
    }
    DSLAM_SYNC();
  }
  // Cholesky solve of H dz = b
  PFOR(idx, n * n) {
    int i = idx / n, j = idx % n;
    w->L[i * NZ + j] = w->H[i * NZ + j];
  }
  PFOR(i, n) w->dz[i] = w->b[i];
  DSLAM_SYNC();
  int bad = cholesky(par, w->L, n, NZ, &w->status);
  if (bad) {
    SERIAL w->status = DSLAM_ERR_SINGULAR;
    DSLAM_SYNC();
    return DSLAM_ERR_SINGULAR;
  }
  SERIAL {
    for (int i = 0; i < n; ++i) {
      double s = w->dz[i];
      for (int k = 0; k < i; ++k) s -= w->L[i * NZ + k] * w->dz[k];
      w->dz[i] = s / w->L[i * NZ + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = w->dz[i];
      for (int k = i + 1; k < n; ++k) s -= w->L[k * NZ + i] * w->dz[k];
      w->dz[i] = s / w->L[i * NZ + i];
    }
    bool finite = true;
    for (int i = 0; i < n; ++i) finite = finite && (w->dz[i] == w->dz[i]) && fabs(w->dz[i]) < 1e30;
    w->status = finite ? DSLAM_OK : DSLAM_ERR_SINGULAR;
    if (finite) {
      if (full) {
        state_boxplus(x0, w->dz);
        state_boxplus(x1, w->dz + 15);
        qboxplus(qIW, v3(w->dz[30], w->dz[31], w->dz[32]));
      } else {
        double d15[15] = {w->dz[0], w->dz[1], w->dz[2], w->dz[3], w->dz[4], w->dz[5], 0, 0, 0, 0, 0, 0, 0, 0, 0};
        state_boxplus(x1, d15);
      }
    }
  }
  DSLAM_SYNC();
  if (w->status != DSLAM_OK) return w->status;
  if (full && sp.marginalise && marg_out != nullptr) {
    // b' = b - H dz (re-expressed at the updated point)
    PFOR(i, NZ) {
      double a = w->b[i];
      for (int k = 0; k < NZ; ++k) a -= w->H[i * NZ + k] * w->dz[k];
      w->y[i] = a;
    }
    // Cholesky of H00 (15x15) in L
    PFOR(idx, 15 * 15) {
      int i = idx / 15, j = idx % 15;
      w->L[i * NZ + j] = w->H[i * NZ + j];
    }
    DSLAM_SYNC();
    if (cholesky(par, w->L, 15, NZ, &w->status)) {
      SERIAL w->status = DSLAM_ERR_SINGULAR;
      DSLAM_SYNC();
      return DSLAM_ERR_SINGULAR;
    }
    // Y = H00^-1 [H0k (15x18), b'0]
    PFOR(idx, 15 * 19) {
      int i = idx / 19, c = idx % 19;
      w->Y[idx] = c < 18 ? w->H[i * NZ + 15 + c] : w->y[i];
    }
    DSLAM_SYNC();
    chol_solve_cols(par, w->L, 15, NZ, w->Y, 19, 19);
    PFOR(idx, 18 * 18) {
      int i = idx / 18, j = idx % 18;
      double a = w->H[(15 + i) * NZ + 15 + j];
      for (int k = 0; k < 15; ++k) a -= w->H[(15 + i) * NZ + k] * w->Y[k * 19 + j];
      marg_out->H[idx] = a;
    }
    PFOR(i, 18) {
      double a = w->y[15 + i];
      for (int k = 0; k < 15; ++k) a -= w->H[(15 + i) * NZ + k] * w->Y[k * 19 + 18];
      marg_out->b[i] = a;
    }
    DSLAM_SYNC();
    SERIAL {
      for (int i = 0; i < 18; ++i)
        for (int j = i + 1; j < 18; ++j) {
          double a = 0.5 * (marg_out->H[18 * i + j] + marg_out->H[18 * j + i]);
          marg_out->H[18 * i + j] = a;
          marg_out->H[18 * j + i] = a;
        }
      marg_out->xbar = *x1;
      for (int i = 0; i < 4; ++i) marg_out->q_IW_bar[i] = qIW[i];
    }
    DSLAM_SYNC();
  }
  return DSLAM_OK;
}

}  // namespace dslam
