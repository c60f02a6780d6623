// IMU preintegration and the IMU error term (Section IV-C, eq. (5)), float64,
// shared by the host entry points and the device kernels.
//
// Preintegration: zero-order hold over the sub-intervals of [t0, t1); within a
// sub-interval of length dt the held rate w and specific force a integrate
// exactly:
//   dp <- dp + dv dt + dR G2(w dt) a dt^2,  dv <- dv + dR G1(w dt) a dt,
//   dR <- dR Exp(w dt),  G1 = sum [phi]^k/(k+1)!,  G2 = sum [phi]^k/(k+2)!.
// The error state (dphi, dv, dp), with dR <- dR Exp(dphi), is propagated
// with the analytic step Jacobians: bias Jacobians J <- A J + B and noise
// covariance Sigma <- A Sigma A^T + B diag(sigma^2/dt) B^T.
//
// Code in this file runs on one thread or on the lanes of one workgroup: loops
// written PFOR are split across lanes, SERIAL blocks run on lane 0 and
// DSLAM_SYNC() separates phases (a no-op on the host).
#pragma once
#include "mathx.h"
#include "../../include/dslam.h"

#ifdef __HIP_DEVICE_COMPILE__
#define DSLAM_SYNC() __syncthreads()
#else
#define DSLAM_SYNC() ((void)0)
#endif
#define PFOR(i, n) for (int i = par.lane; i < (n); i += par.nl)
#define SERIAL if (par.lane == 0)

namespace dslam {

struct Par {
  int lane, nl;
};

// Coefficients of G1, G2 and their theta-derivatives divided by theta:
// c1 = (1-cos)/t^2, c2 = (t-sin)/t^3, c3 = (t^2/2+cos-1)/t^4 and d_i = c_i'(t)/t.
// Taylor series below 0.25 rad, where the closed forms cancel.
DX void gamma_coeffs(double th, double* c, double* d) {
  double t2 = th * th;
  if (th < 0.25) {
    double t4 = t2 * t2, t6 = t4 * t2;
    c[0] = 0.5 - t2 / 24.0 + t4 / 720.0 - t6 / 40320.0;
    c[1] = 1.0 / 6.0 - t2 / 120.0 + t4 / 5040.0 - t6 / 362880.0;
    c[2] = 1.0 / 24.0 - t2 / 720.0 + t4 / 40320.0 - t6 / 3628800.0;
    d[0] = -1.0 / 12.0 + t2 / 180.0 - t4 / 6720.0 + t6 / 453600.0;
    d[1] = -1.0 / 60.0 + t2 / 1260.0 - t4 / 60480.0 + t6 / 4989600.0;
    d[2] = -1.0 / 360.0 + t2 / 10080.0 - t4 / 604800.0 + t6 / 59875200.0;
    return;
  }
  double s = sin(th), co = cos(th), t3 = t2 * th, t4 = t2 * t2, t5 = t4 * th, t6 = t4 * t2;
  c[0] = (1.0 - co) / t2;
  c[1] = (th - s) / t3;
  c[2] = (0.5 * t2 + co - 1.0) / t4;
  d[0] = s / t3 - 2.0 * (1.0 - co) / t4;
  d[1] = (1.0 - co) / t4 - 3.0 * (th - s) / t5;
  d[2] = (th - s) / t5 - 4.0 * (0.5 * t2 + co - 1.0) / t6;
}

// Gk(phi) a and its derivative with respect to phi, for Gk = k0 I + ca K + cb K^2.
DX void gamma_apply(V3 phi, V3 a, double k0, double ca, double cb, double da, double db, V3* out, M3* D) {
  V3 pa = cross(phi, a);
  V3 ppa = cross(phi, pa);
  *out = k0 * a + ca * pa + cb * ppa;
  double pda = dot(phi, a);
  M3 Dm;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double pj = phi[j];
      double v = pa[i] * da * pj + ppa[i] * db * pj;
      // d(phi x (phi x a))/dphi = (phi.a) I + phi a^T - 2 a phi^T
      v += cb * ((i == j ? pda : 0.0) + phi[i] * a[j] - 2.0 * a[i] * pj);
      Dm(i, j) = v;
    }
  M3 ha = hat(a);
  *D = Dm - ca * ha;
}

// Working storage for the preintegration (LDS on the device).
struct PreintStep {
  M3 E, Jr, G1, G2, D1, D2;  // Exp(phi), right Jacobian, G1, G2 and d(Gk a)/dphi
  V3 g1a, g2a;               // G1 a, G2 a
  M3 dR;                     // dR at the start of the step
  double dt;
};
struct PreintWork {
  PreintStep st[DSLAM_MAX_IMU_SAMPLES];
  double A[DSLAM_MAX_IMU_SAMPLES][81];
  double B[DSLAM_MAX_IMU_SAMPLES][54];
  double T[81], TB[54];
  double dR[9], dv[3], dp[3];
  int nsub;
  int ksub[DSLAM_MAX_IMU_SAMPLES];
  double dtsub[DSLAM_MAX_IMU_SAMPLES];
};

// Validates the samples and lists the zero-order-hold sub-intervals of [t0, t1).
// Returns DSLAM_OK or DSLAM_ERR_INVALID.  Serial.
DX int imu_subintervals(const dslam_imu_sample* s, int n, double t0, double t1, PreintWork* w) {
  if (n < 1 || n > DSLAM_MAX_IMU_SAMPLES || !(t1 > t0) || !(s[0].t <= t0)) return DSLAM_ERR_INVALID;
  for (int k = 1; k < n; ++k)
    if (!(s[k].t > s[k - 1].t)) return DSLAM_ERR_INVALID;
  int m = 0;
  for (int k = 0; k < n; ++k) {
    double a = s[k].t > t0 ? s[k].t : t0;
    double b = (k + 1 < n && s[k + 1].t < t1) ? s[k + 1].t : t1;
    if (b > a) {
      w->ksub[m] = k;
      w->dtsub[m] = b - a;
      ++m;
    }
  }
  w->nsub = m;
  return m > 0 ? DSLAM_OK : DSLAM_ERR_INVALID;
}

// Preintegration over [t0, t1) at biases (bg, ba).  Runs on the lanes of `par`
// (one lane per sub-interval for the step quantities, then the covariance and
// bias-Jacobian recursions split over matrix entries); `out` and `w` are
// visible to all lanes.  Returns DSLAM_OK / DSLAM_ERR_INVALID.
DX int preintegrate(Par par, const dslam_imu_sample* s, int n, double t0, double t1, const double* bg,
                    const double* ba, double sigma_g, double sigma_a, PreintWork* w, dslam_preint* out) {
  SERIAL {
    int st = imu_subintervals(s, n, t0, t1, w);
    if (st != DSLAM_OK) w->nsub = -1;
  }
  PFOR(i, 81) out->Sigma[i] = 0.0;
  PFOR(i, 54) out->J[i] = 0.0;
  DSLAM_SYNC();
  const int nsub = w->nsub;
  if (nsub < 0) return DSLAM_ERR_INVALID;
  // per-step quantities, independent across steps, in three independent
  // parts (the Gamma terms, Exp, the right Jacobian): index 64 part + m, so
  // that on the device each part runs on a wavefront of its own (nsub <= 33)
  PFOR(i, 3 * 64) {
    const int part = i >> 6, m = i & 63;
    if (m < nsub) {
      const dslam_imu_sample& smp = s[w->ksub[m]];
      const double dt = w->dtsub[m];
      const V3 wv = v3(smp.gyro[0] - bg[0], smp.gyro[1] - bg[1], smp.gyro[2] - bg[2]);
      const V3 phi = dt * wv;
      PreintStep& P = w->st[m];
      if (part == 0) {
        const V3 av = v3(smp.acc[0] - ba[0], smp.acc[1] - ba[1], smp.acc[2] - ba[2]);
        double c[3], d[3];
        gamma_coeffs(norm(phi), c, d);
        gamma_apply(phi, av, 1.0, c[0], c[1], d[0], d[1], &P.g1a, &P.D1);
        gamma_apply(phi, av, 0.5, c[1], c[2], d[1], d[2], &P.g2a, &P.D2);
        M3 K = hat(phi);
        P.G1 = eye3() + c[0] * K + c[1] * (K * K);
        P.G2 = 0.5 * eye3() + c[1] * K + c[2] * (K * K);
        P.dt = dt;
      } else if (part == 1) {
        P.E = Exp(phi);
      } else {
        P.Jr = Jr(phi);
      }
    }
  }
  DSLAM_SYNC();
  // the rotation chain and the integrated velocity and position (cheap, serial)
  SERIAL {
    M3 dR = eye3();
    V3 dv = v3(0, 0, 0), dp = v3(0, 0, 0);
    for (int m = 0; m < nsub; ++m) {
      PreintStep& P = w->st[m];
      double dt = P.dt;
      P.dR = dR;
      dp = dp + dt * dv + (dt * dt) * (dR * P.g2a);
      dv = dv + dt * (dR * P.g1a);
      dR = dR * P.E;
    }
    for (int i = 0; i < 9; ++i) w->dR[i] = dR.m[i];
    store3(w->dv, dv);
    store3(w->dp, dp);
  }
  DSLAM_SYNC();
  // step Jacobians A (error state [dphi, dv, dp]) and B (biases [bg, ba]), in
  // three parts writing disjoint entries (A; B's gyro columns; B's
  // accelerometer columns), each part on a wavefront of its own as above
  PFOR(i, 3 * 64) {
    const int part = i >> 6, m = i & 63;
    if (m < nsub) {
      const PreintStep& P = w->st[m];
      const double dt = P.dt;
      double* A = w->A[m];
      double* B = w->B[m];
      if (part == 0) {
        for (int k = 0; k < 81; ++k) A[k] = (k % 10 == 0) ? 1.0 : 0.0;
        const M3 Et = tr(P.E);
        const M3 Av_phi = (-dt) * (P.dR * hat(P.g1a));
        const M3 Ap_phi = (-dt * dt) * (P.dR * hat(P.g2a));
        for (int r = 0; r < 3; ++r) {
          A[9 * (6 + r) + 3 + r] = dt;
          for (int j = 0; j < 3; ++j) {
            A[9 * r + j] = Et(r, j);
            A[9 * (3 + r) + j] = Av_phi(r, j);
            A[9 * (6 + r) + j] = Ap_phi(r, j);
          }
        }
      } else if (part == 1) {
        const M3 Bphi_g = (-dt) * P.Jr;
        const M3 Bv_g = (-dt * dt) * (P.dR * P.D1);
        const M3 Bp_g = (-dt * dt * dt) * (P.dR * P.D2);
        for (int r = 0; r < 3; ++r)
          for (int j = 0; j < 3; ++j) {
            B[6 * r + j] = Bphi_g(r, j);
            B[6 * (3 + r) + j] = Bv_g(r, j);
            B[6 * (6 + r) + j] = Bp_g(r, j);
          }
      } else {
        const M3 Bv_a = (-dt) * (P.dR * P.G1);
        const M3 Bp_a = (-dt * dt) * (P.dR * P.G2);
        for (int r = 0; r < 3; ++r)
          for (int j = 0; j < 3; ++j) {
            B[6 * r + 3 + j] = 0.0;
            B[6 * (3 + r) + 3 + j] = Bv_a(r, j);
            B[6 * (6 + r) + 3 + j] = Bp_a(r, j);
          }
      }
    }
  }
  DSLAM_SYNC();
  // Sigma <- A Sigma A^T + B diag(sigma^2/dt) B^T,  J <- A J + B
  for (int m = 0; m < nsub; ++m) {
    const double* A = w->A[m];
    const double* B = w->B[m];
    PFOR(idx, 81 + 54) {
      if (idx < 81) {
        int i = idx / 9, j = idx % 9;
        w->T[idx] = dotN<9>(A + 9 * i, 1, out->Sigma + j, 9);
      } else {
        int q = idx - 81, i = q / 6, j = q % 6;
        w->TB[q] = dotN<9>(A + 9 * i, 1, out->J + j, 6);
      }
    }
    DSLAM_SYNC();
    double dt = w->st[m].dt;
    double vg = sigma_g * sigma_g / dt, va = sigma_a * sigma_a / dt;
    PFOR(idx, 81 + 54) {
      if (idx < 81) {
        int i = idx / 9, j = idx % 9;
        const double acc = dotN<9>(w->T + 9 * i, 1, A + 9 * j, 1);
        const double q = dotN<3>(B + 6 * i, 1, B + 6 * j, 1);
        const double r = dotN<3>(B + 6 * i + 3, 1, B + 6 * j + 3, 1);
        out->Sigma[idx] = acc + vg * q + va * r;
      } else {
        out->J[idx - 81] = w->TB[idx - 81] + B[idx - 81];
      }
    }
    DSLAM_SYNC();
  }
  // the measurement and the symmetrised covariance, entry by entry
  PFOR(q, 9 + 12 + 1 + 36) {
    if (q < 9) {
      out->dR[q] = w->dR[q];
    } else if (q < 21) {
      const int i = (q - 9) % 3, k = (q - 9) / 3;
      if (k == 0) out->dv[i] = w->dv[i];
      else if (k == 1) out->dp[i] = w->dp[i];
      else if (k == 2) out->bg[i] = bg[i];
      else out->ba[i] = ba[i];
    } else if (q == 21) {
      out->dt = t1 - t0;
    } else {
      int i = 0, r = q - 22;  // pair r of the upper triangle (i < j), row by row
      while (r >= 8 - i) {
        r -= 8 - i;
        ++i;
      }
      const int j = i + 1 + r;
      const double a = 0.5 * (out->Sigma[9 * i + j] + out->Sigma[9 * j + i]);
      out->Sigma[9 * i + j] = a;
      out->Sigma[9 * j + i] = a;
    }
  }
  DSLAM_SYNC();
  return DSLAM_OK;
}

struct ImuParamsD {
  double gravity, sigma_bg_rw, sigma_ba_rw;
  double R_CS[9], t_CS[3];
};

// Quantities shared by the IMU error and its Jacobian blocks.
struct ImuCommon {
  // operands of the Jacobian blocks (see imu_block_entry) and of the noise
  // map's inverse; mats[0] is the identity
  M3 mats[27];
  double T;
};

// indices into ImuCommon::mats
enum {
  IC_I = 0, IC_NEG_I, IC_HAT_R0YR, IC_QT, IC_S, IC_JPG, IC_KROT, IC_JRG, IC_JPA, IC_JRA, IC_HAT_YG, IC_JLI, IC_KAL,
  IC_JRI, IC_Q, IC_HAT_SDV, IC_QS, IC_JVG, IC_JVA, IC_HAT_QSDV,
  // the noise map's inverse (see imu_whitening)
  IC_YI, IC_ST, IC_QST, IC_SXY, IC_COUNT
};

enum { IMU_BLOCKS = 17 };

// IMU error e = x1_hat(x0) [-] x1 (eq. (5)), ordered [r, alpha, v, bg, ba]
// (the staged form below also produces the Jacobian operands).  The derivation uses the left perturbations of Section IV-A; with
// S = R0 R_CS, dR~ = dR Exp(J_R db) and y_r = t_CS + R_CS dp~ - R_CS dR~ R_CS^T t_CS:
//   r_hat = r0 + R0 y_r + R_IW^T (v0 T + g T^2/2),
//   R_hat = S dR~ R_CS^T,  v_hat = v0 + g T + R_IW S dv~.
// Serial.
DX void imu_common(const dslam_frame_state& x0, const dslam_frame_state& x1, const double* qIW,
                   const dslam_preint& pre, const ImuParamsD& ip, double* e) {
  M3 R0 = q2R(x0.q), R1 = q2R(x1.q), Q = q2R(qIW);
  M3 Rcs = load33(ip.R_CS);
  V3 tcs = load3(ip.t_CS);
  V3 g = v3(0.0, 0.0, -ip.gravity);
  double T = pre.dt;
  double db[6];
  for (int i = 0; i < 3; ++i) {
    db[i] = x0.bg[i] - pre.bg[i];
    db[3 + i] = x0.ba[i] - pre.ba[i];
  }
  // first-order bias correction
  double pb[3], dvt[3], dpt[3];
  for (int i = 0; i < 3; ++i) {
    double a = 0.0, bv = 0.0, bp = 0.0;
    for (int k = 0; k < 6; ++k) {
      a += pre.J[6 * i + k] * db[k];
      bv += pre.J[6 * (3 + i) + k] * db[k];
      bp += pre.J[6 * (6 + i) + k] * db[k];
    }
    pb[i] = a;
    dvt[i] = pre.dv[i] + bv;
    dpt[i] = pre.dp[i] + bp;
  }
  V3 phib = load3(pb);
  M3 Rb = Exp(phib);
  M3 dRt = load33(pre.dR) * Rb;
  V3 dvv = load3(dvt), dpv = load3(dpt);
  M3 S = R0 * Rcs;
  M3 SdRt = S * dRt;
  M3 Rh1 = SdRt * tr(Rcs);
  V3 wt = tr(Rcs) * tcs;
  V3 v0 = load3(x0.v), r0 = load3(x0.r);
  M3 Qt = tr(Q);
  V3 yg = T * v0 + (0.5 * T * T) * g;
  V3 yr = tcs + Rcs * dpv - Rcs * (dRt * wt);
  V3 rh = r0 + R0 * yr + Qt * yg;
  V3 Sdv = S * dvv;
  V3 QSdv = Q * Sdv;
  V3 vh = v0 + T * g + QSdv;
  V3 ea = Log(Rh1 * tr(R1));
  V3 er = rh - load3(x1.r);
  V3 ev = vh - load3(x1.v);
  for (int i = 0; i < 3; ++i) {
    e[i] = er[i];
    e[3 + i] = ea[i];
    e[6 + i] = ev[i];
    e[9 + i] = x0.bg[i] - x1.bg[i];
    e[12 + i] = x0.ba[i] - x1.ba[i];
  }
}

// Intermediates of imu_common_par shared between its lanes.
struct ImuStage {
  M3 R0, R1, Q, Rb, Jrb, SdRt, Jli;
  M3 G, K, Jl;  // noise-map inverse operands: Y^-1 = G Jl, S^T X Y^-1 = -K Jl
  M3 SdRtJrb;   // S dR~ Jr(phi_b)
  V3 phib, dvt, dpt, ea, yr, yg, Sdv, QSdv;
};

// Independent serial tasks run on the first lane of different wavefronts
// (concurrently on the device, one after the other on the host).
DX int task_lane(Par par, int t) { return t * 64 < par.nl ? t * 64 : 0; }
#define TASK(t) if (par.lane == task_lane(par, (t)))

// imu_common split into three stages over the first lanes of the wavefronts
// tb, tb + 1, tb + 2 (and tb + 3 for `side`): the three rotations and the
// bias-corrected preintegration first, then the residual, then the Jacobian
// operands.  Same arithmetic as imu_common.  The caller separates the stages
// by barriers (imu_common_par below, or a caller that interleaves other work).
DX void imu_stage0(Par par, int tb, const dslam_frame_state& x0, const dslam_frame_state& x1, const double* qIW,
                   const dslam_preint& pre, ImuCommon* c, ImuStage* t) {
  // the operands that are copies of the preintegration's bias Jacobians and
  // the constant blocks, one entry per lane
  PFOR(q, 54 + 18) {
    M3* m = c->mats;
    if (q < 54) {
      const int r = q / 6, k = q % 6, blk = r / 3, i = r % 3, j = k % 3;
      const int id = blk == 0 ? (k < 3 ? IC_JRG : IC_JRA) : (blk == 1 ? (k < 3 ? IC_JVG : IC_JVA)
                                                                     : (k < 3 ? IC_JPG : IC_JPA));
      m[id](i, j) = pre.J[q];
    } else {
      const int e = q - 54, i = (e % 9) / 3, j = e % 3;
      m[e < 9 ? IC_I : IC_NEG_I](i, j) = e < 9 ? (i == j ? 1.0 : 0.0) : (i == j ? -1.0 : 0.0);
    }
  }
  TASK(tb) {
    double q0[4];
    for (int i = 0; i < 4; ++i) q0[i] = x0.q[i];
    t->R0 = q2R(q0);
    c->T = pre.dt;
  }
  TASK(tb + 1) {
    t->R1 = q2R(x1.q);
    t->Q = q2R(qIW);
  }
  TASK(tb + 2) {
    double db[6];
    for (int i = 0; i < 3; ++i) {
      db[i] = x0.bg[i] - pre.bg[i];
      db[3 + i] = x0.ba[i] - pre.ba[i];
    }
    double pb[3], dvt[3], dpt[3];
    for (int i = 0; i < 3; ++i) {
      double a = 0.0, bv = 0.0, bp = 0.0;
      for (int k = 0; k < 6; ++k) {
        a += pre.J[6 * i + k] * db[k];
        bv += pre.J[6 * (3 + i) + k] * db[k];
        bp += pre.J[6 * (6 + i) + k] * db[k];
      }
      pb[i] = a;
      dvt[i] = pre.dv[i] + bv;
      dpt[i] = pre.dp[i] + bp;
    }
    t->phib = load3(pb);
    t->dvt = load3(dvt);
    t->dpt = load3(dpt);
    t->Rb = Exp(t->phib);
    t->Jrb = Jr(t->phib);
  }
}

// The IMU residual in three independent parts (position, rotation,
// velocity; the bias rows are differences), each one serial task, with the
// operands the Jacobian blocks reuse.  imu_stage1 runs them on one lane.
DX void imu_residual_r(const dslam_frame_state& x0, const dslam_frame_state& x1, const dslam_preint& pre,
                       const ImuParamsD& ip, double* e, ImuStage* t) {
  const M3 R0 = t->R0, Q = t->Q, Rb = t->Rb, dR = load33(pre.dR);
  const V3 dpt = t->dpt, v0 = load3(x0.v), r0 = load3(x0.r), r1 = load3(x1.r);
  const M3 Rcs = load33(ip.R_CS);
  const V3 tcs = load3(ip.t_CS);
  const V3 g = v3(0.0, 0.0, -ip.gravity);
  const double T = pre.dt;
  const M3 dRt = dR * Rb;
  const V3 wt = tr(Rcs) * tcs;
  const V3 yg = T * v0 + (0.5 * T * T) * g;
  const V3 yr = tcs + Rcs * dpt - Rcs * (dRt * wt);
  const V3 rh = r0 + R0 * yr + tr(Q) * yg;
  const V3 er = rh - r1;
  for (int i = 0; i < 3; ++i) e[i] = er[i];
  t->yr = yr;
  t->yg = yg;
}

DX void imu_residual_a(const dslam_frame_state& x1, const dslam_preint& pre, const ImuParamsD& ip, double* e,
                       ImuStage* t) {
  const M3 R0 = t->R0, R1 = t->R1, Rb = t->Rb, dR = load33(pre.dR);
  const M3 Rcs = load33(ip.R_CS);
  const M3 dRt = dR * Rb;
  const M3 S = R0 * Rcs;
  const M3 SdRt = S * dRt;
  const M3 Rh1 = SdRt * tr(Rcs);
  const V3 ea = Log(Rh1 * tr(R1));
  for (int i = 0; i < 3; ++i) e[3 + i] = ea[i];
  t->SdRt = SdRt;
  t->ea = ea;
}

DX void imu_residual_v(const dslam_frame_state& x0, const dslam_frame_state& x1, const dslam_preint& pre,
                       const ImuParamsD& ip, double* e, ImuStage* t) {
  const M3 R0 = t->R0, Q = t->Q;
  const V3 dvt = t->dvt, v0 = load3(x0.v), v1 = load3(x1.v);
  const M3 Rcs = load33(ip.R_CS);
  const V3 g = v3(0.0, 0.0, -ip.gravity);
  const double T = pre.dt;
  const M3 S = R0 * Rcs;
  const V3 Sdv = S * dvt;
  const V3 QSdv = Q * Sdv;
  const V3 vh = v0 + T * g + QSdv;
  const V3 ev = vh - v1;
  double eb[6];  // read before the first store (see state_boxplus)
  for (int i = 0; i < 3; ++i) {
    eb[i] = x0.bg[i] - x1.bg[i];
    eb[3 + i] = x0.ba[i] - x1.ba[i];
  }
  for (int i = 0; i < 3; ++i) {
    e[6 + i] = ev[i];
    e[9 + i] = eb[i];
    e[12 + i] = eb[3 + i];
  }
  t->Sdv = Sdv;
  t->QSdv = QSdv;
}

DX void imu_stage1(Par par, int tb, const dslam_frame_state& x0, const dslam_frame_state& x1,
                   const dslam_preint& pre, const ImuParamsD& ip, double* e, ImuStage* t) {
  TASK(tb) {
    imu_residual_r(x0, x1, pre, ip, e, t);
    imu_residual_a(x1, pre, ip, e, t);
    imu_residual_v(x0, x1, pre, ip, e, t);
  }
}

// Jacobian operands that need only the stage-0 rotations, so idle lanes can
// compute them during stage 1, in two serial tasks.  With S = R0 R_CS and
// dR~ = dR Rb (the same operations as the stage-1 residual task):
// imu_rotation_operands: S, R_IW S, T R_IW^T, -R_IW and the transposes the
// noise map's inverse uses;
// imu_krot_operands: KROT = S dR~ [w]x Jr(phi_b) and S dR~ Jr(phi_b);
// imu_noise_inverse_factors: the factors of the noise map's inverse (see
// imu_whitening)
//   Y^-1 = Rb (S dR~)^T Jl(e_a) = G Jl,
//   S^T X Y^-1 = S^T (S dR~ [w]x Rb^T) Rb (S dR~)^T Jl = dR~ [w]x (S dR~)^T Jl = -K Jl
// (S^T S = Rb^T Rb = I).
DX void imu_rotation_operands(const dslam_preint& pre, const ImuParamsD& ip, ImuCommon* c, const ImuStage* t) {
  M3* m = c->mats;
  const M3 Rcs = load33(ip.R_CS);
  const M3 R0 = t->R0, Q = t->Q;
  const double T = pre.dt;
  const M3 S = R0 * Rcs;
  const M3 QS = Q * S;
  m[IC_S] = S;
  m[IC_QS] = QS;
  m[IC_QT] = T * tr(Q);
  m[IC_Q] = (-1.0) * Q;
  m[IC_ST] = tr(S);
  m[IC_QST] = tr(QS);
}

DX void imu_krot_operands(const dslam_preint& pre, const ImuParamsD& ip, ImuCommon* c, ImuStage* t) {
  const M3 Rcs = load33(ip.R_CS);
  const V3 wt = tr(Rcs) * load3(ip.t_CS);
  const M3 Rb = t->Rb, R0 = t->R0, Jrb = t->Jrb, dR = load33(pre.dR);
  const M3 SdRt = (R0 * Rcs) * (dR * Rb);
  const M3 KROT = (SdRt * hat(wt)) * Jrb, SJ = SdRt * Jrb;
  c->mats[IC_KROT] = KROT;
  t->SdRtJrb = SJ;
}

DX void imu_noise_inverse_factors(const dslam_preint& pre, const ImuParamsD& ip, ImuStage* t) {
  const M3 Rcs = load33(ip.R_CS);
  const V3 wt = tr(Rcs) * load3(ip.t_CS);
  const M3 Rb = t->Rb, R0 = t->R0, dR = load33(pre.dR);
  const M3 dRt = dR * Rb;
  const M3 SdRtT = tr((R0 * Rcs) * dRt);
  const M3 G = Rb * SdRtT;
  const M3 K = (-1.0) * ((dRt * hat(wt)) * SdRtT);
  t->G = G;
  t->K = K;
}

// Entry q (0 <= q < 18) of Y^-1 (q < 9) and of -S^T X Y^-1 (the operands
// IC_YI, IC_SXY of imu_whitening), one lane each, once Jl is known.
DX void imu_noise_inverse_entry(const ImuStage& t, int q, ImuCommon* c) {
  const int e = q % 9, i = e / 3, j = e % 3;
  const M3& F = q < 9 ? t.G : t.K;
  const double r = F(i, 0) * t.Jl(0, j) + F(i, 1) * t.Jl(1, j) + F(i, 2) * t.Jl(2, j);
  c->mats[q < 9 ? IC_YI : IC_SXY](i, j) = r;
}

// Stage 2: the operands that need the stage-1 residual, on the first lanes of
// wavefronts tb, tb + 1 and tj (tj also runs `side`).
template <class Side>
DX void imu_stage2(Par par, int tb, int tj, const dslam_preint& pre, const ImuParamsD& ip, ImuCommon* c,
                   ImuStage* t, Side side) {
  (void)pre;
  (void)ip;
  M3* m = c->mats;
  // (each task reads its operands before its first store, see state_boxplus)
  TASK(tb) {
    const V3 ea = t->ea;
    const M3 SdRtJrb = t->SdRtJrb;
    const M3 Jli = JlInv(ea);
    const M3 KAL = Jli * SdRtJrb;
    m[IC_JLI] = Jli;
    m[IC_KAL] = KAL;
    m[IC_JRI] = (-1.0) * tr(Jli);
  }
  TASK(tb + 1) {
    const M3 R0 = t->R0, Q = t->Q;
    const V3 yr = t->yr, yg = t->yg, Sdv = t->Sdv, QSdv = t->QSdv;
    const M3 A = (-1.0) * hat(R0 * yr), B = tr(Q) * hat(yg);
    m[IC_HAT_R0YR] = A;
    m[IC_HAT_YG] = B;
    m[IC_HAT_SDV] = hat(Sdv);
    m[IC_HAT_QSDV] = (-1.0) * hat(QSdv);
  }
  TASK(tj) {
    const V3 ea = t->ea;
    t->Jl = Jr((-1.0) * ea);  // Jl(a) = Jr(-a)
    side();
  }
}

template <class Side>
DX void imu_common_par(Par par, const dslam_frame_state& x0, const dslam_frame_state& x1, const double* qIW,
                       const dslam_preint& pre, const ImuParamsD& ip, double* e, ImuCommon* c, ImuStage* t,
                       Side side) {
  imu_stage0(par, 0, x0, x1, qIW, pre, c, t);
  DSLAM_SYNC();
  imu_stage1(par, 0, x0, x1, pre, ip, e, t);
  TASK(1) imu_rotation_operands(pre, ip, c, t);
  TASK(2) imu_krot_operands(pre, ip, c, t);
  TASK(3) imu_noise_inverse_factors(pre, ip, t);
  DSLAM_SYNC();
  imu_stage2(par, 0, 2, pre, ip, c, t, side);
  DSLAM_SYNC();
  PFOR(q, 18) imu_noise_inverse_entry(*t, q, c);
  DSLAM_SYNC();
}

DX void put_block(double* M, int ld, int r0, int c0, const M3& B) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[(r0 + i) * ld + c0 + j] = B(i, j);
}

// Jacobian block table: block b is J9[row, col] = A1 A2 + A3 A4 with the
// operands taken from ImuCommon::mats (the identity pads unused factors, and
// A3 A4 = 0 when A3 is IC_COUNT).
struct ImuBlockSpec {
  signed char row, col, a1, a2, a3, a4;
};

// Block b (0 <= b < IMU_BLOCKS) of the Jacobian rows J9 (9x33 over
// [x0 (15), x1 (15), dg (3)]) of the first nine IMU error entries.  J9 must be
// zero-filled first; blocks write disjoint entries.  Every block runs the same
// instructions on different operands, so lanes do not diverge.
DX ImuBlockSpec imu_block_spec(int b) {
  switch (b) {
    case 0: return {0, 0, IC_I, IC_I, IC_COUNT, 0};               // e_r / dr0 = I
    case 1: return {0, 15, IC_NEG_I, IC_I, IC_COUNT, 0};          // e_r / dr1 = -I
    case 2: return {0, 3, IC_HAT_R0YR, IC_I, IC_COUNT, 0};        // e_r / da0 = -[R0 y_r]x
    case 3: return {0, 6, IC_QT, IC_I, IC_COUNT, 0};              // e_r / dv0 = T R_IW^T
    case 4: return {0, 9, IC_S, IC_JPG, IC_KROT, IC_JRG};         // e_r / dbg0
    case 5: return {0, 12, IC_S, IC_JPA, IC_KROT, IC_JRA};        // e_r / dba0
    case 6: return {0, 30, IC_HAT_YG, IC_I, IC_COUNT, 0};         // e_r / dg = R_IW^T [y_g]x
    case 7: return {3, 3, IC_JLI, IC_I, IC_COUNT, 0};             // e_a / da0 = Jl^-1
    case 8: return {3, 9, IC_KAL, IC_JRG, IC_COUNT, 0};           // e_a / dbg0
    case 9: return {3, 12, IC_KAL, IC_JRA, IC_COUNT, 0};          // e_a / dba0
    case 10: return {3, 18, IC_JRI, IC_I, IC_COUNT, 0};           // e_a / da1 = -Jr^-1
    case 11: return {6, 6, IC_I, IC_I, IC_COUNT, 0};              // e_v / dv0 = I
    case 12: return {6, 21, IC_NEG_I, IC_I, IC_COUNT, 0};         // e_v / dv1 = -I
    case 13: return {6, 3, IC_Q, IC_HAT_SDV, IC_COUNT, 0};        // e_v / da0 = -R_IW [S dv~]x
    case 14: return {6, 9, IC_QS, IC_JVG, IC_COUNT, 0};           // e_v / dbg0
    case 15: return {6, 12, IC_QS, IC_JVA, IC_COUNT, 0};          // e_v / dba0
    default: return {6, 30, IC_HAT_QSDV, IC_I, IC_COUNT, 0};      // e_v / dg = -[R_IW S dv~]x
  }
}

// Entry q (0 <= q < IMU_BLOCK_ENTRIES) of the block table: entry (i, j) =
// (q % 9 / 3, q % 3) of block q / 9, with the arithmetic of the 3x3 products
// (A1 A2)(i, j) + (A3 A4)(i, j), so nine lanes compute a block together.
enum { IMU_BLOCK_ENTRIES = 9 * IMU_BLOCKS };
DX void imu_block_entry(const ImuCommon& c, int q, double* J9) {
  const int b = q / 9, i = (q % 9) / 3, j = q % 3;
  const ImuBlockSpec t = imu_block_spec(b);
  const M3 &a1 = c.mats[t.a1], &a2 = c.mats[t.a2];
  double r = a1(i, 0) * a2(0, j) + a1(i, 1) * a2(1, j) + a1(i, 2) * a2(2, j);
  if (t.a3 != IC_COUNT) {
    const M3 &a3 = c.mats[t.a3], &a4 = c.mats[t.a4];
    r = r + (a3(i, 0) * a4(0, j) + a3(i, 1) * a4(1, j) + a3(i, 2) * a4(2, j));
  }
  J9[(t.row + i) * 33 + t.col + j] = r;
}

// The IMU factor's weight W = (A Sigma A^T)^-1 in factored form.  The map A
// (9x9) from the preintegration noise (dphi, dv, dp) to the error rows
// (r, alpha, v) has the block structure
//   r = X dphi + S dp,  alpha = Y dphi,  v = R_IW S dv
// with X = S dR~ [w]x Rb^T, Y = Jl^-1(e_a) S dR~ Rb^T (w = R_CS^T t_CS), so
//   A^-1 = [[0, Y^-1, 0], [0, 0, (R_IW S)^T], [S^T, -S^T X Y^-1, 0]]
// (rows dphi, dv, dp; columns r, alpha, v), where every factor but Jl^-1 is a
// rotation.  With Sigma = L L^T (Cholesky, once per step) and M = L^-1 A^-1,
// W = M^T M: the whitened rows M J and M e replace the 9x9 inverse.
// Entry (i, c) of M from Linv = L^-1 (lower triangular, row-major) and the
// operands IC_YI, IC_ST, IC_QST, IC_SXY (the sign of the last included).
DX double imu_whitening(const ImuCommon& ic, const double* Linv, int i, int c) {
  const M3* m = ic.mats;
  const int j = c % 3;
  double a = 0.0;
  if (c < 3) {  // r: dp rows of A^-1
    for (int k = 0; k < 3; ++k) a += Linv[9 * i + 6 + k] * m[IC_ST](k, j);
  } else if (c < 6) {  // alpha: dphi and dp rows
    for (int k = 0; k < 3; ++k) a += Linv[9 * i + k] * m[IC_YI](k, j);
    for (int k = 0; k < 3; ++k) a += Linv[9 * i + 6 + k] * m[IC_SXY](k, j);
  } else {  // v: dv rows
    for (int k = 0; k < 3; ++k) a += Linv[9 * i + 3 + k] * m[IC_QST](k, j);
  }
  return a;
}

// Gyro-only prediction: x1 = x0 with the orientation rotated by the
// gyro-integrated rotation, R1 = R0 R_CS dR R_CS^T (dR at x0's gyro bias).
DX void imu_predict_gyro(const dslam_frame_state& x0, const dslam_preint& pre, const ImuParamsD& ip,
                         dslam_frame_state* x1) {
  double pb[3];
  for (int i = 0; i < 3; ++i) {
    double a = 0.0;
    for (int k = 0; k < 3; ++k) a += pre.J[6 * i + k] * (x0.bg[k] - pre.bg[k]);
    pb[i] = a;
  }
  const M3 Rcs = load33(ip.R_CS);
  const M3 dR = load33(pre.dR) * Exp(load3(pb));
  const M3 R0 = q2R(x0.q);
  const M3 R1 = R0 * Rcs * dR * tr(Rcs);
  *x1 = x0;
  qboxplus(x1->q, Log(R1 * tr(R0)));
}

// IMU prediction of the current state from x0 (x1 <- x1_hat(x0)).  Serial.
DX void imu_predict(const dslam_frame_state& x0, const double* qIW, const dslam_preint& pre, const ImuParamsD& ip,
                    dslam_frame_state* x1) {
  double e[15];
  imu_common(x0, x0, qIW, pre, ip, e);
  // e = x1_hat [-] x0 with x1 := x0; recover x1_hat
  *x1 = x0;
  for (int i = 0; i < 3; ++i) {
    x1->r[i] = x0.r[i] + e[i];
    x1->v[i] = x0.v[i] + e[6 + i];
  }
  qboxplus(x1->q, v3(e[3], e[4], e[5]));
}

}  // namespace dslam
