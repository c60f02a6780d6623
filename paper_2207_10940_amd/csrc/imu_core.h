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
struct PreintWork {
  double A[81], B[54], T[81], TB[54];
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

// Preintegration over [t0, t1) at biases (bg, ba).  Runs on the lanes of `par`;
// `out` and `w` are visible to all lanes.  Returns DSLAM_OK / DSLAM_ERR_INVALID.
DX int preintegrate(Par par, const dslam_imu_sample* s, int n, double t0, double t1, const double* bg,
                    const double* ba, double sigma_g, double sigma_a, PreintWork* w, dslam_preint* out) {
  SERIAL {
    w->nsub = -1;
    int st = imu_subintervals(s, n, t0, t1, w);
    if (st != DSLAM_OK) w->nsub = -1;
    for (int i = 0; i < 9; ++i) w->dR[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int i = 0; i < 3; ++i) { w->dv[i] = 0.0; w->dp[i] = 0.0; }
  }
  PFOR(i, 81) out->Sigma[i] = 0.0;
  PFOR(i, 54) out->J[i] = 0.0;
  DSLAM_SYNC();
  int nsub = w->nsub;
  if (nsub < 0) return DSLAM_ERR_INVALID;
  for (int m = 0; m < nsub; ++m) {
    const dslam_imu_sample& smp = s[w->ksub[m]];
    double dt = w->dtsub[m];
    SERIAL {
      V3 wv = v3(smp.gyro[0] - bg[0], smp.gyro[1] - bg[1], smp.gyro[2] - bg[2]);
      V3 av = v3(smp.acc[0] - ba[0], smp.acc[1] - ba[1], smp.acc[2] - ba[2]);
      V3 phi = dt * wv;
      double c[3], d[3];
      gamma_coeffs(norm(phi), c, d);
      V3 g1a, g2a;
      M3 D1, D2;
      gamma_apply(phi, av, 1.0, c[0], c[1], d[0], d[1], &g1a, &D1);
      gamma_apply(phi, av, 0.5, c[1], c[2], d[1], d[2], &g2a, &D2);
      M3 K = hat(phi);
      M3 G1 = eye3() + c[0] * K + c[1] * (K * K);
      M3 G2 = 0.5 * eye3() + c[1] * K + c[2] * (K * K);
      M3 dR = load33(w->dR);
      M3 E = Exp(phi);
      // step Jacobian w.r.t. the incoming error state [dphi, dv, dp]
      for (int i = 0; i < 81; ++i) w->A[i] = (i % 10 == 0) ? 1.0 : 0.0;
      M3 Et = tr(E);
      M3 Av_phi = (-dt) * (dR * hat(g1a));
      M3 Ap_phi = (-dt * dt) * (dR * hat(g2a));
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          w->A[9 * i + j] = Et(i, j);
          w->A[9 * (3 + i) + j] = Av_phi(i, j);
          w->A[9 * (6 + i) + j] = Ap_phi(i, j);
        }
      for (int i = 0; i < 3; ++i) w->A[9 * (6 + i) + 3 + i] = dt;
      // step Jacobian w.r.t. the biases [bg, ba] (the noise enters with the opposite sign)
      M3 Bphi_g = (-dt) * Jr(phi);
      M3 Bv_g = (-dt * dt) * (dR * D1);
      M3 Bp_g = (-dt * dt * dt) * (dR * D2);
      M3 Bv_a = (-dt) * (dR * G1);
      M3 Bp_a = (-dt * dt) * (dR * G2);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          w->B[6 * i + j] = Bphi_g(i, j);
          w->B[6 * i + 3 + j] = 0.0;
          w->B[6 * (3 + i) + j] = Bv_g(i, j);
          w->B[6 * (3 + i) + 3 + j] = Bv_a(i, j);
          w->B[6 * (6 + i) + j] = Bp_g(i, j);
          w->B[6 * (6 + i) + 3 + j] = Bp_a(i, j);
        }
      // state update (uses the old dR, dv)
      V3 dRg2a = dR * g2a, dRg1a = dR * g1a;
      for (int i = 0; i < 3; ++i) {
        w->dp[i] = w->dp[i] + w->dv[i] * dt + dRg2a[i] * dt * dt;
        w->dv[i] = w->dv[i] + dRg1a[i] * dt;
      }
      M3 dRn = dR * E;
      for (int i = 0; i < 9; ++i) w->dR[i] = dRn.m[i];
    }
    DSLAM_SYNC();
    // T = A Sigma, TB = A J
    PFOR(idx, 81) {
      int i = idx / 9, j = idx % 9;
      double acc = 0.0;
      for (int k = 0; k < 9; ++k) acc += w->A[9 * i + k] * out->Sigma[9 * k + j];
      w->T[idx] = acc;
    }
    PFOR(idx, 54) {
      int i = idx / 6, j = idx % 6;
      double acc = 0.0;
      for (int k = 0; k < 9; ++k) acc += w->A[9 * i + k] * out->J[6 * k + j];
      w->TB[idx] = acc;
    }
    DSLAM_SYNC();
    double vg = sigma_g * sigma_g / dt, va = sigma_a * sigma_a / dt;
    PFOR(idx, 81) {
      int i = idx / 9, j = idx % 9;
      double acc = 0.0;
      for (int k = 0; k < 9; ++k) acc += w->T[9 * i + k] * w->A[9 * j + k];
      double q = 0.0;
      for (int k = 0; k < 3; ++k) q += w->B[6 * i + k] * w->B[6 * j + k];
      double r = 0.0;
      for (int k = 3; k < 6; ++k) r += w->B[6 * i + k] * w->B[6 * j + k];
      out->Sigma[idx] = acc + vg * q + va * r;
    }
    PFOR(idx, 54) out->J[idx] = w->TB[idx] + w->B[idx];
    DSLAM_SYNC();
  }
  SERIAL {
    for (int i = 0; i < 9; ++i) out->dR[i] = w->dR[i];
    for (int i = 0; i < 3; ++i) {
      out->dv[i] = w->dv[i];
      out->dp[i] = w->dp[i];
      out->bg[i] = bg[i];
      out->ba[i] = ba[i];
    }
    out->dt = t1 - t0;
    // symmetrise
    for (int i = 0; i < 9; ++i)
      for (int j = i + 1; j < 9; ++j) {
        double a = 0.5 * (out->Sigma[9 * i + j] + out->Sigma[9 * j + i]);
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

// IMU error e = x1_hat(x0) [-] x1 (eq. (5)), ordered [r, alpha, v, bg, ba], with
// the Jacobian rows of its first nine entries (9x33 over [x0, x1, dg]) and the
// map A9 (9x9) from the preintegration noise (dphi, dv, dp) to those entries
// (J9 == nullptr: residual only).  The bias rows are [I at x0's bias, -I at
// x1's bias].  Serial.
DX void imu_factor(const dslam_frame_state& x0, const dslam_frame_state& x1, const double* qIW,
                   const dslam_preint& pre, const ImuParamsD& ip, double* e, double* J9, double* A9) {
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
  V3 rh = r0 + R0 * tcs + Qt * yg + S * dpv - Rh1 * tcs;
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
  if (J9 == nullptr) return;
  for (int i = 0; i < 9 * 33; ++i) J9[i] = 0.0;
  for (int i = 0; i < 81; ++i) A9[i] = 0.0;
  M3 Jli = JlInv(ea);
  M3 Jri = tr(Jli);
  M3 Jrb = Jr(phib);
  M3 JRg, JRa, Jpg, Jpa, Jvg, Jva;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      JRg(i, j) = pre.J[6 * i + j];
      JRa(i, j) = pre.J[6 * i + 3 + j];
      Jvg(i, j) = pre.J[6 * (3 + i) + j];
      Jva(i, j) = pre.J[6 * (3 + i) + 3 + j];
      Jpg(i, j) = pre.J[6 * (6 + i) + j];
      Jpa(i, j) = pre.J[6 * (6 + i) + 3 + j];
    }
  // e_r rows
  V3 yr = tcs + Rcs * dpv - Rcs * (dRt * wt);
  M3 Er_a0 = (-1.0) * hat(R0 * yr);
  M3 Er_v0 = T * Qt;
  M3 Krot = SdRt * hat(wt) * Jrb;
  M3 Er_bg = S * Jpg + Krot * JRg;
  M3 Er_ba = S * Jpa + Krot * JRa;
  M3 Er_g = Qt * hat(yg);
  // e_alpha rows
  M3 Kal = Jli * SdRt * Jrb;
  M3 Ea_bg = Kal * JRg;
  M3 Ea_ba = Kal * JRa;
  // e_v rows
  M3 Ev_a0 = (-1.0) * (Q * hat(Sdv));
  M3 Ev_bg = Q * S * Jvg;
  M3 Ev_ba = Q * S * Jva;
  M3 Ev_g = (-1.0) * hat(QSdv);
  // noise map
  M3 RbT = tr(Rb);
  M3 Nr_phi = SdRt * hat(wt) * RbT;
  M3 Na_phi = Jli * SdRt * RbT;
  M3 Nv_v = Q * S;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double d = (i == j) ? 1.0 : 0.0;
      double* rr = J9 + 33 * i;
      double* ra = J9 + 33 * (3 + i);
      double* rv = J9 + 33 * (6 + i);
      rr[0 + j] = d;
      rr[3 + j] = Er_a0(i, j);
      rr[6 + j] = Er_v0(i, j);
      rr[9 + j] = Er_bg(i, j);
      rr[12 + j] = Er_ba(i, j);
      rr[15 + j] = -d;
      rr[30 + j] = Er_g(i, j);
      ra[3 + j] = Jli(i, j);
      ra[9 + j] = Ea_bg(i, j);
      ra[12 + j] = Ea_ba(i, j);
      ra[18 + j] = -Jri(i, j);
      rv[3 + j] = Ev_a0(i, j);
      rv[6 + j] = d;
      rv[9 + j] = Ev_bg(i, j);
      rv[12 + j] = Ev_ba(i, j);
      rv[21 + j] = -d;
      rv[30 + j] = Ev_g(i, j);
      A9[9 * i + j] = Nr_phi(i, j);
      A9[9 * i + 6 + j] = S(i, j);
      A9[9 * (3 + i) + j] = Na_phi(i, j);
      A9[9 * (6 + i) + 3 + j] = Nv_v(i, j);
    }
}

// IMU prediction of the current state from x0 (x1 <- x1_hat(x0)).  Serial.
DX void imu_predict(const dslam_frame_state& x0, const double* qIW, const dslam_preint& pre, const ImuParamsD& ip,
                    dslam_frame_state* x1) {
  double e[15];
  imu_factor(x0, x0, qIW, pre, ip, e, nullptr, nullptr);
  // e = x1_hat [-] x0 with x1 := x0; recover x1_hat
  *x1 = x0;
  for (int i = 0; i < 3; ++i) {
    x1->r[i] = x0.r[i] + e[i];
    x1->v[i] = x0.v[i] + e[6 + i];
  }
  qboxplus(x1->q, v3(e[3], e[4], e[5]));
}

}  // namespace dslam
