// Small float64 linear algebra and SO(3) helpers shared by the host solve and
// the device solve kernel (__host__ __device__).  3x3 matrices are row-major
// double[9]; quaternions are Hamilton (w, x, y, z); perturbations are on the
// left, R <- Exp(da) R (Section IV-A).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#define DX __host__ __device__ inline

namespace dslam {

struct M3 {
  double m[9];
  DX double& operator()(int r, int c) { return m[3 * r + c]; }
  DX double operator()(int r, int c) const { return m[3 * r + c]; }
};
struct V3 {
  double x, y, z;
  DX double operator[](int i) const { return i == 0 ? x : (i == 1 ? y : z); }
};

DX V3 v3(double x, double y, double z) { return V3{x, y, z}; }
DX V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
DX V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
DX V3 operator-(V3 a) { return v3(-a.x, -a.y, -a.z); }
DX V3 operator*(double s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
DX double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
DX V3 cross(V3 a, V3 b) { return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
DX double norm(V3 a) { return sqrt(dot(a, a)); }
DX V3 load3(const double* p) { return v3(p[0], p[1], p[2]); }
DX void store3(double* p, V3 a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }

DX M3 eye3() { M3 r = {{1, 0, 0, 0, 1, 0, 0, 0, 1}}; return r; }
DX M3 zero3() { M3 r = {{0, 0, 0, 0, 0, 0, 0, 0, 0}}; return r; }
DX M3 load33(const double* p) { M3 r; for (int i = 0; i < 9; ++i) r.m[i] = p[i]; return r; }
DX M3 hat(V3 w) { M3 r = {{0, -w.z, w.y, w.z, 0, -w.x, -w.y, w.x, 0}}; return r; }
DX M3 operator*(const M3& a, const M3& b) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r(i, j) = a(i, 0) * b(0, j) + a(i, 1) * b(1, j) + a(i, 2) * b(2, j);
  return r;
}
DX V3 operator*(const M3& a, V3 v) {
  return v3(a(0, 0) * v.x + a(0, 1) * v.y + a(0, 2) * v.z, a(1, 0) * v.x + a(1, 1) * v.y + a(1, 2) * v.z,
            a(2, 0) * v.x + a(2, 1) * v.y + a(2, 2) * v.z);
}
DX M3 operator+(const M3& a, const M3& b) { M3 r; for (int i = 0; i < 9; ++i) r.m[i] = a.m[i] + b.m[i]; return r; }
DX M3 operator-(const M3& a, const M3& b) { M3 r; for (int i = 0; i < 9; ++i) r.m[i] = a.m[i] - b.m[i]; return r; }
DX M3 operator*(double s, const M3& a) { M3 r; for (int i = 0; i < 9; ++i) r.m[i] = s * a.m[i]; return r; }
DX M3 tr(const M3& a) { M3 r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r(i, j) = a(j, i); return r; }

// sum_{k<N} a[k sa] b[k sb], accumulated from 0 in the order k = 0..N-1 (the
// arithmetic of the plain loop), with all 2N shared-memory reads issued before
// the first product: left to itself the compiler waits on each read in turn.
template <int N>
DX double dotN(const double* a, int sa, const double* b, int sb) {
  double x[N], y[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    x[k] = a[k * sa];
    y[k] = b[k * sb];
  }
#ifdef __HIP_DEVICE_COMPILE__
  __builtin_amdgcn_sched_barrier(0);
#endif
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) s += x[k] * y[k];
  return s;
}

// sum_{k<N} (a[k] b[k] + c[k] d[k]) in the same way (each step adds the sum of
// the two products).
template <int N>
DX double dot2N(const double* a, const double* b, const double* c, const double* d) {
  double x[N], y[N], u[N], v[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    x[k] = a[k];
    y[k] = b[k];
    u[k] = c[k];
    v[k] = d[k];
  }
#ifdef __HIP_DEVICE_COMPILE__
  __builtin_amdgcn_sched_barrier(0);
#endif
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) s += x[k] * y[k] + u[k] * v[k];
  return s;
}

// Rodrigues' formula; below 0.1 rad its coefficients come from their Taylor
// series (exact to double precision there), which avoids sin/cos for the small
// rotations of a Gauss-Newton step or an IMU sample.
DX M3 Exp(V3 phi) {
  double t2 = dot(phi, phi), th = sqrt(t2);
  double a, b;
  if (th < 0.1) {
    a = 1.0 + t2 * (-1.0 / 6.0 + t2 * (1.0 / 120.0 + t2 * (-1.0 / 5040.0 + t2 * (1.0 / 362880.0))));
    b = 0.5 + t2 * (-1.0 / 24.0 + t2 * (1.0 / 720.0 + t2 * (-1.0 / 40320.0 + t2 * (1.0 / 3628800.0))));
  } else {
    a = sin(th) / th;
    b = (1.0 - cos(th)) / t2;
  }
  M3 K = hat(phi);
  return eye3() + a * K + b * (K * K);
}

// Inverse of Exp for angles in [0, pi).  With w the skew part (|w| = 2 sin th),
// Log = (th / (2 sin th)) w; for small angles th / sin th is the series of
// asin(s)/s in s = |w|/2 (no inverse trigonometry).
DX V3 Log(const M3& R) {
  double c = 0.5 * (R(0, 0) + R(1, 1) + R(2, 2) - 1.0);
  V3 w = v3(R(2, 1) - R(1,2), R(0, 2) - R(2, 0), R(1, 0) - R(0, 1));
  double s2 = 0.25 * dot(w, w);
  if (c > 0.0 && s2 < 0.0025) {  // th < ~0.05 rad
    double f = 1.0 + s2 * (1.0 / 6.0 + s2 * (3.0 / 40.0 + s2 * (5.0 / 112.0 + s2 * (35.0 / 1152.0))));
    return (0.5 * f) * w;
  }
  c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
  double th = acos(c);
  if (th < 1e-5) return (0.5 * (1.0 + th * th / 6.0)) * w;
  if (M_PI - th < 1e-6) {
    // near pi: the axis from the column of R + I with the largest diagonal
    // (columns picked by value, no run-time indexing of R)
    const bool c1 = R(1, 1) > R(0, 0) && R(1, 1) >= R(2, 2);
    const bool c2 = !c1 && R(2, 2) > R(0, 0);
    V3 col = c2 ? v3(R(0, 2), R(1, 2), R(2, 2) + 1.0)
                : (c1 ? v3(R(0, 1), R(1, 1) + 1.0, R(2, 1)) : v3(R(0, 0) + 1.0, R(1, 0), R(2, 0)));
    V3 a = 0.5 * col;
    const double akk = c2 ? a.z : (c1 ? a.y : a.x);
    a = (1.0 / sqrt(akk)) * a;
    return (th / norm(a)) * a;
  }
  return (th / (2.0 * sin(th))) * w;
}

// Right Jacobian of SO(3): Exp(phi + d) ~ Exp(phi) Exp(Jr(phi) d).
DX M3 Jr(V3 phi) {
  double t2 = dot(phi, phi), th = sqrt(t2);
  double a, b;
  if (th < 0.1) {
    a = 0.5 + t2 * (-1.0 / 24.0 + t2 * (1.0 / 720.0 + t2 * (-1.0 / 40320.0 + t2 * (1.0 / 3628800.0))));
    b = 1.0 / 6.0 + t2 * (-1.0 / 120.0 + t2 * (1.0 / 5040.0 + t2 * (-1.0 / 362880.0 + t2 * (1.0 / 39916800.0))));
  } else {
    a = (1.0 - cos(th)) / t2;
    b = (th - sin(th)) / (t2 * th);
  }
  M3 K = hat(phi);
  return eye3() - a * K + b * (K * K);
}

// Inverse left Jacobian: Log(Exp(d) Exp(phi)) ~ phi + Jl^-1(phi) d.
DX M3 JlInv(V3 phi) {
  double t2 = dot(phi, phi), th = sqrt(t2);
  double c;
  if (th < 0.1) c = 1.0 / 12.0 + t2 * (1.0 / 720.0 + t2 * (1.0 / 30240.0 + t2 * (1.0 / 1209600.0)));
  else c = 1.0 / t2 - (1.0 + cos(th)) / (2.0 * th * sin(th));
  M3 K = hat(phi);
  return eye3() - 0.5 * K + c * (K * K);
}

// Quaternion helpers (w, x, y, z).
DX void qmul(const double* p, const double* q, double* r) {
  double w = p[0] * q[0] - p[1] * q[1] - p[2] * q[2] - p[3] * q[3];
  double x = p[0] * q[1] + p[1] * q[0] + p[2] * q[3] - p[3] * q[2];
  double y = p[0] * q[2] - p[1] * q[3] + p[2] * q[0] + p[3] * q[1];
  double z = p[0] * q[3] + p[1] * q[2] - p[2] * q[1] + p[3] * q[0];
  r[0] = w; r[1] = x; r[2] = y; r[3] = z;
}
DX M3 q2R(const double* qin) {
  double inv = 1.0 / sqrt(qin[0] * qin[0] + qin[1] * qin[1] + qin[2] * qin[2] + qin[3] * qin[3]);
  double w = qin[0] * inv, x = qin[1] * inv, y = qin[2] * inv, z = qin[3] * inv;
  M3 R = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
           2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
           2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
  return R;
}
DX void qexp(V3 phi, double* q) {
  double t2 = dot(phi, phi);
  if (t2 < 0.01) {  // th < 0.1: Taylor series of cos(th/2) and sin(th/2)/th
    double h2 = 0.25 * t2;
    double co = 1.0 + h2 * (-0.5 + h2 * (1.0 / 24.0 + h2 * (-1.0 / 720.0 + h2 * (1.0 / 40320.0))));
    double s = 0.5 * (1.0 + h2 * (-1.0 / 6.0 + h2 * (1.0 / 120.0 + h2 * (-1.0 / 5040.0 + h2 * (1.0 / 362880.0)))));
    q[0] = co; q[1] = s * phi.x; q[2] = s * phi.y; q[3] = s * phi.z;
    return;
  }
  double th = sqrt(t2);
  double s = sin(0.5 * th) / th;
  q[0] = cos(0.5 * th); q[1] = s * phi.x; q[2] = s * phi.y; q[3] = s * phi.z;
}
// q <- Exp(da) (x) q, renormalised, scalar part kept non-negative.
DX void qboxplus(double* q, V3 da) {
  double e[4], r[4];
  qexp(da, e);
  qmul(e, q, r);
  double n = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
  double s = (r[0] < 0 ? -1.0 : 1.0) / n;
  for (int i = 0; i < 4; ++i) q[i] = r[i] * s;
}
// p [-] q = Log(R(p) R(q)^T)
DX V3 qboxminus(const double* p, const double* q) { return Log(q2R(p) * tr(q2R(q))); }

}  // namespace dslam
