// Deformation graph with the gravity term (Section V, eqs. (10)-(17)) on the
// GPU: Gauss-Newton over the node matrices A_l (the paper's node "rotation",
// held orthonormal by E_rot only) and translations t_l.  Readings:
//   * influence of the nodes on a point v: its K = 4 nearest nodes (ties by
//     index), weights w_k = (1 - |v - g_k| / d_max)^2 with d_max the distance
//     of the (K+1)-th nearest node, normalised (equal weights if all vanish);
//     phi(v) = sum_k w_k (A_k (v - g_k) + g_k + t_k);
//   * E_reg's neighbours N(l): the K nearest other nodes;
//   * E_rot = sum_l |A_l^T A_l - I|_F^2 (all nine entries), E_reg, E_con,
//     E_pin, E_rel (global closures only) and E_imu as written, weights
//     w_f = 1, w_r = 10, w_c = w_i = 100;
//   * each step forms every term's residual and Jacobian rows scaled by the
//     square root of its weight (one thread per term, dense rows of
//     [J | r]), the normal equations as [J r]^T [J r] (tiled, every entry
//     summed over the rows in row order: the last column holds J^T r and the
//     corner the cost), and solves them by a blocked Cholesky (panels of 16
//     columns factored in one workgroup, trailing updates over the chip).
// Everything is float64; the neighbour lists and influences are computed on
// the host.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "host.h"

namespace dslam {

constexpr int DEF_K = 4;
constexpr double DEF_W_ROT = 1.0, DEF_W_REG = 10.0, DEF_W_CON = 100.0, DEF_W_IMU = 100.0;
constexpr int DEF_TILE = 16;

struct DefDev {
  int N, P, Pp, Pr, global;
  int m, n, ld;       // rows of [J | r], unknowns (12 N), row length (n + 1 rounded up to the tile)
  const double* nodes;  // N x 3
  const int* nbr;       // N x K
  const double* con;    // P x 6: source, destination
  const int* con_idx;   // P x K
  const double* con_w;
  const double* pin;    // Pp x 3
  const int* pin_idx;
  const double* pin_w;
  const double* rel;    // Pr x 6
  const int* rel_idx;   // Pr x 2K: the source's influence, then the destination's
  const double* rel_w;
  double g[3];
  double* x;   // 12 N: A_l row-major, t_l
  double* Jr;  // m x ld
  double* H;   // ld x ld
  double* L;   // ld x ld: the Cholesky factor (lower triangle; off-diagonal panels also transposed above it)
  double* cost;
  int* bad;
  double* tiny;
};

__global__ __launch_bounds__(256) void def_zero_kernel(double* p, size_t n) {
  for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0.0;
}

// phi at v with the given influence, added with sign `sg` to the three rows
// starting at `row` (Jacobian entries and residual column).
__device__ __forceinline__ void def_phi_rows(const DefDev& d, const int* idx, const double* w, const double* v,
                                             double sg, double sw, int row, double* r) {
  for (int k = 0; k < DEF_K; ++k) {
    const int nd = idx[k];
    const double wk = w[k];
    const double* g = d.nodes + 3 * nd;
    const double dv[3] = {v[0] - g[0], v[1] - g[1], v[2] - g[2]};
    const double* A = d.x + 12 * nd;
    for (int a = 0; a < 3; ++a) {
      double* J = d.Jr + (size_t)(row + a) * d.ld;
      for (int b = 0; b < 3; ++b) J[12 * nd + 3 * a + b] += sg * sw * wk * dv[b];
      J[12 * nd + 9 + a] += sg * sw * wk;
      const double pa = A[3 * a] * dv[0] + A[3 * a + 1] * dv[1] + A[3 * a + 2] * dv[2] + g[a] + A[9 + a];
      r[a] += sg * wk * pa;
    }
  }
}

// One thread per term: its rows of [J | r], scaled by sqrt(weight).
__global__ __launch_bounds__(256) void def_jacobian_kernel(DefDev d) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  const int N = d.N, nrot = N, nreg = N * DEF_K, ncon = d.P, npin = d.Pp, nrel = d.global ? d.Pr : 0;
  const int T = nrot + nreg + ncon + npin + nrel + N;
  if (q >= T) return;
  const int n = d.n;
  if (q < nrot) {  // E_rot
    const int l = q;
    const double sw = sqrt(DEF_W_ROT);
    const double* A = d.x + 12 * l;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double* J = d.Jr + (size_t)(9 * l + 3 * i + j) * d.ld;
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
          s += A[3 * a + i] * A[3 * a + j];
          J[12 * l + 3 * a + j] += sw * A[3 * a + i];
          J[12 * l + 3 * a + i] += sw * A[3 * a + j];
        }
        J[n] = sw * (s - (i == j ? 1.0 : 0.0));
      }
    return;
  }
  int row = 9 * N;
  int t = q - nrot;
  if (t < nreg) {  // E_reg
    const int l = t / DEF_K, nb = d.nbr[t];
    const double sw = sqrt(DEF_W_REG);
    const double* gl = d.nodes + 3 * l;
    const double* gn = d.nodes + 3 * nb;
    const double dv[3] = {gn[0] - gl[0], gn[1] - gl[1], gn[2] - gl[2]};
    const double* A = d.x + 12 * l;
    for (int a = 0; a < 3; ++a) {
      double* J = d.Jr + (size_t)(row + 3 * t + a) * d.ld;
      for (int b = 0; b < 3; ++b) J[12 * l + 3 * a + b] = sw * dv[b];
      J[12 * l + 9 + a] += sw;
      J[12 * nb + 9 + a] -= sw;
      const double r = A[3 * a] * dv[0] + A[3 * a + 1] * dv[1] + A[3 * a + 2] * dv[2] + gl[a] + A[9 + a] -
                       (gn[a] + d.x[12 * nb + 9 + a]);
      J[n] = sw * r;
    }
    return;
  }
  row += 3 * nreg;
  t -= nreg;
  const double sw = sqrt(DEF_W_CON);
  double r[3] = {0.0, 0.0, 0.0};
  if (t < ncon) {  // E_con: phi(source) - destination
    const double* c = d.con + 6 * t;
    def_phi_rows(d, d.con_idx + DEF_K * t, d.con_w + DEF_K * t, c, 1.0, sw, row + 3 * t, r);
    for (int a = 0; a < 3; ++a) d.Jr[(size_t)(row + 3 * t + a) * d.ld + n] = sw * (r[a] - c[3 + a]);
    return;
  }
  row += 3 * ncon;
  t -= ncon;
  if (t < npin) {  // E_pin: phi(destination) - destination
    const double* c = d.pin + 3 * t;
    def_phi_rows(d, d.pin_idx + DEF_K * t, d.pin_w + DEF_K * t, c, 1.0, sw, row + 3 * t, r);
    for (int a = 0; a < 3; ++a) d.Jr[(size_t)(row + 3 * t + a) * d.ld + n] = sw * (r[a] - c[a]);
    return;
  }
  row += 3 * npin;
  t -= npin;
  if (t < nrel) {  // E_rel: phi(source) - phi(destination)
    const double* c = d.rel + 6 * t;
    def_phi_rows(d, d.rel_idx + 2 * DEF_K * t, d.rel_w + 2 * DEF_K * t, c, 1.0, sw, row + 3 * t, r);
    def_phi_rows(d, d.rel_idx + 2 * DEF_K * t + DEF_K, d.rel_w + 2 * DEF_K * t + DEF_K, c + 3, -1.0, sw,
                 row + 3 * t, r);
    for (int a = 0; a < 3; ++a) d.Jr[(size_t)(row + 3 * t + a) * d.ld + n] = sw * r[a];
    return;
  }
  row += 3 * nrel;
  t -= nrel;
  {  // E_imu: A_l g - g
    const int l = t;
    const double si = sqrt(DEF_W_IMU);
    const double* A = d.x + 12 * l;
    for (int a = 0; a < 3; ++a) {
      double* J = d.Jr + (size_t)(row + 3 * l + a) * d.ld;
      for (int b = 0; b < 3; ++b) J[12 * l + 3 * a + b] = si * d.g[b];
      J[n] = si * (A[3 * a] * d.g[0] + A[3 * a + 1] * d.g[1] + A[3 * a + 2] * d.g[2] - d.g[a]);
    }
  }
}

// [J r]^T [J r] on its lower tiles (all that the factorisation and the solves
// read), one 16 x 16 tile per workgroup.  A tile sums, in row order, only the
// rows with entries in both of its column blocks: the host lists them per
// tile (the pattern of J is the same at every Gauss-Newton step), and a row
// left out would add exact zeros.  The one exception is the corner entry
// r^T r, left incomplete here: nothing reads it (the cost is summed apart).
__global__ __launch_bounds__(256) void def_normal_kernel(DefDev d, const int* tile_ij, const int* off,
                                                         const int* rows) {
  __shared__ double As[DEF_TILE][DEF_TILE + 1], Bs[DEF_TILE][DEF_TILE + 1];
  const int tx = threadIdx.x % DEF_TILE, ty = threadIdx.x / DEF_TILE;
  const int p = blockIdx.x;
  const int i0 = tile_ij[2 * p] * DEF_TILE, j0 = tile_ij[2 * p + 1] * DEF_TILE;
  const int beg = off[p], end = off[p + 1];
  double acc = 0.0;
  for (int k0 = beg; k0 < end; k0 += DEF_TILE) {
    const int r = k0 + ty < end ? rows[k0 + ty] : -1;
    As[ty][tx] = r >= 0 ? d.Jr[(size_t)r * d.ld + i0 + tx] : 0.0;
    Bs[ty][tx] = r >= 0 ? d.Jr[(size_t)r * d.ld + j0 + tx] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < DEF_TILE; ++k) acc += As[k][ty] * Bs[k][tx];
    __syncthreads();
  }
  d.H[(size_t)(i0 + ty) * d.ld + j0 + tx] = acc;
}

// Blocked right-looking Cholesky of the n x n normal matrix (lower triangle,
// into L), panel by panel of DEF_PANEL columns, one launch of def_chol_kernel
// per DEF_NP panels; def_solve_kernel then solves L L^T dx = -J^T r and updates the
// parameters.  A pivot at or below 1e-12 of the largest diagonal entry of the
// normal matrix marks the system singular (def_prepare_kernel also records
// the step's cost r^T r, summed over the residual column of [J r]).
constexpr int DEF_PANEL = 16;

__global__ __launch_bounds__(256) void def_prepare_kernel(DefDev d, int it) {
  __shared__ double part[256], cost[256];
  const int n = d.n, ld = d.ld, tid = threadIdx.x;
  double m = 0.0, c = 0.0;
  for (int i = tid; i < n; i += 256) m = fmax(m, d.H[(size_t)i * ld + i]);
  for (int r = tid; r < d.m; r += 256) {
    const double v = d.Jr[(size_t)r * ld + n];
    c += v * v;
  }
  part[tid] = m;
  cost[tid] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      part[tid] = fmax(part[tid], part[tid + s]);
      cost[tid] += cost[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    d.cost[it] = cost[0];
    *d.tiny = 1e-12 * part[0];
  }
}

// A lane's double from lane l of the wave (l the same for every lane).
__device__ __forceinline__ double def_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// One step of the blocked right-looking Cholesky, for the macro panel of up
// to DEF_NP panels of DEF_PANEL columns at kb, in a single launch.  The
// factor goes to the separate matrix L, so that the macro panel's columns of H
// stay as they were for every workgroup to read; its part below each panel's
// diagonal block is also written transposed into L's otherwise unused upper
// triangle, where the forward solve reads it by rows.  Workgroup p owns the
// p-th lower trailing tile (rows i0, columns j0, both past the macro panel).
// Panel by panel (left-looking within the macro panel) it updates the
// panel's diagonal block, the later panels' rows and its own two row blocks
// with the earlier panels' columns, factors the diagonal block in LDS and
// solves those rows against it (x L^T = h, one thread per row); it then
// subtracts its row blocks' product from its tile of H.  A tile in the first
// trailing column writes its row blocks of the factor (the first tile also
// the macro panel's diagonal part and the bad-pivot flag).  The last macro
// panel has no trailing tile and runs one workgroup that only factors.
constexpr int DEF_NP = 2;

__global__ __launch_bounds__(256) void def_chol_kernel(DefDev d, int kb) {
  // Dd[c][a]: rows of panel c, columns of panel a (a <= c); R[s][a]: the
  // tile's row block s (0: rows i0.., 1: rows j0..), columns of panel a
  __shared__ double Dd[DEF_NP][DEF_NP][DEF_PANEL][DEF_PANEL + 1];
  __shared__ double R[2][DEF_NP][DEF_TILE][DEF_PANEL + 1];
  const int n = d.n, ld = d.ld, tid = threadIdx.x;
  const int np = min(DEF_NP, (n - kb + DEF_PANEL - 1) / DEF_PANEL);
  const int base = min(kb + DEF_NP * DEF_PANEL, n);
  const int p = blockIdx.x;
  int ti = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > p) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= p) ++ti;
  const int tj = p - ti * (ti + 1) / 2;
  const int i0 = base + ti * DEF_TILE, j0 = base + tj * DEF_TILE;
  const bool first = p == 0;
  double* H = d.H;
  double* L = d.L;
  auto width = [&](int a) { return min(DEF_PANEL, n - (kb + DEF_PANEL * a)); };
  const int r = tid / DEF_PANEL, col = tid % DEF_PANEL;
  for (int c = 0; c < DEF_NP; ++c)
    for (int a = 0; a < DEF_NP; ++a) {
      const bool in = c < np && a <= c && r < width(c) && col < width(a) && (a < c || col <= r);
      Dd[c][a][r][col] = in ? H[(size_t)(kb + DEF_PANEL * c + r) * ld + kb + DEF_PANEL * a + col] : 0.0;
    }
  for (int sb = 0; sb < 2; ++sb) {
    const int row = (sb ? j0 : i0) + r;
    for (int a = 0; a < DEF_NP; ++a)
      R[sb][a][r][col] = (a < np && row < n && col < width(a)) ? H[(size_t)row * ld + kb + DEF_PANEL * a + col] : 0.0;
  }
  __syncthreads();
  const double tiny = *d.tiny;
  for (int a = 0; a < np; ++a) {
    const int bs = width(a);
    if (a > 0) {  // the earlier panels' contribution to this panel's columns
      const int blocks = np - a + 2;
      for (int e = tid; e < blocks * 256; e += 256) {
        const int blk = e / 256, rr = (e % 256) / DEF_PANEL, cc = e % DEF_PANEL;
        const int c = a + blk;
        if (blk < np - a && c == a && cc > rr) continue;
        double* X = blk < np - a ? &Dd[c][a][rr][cc] : &R[blk - (np - a)][a][rr][cc];
        double acc = 0.0;
        for (int b2 = 0; b2 < a; ++b2) {
          const double* xr = blk < np - a ? Dd[c][b2][rr] : R[blk - (np - a)][b2][rr];
#pragma unroll
          for (int k = 0; k < DEF_PANEL; ++k) acc += xr[k] * Dd[a][b2][cc][k];
        }
        *X -= acc;
      }
      __syncthreads();
    }
    double (*D)[DEF_PANEL + 1] = Dd[a][a];
    for (int k = 0; k < bs; ++k) {  // unblocked Cholesky of the diagonal block
      if (tid == 0) {
        const double pv = D[k][k];
        if (first && (!(pv > tiny) || !(pv < 1e300))) *d.bad = 1;
        D[k][k] = sqrt(pv > 0.0 ? pv : 1.0);
      }
      __syncthreads();
      const double piv = D[k][k];
      if (tid > k && tid < bs) D[tid][k] /= piv;
      __syncthreads();
      if (col > k && r >= col && r < bs) D[r][col] -= D[r][k] * D[col][k];
      __syncthreads();
    }
    // a short last block is padded with identity rows, so that the solves
    // below run over all DEF_PANEL columns with the row in registers
    if (tid >= bs && tid < DEF_PANEL) D[tid][tid] = 1.0;
    __syncthreads();
    // rows of the later panels, then the tile's two row blocks, against D
    const int nrows = DEF_PANEL * (np - 1 - a) + 2 * DEF_TILE;
    if (tid < nrows) {
      const int blk = tid / DEF_PANEL, rr = tid % DEF_PANEL;
      double* xr = blk < np - 1 - a ? Dd[a + 1 + blk][a][rr] : R[blk - (np - 1 - a)][a][rr];
      double x[DEF_PANEL];
#pragma unroll
      for (int c = 0; c < DEF_PANEL; ++c) x[c] = xr[c];
#pragma unroll
      for (int c = 0; c < DEF_PANEL; ++c) {
        double v = x[c];
#pragma unroll
        for (int c2 = 0; c2 < c; ++c2) v -= x[c2] * D[c][c2];
        x[c] = v / D[c][c];
      }
#pragma unroll
      for (int c = 0; c < DEF_PANEL; ++c) xr[c] = c < bs ? x[c] : 0.0;
    }
    __syncthreads();
  }
  if (first)  // the macro panel's diagonal part
    for (int c = 0; c < np; ++c)
      for (int a = 0; a <= c; ++a)
        if (r < width(c) && col < width(a) && (a < c || col <= r)) {
          const int gr = kb + DEF_PANEL * c + r, gc = kb + DEF_PANEL * a + col;
          L[(size_t)gr * ld + gc] = Dd[c][a][r][col];
          if (a < c) L[(size_t)gc * ld + gr] = Dd[c][a][r][col];
        }
  if (tj == 0 && i0 + r < n)  // the first trailing column's row blocks
    for (int a = 0; a < np; ++a)
      if (col < width(a)) {
        const int gr = i0 + r, gc = kb + DEF_PANEL * a + col;
        L[(size_t)gr * ld + gc] = R[0][a][r][col];
        L[(size_t)gc * ld + gr] = R[0][a][r][col];
      }
  const int tx = tid % DEF_TILE, ty = tid / DEF_TILE;
  const int i = i0 + ty, j = j0 + tx;
  if (i < n && j <= i) {
    double acc = 0.0;
    for (int a = 0; a < np; ++a)
#pragma unroll
      for (int c = 0; c < DEF_PANEL; ++c) acc += R[0][a][ty][c] * R[1][a][tx][c];
    H[(size_t)i * ld + j] -= acc;
  }
}

// The two triangular solves, panel by panel of DEF_PANEL rows.  Wave 0 solves
// the panel's diagonal block, lane i holding row i (forward) or column i
// (backward) of it and the reciprocal of its diagonal entry, the finished
// entries read across lanes; the other
// waves then update the remaining right-hand-side entries with the panel's
// columns (forward) or rows (backward), one entry per thread.  Both sides
// load the next panel's part of L while they work on this one.  Each entry
// takes its updates in column order (forward) and in panel order, columns in
// order within a panel (backward).  The right-hand side lives in LDS
// (n <= 12 x 256).
constexpr int DEF_MAX_N = 12 * 256;
constexpr int DEF_SOLVE_THREADS = 1024, DEF_UPD = DEF_SOLVE_THREADS - 64;

__global__ __launch_bounds__(DEF_SOLVE_THREADS) void def_solve_kernel(DefDev d) {
  __shared__ double y[DEF_MAX_N];
  const int n = d.n, ld = d.ld, tid = threadIdx.x, lane = tid & 63, ut = tid - 64;
  const bool diag = tid < 64;  // wave 0
  if (*d.bad) return;          // the same value for every thread
  const double* L = d.L;
  const double* jtr = d.H + (size_t)n * ld;  // row n of the symmetric [J r]^T [J r] is (J^T r)^T
  for (int i = tid; i < n; i += DEF_SOLVE_THREADS) y[i] = -jtr[i];
  const int last = ((n - 1) / DEF_PANEL) * DEF_PANEL;
  // forward: L y = -J^T r
  double cur[DEF_PANEL], nxt[DEF_PANEL] = {}, cur_d = 1.0, nxt_d = 1.0;
  auto fwd_load = [&](int pb, double* v, double* dg) {
    const int bs = min(DEF_PANEL, n - pb);
    if (diag) {
#pragma unroll
      for (int c = 0; c < DEF_PANEL; ++c)
        v[c] = (lane < bs && c <= lane) ? L[(size_t)(pb + lane) * ld + pb + c] : 1.0;
      *dg = lane < bs ? L[(size_t)(pb + lane) * ld + pb + lane] : 1.0;
    } else {  // L[r][pb + c], from its transposed copy above the diagonal
      const int r = pb + bs + ut;
#pragma unroll
      for (int c = 0; c < DEF_PANEL; ++c) v[c] = (r < n && c < bs) ? L[(size_t)(pb + c) * ld + r] : 0.0;
    }
  };
  fwd_load(0, cur, &cur_d);
  double cur_inv = 1.0 / cur_d;
  __syncthreads();
  for (int pb = 0; pb < n; pb += DEF_PANEL) {
    const int bs = min(DEF_PANEL, n - pb);
    if (pb + DEF_PANEL < n) fwd_load(pb + DEF_PANEL, nxt, &nxt_d);
    if (diag) {
      double yi = lane < bs ? y[pb + lane] : 0.0;
#pragma unroll
      for (int c = 0; c < DEF_PANEL; ++c) {
        if (lane == c) yi *= cur_inv;
        const double yc = def_lane(yi, c);
        if (lane > c) yi -= cur[c] * yc;
      }
      if (lane < bs) y[pb + lane] = yi;
    }
    __syncthreads();
    if (!diag) {
      const int r0 = pb + bs + ut;
      if (r0 < n) {
        double v = y[r0];
#pragma unroll
        for (int c = 0; c < DEF_PANEL; ++c) v -= cur[c] * y[pb + min(c, bs - 1)];
        y[r0] = v;
      }
      for (int r = r0 + DEF_UPD; r < n; r += DEF_UPD) {
        double v = y[r];
        for (int c = 0; c < bs; ++c) v -= L[(size_t)(pb + c) * ld + r] * y[pb + c];
        y[r] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < DEF_PANEL; ++c) cur[c] = nxt[c];
    cur_inv = 1.0 / nxt_d;
  }
  // backward: L^T dx = y
  auto bwd_load = [&](int pb, double* v, double* dg) {
    const int bs = min(DEF_PANEL, n - pb);
    if (diag) {
#pragma unroll
      for (int c = 0; c < DEF_PANEL; ++c)
        v[c] = (lane < bs && c < bs && c >= lane) ? L[(size_t)(pb + c) * ld + pb + lane] : 1.0;
      *dg = lane < bs ? L[(size_t)(pb + lane) * ld + pb + lane] : 1.0;
    } else {
#pragma unroll
      for (int c = 0; c < DEF_PANEL; ++c) v[c] = (ut < pb && c < bs) ? L[(size_t)(pb + c) * ld + ut] : 0.0;
    }
  };
  bwd_load(last, cur, &cur_d);
  cur_inv = 1.0 / cur_d;
  for (int pb = last; pb >= 0; pb -= DEF_PANEL) {
    const int bs = min(DEF_PANEL, n - pb);
    if (pb > 0) bwd_load(pb - DEF_PANEL, nxt, &nxt_d);
    if (diag) {
      double yi = lane < bs ? y[pb + lane] : 0.0;
#pragma unroll
      for (int c = DEF_PANEL - 1; c >= 0; --c) {
        if (lane == c) yi *= cur_inv;
        const double yc = def_lane(yi, c);
        if (lane < c) yi -= cur[c] * yc;
      }
      if (lane < bs) y[pb + lane] = yi;
    }
    __syncthreads();
    if (!diag) {
      if (ut < pb) {
        double v = y[ut];
#pragma unroll
        for (int c = 0; c < DEF_PANEL; ++c) v -= cur[c] * y[pb + min(c, bs - 1)];
        y[ut] = v;
      }
      for (int r = ut + DEF_UPD; r < pb; r += DEF_UPD) {
        double v = y[r];
        for (int c = 0; c < bs; ++c) v -= L[(size_t)(pb + c) * ld + r] * y[pb + c];
        y[r] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < DEF_PANEL; ++c) cur[c] = nxt[c];
    cur_inv = 1.0 / nxt_d;
  }
  for (int i = tid; i < n; i += DEF_SOLVE_THREADS) d.x[i] += y[i];
}

}  // namespace dslam

// ---------------------------------------------------------------------------
// C ABI (include/dslam.h)
// ---------------------------------------------------------------------------
using namespace dslam;

struct dslam_deform {
  dslam_context* ctx;
  int max_nodes, max_points;
  uint64_t bytes;
  void* arena;
  double* nodes;
  int* nbr;
  double* pts;   // constraint coordinates
  int* idx;      // influences
  double* w;
  double* x;
  double* Jr;
  double* H;
  double* L;
  double* cost;
  int* bad;
  double* tiny;
  int* pairs;         // per lower tile pair: its two tiles, then the list offsets, then the row lists
  size_t pairs_cap;   // ints
  hipEvent_t done;    // recorded after every solve's work (dslam_deform_destroy waits on it)
  bool recorded;
  std::mutex mu;
};

#define DEF_HIP(expr)                                 \
  do {                                                \
    if ((expr) != hipSuccess) return DSLAM_ERR_DEVICE; \
  } while (0)

static size_t def_align(size_t n) { return (n + 255) & ~size_t(255); }
static int def_round(int v) { return (v + DEF_TILE - 1) / DEF_TILE * DEF_TILE; }

static void def_sizes(int N, int points, int* m, int* n, int* ld) {
  *n = 12 * N;
  *ld = def_round(*n + 1);
  *m = def_round(9 * N + 3 * N * DEF_K + 3 * points + 3 * N);
}

// A row of J has entries in at most 8 nodes (E_rel), each across at most two
// column tiles, plus the residual column's tile: at most 17 tiles, so it
// appears in at most 17 * 18 / 2 lower tile pairs.
constexpr int DEF_ROW_PAIRS = 17 * 18 / 2;

static size_t def_pairs_cap(int m, int ld) {
  const size_t nt = ld / DEF_TILE;
  return (size_t)m * DEF_ROW_PAIRS + 3 * (nt * (nt + 1) / 2) + 1;
}

// The row lists of the lower tile pairs of [J r]^T [J r] for the row layout
// of def_jacobian_kernel: E_rot (9 rows per node), E_reg (3 per node and
// neighbour), E_con, E_pin, E_rel (3 per point), E_imu (3 per node).  `idx`
// holds the influences (K per con and pin point, 2K per rel pair).  Every row
// has the residual column, in the last tile; the corner pair takes only the
// rows with node entries in that tile.  Packs [tile pairs (2 ints each) |
// offsets (pairs + 1) | rows] into `out`.
static void def_pair_lists(int N, int P, int Pp, int Pr, int n, int ld, const int* nbr, const int* idx,
                           std::vector<int>* out) {
  const int nt = ld / DEF_TILE, rt = n / DEF_TILE, W = (nt + 63) / 64;
  const int mr = 9 * N + 3 * N * DEF_K + 3 * (P + Pp + Pr) + 3 * N;
  std::vector<uint64_t> mask((size_t)mr * W, 0);
  auto mark = [&](int row, int node) {
    for (int t = 12 * node / DEF_TILE; t <= (12 * node + 11) / DEF_TILE; ++t)
      mask[(size_t)row * W + t / 64] |= 1ull << (t % 64);
  };
  int row = 0;
  for (int l = 0; l < N; ++l)
    for (int q = 0; q < 9; ++q) mark(row++, l);
  for (int t = 0; t < N * DEF_K; ++t)
    for (int a = 0; a < 3; ++a, ++row) {
      mark(row, t / DEF_K);
      mark(row, nbr[t]);
    }
  for (int t = 0; t < P + Pp; ++t)
    for (int a = 0; a < 3; ++a, ++row)
      for (int k = 0; k < DEF_K; ++k) mark(row, idx[DEF_K * t + k]);
  for (int t = 0; t < Pr; ++t)
    for (int a = 0; a < 3; ++a, ++row)
      for (int k = 0; k < 2 * DEF_K; ++k) mark(row, idx[DEF_K * (P + Pp) + 2 * DEF_K * t + k]);
  for (int l = 0; l < N; ++l)
    for (int a = 0; a < 3; ++a) mark(row++, l);
  // the corner tile pair lists only the rows with node entries in its tile
  std::vector<int> corner;
  std::vector<std::vector<int>> trows(nt);
  for (int r = 0; r < mr; ++r) {
    if ((mask[(size_t)r * W + rt / 64] >> (rt % 64)) & 1) corner.push_back(r);
    mask[(size_t)r * W + rt / 64] |= 1ull << (rt % 64);
    for (int w = 0; w < W; ++w)
      for (uint64_t b = mask[(size_t)r * W + w]; b; b &= b - 1) trows[64 * w + __builtin_ctzll(b)].push_back(r);
  }
  const int np = nt * (nt + 1) / 2;
  out->assign(3 * (size_t)np + 1, 0);
  int p = 0;
  for (int I = 0; I < nt; ++I)
    for (int J = 0; J <= I; ++J, ++p) {
      (*out)[2 * p] = I;
      (*out)[2 * p + 1] = J;
      (*out)[2 * np + p] = (int)(out->size() - (3 * (size_t)np + 1));
      if (I == rt && J == rt) {
        out->insert(out->end(), corner.begin(), corner.end());
        continue;
      }
      const bool a_is_i = trows[I].size() <= trows[J].size();
      const int o = a_is_i ? J : I;
      for (int r : a_is_i ? trows[I] : trows[J])
        if ((mask[(size_t)r * W + o / 64] >> (o % 64)) & 1) out->push_back(r);
    }
  (*out)[3 * np] = (int)(out->size() - (3 * (size_t)np + 1));
}

// The K nearest nodes to v (ties by index, skipping `exclude`) and the
// distance of the next one.
static void def_nearest(const double* nodes, int N, const double* v, int exclude, int* idx, double* dist,
                        double* dmax) {
  // the K + 1 smallest (distance, index) pairs, kept sorted by insertion
  std::pair<double, int> best[DEF_K + 1];
  int nb = 0;
  for (int k = 0; k < N; ++k) {
    if (k == exclude) continue;
    const double dx = v[0] - nodes[3 * k], dy = v[1] - nodes[3 * k + 1], dz = v[2] - nodes[3 * k + 2];
    const std::pair<double, int> e{std::sqrt(dx * dx + dy * dy + dz * dz), k};
    if (nb == DEF_K + 1 && !(e < best[DEF_K])) continue;
    int j = nb < DEF_K + 1 ? nb++ : DEF_K;
    for (; j > 0 && e < best[j - 1]; --j) best[j] = best[j - 1];
    best[j] = e;
  }
  for (int k = 0; k < DEF_K; ++k) {
    idx[k] = best[k].second;
    dist[k] = best[k].first;
  }
  *dmax = best[DEF_K].first;
}

static void def_influence(const double* nodes, int N, const double* v, int* idx, double* w) {
  double dist[DEF_K], dmax;
  def_nearest(nodes, N, v, -1, idx, dist, &dmax);
  double s = 0.0;
  for (int k = 0; k < DEF_K; ++k) {
    const double a = 1.0 - dist[k] / dmax;
    w[k] = a * a;
    s += w[k];
  }
  for (int k = 0; k < DEF_K; ++k) w[k] = s > 0.0 ? w[k] / s : 1.0 / DEF_K;
}

extern "C" {

dslam_status dslam_deform_create(dslam_context* ctx, int32_t max_nodes, int32_t max_points, dslam_deform** out) {
  if (!ctx || !out || max_nodes < DEF_K + 2 || max_nodes > 256 || max_points < 0 || max_points > (1 << 20))
    return DSLAM_ERR_INVALID;
  int m, n, ld;
  def_sizes(max_nodes, max_points, &m, &n, &ld);
  const size_t N = max_nodes, Pt = max_points;
  const size_t pairs_cap = def_pairs_cap(m, ld);
  const uint64_t bytes = def_align(N * 3 * 8) + def_align(N * DEF_K * 4) + def_align(Pt * 6 * 8) +
                         def_align(Pt * 2 * DEF_K * 4) + def_align(Pt * 2 * DEF_K * 8) + def_align(N * 12 * 8) +
                         def_align((size_t)m * ld * 8) + 2 * def_align((size_t)ld * ld * 8) + def_align(64 * 8) +
                         def_align(4) + def_align(8) + def_align(pairs_cap * 4);
  const uint64_t prev = ctx->used.fetch_add(bytes);
  if (ctx->budget && prev + bytes > ctx->budget) {
    ctx->used.fetch_sub(bytes);
    return DSLAM_ERR_NO_CAPACITY;
  }
  dslam_deform* d = new (std::nothrow) dslam_deform;
  if (!d) {
    ctx->used.fetch_sub(bytes);
    return DSLAM_ERR_NO_CAPACITY;
  }
  d->ctx = ctx;
  d->max_nodes = max_nodes;
  d->max_points = max_points;
  d->bytes = bytes;
  if (hipSetDevice(ctx->device) != hipSuccess || hipMalloc(&d->arena, bytes) != hipSuccess) {
    ctx->used.fetch_sub(bytes);
    delete d;
    return DSLAM_ERR_NO_CAPACITY;
  }
  char* q = (char*)d->arena;
  d->nodes = (double*)q; q += def_align(N * 3 * 8);
  d->nbr = (int*)q; q += def_align(N * DEF_K * 4);
  d->pts = (double*)q; q += def_align(Pt * 6 * 8);
  d->idx = (int*)q; q += def_align(Pt * 2 * DEF_K * 4);
  d->w = (double*)q; q += def_align(Pt * 2 * DEF_K * 8);
  d->x = (double*)q; q += def_align(N * 12 * 8);
  d->Jr = (double*)q; q += def_align((size_t)m * ld * 8);
  d->H = (double*)q; q += def_align((size_t)ld * ld * 8);
  d->L = (double*)q; q += def_align((size_t)ld * ld * 8);
  d->cost = (double*)q; q += def_align(64 * 8);
  d->bad = (int*)q; q += def_align(4);
  d->tiny = (double*)q; q += def_align(8);
  d->pairs = (int*)q;
  d->pairs_cap = pairs_cap;
  d->recorded = false;
  if (hipEventCreateWithFlags(&d->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipFree(d->arena);
    ctx->used.fetch_sub(bytes);
    delete d;
    return DSLAM_ERR_DEVICE;
  }
  *out = d;
  return DSLAM_OK;
}

dslam_status dslam_deform_destroy(dslam_deform* d) {
  if (!d) return DSLAM_ERR_INVALID;
  (void)hipSetDevice(d->ctx->device);
  if (d->recorded) (void)hipEventSynchronize(d->done);  // the last solve's work (not the whole device)
  (void)hipEventDestroy(d->done);
  (void)hipFree(d->arena);
  d->ctx->used.fetch_sub(d->bytes);
  delete d;
  return DSLAM_OK;
}

dslam_status dslam_deform_solve(dslam_deform* d, const dslam_deform_problem* p, int32_t iters, double* params_out,
                                double* cost_out, void* stream) {
  if (!d || !p || !params_out || iters < 1 || iters > 63) return DSLAM_ERR_INVALID;
  const int N = p->n_nodes, P = p->n_con, Pp = p->n_pin, Pr = p->global ? p->n_rel : 0;
  if (N < DEF_K + 2 || N > d->max_nodes || P < 0 || Pp < 0 || Pr < 0 || P + Pp + Pr > d->max_points) return DSLAM_ERR_INVALID;
  if (!p->nodes || (P && !p->con) || (Pp && !p->pin) || (Pr && !p->rel)) return DSLAM_ERR_INVALID;
  auto finite = [](const double* a, int n) {
    for (int i = 0; i < n; ++i)
      if (!std::isfinite(a[i])) return false;
    return true;
  };
  if (!finite(p->nodes, 3 * N) || (P && !finite(p->con, 6 * P)) || (Pp && !finite(p->pin, 3 * Pp)) ||
      (Pr && !finite(p->rel, 6 * Pr)) || !finite(p->g_W, 3))
    return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(d->mu);
  DEF_HIP(hipSetDevice(d->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  // whatever path returns from here, the work enqueued so far is marked for dslam_deform_destroy
  struct MarkDone {
    dslam_deform* d;
    hipStream_t st;
    ~MarkDone() { d->recorded = hipEventRecord(d->done, st) == hipSuccess || d->recorded; }
  } mark{d, st};
  // host: neighbour lists and influences
  std::vector<int> nbr(N * DEF_K);
  for (int l = 0; l < N; ++l) {
    double dist[DEF_K], dmax;
    def_nearest(p->nodes, N, p->nodes + 3 * l, l, &nbr[DEF_K * l], dist, &dmax);
  }
  std::vector<double> pts;
  std::vector<int> idx;
  std::vector<double> w;
  auto add_inf = [&](const double* v) {
    int i4[DEF_K];
    double w4[DEF_K];
    def_influence(p->nodes, N, v, i4, w4);
    idx.insert(idx.end(), i4, i4 + DEF_K);
    w.insert(w.end(), w4, w4 + DEF_K);
  };
  for (int k = 0; k < P; ++k) add_inf(p->con + 6 * k);
  for (int k = 0; k < Pp; ++k) add_inf(p->pin + 3 * k);
  for (int k = 0; k < Pr; ++k) {
    add_inf(p->rel + 6 * k);
    add_inf(p->rel + 6 * k + 3);
  }
  pts.insert(pts.end(), p->con, p->con + 6 * P);
  pts.insert(pts.end(), p->pin, p->pin + 3 * Pp);
  if (Pr) pts.insert(pts.end(), p->rel, p->rel + 6 * Pr);
  std::vector<double> x(12 * N, 0.0);
  for (int l = 0; l < N; ++l) x[12 * l] = x[12 * l + 4] = x[12 * l + 8] = 1.0;
  DEF_HIP(hipMemcpyAsync(d->nodes, p->nodes, sizeof(double) * 3 * N, hipMemcpyHostToDevice, st));
  DEF_HIP(hipMemcpyAsync(d->nbr, nbr.data(), sizeof(int) * nbr.size(), hipMemcpyHostToDevice, st));
  if (!pts.empty()) DEF_HIP(hipMemcpyAsync(d->pts, pts.data(), sizeof(double) * pts.size(), hipMemcpyHostToDevice, st));
  if (!idx.empty()) {
    DEF_HIP(hipMemcpyAsync(d->idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice, st));
    DEF_HIP(hipMemcpyAsync(d->w, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, st));
  }
  DEF_HIP(hipMemcpyAsync(d->x, x.data(), sizeof(double) * x.size(), hipMemcpyHostToDevice, st));
  int zero = 0;
  DEF_HIP(hipMemcpyAsync(d->bad, &zero, sizeof(int), hipMemcpyHostToDevice, st));
  int m, n, ld;
  def_sizes(N, P + Pp + Pr, &m, &n, &ld);
  std::vector<int> pairs;
  def_pair_lists(N, P, Pp, Pr, n, ld, nbr.data(), idx.data(), &pairs);
  if (pairs.size() > d->pairs_cap) return DSLAM_ERR_DEVICE;  // cannot happen: a row is in at most DEF_ROW_PAIRS pairs
  DEF_HIP(hipMemcpyAsync(d->pairs, pairs.data(), sizeof(int) * pairs.size(), hipMemcpyHostToDevice, st));
  const int np = (ld / DEF_TILE) * (ld / DEF_TILE + 1) / 2;
  DefDev dv;
  dv.N = N; dv.P = P; dv.Pp = Pp; dv.Pr = Pr; dv.global = p->global ? 1 : 0;
  def_sizes(N, P + Pp + Pr, &dv.m, &dv.n, &dv.ld);
  dv.nodes = d->nodes;
  dv.nbr = d->nbr;
  dv.con = d->pts;
  dv.con_idx = d->idx;
  dv.con_w = d->w;
  dv.pin = d->pts + 6 * P;
  dv.pin_idx = d->idx + DEF_K * P;
  dv.pin_w = d->w + DEF_K * P;
  dv.rel = d->pts + 6 * P + 3 * Pp;
  dv.rel_idx = d->idx + DEF_K * (P + Pp);
  dv.rel_w = d->w + DEF_K * (P + Pp);
  for (int i = 0; i < 3; ++i) dv.g[i] = p->g_W[i];
  dv.x = d->x;
  dv.Jr = d->Jr;
  dv.H = d->H;
  dv.L = d->L;
  dv.cost = d->cost;
  dv.bad = d->bad;
  dv.tiny = d->tiny;
  const int T = N + N * DEF_K + P + Pp + Pr + N;
  const size_t jr = (size_t)dv.m * dv.ld;
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(def_zero_kernel, dim3((unsigned)std::min<size_t>((jr + 255) / 256, 4096)), dim3(256), 0, st,
                       d->Jr, jr);
    hipLaunchKernelGGL(def_jacobian_kernel, dim3((T + 255) / 256), dim3(256), 0, st, dv);
    hipLaunchKernelGGL(def_normal_kernel, dim3(np), dim3(256), 0, st, dv, d->pairs, d->pairs + 2 * np,
                       d->pairs + 3 * np + 1);
    hipLaunchKernelGGL(def_prepare_kernel, dim3(1), dim3(256), 0, st, dv, it);
    for (int kb = 0; kb < dv.n; kb += DEF_NP * DEF_PANEL) {
      const int rest = dv.n - kb - DEF_NP * DEF_PANEL;
      const int t = rest > 0 ? (rest + DEF_TILE - 1) / DEF_TILE : 1;
      hipLaunchKernelGGL(def_chol_kernel, dim3(t * (t + 1) / 2), dim3(256), 0, st, dv, kb);
    }
    hipLaunchKernelGGL(def_solve_kernel, dim3(1), dim3(DEF_SOLVE_THREADS), 0, st, dv);
  }
  DEF_HIP(hipGetLastError());
  std::vector<double> cost(iters);
  int bad = 0;
  DEF_HIP(hipMemcpyAsync(params_out, d->x, sizeof(double) * 12 * N, hipMemcpyDeviceToHost, st));
  DEF_HIP(hipMemcpyAsync(cost.data(), d->cost, sizeof(double) * iters, hipMemcpyDeviceToHost, st));
  DEF_HIP(hipMemcpyAsync(&bad, d->bad, sizeof(int), hipMemcpyDeviceToHost, st));
  DEF_HIP(hipStreamSynchronize(st));
  if (cost_out)
    for (int i = 0; i < iters; ++i) cost_out[i] = cost[i];
  return bad ? DSLAM_ERR_SINGULAR : DSLAM_OK;
}

}  // extern "C"
