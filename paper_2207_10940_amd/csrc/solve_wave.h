// Device back ends of the dense SPD solves of the Gauss-Newton step: one
// wavefront holds the augmented system one row per lane, in registers, and
// runs Gauss-Jordan elimination without pivoting (positive pivots exist for
// every SPD matrix; a non-positive pivot reports the system as singular).
// Symmetry lets one shared-memory store per lane publish each pivot row (see
// gauss_jordan), so a step costs one store, a few wide broadcast loads and one
// FMA per remaining column.
//
// Eliminating the first 15 pivot columns of [H | b] leaves, in rows 15..32,
// exactly the Schur complement [H* | S(b)] of the previous state's block
// (Section IV-E, eq. (8)); the solve captures it on the way.
#pragma once
#include <hip/hip_runtime.h>

namespace dslam {

__device__ __forceinline__ double readlane_d(double v, int lane) {
  unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  unsigned lo = __builtin_amdgcn_readlane((unsigned)u, lane);
  unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Gauss-Jordan on the rows held by the lanes of one wavefront: lane i < NSYM
// holds R[0..NC) = row i of [A | B] with A (NSYM x NSYM) symmetric and its
// leading NSTEP x NSTEP block positive definite; the first NSTEP columns are
// eliminated (NSYM = NSTEP: a plain solve; NSYM > NSTEP: the trailing rows
// end as the Schur complement of the leading block).  After the loop every
// pivot column k < NSTEP is zero in every row but row k, whose entries are
// left unscaled: lane k's own diagonal entry R[k] is step k's pivot, which
// pivots_ok tests (the loop itself never branches on a pivot; a bad one only
// makes the eliminated values meaningless).  If cap != nullptr, rows CAP..NSTEP-1, columns CAP..NC-1 are
// stored there just before step CAP (row-major, NC - CAP per row).
//
// The trailing block of a symmetric matrix stays symmetric under elimination,
// so the pivot row's entries A[k][j], k < j < NSYM, equal column k's entries
// A[j][k], which lane j holds: one shared-memory store per lane publishes the
// whole pivot row, and every lane reads it back with wide broadcast loads.
// The pivot row's right-hand-side entries (columns NSYM..NC-1) are published
// by lane k.
//
// With FWD, rows above the pivot are left alone (forward elimination only):
// lane i then ends with row i of [U | E] where S = E^-1 U, E unit lower
// triangular and U upper triangular with U_ii the pivots.
template <int NC, int NSTEP, int CAP, bool FWD = false, int NSYM = NSTEP>
__device__ __forceinline__ void gauss_jordan(double (&R)[NC], int lane, double* col, double* cap) {
  static_assert(NSYM >= NSTEP && NSYM <= NC && NSYM <= 64, "symmetric block");
  constexpr int NR = NC - NSYM;  // right-hand-side columns
  // Software-pipelined: step k updates the next pivot column (and the
  // right-hand side) first, publishes it and starts step k+1's pivot and
  // column reads, and only then applies its remaining updates, so that one
  // step's shared-memory round trip and pivot chain overlap the previous
  // step's updates.  Every entry gets the same FMAs in the same order as
  // without the pipelining.
  double cv[NSYM];                // this step's pivot column (entries k+1..)
  double rhs[NR > 0 ? NR : 1];    // the pivot row's right-hand-side entries
  col[lane] = R[0];
  double p = readlane_d(R[0], 0);
#pragma unroll
  for (int j = 0; j < NR; ++j) rhs[j] = readlane_d(R[NSYM + j], 0);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
  for (int j = 0; j < NSYM; j += 2) {
    if (j + 1 < NSYM) {
      const double2 t = *reinterpret_cast<const double2*>(col + j);
      cv[j] = t.x;
      cv[j + 1] = t.y;
    } else {
      cv[j] = col[j];
    }
  }
#pragma unroll
  for (int k = 0; k < NSTEP; ++k) {
    if (k == CAP && cap != nullptr && lane >= CAP && lane < NSTEP) {
#pragma unroll
      for (int j = CAP; j < NC; ++j) cap[(lane - CAP) * (NC - CAP) + (j - CAP)] = R[j];
    }
    // reciprocal: hardware estimate refined by two Newton steps (full precision)
    double inv = __builtin_amdgcn_rcp(p);
    inv = fma(inv, fma(-p, inv, 1.0), inv);
    inv = fma(inv, fma(-p, inv, 1.0), inv);
    const double m = (FWD ? lane <= k : lane == k) ? 0.0 : R[k] * inv;
    if (k + 1 < NSTEP) {
      R[k + 1] = fma(-m, cv[k + 1], R[k + 1]);
#pragma unroll
      for (int j = 0; j < NR; ++j) R[NSYM + j] = fma(-m, rhs[j], R[NSYM + j]);
      // publish step k+1's column (two buffers alternate) and fetch its pivot,
      // right-hand-side entries and the column itself with 16-byte broadcast
      // reads, all in flight before this step's remaining updates
      double* c = col + ((k + 1) & 1) * 64;
      c[lane] = R[k + 1];
      const double pn = readlane_d(R[k + 1], k + 1);
      double rn[NR > 0 ? NR : 1];
#pragma unroll
      for (int j = 0; j < NR; ++j) rn[j] = readlane_d(R[NSYM + j], k + 1);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      double cn[NSYM];
#pragma unroll
      for (int j = (k + 2) & ~1; j < NSYM; j += 2) {
        if (j + 1 < NSYM) {
          const double2 t = *reinterpret_cast<const double2*>(c + j);
          cn[j] = t.x;
          cn[j + 1] = t.y;
        } else {
          cn[j] = c[j];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = k + 2; j < NSYM; ++j) R[j] = fma(-m, cv[j], R[j]);
      p = pn;
#pragma unroll
      for (int j = 0; j < NR; ++j) rhs[j] = rn[j];
#pragma unroll
      for (int j = (k + 2) & ~1; j < NSYM; ++j) cv[j] = cn[j];
    } else {
#pragma unroll
      for (int j = k + 1; j < NSYM; ++j) R[j] = fma(-m, cv[j], R[j]);
#pragma unroll
      for (int j = 0; j < NR; ++j) R[NSYM + j] = fma(-m, rhs[j], R[NSYM + j]);
    }
  }
}

template <int NC>
__device__ __forceinline__ double own_diag(const double (&R)[NC], int lane) {
  double d = 1.0;
#pragma unroll
  for (int i = 0; i < NC; ++i) d = (lane == i) ? R[i] : d;
  return d;
}

// After gauss_jordan: every pivot (lane k's own diagonal d, k < NSTEP) is
// positive and finite (uniform over the wavefront).
__device__ __forceinline__ bool pivots_ok(double d, int lane, int nstep) {
  return !__any(lane < nstep && !(d > 0.0 && d < 1e300));
}

// Linv = L^-1 for the 9x9 SPD S = L L^T (row-major, shared memory) on the
// wavefront of the calling lanes (lane < 64 of the wave): forward elimination
// of [S | I] leaves row i of [U | E] in lane i with S = E^-1 U and U = D E^-T,
// D = diag(U_ii), so L = E^-1 D^1/2 and row i of L^-1 is row i of E scaled by
// U_ii^-1/2.  col: 128 doubles of shared memory.  Returns false if S is not
// positive definite.
__device__ __forceinline__ bool chol_inv_lower9_wave(const double* S, double* Linv, int lane, double* col) {
  double R[18];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    R[j] = lane < 9 ? S[9 * lane + j] : (lane == j ? 1.0 : 0.0);
    R[9 + j] = (lane == j) ? 1.0 : 0.0;
  }
  gauss_jordan<18, 9, -1, true>(R, lane, col, nullptr);
  const double d = own_diag(R, lane);
  const bool ok = pivots_ok(d, lane, 9);
  if (lane < 9) {
    const double s = 1.0 / sqrt(d);
#pragma unroll
    for (int j = 0; j < 9; ++j) Linv[9 * lane + j] = (j <= lane) ? R[9 + j] * s : 0.0;
  }
  return ok;
}

template <int N, int CAP>
__device__ __forceinline__ bool solve_rows(const double* H, const double* b, int lane, double* dz, double* col,
                                           double* cap) {
  double R[N + 1];
  // every lane reads a row (lanes past N read row 0 and discard it), so the
  // loads need no per-entry branches
  const int row = lane < N ? lane : 0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double h = H[row * 33 + j];
    R[j] = lane < N ? h : (lane == j ? 1.0 : 0.0);
  }
  const double bb = b[row];
  R[N] = lane < N ? bb : 0.0;
  gauss_jordan<N + 1, N, CAP>(R, lane, col, cap);
  const double d = own_diag(R, lane);
  const double x = R[N] / d;
  const bool finite = lane >= N || (x == x && fabs(x) < 1e30);
  if (lane < N) dz[lane] = x;
  return pivots_ok(d, lane, N) && !__any(!finite);
}

// dz = H^-1 b (H leading dimension 33, shared memory); n is 33 or 6.  With
// schur != nullptr (n == 33) also writes the 18 x 19 Schur complement of the
// leading 15x15 block of [H | b].  Called by every thread; wave 0 computes.
__device__ int spd_solve_dev(const double* H, const double* b, int n, double* dz, double* schur) {
  __shared__ int bad;
  __shared__ __attribute__((aligned(16))) double col[128];
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    bool ok = false;
    if (n == 33) ok = solve_rows<33, 15>(H, b, lane, dz, col, schur);
    else if (n == 6) ok = solve_rows<6, -1>(H, b, lane, dz, col, nullptr);
    if (lane == 0) bad = ok ? 0 : 1;
  }
  __syncthreads();
  return bad;
}

}  // namespace dslam
