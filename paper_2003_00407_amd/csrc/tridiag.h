// Symmetric tridiagonal eigen-solver pieces (FP64), one GPU thread each.
//
//  * sturm_count: number of eigenvalues of T below x (LDL^T pivot signs);
//  * tri_lu / tri_solve: LU factors of T - sI with partial pivoting and
//    solves with them, the step of inverse iteration for one eigenvector
//    (vectors of a cluster are re-orthogonalised by the caller, as LAPACK's
//    dstein does).
// T has diagonal d[0..n) and off-diagonal e[0..n-1). Divisions use the
// hardware reciprocal refined by two Newton steps (error of a few ulps), so
// that the sequential recurrences carry five dependent operations per step
// instead of a full division.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace dg {

__device__ __forceinline__ double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double t = fma(-q, r, 1.0);
  r = fma(r, t, r);
  t = fma(-q, r, 1.0);
  return fma(r, t, r);
}

__device__ inline int sturm_count(const double* d, const double* e, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    const double e2 = e[i - 1] * e[i - 1];
    q = fma(-e2, recip(q), d[i] - x);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// strided views (per-thread arrays interleaved across the threads of a block)
struct StridedD {
  double* p;
  int s;
  __device__ double& operator[](int i) const { return p[(size_t)i * s]; }
};
struct StridedB {
  unsigned char* p;
  int s;
  __device__ unsigned char& operator[](int i) const { return p[(size_t)i * s]; }
};

// deterministic start vector entries in (-1, 1)
__device__ inline double hash_unit(unsigned a, unsigned b) {
  unsigned long long x = (unsigned long long)a * 0x9E3779B97F4A7C15ull ^ ((unsigned long long)b + 0x632BE59BD9B4E019ull);
  x ^= x >> 31;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 29;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 32;
  return (double)(x & 0xFFFFFFFFull) / 2147483648.0 - 1.0;
}

// Factor T - s I = P L U with partial pivoting: on return ai (reciprocal of the
// diagonal of U), b (first super-diagonal), u2 (second), l (multipliers), piv
// (row swaps). A zero pivot is replaced by tiny. The running diagonal entry and
// the next super-diagonal are carried in registers.
template <typename DA, typename BA>
__device__ inline void tri_lu(const double* d, const double* e, int n, double s, double tiny, DA ai, DA b,
                              DA u2, DA l, BA piv) {
  double ak = d[0] - s;            // current diagonal of row k
  double bk = n > 1 ? e[0] : 0.0;  // current first super-diagonal of row k
  for (int k = 0; k < n - 1; ++k) {
    const double ck = e[k];                          // sub-diagonal below the pivot
    const double an = d[k + 1] - s;                  // row k+1 diagonal
    const double bn = (k + 1 < n - 1) ? e[k + 1] : 0.0;   // row k+1 super-diagonal
    if (fabs(ak) >= fabs(ck)) {
      const double a0 = ak != 0.0 ? ak : tiny;
      const double r = recip(a0);
      const double m = ck * r;
      piv[k] = 0;
      l[k] = m;
      ai[k] = r;
      b[k] = bk;
      u2[k] = 0.0;
      ak = fma(-m, bk, an);
      bk = bn;
    } else {
      const double r = recip(ck);
      const double m = ak * r;
      piv[k] = 1;
      l[k] = m;
      ai[k] = r;             // the pivot row is row k+1: diagonal ck
      b[k] = an;
      u2[k] = bn;
      ak = fma(-m, an, bk);
      bk = -m * bn;
    }
  }
  ai[n - 1] = recip(ak != 0.0 ? ak : tiny);
}

// solve (T - s I) x = y in place with the factors of tri_lu
template <typename DA, typename BA>
__device__ inline void tri_solve(int n, DA ai, DA b, DA u2, DA l, BA piv, DA y) {
  double cur = y[0];
  for (int k = 0; k < n - 1; ++k) {
    double nxt = y[k + 1];
    if (piv[k]) {
      const double t = cur;
      cur = nxt;
      nxt = t;
    }
    y[k] = cur;
    cur = fma(-l[k], cur, nxt);
  }
  // back substitution with U (diagonal 1/ai, super-diagonals b and u2)
  double y1 = cur * ai[n - 1];   // y[k+1]
  y[n - 1] = y1;
  double y2 = 0.0;               // y[k+2]
  for (int k = n - 2; k >= 0; --k) {
    const double v = (y[k] - b[k] * y1 - u2[k] * y2) * ai[k];
    y[k] = v;
    y2 = y1;
    y1 = v;
  }
}

}  // namespace dg
