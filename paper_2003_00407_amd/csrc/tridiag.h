// Symmetric tridiagonal eigen-solver pieces (FP64), written so that each
// routine runs either per GPU thread or on the host (for CPU checks).
//
//  * sturm_count: number of eigenvalues of T below x (LDL^T pivot signs);
//  * bisect_eig:  the i-th smallest eigenvalue by bisection on the Sturm count;
//  * invit:       inverse iteration for one eigenvector, tridiagonal LU with
//                 partial pivoting, re-orthogonalised against already computed
//                 vectors of the same cluster (as LAPACK's dstein does).
// T has diagonal d[0..n) and off-diagonal e[0..n-1).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace dg {

__host__ __device__ inline int sturm_count(const double* d, const double* e, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// i-th smallest (0-based) eigenvalue in [lo, hi]
__host__ __device__ inline double bisect_eig(const double* d, const double* e, int n, int i, double lo, double hi,
                                             double pivmin) {
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(d, e, n, mid, pivmin) > i) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// strided views (per-thread arrays interleaved across the threads of a block)
struct StridedD {
  double* p;
  int s;
  __host__ __device__ double& operator[](int i) const { return p[(size_t)i * s]; }
};
struct StridedB {
  unsigned char* p;
  int s;
  __host__ __device__ unsigned char& operator[](int i) const { return p[(size_t)i * s]; }
};

// deterministic start vector entries in (-1, 1)
__host__ __device__ inline double hash_unit(unsigned a, unsigned b) {
  unsigned long long x = (unsigned long long)a * 0x9E3779B97F4A7C15ull ^ ((unsigned long long)b + 0x632BE59BD9B4E019ull);
  x ^= x >> 31;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 29;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 32;
  return (double)(x & 0xFFFFFFFFull) / 2147483648.0 - 1.0;
}

// Factor T - s I with partial pivoting: on return a (diagonal of U), b (first
// super-diagonal), u2 (second), l (multipliers), piv (row swaps).
template <typename DA, typename BA>
__host__ __device__ inline void tri_lu(const double* d, const double* e, int n, double s, double tiny, DA a, DA b,
                                       DA u2, DA l, BA piv) {
  for (int k = 0; k < n; ++k) {
    a[k] = d[k] - s;
    b[k] = (k < n - 1) ? e[k] : 0.0;
    u2[k] = 0.0;
  }
  for (int k = 0; k < n - 1; ++k) {
    const double ck = e[k];
    if (fabs(a[k]) >= fabs(ck)) {
      piv[k] = 0;
      const double m = (a[k] != 0.0) ? ck / a[k] : 0.0;
      l[k] = m;
      a[k + 1] -= m * b[k];
      u2[k] = 0.0;
    } else {
      piv[k] = 1;
      const double m = a[k] / ck;
      l[k] = m;
      a[k] = ck;
      const double t = a[k + 1];
      a[k + 1] = b[k] - m * t;
      u2[k] = (k + 1 < n - 1) ? b[k + 1] : 0.0;
      b[k] = t;
      if (k + 1 < n - 1) b[k + 1] = -m * u2[k];
    }
    if (a[k] == 0.0) a[k] = tiny;
  }
  if (a[n - 1] == 0.0) a[n - 1] = tiny;
}

// solve (T - s I) x = y in place with the factors of tri_lu
template <typename DA, typename BA>
__host__ __device__ inline void tri_solve(int n, DA a, DA b, DA u2, DA l, BA piv, DA y) {
  for (int k = 0; k < n - 1; ++k) {
    if (piv[k]) {
      const double t = y[k];
      y[k] = y[k + 1];
      y[k + 1] = t;
    }
    y[k + 1] -= l[k] * y[k];
  }
  y[n - 1] /= a[n - 1];
  if (n >= 2) y[n - 2] = (y[n - 2] - b[n - 2] * y[n - 1]) / a[n - 2];
  for (int k = n - 3; k >= 0; --k) y[k] = (y[k] - b[k] * y[k + 1] - u2[k] * y[k + 2]) / a[k];
}

}  // namespace dg
