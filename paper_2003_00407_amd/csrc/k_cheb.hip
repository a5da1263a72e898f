// Chebyshev filter steps and the band-energy adjoint (elementwise / reduction kernels).
//
// Algorithm 2 step 2 with Eq. (8)'s three-term recurrence, scaled as in Zhou &
// Saad (2007): with e = (b - a)/2, c = (b + a)/2, sigma_1 = e / (a0 - c),
//   Y_1     = (sigma_1 / e) (H - c) Y_0
//   Y_{k+1} = (2 sigma_{k+1} / e) (H - c) Y_k - sigma_k sigma_{k+1} Y_{k-1},
//   sigma_{k+1} = 1 / (2 / sigma_1 - sigma_k).
// The step coefficients are computed on the device from each element's bounds.
#include "dg_internal.h"

#include <algorithm>

namespace dg {

struct ChebCoef {
  double alpha, beta, c;   // Y_{k+1} = alpha (HY_k - c Y_k) - beta Y_{k-1}
};

__device__ __forceinline__ ChebCoef cheb_coef(double a, double b, double a0, int k) {
  const double e = 0.5 * (b - a), c = 0.5 * (b + a);
  const double s1 = e / (a0 - c);
  if (k == 0) return {s1 / e, 0.0, c};
  double s = s1, sn = s1;
  for (int i = 1; i <= k; ++i) {
    sn = 1.0 / (2.0 / s1 - s);
    if (i < k) s = sn;
  }
  return {2.0 * sn / e, s * sn, c};
}

// bounds of element e: from the context (ChFSI: a = largest Ritz value of the
// block, a0 = smallest, b = upper spectral bound) or from a caller array
__device__ __forceinline__ void elem_bounds(const ElemDev& E, const double* bounds, int e, double& a, double& b,
                                            double& a0) {
  if (bounds) {
    a = bounds[3 * e];
    b = bounds[3 * e + 1];
    a0 = bounds[3 * e + 2];
  } else {
    const int KP = E.kmax3 + 2;
    const double* th = E.small + SmallLayout::vec(KP) + VS_THETA * KP;
    a = th[E.K - 1];
    a0 = th[0];
    b = E.bup;
  }
}

struct ChebStepArgs {
  const ElemDev* elems;
  const int* active;
  int y_blk, hy_blk, prev_blk;   // prev_blk < 0 for the first step
  int k;                         // step index (0 produces Y_1)
  int ncols;                     // <= 0: E.K
  const double* bounds;          // nullptr: context bounds
};

// hy <- alpha (hy - c y) - beta prev   (in place in hy)
template <typename T>
__global__ void __launch_bounds__(256) k_cheb_step(ChebStepArgs A) {
  const int e = blockIdx.z;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int ncols = A.ncols > 0 ? A.ncols : E.K;
  const int j = blockIdx.y;
  if (j >= ncols) return;
  double a, b, a0;
  elem_bounds(E, A.bounds, e, a, b, a0);
  const ChebCoef cf = cheb_coef(a, b, a0, A.k);
  const T* y = reinterpret_cast<const T*>(E.blk[A.y_blk]) + (size_t)j * E.ld;
  T* hy = reinterpret_cast<T*>(E.blk[A.hy_blk]) + (size_t)j * E.ld;
  const T* pv = A.prev_blk >= 0 ? reinterpret_cast<const T*>(E.blk[A.prev_blk]) + (size_t)j * E.ld : nullptr;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < E.N; r += gridDim.x * 256) {
    double v = cf.alpha * (double(hy[r]) - cf.c * double(y[r]));
    if (pv) v -= cf.beta * double(pv[r]);
    hy[r] = T(v);
  }
}

// adjoint step: A_k = alpha_k (H A_{k+1} - c A_{k+1}) - beta_{k+1} A_{k+2}
// (t holds H A_{k+1} on entry and A_k on exit)
struct AdjStepArgs {
  const ElemDev* elems;
  int a1_blk, t_blk, a2_blk;   // a2_blk < 0 when A_{k+2} = 0
  int k, m;                    // step index and filter degree
  int ncols;
  const double* bounds;
};

template <typename T>
__global__ void __launch_bounds__(256) k_adj_step(AdjStepArgs A) {
  const int e = blockIdx.z;
  const ElemDev& E = A.elems[e];
  const int j = blockIdx.y;
  if (j >= A.ncols) return;
  double a, b, a0;
  elem_bounds(E, A.bounds, e, a, b, a0);
  const ChebCoef ck = cheb_coef(a, b, a0, A.k);
  const double beta_next = (A.k + 1 <= A.m - 1) ? cheb_coef(a, b, a0, A.k + 1).beta : 0.0;
  const T* a1 = reinterpret_cast<const T*>(E.blk[A.a1_blk]) + (size_t)j * E.ld;
  T* t = reinterpret_cast<T*>(E.blk[A.t_blk]) + (size_t)j * E.ld;
  const T* a2 = A.a2_blk >= 0 ? reinterpret_cast<const T*>(E.blk[A.a2_blk]) + (size_t)j * E.ld : nullptr;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < E.N; r += gridDim.x * 256) {
    double v = ck.alpha * (double(t[r]) - ck.c * double(a1[r]));
    if (a2) v -= beta_next * double(a2[r]);
    t[r] = T(v);
  }
}

// partial[e][j] = sum_r u_j(r) w_j(r) (FP64 accumulation, fixed order)
template <typename T>
__global__ void __launch_bounds__(256) k_coldot(const ElemDev* elems, int u_blk, int w_blk, int ncols,
                                               double* partial, int pstride) {
  const int e = blockIdx.y, j = blockIdx.x;
  const ElemDev& E = elems[e];
  if (j >= ncols) return;
  const T* u = reinterpret_cast<const T*>(E.blk[u_blk]) + (size_t)j * E.ld;
  const T* w = reinterpret_cast<const T*>(E.blk[w_blk]) + (size_t)j * E.ld;
  double s = 0.0;
  for (int r = threadIdx.x; r < E.N; r += 256) s += double(u[r]) * double(w[r]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[(size_t)e * pstride + j] = sh[0] + sh[1] + sh[2] + sh[3];
}

// E[e] = scale * sum_j f_j partial[e][j]
__global__ void k_wsum(const double* partial, int pstride, const double* f, int ncols, double scale, double* E,
                       int n_elem) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  double s = 0.0;
  for (int j = 0; j < ncols; ++j) s += f[j] * partial[(size_t)e * pstride + j];
  E[e] = scale * s;
}

// vbar[e][r] = beta * vbar[e][r] + sum_j wt_j * u_j(r) y_j(r), wt_j = coef_e * (f ? f_j : 1)
// coef_e: alpha_k of the element (step k >= 0) or the caller's scale (k < 0)
struct VbarArgs {
  const ElemDev* elems;
  int u_blk, y_blk;
  int ncols;
  const double* f;
  const double* scale;        // per element multiplier (dE), may be nullptr
  int k, m;                   // k >= 0: multiply by alpha_k of the filter
  const double* bounds;
  double beta;                // 0: overwrite
  double* vbar;               // FP64, packed N per element
  const long long* off;       // packed offsets (N per element)
};

template <typename T>
__global__ void __launch_bounds__(256) k_vbar(VbarArgs A) {
  const int e = blockIdx.y;
  const ElemDev& E = A.elems[e];
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= E.N) return;
  double coef = A.scale ? A.scale[e] : 1.0;
  if (A.k >= 0) {
    double a, b, a0;
    elem_bounds(E, A.bounds, e, a, b, a0);
    coef *= cheb_coef(a, b, a0, A.k).alpha;
  }
  const T* u = reinterpret_cast<const T*>(E.blk[A.u_blk]);
  const T* y = reinterpret_cast<const T*>(E.blk[A.y_blk]);
  double s = 0.0;
  for (int j = 0; j < A.ncols; ++j) {
    const double w = A.f ? A.f[j] : 1.0;
    s += w * double(u[(size_t)j * E.ld + r]) * double(y[(size_t)j * E.ld + r]);
  }
  double* v = A.vbar + A.off[e] + r;
  *v = (A.beta != 0.0 ? A.beta * *v : 0.0) + coef * s;
}

// out[:, j] = s_e * f_j * in[:, j]
template <typename T>
__global__ void __launch_bounds__(256) k_scale_cols(const ElemDev* elems, int in_blk, int out_blk, int ncols,
                                                    const double* f, const double* scale, double mult) {
  const int e = blockIdx.z, j = blockIdx.y;
  const ElemDev& E = elems[e];
  if (j >= ncols) return;
  const double s = mult * (scale ? scale[e] : 1.0) * (f ? f[j] : 1.0);
  const T* in = reinterpret_cast<const T*>(E.blk[in_blk]) + (size_t)j * E.ld;
  T* out = reinterpret_cast<T*>(E.blk[out_blk]) + (size_t)j * E.ld;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < E.N; r += gridDim.x * 256) out[r] = T(s * double(in[r]));
}

// block copy (same precision); blocks may live outside E.blk (checkpoints)
template <typename T>
__global__ void __launch_bounds__(256) k_copy_cols(const ElemDev* elems, const void* const* src_tab,
                                                   void* const* dst_tab, int src_blk, int dst_blk, int ncols) {
  const int e = blockIdx.z, j = blockIdx.y;
  const ElemDev& E = elems[e];
  if (j >= (ncols > 0 ? ncols : E.K)) return;
  const T* s = reinterpret_cast<const T*>(src_tab ? src_tab[e] : E.blk[src_blk]) + (size_t)j * E.ld;
  T* d = reinterpret_cast<T*>(dst_tab ? dst_tab[e] : E.blk[dst_blk]) + (size_t)j * E.ld;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < E.N; r += gridDim.x * 256) d[r] = s[r];
}

// new V_eff (packed FP64, N per element) into the element arrays
__global__ void __launch_bounds__(256) k_set_potential(const ElemDev* elems, const double* v, const long long* off) {
  const int e = blockIdx.y;
  const ElemDev& E = elems[e];
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= E.N) return;
  const double x = v[off[e] + r];
  const_cast<double*>(E.v64)[r] = x;
  const_cast<float*>(E.v32)[r] = float(x);
}

// spectral upper bound after a potential update: bup = bup_base + max(max V, 0),
// a NaN in V propagates into bup (fmax would drop it)
__global__ void __launch_bounds__(1024) k_update_bounds(ElemDev* elems) {
  const int e = blockIdx.x;
  ElemDev& E = elems[e];
  double m = -1e300;
  bool nan = false;
  for (int r = threadIdx.x; r < E.N; r += 1024) {
    const double x = E.v64[r];
    nan |= !(x == x);
    m = fmax(m, x);
  }
  __shared__ double sh[16];
  __shared__ int snan;
  if (threadIdx.x == 0) snan = 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  if (nan) atomicOr(&snan, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = sh[0];
    for (int w = 1; w < 16; ++w) mm = fmax(mm, sh[w]);
    E.bup = snan ? __builtin_nan("") : E.bup_base + fmax(mm, 0.0);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int maxN(Ctx& c) {
  int m = 0;
  for (int e = 0; e < c.n_elem; ++e) m = std::max(m, c.N[e]);
  return m;
}

static dim3 col_grid(Ctx& c, int ncols) {
  const int gx = std::min(64, (maxN(c) + 255) / 256);
  return dim3(gx, ncols, c.n_elem);
}

int launch_cheb_step(Ctx& c, int prec, int y_blk, int hy_blk, int prev_blk, int k, int ncols, const int* active,
                     const double* bounds) {
  int kmax = ncols;
  if (ncols <= 0)
    for (int e = 0; e < c.n_elem; ++e) kmax = std::max(kmax, c.K[e]);
  ChebStepArgs a{c.elems_dev, active, y_blk, hy_blk, prev_blk, k, ncols, bounds};
  TimedScope ts(c, TC_OTHER);
  if (prec == DG_FP64) hipLaunchKernelGGL(k_cheb_step<double>, col_grid(c, kmax), dim3(256), 0, c.stream, a);
  else hipLaunchKernelGGL(k_cheb_step<float>, col_grid(c, kmax), dim3(256), 0, c.stream, a);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_adj_step(Ctx& c, int prec, int a1_blk, int t_blk, int a2_blk, int k, int m, int ncols,
                    const double* bounds) {
  AdjStepArgs a{c.elems_dev, a1_blk, t_blk, a2_blk, k, m, ncols, bounds};
  TimedScope ts(c, TC_OTHER);
  if (prec == DG_FP64) hipLaunchKernelGGL(k_adj_step<double>, col_grid(c, ncols), dim3(256), 0, c.stream, a);
  else hipLaunchKernelGGL(k_adj_step<float>, col_grid(c, ncols), dim3(256), 0, c.stream, a);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_weighted_dot(Ctx& c, int prec, int u_blk, int w_blk, int ncols, const double* f, double scale,
                        double* E) {
  double* partial = c.gram_part;   // n_elem x ncols scratch
  const int pstride = (int)std::min<long long>(c.gram_part_stride, 1 << 20);
  dim3 g(ncols, c.n_elem);
  if (prec == DG_FP64) hipLaunchKernelGGL(k_coldot<double>, g, dim3(256), 0, c.stream, c.elems_dev, u_blk, w_blk, ncols, partial, pstride);
  else hipLaunchKernelGGL(k_coldot<float>, g, dim3(256), 0, c.stream, c.elems_dev, u_blk, w_blk, ncols, partial, pstride);
  hipLaunchKernelGGL(k_wsum, dim3((c.n_elem + 63) / 64), dim3(64), 0, c.stream, partial, pstride, f, ncols, scale, E,
                     c.n_elem);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_vbar(Ctx& c, int prec, int u_blk, int y_blk, int ncols, const double* f, const double* scale, int k,
                int m, const double* bounds, double beta, double* vbar) {
  VbarArgs a{c.elems_dev, u_blk, y_blk, ncols, f, scale, k, m, bounds, beta, vbar, c.dev_off_grid};
  dim3 g((maxN(c) + 255) / 256, c.n_elem);
  if (prec == DG_FP64) hipLaunchKernelGGL(k_vbar<double>, g, dim3(256), 0, c.stream, a);
  else hipLaunchKernelGGL(k_vbar<float>, g, dim3(256), 0, c.stream, a);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_scale_cols(Ctx& c, int prec, int in_blk, int out_blk, int ncols, const double* f, const double* scale,
                      double mult) {
  if (prec == DG_FP64) hipLaunchKernelGGL(k_scale_cols<double>, col_grid(c, ncols), dim3(256), 0, c.stream, c.elems_dev, in_blk, out_blk, ncols, f, scale, mult);
  else hipLaunchKernelGGL(k_scale_cols<float>, col_grid(c, ncols), dim3(256), 0, c.stream, c.elems_dev, in_blk, out_blk, ncols, f, scale, mult);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_copy_cols(Ctx& c, int prec, const void* const* src_tab, void* const* dst_tab, int src_blk, int dst_blk,
                     int ncols) {
  int gcols = ncols;
  if (gcols <= 0)
    for (int e = 0; e < c.n_elem; ++e) gcols = std::max(gcols, c.K[e]);
  if (prec == DG_FP64) hipLaunchKernelGGL(k_copy_cols<double>, col_grid(c, gcols), dim3(256), 0, c.stream, c.elems_dev, src_tab, dst_tab, src_blk, dst_blk, ncols);
  else hipLaunchKernelGGL(k_copy_cols<float>, col_grid(c, gcols), dim3(256), 0, c.stream, c.elems_dev, src_tab, dst_tab, src_blk, dst_blk, ncols);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int set_potential(Ctx& c, const double* v) {
  if (!v) {
    set_error("v_dev is NULL");
    return DG_ERR_ARG;
  }
  dim3 g((maxN(c) + 255) / 256, c.n_elem);
  hipLaunchKernelGGL(k_set_potential, g, dim3(256), 0, c.stream, c.elems_dev, v, c.dev_off_grid);
  DG_HIP(hipGetLastError());
  int st;
  if ((st = launch_update_bounds(c))) return st;
  // the eigenvectors stay as a warm start, but are no solution of the new H
  c.solved = false;
  // a band energy taken at the old potential can no longer be differentiated
  c.be_valid = false;
  return DG_OK;
}

int launch_update_bounds(Ctx& c) {
  hipLaunchKernelGGL(k_update_bounds, dim3(c.n_elem), dim3(1024), 0, c.stream, c.elems_dev);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace dg
