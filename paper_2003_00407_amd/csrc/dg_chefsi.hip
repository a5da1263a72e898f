// CheFSI on the DG Hamiltonian (Algorithm 2 with the block-row product of Eq. (8)).
//
// The global problem H^DG C = C Lambda is one more "element" to the subspace-iteration
// machinery: a single block of N_b = sum_k J_k rows (the ALBs of every element,
// element-major) and n_vec columns.  Filter steps, Gram matrices, the Cholesky /
// projected eigenproblem and the rotations are the element solver's own kernels; two
// pieces are specific to H^DG:
//   * k_dg_bsr: Y = H^DG X for a block of columns, one workgroup per (element row k,
//     16 columns): Y_k = sum over the nonzero blocks (k, k') of H_{k,k'} X_{k'} (Eq.
//     (8)), X_{k'} staged through LDS, the J_k x J_k' block read from HBM column by
//     column (coalesced along the rows of the block);
//   * the upper bound b_up by a k-step Lanczos run (Algorithm 2, step 1): seeded start,
//     H v by k_dg_bsr, one single-workgroup update kernel per step, and the largest
//     eigenvalue of the Lanczos tridiagonal (Sturm bisection) plus the last residual
//     norm, written straight into the device-side bound the filter reads.
// The lower bounds are the previous Ritz values (largest and smallest of the block),
// as in the element solver.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "dg_internal.h"

namespace dg {

int run_chfsi(Ctx& c, int prec, double tol, int max_iter, int degree, int* iters, int* n_done);

constexpr int kBsrCols = 16;
constexpr int kBsrThreads = 128;   // >= the largest J_k (88)
constexpr int kLanczosMax = 64;

// H^DG X for columns [16 y, 16 y + 16) of block in_blk into out_blk
__global__ void __launch_bounds__(kBsrThreads) k_dg_bsr(const ElemDev* elems, DgOp op, int in_blk, int out_blk,
                                                        int ncols, const int* active) {
  if (active && !active[0]) return;
  const ElemDev& E = elems[0];
  const int K = ncols > 0 ? ncols : E.K;
  const int c0 = blockIdx.y * kBsrCols;
  if (c0 >= K) return;
  const int k = blockIdx.x;
  const int Jk = op.J[k];
  const long long r0 = op.roff[k];
  const double* X = reinterpret_cast<const double*>(E.blk[in_blk]);
  double* Y = reinterpret_cast<double*>(E.blk[out_blk]);
  const int i = threadIdx.x;
  __shared__ double xs[88][kBsrCols + 1];
  double acc[kBsrCols];
#pragma unroll
  for (int c = 0; c < kBsrCols; ++c) acc[c] = 0.0;
  for (long long b = op.row_ptr[k]; b < op.row_ptr[k + 1]; ++b) {
    const int nb = op.col_idx[b];
    const int Jn = op.J[nb];
    const long long rn = op.roff[nb];
    const double* Hb = op.H + op.boff[b];
    __syncthreads();
    for (int x = threadIdx.x; x < Jn * kBsrCols; x += kBsrThreads) {
      const int l = x % Jn, c = x / Jn;
      xs[l][c] = c0 + c < K ? X[rn + l + (long long)(c0 + c) * E.ld] : 0.0;
    }
    __syncthreads();
    if (i < Jk) {
      for (int l = 0; l < Jn; ++l) {
        const double h = Hb[i + (long long)l * Jk];
#pragma unroll
        for (int c = 0; c < kBsrCols; ++c) acc[c] += h * xs[l][c];
      }
    }
  }
  if (i < Jk) {
#pragma unroll
    for (int c = 0; c < kBsrCols; ++c)
      if (c0 + c < K) Y[r0 + i + (long long)(c0 + c) * E.ld] = acc[c];
  }
}

int launch_dg_bsr(Ctx& c, int in_blk, int out_blk, int ncols, const int* active) {
  const int K = ncols > 0 ? ncols : c.K[0];
  TimedScope ts(c, TC_OTHER);
  hipLaunchKernelGGL(k_dg_bsr, dim3(c.dg_op.M, (K + kBsrCols - 1) / kBsrCols), dim3(kBsrThreads), 0, c.stream,
                     c.elems_dev, c.dg_op, in_blk, out_blk, ncols, active);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

// ---------------------------------------------------------------------------
// Lanczos upper bound
// ---------------------------------------------------------------------------
__device__ double lz_block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  return s;
}

// state lz: [0, 64) alpha, [64, 128) beta, 128 steps done, 129 stopped (invariant subspace)
// v = column 0 of blk_v, v_prev = column 1 of blk_v, w = H v = column 0 of blk_w.
// step < 0: normalise the start vector and clear v_prev.
__global__ void __launch_bounds__(1024) k_lz_step(const ElemDev* elems, int blk_v, int blk_w, int step, double* lz) {
  const ElemDev& E = elems[0];
  __shared__ double sh[16];
  double* v = reinterpret_cast<double*>(E.blk[blk_v]);
  double* vp = v + E.ld;
  const double* w = reinterpret_cast<const double*>(E.blk[blk_w]);
  const int N = E.N;
  if (step < 0) {
    double s = 0.0;
    for (int r = threadIdx.x; r < N; r += blockDim.x) s += v[r] * v[r];
    const double nrm = sqrt(lz_block_sum(s, sh));
    for (int r = threadIdx.x; r < N; r += blockDim.x) {
      v[r] = nrm > 0.0 ? v[r] / nrm : 0.0;
      vp[r] = 0.0;
    }
    if (threadIdx.x == 0) {
      lz[128] = 0.0;
      lz[129] = nrm > 0.0 ? 0.0 : 1.0;
    }
    return;
  }
  if (lz[129] != 0.0) return;   // uniform: every thread reads the same flag
  double s = 0.0;
  for (int r = threadIdx.x; r < N; r += blockDim.x) s += v[r] * w[r];
  const double alpha = lz_block_sum(s, sh);
  const double beta_prev = step > 0 ? lz[64 + step - 1] : 0.0;
  double f2 = 0.0;
  for (int r = threadIdx.x; r < N; r += blockDim.x) {
    const double f = w[r] - alpha * v[r] - beta_prev * vp[r];
    f2 += f * f;
  }
  const double beta = sqrt(lz_block_sum(f2, sh));
  for (int r = threadIdx.x; r < N; r += blockDim.x) {
    const double f = w[r] - alpha * v[r] - beta_prev * vp[r];
    vp[r] = v[r];
    v[r] = beta > 0.0 ? f / beta : 0.0;
  }
  if (threadIdx.x == 0) {
    lz[step] = alpha;
    lz[64 + step] = beta;
    lz[128] = step + 1;
    if (!(beta > 0.0)) lz[129] = 1.0;
  }
}

// Sturm count: eigenvalues of the m x m tridiagonal (d, e) below x
__device__ int lz_count_below(const double* d, const double* e, int m, double x) {
  int cnt = 0;
  double q = 1.0;
  for (int i = 0; i < m; ++i) {
    const double off = i > 0 ? e[i - 1] * e[i - 1] : 0.0;
    q = d[i] - x - (i > 0 ? off / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// b_up = lambda_max(T_m) + |beta_m| into the element's filter bound
__global__ void k_lz_bound(ElemDev* elems, const double* lz) {
  if (threadIdx.x != 0) return;
  const int m = (int)lz[128];
  if (m <= 0) return;
  const double* d = lz;
  const double* e = lz + 64;
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-13 * fmax(fabs(lo), fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (lz_count_below(d, e, m, mid) == m) hi = mid;
    else lo = mid;
  }
  elems[0].bup = hi + fabs(e[m - 1]);
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
namespace {
size_t al256(size_t x) { return (x + 255) / 256 * 256; }

struct ChefsiLayout {
  int M = 0, Nb = 0, K = 0, ld = 0, Kpad = 0, part_ld = 0, nsplit = 16;
  size_t part_stride = 0;
  size_t off_elem = 0, off_blk[kMaxBlocks] = {}, off_small = 0, off_part = 0, off_ints = 0, off_dbl = 0,
         off_phase = 0, off_rowptr = 0, off_col = 0, off_boff = 0, off_roff = 0, off_J = 0, off_lz = 0,
         off_offkall = 0, off_v64 = 0, off_v32 = 0, total = 0;
};

ChefsiLayout chefsi_layout(int M, int Nb, int K, int n_blocks) {
  ChefsiLayout L;
  L.M = M;
  L.Nb = Nb;
  L.K = K;
  L.ld = (Nb + 63) / 64 * 64;
  L.Kpad = K + (K & 1);
  L.part_ld = 3 * K;
  L.part_stride = std::max((size_t)L.nsplit * L.part_ld * L.part_ld, (size_t)6 * (L.part_ld + 2) * 512);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = al256(off + bytes);
    return o;
  };
  L.off_elem = take(sizeof(ElemDev));
  for (int b = 0; b < kMaxBlocks; ++b) L.off_blk[b] = take(sizeof(double) * (size_t)L.ld * L.Kpad);
  L.off_small = take(sizeof(double) * SmallLayout::total(3 * K + 2));
  L.off_part = take(sizeof(double) * L.part_stride);
  L.off_ints = take(sizeof(int) * 16);
  L.off_dbl = take(sizeof(double) * 16);
  L.off_phase = take(sizeof(long long) * 16);
  L.off_rowptr = take(sizeof(long long) * (M + 1));
  L.off_col = take(sizeof(int) * std::max(1, n_blocks));
  L.off_boff = take(sizeof(long long) * std::max(1, n_blocks));
  L.off_roff = take(sizeof(long long) * (M + 1));
  L.off_J = take(sizeof(int) * M);
  L.off_lz = take(sizeof(double) * 136);
  L.off_offkall = take(sizeof(long long) * 2);
  // a zero potential: the residual kernel also forms x^T V x for the element solver's
  // preconditioner energy, which the DG iteration does not use
  L.off_v64 = take(sizeof(double) * (size_t)L.ld);
  L.off_v32 = take(sizeof(float) * (size_t)L.ld);
  L.total = off + 256;
  return L;
}
}  // namespace

size_t chefsi_work_bytes(int M, int Nb, int K, int n_blocks) { return chefsi_layout(M, Nb, K, n_blocks).total; }

int chefsi(hipStream_t stream, const std::vector<int>& Js, const dg_chefsi_params& p, int n_blocks,
           const int64_t* row_ptr, const int32_t* col_idx, const int64_t* block_off, const double* hdg,
           double* x, double* eig, double* resid, void* work, size_t work_bytes, int* iters_out) {
  const int M = (int)Js.size();
  std::vector<long long> roff(M + 1, 0);
  for (int k = 0; k < M; ++k) roff[k + 1] = roff[k] + Js[k];
  const int Nb = (int)roff[M];
  const int K = p.n_vec;
  // layout of the blocks: ascending rows, columns in range, sizes J_k x J_col
  if (row_ptr[0] != 0 || row_ptr[M] != n_blocks || block_off[0] != 0) {
    set_error("row_ptr must start at 0 and end at n_blocks; block_off must start at 0");
    return DG_ERR_ARG;
  }
  for (int k = 0; k < M; ++k) {
    if (row_ptr[k + 1] < row_ptr[k]) {
      set_error("row_ptr must be non-decreasing");
      return DG_ERR_ARG;
    }
    for (long long b = row_ptr[k]; b < row_ptr[k + 1]; ++b) {
      if (col_idx[b] < 0 || col_idx[b] >= M) {
        set_error("col_idx out of range in row " + std::to_string(k));
        return DG_ERR_ARG;
      }
      if (block_off[b + 1] - block_off[b] != (long long)Js[k] * Js[col_idx[b]]) {
        set_error("block " + std::to_string(b) + " is not J_k x J_col");
        return DG_ERR_ARG;
      }
    }
  }
  for (int k = 0; k < M; ++k)
    if (Js[k] > 88) {
      set_error("J_k above 88");
      return DG_ERR_SHAPE;
    }
  if (p.n_want < 1 || K < p.n_want || K > 88 || 2 * K > Nb) {
    set_error("need 1 <= n_want <= n_vec <= min(88, N_b / 2); N_b = " + std::to_string(Nb));
    return DG_ERR_SHAPE;
  }
  if (!(p.tol > 0.0) || p.max_iter < 1 || p.degree < 1 || p.degree > 64 || p.lanczos_steps < 0 ||
      p.lanczos_steps > kLanczosMax) {
    set_error("tol > 0, max_iter >= 1, degree in [1, 64], lanczos_steps in [0, 64] (0: 10)");
    return DG_ERR_ARG;
  }
  const ChefsiLayout L = chefsi_layout(M, Nb, K, n_blocks);
  if (work_bytes < L.total) {
    set_error("work_bytes below " + std::to_string(L.total));
    return DG_ERR_OOM;
  }
  char* A = (char*)work;
  // the one-"element" context
  Ctx c;
  c.stream = stream;
  c.n_elem = 1;
  c.J = {p.n_want};
  c.G = {K - p.n_want};
  c.K = {K};
  c.N = {Nb};
  c.ld = {L.ld};
  for (int a = 0; a < 3; ++a) {
    c.elo[a] = {0};
    c.en[a] = {a == 0 ? Nb : 1};
  }
  c.kmax = K;
  c.autotune = false;
  c.gram_part = (double*)(A + L.off_part);
  c.gram_part_stride = (long long)L.part_stride;
  c.gram_part_ld = L.part_ld;
  c.gram_max_split = L.nsplit;
  int* ints = (int*)(A + L.off_ints);
  c.dev_active = ints;
  c.dev_status = ints + 1;
  c.dev_count = ints + 4;
  c.dev_iters = ints + 8;
  c.iota_dev = ints + 9;
  double* dbl = (double*)(A + L.off_dbl);
  c.dev_maxres = dbl;
  c.dev_minpiv = dbl + 1;
  c.dev_bounds = dbl + 4;
  c.dev_de = dbl + 7;
  c.dev_phase = (long long*)(A + L.off_phase);
  c.dev_off_kall = (long long*)(A + L.off_offkall);
  ElemDev E{};
  E.nx = Nb;
  E.ny = 1;
  E.nz = 1;
  E.N = Nb;
  E.ld = L.ld;
  E.K = K;
  E.J = p.n_want;
  E.en[0] = Nb;
  E.en[1] = 1;
  E.en[2] = 1;
  for (int b = 0; b < kMaxBlocks; ++b) E.blk[b] = A + L.off_blk[b];
  E.v64 = (const double*)(A + L.off_v64);
  E.v32 = (const float*)(A + L.off_v32);
  E.small = (double*)(A + L.off_small);
  E.kmax3 = 3 * K;
  E.bup = 0.0;
  c.elems_host = {E};
  c.elems_dev = (ElemDev*)(A + L.off_elem);
  c.dg_op.M = M;
  c.dg_op.H = hdg;
  c.dg_op.row_ptr = (const long long*)(A + L.off_rowptr);
  c.dg_op.col_idx = (const int*)(A + L.off_col);
  c.dg_op.boff = (const long long*)(A + L.off_boff);
  c.dg_op.roff = (const long long*)(A + L.off_roff);
  c.dg_op.J = (const int*)(A + L.off_J);
  c.dg_op.active = true;
  std::vector<long long> rp(row_ptr, row_ptr + M + 1), bo(block_off, block_off + std::max(1, n_blocks));
  std::vector<int> ci(col_idx, col_idx + std::max(0, n_blocks));
  if (ci.empty()) ci.push_back(0);
  const long long kall[2] = {0, K};
  const int iota0 = 0;
  auto put = [&](size_t off, const void* src, size_t bytes) -> int {
    DG_HIP(hipMemcpyAsync(A + off, src, bytes, hipMemcpyHostToDevice, stream));
    return DG_OK;
  };
  int st;
  if ((st = put(L.off_elem, &E, sizeof(ElemDev)))) return st;
  if ((st = put(L.off_rowptr, rp.data(), sizeof(long long) * rp.size()))) return st;
  if ((st = put(L.off_col, ci.data(), sizeof(int) * ci.size()))) return st;
  if ((st = put(L.off_boff, bo.data(), sizeof(long long) * bo.size()))) return st;
  if ((st = put(L.off_roff, roff.data(), sizeof(long long) * roff.size()))) return st;
  if ((st = put(L.off_J, Js.data(), sizeof(int) * M))) return st;
  if ((st = put(L.off_offkall, kall, sizeof(kall)))) return st;
  for (int b = 0; b < kMaxBlocks; ++b)
    DG_HIP(hipMemsetAsync(A + L.off_blk[b], 0, sizeof(double) * (size_t)L.ld * L.Kpad, stream));
  // flags, counters, status, iteration counts, the Lanczos state and the zero potential
  DG_HIP(hipMemsetAsync(A + L.off_ints, 0, sizeof(int) * 16, stream));
  DG_HIP(hipMemsetAsync(A + L.off_dbl, 0, sizeof(double) * 16, stream));
  DG_HIP(hipMemsetAsync(A + L.off_lz, 0, sizeof(double) * 136, stream));
  DG_HIP(hipMemsetAsync(A + L.off_v64, 0, sizeof(double) * (size_t)L.ld, stream));
  DG_HIP(hipMemsetAsync(A + L.off_v32, 0, sizeof(float) * (size_t)L.ld, stream));
  if ((st = put(L.off_ints + 9 * sizeof(int), &iota0, sizeof(int)))) return st;
  // start block
  if ((st = launch_copy_ext(c, DG_FP64, B_X, x, 0, 0, 0, Nb))) return st;
  // b_up by Lanczos from a seeded start (T0 column 0)
  const int steps = p.lanczos_steps > 0 ? p.lanczos_steps : 10;
  double* lz = (double*)(A + L.off_lz);
  if ((st = launch_random_block(c, DG_FP64, B_T0, (unsigned long long)p.seed))) return st;
  hipLaunchKernelGGL(k_lz_step, dim3(1), dim3(1024), 0, stream, c.elems_dev, (int)B_T0, (int)B_T1, -1, lz);
  for (int j = 0; j < steps; ++j) {
    if ((st = launch_dg_bsr(c, B_T0, B_T1, 1, nullptr))) return st;
    hipLaunchKernelGGL(k_lz_step, dim3(1), dim3(1024), 0, stream, c.elems_dev, (int)B_T0, (int)B_T1, j, lz);
  }
  hipLaunchKernelGGL(k_lz_bound, dim3(1), dim3(64), 0, stream, c.elems_dev, lz);
  DG_HIP(hipGetLastError());
  // Algorithm 2 iterations
  int it = 0, done = 0;
  st = run_chfsi(c, DG_FP64, p.tol, p.max_iter, p.degree, &it, &done);
  if (st < 0) return st;
  if ((st = launch_extract_kall(c, eig, resid))) return st;
  if ((st = launch_copy_ext(c, DG_FP64, B_X, x, 0, 0, 1, Nb))) return st;
  DG_HIP(hipStreamSynchronize(stream));
  if (iters_out) *iters_out = it;
  return done == 1 ? DG_OK : DG_WARN_NOT_CONVERGED;
}

}  // namespace dg
