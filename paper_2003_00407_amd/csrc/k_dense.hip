// Subspace linear algebra for the batched eigensolvers on gfx950.
//
//  * Gram matrices S^T S and S^T (H S) (the projected matrices of Eq. (4),
//    Algorithm 1 step 5; and Y^T Y, Y^T H Y of Algorithm 2 steps 3-4):
//    tall-skinny TN products, split over the grid dimension N, FP64 partial
//    tiles, then a fixed-order reduction (deterministic).
//  * Rayleigh-Ritz on the small projected problem, FP64, one workgroup per
//    element: diagonal scaling, Cholesky S^T S = U^T U, U^{-1}, the standard
//    problem U^{-T} A U^{-1}, cyclic Jacobi with a parallel (round-robin)
//    ordering, then the coefficients C = D U^{-1} V of the lowest eigenpairs.
//  * Rotations X <- S C (Eq. (2), Algorithm 1 steps 6-7; Algorithm 2 step 5).
//  * Residual norms ||H x_i - theta_i x_i|| and the preconditioner energy.
#include "dg_internal.h"

#include <algorithm>

namespace dg {

// column-count codes: > 0 explicit, 0 -> E.K, -1 -> E.J
__device__ __forceinline__ int kcode(int k, const ElemDev& E) { return k > 0 ? k : (k == 0 ? E.K : E.J); }
// small-matrix offsets: >= 0 explicit, -1-w -> SmallLayout slot w for this element
__device__ __forceinline__ long long soff(long long o, const ElemDev& E) {
  if (o >= 0) return o;
  const int KP = E.kmax3 + 2;
  switch (-1 - (int)o) {
    case 0: return SmallLayout::G(KP);
    case 1: return SmallLayout::A(KP);
    case 2: return SmallLayout::U(KP);
    case 3: return SmallLayout::V(KP);
    default: return SmallLayout::C(KP);
  }
}
// rows of the blocks a kernel works on: 0 -> N (Q_k grid), 1 -> |E_k|
__device__ __forceinline__ int nrows_of(const ElemDev& E, int rows_e) {
  return rows_e ? E.en[0] * E.en[1] * E.en[2] : E.N;
}

// ---------------------------------------------------------------------------
// virtual column access: column c of the concatenation of nb blocks of K cols
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ const T* vcol(const ElemDev& E, const ColSet& s, int c, int K) {
  const int b = c / K;
  return reinterpret_cast<const T*>(E.blk[s.blk[b]]) + (size_t)(c - b * K) * E.ld;
}

// ---------------------------------------------------------------------------
// Gram: part[e][split][i][j] = sum_{r in split} S[r,i] T[r,j]
// ---------------------------------------------------------------------------
struct GramArgs {
  const ElemDev* elems;
  const int* active;
  ColSet S, T;
  int kS, kT;          // columns per block (per element: <=0 -> E.K) -- multiplied by nb
  int nsplit;
  int tiles_j;         // output tile columns of the launch grid
  int rows_e;          // 1: reduce over the first |E_k| rows only
  double* part;        // per element region of part_stride doubles
  long long part_stride;
  int part_ld;         // leading dim of a partial tile matrix
};

constexpr int GT = 32;  // Gram tile

template <typename T>
__global__ void __launch_bounds__(256) k_gram(GramArgs A) {
  const int e = blockIdx.z;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int kS = kcode(A.kS, E);
  const int kT = kcode(A.kT, E);
  const int ni = A.S.nb * kS, nj = A.T.nb * kT;
  const int ti = blockIdx.x / A.tiles_j, tj = blockIdx.x % A.tiles_j;
  if (ti * GT >= ni || tj * GT >= nj) return;
  const int split = blockIdx.y;
  const int nrows = nrows_of(E, A.rows_e);
  const int rows_per = ((nrows + A.nsplit - 1) / A.nsplit + GT - 1) / GT * GT;
  const int r0 = split * rows_per;
  const int r1 = min(nrows, r0 + rows_per);
  __shared__ double sa[GT][GT + 1];
  __shared__ double sb[GT][GT + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc00 = 0, acc01 = 0, acc10 = 0, acc11 = 0;
  const T* colA[4];
  const T* colB[4];
  int lrow[4], lcol[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = threadIdx.x + 256 * q;
    lcol[q] = idx / GT;
    lrow[q] = idx % GT;
    const int ci = ti * GT + lcol[q], cj = tj * GT + lcol[q];
    colA[q] = ci < ni ? vcol<T>(E, A.S, ci, kS) : nullptr;
    colB[q] = cj < nj ? vcol<T>(E, A.T, cj, kT) : nullptr;
  }
  for (int r = r0; r < r1; r += GT) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = r + lrow[q];
      sa[lcol[q]][lrow[q]] = (colA[q] && rr < r1) ? double(colA[q][rr]) : 0.0;
      sb[lcol[q]][lrow[q]] = (colB[q] && rr < r1) ? double(colB[q][rr]) : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < GT; ++k) {
      const double a0 = sa[2 * ty][k], a1 = sa[2 * ty + 1][k];
      const double b0 = sb[2 * tx][k], b1 = sb[2 * tx + 1][k];
      acc00 += a0 * b0;
      acc01 += a0 * b1;
      acc10 += a1 * b0;
      acc11 += a1 * b1;
    }
    __syncthreads();
  }
  double* out = A.part + (size_t)e * A.part_stride + (size_t)split * A.part_ld * A.part_ld;
  const int i0 = ti * GT + 2 * ty, j0 = tj * GT + 2 * tx;
  if (i0 < ni && j0 < nj) out[(size_t)i0 * A.part_ld + j0] = acc00;
  if (i0 < ni && j0 + 1 < nj) out[(size_t)i0 * A.part_ld + j0 + 1] = acc01;
  if (i0 + 1 < ni && j0 < nj) out[(size_t)(i0 + 1) * A.part_ld + j0] = acc10;
  if (i0 + 1 < ni && j0 + 1 < nj) out[(size_t)(i0 + 1) * A.part_ld + j0 + 1] = acc11;
}

struct GramReduceArgs {
  const ElemDev* elems;
  const int* active;
  int nbS, nbT, kS, kT;
  int nsplit;
  const double* part;
  long long part_stride;
  int part_ld;
  long long out_off;   // doubles, inside E.small
  int out_ld;          // <= 0: ni
};

__global__ void __launch_bounds__(256) k_gram_reduce(GramReduceArgs A) {
  const int e = blockIdx.y;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int kS = kcode(A.kS, E);
  const int kT = kcode(A.kT, E);
  const int ni = A.nbS * kS, nj = A.nbT * kT;
  const int ld = A.out_ld > 0 ? A.out_ld : nj;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= ni * nj) return;
  const int i = idx / nj, j = idx % nj;
  const double* p = A.part + (size_t)e * A.part_stride + (size_t)i * A.part_ld + j;
  double s = 0.0;
  for (int q = 0; q < A.nsplit; ++q) s += p[(size_t)q * A.part_ld * A.part_ld];
  E.small[soff(A.out_off, E) + (size_t)i * ld + j] = s;
}

// ---------------------------------------------------------------------------
// block reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// sum over the block, result broadcast to every thread (fixed order)
__device__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  __syncthreads();
  return s;
}

__device__ double block_max(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = sh[0];
  for (int i = 1; i < nw; ++i) s = fmax(s, sh[i]);
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz / symmetric eigen, one workgroup per element (FP64)
// ---------------------------------------------------------------------------
struct RRArgs {
  const ElemDev* elems;
  const int* active;
  int nb;              // K3 = nb * E.K (RR_GEN); RR_SVD: K3 = kfix
  int kfix;            // RR_SVD: matrix order
  int nkeep;           // columns of C to produce (<= 0: E.K)
  int mode;
  int max_sweeps;
  int* status;         // per element: 0 ok, 1 breakdown
};

constexpr int kRRThreads = 512;

__device__ __forceinline__ void jacobi_cs(double app, double aqq, double apq, double& c, double& s,
                                          double& t) {
  if (apq == 0.0) {
    c = 1.0;
    s = 0.0;
    t = 0.0;
    return;
  }
  const double th = (aqq - app) / (2.0 * apq);
  t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

__global__ void __launch_bounds__(kRRThreads) k_rr(RRArgs A) {
  const int e = blockIdx.x;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int K = E.K;
  const int n = (A.mode == RR_GEN) ? A.nb * K : kcode(A.kfix, E);
  const int np = n + (n & 1);             // padded even order for the pairing
  const int nkeep = kcode(A.nkeep, E);
  const int KP = E.kmax3 + 2;             // storage order of the work matrices
  double* G = E.small + SmallLayout::G(KP);     // Gram / U / Z (KP x KP)
  double* Am = E.small + SmallLayout::A(KP);    // A, then the standard problem
  double* Um = E.small + SmallLayout::U(KP);
  double* Vm = E.small + SmallLayout::V(KP);
  double* Cm = E.small + SmallLayout::C(KP);
  double* vec = E.small + SmallLayout::vec(KP);
  double* d = vec + VS_D * KP;
  double* lam = vec + VS_T0 * KP;
  double* csv = vec + VS_T1 * KP;   // c of each pair
  double* ssv = vec + VS_T2 * KP;   // s of each pair
  double* tsv = vec + VS_T2 * KP + KP / 2 + 1;
  __shared__ double sh[16];
  __shared__ int brk;
  const int tid = threadIdx.x, nt = blockDim.x;
  // Inputs: G and A (n x n, ld n) as written by the Gram reduction.  For the
  // generalised problem the leading blocks of S are tried in turn when the
  // overlap Cholesky breaks down: [X W P], then [X W], then [X]; the
  // coefficients of dropped blocks are zero (restart without P).
  int n_cur = n;
  if (A.mode == RR_GEN) {
    int attempt = 0;
    for (;;) {
      const int m = n_cur;
      if (tid == 0) brk = 0;
      __syncthreads();
      for (int idx = tid; idx < np * np; idx += nt) {
        const int i = idx / np, j = idx % np;
        const bool in = (i < m && j < m);
        Um[idx] = in ? G[(size_t)i * n + j] : (i == j ? 1.0 : 0.0);
        Vm[idx] = in ? 0.5 * (Am[(size_t)i * n + j] + Am[(size_t)j * n + i]) : 0.0;
      }
      __syncthreads();
      for (int i = tid; i < np; i += nt) {
        const double gii = Um[(size_t)i * np + i];
        if (!(gii > 0.0)) brk = 1;
        d[i] = (i < m && gii > 0.0) ? 1.0 / sqrt(gii) : (i < m ? 0.0 : 1.0);
      }
      __syncthreads();
      for (int idx = tid; idx < np * np; idx += nt) {
        const int i = idx / np, j = idx % np;
        Um[idx] *= d[i] * d[j];
        Vm[idx] *= d[i] * d[j];
      }
      __syncthreads();
      // Cholesky (upper, in place in Um): Um = U^T U
      for (int j = 0; j < m; ++j) {
        const double piv = Um[(size_t)j * np + j];
        if (!(piv > 1e-13) && tid == 0) brk = 1;
        const double ujj = sqrt(fmax(piv, 1e-300));
        __syncthreads();
        for (int k = j + 1 + tid; k < m; k += nt) Um[(size_t)j * np + k] /= ujj;
        __syncthreads();
        if (tid == 0) Um[(size_t)j * np + j] = ujj;
        const int mm = m - j - 1;
        for (int idx = tid; idx < mm * mm; idx += nt) {
          const int i = j + 1 + idx / mm, k = j + 1 + idx % mm;
          if (k >= i) Um[(size_t)i * np + k] -= Um[(size_t)j * np + i] * Um[(size_t)j * np + k];
        }
        __syncthreads();
      }
      if (!brk) break;
      ++attempt;
      if (n_cur > K) {
        n_cur -= K;
      } else {
        if (tid == 0) A.status[e] = 2;
        return;   // unrecoverable: C is left as is and the status reports it
      }
      __syncthreads();
    }
    if (tid == 0) A.status[e] = attempt;
    for (int idx = tid; idx < np * np; idx += nt) {
      const int i = idx / np, j = idx % np;
      if (j < i) Um[idx] = 0.0;
    }
    __syncthreads();
    // Z = U^{-1} (upper), column j by back substitution, into G (inputs are no longer needed)
    for (int j = tid; j < np; j += nt) {
      for (int i = np - 1; i >= 0; --i) {
        double s = (i == j) ? 1.0 : 0.0;
        for (int k = i + 1; k <= j; ++k) s -= Um[(size_t)i * np + k] * G[(size_t)k * np + j];
        G[(size_t)i * np + j] = (i <= j) ? s / Um[(size_t)i * np + i] : 0.0;
      }
    }
    __syncthreads();
    // Am = A' Z ; Um = Z^T Am ; Am = sym(Um)  (standard problem)
    for (int idx = tid; idx < np * np; idx += nt) {
      const int i = idx / np, j = idx % np;
      double s = 0.0;
      for (int k = 0; k <= j; ++k) s += Vm[(size_t)i * np + k] * G[(size_t)k * np + j];
      Am[idx] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < np * np; idx += nt) {
      const int i = idx / np, j = idx % np;
      double s = 0.0;
      for (int k = 0; k <= i; ++k) s += G[(size_t)k * np + i] * Am[(size_t)k * np + j];
      Um[idx] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < np * np; idx += nt) {
      const int i = idx / np, j = idx % np;
      Am[idx] = (i < n_cur && j < n_cur) ? 0.5 * (Um[idx] + Um[(size_t)j * np + i]) : 0.0;
    }
  } else {
    // RR_SVD: eigen-decomposition of the Gram matrix itself
    for (int idx = tid; idx < np * np; idx += nt) {
      const int i = idx / np, j = idx % np;
      Um[idx] = (i < n && j < n) ? G[(size_t)i * n + j] : 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < np * np; idx += nt) Am[idx] = Um[idx];
  }
  __syncthreads();
  // ---- cyclic Jacobi, round-robin pairs, V accumulated in Vm
  for (int idx = tid; idx < np * np; idx += nt) {
    const int i = idx / np, j = idx % np;
    Vm[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int half = np / 2;
  for (int sweep = 0; sweep < A.max_sweeps; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int idx = tid; idx < np * np; idx += nt) {
      const int i = idx / np, j = idx % np;
      const double a = Am[idx];
      if (i != j) off += a * a;
      else dia += a * a;
    }
    off = block_sum(off, sh);
    dia = block_sum(dia, sh);
    if (off <= 1e-30 * dia || off == 0.0) break;
    for (int r = 0; r < np - 1; ++r) {
      for (int pi = tid; pi < half; pi += nt) {
        const int a = pi, b = np - 1 - pi;
        const int ia = a == 0 ? 0 : ((a - 1 + r) % (np - 1)) + 1;
        const int ib = b == 0 ? 0 : ((b - 1 + r) % (np - 1)) + 1;
        const int p = min(ia, ib), q = max(ia, ib);
        double c, s, t;
        jacobi_cs(Am[(size_t)p * np + p], Am[(size_t)q * np + q], Am[(size_t)p * np + q], c, s, t);
        csv[pi] = c;
        ssv[pi] = s;
        tsv[pi] = t;
      }
      __syncthreads();
      // 2x2 block updates A' = J^T A J over all (pair i, pair j) blocks; then V J
      for (int idx = tid; idx < half * half + half * np; idx += nt) {
        if (idx < half * half) {
          const int bi = idx / half, bj = idx % half;
          auto pq = [&](int pi, int& p, int& q) {
            const int a = pi, b = np - 1 - pi;
            const int ia = a == 0 ? 0 : ((a - 1 + r) % (np - 1)) + 1;
            const int ib = b == 0 ? 0 : ((b - 1 + r) % (np - 1)) + 1;
            p = min(ia, ib);
            q = max(ia, ib);
          };
          int pI, qI, pJ, qJ;
          pq(bi, pI, qI);
          pq(bj, pJ, qJ);
          const double ci = csv[bi], si = ssv[bi], cj = csv[bj], sj = ssv[bj];
          double* a00 = &Am[(size_t)pI * np + pJ];
          double* a01 = &Am[(size_t)pI * np + qJ];
          double* a10 = &Am[(size_t)qI * np + pJ];
          double* a11 = &Am[(size_t)qI * np + qJ];
          if (bi == bj) {
            const double t = tsv[bi];
            const double apq = *a01;
            *a00 = *a00 - t * apq;
            *a11 = *a11 + t * apq;
            *a01 = 0.0;
            *a10 = 0.0;
          } else {
            const double m00 = *a00, m01 = *a01, m10 = *a10, m11 = *a11;
            const double b00 = ci * m00 - si * m10, b01 = ci * m01 - si * m11;
            const double b10 = si * m00 + ci * m10, b11 = si * m01 + ci * m11;
            *a00 = cj * b00 - sj * b01;
            *a01 = sj * b00 + cj * b01;
            *a10 = cj * b10 - sj * b11;
            *a11 = sj * b10 + cj * b11;
          }
        } else {
          const int k = idx - half * half;
          const int row = k / half, pj = k % half;
          const int a = pj, b = np - 1 - pj;
          const int ia = a == 0 ? 0 : ((a - 1 + r) % (np - 1)) + 1;
          const int ib = b == 0 ? 0 : ((b - 1 + r) % (np - 1)) + 1;
          const int p = min(ia, ib), q = max(ia, ib);
          const double c = csv[pj], s = ssv[pj];
          const double vp = Vm[(size_t)row * np + p], vq = Vm[(size_t)row * np + q];
          Vm[(size_t)row * np + p] = c * vp - s * vq;
          Vm[(size_t)row * np + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }
  // eigenvalues on the diagonal; rank them (ascending for RR_GEN, descending for RR_SVD)
  for (int i = tid; i < np; i += nt) lam[i] = (i < n_cur) ? Am[(size_t)i * np + i] : 0.0;
  __syncthreads();
  int* rank_of = reinterpret_cast<int*>(csv);   // reuse: position -> original index
  for (int i = tid; i < n_cur; i += nt) {
    int rk = 0;
    for (int j = 0; j < n_cur; ++j) {
      const bool before = (A.mode == RR_GEN) ? (lam[j] < lam[i] || (lam[j] == lam[i] && j < i))
                                             : (lam[j] > lam[i] || (lam[j] == lam[i] && j < i));
      rk += before;
    }
    rank_of[rk] = i;
  }
  __syncthreads();
  double* theta = vec + VS_THETA * KP;
  if (A.mode == RR_GEN) {
    // C = D Z V[:, sel]  (n x nkeep, ld nkeep)
    for (int idx = tid; idx < n * nkeep; idx += nt) {
      const int i = idx / nkeep, j = idx % nkeep;
      if (i >= n_cur) {
        Cm[(size_t)i * nkeep + j] = 0.0;
        continue;
      }
      const int col = rank_of[j];
      double s = 0.0;
      for (int k = i; k < n_cur; ++k) s += G[(size_t)i * np + k] * Vm[(size_t)k * np + col];
      Cm[(size_t)i * nkeep + j] = d[i] * s;
    }
    for (int j = tid; j < nkeep; j += nt) theta[j] = lam[rank_of[j]];
  } else {
    // C = V[:, sel] / sigma ; theta = sigma (descending)
    for (int idx = tid; idx < n * nkeep; idx += nt) {
      const int i = idx / nkeep, j = idx % nkeep;
      const int col = rank_of[j];
      const double sg = sqrt(fmax(lam[col], 0.0));
      Cm[(size_t)i * nkeep + j] = sg > 0.0 ? Vm[(size_t)i * np + col] / sg : 0.0;
    }
    for (int j = tid; j < nkeep; j += nt) theta[j] = sqrt(fmax(lam[rank_of[j]], 0.0));
  }
}

// ---------------------------------------------------------------------------
// rotation: out_o[:, j] = beta_o out_o[:, j] + alpha sum_{c in [c0_o, c1_o)} S[:, c] C[c, j]
// ---------------------------------------------------------------------------
constexpr int RT_ROWS = 64;
constexpr int RT_CC = 16;
constexpr int RT_MAXC = 96;   // max output columns
constexpr int RT_PER = RT_MAXC / 4;

template <typename T>
__global__ void __launch_bounds__(256) k_rotate(RotArgs A) {
  const int e = blockIdx.y;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int kS = kcode(A.kS, E);
  const int ncol = kcode(A.ncol, E);
  const int cld = A.c_ld > 0 ? A.c_ld : ncol;
  const int nrows = nrows_of(E, A.rows_e);
  const int r0 = blockIdx.x * RT_ROWS;
  if (r0 >= nrows) return;
  int c0[2], c1[2];
  for (int o = 0; o < 2; ++o) {
    c0[o] = A.c_blockrows > 0 ? A.c0[o] * kS : A.c0[o];
    c1[o] = A.c_blockrows > 0 ? A.c1[o] * kS : A.c1[o];
  }
  const int cmin = min(c0[0], A.nout > 1 ? c0[1] : c0[0]);
  const int cmax = max(c1[0], A.nout > 1 ? c1[1] : c1[0]);
  __shared__ double ss[RT_CC][RT_ROWS + 1];
  __shared__ double sc[RT_CC][RT_MAXC];
  const int row = threadIdx.x % RT_ROWS;
  const int cg = threadIdx.x / RT_ROWS;   // 0..3, uniform per wave
  double acc[2][RT_PER];
#pragma unroll
  for (int o = 0; o < 2; ++o)
#pragma unroll
    for (int q = 0; q < RT_PER; ++q) acc[o][q] = 0.0;
  const double* Cm = E.small + soff(A.c_off, E);
  for (int cb = cmin; cb < cmax; cb += RT_CC) {
    for (int idx = threadIdx.x; idx < RT_CC * RT_ROWS; idx += 256) {
      const int cc = idx / RT_ROWS, rr = idx % RT_ROWS;
      const int c = cb + cc, r = r0 + rr;
      ss[cc][rr] = (c < cmax && r < nrows) ? double(vcol<T>(E, A.S, c, kS)[r]) : 0.0;
    }
    for (int idx = threadIdx.x; idx < RT_CC * RT_MAXC; idx += 256) {
      const int cc = idx / RT_MAXC, j = idx % RT_MAXC;
      const int c = cb + cc;
      sc[cc][j] = (c < cmax && j < ncol) ? Cm[(size_t)c * cld + j] : 0.0;
    }
    __syncthreads();
    for (int cc = 0; cc < RT_CC; ++cc) {
      const int c = cb + cc;
      const double s = ss[cc][row];
      const bool in0 = (c >= c0[0] && c < c1[0]);
      const bool in1 = (A.nout > 1 && c >= c0[1] && c < c1[1]);
#pragma unroll
      for (int q = 0; q < RT_PER; ++q) {
        const double cv = s * sc[cc][cg + 4 * q];
        if (in0) acc[0][q] += cv;
        if (in1) acc[1][q] += cv;
      }
    }
    __syncthreads();
  }
  const int r = r0 + row;
  if (r >= nrows) return;
  for (int o = 0; o < A.nout; ++o) {
    T* out = reinterpret_cast<T*>(E.blk[A.out_blk[o]]);
#pragma unroll
    for (int q = 0; q < RT_PER; ++q) {
      const int j = cg + 4 * q;
      if (j < ncol) {
        T* p = out + (size_t)j * E.ld + r;
        const double prev = A.beta[o] != 0.0 ? A.beta[o] * double(*p) : 0.0;
        *p = T(prev + A.alpha * acc[o][q]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// residual norms and preconditioner energies
// res_i = ||hx_i - theta_i x_i||,  ekin_i = max(theta_i - x_i^T V x_i, 0.05)
// ---------------------------------------------------------------------------
struct ResArgs {
  const ElemDev* elems;
  const int* active;
  int x_blk, hx_blk;
  int ncol;
  int kp;              // small storage order (kmax3 + 2)
};

template <typename T>
__global__ void __launch_bounds__(256) k_residual(ResArgs A) {
  const int e = blockIdx.y;
  const ElemDev& E = A.elems[e];
  const int i = blockIdx.x;
  const int ncol = kcode(A.ncol, E);
  if (i >= ncol) return;
  if (A.active && !A.active[e]) return;
  const int KP = E.kmax3 + 2;
  double* vec = E.small + SmallLayout::vec(KP);
  const double th = vec[VS_THETA * KP + i];
  const T* x = reinterpret_cast<const T*>(E.blk[A.x_blk]) + (size_t)i * E.ld;
  const T* hx = reinterpret_cast<const T*>(E.blk[A.hx_blk]) + (size_t)i * E.ld;
  double s1 = 0.0, s2 = 0.0;
  for (int r = threadIdx.x; r < E.N; r += blockDim.x) {
    const double xv = double(x[r]);
    const double rv = double(hx[r]) - th * xv;
    s1 += rv * rv;
    s2 += E.v64[r] * xv * xv;
  }
  __shared__ double sh[16];
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    vec[VS_RES * KP + i] = sqrt(s1);
    vec[VS_EKIN * KP + i] = fmax(th - s2, 0.05);
  }
}

// per element: active = max_{i<J} res_i > tol ; count of active elements
__global__ void k_check(const ElemDev* elems, int n_elem, int* active, double tol, int* count,
                        double* maxres) {
  __shared__ double sh[16];
  for (int e = 0; e < n_elem; ++e) {
    const ElemDev& E = elems[e];
    const int KP = E.kmax3 + 2;
    const double* res = E.small + SmallLayout::vec(KP) + VS_RES * KP;
    double m = 0.0;
    for (int i = threadIdx.x; i < E.J; i += blockDim.x) m = fmax(m, res[i]);
    m = block_max(m, sh);
    if (threadIdx.x == 0) {
      if (active[e] && !(m <= tol)) {
      } else {
        active[e] = 0;
      }
      if (!(m == m)) active[e] = -1;   // NaN
      maxres[e] = m;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int c = 0, nan = 0;
    for (int e = 0; e < n_elem; ++e) {
      c += active[e] > 0;
      nan += active[e] < 0;
    }
    count[0] = c;
    count[1] = nan;
  }
}

// ---------------------------------------------------------------------------
// copies between caller buffers (packed) and blocks
// mode 0: packed <-> block (all N rows)      mode 1: block E_k rows -> packed
// mode 2: block E_k rows -> block rows 0..|E_k|-1
// ---------------------------------------------------------------------------
struct CopyArgs {
  const ElemDev* elems;
  int blk, blk2;
  void* ptr;                  // packed caller buffer (FP64 or FP32 as prec)
  const long long* off;       // per element offsets into ptr (elements), or nullptr
  long long off_mult;         // multiplier applied to off[e]
  int elem_only;              // >= 0: this element only, ptr offset 0
  int ncol;                   // column code
  int to_packed;              // 1: block -> ptr
  int mode;
};

template <typename T>
__global__ void __launch_bounds__(256) k_copy(CopyArgs A) {
  const int e = A.elem_only >= 0 ? A.elem_only : blockIdx.z;
  const ElemDev& E = A.elems[e];
  const int ncol = kcode(A.ncol, E);
  const int j = blockIdx.y;
  if (j >= ncol) return;
  const int ne = E.en[0] * E.en[1] * E.en[2];
  const int nrows = A.mode == 0 ? E.N : ne;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nrows) return;
  int gr = r;
  if (A.mode != 0) {
    const int x = r % E.en[0], y = (r / E.en[0]) % E.en[1], z = r / (E.en[0] * E.en[1]);
    gr = (x + E.elo[0]) + E.nx * ((y + E.elo[1]) + E.ny * (z + E.elo[2]));
  }
  T* b = reinterpret_cast<T*>(E.blk[A.blk]) + (size_t)j * E.ld;
  if (A.mode == 2) {
    T* d = reinterpret_cast<T*>(E.blk[A.blk2]) + (size_t)j * E.ld;
    d[r] = b[gr];
    return;
  }
  const long long base = (A.elem_only >= 0 || !A.off) ? 0 : A.off[e] * A.off_mult;
  T* p = reinterpret_cast<T*>(A.ptr) + base + (size_t)j * nrows + r;
  if (A.to_packed) *p = b[gr];
  else b[gr] = *p;
}

// packed FP64 source (x0) into a block of either precision
template <typename T>
__global__ void __launch_bounds__(256) k_copy_in64(const ElemDev* elems, int blk, const double* src,
                                                    const long long* off, int ncol_code) {
  const int e = blockIdx.z;
  const ElemDev& E = elems[e];
  const int ncol = kcode(ncol_code, E);
  const int j = blockIdx.y;
  if (j >= ncol) return;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= E.N) return;
  reinterpret_cast<T*>(E.blk[blk])[(size_t)j * E.ld + r] = T(src[off[e] + (size_t)j * E.N + r]);
}

// convert a block between precisions (separate blocks)
__global__ void __launch_bounds__(256) k_convert(const ElemDev* elems, int src_blk, int src_prec,
                                                  int dst_blk, int dst_prec, int ncol_code) {
  const int e = blockIdx.z;
  const ElemDev& E = elems[e];
  const int ncol = kcode(ncol_code, E);
  const int j = blockIdx.y;
  if (j >= ncol) return;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= E.N) return;
  const size_t o = (size_t)j * E.ld + r;
  double v = src_prec == DG_FP64 ? reinterpret_cast<const double*>(E.blk[src_blk])[o]
                                 : double(reinterpret_cast<const float*>(E.blk[src_blk])[o]);
  if (dst_prec == DG_FP64) reinterpret_cast<double*>(E.blk[dst_blk])[o] = v;
  else reinterpret_cast<float*>(E.blk[dst_blk])[o] = float(v);
}

// J values per element from the small-vector slots into packed outputs
__global__ void k_extract(const ElemDev* elems, const long long* off, int slot0, double* out0,
                          int slot1, double* out1) {
  const int e = blockIdx.x;
  const ElemDev& E = elems[e];
  const int KP = E.kmax3 + 2;
  const double* vec = E.small + SmallLayout::vec(KP);
  for (int i = threadIdx.x; i < E.J; i += blockDim.x) {
    if (out0) out0[off[e] + i] = vec[slot0 * KP + i];
    if (out1) out1[off[e] + i] = vec[slot1 * KP + i];
  }
}

// first |E_k| rows of a block -> packed |E_k| x J output
__global__ void __launch_bounds__(256) k_copy_rows(const ElemDev* elems, int blk, double* out,
                                                    const long long* off) {
  const int e = blockIdx.z;
  const ElemDev& E = elems[e];
  const int j = blockIdx.y;
  if (j >= E.J) return;
  const int ne = E.en[0] * E.en[1] * E.en[2];
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= ne) return;
  out[off[e] + (size_t)j * ne + r] = reinterpret_cast<const double*>(E.blk[blk])[(size_t)j * E.ld + r];
}

// Block roles move with each element: after a rotation the logical blocks of
// every active element are re-pointed (new[i] = old[perm[i]]); converged
// elements keep theirs.
struct Perm8 {
  int p[kMaxBlocks];
};

__global__ void k_permute_blocks(ElemDev* elems, int n_elem, const int* active, Perm8 perm) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  if (active && active[e] <= 0) return;
  void* old[kMaxBlocks];
  for (int i = 0; i < kMaxBlocks; ++i) old[i] = elems[e].blk[i];
  for (int i = 0; i < kMaxBlocks; ++i) elems[e].blk[i] = old[perm.p[i]];
}

int launch_permute(Ctx& c, const int* perm, const int* active) {
  Perm8 p;
  for (int i = 0; i < kMaxBlocks; ++i) p.p[i] = perm[i];
  hipLaunchKernelGGL(k_permute_blocks, dim3((c.n_elem + 63) / 64), dim3(64), 0, c.stream, c.elems_dev,
                     c.n_elem, active, p);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static void max_dims(Ctx& c, int code, int* maxk, int* maxN, int* maxE) {
  *maxk = *maxN = *maxE = 0;
  for (int e = 0; e < c.n_elem; ++e) {
    const int k = code > 0 ? code : (code == 0 ? c.K[e] : c.J[e]);
    *maxk = std::max(*maxk, k);
    *maxN = std::max(*maxN, c.N[e]);
    *maxE = std::max(*maxE, c.en[0][e] * c.en[1][e] * c.en[2][e]);
  }
}

static int gram_impl(Ctx& c, int prec, const ColSet& S, int kS, const ColSet& T, int kT,
                     long long out_off, const int* active, int rows_e) {
  int ks, kt, maxN, maxE;
  max_dims(c, kS, &ks, &maxN, &maxE);
  max_dims(c, kT, &kt, &maxN, &maxE);
  const int maxni = S.nb * ks, maxnj = T.nb * kt;
  const int rows = rows_e ? maxE : maxN;
  const int tiles = ((maxni + GT - 1) / GT) * ((maxnj + GT - 1) / GT);
  int nsplit = std::max(1, std::min(c.gram_max_split, (2048 + tiles * c.n_elem - 1) / (tiles * c.n_elem)));
  nsplit = std::min(nsplit, std::max(1, rows / 1024));
  GramArgs ga{c.elems_dev, active, S, T, kS, kT, nsplit, (maxnj + GT - 1) / GT, rows_e, c.gram_part,
              c.gram_part_stride, c.gram_part_ld};
  double flops = 0.0;
  for (int e = 0; e < c.n_elem; ++e) {
    if (active && !c.active_host.empty() && !c.active_host[e]) continue;
    const int ke = kS > 0 ? kS : (kS == 0 ? c.K[e] : c.J[e]);
    const int kt = kT > 0 ? kT : (kT == 0 ? c.K[e] : c.J[e]);
    const double r = rows_e ? (double)c.en[0][e] * c.en[1][e] * c.en[2][e] : (double)c.N[e];
    flops += 2.0 * r * (S.nb * ke) * (T.nb * kt);
  }
  TimedScope ts(c, TC_GRAM, flops);
  dim3 g1(tiles, nsplit, c.n_elem);
  if (prec == DG_FP64) hipLaunchKernelGGL(k_gram<double>, g1, dim3(256), 0, c.stream, ga);
  else hipLaunchKernelGGL(k_gram<float>, g1, dim3(256), 0, c.stream, ga);
  GramReduceArgs ra{c.elems_dev, active, S.nb, T.nb, kS, kT, nsplit, c.gram_part,
                    c.gram_part_stride, c.gram_part_ld, out_off, 0};
  dim3 g2((maxni * maxnj + 255) / 256, c.n_elem);
  hipLaunchKernelGGL(k_gram_reduce, g2, dim3(256), 0, c.stream, ra);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_gram(Ctx& c, int prec, const ColSet& S, int kS, const ColSet& T, int kT,
                long long out_off, const int* active) {
  return gram_impl(c, prec, S, kS, T, kT, out_off, active, 0);
}

int launch_gram_rows(Ctx& c, int prec, const ColSet& S, int kS, const ColSet& T, int kT,
                     long long out_off, int rows_e) {
  return gram_impl(c, prec, S, kS, T, kT, out_off, nullptr, rows_e);
}

int launch_rr(Ctx& c, int nb, int kfix, int nkeep, int mode, const int* active) {
  RRArgs a{c.elems_dev, active, nb, kfix, nkeep, mode, 40, c.dev_status};
  TimedScope ts(c, TC_RR);
  hipLaunchKernelGGL(k_rr, dim3(c.n_elem), dim3(kRRThreads), 0, c.stream, a);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_rotate(Ctx& c, int prec, const RotArgs& a_in) {
  RotArgs a = a_in;
  a.elems = c.elems_dev;
  int k, maxN, maxE;
  max_dims(c, a.ncol, &k, &maxN, &maxE);
  const int rows = a.rows_e ? maxE : maxN;
  dim3 g((rows + RT_ROWS - 1) / RT_ROWS, c.n_elem);
  double flops = 0.0;
  for (int e = 0; e < c.n_elem; ++e) {
    if (a.active && !c.active_host.empty() && !c.active_host[e]) continue;
    const int ks = a.kS > 0 ? a.kS : (a.kS == 0 ? c.K[e] : c.J[e]);
    const int nc = a.ncol > 0 ? a.ncol : (a.ncol == 0 ? c.K[e] : c.J[e]);
    const double r = a.rows_e ? (double)c.en[0][e] * c.en[1][e] * c.en[2][e] : (double)c.N[e];
    for (int o = 0; o < a.nout; ++o) {
      const int span = a.c_blockrows > 0 ? (a.c1[o] - a.c0[o]) * ks : (a.c1[o] - a.c0[o]);
      flops += 2.0 * r * span * nc;
    }
  }
  TimedScope ts(c, TC_ROT, flops);
  if (prec == DG_FP64) hipLaunchKernelGGL(k_rotate<double>, g, dim3(256), 0, c.stream, a);
  else hipLaunchKernelGGL(k_rotate<float>, g, dim3(256), 0, c.stream, a);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_residual(Ctx& c, int prec, int x_blk, int hx_blk, int ncol, const int* active) {
  int maxk, maxN, maxE;
  max_dims(c, ncol, &maxk, &maxN, &maxE);
  ResArgs a{c.elems_dev, active, x_blk, hx_blk, ncol, 0};
  dim3 g(maxk, c.n_elem);
  TimedScope ts(c, TC_OTHER);
  if (prec == DG_FP64) hipLaunchKernelGGL(k_residual<double>, g, dim3(256), 0, c.stream, a);
  else hipLaunchKernelGGL(k_residual<float>, g, dim3(256), 0, c.stream, a);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_check(Ctx& c, int* active, double tol) {
  hipLaunchKernelGGL(k_check, dim3(1), dim3(256), 0, c.stream, c.elems_dev, c.n_elem, active, tol,
                     c.dev_count, c.dev_maxres);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_copy_ext(Ctx& c, int prec, int blk, const void* ptr, int elem, int ncol, int to_packed) {
  int maxk, maxN, maxE;
  max_dims(c, ncol, &maxk, &maxN, &maxE);
  CopyArgs a{c.elems_dev, blk, 0, const_cast<void*>(ptr), c.dev_off_grid, ncol, elem, ncol, to_packed, 0};
  dim3 g((maxN + 255) / 256, maxk, elem >= 0 ? 1 : c.n_elem);
  if (prec == DG_FP64) hipLaunchKernelGGL(k_copy<double>, g, dim3(256), 0, c.stream, a);
  else hipLaunchKernelGGL(k_copy<float>, g, dim3(256), 0, c.stream, a);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_copy_packed(Ctx& c, int prec, int blk, const double* ptr, const long long* off, int ncol,
                       int to_packed) {
  int maxk, maxN, maxE;
  max_dims(c, ncol, &maxk, &maxN, &maxE);
  dim3 g((maxN + 255) / 256, maxk, c.n_elem);
  if (!to_packed) {
    if (prec == DG_FP64) hipLaunchKernelGGL(k_copy_in64<double>, g, dim3(256), 0, c.stream, c.elems_dev, blk, ptr, off, ncol);
    else hipLaunchKernelGGL(k_copy_in64<float>, g, dim3(256), 0, c.stream, c.elems_dev, blk, ptr, off, ncol);
  } else {
    CopyArgs a{c.elems_dev, blk, 0, const_cast<double*>(ptr), off, 1, -1, ncol, 1, 0};
    hipLaunchKernelGGL(k_copy<double>, g, dim3(256), 0, c.stream, a);
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_gather_e(Ctx& c, int src_blk, int dst_blk) {
  int maxk, maxN, maxE;
  max_dims(c, -1, &maxk, &maxN, &maxE);
  CopyArgs a{c.elems_dev, src_blk, dst_blk, nullptr, nullptr, 0, -1, -1, 0, 2};
  dim3 g((maxE + 255) / 256, maxk, c.n_elem);
  hipLaunchKernelGGL(k_copy<double>, g, dim3(256), 0, c.stream, a);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_copy_rows_out(Ctx& c, int blk, double* out) {
  // blk holds |E_k| x J in its first rows: mode 0 semantics over |E_k| rows
  int maxk, maxN, maxE;
  max_dims(c, -1, &maxk, &maxN, &maxE);
  dim3 g((maxE + 255) / 256, maxk, c.n_elem);
  hipLaunchKernelGGL(k_copy_rows, g, dim3(256), 0, c.stream, c.elems_dev, blk, out, c.dev_off_alb);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_convert(Ctx& c, int src_blk, int src_prec, int dst_blk, int dst_prec, int ncol) {
  int maxk, maxN, maxE;
  max_dims(c, ncol, &maxk, &maxN, &maxE);
  dim3 g((maxN + 255) / 256, maxk, c.n_elem);
  hipLaunchKernelGGL(k_convert, g, dim3(256), 0, c.stream, c.elems_dev, src_blk, src_prec, dst_blk,
                     dst_prec, ncol);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_extract_eig(Ctx& c, double* eig, double* resid) {
  hipLaunchKernelGGL(k_extract, dim3(c.n_elem), dim3(128), 0, c.stream, c.elems_dev, c.dev_off_eig,
                     (int)VS_THETA, eig, (int)VS_RES, resid);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_extract_theta(Ctx& c, double* out) {
  hipLaunchKernelGGL(k_extract, dim3(c.n_elem), dim3(128), 0, c.stream, c.elems_dev, c.dev_off_eig,
                     (int)VS_THETA, out, (int)VS_THETA, (double*)nullptr);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace dg
