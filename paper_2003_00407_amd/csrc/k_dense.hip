// Subspace linear algebra for the batched eigensolvers on gfx950.
//
//  * Gram matrices S^T S and S^T (H S) (the projected matrices of Eq. (4),
//    Algorithm 1 step 5; and Y^T Y, Y^T H Y of Algorithm 2 steps 3-4):
//    tall-skinny TN products, split over the grid dimension N, FP64 partial
//    tiles, then a fixed-order reduction (deterministic).
//  * Rayleigh-Ritz on the small projected problem, FP64, one workgroup per
//    element: diagonal scaling, Cholesky S^T S = U^T U, U^{-1}, the standard
//    problem U^{-T} A U^{-1}, Householder tridiagonalisation, Sturm
//    multisection and inverse iteration, then the coefficients C = D U^{-1} V
//    of the lowest eigenpairs.
//  * Rotations X <- S C (Eq. (2), Algorithm 1 steps 6-7; Algorithm 2 step 5).
//  * Residual norms ||H x_i - theta_i x_i|| and the preconditioner energy.
#include "dg_internal.h"
#include "tridiag.h"
#include "wave_ops.h"

#include <algorithm>
#include <cstdio>

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

// Loads through a global-address-space pointer: the block pointers come from tables
// in memory, so the compiler cannot infer the address space and would otherwise use
// flat loads, which also count against the LDS counter and get conservative waits.
typedef double gd2 __attribute__((ext_vector_type(2)));
template <typename V>
__device__ __forceinline__ V gload(const void* p) {
  return *(const __attribute__((address_space(1))) V*)(p);
}
__device__ __forceinline__ double2 gload2(const void* p) {
  const gd2 v = *(const __attribute__((address_space(1))) gd2*)(p);
  return double2{v.x, v.y};
}
typedef float gf2 __attribute__((ext_vector_type(2)));
typedef float gf4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float2 gload2f(const void* p) {
  const gf2 v = *(const __attribute__((address_space(1))) gf2*)(p);
  return float2{v.x, v.y};
}
__device__ __forceinline__ void gstore2f(void* p, float x, float y) {
  *(__attribute__((address_space(1))) gf2*)(p) = gf2{x, y};
}
__device__ __forceinline__ void gstore2(void* p, double x, double y) {
  *(__attribute__((address_space(1))) gd2*)(p) = gd2{x, y};
}

// ---------------------------------------------------------------------------
// Gram: part[e][split][i][j] = sum_{r in split} S[r,i] T[r,j]
//
// Tiled row-panel design.  The 16x16 output blocks form a grid (bi x bj, the
// upper triangle when the result is symmetric); it is cut into square tiles of
// tb x tb blocks.  A workgroup owns one element, one tile and one contiguous
// range of grid rows: per step it stages GP_R rows of only the columns its tile
// touches (S columns of the tile's block rows, T columns of its block columns)
// in LDS and accumulates the tile's blocks in MFMA registers.  In pair mode a
// tile also holds the same blocks of S^T S, whose columns are S's (staged once
// on the diagonal).  With tb >= bi there is one tile: every column is staged
// once and read from HBM once per Gram.  Partial sums of the row ranges are
// reduced in a fixed order afterwards (deterministic).
// ---------------------------------------------------------------------------
struct GramArgs {
  const ElemDev* elems;
  const int* active;
  ColSet S, T;
  int kS, kT;          // columns per block (per element: <=0 -> E.K) -- multiplied by nb
  int nsplit;
  int rows_e;          // 1: reduce over the first |E_k| rows only
  int sym;             // 1: the result is symmetric, only 16x16 blocks with p <= q are computed
  int same;            // 1: T is the same column set as S
  int tb;              // tile side in 16x16 blocks
  int ntile;           // tiles of the largest element (work items per row range)
  int n_elem;          // elements in the launch
  double* part;        // per element region of part_stride doubles
  long long part_stride;
  int part_ld;         // leading dim of a partial matrix
  int pair;            // 1: also S^T S (symmetric) from the same staged S columns
  long long part_pair; // offset (doubles) of the S^T S partials inside an element's region
};

constexpr int GP_THREADS = 512;
constexpr int GP_R = 16;        // grid rows staged per step
constexpr int GP_MAXCOL = 384;  // staged columns per workgroup (tiles are chosen to fit)

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 lane layout (checked on the device): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; result register q of lane l is D[l/16 + 4q][l%16].
__device__ __forceinline__ d4v mfma16x16x4(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 16x16 output block number b -> (p, q): row-major over p <= q when sym, else over all
__host__ __device__ __forceinline__ void gram_block(int b, int bi, int bj, int sym, int& p, int& q) {
  if (!sym) {
    p = b / bj;
    q = b - p * bj;
    return;
  }
  p = 0;
  while (b >= bj - p) {
    b -= bj - p;
    ++p;
  }
  q = p + b;
}

// One tile of a Gram launch, for an element with bi x bj output blocks.
struct GramTile {
  int P0, P1, Q0, Q1;   // block rows / columns
  bool diag;            // symmetric result, tile on the diagonal: blocks p <= q only
  int ncA, ncB, ncC;    // staged columns: S rows-range, T cols-range, S cols-range (pair, off-diagonal)
  int nloc;             // blocks per product
};

__host__ __device__ __forceinline__ int gram_ntiles(int bi, int bj, int tb, int sym) {
  const int ti = (bi + tb - 1) / tb, tj = (bj + tb - 1) / tb;
  return sym ? ti * (ti + 1) / 2 : ti * tj;
}

__host__ __device__ __forceinline__ GramTile gram_tile(int tile, int bi, int bj, int tb, int sym, int same,
                                                       int pair) {
  const int ti = (bi + tb - 1) / tb, tj = (bj + tb - 1) / tb;
  int I, J;
  gram_block(tile, ti, tj, sym, I, J);
  GramTile g;
  g.P0 = I * tb;
  g.P1 = min(bi, g.P0 + tb);
  g.Q0 = J * tb;
  g.Q1 = min(bj, g.Q0 + tb);
  g.diag = sym && I == J;
  const int np = g.P1 - g.P0, nq = g.Q1 - g.Q0;
  g.ncA = 16 * np;
  g.ncB = (same && g.diag) ? 0 : 16 * nq;
  g.ncC = (pair && !g.diag) ? 16 * nq : 0;
  g.nloc = g.diag ? np * (np + 1) / 2 : np * nq;
  return g;
}

// Block b of a tile's list (blocks nloc .. 2 nloc - 1 are those of S^T S in pair
// mode): LDS columns of its A and B operands, and its output position packed as
// (row block << 16) | (column block << 1) | second product.
__host__ __device__ __forceinline__ void gram_tile_block(const GramTile& g, int b, int offB, int offC, int& acol,
                                                         int& bcol, int& pos) {
  const int np = g.P1 - g.P0, nq = g.Q1 - g.Q0;
  const int second = b >= g.nloc;
  const int lb = b - second * g.nloc;
  int dp, dq;
  if (g.diag) {
    gram_block(lb, np, np, 1, dp, dq);
  } else {
    dp = lb / nq;
    dq = lb - dp * nq;
  }
  acol = dp * 16;
  bcol = (second ? offC : offB) + dq * 16;
  pos = ((g.P0 + dp) << 16) | ((g.Q0 + dq) << 1) | second;
}

// Work item of a Gram workgroup on the 1D grid (ntile x row ranges, the row ranges
// padded to a multiple of 8).  Workgroup p is dispatched to XCD p % 8; its item is
// chosen so that each XCD runs every tile of its row ranges (split, element) back
// to back: the tiles of one row range stage overlapping columns, which that XCD's
// L2 then serves, and the row ranges are interleaved over the XCDs for balance.
struct GramItem {
  int tile, split, e;
  bool valid;
};

__device__ __forceinline__ GramItem gram_item(const GramArgs& A) {
  const int p = blockIdx.x;
  const int xcd = p & 7, slot = p >> 3;
  const int tile = slot % A.ntile, j = slot / A.ntile;
  const int rr = j * 8 + xcd;
  GramItem it;
  it.tile = tile;
  it.split = rr % A.nsplit;
  it.e = rr / A.nsplit;
  it.valid = it.e < A.n_elem;
  return it;
}

// FP64 staging: column-major panels, GP_RP doubles per staged column (16 rows + 2 pad;
// about 57 KB for 384 columns).  Lane l reads rows 4 (l / 16) .. 4 (l / 16) + 3 of
// column (l % 16) of a 16-column fragment as two 16-byte loads.  MFMA k-step j takes
// row 4 (l / 16) + j from every lane group: the four k-steps cover the 16 rows of the
// panel, the same assignment for both operands (a Gram sums over rows in any order).
// Occupancy decides the rate: with at most 6 output blocks per wave (<= 128 VGPRs)
// and 16-row panels two workgroups share a CU and one's barrier and load waits
// overlap the other's matrix work (measured on the C4 batch in one stream: 26.2
// TFLOP/s with 12 blocks, 32-row panels and one workgroup per CU; 35.2 with this;
// 34.9 with three workgroups per CU at 4 blocks).
constexpr int GP_RP = GP_R + 2;
constexpr int GP_LDS_LIMIT = 120000;

// Block b' of a wave's contiguous run: in pair mode the two products of one (p, q)
// are adjacent (they share the A operand, S's column block p); blocks follow the
// tile's row-major order, so runs share p as well.
__device__ __forceinline__ void gram_run_block(const GramTile& g, int bprime, int pair, int offB, int offC,
                                               int& acol, int& bcol, int& pos) {
  const int lb = pair ? (bprime >> 1) : bprime;
  const int second = pair ? (bprime & 1) : 0;
  gram_tile_block(g, lb + second * g.nloc, offB, offC, acol, bcol, pos);
}

// PF: staged values per thread and step (32 columns per pass of the workgroup)
template <typename T, int MAXB, int PF>
__global__ void __launch_bounds__(GP_THREADS, MAXB <= 6 ? 4 : 2) k_gram(GramArgs A) {
  const GramItem item = gram_item(A);
  if (!item.valid) return;
  const int e = item.e;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int kS = kcode(A.kS, E);
  const int kT = kcode(A.kT, E);
  const int ni = A.S.nb * kS, nj = A.T.nb * kT;
  const int bi = (ni + 15) >> 4, bj = (nj + 15) >> 4;
  if (item.tile >= gram_ntiles(bi, bj, A.tb, A.sym)) return;
  const GramTile g = gram_tile(item.tile, bi, bj, A.tb, A.sym, A.same, A.pair);
  const int nblk_all = A.pair ? 2 * g.nloc : g.nloc;
  const int split = item.split;
  const int nrows = nrows_of(E, A.rows_e);
  const int rows_per = ((nrows + A.nsplit - 1) / A.nsplit + GP_R - 1) / GP_R * GP_R;
  const int r0 = split * rows_per;
  const int r1 = min(nrows, r0 + rows_per);
  const int nc = g.ncA + g.ncB + g.ncC;
  // LDS column of the B operand's first staged column, per product
  const int offB = (A.same && g.diag) ? 0 : g.ncA;
  const int offC = g.diag ? 0 : g.ncA + g.ncB;
  extern __shared__ double gsm[];
  double* sm = gsm;                                       // [nc][GP_RP]
  const T** cp = reinterpret_cast<const T**>(gsm + (size_t)nc * GP_RP);   // [nc]
  for (int c = threadIdx.x; c < nc; c += GP_THREADS) {
    const T* ptr = nullptr;
    if (c < g.ncA) {
      const int v = 16 * g.P0 + c;
      if (v < ni) ptr = vcol<T>(E, A.S, v, kS);
    } else if (c < g.ncA + g.ncB) {
      const int v = 16 * g.Q0 + c - g.ncA;
      if (A.same) {
        if (v < ni) ptr = vcol<T>(E, A.S, v, kS);
      } else if (v < nj) {
        ptr = vcol<T>(E, A.T, v, kT);
      }
    } else {
      const int v = 16 * g.Q0 + c - g.ncA - g.ncB;
      if (v < ni) ptr = vcol<T>(E, A.S, v, kS);
    }
    cp[c] = ptr;
  }
  // the wave index is uniform: the block bookkeeping below stays in scalar registers.
  // Wave w owns the contiguous run [w cs, (w + 1) cs) of the tile's blocks; bp, bq: LDS
  // columns of the A and B operands, bo: output position (row block, column block)
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cs = (nblk_all + 7) >> 3;
  int bp[MAXB], bq[MAXB], bo[MAXB];
  bool bv[MAXB];
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int b = w * cs + t;
    bv[t] = t < cs && b < nblk_all;
    bp[t] = bq[t] = bo[t] = 0;
    if (bv[t]) gram_run_block(g, b, A.pair, offB, offC, bp[t], bq[t], bo[t]);
  }
  const int l16 = lane & 15;
  const int lrow = (lane >> 4) * (GP_R / 4);
  d4v acc[MAXB];
#pragma unroll
  for (int t = 0; t < MAXB; ++t) acc[t] = d4v{0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  // staging map: thread -> grid row (tid % 32) of columns tid / 32 + 16 u
  constexpr int kCPP = GP_THREADS / GP_R;   // columns per pass of the workgroup
  const int srow = threadIdx.x & (GP_R - 1), scol = threadIdx.x / GP_R;
  double pre[PF];
  auto load = [&](int rbase) {
    const int rr = rbase + srow;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int c = scol + kCPP * u;
      double v = 0.0;
      if (c < nc) {
        const T* ptr = cp[c];
        // a global load: a flat load would also count against the LDS counter, and
        // the fragment reads' waits would then wait for this prefetch as well
        if (ptr && rr < r1) v = double(gload<T>(ptr + rr));
      }
      pre[u] = v;
    }
  };
  constexpr int KF = GP_R / 4;   // k-steps per panel = values per lane and fragment
  auto frag = [&](int col, double (&f)[KF]) {
    const double2* q = reinterpret_cast<const double2*>(sm + (size_t)(col + l16) * GP_RP + lrow);
#pragma unroll
    for (int m = 0; m < KF / 2; ++m) {
      const double2 x = q[m];
      f[2 * m] = x.x;
      f[2 * m + 1] = x.y;
    }
  };
  if (r0 < r1) load(r0);
  for (int r = r0; r < r1; r += GP_R) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int c = scol + kCPP * u;
      if (c < nc) sm[(size_t)c * GP_RP + srow] = pre[u];
    }
    __syncthreads();
    if (r + GP_R < r1) load(r + GP_R);
    double fa[KF];
#pragma unroll
    for (int j = 0; j < KF; ++j) fa[j] = 0.0;
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
      if (!bv[t]) continue;
      if (t == 0 || bp[t] != bp[t - 1]) frag(bp[t], fa);   // uniform branch: bp is wave-uniform
      double fb[KF];
      frag(bq[t], fb);
#pragma unroll
      for (int j = 0; j < KF; ++j) acc[t] = mfma16x16x4(fa[j], fb[j], acc[t]);
    }
  }
  double* out = A.part + (size_t)e * A.part_stride + (size_t)split * A.part_ld * A.part_ld;
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    if (!bv[t]) continue;
    const bool second = bo[t] & 1;
    double* o = second ? out + A.part_pair : out;
    const int i0 = (bo[t] >> 16) * 16, j = ((bo[t] >> 1) & 0x7FFF) * 16 + l16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + (lane >> 4) + 4 * q;
      if (i < ni && j < (second ? ni : nj)) o[(size_t)i * A.part_ld + j] = acc[t][q];
    }
  }
}

// ---------------------------------------------------------------------------
// Gram of FP32 blocks on FP32 matrix cores (the FP32 parts of the mixed path).
// Same tiles, work items, pair mode and partial sums as k_gram.  A workgroup stages
// 32-row panels of FP32 values column-major in LDS (pitch 36 floats: the sixteen
// columns of a fragment start on distinct 4-bank groups, so the 16-byte fragment
// reads are conflict-free); per panel and output block the eight k-steps of
// v_mfma_f32_16x16x4f32 are summed in FP32 and the panel's sum is added to FP64
// accumulators, so rounding grows with the 32 products of a panel, not with N.
// v_mfma_f32_16x16x4f32 (checked on the device): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; result register q of lane l is D[4 (l/16) + q][l%16].
// ---------------------------------------------------------------------------
constexpr int G3_R = 32;            // grid rows staged per step
constexpr int G3_RP = G3_R + 4;     // floats per staged column
constexpr int G3_MAXCOL = 384;

__device__ __forceinline__ f4v mfma32_16x16x4(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// PF: staged values per thread and step (16 columns per pass of the workgroup)
template <int MAXB, int PF>
__global__ void __launch_bounds__(GP_THREADS, 4) k_gram32(GramArgs A) {
  const GramItem item = gram_item(A);
  if (!item.valid) return;
  const int e = item.e;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int kS = kcode(A.kS, E);
  const int kT = kcode(A.kT, E);
  const int ni = A.S.nb * kS, nj = A.T.nb * kT;
  const int bi = (ni + 15) >> 4, bj = (nj + 15) >> 4;
  if (item.tile >= gram_ntiles(bi, bj, A.tb, A.sym)) return;
  const GramTile g = gram_tile(item.tile, bi, bj, A.tb, A.sym, A.same, A.pair);
  const int nblk_all = A.pair ? 2 * g.nloc : g.nloc;
  const int split = item.split;
  const int nrows = nrows_of(E, A.rows_e);
  const int rows_per = ((nrows + A.nsplit - 1) / A.nsplit + G3_R - 1) / G3_R * G3_R;
  const int r0 = split * rows_per;
  const int r1 = min(nrows, r0 + rows_per);
  const int nc = g.ncA + g.ncB + g.ncC;
  const int offB = (A.same && g.diag) ? 0 : g.ncA;
  const int offC = g.diag ? 0 : g.ncA + g.ncB;
  extern __shared__ double gsm[];
  float* sm = reinterpret_cast<float*>(gsm);                              // [nc][G3_RP]
  const float** cp = reinterpret_cast<const float**>(sm + (size_t)nc * G3_RP);   // [nc]
  for (int c = threadIdx.x; c < nc; c += GP_THREADS) {
    const float* ptr = nullptr;
    if (c < g.ncA) {
      const int v = 16 * g.P0 + c;
      if (v < ni) ptr = vcol<float>(E, A.S, v, kS);
    } else if (c < g.ncA + g.ncB) {
      const int v = 16 * g.Q0 + c - g.ncA;
      if (A.same) {
        if (v < ni) ptr = vcol<float>(E, A.S, v, kS);
      } else if (v < nj) {
        ptr = vcol<float>(E, A.T, v, kT);
      }
    } else {
      const int v = 16 * g.Q0 + c - g.ncA - g.ncB;
      if (v < ni) ptr = vcol<float>(E, A.S, v, kS);
    }
    cp[c] = ptr;
  }
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cs = (nblk_all + 7) >> 3;
  int bp[MAXB], bq[MAXB], bo[MAXB];
  bool bv[MAXB];
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int b = w * cs + t;
    bv[t] = t < cs && b < nblk_all;
    bp[t] = bq[t] = bo[t] = 0;
    if (bv[t]) gram_run_block(g, b, A.pair, offB, offC, bp[t], bq[t], bo[t]);
  }
  const int l16 = lane & 15;
  const int lrow = (lane >> 4) * (G3_R / 4);
  d4v acc[MAXB];
#pragma unroll
  for (int t = 0; t < MAXB; ++t) acc[t] = d4v{0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  constexpr int kCPP = GP_THREADS / G3_R;   // columns per pass of the workgroup
  const int srow = threadIdx.x & (G3_R - 1), scol = threadIdx.x / G3_R;
  float pre[PF];
  auto load = [&](int rbase) {
    const int rr = rbase + srow;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int c = scol + kCPP * u;
      float v = 0.f;
      if (c < nc) {
        const float* ptr = cp[c];
        if (ptr && rr < r1) v = gload<float>(ptr + rr);
      }
      pre[u] = v;
    }
  };
  constexpr int KF = G3_R / 4;   // k-steps per panel = values per lane and fragment
  auto frag = [&](int col, float (&f)[KF]) {
    const float4* q = reinterpret_cast<const float4*>(sm + (size_t)(col + l16) * G3_RP + lrow);
#pragma unroll
    for (int m = 0; m < KF / 4; ++m) {
      const float4 x = q[m];
      f[4 * m] = x.x;
      f[4 * m + 1] = x.y;
      f[4 * m + 2] = x.z;
      f[4 * m + 3] = x.w;
    }
  };
  if (r0 < r1) load(r0);
  for (int r = r0; r < r1; r += G3_R) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int c = scol + kCPP * u;
      if (c < nc) sm[(size_t)c * G3_RP + srow] = pre[u];
    }
    __syncthreads();
    if (r + G3_R < r1) load(r + G3_R);
    float fa[KF];
#pragma unroll
    for (int j = 0; j < KF; ++j) fa[j] = 0.f;
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
      if (!bv[t]) continue;
      if (t == 0 || bp[t] != bp[t - 1]) frag(bp[t], fa);   // uniform branch: bp is wave-uniform
      float fb[KF];
      frag(bq[t], fb);
      f4v s = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < KF; ++j) s = mfma32_16x16x4(fa[j], fb[j], s);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[t][q] += (double)s[q];
    }
  }
  double* out = A.part + (size_t)e * A.part_stride + (size_t)split * A.part_ld * A.part_ld;
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    if (!bv[t]) continue;
    const bool second = bo[t] & 1;
    double* o = second ? out + A.part_pair : out;
    const int i0 = (bo[t] >> 16) * 16, j = ((bo[t] >> 1) & 0x7FFF) * 16 + l16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + 4 * (lane >> 4) + q;
      if (i < ni && j < (second ? ni : nj)) o[(size_t)i * A.part_ld + j] = acc[t][q];
    }
  }
}

// ---------------------------------------------------------------------------
// Gram of FP32 blocks with BF16 matrix cores (the FP32 stage of the mixed path):
// every FP32 value is split into three BF16 pieces x = x0 + x1 + x2 (24 significant
// bits), the six products x_a y_b with a + b <= 2 of a 32-row stage are summed by
// v_mfma_f32_16x16x32_bf16 in FP32, and each stage's sum is added to FP64
// accumulators.  Same row-panel structure as k_gram: a workgroup stages 32 rows of
// every column (three BF16 planes, column-major in LDS) and owns all output blocks.
// v_mfma_f32_16x16x32_bf16 (checked on the device): lane l supplies A[l%16][k] and
// B[k][l%16] for eight k that A and B share; result register q is D[4(l/16)+q][l%16].
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int GB_R = 32;          // rows per stage (the MFMA's k)
constexpr int GB_PITCH = 40;      // BF16 per staged column (32 rows + pad)

__device__ __forceinline__ unsigned short bf16_bits_rn(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_float(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// PF: staged values per thread and stage (16 columns per pass of the workgroup)
template <int MAXB, int PF>
__global__ void __launch_bounds__(GP_THREADS, MAXB <= 6 && PF <= 8 ? 4 : 2) k_gram_bf16(GramArgs A) {
  const GramItem item = gram_item(A);
  if (!item.valid) return;
  const int e = item.e;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int kS = kcode(A.kS, E);
  const int kT = kcode(A.kT, E);
  const int ni = A.S.nb * kS, nj = A.T.nb * kT;
  const int bi = (ni + 15) >> 4, bj = (nj + 15) >> 4;
  if (item.tile >= gram_ntiles(bi, bj, A.tb, A.sym)) return;
  const GramTile g = gram_tile(item.tile, bi, bj, A.tb, A.sym, A.same, A.pair);
  const int nblk_all = A.pair ? 2 * g.nloc : g.nloc;
  const int split = item.split;
  const int nrows = nrows_of(E, A.rows_e);
  const int rows_per = ((nrows + A.nsplit - 1) / A.nsplit + GB_R - 1) / GB_R * GB_R;
  const int r0 = split * rows_per;
  const int r1 = min(nrows, r0 + rows_per);
  const int nc = g.ncA + g.ncB + g.ncC;
  const int offB = (A.same && g.diag) ? 0 : g.ncA;
  const int offC = g.diag ? 0 : g.ncA + g.ncB;
  extern __shared__ double gsm[];
  unsigned short* sm = reinterpret_cast<unsigned short*>(gsm);          // [3][nc][GB_PITCH]
  const float** cp = reinterpret_cast<const float**>(sm + 3 * nc * GB_PITCH);   // [nc]
  for (int c = threadIdx.x; c < nc; c += GP_THREADS) {
    const float* ptr = nullptr;
    if (c < g.ncA) {
      const int v = 16 * g.P0 + c;
      if (v < ni) ptr = vcol<float>(E, A.S, v, kS);
    } else if (c < g.ncA + g.ncB) {
      const int v = 16 * g.Q0 + c - g.ncA;
      if (A.same) {
        if (v < ni) ptr = vcol<float>(E, A.S, v, kS);
      } else if (v < nj) {
        ptr = vcol<float>(E, A.T, v, kT);
      }
    } else {
      const int v = 16 * g.Q0 + c - g.ncA - g.ncB;
      if (v < ni) ptr = vcol<float>(E, A.S, v, kS);
    }
    cp[c] = ptr;
  }
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int bp[MAXB], bq[MAXB], bo[MAXB];
  bool bv[MAXB];
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int b = w + 8 * t;
    bv[t] = b < nblk_all;
    bp[t] = bq[t] = bo[t] = 0;
    if (bv[t]) gram_tile_block(g, b, offB, offC, bp[t], bq[t], bo[t]);
  }
  double acc[MAXB][4];
#pragma unroll
  for (int t = 0; t < MAXB; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[t][q] = 0.0;
  __syncthreads();
  // staging map: thread -> grid row (tid % 32) of columns tid / 32 + 16 u
  const int srow = threadIdx.x & (GB_R - 1), scol = threadIdx.x >> 5;
  float pre[PF];
  auto load = [&](int rbase) {
    const int rr = rbase + srow;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int c = scol + 16 * u;
      float v = 0.f;
      if (c < nc) {
        const float* ptr = cp[c];
        if (ptr && rr < r1) v = ptr[rr];
      }
      pre[u] = v;
    }
  };
  const int plane = nc * GB_PITCH;
  const int koff = 8 * (lane >> 4);
  if (r0 < r1) load(r0);
  for (int r = r0; r < r1; r += GB_R) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int c = scol + 16 * u;
      if (c < nc) {
        const float x = pre[u];
        const unsigned short h0 = bf16_bits_rn(x);
        const float x1 = x - bf16_to_float(h0);
        const unsigned short h1 = bf16_bits_rn(x1);
        const unsigned short h2 = bf16_bits_rn(x1 - bf16_to_float(h1));
        const int o = c * GB_PITCH + srow;
        sm[o] = h0;
        sm[plane + o] = h1;
        sm[2 * plane + o] = h2;
      }
    }
    __syncthreads();
    if (r + GB_R < r1) load(r + GB_R);
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
      if (!bv[t]) continue;
      const int ca = (bp[t] + (lane & 15)) * GB_PITCH + koff;
      const int cb = (bq[t] + (lane & 15)) * GB_PITCH + koff;
      const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(sm + ca);
      const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(sm + plane + ca);
      const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(sm + 2 * plane + ca);
      const bf16x8 c0 = *reinterpret_cast<const bf16x8*>(sm + cb);
      const bf16x8 c1 = *reinterpret_cast<const bf16x8*>(sm + plane + cb);
      const bf16x8 c2 = *reinterpret_cast<const bf16x8*>(sm + 2 * plane + cb);
      f4v sacc = {0.f, 0.f, 0.f, 0.f};
      sacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, c1, sacc, 0, 0, 0);
      sacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, c2, sacc, 0, 0, 0);
      sacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, c0, sacc, 0, 0, 0);
      sacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, c1, sacc, 0, 0, 0);
      sacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, c0, sacc, 0, 0, 0);
      sacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, c0, sacc, 0, 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[t][q] += (double)sacc[q];
    }
  }
  double* out = A.part + (size_t)e * A.part_stride + (size_t)split * A.part_ld * A.part_ld;
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    if (!bv[t]) continue;
    const bool second = bo[t] & 1;
    double* o = second ? out + A.part_pair : out;
    const int j = ((bo[t] >> 1) & 0x7FFF) * 16 + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = (bo[t] >> 16) * 16 + 4 * (lane >> 4) + q;
      if (i < ni && j < (second ? ni : nj)) o[(size_t)i * A.part_ld + j] = acc[t][q];
    }
  }
}

struct GramReduceArgs {
  const ElemDev* elems;
  const int* active;
  int sym;
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
  const bool mirror = A.sym && (i >> 4) > (j >> 4);
  const double* p = A.part + (size_t)e * A.part_stride +
                    (mirror ? (size_t)j * A.part_ld + i : (size_t)i * A.part_ld + j);
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

// Eigenvalues 0..nwant-1 (ascending) of the symmetric tridiagonal T (diagonal sd,
// off-diagonal se) by multisection on Sturm counts: a group of 8 lanes owns one
// eigenvalue and counts at the 8 interior points of its bracket, which shrinks
// 9-fold per round; the round's bracket is read off the group's ballot. The
// bracket keeps count(lo) <= j < count(hi) and stops below abstol or a few ulps of
// its end points. Each lane of a group computes the same bracket, so the group
// stays converged together. Ends with a barrier.
__device__ void multisect_eigs(const double* sd, const double* se, int m, int nwant, double lo0, double hi0,
                               double pivmin, double abstol, double* lam) {
  const int lane = threadIdx.x & 63;
  const int t = lane & 7, gsh = lane & 56;
  const int per_pass = blockDim.x >> 3;
  for (int j0 = 0; j0 < nwant; j0 += per_pass) {
    const int j = j0 + (threadIdx.x >> 3);
    if (j < nwant) {
      double lo = lo0, hi = hi0;
      for (int r = 0; r < 80; ++r) {
        const double w = hi - lo;
        if (!(w > fmax(abstol, 4.0 * 2.2204460492503131e-16 * fmax(fabs(lo), fabs(hi))))) break;
        const double step = w * (1.0 / 9.0);
        const int cnt = sturm_count(sd, se, m, lo + step * (double)(t + 1), pivmin);
        const unsigned bits = (unsigned)(__ballot(cnt > j) >> gsh) & 0xFFu;
        if (bits == 0) {
          lo = lo + step * 8.0;
        } else {
          const int f = __ffs(bits) - 1;   // first point whose count exceeds j
          const double nlo = f > 0 ? lo + step * (double)f : lo;
          hi = lo + step * (double)(f + 1);
          lo = nlo;
        }
      }
      if (t == 0) lam[j] = 0.5 * (lo + hi);
    }
  }
  __syncthreads();
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
  int* status;         // per element: 0 ok, 2 breakdown of the X block
  long long* phase_clk;  // optional: 16 timestamps per element (diagnostics)
  double* work;          // per element work region (the working matrix above kRRLdsOrder)
  long long work_stride;
  double pivot_tol;      // X-column overlap pivots below this (after unit-diagonal scaling) = breakdown
  double drop_tol;       // W/P columns whose scaled pivot is below this are left out of the basis
  double* minpiv;        // optional: smallest scaled pivot, its column, dropped count (diagnostics)
  double ortol;          // eigenvalues closer than ortol * ||T|| are treated as one cluster
  int lds_dyn;           // dynamic LDS bytes of the launch (LDS variant)
  int* hp_flag;          // optional, per element: 1 when the smallest scaled pivot is below hp_tol
                         // (the rotated H P' would carry cancellation error), 0 otherwise and
                         // for inactive elements
  double hp_tol;
};

constexpr int kRRThreads = 512;     // LDS variant (orders up to kRRLdsOrder)
constexpr int kRRThreadsL2 = 1024;  // L2-resident variant: more loads in flight for its latency-bound sweeps
constexpr int kTriMax = 272;   // largest projected problem handled (3 x 88 + pad)

// ---------------------------------------------------------------------------
// Rayleigh-Ritz for the generalised problem (S = [X W P]), one workgroup per
// element:
//   scaled overlap -> Cholesky with column dropping -> in-place U^{-1} = Z
//   -> T = A~ Z, A^ = Z^T T (FP64 MFMA) -> Householder tridiagonal
//   -> Sturm multisection -> inverse iteration (batches of vectors)
//   -> in-order Gram-Schmidt and back-transformation -> C = D Z V.
// The working region W (the matrix, then the inverse-iteration factors, then
// the eigenvectors and reflectors) is dynamic LDS for orders up to
// kRRLdsOrder (kLds = true) and the element's slice of the Gram partial-sum
// area in global memory above that (kLds = false; L2-resident). G keeps Z, Vm
// the scaled A and then the packed reflectors, Um the eigenvectors of T
// between phases.
// ---------------------------------------------------------------------------
constexpr int kLdsPerCU = 163840;                 // 160 KB of LDS per compute unit
constexpr int kRRStaticLds = 21504;               // bound on k_rr_lds's static LDS
constexpr int kRRLdsBytes = kLdsPerCU - kRRStaticLds;
constexpr int kRRLdsOrder = 132;                  // np * np doubles fit in kRRLdsBytes

__device__ __forceinline__ int refl_off(int kk, int m) { return kk * (m - 1) - kk * (kk - 1) / 2; }

template <bool kLds>
__global__ void __launch_bounds__(kLds ? kRRThreads : kRRThreadsL2) k_rr_lds(RRArgs A) {
  const int e = blockIdx.x;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) {
    if (A.hp_flag && threadIdx.x == 0) A.hp_flag[e] = 0;
    return;
  }
  const int K = E.K;
  const bool gen = A.mode == RR_GEN, svd = A.mode == RR_SVD;
  const int n = gen ? A.nb * K : kcode(A.kfix, E);
  const int kx = gen ? K : n;             // leading columns that are never left out
  const int np = n + (n & 1);
  const int nkeep = kcode(A.nkeep, E);
  const int KP = E.kmax3 + 2;
  double* G = E.small + SmallLayout::G(KP);     // in: S^T S (ld n); out: Z (ld np)
  double* Am = E.small + SmallLayout::A(KP);    // in: S^T H S (ld n); then T; then A^
  double* Um = E.small + SmallLayout::U(KP);    // staging: Z^T T, then eigenvectors of the tridiagonal
  double* Vm = E.small + SmallLayout::V(KP);    // scaled A, then packed reflectors
  double* Cm = E.small + SmallLayout::C(KP);
  double* vec = E.small + SmallLayout::vec(KP);
  double* d = vec + VS_D * KP;
  double* theta = vec + VS_THETA * KP;
  double* lam_s = vec + VS_FLAGS * KP;
  extern __shared__ double rr_lds[];
  double* const L = kLds ? rr_lds : A.work + (size_t)e * A.work_stride;
  __shared__ double sh[16];
  __shared__ int brk;
  __shared__ double sd[kTriMax], se[kTriMax], stau[kTriMax];
  __shared__ double vs[kTriMax], ps[kTriMax], ws[kTriMax];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
  auto stamp = [&](int k) {
    if (A.phase_clk && tid == 0) A.phase_clk[e * 16 + k] = wall_clock64();
  };
  stamp(0);
  if (tid == 0) brk = 0;
  __syncthreads();
  int ndrop = 0;
  if (svd) {
    // eigen-decomposition of the Gram matrix itself
    for (int idx = tid; idx < np * np; idx += nt) {
      const int i = idx / np, j = idx % np;
      L[idx] = (i < n && j < n) ? G[(size_t)i * n + j] : 0.0;
    }
    __syncthreads();
  } else {
  // ---- scaled overlap in LDS, scaled A in Vm
  for (int i = tid; i < np; i += nt) {
    const double gii = i < n ? G[(size_t)i * n + i] : 1.0;
    if (!(gii > 0.0) && i < kx) brk = 1;
    d[i] = (i < n && gii > 0.0) ? 1.0 / sqrt(gii) : (i < n ? 0.0 : 1.0);
  }
  __syncthreads();
  for (int idx = tid; idx < np * np; idx += nt) {
    const int i = idx / np, j = idx % np;
    const bool in = i < n && j < n;
    const double s2 = d[i] * d[j];
    L[idx] = in ? G[(size_t)i * n + j] * s2 : (i == j ? 1.0 : 0.0);
    if (gen) Vm[idx] = in ? 0.5 * (Am[(size_t)i * n + j] + Am[(size_t)j * n + i]) * s2 : 0.0;
  }
  __syncthreads();
  // ---- Cholesky L = U^T U (upper, in place); nearly dependent W/P columns leave the basis.
  // Rows keep their unscaled values during the elimination (one barrier per
  // column); the rows are divided by sqrt(pivot) at the end.
  double pmin = 1.0;
  int jmin = -1;
  for (int j = 0; j < n; ++j) {
    const double piv = L[j * np + j];
    if (piv < pmin) {
      pmin = piv;
      jmin = j;
    }
    if (j >= kx && !(piv > A.drop_tol)) {
      __syncthreads();
      for (int i = tid; i < n; i += nt) {
        if (i == j) continue;
        L[i * np + j] = 0.0;
        L[j * np + i] = 0.0;
        Vm[(size_t)i * np + j] = 0.0;
        Vm[(size_t)j * np + i] = 0.0;
      }
      if (tid == 0) {
        L[j * np + j] = 1.0;
        Vm[(size_t)j * np + j] = 0.0;
        d[j] = 0.0;
        ws[j] = 1.0;
      }
      ++ndrop;
      __syncthreads();
      continue;
    }
    if (!(piv > A.pivot_tol) && tid == 0) brk = 1;
    const double pinv = 1.0 / fmax(piv, 1e-300);
    if (tid == 0) ws[j] = sqrt(fmax(piv, 1e-300));
    for (int i = j + 1 + wv; i < n; i += nw) {
      const double f = L[j * np + i] * pinv;
      double* row = L + i * np;
      const double* rj = L + j * np;
      for (int k = i + lane; k < n; k += 64) row[k] -= f * rj[k];
    }
    __syncthreads();
  }
  // divide row j by sqrt(pivot_j): U
  for (int j = wv; j < n; j += nw) {
    const double u = ws[j];
    double* row = L + j * np;
    for (int k = j + 1 + lane; k < n; k += 64) row[k] = (d[j] == 0.0 && k != j) ? 0.0 : row[k] / u;
    if (lane == 0) row[j] = u;
  }
  __syncthreads();
  if (A.hp_flag && tid == 0) A.hp_flag[e] = (brk || !(pmin >= A.hp_tol)) ? 1 : 0;
  if (A.minpiv && tid == 0) {
    A.minpiv[3 * e] = pmin;
    A.minpiv[3 * e + 1] = jmin;
    A.minpiv[3 * e + 2] = ndrop;
  }
  if (brk) {
    // X itself is not positive definite: keep X (C = [I; 0; 0]) and report it
    for (int idx = tid; idx < n * nkeep; idx += nt) {
      const int i = idx / nkeep, j = idx % nkeep;
      Cm[idx] = (i == j) ? 1.0 : 0.0;
    }
    if (tid == 0) A.status[e] = 2;
    return;
  }
  if (tid == 0) A.status[e] = 0;
  stamp(1);
  if constexpr (kLds) {
    // ---- Z = U^{-1}: rows are independent, Z[i][j] = -(1/U[j][j]) sum_{k=i}^{j-1} Z[i][k] U[k][j]
    // left to right. A quad of lanes owns a row (the k sum split four ways, DPP quad
    // reduction); Z[i][j] is kept transposed in the free strictly lower triangle
    // (L[j][i]), the reciprocal diagonal in ws, so U stays intact until every row is
    // done; then Z moves to the upper triangle.
    for (int i = tid; i < n; i += nt) ws[i] = 1.0 / L[i * np + i];
    __syncthreads();
    {
      const int ql = tid & 3;
      for (int i = tid >> 2; i < n; i += nt >> 2) {
        const double zii = ws[i];
        for (int j = i + 1; j < n; ++j) {
          double t = 0.0;
          for (int k = i + ql; k < j; k += 4) t += (k == i ? zii : L[k * np + i]) * L[k * np + j];
          t += dpp_mov<0xB1>(t);   // quad_perm [1,0,3,2]
          t += dpp_mov<0x4E>(t);   // quad_perm [2,3,0,1]
          if (ql == 0) L[j * np + i] = -ws[j] * t;
        }
      }
    }
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += nt) {
      const int i = idx / n, j = idx % n;
      if (i < j) L[i * np + j] = L[j * np + i];
      else if (i == j) L[i * np + i] = ws[i];
    }
    __syncthreads();
  } else {
    // ---- Z = U^{-1} in place, column by column (column j uses the inverted leading block):
    // Z[i][j] = -(1/U[j][j]) sum_{k=i}^{j-1} Z[i][k] U[k][j]
    for (int j = 0; j < n; ++j) {
      for (int k = tid; k < j; k += nt) vs[k] = L[k * np + j];
      __syncthreads();
      const double ajj = 1.0 / L[j * np + j];
      for (int i = wv; i < j; i += nw) {
        const double* zi = L + i * np;
        double t = 0.0;
        for (int k = i + lane; k < j; k += 64) t += zi[k] * vs[k];
        t = wave_sum_dpp(t);
        if (lane == 0) ps[i] = -ajj * t;
      }
      __syncthreads();
      for (int i = tid; i < j; i += nt) L[i * np + j] = ps[i];
      if (tid == 0) L[j * np + j] = ajj;
    }
    __syncthreads();
  }
  if (!gen) {
    // Cholesky QR: C = D Z orthonormalises the columns (n x nkeep)
    for (int idx = tid; idx < n * nkeep; idx += nt) {
      const int i = idx / nkeep, j = idx % nkeep;
      Cm[idx] = (i <= j && j < n) ? d[i] * L[i * np + j] : 0.0;
    }
    stamp(9);
    return;
  }
  // keep Z for the coefficients
  for (int idx = tid; idx < np * np; idx += nt) {
    const int i = idx / np, j = idx % np;
    G[idx] = (i <= j && j < n) ? L[idx] : 0.0;
  }
  stamp(2);
  // ---- T = A~ Z (Am), then A^ = Z^T T (Um), as 16x16 FP64 MFMA tiles (one wave per tile)
  {
    const int nt16 = (n + 15) >> 4;
    const int kst = (n + 3) >> 2;
    for (int t = wv; t < nt16 * nt16; t += nw) {
      const int ti = t / nt16, tj = t % nt16;
      const int ia = ti * 16 + (lane & 15), jb = tj * 16 + (lane & 15);
      const int kmax = min(kst, (tj * 16 + 16 + 3) >> 2);   // Z[k][j] = 0 for k > j
      d4v acc = {0.0, 0.0, 0.0, 0.0};
      for (int ks = 0; ks < kmax; ++ks) {
        const int k = ks * 4 + (lane >> 4);
        const double av = (ia < n && k < n) ? Vm[(size_t)ia * np + k] : 0.0;
        const double bv = (jb < n && k <= jb) ? L[k * np + jb] : 0.0;
        acc = mfma16x16x4(av, bv, acc);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ti * 16 + (lane >> 4) + 4 * q;
        if (i < n && jb < n) Am[(size_t)i * np + jb] = acc[q];
      }
    }
    __syncthreads();
    for (int t = wv; t < nt16 * nt16; t += nw) {
      const int ti = t / nt16, tj = t % nt16;
      const int ia = ti * 16 + (lane & 15), jb = tj * 16 + (lane & 15);
      const int kmax = min(kst, (ti * 16 + 16 + 3) >> 2);   // Z[k][i] = 0 for k > i
      d4v acc = {0.0, 0.0, 0.0, 0.0};
      for (int ks = 0; ks < kmax; ++ks) {
        const int k = ks * 4 + (lane >> 4);
        const double av = (ia < n && k <= ia) ? L[k * np + ia] : 0.0;
        const double bv = (jb < n && k < n) ? Am[(size_t)k * np + jb] : 0.0;
        acc = mfma16x16x4(av, bv, acc);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ti * 16 + (lane >> 4) + 4 * q;
        if (i < n && jb < n) Um[(size_t)i * np + jb] = acc[q];
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += nt) {
    const int i = idx / n, j = idx % n;
    L[(size_t)i * np + j] = 0.5 * (Um[(size_t)i * np + j] + Um[(size_t)j * np + i]);
  }
  __syncthreads();
  if (ndrop > 0) {
    // left-out columns get an eigenvalue above the whole spectrum (Gershgorin bound)
    double rmax = 0.0;
    for (int i = tid; i < n; i += nt) {
      double sacc = 0.0;
      for (int k = 0; k < n; ++k) sacc += fabs(L[(size_t)i * np + k]);
      rmax = fmax(rmax, sacc);
    }
    rmax = block_max(rmax, sh);
    for (int j = tid; j < n; j += nt)
      if (d[j] == 0.0) L[(size_t)j * np + j] = 2.0 * rmax + 1.0;
    __syncthreads();
  }
  }   // !svd
  stamp(3);
  // ---- Householder tridiagonalisation in LDS; reflector kk kept in column kk below the diagonal
  const int m = n;
  __shared__ int skip;
  // the product p = tau A v splits the rows between sets of 256 threads
  constexpr int kSets = (kLds ? kRRThreads : kRRThreadsL2) / 256;
  __shared__ double pq[kSets][kTriMax];
  for (int kk = 0; kk < m - 2; ++kk) {
    const int mr = m - kk - 1;
    if (wv == 0) {
      // reflector from column kk (one wave)
      double part = 0.0;
      for (int i = lane; i < mr; i += 64) {
        const double x = L[(kk + 1 + i) * np + kk];
        part += x * x;
      }
      const double ss = wave_sum_dpp(part);
      const double x0 = L[(kk + 1) * np + kk];
      const double alpha = x0 >= 0.0 ? -sqrt(ss) : sqrt(ss);
      const double vv = ss - x0 * x0 + (x0 - alpha) * (x0 - alpha);
      const bool zero = !(ss > 0.0);
      for (int i = lane; i < mr; i += 64) vs[i] = (i == 0) ? x0 - alpha : L[(kk + 1 + i) * np + kk];
      if (lane == 0) {
        sd[kk] = L[kk * np + kk];
        stau[kk] = zero ? 0.0 : 2.0 / vv;
        se[kk] = zero ? 0.0 : alpha;
        skip = zero ? 1 : 0;
      }
    }
    __syncthreads();
    if (skip) continue;
    const double tau = stau[kk];
    // p = tau A v; A is symmetric, so row i is read as column i (consecutive threads,
    // consecutive addresses): two threads per row, each over half of the rows
    {
      const int q = tid >> 8, qn = (mr + kSets - 1) / kSets;
      const int j0 = q * qn, j1 = min(mr, j0 + qn);
      for (int i = tid & 255; i < mr; i += 256) {
        const double* col = L + (kk + 1) * np + kk + 1 + i;
        double acc = 0.0;
        for (int j = j0; j < j1; ++j) acc += col[j * np] * vs[j];
        pq[q][i] = acc;
      }
    }
    __syncthreads();
    if (wv == 0) {
      double kp = 0.0;
      for (int i = lane; i < mr; i += 64) {
        double p = 0.0;
#pragma unroll
        for (int q = 0; q < kSets; ++q) p += pq[q][i];
        p *= tau;
        ps[i] = p;
        kp += vs[i] * p;
      }
      const double Kc = 0.5 * tau * wave_sum_dpp(kp);
      for (int i = lane; i < mr; i += 64) ws[i] = ps[i] - Kc * vs[i];
    }
    __syncthreads();
    {
      // this lane's entries of v and w stay in registers across the rows
      constexpr int NQ = ((kLds ? kRRLdsOrder : kTriMax) + 63) / 64;
      double vj[NQ], wj[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int j = lane + 64 * q;
        vj[q] = j < mr ? vs[j] : 0.0;
        wj[q] = j < mr ? ws[j] : 0.0;
      }
      for (int i = wv; i < mr; i += nw) {
        double* row = L + (kk + 1 + i) * np + kk + 1;
        const double vi = vs[i], wi = ws[i];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int j = lane + 64 * q;
          if (j < mr) row[j] -= vi * wj[q] + wi * vj[q];
        }
        if (lane == 0) L[(kk + 1 + i) * np + kk] = vi;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (m >= 2) {
      sd[m - 2] = L[(size_t)(m - 2) * np + m - 2];
      se[m - 2] = L[(size_t)(m - 1) * np + m - 2];
      stau[m - 2] = 0.0;
    }
    sd[m - 1] = L[(size_t)(m - 1) * np + m - 1];
    se[m - 1] = 0.0;
  }
  // reflectors to Vm, packed by column (rows kk+1 .. m-1 of column kk)
  for (int kk = wv; kk < m - 2; kk += nw) {
    double* dst = Vm + refl_off(kk, m);
    for (int i = lane; i < m - 1 - kk; i += 64) dst[i] = L[(size_t)(kk + 1 + i) * np + kk];
  }
  __syncthreads();
  stamp(4);
  // ---- eigenvalues by bisection on Sturm counts (thread j -> j-th smallest)
  __shared__ double sb_lo, sb_hi, sb_norm;
  if (tid == 0) {
    double lo = 1e300, hi = -1e300, nrm = 0.0;
    for (int i = 0; i < m; ++i) {
      const double r = (i > 0 ? fabs(se[i - 1]) : 0.0) + (i < m - 1 ? fabs(se[i]) : 0.0);
      lo = fmin(lo, sd[i] - r);
      hi = fmax(hi, sd[i] + r);
      nrm = fmax(nrm, fabs(sd[i]) + r);
    }
    sb_norm = fmax(nrm, 1e-300);
    sb_lo = lo - 1e-12 * sb_norm - 1e-300;
    sb_hi = hi + 1e-12 * sb_norm + 1e-300;
  }
  __syncthreads();
  const double onenorm = sb_norm;
  const double pivmin = 1e-300 + 1e-30 * onenorm * onenorm;
  const int nwant = svd ? m : min(nkeep, m);
  multisect_eigs(sd, se, m, nwant, sb_lo, sb_hi, pivmin, 2.0 * 2.2204460492503131e-16 * onenorm, lam_s);
  stamp(5);
  // ---- eigenvectors of T by inverse iteration, factors in LDS, R vectors per batch;
  // eigenvalues closer than ortol ||T|| form a cluster whose vectors are computed in
  // order, each re-orthogonalised against the earlier ones (read back from Um)
  __shared__ int cst[kTriMax];
  __shared__ double shf[kTriMax];
  __shared__ int maxrank;
  if (tid == 0) {
    const double ortol = A.ortol * onenorm, pertol = 10.0 * 2.2e-16 * onenorm;
    int mr = 0;
    for (int j = 0; j < nwant; ++j) {
      cst[j] = (j > 0 && lam_s[j] - lam_s[j - 1] <= ortol) ? cst[j - 1] : j;
      shf[j] = lam_s[j];
      if (j > 0 && cst[j] != j && shf[j] < shf[j - 1] + pertol) shf[j] = shf[j - 1] + pertol;
      mr = max(mr, j - cst[j]);
    }
    maxrank = mr;
  }
  __syncthreads();
  double* Zv = Um;   // eigenvector j of T at Zv[j * np + i]
  // R vectors per batch, each with five FP64 arrays and a byte array of length np
  const long long wbytes = kLds ? (long long)A.lds_dyn : A.work_stride * (long long)sizeof(double);
  const int R = (int)min((long long)nt, wbytes / (np * (5 * (int)sizeof(double) + 1)));
  // vector of this thread: spread over the waves (latency hiding); its storage
  // column: consecutive lanes adjacent when the whole block has a slot
  const int slot = (lane < (R + nw - 1) / nw) ? lane * nw + wv : R;
  const int col = R == nt ? wv * 64 + lane : slot;
  for (int cb = 0; cb < nwant; cb += R) {
    for (int rnd = 0; rnd <= maxrank; ++rnd) {
      const int j = cb + slot;
      if (slot < R && j < nwant && j - cst[j] == rnd) {
        StridedD ta{L + 0 * (size_t)np * R + col, R};
        StridedD tb{L + 1 * (size_t)np * R + col, R};
        StridedD tu{L + 2 * (size_t)np * R + col, R};
        StridedD tl{L + 3 * (size_t)np * R + col, R};
        StridedD z{L + 4 * (size_t)np * R + col, R};
        StridedB pv{reinterpret_cast<unsigned char*>(L + 5 * (size_t)np * R) + col, R};
        tri_lu(sd, se, m, shf[j], 2.2e-16 * onenorm, ta, tb, tu, tl, pv);
        for (int i = 0; i < m; ++i) z[i] = hash_unit(j, i);
        // an isolated eigenvalue needs no re-orthogonalisation: two solves (growth
        // at most ~1/(eps ||T||) each, far from overflow), one normalisation
        const bool single = cst[j] == j && (j + 1 >= nwant || cst[j + 1] == j + 1);
        const int n_it = single ? 2 : 4;
        for (int it = 0; it < n_it; ++it) {
          tri_solve(m, ta, tb, tu, tl, pv, z);
          if (single && it + 1 < n_it) continue;
          for (int q = cst[j]; q < j; ++q) {
            const double* zq = Zv + (size_t)q * np;
            double dot = 0.0;
            for (int i = 0; i < m; ++i) dot += zq[i] * z[i];
            for (int i = 0; i < m; ++i) z[i] -= dot * zq[i];
          }
          double nn = 0.0;
          for (int i = 0; i < m; ++i) nn += z[i] * z[i];
          nn = 1.0 / sqrt(nn);
          for (int i = 0; i < m; ++i) z[i] *= nn;
        }
        for (int i = 0; i < np; ++i) Zv[(size_t)j * np + i] = (i < m) ? z[i] : 0.0;
      }
      __syncthreads();
    }
  }
  stamp(6);
  // ---- eigenvectors and reflectors into LDS: in-order Gram-Schmidt, back-transformation
  double* zl = L;                                  // nwant x np
  double* rl = L + (size_t)nwant * np;             // packed reflectors
  const int nrefl = m >= 2 ? refl_off(m - 2, m) : 0;
  for (int idx = tid; idx < nwant * np; idx += nt) zl[idx] = Zv[idx];
  for (int idx = tid; idx < nrefl; idx += nt) rl[idx] = Vm[idx];
  __syncthreads();
  for (int j = 1; j < nwant; ++j) {
    double* zj = zl + j * np;
    for (int q = wv; q < j; q += nw) {
      const double* zq = zl + q * np;
      double dot = 0.0;
      for (int i = lane; i < m; i += 64) dot += zq[i] * zj[i];
      dot = wave_sum_dpp(dot);
      if (lane == 0) ps[q] = dot;
    }
    __syncthreads();
    // z_j -= sum_q (z_q . z_j) z_q: a quad of lanes per row, the q sum split four ways;
    // per-wave sums of squares for the norm
    {
      const int ql = tid & 3;
      double part = 0.0;
      for (int i = tid >> 2; i < m; i += nt >> 2) {
        double t = 0.0;
        for (int q = ql; q < j; q += 4) t += ps[q] * zl[q * np + i];
        t += dpp_mov<0xB1>(t);   // quad_perm [1,0,3,2]
        t += dpp_mov<0x4E>(t);   // quad_perm [2,3,0,1]
        if (ql == 0) {
          const double v = zj[i] - t;
          zj[i] = v;
          part += v * v;
        }
      }
      part = wave_sum_dpp(part);
      if (lane == 0) sh[wv] = part;
    }
    __syncthreads();
    {
      double nn2 = 0.0;
      for (int q = 0; q < nw; ++q) nn2 += sh[q];
      const double nn = 1.0 / sqrt(nn2);
      for (int i = tid; i < m; i += nt) zj[i] *= nn;
    }
    __syncthreads();
  }
  stamp(7);
  if constexpr (kLds) {
    // back-transform: z <- H_0 ... H_{m-3} z with eight lanes per vector (the dot
    // product reduced within the lane group) and every vector at once: the reflectors
    // are read-only, so the vectors need no barriers between reflectors
    {
      const int l8 = tid & 7;
      for (int j = tid >> 3; j < nwant; j += nt >> 3) {
        double* z = zl + (size_t)j * np;
        for (int kk = m - 3; kk >= 0; --kk) {
          const double tau = stau[kk];
          if (tau == 0.0) continue;
          const double* v = rl + refl_off(kk, m);   // rows kk+1 .. m-1
          const int len = m - 1 - kk;
          double dot = 0.0;
          for (int i = l8; i < len; i += 8) dot += v[i] * z[kk + 1 + i];
          dot = group8_sum(dot) * tau;
          for (int i = l8; i < len; i += 8) z[kk + 1 + i] -= dot * v[i];
        }
      }
    }
  } else {
    // back-transform: z <- H_0 ... H_{m-3} z (lanes over rows); a wave carries four of
    // its vectors through the reflectors together, so that their dot products and
    // reductions overlap
    {
      constexpr int BV = 4;
      for (int j0 = wv; j0 < nwant; j0 += BV * nw) {
        double* z[BV];
        bool on[BV];
#pragma unroll
        for (int b = 0; b < BV; ++b) {
          const int j = j0 + b * nw;
          on[b] = j < nwant;
          z[b] = zl + (size_t)(on[b] ? j : j0) * np;
        }
        for (int kk = m - 3; kk >= 0; --kk) {
          const double tau = stau[kk];
          if (tau == 0.0) continue;
          const double* v = rl + refl_off(kk, m);   // rows kk+1 .. m-1
          double dot[BV];
#pragma unroll
          for (int b = 0; b < BV; ++b) dot[b] = 0.0;
          for (int i = lane; i < m - 1 - kk; i += 64) {
            const double vi = v[i];
#pragma unroll
            for (int b = 0; b < BV; ++b) dot[b] += vi * z[b][kk + 1 + i];
          }
#pragma unroll
          for (int b = 0; b < BV; ++b) dot[b] = wave_sum_dpp(dot[b]) * tau;
          for (int i = lane; i < m - 1 - kk; i += 64) {
            const double vi = v[i];
#pragma unroll
            for (int b = 0; b < BV; ++b)
              if (on[b]) z[b][kk + 1 + i] -= dot[b] * vi;
          }
        }
      }
    }
  }
  __syncthreads();
  stamp(8);
  if (svd) {
    // C = V[:, sel] / sigma with sigma = sqrt(eigenvalue), descending
    for (int idx = tid; idx < n * nkeep; idx += nt) {
      const int i = idx / nkeep, j = idx % nkeep;
      const int col = m - 1 - j;
      const double sg = (col >= 0) ? sqrt(fmax(lam_s[col], 0.0)) : 0.0;
      Cm[idx] = (col >= 0 && sg > 0.0) ? zl[col * np + i] / sg : 0.0;
    }
    for (int j = tid; j < nkeep; j += nt) theta[j] = (m - 1 - j >= 0) ? sqrt(fmax(lam_s[m - 1 - j], 0.0)) : 0.0;
    __syncthreads();
    stamp(9);
    return;
  }
  // ---- C = D Z V[:, :nkeep] (n x nkeep, ld nkeep) as 16x16 FP64 MFMA tiles (one wave
  // per tile; Z[i][k] = 0 for k < i, so a tile's k range starts at its first row);
  // left-out rows are zero (d = 0)
  {
    const int nti = (n + 15) >> 4, ntj = (nkeep + 15) >> 4;
    const int kst = (n + 3) >> 2;
    for (int tile = wv; tile < nti * ntj; tile += nw) {
      const int ti = tile / ntj, tj = tile % ntj;
      const int ia = ti * 16 + (lane & 15), jb = tj * 16 + (lane & 15);
      d4v acc = {0.0, 0.0, 0.0, 0.0};
      for (int ks = ti * 4; ks < kst; ++ks) {
        const int k = ks * 4 + (lane >> 4);
        const double av = (ia < n && k < n && k >= ia) ? G[(size_t)ia * np + k] : 0.0;
        const double bv = (jb < nwant && k < n) ? zl[(size_t)jb * np + k] : 0.0;
        acc = mfma16x16x4(av, bv, acc);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ti * 16 + (lane >> 4) + 4 * q;
        if (i < n && jb < nkeep) Cm[(size_t)i * nkeep + jb] = jb < nwant ? d[i] * acc[q] : 0.0;
      }
    }
  }
  for (int j = tid; j < nkeep; j += nt) theta[j] = j < nwant ? lam_s[j] : 0.0;
  __syncthreads();
  stamp(9);
}

// ---------------------------------------------------------------------------
// rotation: out_o[:, j] = beta_o out_o[:, j] + alpha sum_{c in [c0_o, c1_o)} S[:, c] C[c, j]
// ---------------------------------------------------------------------------
constexpr int RT_THREADS = 512;
constexpr int RT_RT = 2;                            // 16-row tiles per wave
constexpr int RT_ROWS = (RT_THREADS / 64) * RT_RT * 16;   // rows per workgroup (256)
constexpr int RT_CC = 32;     // C rows staged per step
constexpr int RT_MAXC = 96;   // max output columns (6 MFMA column tiles)
constexpr int RT_NCT = RT_MAXC / 16;

// out_o[:, j] = beta_o out_o[:, j] + alpha sum_c S[:, c] C[c, j] with FP64 MFMA.
// The product is formed transposed, out^T = C^T S^T, so that each lane's
// results are 16 consecutive grid rows of one column (128-byte stores).
// With two outputs whose C row ranges nest (range 1 is a suffix of range 0),
// the suffix is accumulated first, stored as output 1, then completed.
// C rows of a chunk are staged transposed: for each output column n, its RT_CC
// coefficients contiguous (pitch RT_CP doubles).  Lane l takes the 8 coefficients
// k = 8 (l / 16) .. 8 (l / 16) + 7 of column (l % 16) of a 16-column tile with four
// 16-byte LDS loads (pitch 272 bytes: 8 or 16 consecutive lanes on distinct banks);
// MFMA k-step ks uses k = 8 (l / 16) + ks, and the S operand follows the same
// assignment.  The two 16-row tiles of a wave interleave (lane row 2 (l % 16) + u), so
// a lane's two S values of a column, and its two outputs, are adjacent in memory and
// move as one 16-byte access.
constexpr int RT_CP = RT_CC + 2;

template <typename T, int NCT>
__global__ void __launch_bounds__(RT_THREADS, NCT <= 3 ? 3 : 2) k_rotate(RotArgs A) {
  static_assert(sizeof(T) == 8 && RT_RT == 2, "FP64 rotation with two interleaved row tiles per lane");
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
  __shared__ double sc[NCT * 16][RT_CP];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kl = lane >> 4;
  // rows of this lane: rr0, rr0 + 1 (u = 0, 1)
  const int rr0 = r0 + w * RT_RT * 16 + 2 * (lane & 15);
  const bool in0 = rr0 < nrows, in1 = rr0 + 1 < nrows;
  const int nct = (ncol + 15) / 16;
  const double* Cm = E.small + soff(A.c_off, E);
  d4v acc[RT_RT][NCT];
#pragma unroll
  for (int u = 0; u < RT_RT; ++u)
#pragma unroll
    for (int t = 0; t < NCT; ++t) acc[u][t] = d4v{0.0, 0.0, 0.0, 0.0};
  const int nseg = A.nout > 1 ? 2 : 1;
  for (int sg = 0; sg < nseg; ++sg) {
    // segment bounds
    int lo, hi;
    if (A.nout > 1) {
      lo = sg == 0 ? c0[1] : c0[0];
      hi = sg == 0 ? c1[1] : c0[1];
    } else {
      lo = c0[0];
      hi = c1[0];
    }
    // S values of the next C chunk are loaded while the current one is multiplied.
    // The (at most three) block bases of S are resolved once: a per-column lookup of
    // the block table would put a dependent pointer load before every column load.
    const T* sb0 = reinterpret_cast<const T*>(E.blk[A.S.blk[0]]);
    const long long d1 = A.S.nb > 1 ? reinterpret_cast<const T*>(E.blk[A.S.blk[1]]) - sb0 : 0;
    const long long d2 = A.S.nb > 2 ? reinterpret_cast<const T*>(E.blk[A.S.blk[2]]) - sb0 : 0;
    const long long ldS = E.ld;
    auto scol = [&](int c) -> const T* {
      const bool in1 = c >= kS, in2 = c >= 2 * kS;
      const long long off = (in2 ? d2 : (in1 ? d1 : 0LL)) + (long long)(c - (in2 ? 2 * kS : (in1 ? kS : 0))) * ldS;
      return sb0 + off;
    };
    double av[RT_CC / 4][RT_RT], an[RT_CC / 4][RT_RT];
    // branch-free: every lane loads one 16-byte pair from a valid address (the column
    // clamped to lo, the row pair to 0; a lone last row's partner lies inside the
    // leading dimension, which is even and at least N + 1 for odd N) and zeroes what
    // is out of range
    auto load_s = [&](int cb, double (&dst)[RT_CC / 4][RT_RT]) {
#pragma unroll
      for (int ks = 0; ks < RT_CC / 4; ++ks) {
        const int c = cb + kl * (RT_CC / 4) + ks;
        const bool cin = c < hi;
        const T* col = scol(cin ? c : lo);
        const double2 v = gload2(col + (in0 ? rr0 : 0));
        dst[ks][0] = (cin && in0) ? v.x : 0.0;
        dst[ks][1] = (cin && in1) ? v.y : 0.0;
      }
    };
    // with six column tiles (two waves per SIMD, registers to spare) the C rows of the
    // next chunk are prefetched into registers as well; with three (three waves per
    // SIMD) they are read when staged
    constexpr bool kPrefC = NCT > 3;
    constexpr int CPT = kPrefC ? (RT_CC * NCT * 16 + RT_THREADS - 1) / RT_THREADS : 1;
    double cn[CPT];
    auto load_c = [&](int cb) {
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int idx = threadIdx.x + u * RT_THREADS;
        const int cc = idx / (NCT * 16), j = idx % (NCT * 16);
        const int c = cb + cc;
        const bool ok = idx < RT_CC * NCT * 16 && c < hi && j < ncol;
        const double v = gload<double>(Cm + (ok ? (size_t)c * cld + j : 0));
        cn[u] = ok ? v : 0.0;
      }
    };
    if (lo < hi) {
      load_s(lo, an);
      if constexpr (kPrefC) load_c(lo);
    }
    for (int cb = lo; cb < hi; cb += RT_CC) {
      __syncthreads();
      if constexpr (kPrefC) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
          const int idx = threadIdx.x + u * RT_THREADS;
          if (idx < RT_CC * NCT * 16) sc[idx % (NCT * 16)][idx / (NCT * 16)] = cn[u];
        }
      } else {
        for (int idx = threadIdx.x; idx < RT_CC * NCT * 16; idx += RT_THREADS) {
          const int cc = idx / (NCT * 16), j = idx % (NCT * 16);
          const int c = cb + cc;
          sc[j][cc] = (c < hi && j < ncol) ? Cm[(size_t)c * cld + j] : 0.0;
        }
      }
#pragma unroll
      for (int ks = 0; ks < RT_CC / 4; ++ks)
#pragma unroll
        for (int u = 0; u < RT_RT; ++u) av[ks][u] = an[ks][u];
      __syncthreads();
      if (cb + RT_CC < hi) {
        load_s(cb + RT_CC, an);
        if constexpr (kPrefC) load_c(cb + RT_CC);
      }
#pragma unroll
      for (int t = 0; t < NCT; ++t) {
        if (t >= nct) continue;
        const double2* q = reinterpret_cast<const double2*>(&sc[t * 16 + (lane & 15)][kl * (RT_CC / 4)]);
        double cf[RT_CC / 4];
#pragma unroll
        for (int m = 0; m < RT_CC / 8; ++m) {
          const double2 v = q[m];
          cf[2 * m] = v.x;
          cf[2 * m + 1] = v.y;
        }
#pragma unroll
        for (int ks = 0; ks < RT_CC / 4; ++ks)
#pragma unroll
          for (int u = 0; u < RT_RT; ++u) acc[u][t] = mfma16x16x4(cf[ks], av[ks][u], acc[u][t]);
      }
    }
    // store the output this segment completes: lane holds out[rows rr0, rr0 + 1][col 16 t + kl + 4 q]
    const int o = (A.nout > 1 && sg == 0) ? 1 : 0;
    T* out = reinterpret_cast<T*>(E.blk[A.out_blk[o]]);
    const double beta = A.beta[o];
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      if (t >= nct) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = t * 16 + kl + 4 * q;
        if (j >= ncol) continue;
        T* p = out + (size_t)j * E.ld + rr0;
        // the beta term: the output's own values, or those of an FP32 block
        const float* p32 = A.add32 ? reinterpret_cast<const float*>(E.blk[A.add32_blk[o]]) + (size_t)j * E.ld + rr0
                                   : nullptr;
        if (in1) {
          double2 v = {A.alpha * acc[0][t][q], A.alpha * acc[1][t][q]};
          if (beta != 0.0) {
            double2 prev;
            if (p32) {
              const float2 f = gload2f(p32);
              prev = double2{(double)f.x, (double)f.y};
            } else {
              prev = gload2(p);
            }
            v.x += beta * prev.x;
            v.y += beta * prev.y;
          }
          gstore2(p, v.x, v.y);
        } else if (in0) {
          const double prev = beta != 0.0 ? beta * (p32 ? (double)*p32 : double(*p)) : 0.0;
          *p = T(prev + A.alpha * acc[0][t][q]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same rotation for FP32 blocks on FP32 matrix cores (v_mfma_f32_16x16x4f32,
// FP32 sums): C chunks of 32 rows staged transposed as FP32 (pitch 36 floats, the
// eight coefficients of a lane two 16-byte reads), each lane's two row tiles are
// adjacent rows, so S loads and output stores move 8 bytes per column.  Lane l's
// result q of column tile t is output column 16 t + 4 (l / 16) + q.
// ---------------------------------------------------------------------------
constexpr int R3_CP = RT_CC + 4;

template <int NCT>
__global__ void __launch_bounds__(RT_THREADS, NCT <= 3 ? 4 : 2) k_rotate32(RotArgs A) {
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
  __shared__ __attribute__((aligned(16))) float sc[NCT * 16][R3_CP];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kl = lane >> 4;
  const int rr0 = r0 + w * RT_RT * 16 + 2 * (lane & 15);
  const bool in0 = rr0 < nrows, in1 = rr0 + 1 < nrows;
  const int nct = (ncol + 15) / 16;
  const double* Cm = E.small + soff(A.c_off, E);
  f4v acc[RT_RT][NCT];
#pragma unroll
  for (int u = 0; u < RT_RT; ++u)
#pragma unroll
    for (int t = 0; t < NCT; ++t) acc[u][t] = f4v{0.f, 0.f, 0.f, 0.f};
  const int nseg = A.nout > 1 ? 2 : 1;
  for (int sg = 0; sg < nseg; ++sg) {
    int lo, hi;
    if (A.nout > 1) {
      lo = sg == 0 ? c0[1] : c0[0];
      hi = sg == 0 ? c1[1] : c0[1];
    } else {
      lo = c0[0];
      hi = c1[0];
    }
    const float* sb0 = reinterpret_cast<const float*>(E.blk[A.S.blk[0]]);
    const long long d1 = A.S.nb > 1 ? reinterpret_cast<const float*>(E.blk[A.S.blk[1]]) - sb0 : 0;
    const long long d2 = A.S.nb > 2 ? reinterpret_cast<const float*>(E.blk[A.S.blk[2]]) - sb0 : 0;
    const long long ldS = E.ld;
    auto scol = [&](int c) -> const float* {
      const bool b1 = c >= kS, b2 = c >= 2 * kS;
      const long long off = (b2 ? d2 : (b1 ? d1 : 0LL)) + (long long)(c - (b2 ? 2 * kS : (b1 ? kS : 0))) * ldS;
      return sb0 + off;
    };
    float av[RT_CC / 4][RT_RT], an[RT_CC / 4][RT_RT];
    // branch-free, as in k_rotate: one 8-byte pair from a valid address per column
    auto load_s = [&](int cb, float (&dst)[RT_CC / 4][RT_RT]) {
#pragma unroll
      for (int ks = 0; ks < RT_CC / 4; ++ks) {
        const int c = cb + kl * (RT_CC / 4) + ks;
        const bool cin = c < hi;
        const float* col = scol(cin ? c : lo);
        const float2 v = gload2f(col + (in0 ? rr0 : 0));
        dst[ks][0] = (cin && in0) ? v.x : 0.f;
        dst[ks][1] = (cin && in1) ? v.y : 0.f;
      }
    };
    constexpr int CPT = (RT_CC * NCT * 16 + RT_THREADS - 1) / RT_THREADS;
    double cn[CPT];
    auto load_c = [&](int cb) {
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int idx = threadIdx.x + u * RT_THREADS;
        const int cc = idx / (NCT * 16), j = idx % (NCT * 16);
        const int c = cb + cc;
        const bool ok = idx < RT_CC * NCT * 16 && c < hi && j < ncol;
        const double v = gload<double>(Cm + (ok ? (size_t)c * cld + j : 0));
        cn[u] = ok ? v : 0.0;
      }
    };
    if (lo < hi) {
      load_s(lo, an);
      load_c(lo);
    }
    for (int cb = lo; cb < hi; cb += RT_CC) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int idx = threadIdx.x + u * RT_THREADS;
        if (idx < RT_CC * NCT * 16) sc[idx % (NCT * 16)][idx / (NCT * 16)] = (float)cn[u];
      }
#pragma unroll
      for (int ks = 0; ks < RT_CC / 4; ++ks)
#pragma unroll
        for (int u = 0; u < RT_RT; ++u) av[ks][u] = an[ks][u];
      __syncthreads();
      if (cb + RT_CC < hi) {
        load_s(cb + RT_CC, an);
        load_c(cb + RT_CC);
      }
#pragma unroll
      for (int t = 0; t < NCT; ++t) {
        if (t >= nct) continue;
        const float4* q = reinterpret_cast<const float4*>(&sc[t * 16 + (lane & 15)][kl * (RT_CC / 4)]);
        float cf[RT_CC / 4];
#pragma unroll
        for (int m = 0; m < RT_CC / 16; ++m) {
          const float4 v = q[m];
          cf[4 * m] = v.x;
          cf[4 * m + 1] = v.y;
          cf[4 * m + 2] = v.z;
          cf[4 * m + 3] = v.w;
        }
#pragma unroll
        for (int ks = 0; ks < RT_CC / 4; ++ks)
#pragma unroll
          for (int u = 0; u < RT_RT; ++u) acc[u][t] = mfma32_16x16x4(cf[ks], av[ks][u], acc[u][t]);
      }
    }
    // store the output this segment completes: lane holds out[rows rr0, rr0 + 1][col 16 t + 4 kl + q]
    const int o = (A.nout > 1 && sg == 0) ? 1 : 0;
    float* out = reinterpret_cast<float*>(E.blk[A.out_blk[o]]);
    const double beta = A.beta[o];
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      if (t >= nct) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = t * 16 + 4 * kl + q;
        if (j >= ncol) continue;
        float* p = out + (size_t)j * E.ld + rr0;
        if (in1) {
          double v0 = A.alpha * (double)acc[0][t][q], v1 = A.alpha * (double)acc[1][t][q];
          if (beta != 0.0) {
            const float2 prev = gload2f(p);
            v0 += beta * (double)prev.x;
            v1 += beta * (double)prev.y;
          }
          gstore2f(p, (float)v0, (float)v1);
        } else if (in0) {
          const double prev = beta != 0.0 ? beta * (double)*p : 0.0;
          *p = (float)(prev + A.alpha * (double)acc[0][t][q]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same rotation for FP32 blocks on BF16 matrix cores (the FP32 stage of the
// mixed path): S values and C coefficients are split into three BF16 pieces each
// (24 significant bits), and the six products s_a c_b with a + b <= 2 of every
// 32-row step of C go to v_mfma_f32_16x16x32_bf16, smallest first, summed in FP32.
// out^T = C^T S^T as in k_rotate: the A operand is a 16-column tile of C^T (staged
// as three BF16 planes in LDS, the 32 C rows of a step contiguous per column), the
// B operand 32 S columns of 16 grid rows (eight per lane, split in registers).
// ---------------------------------------------------------------------------
constexpr int RB_K = 32;        // C rows per MFMA step
constexpr int RB_PITCH = 40;    // BF16 per staged C column (32 rows + pad)

typedef unsigned short us8v __attribute__((ext_vector_type(8)));

template <int NCT>
__global__ void __launch_bounds__(RT_THREADS, 2) k_rotate_bf16(RotArgs A) {
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
  __shared__ __attribute__((aligned(16))) unsigned short scb[3][NCT * 16][RB_PITCH];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kl = lane >> 4;
  int rrow[RT_RT];
#pragma unroll
  for (int u = 0; u < RT_RT; ++u) rrow[u] = r0 + (w * RT_RT + u) * 16 + (lane & 15);
  const int nct = (ncol + 15) / 16;
  const double* Cm = E.small + soff(A.c_off, E);
  f4v acc[RT_RT][NCT];
#pragma unroll
  for (int u = 0; u < RT_RT; ++u)
#pragma unroll
    for (int t = 0; t < NCT; ++t) acc[u][t] = f4v{0.f, 0.f, 0.f, 0.f};
  const int nseg = A.nout > 1 ? 2 : 1;
  for (int sg = 0; sg < nseg; ++sg) {
    int lo, hi;
    if (A.nout > 1) {
      lo = sg == 0 ? c0[1] : c0[0];
      hi = sg == 0 ? c1[1] : c0[1];
    } else {
      lo = c0[0];
      hi = c1[0];
    }
    // S values of the next step (columns cb + 8 kl + i, rows rrow[u]) are loaded
    // while the current step is multiplied
    // block bases resolved once (a per-column lookup of the block table puts a
    // dependent pointer load before every column load); branch-free global loads from
    // clamped valid addresses, out-of-range values zeroed
    const float* sb0 = reinterpret_cast<const float*>(E.blk[A.S.blk[0]]);
    const long long d1 = A.S.nb > 1 ? reinterpret_cast<const float*>(E.blk[A.S.blk[1]]) - sb0 : 0;
    const long long d2 = A.S.nb > 2 ? reinterpret_cast<const float*>(E.blk[A.S.blk[2]]) - sb0 : 0;
    const long long ldS = E.ld;
    auto scol = [&](int c) -> const float* {
      const bool b1 = c >= kS, b2 = c >= 2 * kS;
      const long long off = (b2 ? d2 : (b1 ? d1 : 0LL)) + (long long)(c - (b2 ? 2 * kS : (b1 ? kS : 0))) * ldS;
      return sb0 + off;
    };
    float sv[RT_RT][8], sn[RT_RT][8];
    auto load_s = [&](int cb, float (&dst)[RT_RT][8]) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int c = cb + 8 * kl + i;
        const bool cin = c < hi;
        const float* col = scol(cin ? c : lo);
#pragma unroll
        for (int u = 0; u < RT_RT; ++u) {
          const bool ok = cin && rrow[u] < nrows;
          const float v = gload<float>(col + (rrow[u] < nrows ? rrow[u] : 0));
          dst[u][i] = ok ? v : 0.f;
        }
      }
    };
    // with six column tiles the C rows of the next step are prefetched into registers
    // too; with three they are read when staged (the registers would cost occupancy)
    constexpr bool kPrefC = NCT > 3;
    constexpr int CPT = (RB_K * NCT * 16 + RT_THREADS - 1) / RT_THREADS;
    double cn[kPrefC ? CPT : 1];
    auto load_c = [&](int cb) {
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int idx = threadIdx.x + u * RT_THREADS;
        const int j = idx % (NCT * 16), k = idx / (NCT * 16);
        const int c = cb + k;
        if constexpr (kPrefC) {
          const bool ok = idx < RB_K * NCT * 16 && c < hi && j < ncol;
          const double v = gload<double>(Cm + (ok ? (size_t)c * cld + j : 0));
          cn[u] = ok ? v : 0.0;
        }
      }
    };
    if (lo < hi) {
      load_s(lo, sn);
      if constexpr (kPrefC) load_c(lo);
    }
    for (int cb = lo; cb < hi; cb += RB_K) {
      __syncthreads();
      // C rows cb .. cb+31 as three BF16 planes, transposed (scb[piece][column j][row k])
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int idx = threadIdx.x + u * RT_THREADS;
        if (idx >= RB_K * NCT * 16) continue;
        const int j = idx % (NCT * 16), k = idx / (NCT * 16);
        double v;
        if constexpr (kPrefC) {
          v = cn[u];
        } else {
          const int c = cb + k;
          v = (c < hi && j < ncol) ? Cm[(size_t)c * cld + j] : 0.0;
        }
        const unsigned short h0 = bf16_bits_rn((float)v);
        const double v1 = v - (double)bf16_to_float(h0);
        const unsigned short h1 = bf16_bits_rn((float)v1);
        const unsigned short h2 = bf16_bits_rn((float)(v1 - (double)bf16_to_float(h1)));
        scb[0][j][k] = h0;
        scb[1][j][k] = h1;
        scb[2][j][k] = h2;
      }
#pragma unroll
      for (int u = 0; u < RT_RT; ++u)
#pragma unroll
        for (int i = 0; i < 8; ++i) sv[u][i] = sn[u][i];
      __syncthreads();
      if (cb + RB_K < hi) {
        load_s(cb + RB_K, sn);
        if constexpr (kPrefC) load_c(cb + RB_K);
      }
      bf16x8 b0[RT_RT], b1[RT_RT], b2[RT_RT];
#pragma unroll
      for (int u = 0; u < RT_RT; ++u) {
        us8v p0, p1, p2;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float x = sv[u][i];
          const unsigned short h0 = bf16_bits_rn(x);
          const float x1 = x - bf16_to_float(h0);
          const unsigned short h1 = bf16_bits_rn(x1);
          p0[i] = h0;
          p1[i] = h1;
          p2[i] = bf16_bits_rn(x1 - bf16_to_float(h1));
        }
        b0[u] = __builtin_bit_cast(bf16x8, p0);
        b1[u] = __builtin_bit_cast(bf16x8, p1);
        b2[u] = __builtin_bit_cast(bf16x8, p2);
      }
#pragma unroll
      for (int t = 0; t < NCT; ++t) {
        if (t >= nct) continue;
        const int j = t * 16 + (lane & 15);
        const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&scb[0][j][8 * kl]);
        const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&scb[1][j][8 * kl]);
        const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(&scb[2][j][8 * kl]);
#pragma unroll
        for (int u = 0; u < RT_RT; ++u) {
          f4v s = acc[u][t];
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0[u], s, 0, 0, 0);
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1[u], s, 0, 0, 0);
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b2[u], s, 0, 0, 0);
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0[u], s, 0, 0, 0);
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1[u], s, 0, 0, 0);
          acc[u][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0[u], s, 0, 0, 0);
        }
      }
    }
    // store the output this segment completes: lane holds out[row rrow[u]][col 16 t + 4 kl + q]
    const int o = (A.nout > 1 && sg == 0) ? 1 : 0;
    float* out = reinterpret_cast<float*>(E.blk[A.out_blk[o]]);
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      if (t >= nct) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = t * 16 + 4 * kl + q;
        if (j >= ncol) continue;
#pragma unroll
        for (int u = 0; u < RT_RT; ++u) {
          if (rrow[u] >= nrows) continue;
          float* p = out + (size_t)j * E.ld + rrow[u];
          const double prev = A.beta[o] != 0.0 ? A.beta[o] * (double)*p : 0.0;
          *p = (float)(prev + A.alpha * (double)acc[u][t][q]);
        }
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

// one workgroup of RES_THREADS per column; each thread keeps four rows in flight
constexpr int RES_THREADS = 1024;

template <typename T>
__global__ void __launch_bounds__(RES_THREADS) k_residual(ResArgs A) {
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
  double s1[4] = {0.0, 0.0, 0.0, 0.0}, s2[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = threadIdx.x; r0 < E.N; r0 += 4 * RES_THREADS) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + u * RES_THREADS;
      if (r < E.N) {
        const double xv = double(x[r]);
        const double rv = double(hx[r]) - th * xv;
        s1[u] += rv * rv;
        s2[u] += E.v64[r] * xv * xv;
      }
    }
  }
  __shared__ double sh[16];
  const double t1 = block_sum((s1[0] + s1[1]) + (s1[2] + s1[3]), sh);
  const double t2 = block_sum((s2[0] + s2[1]) + (s2[2] + s2[3]), sh);
  if (threadIdx.x == 0) {
    vec[VS_RES * KP + i] = sqrt(t1);
    vec[VS_EKIN * KP + i] = fmax(th - t2, 0.05);
  }
}

// per element: active = max_{i<J} res_i > tol ; count of active elements; the
// Rayleigh-Ritz breakdowns (status 2) since the last check are added to count[2]
// and their flags cleared
__global__ void k_check(const ElemDev* elems, int n_elem, int* active, double tol, int* count,
                        double* maxres, int* iter_count, int* status) {
  __shared__ double sh[16];
  if (threadIdx.x == 0) {
    int brk = 0;
    for (int e = 0; e < n_elem; ++e)
      if (status[e] != 0) {
        ++brk;
        status[e] = 0;
      }
    count[2] += brk;
  }
  __syncthreads();
  for (int e = 0; e < n_elem; ++e) {
    const ElemDev& E = elems[e];
    const int KP = E.kmax3 + 2;
    const double* res = E.small + SmallLayout::vec(KP) + VS_RES * KP;
    double m = 0.0;
    int bad = 0;
    for (int i = threadIdx.x; i < E.J; i += blockDim.x) {
      const double r = res[i];
      bad |= !(r == r);          // fmax drops NaN: flag it separately
      m = fmax(m, r);
    }
    m = block_max(m, sh);
    if (__syncthreads_or(bad)) m = __builtin_nan("");
    if (threadIdx.x == 0) {
      if (active[e] && !(m <= tol)) {
      } else {
        active[e] = 0;
      }
      if (!(m == m)) active[e] = -1;   // NaN
      maxres[e] = m;
      if (iter_count && active[e] > 0) ++iter_count[e];
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
  long long ld;               // mode 0: > 0 caller leading dimension (element blocks ld * ncol apart)
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
  long long base, cstride = nrows;
  if (A.ld > 0) {
    base = A.elem_only >= 0 ? 0 : (long long)e * A.ld * ncol;
    cstride = A.ld;
  } else {
    base = (A.elem_only >= 0 || !A.off) ? 0 : A.off[e] * A.off_mult;
  }
  T* p = reinterpret_cast<T*>(A.ptr) + base + (size_t)j * cstride + r;
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

// Mixed refinement, per active element and column j < K: the residual
// r_j = hx_j - theta_j x_j, formed in FP64 and stored in FP32 (its rounding is relative
// to r, not to hx), and x_j rounded to FP32.
__global__ void __launch_bounds__(256) k_mixed_split(const ElemDev* elems, const int* active, int x_blk,
                                                     int hx_blk, int r_blk, int x32_blk) {
  const int e = blockIdx.z;
  const ElemDev& E = elems[e];
  if (active && !active[e]) return;
  const int j = blockIdx.y;
  if (j >= E.K) return;
  const int KP = E.kmax3 + 2;
  const double th = E.small[SmallLayout::vec(KP) + VS_THETA * KP + j];
  const double* X = reinterpret_cast<const double*>(E.blk[x_blk]) + (size_t)j * E.ld;
  const double* HX = reinterpret_cast<const double*>(E.blk[hx_blk]) + (size_t)j * E.ld;
  float* R = reinterpret_cast<float*>(E.blk[r_blk]) + (size_t)j * E.ld;
  float* X32 = reinterpret_cast<float*>(E.blk[x32_blk]) + (size_t)j * E.ld;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = blockIdx.x * 1024 + u * 256 + threadIdx.x;
    if (r >= E.N) break;
    const double x = X[r];
    R[r] = (float)(HX[r] - th * x);
    X32[r] = (float)x;
  }
}

// Mixed refinement: the projected matrices of [X W P] (G: overlap, A: H) from the FP32
// Grams of S' = [W P X32] (Gs = S'^T S') and T' = [HW HP R] (As = S'^T T', upper blocks):
//   G_XX = I and A_XX = Theta (X holds Ritz vectors),
//   G_QX = Gs_QX and A_QX = Q^T R + G_QX Theta for Q = W, P,
//   G_QQ', A_QQ' = Gs, As,
// both symmetric.  A_QX - theta_j G_QX e_j = Q^T r_j holds whatever the rounding of
// G_QX, so the FP32 Grams perturb the correction only in second order.
__global__ void __launch_bounds__(256) k_mixed_fix(const ElemDev* elems, const int* active, int nb) {
  const int e = blockIdx.x;
  const ElemDev& E = elems[e];
  if (active && !active[e]) return;
  const int K = E.K, n = nb * K;
  const int KP = E.kmax3 + 2;
  const double* Gs = E.small + SmallLayout::V(KP);
  const double* As = E.small + SmallLayout::U(KP);
  double* G = E.small + SmallLayout::G(KP);
  double* Am = E.small + SmallLayout::A(KP);
  const double* th = E.small + SmallLayout::vec(KP) + VS_THETA * KP;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    const int bi = i / K, bj = j / K;
    // [X W P] index -> [W P X] index
    const int oi = (bi == 0 ? nb - 1 : bi - 1) * K + (i - bi * K);
    const int oj = (bj == 0 ? nb - 1 : bj - 1) * K + (j - bj * K);
    double g, a;
    if (bi == 0 && bj == 0) {
      g = i == j ? 1.0 : 0.0;
      a = i == j ? th[i] : 0.0;
    } else if (bi == 0 || bj == 0) {
      // one index in X: read the (Q row, X column) entries, computed directly in As
      const int q = bi == 0 ? oj : oi, x = bi == 0 ? oi : oj;
      const int xi = bi == 0 ? i : j;
      g = Gs[(size_t)q * n + x];
      a = As[(size_t)q * n + x] + g * th[xi];
    } else {
      g = Gs[(size_t)oi * n + oj];
      a = As[(size_t)oi * n + oj];
    }
    G[(size_t)i * n + j] = g;
    Am[(size_t)i * n + j] = a;
  }
}

// Seeded Gaussian start: value (row r, column j) of element g = e + elem_base is a
// Box-Muller normal from two SplitMix64 outputs of the counter (seed, g, j, r), so
// the block does not depend on how the batch is split into element groups.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

template <typename T>
__global__ void __launch_bounds__(256) k_random_block(const ElemDev* elems, int blk, unsigned long long seed,
                                                       int elem_base) {
  const int e = blockIdx.z;
  const ElemDev& E = elems[e];
  const int j = blockIdx.y;
  if (j >= E.K) return;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= E.N) return;
  const unsigned long long key =
      splitmix64(seed ^ splitmix64(((unsigned long long)(e + elem_base) << 32) | (unsigned)j)) ^ (unsigned long long)r;
  const unsigned long long h1 = splitmix64(2 * key), h2 = splitmix64(2 * key + 1);
  // u1 in (0, 1], u2 in [0, 1)
  const double u1 = ((double)(h1 >> 11) + 1.0) * (1.0 / 9007199254740992.0);
  const double u2 = (double)(h2 >> 11) * (1.0 / 9007199254740992.0);
  const double v = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
  reinterpret_cast<T*>(E.blk[blk])[(size_t)j * E.ld + r] = T(v);
}

// J (all = 0) or J + g (all = 1) values per element from the small-vector slots
// into packed outputs
__global__ void k_extract(const ElemDev* elems, const long long* off, int slot0, double* out0,
                          int slot1, double* out1, int all) {
  const int e = blockIdx.x;
  const ElemDev& E = elems[e];
  const int KP = E.kmax3 + 2;
  const double* vec = E.small + SmallLayout::vec(KP);
  const int n = all ? E.K : E.J;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
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

static bool set_lds_limit(const void* fn, int bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
}

// Gram instantiations: FP64 blocks per wave {1,2,3,4,6,8,12} x staged values
// per thread {4,8,12} (up to 128, 256, 384 columns); BF16x3 {1,2,3,4,6,8} x {8,18}
// (up to 128, 288 columns), which keeps the FP32 staging and the FP64 accumulators
// in registers.
template <int MB>
static void gram_attrs() {
  set_lds_limit((const void*)k_gram<double, MB, 8>, GP_LDS_LIMIT);
  set_lds_limit((const void*)k_gram<double, MB, 16>, GP_LDS_LIMIT);
  set_lds_limit((const void*)k_gram<double, MB, 24>, GP_LDS_LIMIT);
  if constexpr (MB <= 8) {
    set_lds_limit((const void*)k_gram_bf16<MB, 8>, 96000);
    set_lds_limit((const void*)k_gram_bf16<MB, 18>, 96000);
  }
  if constexpr (MB <= 6) {
    set_lds_limit((const void*)k_gram32<MB, 8>, GP_LDS_LIMIT);
    set_lds_limit((const void*)k_gram32<MB, 16>, GP_LDS_LIMIT);
    set_lds_limit((const void*)k_gram32<MB, 24>, GP_LDS_LIMIT);
  }
}

template <int MB>
static void launch_gram_mb(int prec, int pf, dim3 g, size_t lds, hipStream_t s, const GramArgs& ga, bool bf16) {
  if (prec != DG_FP64 && !bf16) {
    if constexpr (MB <= 6) {
      if (pf <= 8) hipLaunchKernelGGL((k_gram32<MB, 8>), g, dim3(GP_THREADS), lds, s, ga);
      else if (pf <= 16) hipLaunchKernelGGL((k_gram32<MB, 16>), g, dim3(GP_THREADS), lds, s, ga);
      else hipLaunchKernelGGL((k_gram32<MB, 24>), g, dim3(GP_THREADS), lds, s, ga);
    }
    return;
  }
  if (prec == DG_FP64) {
    if (pf <= 8) hipLaunchKernelGGL((k_gram<double, MB, 8>), g, dim3(GP_THREADS), lds, s, ga);
    else if (pf <= 16) hipLaunchKernelGGL((k_gram<double, MB, 16>), g, dim3(GP_THREADS), lds, s, ga);
    else hipLaunchKernelGGL((k_gram<double, MB, 24>), g, dim3(GP_THREADS), lds, s, ga);
  } else if constexpr (MB <= 8) {
    if (pf <= 8) hipLaunchKernelGGL((k_gram_bf16<MB, 8>), g, dim3(GP_THREADS), lds, s, ga);
    else hipLaunchKernelGGL((k_gram_bf16<MB, 18>), g, dim3(GP_THREADS), lds, s, ga);
  }
}

// dynamic-LDS limits of every kernel variant, set once before any launch (and so
// never from inside a stream capture)
void init_kernel_attributes() {
  static const bool done = [] {
    gram_attrs<1>();
    gram_attrs<2>();
    gram_attrs<3>();
    gram_attrs<4>();
    gram_attrs<6>();
    gram_attrs<8>();
    gram_attrs<12>();
    set_lds_limit((const void*)k_rr_lds<true>, kRRLdsBytes);
    return true;
  }();
  (void)done;
}

// pair: also S^T S (to out_off_ss) from the same staging of [S | T]
// Tile side for a Gram launch: the tb that stages the fewest columns in total
// (over the tiles of every element shape in the launch) while each tile's blocks
// fit 8 waves x max_blocks and its staged columns max_cols.
struct GramPlan {
  int tb = 1, maxblk = 0, maxnc = 0, ntiles = 0;
};

static GramPlan plan_gram_tiles(const std::vector<int>& bis, int bj_max, int sym, int same, int pair,
                                int max_blocks, int max_cols) {
  int bi_max = 0;
  for (int b : bis) bi_max = std::max(bi_max, b);
  GramPlan best;
  long long best_staged = -1;
  for (int tb = std::max(bi_max, bj_max); tb >= 1; --tb) {
    GramPlan pl;
    pl.tb = tb;
    long long staged = 0;
    for (int bi : bis) {
      const int bj = sym ? bi : bj_max;
      const int nt = gram_ntiles(bi, bj, tb, sym);
      if (bi == bi_max) pl.ntiles = nt;
      for (int t = 0; t < nt; ++t) {
        const GramTile g = gram_tile(t, bi, bj, tb, sym, same, pair);
        pl.maxblk = std::max(pl.maxblk, g.nloc * (pair ? 2 : 1));
        pl.maxnc = std::max(pl.maxnc, g.ncA + g.ncB + g.ncC);
        if (bi == bi_max) staged += g.ncA + g.ncB + g.ncC;
      }
    }
    if (pl.maxblk > 8 * max_blocks || pl.maxnc > max_cols) continue;
    if (best_staged < 0 || staged < best_staged) {
      best = pl;
      best_staged = staged;
    }
  }
  return best;
}

static int gram_impl(Ctx& c, int prec, const ColSet& S, int kS, const ColSet& T, int kT,
                     long long out_off, const int* active, int rows_e, int sym, bool pair = false,
                     long long out_off_ss = 0) {
  int ks, kt, maxN, maxE;
  max_dims(c, kS, &ks, &maxN, &maxE);
  max_dims(c, kT, &kt, &maxN, &maxE);
  const int maxni = S.nb * ks, maxnj = T.nb * kt;
  const int rows = rows_e ? maxE : maxN;
  const bool same = S.nb == T.nb && kS == kT &&
                    std::equal(S.blk, S.blk + S.nb, T.blk);
  if (sym && maxni != maxnj) { set_error("symmetric Gram of a non-square shape"); return DG_ERR_ARG; }
  const long long part_sq = (long long)c.gram_part_ld * c.gram_part_ld;
  if (pair) {
    // both products from one staging of S (symmetric, T != S) when the partial area
    // holds both sets of partial sums; else two separate Grams
    const bool fits = sym && !same && c.gram_part_stride >= 2 * part_sq;
    if (!fits) {
      if (int st = gram_impl(c, prec, S, kS, S, kS, out_off_ss, active, rows_e, sym)) return st;
      return gram_impl(c, prec, S, kS, T, kT, out_off, active, rows_e, sym);
    }
  }
  // block-row counts of the element shapes in this launch
  std::vector<int> bis;
  for (int e = 0; e < c.n_elem; ++e) {
    const int ke = kS > 0 ? kS : (kS == 0 ? c.K[e] : c.J[e]);
    const int b = (S.nb * ke + 15) / 16;
    if (std::find(bis.begin(), bis.end(), b) == bis.end()) bis.push_back(b);
  }
  const int bj_max = (maxnj + 15) / 16;
  // FP64: up to 12 blocks per wave (16 spill registers) and 384 staged columns; BF16x3: 8 and 288
  // FP64 and FP32 (FP32 matrix cores): at most 6 blocks per wave and 384 staged columns;
  // BF16x3 (DG_BF16=1): 6 blocks and 128 columns
  const bool bf16 = prec != DG_FP64 && c.bf16;
  const int cap_blocks = 6;
  const int cap_cols = prec == DG_FP64 ? GP_MAXCOL : (bf16 ? 128 : G3_MAXCOL);
  const GramPlan pl = plan_gram_tiles(bis, bj_max, sym, same ? 1 : 0, pair ? 1 : 0, cap_blocks, cap_cols);
  if (pl.maxblk == 0) {
    set_error("Gram: no tile fits the per-workgroup limits");
    return DG_ERR_SHAPE;
  }
  static const int kMaxbList[] = {1, 2, 3, 4, 6, 8, 12};
  int maxb = cap_blocks;
  for (int m : kMaxbList)
    if (m <= cap_blocks && 8 * m >= pl.maxblk) {
      maxb = m;
      break;
    }
  // staged values per thread: FP64 GP_THREADS / GP_R columns per pass; FP32 and BF16: 16 per pass
  const int pf = prec == DG_FP64 ? (pl.maxnc + GP_THREADS / GP_R - 1) / (GP_THREADS / GP_R) : (pl.maxnc + 15) / 16;
  const int groups = pl.ntiles;
  // row-range split: row ranges of about 8192 rows of the largest element, and at least
  // 2048 workgroups over the launch (long single ranges leave the launch to a tail of
  // the largest elements), at least 256 rows each; the autotuner below may replace it
  // by half or twice that for this Gram shape (the pair keeps two sets of partials)
  const int split_cap = std::max(1, std::min(pair ? (int)(c.gram_part_stride / (2 * part_sq)) : c.gram_max_split,
                                             rows / 256));
  int nsplit = std::max((rows + 8191) / 8192, (2048 + groups * c.n_elem - 1) / (groups * c.n_elem));
  nsplit = std::max(1, std::min(split_cap, nsplit));
  const long long key =
      ((((((long long)prec * 1024 + maxni) * 1024 + maxnj) * 2 + sym) * 2 + (same ? 1 : 0)) * 2 + rows_e) * 2 +
      (pair ? 1 : 0);
  auto tuned = c.gram_split_table.find(key);
  if (tuned != c.gram_split_table.end()) nsplit = tuned->second;
  GramArgs ga{c.elems_dev, active, S, T, kS, kT, nsplit, rows_e, sym, same ? 1 : 0, pl.tb, pl.ntiles,
              c.n_elem, c.gram_part, c.gram_part_stride, c.gram_part_ld, pair ? 1 : 0, 0};
  // algorithmic flops: 2 r n_i n_j per product, n (n + 1) r for a symmetric n x n result
  double flops = 0.0;
  for (int e = 0; e < c.n_elem; ++e) {
    if (active && !c.active_host.empty() && !c.active_host[e]) continue;
    const int ke = kS > 0 ? kS : (kS == 0 ? c.K[e] : c.J[e]);
    const int kt = kT > 0 ? kT : (kT == 0 ? c.K[e] : c.J[e]);
    const double r = rows_e ? (double)c.en[0][e] * c.en[1][e] * c.en[2][e] : (double)c.N[e];
    const double ni = S.nb * ke, nj = T.nb * kt;
    flops += (sym ? r * ni * (ni + 1.0) : 2.0 * r * ni * nj) * (pair ? 2.0 : 1.0);
  }
  const size_t lds = prec == DG_FP64 ? (size_t)GP_RP * pl.maxnc * sizeof(double) + (size_t)pl.maxnc * sizeof(void*)
                     : !bf16       ? (size_t)G3_RP * pl.maxnc * sizeof(float) + (size_t)pl.maxnc * sizeof(void*)
                                   : (size_t)3 * pl.maxnc * GB_PITCH * 2 + (size_t)pl.maxnc * sizeof(void*);
  auto launch = [&](int ns) -> int {
    ga.nsplit = ns;
    ga.part_pair = ns * part_sq;
    // 1D grid: tiles x row ranges (split, element), the row ranges padded to a multiple of 8
    const long long n_rr8 = ((long long)ns * c.n_elem + 7) / 8 * 8;
    dim3 g1((unsigned)(groups * n_rr8));
    switch (maxb) {
      case 1: launch_gram_mb<1>(prec, pf, g1, lds, c.stream, ga, bf16); break;
      case 2: launch_gram_mb<2>(prec, pf, g1, lds, c.stream, ga, bf16); break;
      case 3: launch_gram_mb<3>(prec, pf, g1, lds, c.stream, ga, bf16); break;
      case 4: launch_gram_mb<4>(prec, pf, g1, lds, c.stream, ga, bf16); break;
      case 6: launch_gram_mb<6>(prec, pf, g1, lds, c.stream, ga, bf16); break;
      case 8: launch_gram_mb<8>(prec, pf, g1, lds, c.stream, ga, bf16); break;
      case 12: launch_gram_mb<12>(prec, pf, g1, lds, c.stream, ga, bf16); break;
      default:
        set_error("Gram: unsupported block count");
        return DG_ERR_SHAPE;
    }
    return DG_OK;
  };
  if (tuned == c.gram_split_table.end() && c.autotune && !c.capturing) {
    // autotuner: time the candidate splits on this launch's data (the best of three
    // launches each, since other element groups may share the GPU meanwhile) and keep
    // the heuristic split unless another is at least 3 % faster
    const int cand[3] = {nsplit, std::max(1, nsplit / 2), std::min(split_cap, nsplit * 2)};
    float best = 1e30f, base = 1e30f;
    int best_ns = nsplit;
    struct Events {   // destroyed on every return path
      hipEvent_t e[2] = {nullptr, nullptr};
      ~Events() {
        for (hipEvent_t x : e)
          if (x) (void)hipEventDestroy(x);
      }
    } evs;
    hipEvent_t* ev = evs.e;
    DG_HIP(hipEventCreate(&ev[0]));
    DG_HIP(hipEventCreate(&ev[1]));
    for (int ci = 0; ci < 3; ++ci) {
      if (ci > 0 && cand[ci] == nsplit) continue;
      float ms_min = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        DG_HIP(hipEventRecord(ev[0], c.stream));
        if (int st = launch(cand[ci])) return st;
        DG_HIP(hipEventRecord(ev[1], c.stream));
        DG_HIP(hipEventSynchronize(ev[1]));
        float ms = 0.f;
        DG_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        ms_min = std::min(ms_min, ms);
      }
      if (ci == 0) base = ms_min;
      if (ms_min < best && (ci == 0 || ms_min < 0.97f * base)) {
        best = ms_min;
        best_ns = cand[ci];
      }
    }
    c.gram_split_table[key] = best_ns;
    nsplit = best_ns;
    if (c.log_level > 0)
      fprintf(stderr, "[dg] gram autotune %dx%d sym=%d prec=%d pair=%d tile=%d (%d tiles, %d blocks/wg): split %d "
              "(%.3f ms)\n", maxni, maxnj, sym, prec, pair ? 1 : 0, pl.tb, groups, pl.maxblk, best_ns, best);
  }
  TimedScope ts(c, TC_GRAM, flops);
  if (int st = launch(nsplit)) return st;
  GramReduceArgs ra{c.elems_dev, active, sym, S.nb, T.nb, kS, kT, nsplit, c.gram_part,
                    c.gram_part_stride, c.gram_part_ld, out_off, 0};
  dim3 g2((maxni * maxnj + 255) / 256, c.n_elem);
  hipLaunchKernelGGL(k_gram_reduce, g2, dim3(256), 0, c.stream, ra);
  if (pair) {
    GramReduceArgs rs{c.elems_dev, active, sym, S.nb, S.nb, kS, kS, nsplit, c.gram_part + nsplit * part_sq,
                      c.gram_part_stride, c.gram_part_ld, out_off_ss, 0};
    hipLaunchKernelGGL(k_gram_reduce, g2, dim3(256), 0, c.stream, rs);
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_gram(Ctx& c, int prec, const ColSet& S, int kS, const ColSet& T, int kT,
                long long out_off, const int* active, int sym) {
  return gram_impl(c, prec, S, kS, T, kT, out_off, active, 0, sym);
}

int launch_gram_rows(Ctx& c, int prec, const ColSet& S, int kS, const ColSet& T, int kT,
                     long long out_off, int rows_e, int sym) {
  return gram_impl(c, prec, S, kS, T, kT, out_off, nullptr, rows_e, sym);
}

int launch_gram_pair(Ctx& c, int prec, const ColSet& S, int kS, const ColSet& T, int kT, long long out_off_st,
                     long long out_off_ss, const int* active) {
  return gram_impl(c, prec, S, kS, T, kT, out_off_st, active, 0, 1, true, out_off_ss);
}

int launch_rr(Ctx& c, int nb, int kfix, int nkeep, int mode, const int* active) {
  // algorithmic flop estimate: Cholesky + inverse (n^3/3 each), two n^3 products,
  // tridiagonalisation (4n^3/3), back-transformation and coefficients (4 n^2 k)
  double flops = 0.0;
  int npmax = 0;
  size_t need = 0;   // bytes of the working region: matrix, then eigenvectors + reflectors
  for (int e = 0; e < c.n_elem; ++e) {
    const int n = mode == RR_GEN ? nb * c.K[e] : (kfix > 0 ? kfix : (kfix == 0 ? c.K[e] : c.J[e]));
    const int npe = n + (n & 1);
    const int nk = nkeep > 0 ? nkeep : (nkeep == 0 ? c.K[e] : c.J[e]);
    const int nw = mode == RR_SVD ? n : std::min(nk, n);
    npmax = std::max(npmax, npe);
    need = std::max({need, (size_t)(nw * npe + n * (n - 1) / 2) * sizeof(double),
                     (size_t)npe * npe * sizeof(double), (size_t)npe * 41});
    if (active && !c.active_host.empty() && !c.active_host[e]) continue;
    flops += (mode == RR_GEN ? 2.0 / 3.0 + 2.0 : 0.0) * (double)n * n * n + 4.0 / 3.0 * (double)n * n * n +
             4.0 * (double)n * n * nk;
  }
  if (npmax > kTriMax) {
    set_error("projected problem of order " + std::to_string(npmax) + " above the limit " +
              std::to_string(kTriMax));
    return DG_ERR_SHAPE;
  }
  // the working region lives in LDS when the orders allow it, else in the element's
  // slice of the Gram partial-sum area (free between the Gram reduction and the rotation)
  const bool in_lds = npmax <= kRRLdsOrder && need <= (size_t)kRRLdsBytes;
  if (!in_lds && need > (size_t)c.gram_part_stride * sizeof(double)) {
    set_error("Rayleigh-Ritz work region of " + std::to_string(need) + " bytes above the partial-sum slice");
    return DG_ERR_SHAPE;
  }
  RRArgs a{c.elems_dev, active, nb, kfix, nkeep, mode, c.dev_status,
           c.log_level >= 2 ? c.dev_phase : nullptr, c.gram_part, c.gram_part_stride,
           c.rr_pivot_tol, c.rr_drop_tol, c.log_level >= 3 ? c.dev_minpiv : nullptr, c.rr_ortol,
           in_lds ? (int)need : 0, mode == RR_GEN ? c.dev_hpflag : nullptr, c.hp_tol};
  TimedScope ts(c, TC_RR, flops);
  if (in_lds) {
    hipLaunchKernelGGL(k_rr_lds<true>, dim3(c.n_elem), dim3(kRRThreads), need, c.stream, a);
  } else {
    hipLaunchKernelGGL(k_rr_lds<false>, dim3(c.n_elem), dim3(kRRThreadsL2), 0, c.stream, a);
  }
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
  // output column tiles: 3 (up to 48 columns) or 6 (up to 96); FP32 blocks on FP32 matrix
  // cores (BF16 matrix cores with DG_BF16=1)
  const bool k3 = k <= 48;
  if (prec == DG_FP64) {
    if (k3) hipLaunchKernelGGL((k_rotate<double, 3>), g, dim3(RT_THREADS), 0, c.stream, a);
    else hipLaunchKernelGGL((k_rotate<double, 6>), g, dim3(RT_THREADS), 0, c.stream, a);
  } else if (!c.bf16) {
    if (k3) hipLaunchKernelGGL((k_rotate32<3>), g, dim3(RT_THREADS), 0, c.stream, a);
    else hipLaunchKernelGGL((k_rotate32<6>), g, dim3(RT_THREADS), 0, c.stream, a);
  } else {
    if (k3) hipLaunchKernelGGL((k_rotate_bf16<3>), g, dim3(RT_THREADS), 0, c.stream, a);
    else hipLaunchKernelGGL((k_rotate_bf16<6>), g, dim3(RT_THREADS), 0, c.stream, a);
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_residual(Ctx& c, int prec, int x_blk, int hx_blk, int ncol, const int* active) {
  int maxk, maxN, maxE;
  max_dims(c, ncol, &maxk, &maxN, &maxE);
  ResArgs a{c.elems_dev, active, x_blk, hx_blk, ncol, 0};
  dim3 g(maxk, c.n_elem);
  TimedScope ts(c, TC_OTHER);
  if (prec == DG_FP64) hipLaunchKernelGGL(k_residual<double>, g, dim3(RES_THREADS), 0, c.stream, a);
  else hipLaunchKernelGGL(k_residual<float>, g, dim3(RES_THREADS), 0, c.stream, a);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_check(Ctx& c, int* active, double tol) {
  hipLaunchKernelGGL(k_check, dim3(1), dim3(256), 0, c.stream, c.elems_dev, c.n_elem, active, tol,
                     c.dev_count, c.dev_maxres, c.dev_iters, c.dev_status);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_copy_ext(Ctx& c, int prec, int blk, const void* ptr, int elem, int ncol, int to_packed,
                    long long ld) {
  int maxk, maxN, maxE;
  max_dims(c, ncol, &maxk, &maxN, &maxE);
  CopyArgs a{c.elems_dev, blk, 0, const_cast<void*>(ptr), c.dev_off_grid, ncol, elem, ncol, to_packed, 0, ld};
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
    CopyArgs a{c.elems_dev, blk, 0, const_cast<double*>(ptr), off, 1, -1, ncol, 1, 0, 0};
    hipLaunchKernelGGL(k_copy<double>, g, dim3(256), 0, c.stream, a);
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_gather_e(Ctx& c, int src_blk, int dst_blk) {
  int maxk, maxN, maxE;
  max_dims(c, -1, &maxk, &maxN, &maxE);
  CopyArgs a{c.elems_dev, src_blk, dst_blk, nullptr, nullptr, 0, -1, -1, 0, 2, 0};
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

int launch_random_block(Ctx& c, int prec, int blk, unsigned long long seed) {
  int maxk, maxN, maxE;
  max_dims(c, 0, &maxk, &maxN, &maxE);
  dim3 g((maxN + 255) / 256, maxk, c.n_elem);
  if (prec == DG_FP64)
    hipLaunchKernelGGL(k_random_block<double>, g, dim3(256), 0, c.stream, c.elems_dev, blk, seed, c.elem_base);
  else
    hipLaunchKernelGGL(k_random_block<float>, g, dim3(256), 0, c.stream, c.elems_dev, blk, seed, c.elem_base);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_mixed_split(Ctx& c, int x_blk, int hx_blk, int r_blk, int x32_blk, const int* active) {
  int maxk, maxN, maxE;
  max_dims(c, 0, &maxk, &maxN, &maxE);
  dim3 g((maxN + 1023) / 1024, maxk, c.n_elem);
  TimedScope ts(c, TC_OTHER);
  hipLaunchKernelGGL(k_mixed_split, g, dim3(256), 0, c.stream, c.elems_dev, active, x_blk, hx_blk, r_blk, x32_blk);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_mixed_fix(Ctx& c, int nb, const int* active) {
  TimedScope ts(c, TC_OTHER);
  hipLaunchKernelGGL(k_mixed_fix, dim3(c.n_elem), dim3(256), 0, c.stream, c.elems_dev, active, nb);
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
                     (int)VS_THETA, eig, (int)VS_RES, resid, 0);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_extract_kall(Ctx& c, double* theta, double* resid) {
  hipLaunchKernelGGL(k_extract, dim3(c.n_elem), dim3(128), 0, c.stream, c.elems_dev, c.dev_off_kall,
                     (int)VS_THETA, theta, (int)VS_RES, resid, 1);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_extract_theta(Ctx& c, double* out) {
  hipLaunchKernelGGL(k_extract, dim3(c.n_elem), dim3(128), 0, c.stream, c.elems_dev, c.dev_off_eig,
                     (int)VS_THETA, out, (int)VS_THETA, (double*)nullptr, 0);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace dg
