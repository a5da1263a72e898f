// H*psi on gfx950: kinetic term by line FFTs, local potential, nonlocal projectors;
// and the Teter preconditioner by a 3D FFT built from the same line FFTs.
//
// Eq. (1): H = -1/2 Laplacian + V_eff + sum gamma |b><b|, plane waves on Q_k.
// The kinetic symbol |G|^2/2 = gx(kx) + gy(ky) + gz(kz) separates, so
//   T x = Tx x + Ty x + Tz x,  T_axis = F_axis^{-1} diag(g_axis) F_axis,
// exactly (up to rounding) the 3D FFT definition.  Two passes over HBM:
//   pass 1 (per z-plane, LDS):   y1 = Tx x + Ty x + V x
//   pass 2 (per z-column, regs): y  = y1 + Tz x
// then the projector term y += B diag(gamma) B^T x (overlap before, apply after).
//
// The Teter preconditioner (Eq. (3)) multiplies the full 3D spectrum by a
// non-separable K(|G|^2 / 2E); it uses three passes: 2D forward per plane,
// z forward * K * z inverse per column, 2D inverse per plane, in place in W.
//
// Real vectors are processed in pairs (columns 2p, 2p+1) packed as one complex
// line; an odd last column pairs with zero.
#include "dg_internal.h"
#include "fft_line.h"
#include "wave_ops.h"

#include <algorithm>

namespace dg {

template <typename T>
__device__ __forceinline__ const T* vptr(const ElemDev& E);
template <>
__device__ __forceinline__ const double* vptr<double>(const ElemDev& E) { return E.v64; }
template <>
__device__ __forceinline__ const float* vptr<float>(const ElemDev& E) { return E.v32; }

__device__ __forceinline__ int signed_freq(int k, int n) { return (2 * k < n) ? k : k - n; }
// column-count code of the H*psi-family kernels for "the element's J" (<= 0 otherwise: K)
constexpr int kNcolsJ = -2;

// frequency of a first derivative: the Nyquist mode's odd derivative vanishes on the grid
__device__ __forceinline__ int deriv_freq(int k, int n) { return (2 * k == n) ? 0 : signed_freq(k, n); }

// 1/q from the hardware reciprocal (FP64: two Newton steps, a few ulps; FP32: one ulp)
__device__ __forceinline__ double fast_recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double t = fma(-q, r, 1.0);
  r = fma(r, t, r);
  t = fma(-q, r, 1.0);
  return fma(r, t, r);
}
__device__ __forceinline__ float fast_recip(float q) { return __builtin_amdgcn_rcpf(q); }

// HPSI: y = (T_x + T_y + V) x; TFWD/TINV: Teter passes; DX/DY: y = d/dx x, d/dy x
enum PlaneMode { PM_HPSI = 0, PM_TFWD = 1, PM_TINV = 2, PM_DX = 3, PM_DY = 4 };

struct PlaneArgs {
  const ElemDev* elems;
  const int* elem_list;   // shape class members
  const int* active;      // per element flag (nullptr = all)
  int in_blk, out_blk, aux_blk;   // HPSI: x -> y ; TFWD: x=X, aux=HX, out=W ; TINV: out=W (in place)
  int ncols;              // columns per element (<= 0: E.K)
  const double* theta_base;  // TFWD: per-element theta at small + vec(VS_THETA)
  int k3;                 // small-layout K3 (for theta lookup)
  ExtBufs ext;            // caller buffers for block ids kExtX / kExtY
  int r_given = 0;        // TFWD: aux already holds r = HX - X theta (in_blk is not read)
};

// Columns 2p and 2p+1 of a block (the second may be absent).
template <typename T>
struct PairCols {
  T* a;
  T* b;
};

// First value and leading dimension of element e's columns in block blk, or in a
// caller buffer (blk = kExtX / kExtY)
template <typename T>
__device__ __forceinline__ T* block_base(const ElemDev& E, int e, int blk, const ExtBufs& X, long long& ld) {
  if (blk >= 0) {
    ld = E.ld;
    return reinterpret_cast<T*>(E.blk[blk]);
  }
  const long long l = blk == kExtX ? X.ldx : X.ldy;
  T* p = reinterpret_cast<T*>(blk == kExtX ? const_cast<void*>(X.x) : X.y);
  ld = l > 0 ? l : E.N;
  if (X.elem_only >= 0) return p;
  return p + (l > 0 ? (long long)e * l * X.nvec : X.off_grid[e] * X.nvec);
}

template <typename T>
__device__ __forceinline__ PairCols<T> pair_cols(const ElemDev& E, int e, int blk, int pair, int ncols,
                                                 const ExtBufs& X) {
  long long ld;
  T* base = block_base<T>(E, e, blk, X, ld);
  PairCols<T> pc;
  pc.a = base + (size_t)(2 * pair) * ld;
  pc.b = (2 * pair + 1 < ncols) ? pc.a + ld : nullptr;
  return pc;
}

// ---------------------------------------------------------------------------
// plane pass: x-lines and y-lines of one z-plane, several planes per block
// ---------------------------------------------------------------------------
template <typename T, int NX, int NY, int TL, int MODE>
__global__ void __launch_bounds__(512) k_plane(PlaneArgs A) {
  constexpr int NL = NX > NY ? NX : NY;
  constexpr int TPP = NL * TL;
  constexpr int PPW = (256 / TPP) > 0 ? 256 / TPP : 1;
  // LDS row pitch: with 8 lanes per line, NX + 2 (complex) makes the column reads of
  // a 16-lane group (2 lines x 8 lanes) fall in distinct banks
  constexpr int PITCH = NX + (TL == 8 ? 2 : 1);
  constexpr int MX = NX / TL, MY = NY / TL;
  using FX = LineFFT<T, NX, TL>;
  using FY = LineFFT<T, NY, TL>;
  __shared__ cplx<T> sm[PPW * NY * PITCH];

  const int e = A.elem_list[blockIdx.z];
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int ncols = A.ncols > 0 ? A.ncols : (A.ncols == kNcolsJ ? E.J : E.K);
  const int pair = blockIdx.y;
  if (2 * pair >= ncols) return;
  const int slot = threadIdx.x / TPP;
  const int lt = threadIdx.x % TPP;
  const int line = lt / TL;
  const int t = lt % TL;
  const int z = blockIdx.x * PPW + slot;
  const bool zok = (slot < PPW) && (z < E.nz);
  constexpr int NXY = NX * NY;
  const size_t zoff = (size_t)z * NXY;
  cplx<T>* P = sm + (slot < PPW ? slot : 0) * NY * PITCH;

  // ---- load the plane (pair) into LDS
  if constexpr (MODE == PM_HPSI || MODE == PM_TINV || MODE == PM_DX || MODE == PM_DY) {
    const int blk = (MODE == PM_TINV) ? A.out_blk : A.in_blk;
    PairCols<T> in = pair_cols<T>(E, e, blk, pair, MODE == PM_TINV ? 2 * pair + 2 : ncols, A.ext);
    if (zok) {
      for (int i = lt; i < NXY; i += TPP) {
        T re = in.a[zoff + i];
        T im = in.b ? in.b[zoff + i] : T(0);
        P[(i / NX) * PITCH + (i % NX)] = {re, im};
      }
    }
  } else {  // PM_TFWD: r = HX - theta X
    PairCols<T> xx = pair_cols<T>(E, e, A.in_blk, pair, ncols, A.ext);
    PairCols<T> hx = pair_cols<T>(E, e, A.aux_blk, pair, ncols, A.ext);
    const int KP = E.kmax3 + 2;
    const double* th = E.small + SmallLayout::vec(KP) + VS_THETA * KP;
    const T ta = T(th[2 * pair]);
    const T tb = xx.b ? T(th[2 * pair + 1]) : T(0);
    if (zok && A.r_given) {
      for (int i = lt; i < NXY; i += TPP) {
        T re = hx.a[zoff + i];
        T im = hx.b ? hx.b[zoff + i] : T(0);
        P[(i / NX) * PITCH + (i % NX)] = {re, im};
      }
    } else if (zok) {
      for (int i = lt; i < NXY; i += TPP) {
        T re = hx.a[zoff + i] - ta * xx.a[zoff + i];
        T im = xx.b ? (hx.b[zoff + i] - tb * xx.b[zoff + i]) : T(0);
        P[(i / NX) * PITCH + (i % NX)] = {re, im};
      }
    }
  }
  __syncthreads();

  if constexpr (MODE == PM_HPSI) {
    const T* V = vptr<T>(E);
    const T gys = T(E.ky / NY), gxs = T(E.kx / NX);
    cplx<T> acc[MY];
    // y-lines (line = x): Ty x + V x
    if (zok && line < NX) {
      cplx<T> v[MY];
      sfor<0, MY>([&](auto i) {
        const int y = t + TL * CV(i);
        v[CV(i)] = P[y * PITCH + line];
        const T vv = V[zoff + y * NX + line];
        acc[CV(i)] = {vv * v[CV(i)].re, vv * v[CV(i)].im};
      });
      FY::forward(v, t);
      sfor<0, MY>([&](auto i) {
        const int f = signed_freq(FY::freq(CV(i), t), NY);
        const T g = gys * T(f * f);
        v[CV(i)].re *= g;
        v[CV(i)].im *= g;
      });
      FY::inverse(v, t);
      sfor<0, MY>([&](auto i) { acc[CV(i)] = cadd(acc[CV(i)], v[CV(i)]); });
    }
    // x-lines (line = y): Tx x
    cplx<T> w[MX];
    const bool xl = zok && line < NY;
    if (xl) {
      sfor<0, MX>([&](auto i) { w[CV(i)] = P[line * PITCH + t + TL * CV(i)]; });
      FX::forward(w, t);
      sfor<0, MX>([&](auto i) {
        const int f = signed_freq(FX::freq(CV(i), t), NX);
        const T g = gxs * T(f * f);
        w[CV(i)].re *= g;
        w[CV(i)].im *= g;
      });
      FX::inverse(w, t);
    }
    __syncthreads();
    if (xl) sfor<0, MX>([&](auto i) { P[line * PITCH + t + TL * CV(i)] = w[CV(i)]; });
    __syncthreads();
    if (zok && line < NX) {
      PairCols<T> out = pair_cols<T>(E, e, A.out_blk, pair, ncols, A.ext);
      sfor<0, MY>([&](auto i) {
        const int y = t + TL * CV(i);
        cplx<T> r = cadd(acc[CV(i)], P[y * PITCH + line]);
        out.a[zoff + y * NX + line] = r.re;
        if (out.b) out.b[zoff + y * NX + line] = r.im;
      });
    }
  } else if constexpr (MODE == PM_DX) {
    // d/dx along the rows: multiply the spectrum by i 2 pi f / L_x (normalised by 1/NX)
    const T g = T(sqrt(2.0 * E.kx) / NX);
    if (zok && line < NY) {
      cplx<T> w[MX];
      sfor<0, MX>([&](auto i) { w[CV(i)] = P[line * PITCH + t + TL * CV(i)]; });
      FX::forward(w, t);
      sfor<0, MX>([&](auto i) {
        const T m = g * T(deriv_freq(FX::freq(CV(i), t), NX));
        w[CV(i)] = {-m * w[CV(i)].im, m * w[CV(i)].re};
      });
      FX::inverse(w, t);
      PairCols<T> out = pair_cols<T>(E, e, A.out_blk, pair, ncols, A.ext);
      sfor<0, MX>([&](auto i) {
        const int x = t + TL * CV(i);
        out.a[zoff + line * NX + x] = w[CV(i)].re;
        if (out.b) out.b[zoff + line * NX + x] = w[CV(i)].im;
      });
    }
  } else if constexpr (MODE == PM_DY) {
    // d/dy along the columns
    const T g = T(sqrt(2.0 * E.ky) / NY);
    if (zok && line < NX) {
      cplx<T> v[MY];
      sfor<0, MY>([&](auto i) { v[CV(i)] = P[(t + TL * CV(i)) * PITCH + line]; });
      FY::forward(v, t);
      sfor<0, MY>([&](auto i) {
        const T m = g * T(deriv_freq(FY::freq(CV(i), t), NY));
        v[CV(i)] = {-m * v[CV(i)].im, m * v[CV(i)].re};
      });
      FY::inverse(v, t);
      PairCols<T> out = pair_cols<T>(E, e, A.out_blk, pair, ncols, A.ext);
      sfor<0, MY>([&](auto i) {
        const int y = t + TL * CV(i);
        out.a[zoff + y * NX + line] = v[CV(i)].re;
        if (out.b) out.b[zoff + y * NX + line] = v[CV(i)].im;
      });
    }
  } else if constexpr (MODE == PM_TFWD) {
    // forward along x (rows), back to LDS at frequency positions, then along y
    cplx<T> w[MX];
    const bool xl = zok && line < NY;
    if (xl) {
      sfor<0, MX>([&](auto i) { w[CV(i)] = P[line * PITCH + t + TL * CV(i)]; });
      FX::forward(w, t);
    }
    __syncthreads();
    if (xl) sfor<0, MX>([&](auto i) { P[line * PITCH + FX::freq(CV(i), t)] = w[CV(i)]; });
    __syncthreads();
    if (zok && line < NX) {
      cplx<T> v[MY];
      sfor<0, MY>([&](auto i) { v[CV(i)] = P[(t + TL * CV(i)) * PITCH + line]; });
      FY::forward(v, t);
      PairCols<T> out = pair_cols<T>(E, e, A.out_blk, pair, 2 * pair + 2, A.ext);
      sfor<0, MY>([&](auto i) {
        const int ky = FY::freq(CV(i), t);
        out.a[zoff + ky * NX + line] = v[CV(i)].re;
        out.b[zoff + ky * NX + line] = v[CV(i)].im;
      });
    }
  } else {  // PM_TINV: inverse along y (columns), then x (rows); real pair out
    const bool yl = zok && line < NX;
    cplx<T> v[MY];
    if (yl) {
      // LDS holds [ky][kx]; register i of lane t takes frequency FY::freq(i, t)
      sfor<0, MY>([&](auto i) { v[CV(i)] = P[FY::freq(CV(i), t) * PITCH + line]; });
      FY::inverse(v, t);
    }
    __syncthreads();
    // after the inverse, register i of lane t is grid row y = t + TL * i
    if (yl) sfor<0, MY>([&](auto i) { P[(t + TL * CV(i)) * PITCH + line] = v[CV(i)]; });
    __syncthreads();
    if (zok && line < NY) {
      cplx<T> w[MX];
      sfor<0, MX>([&](auto i) { w[CV(i)] = P[line * PITCH + FX::freq(CV(i), t)]; });
      FX::inverse(w, t);
      PairCols<T> out = pair_cols<T>(E, e, A.out_blk, pair, ncols, A.ext);
      sfor<0, MX>([&](auto i) {
        const int x = t + TL * CV(i);
        out.a[zoff + line * NX + x] = w[CV(i)].re;
        if (out.b) out.b[zoff + line * NX + x] = w[CV(i)].im;
      });
    }
  }
}

// ---------------------------------------------------------------------------
// z-column pass
// ---------------------------------------------------------------------------
enum ZMode { ZM_HPSI = 0, ZM_TETER = 1, ZM_DZ = 2 };

struct ZArgs {
  const ElemDev* elems;
  const int* elem_list;
  const int* active;
  int in_blk, out_blk;
  int ncols;
  int k3;
  ExtBufs ext;
};

template <typename T, int NZ, int TL, int MODE>
__global__ void __launch_bounds__(256) k_zcol(ZArgs A) {
  constexpr int M = NZ / TL;
  using FZ = LineFFT<T, NZ, TL>;
  const int e = A.elem_list[blockIdx.z];
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int ncols = A.ncols > 0 ? A.ncols : (A.ncols == kNcolsJ ? E.J : E.K);
  const int pair = blockIdx.y;
  if (2 * pair >= ncols) return;
  const int nxy = E.nx * E.ny;
  const int col = blockIdx.x * (256 / TL) + threadIdx.x / TL;
  const int t = threadIdx.x % TL;
  if (col >= nxy) return;  // whole lane groups leave together
  const cplx<T> wz = FZ::root(t);   // one root selection for both transforms

  cplx<T> v[M];
  if constexpr (MODE == ZM_HPSI) {
    PairCols<T> in = pair_cols<T>(E, e, A.in_blk, pair, ncols, A.ext);
    sfor<0, M>([&](auto i) {
      const size_t o = (size_t)(t + TL * CV(i)) * nxy + col;
      v[CV(i)] = {in.a[o], in.b ? in.b[o] : T(0)};
    });
    FZ::forward(v, t, wz);
    const T gzs = T(E.kz / NZ);
    sfor<0, M>([&](auto i) {
      const int f = signed_freq(FZ::freq(CV(i), t), NZ);
      const T g = gzs * T(f * f);
      v[CV(i)].re *= g;
      v[CV(i)].im *= g;
    });
    FZ::inverse(v, t, wz);
    PairCols<T> out = pair_cols<T>(E, e, A.out_blk, pair, ncols, A.ext);
    sfor<0, M>([&](auto i) {
      const size_t o = (size_t)(t + TL * CV(i)) * nxy + col;
      out.a[o] += v[CV(i)].re;
      if (out.b) out.b[o] += v[CV(i)].im;
    });
  } else if constexpr (MODE == ZM_DZ) {
    // d/dz along the columns of z
    PairCols<T> in = pair_cols<T>(E, e, A.in_blk, pair, ncols, A.ext);
    sfor<0, M>([&](auto i) {
      const size_t o = (size_t)(t + TL * CV(i)) * nxy + col;
      v[CV(i)] = {in.a[o], in.b ? in.b[o] : T(0)};
    });
    FZ::forward(v, t, wz);
    const T g = T(sqrt(2.0 * E.kz) / NZ);
    sfor<0, M>([&](auto i) {
      const T m = g * T(deriv_freq(FZ::freq(CV(i), t), NZ));
      v[CV(i)] = {-m * v[CV(i)].im, m * v[CV(i)].re};
    });
    FZ::inverse(v, t, wz);
    PairCols<T> out = pair_cols<T>(E, e, A.out_blk, pair, ncols, A.ext);
    sfor<0, M>([&](auto i) {
      const size_t o = (size_t)(t + TL * CV(i)) * nxy + col;
      out.a[o] = v[CV(i)].re;
      if (out.b) out.b[o] = v[CV(i)].im;
    });
  } else {
    // Teter: complex spectrum pair in W columns (2p: re, 2p+1: im), in place
    PairCols<T> w = pair_cols<T>(E, e, A.out_blk, pair, 2 * pair + 2, A.ext);
    sfor<0, M>([&](auto i) {
      const size_t o = (size_t)(t + TL * CV(i)) * nxy + col;
      v[CV(i)] = {w.a[o], w.b[o]};
    });
    FZ::forward(v, t, wz);
    const int KP = E.kmax3 + 2;
    const double* ek = E.small + SmallLayout::vec(KP) + VS_EKIN * KP;
    const double ea = ek[2 * pair];
    const double eb = (2 * pair + 1 < ncols) ? ek[2 * pair + 1] : ea;
    const T inv_e = T(2.0 / (ea + eb));
    const int kx = signed_freq(col % E.nx, E.nx);
    const int ky = signed_freq(col / E.nx, E.ny);
    const T gxy = T(E.kx * (double)(kx * kx) + E.ky * (double)(ky * ky));
    const T norm = T(1.0 / (double(E.nx) * E.ny * NZ));
    sfor<0, M>([&](auto i) {
      const int f = signed_freq(FZ::freq(CV(i), t), NZ);
      const T x = (gxy + T(E.kz) * T(f * f)) * inv_e;
      const T num = T(27) + x * (T(18) + x * (T(12) + T(8) * x));
      const T x2 = x * x;
      const T kf = norm * num * fast_recip(num + T(16) * x2 * x2);
      v[CV(i)].re *= kf;
      v[CV(i)].im *= kf;
    });
    FZ::inverse(v, t, wz);
    sfor<0, M>([&](auto i) {
      const size_t o = (size_t)(t + TL * CV(i)) * nxy + col;
      w.a[o] = v[CV(i)].re;
      w.b[o] = v[CV(i)].im;
    });
  }
}

// ---------------------------------------------------------------------------
// nonlocal projectors: C = B^T X (per group of projectors sharing a support)
// ---------------------------------------------------------------------------
struct NlArgs {
  const ElemDev* elems;
  const int* active;
  int in_blk, out_blk;
  int ncols;
  int elem_only;   // >= 0: only this element (gridDim.z == 1)
  ExtBufs ext;
};

// projector overlaps of element e: the element's own slice (nproj x kmax3), or the
// caller-independent scratch (nproj x nvec) of the no-allocation H*psi
__device__ __forceinline__ double* nlc_base(const ElemDev& E, int e, const ExtBufs& X, int& ld) {
  if (X.nlc) {
    ld = X.nvec;
    return X.nlc + (X.elem_only >= 0 ? 0 : X.nproj_off[e] * X.nvec);
  }
  ld = E.kmax3;
  return E.nlc;
}

constexpr int kNlCols = 8;

template <typename T>
__global__ void __launch_bounds__(256) k_nl_overlap(NlArgs A) {
  const int e = A.elem_only >= 0 ? A.elem_only : blockIdx.z;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int g = blockIdx.x;
  if (g >= E.ngrp) return;
  const int ncols = A.ncols > 0 ? A.ncols : (A.ncols == kNcolsJ ? E.J : E.K);
  const int c0 = blockIdx.y * kNlCols;
  if (c0 >= ncols) return;
  const int s0 = E.grp_sptr[g], s1 = E.grp_sptr[g + 1];
  const int len = s1 - s0;
  const int p0 = E.grp_pbase[g], np = E.grp_pbase[g + 1] - p0;
  const long long vb = E.grp_vbase[g];
  long long ldx;
  const T* X = block_base<T>(E, e, A.in_blk, A.ext, ldx);
  int nld;
  double* nlc = nlc_base(E, e, A.ext, nld);
  const T* val = nullptr;
  if constexpr (sizeof(T) == 8) val = reinterpret_cast<const T*>(E.grp_val64);
  else val = reinterpret_cast<const T*>(E.grp_val32);
  double acc[4][kNlCols];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < kNlCols; ++j) acc[q][j] = 0.0;
  for (int s = threadIdx.x; s < len; s += blockDim.x) {
    const int r = E.grp_idx[s0 + s];
    T b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) b[q] = (q < np) ? val[vb + (long long)q * len + s] : T(0);
#pragma unroll
    for (int j = 0; j < kNlCols; ++j) {
      if (c0 + j < ncols) {
        const T x = X[(size_t)(c0 + j) * ldx + r];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q][j] += double(b[q]) * double(x);
      }
    }
  }
  // block reduction in a fixed order: DPP wave sums, then across waves
  __shared__ double red[4][4 * kNlCols];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < kNlCols; ++j) {
      const double v = wave_sum_dpp(acc[q][j]);
      if (lane == 0) red[wv][q * kNlCols + j] = v;
    }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  for (int w = threadIdx.x; w < 4 * kNlCols; w += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i][w];
    const int q = w / kNlCols, j = w % kNlCols;
    if (q < np && c0 + j < ncols) nlc[(size_t)(p0 + q) * nld + c0 + j] = s;
  }
}

// y[r, j] += sum_{p in row r} b_p(r) gamma_p C[p, j] over the active points
constexpr int kNlApplyCols = 16;
// LDS row pitch of the gamma C table: odd in doubles, so that lanes reading the rows
// of different projectors fall in different banks
constexpr int kNlApplyPitch = kNlApplyCols + 1;

template <typename T>
__global__ void __launch_bounds__(256) k_nl_apply(NlArgs A) {
  const int e = A.elem_only >= 0 ? A.elem_only : blockIdx.z;
  const ElemDev& E = A.elems[e];
  if (A.active && !A.active[e]) return;
  const int ncols = A.ncols > 0 ? A.ncols : (A.ncols == kNcolsJ ? E.J : E.K);
  const int c0 = blockIdx.y * kNlApplyCols;
  if (c0 >= ncols || E.nact == 0) return;
  const int nc = min(kNlApplyCols, ncols - c0);
  extern __shared__ double gc[];   // nproj x kNlApplyPitch: gamma_p C[p, c0 + j]
  int nld;
  const double* nlc = nlc_base(E, e, A.ext, nld);
  for (int i = threadIdx.x; i < E.nproj * kNlApplyCols; i += blockDim.x) {
    const int p = i / kNlApplyCols, j = i % kNlApplyCols;
    gc[p * kNlApplyPitch + j] = (j < nc) ? E.gamma[p] * nlc[(size_t)p * nld + c0 + j] : 0.0;
  }
  __syncthreads();
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= E.nact) return;
  const int r = E.act_idx[a];
  const int q0 = E.act_ptr[a], q1 = E.act_ptr[a + 1];
  double acc[kNlApplyCols];
#pragma unroll
  for (int j = 0; j < kNlApplyCols; ++j) acc[j] = 0.0;
  const T* ev = nullptr;
  if constexpr (sizeof(T) == 8) ev = reinterpret_cast<const T*>(E.ent_val64);
  else ev = reinterpret_cast<const T*>(E.ent_val32);
  for (int q = q0; q < q1; ++q) {
    const int p = E.ent_proj[q];
    const double bv = double(ev[q]);
#pragma unroll
    for (int j = 0; j < kNlApplyCols; ++j) acc[j] += bv * gc[p * kNlApplyPitch + j];
  }
  long long ldy;
  T* Y = block_base<T>(E, e, A.out_blk, A.ext, ldy);
#pragma unroll
  for (int j = 0; j < kNlApplyCols; ++j)
    if (j < nc) Y[(size_t)(c0 + j) * ldy + r] += T(acc[j]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int NXY, int TL, int MODE>
static void plane_launch(const PlaneArgs& a, int nz, int npairs, int nel, hipStream_t s) {
  constexpr int TPP = NXY * TL;
  constexpr int PPW = (256 / TPP) > 0 ? 256 / TPP : 1;
  dim3 grid((nz + PPW - 1) / PPW, npairs, nel);
  hipLaunchKernelGGL((k_plane<T, NXY, NXY, TL, MODE>), grid, dim3(PPW * TPP), 0, s, a);
}

template <typename T, int NZ, int TL, int MODE>
static void z_launch(const ZArgs& a, int nxy, int npairs, int nel, hipStream_t s) {
  dim3 grid((nxy + (256 / TL) - 1) / (256 / TL), npairs, nel);
  hipLaunchKernelGGL((k_zcol<T, NZ, TL, MODE>), grid, dim3(256), 0, s, a);
}

// lanes per FFT line: lines of 32..64 points on 8 lanes (M = 4..8 values per
// lane), shorter lines on 4; the same for FP32 and FP64 (fewer values per lane keep
// the register count, and so the occupancy, of the long-line kernels up)
template <typename T, int N>
constexpr int lanes_per_line() {
  return N >= 32 ? 8 : 4;
}

template <typename T, int MODE>
static bool dispatch_plane(int nxy, const PlaneArgs& a, int nz, int npairs, int nel, hipStream_t s) {
  switch (nxy) {
    case 8: plane_launch<T, 8, lanes_per_line<T, 8>(), MODE>(a, nz, npairs, nel, s); return true;
    case 12: plane_launch<T, 12, lanes_per_line<T, 12>(), MODE>(a, nz, npairs, nel, s); return true;
    case 16: plane_launch<T, 16, lanes_per_line<T, 16>(), MODE>(a, nz, npairs, nel, s); return true;
    case 24: plane_launch<T, 24, lanes_per_line<T, 24>(), MODE>(a, nz, npairs, nel, s); return true;
    case 32: plane_launch<T, 32, lanes_per_line<T, 32>(), MODE>(a, nz, npairs, nel, s); return true;
    case 48: plane_launch<T, 48, lanes_per_line<T, 48>(), MODE>(a, nz, npairs, nel, s); return true;
    case 64: plane_launch<T, 64, lanes_per_line<T, 64>(), MODE>(a, nz, npairs, nel, s); return true;
    default: return false;
  }
}

template <typename T, int MODE>
static bool dispatch_z(int nz, const ZArgs& a, int nxy, int npairs, int nel, hipStream_t s) {
  switch (nz) {
    case 8: z_launch<T, 8, lanes_per_line<T, 8>(), MODE>(a, nxy, npairs, nel, s); return true;
    case 12: z_launch<T, 12, lanes_per_line<T, 12>(), MODE>(a, nxy, npairs, nel, s); return true;
    case 16: z_launch<T, 16, lanes_per_line<T, 16>(), MODE>(a, nxy, npairs, nel, s); return true;
    case 24: z_launch<T, 24, lanes_per_line<T, 24>(), MODE>(a, nxy, npairs, nel, s); return true;
    case 32: z_launch<T, 32, lanes_per_line<T, 32>(), MODE>(a, nxy, npairs, nel, s); return true;
    case 48: z_launch<T, 48, lanes_per_line<T, 48>(), MODE>(a, nxy, npairs, nel, s); return true;
    case 64: z_launch<T, 64, lanes_per_line<T, 64>(), MODE>(a, nxy, npairs, nel, s); return true;
    default: return false;
  }
}

// algorithmic bytes of the H*psi passes for the elements a launch covers
struct HpsiWork {
  double plane = 0, zcol = 0, nl = 0;
};

static HpsiWork hpsi_work(Ctx& c, int elem, int ncols, size_t sz, const std::vector<int>& members,
                          const int* active_host) {
  HpsiWork w;
  for (int e : members) {
    if (elem >= 0 && e != elem) continue;
    if (active_host && !active_host[e]) continue;
    const double N = c.N[e], k = ncols > 0 ? ncols : c.K[e];
    w.plane += (2.0 * k + 1.0) * N * sz;          // read x, write y1, read V
    w.zcol += 3.0 * k * N * sz;                   // read x, read y1, write y
    const double nnz = c.nnz[e], nact = c.elems_host[e].nact;
    w.nl += nnz * (sz + 4) + 3.0 * nact * k * sz;  // projectors; x read, y read+write at active points
  }
  return w;
}

template <typename T>
static int hpsi_typed(Ctx& c, int elem, int ncols, int in_blk, int out_blk, const int* active,
                      const ExtBufs& ext = ExtBufs()) {
  hipStream_t s = c.stream;
  const int* act_host = (active && !c.active_host.empty()) ? c.active_host.data() : nullptr;
  const int* iota = c.iota_dev;
  if (c.timing && !c.capturing) {
    // algorithmic bytes of the state applications: read psi, write H psi, V and the
    // projectors (nnz values + int32 indices) amortised over the J wanted states
    const double sz = sizeof(T);
    for (int e = 0; e < c.n_elem; ++e) {
      if ((elem >= 0 && e != elem) || (act_host && !act_host[e])) continue;
      const double N = c.N[e], k = ncols > 0 ? ncols : c.K[e], J = c.J[e];
      c.tacc.hpsi_alg += k * (2.0 * N * sz + N * sz / J + c.nnz[e] * (sz + 4.0) / J);
    }
  }
  // projector overlaps first (reads x only)
  {
    NlArgs na{c.elems_dev, active, in_blk, out_blk, ncols, elem, ext};
    int ng = 0, np = 0, kk = 0;
    for (int e = 0; e < c.n_elem; ++e) {
      if (elem >= 0 && e != elem) continue;
      ng = std::max(ng, c.elems_host[e].ngrp);
      np = std::max(np, c.elems_host[e].nproj);
      kk = std::max(kk, ncols > 0 ? ncols : c.K[e]);
    }
    if (ng > 0) {
      std::vector<int> all(c.n_elem);
      for (int e = 0; e < c.n_elem; ++e) all[e] = e;
      TimedScope ts(c, TC_NL, hpsi_work(c, elem, ncols, sizeof(T), all, act_host).nl);
      dim3 g1(ng, (kk + kNlCols - 1) / kNlCols, elem >= 0 ? 1 : c.n_elem);
      hipLaunchKernelGGL(k_nl_overlap<T>, g1, dim3(256), 0, s, na);
    }
    c.nl_pending_np = np;
    c.nl_pending_kk = kk;
  }
  for (const ShapeClass& sc : c.classes) {
    const int* list = sc.elem_list_dev;
    int nel = sc.nelem;
    int maxk = 0;
    if (elem >= 0) {
      bool member = false;
      for (int x : sc.elem_list_host) member |= (x == elem);
      if (!member) continue;
      list = iota + elem;
      nel = 1;
      maxk = ncols > 0 ? ncols : c.K[elem];
    } else {
      maxk = ncols > 0 ? ncols : sc.max_k;
    }
    const int npairs = (maxk + 1) / 2;
    PlaneArgs pa{c.elems_dev, list, active, in_blk, out_blk, -1, ncols, nullptr, 0, ext};
    const HpsiWork hw = hpsi_work(c, elem, ncols, sizeof(T), sc.elem_list_host, act_host);
    {
      TimedScope ts(c, TC_PLANE, hw.plane);
      if (!dispatch_plane<T, PM_HPSI>(sc.nx, pa, sc.nz, npairs, nel, s)) {
        set_error("unsupported grid");
        return DG_ERR_SHAPE;
      }
    }
    ZArgs za{c.elems_dev, list, active, in_blk, out_blk, ncols, 0, ext};
    {
      TimedScope ts(c, TC_ZCOL, hw.zcol);
      if (!dispatch_z<T, ZM_HPSI>(sc.nz, za, sc.nx * sc.ny, npairs, nel, s)) {
        set_error("unsupported grid");
        return DG_ERR_SHAPE;
      }
    }
  }
  if (c.nl_pending_np > 0) {
    NlArgs na{c.elems_dev, active, in_blk, out_blk, ncols, elem, ext};
    int nact = 0;
    for (int e = 0; e < c.n_elem; ++e)
      if (elem < 0 || e == elem) nact = std::max(nact, c.elems_host[e].nact);
    dim3 g2((nact + 255) / 256, (c.nl_pending_kk + kNlApplyCols - 1) / kNlApplyCols,
            elem >= 0 ? 1 : c.n_elem);
    size_t shm = (size_t)c.nl_pending_np * kNlApplyPitch * sizeof(double);
    TimedScope ts(c, TC_NL);
    hipLaunchKernelGGL(k_nl_apply<T>, g2, dim3(256), shm, s, na);
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_hpsi(Ctx& c, int elem, int ncols, int prec, int in_blk, int out_blk, const int* active) {
  if (c.dg_op.active) return launch_dg_bsr(c, in_blk, out_blk, ncols, active);
  return prec == DG_FP64 ? hpsi_typed<double>(c, elem, ncols, in_blk, out_blk, active)
                         : hpsi_typed<float>(c, elem, ncols, in_blk, out_blk, active);
}

int launch_hpsi_ext(Ctx& c, int elem, int ncols, int prec, const ExtBufs& ext) {
  return prec == DG_FP64 ? hpsi_typed<double>(c, elem, ncols, kExtX, kExtY, nullptr, ext)
                         : hpsi_typed<float>(c, elem, ncols, kExtX, kExtY, nullptr, ext);
}

// W <- Teter(HX - X theta), three passes, for every element in place in W (r_given:
// hx_blk already holds the residual)
template <typename T>
static int teter_typed(Ctx& c, int x_blk, int hx_blk, int w_blk, int k3, const int* active, bool r_given) {
  hipStream_t s = c.stream;
  double tw = 0.0;
  for (int e = 0; e < c.n_elem; ++e)
    if (c.active_host.empty() || c.active_host[e]) tw += 3.0 * c.K[e] * (double)c.N[e] * sizeof(T);
  TimedScope ts(c, TC_TETER, tw);   // read X, HX, write W
  for (const ShapeClass& sc : c.classes) {
    const int npairs = (sc.max_k + 1) / 2;
    PlaneArgs pa{c.elems_dev, sc.elem_list_dev, active, r_given ? hx_blk : x_blk, w_blk, hx_blk, -1, nullptr, k3};
    pa.r_given = r_given ? 1 : 0;
    if (!dispatch_plane<T, PM_TFWD>(sc.nx, pa, sc.nz, npairs, sc.nelem, s)) return DG_ERR_SHAPE;
    ZArgs za{c.elems_dev, sc.elem_list_dev, active, w_blk, w_blk, -1, k3};
    if (!dispatch_z<T, ZM_TETER>(sc.nz, za, sc.nx * sc.ny, npairs, sc.nelem, s)) return DG_ERR_SHAPE;
    PlaneArgs pc{c.elems_dev, sc.elem_list_dev, active, w_blk, w_blk, -1, -1, nullptr, k3};
    if (!dispatch_plane<T, PM_TINV>(sc.nx, pc, sc.nz, npairs, sc.nelem, s)) return DG_ERR_SHAPE;
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_teter(Ctx& c, int prec, int x_blk, int hx_blk, int w_blk, int k3, const int* active, bool r_given) {
  return prec == DG_FP64 ? teter_typed<double>(c, x_blk, hx_blk, w_blk, k3, active, r_given)
                         : teter_typed<float>(c, x_blk, hx_blk, w_blk, k3, active, r_given);
}

// d/dx, d/dy, d/dz of the first J_k columns of block in_blk into out blocks (FP64,
// every element)
int launch_gradient(Ctx& c, int in_blk, const int out_blk[3]) {
  hipStream_t s = c.stream;
  const int ncols = kNcolsJ;
  for (const ShapeClass& sc : c.classes) {
    int maxk = 0;
    for (int e : sc.elem_list_host) maxk = std::max(maxk, c.J[e]);
    const int npairs = (maxk + 1) / 2;
    PlaneArgs px{c.elems_dev, sc.elem_list_dev, nullptr, in_blk, out_blk[0], -1, ncols, nullptr, 0};
    if (!dispatch_plane<double, PM_DX>(sc.nx, px, sc.nz, npairs, sc.nelem, s)) return DG_ERR_SHAPE;
    PlaneArgs py{c.elems_dev, sc.elem_list_dev, nullptr, in_blk, out_blk[1], -1, ncols, nullptr, 0};
    if (!dispatch_plane<double, PM_DY>(sc.nx, py, sc.nz, npairs, sc.nelem, s)) return DG_ERR_SHAPE;
    ZArgs zz{c.elems_dev, sc.elem_list_dev, nullptr, in_blk, out_blk[2], ncols, 0};
    if (!dispatch_z<double, ZM_DZ>(sc.nz, zz, sc.nx * sc.ny, npairs, sc.nelem, s)) return DG_ERR_SHAPE;
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}

bool grid_supported(int nx, int ny, int nz) {
  auto ok = [](int n) { return n == 8 || n == 12 || n == 16 || n == 24 || n == 32 || n == 48 || n == 64; };
  return nx == ny && ok(nx) && ok(nz);
}

}  // namespace dg
