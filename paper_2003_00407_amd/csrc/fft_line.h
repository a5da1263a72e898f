// Line FFTs for the plane-wave kinetic operator on gfx950.
//
// The kinetic term of the local Kohn-Sham operator (Eq. (1)) in the full
// plane-wave box is T = F^{-1} diag(|G|^2/2) F.  Because |G|^2 = Gx^2 + Gy^2 +
// Gz^2, T is the sum of three 1D spectral operators, one per axis; each is a
// forward 1D DFT along grid lines, a multiply by (G_axis^2 / 2) and an inverse
// DFT.  The lines are transformed here in registers:
//
//  * a line of N complex points is held by a group of TL adjacent lanes
//    (TL in {1, 2, 4, 8}); lane t of the group holds the M = N / TL points
//    j = t + TL * i, i = 0..M-1;
//  * forward: per-lane DFT_M over i (mixed radix 4/3/2, unrolled, every index
//    a compile-time constant so the data stays in VGPRs), twiddle W_N^{t k1},
//    then a DFT_TL across the lane group (butterflies over __shfl_xor);
//  * afterwards lane t holds frequencies k1 + M * bitrev_TL(t), k1 = 0..M-1;
//  * the inverse is the exact mirror (unnormalised; the 1/N is folded into the
//    spectral multiplier).
//
// Two real grid vectors are packed as one complex line (re = state a,
// im = state b).  A real, even multiplier m(k) = m(-k) keeps the two halves
// apart: F^{-1} m F (a + i b) = (F^{-1} m F a) + i (F^{-1} m F b).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dg {

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul(cplx<T> a, T wr, T wi) {
  return {a.re * wr - a.im * wi, a.re * wi + a.im * wr};
}
// multiply by -i (DIR = -1) or +i (DIR = +1)
template <int DIR, typename T>
__host__ __device__ __forceinline__ cplx<T> cmul_i(cplx<T> a) {
  if constexpr (DIR < 0) return {a.im, -a.re};
  else return {-a.im, a.re};
}

// ---------------------------------------------------------------------------
// compile-time trigonometry: cos / sin of 2 pi p / q for integers, double
// precision (octant reduction with exact integer arithmetic, then Taylor
// series on [0, pi/4]; error ~1 ulp).
// ---------------------------------------------------------------------------
struct TrigPair {
  double c, s;
};

constexpr double kTwoPi = 6.283185307179586476925286766559;

constexpr TrigPair taylor_cs(double x) {
  // Horner evaluation, smallest terms first
  double x2 = x * x;
  double c = 0.0, s = 0.0;
  for (int n = 14; n >= 1; --n) {
    c = 1.0 - c * x2 / double((2 * n - 1) * (2 * n)) ;
    s = 1.0 - s * x2 / double((2 * n) * (2 * n + 1));
  }
  // the loop above leaves c = 1 - x2/2 (1 - ...), s = 1 - x2/6 (1 - ...)
  return {c, x * s};
}

// cos and sin of 2 pi p / q
constexpr TrigPair turn_cs(long p, long q) {
  p %= q;
  if (p < 0) p += q;
  // x = p/q in [0, 1)
  bool neg_s = false, neg_c = false, swap = false;
  if (2 * p > q) {  // x > 1/2: angle -> 1 - x, sin flips
    p = q - p;
    neg_s = true;
  }
  if (4 * p > q) {  // x in (1/4, 1/2]: -> 1/2 - x, cos flips
    p = q - 2 * p;
    q = 2 * q;
    neg_c = true;
  }
  if (8 * p > q) {  // x in (1/8, 1/4]: -> 1/4 - x, cos <-> sin
    p = q - 4 * p;
    q = 4 * q;
    swap = true;
  }
  TrigPair t = taylor_cs(kTwoPi * double(p) / double(q));
  double c = swap ? t.s : t.c;
  double s = swap ? t.c : t.s;
  if (neg_c) c = -c;
  if (neg_s) s = -s;
  return {c, s};
}

// W_n^{e} = exp(DIR * 2 pi i e / n), DIR = -1 forward
template <typename T, int N, int DIR>
struct Tw {
  static constexpr T re(int e) { return T(turn_cs(e, N).c); }
  static constexpr T im(int e) { return T(DIR * turn_cs(e, N).s); }
};

// ---------------------------------------------------------------------------
// compile-time loops: sfor<B, E>(f) calls f(IC<i>{}) for i = B..E-1; the index
// is read back as a constant expression with CV(x)
// ---------------------------------------------------------------------------
#define CV(x) (decltype(x)::value)

template <int I>
struct IC {
  static constexpr int value = I;
};

template <int B, int E, typename F>
__host__ __device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(IC<B>{});
    sfor<B + 1, E>(f);
  }
}

// ---------------------------------------------------------------------------
// per-lane DFT of compile-time length M, natural order in and out
// ---------------------------------------------------------------------------
template <typename T, int DIR>
__host__ __device__ __forceinline__ void dft2(cplx<T>& a, cplx<T>& b) {
  cplx<T> s = cadd(a, b), d = csub(a, b);
  a = s;
  b = d;
}

template <typename T, int DIR>
__host__ __device__ __forceinline__ void dft3(cplx<T>& a, cplx<T>& b, cplx<T>& c) {
  // X0 = a+b+c; X1 = a + w b + w^2 c; X2 = a + w^2 b + w c, w = exp(DIR 2 pi i / 3)
  constexpr T h = T(-0.5);
  constexpr T r = T(DIR * 0.86602540378443864676372317075294);  // DIR * sin(2 pi / 3)
  cplx<T> s = cadd(b, c), d = csub(b, c);
  cplx<T> m = {a.re + h * s.re, a.im + h * s.im};
  cplx<T> x0 = cadd(a, s);
  // i * r * d
  cplx<T> jd = {-r * d.im, r * d.re};
  a = x0;
  b = cadd(m, jd);
  c = csub(m, jd);
}

template <typename T, int DIR>
__host__ __device__ __forceinline__ void dft4(cplx<T>& a, cplx<T>& b, cplx<T>& c, cplx<T>& d) {
  cplx<T> s0 = cadd(a, c), d0 = csub(a, c);
  cplx<T> s1 = cadd(b, d), d1 = csub(b, d);
  cplx<T> jd1 = cmul_i<DIR>(d1);
  a = cadd(s0, s1);
  c = csub(s0, s1);
  b = cadd(d0, jd1);
  d = csub(d0, jd1);
}

template <int M>
constexpr int first_radix() {
  return (M % 4 == 0 && M != 8) ? 4 : (M % 2 == 0 ? 2 : (M % 3 == 0 ? 3 : M));
}

template <typename T, int M, int DIR>
__host__ __device__ __forceinline__ void dft_reg(cplx<T> (&x)[M]) {
  if constexpr (M == 1) {
  } else if constexpr (M == 2) {
    dft2<T, DIR>(x[0], x[1]);
  } else if constexpr (M == 3) {
    dft3<T, DIR>(x[0], x[1], x[2]);
  } else if constexpr (M == 4) {
    dft4<T, DIR>(x[0], x[1], x[2], x[3]);
  } else {
    constexpr int R = first_radix<M>();
    constexpr int Q = M / R;
    static_assert(R * Q == M && R <= 4, "unsupported DFT length (radix 2/3/4 only)");
    cplx<T> sub[R][Q];
    sfor<0, R>([&](auto s) {
      sfor<0, Q>([&](auto i) { sub[CV(s)][CV(i)] = x[CV(s) + R * CV(i)]; });
      dft_reg<T, Q, DIR>(sub[CV(s)]);
    });
    // X[k + Q u] = sum_s W_R^{s u} (W_M^{s k} sub[s][k])
    sfor<0, Q>([&](auto k) {
      cplx<T> t[R];
      sfor<0, R>([&](auto s) {
        constexpr int e = CV(s) * CV(k);
        if constexpr (e == 0) {
          t[CV(s)] = sub[CV(s)][CV(k)];
        } else {
          constexpr T wr = Tw<T, M, DIR>::re(e);
          constexpr T wi = Tw<T, M, DIR>::im(e);
          t[CV(s)] = cmul(sub[CV(s)][CV(k)], wr, wi);
        }
      });
      dft_reg<T, R, DIR>(t);
      sfor<0, R>([&](auto u) { x[CV(k) + Q * CV(u)] = t[CV(u)]; });
    });
  }
}

template <int TL>
__host__ __device__ constexpr int bitrev_lane(int t) {
  if constexpr (TL == 4) return ((t & 1) << 1) | ((t >> 1) & 1);
  else if constexpr (TL == 8) return ((t & 1) << 2) | (t & 2) | ((t >> 2) & 1);
  else return t;
}

// ---------------------------------------------------------------------------
// lane-group line FFT (device)
// ---------------------------------------------------------------------------
// value of lane (l xor MASK): within a quad (MASK 1, 2) by a DPP quad permute on the
// vector ALU, else through the LDS crossbar (ds_bpermute; two row-shift DPP moves
// with bank masks measured slower for MASK 4)
template <int MASK, typename T>
__device__ __forceinline__ T lane_xor(T v) {
  if constexpr (MASK == 1 || MASK == 2) {
    constexpr int ctrl = MASK == 1 ? 0xB1 : 0x4E;   // quad_perm [1,0,3,2] / [2,3,0,1]
    // every lane reads a lane of its own quad, so no "old" value is needed
    if constexpr (sizeof(T) == 8) {
      const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, true);
      const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, true);
      return __hiloint2double(hi, lo);
    } else {
      return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xF, 0xF, true));
    }
  } else {
    return __shfl_xor(v, MASK);
  }
}

template <int MASK, typename T>
__device__ __forceinline__ cplx<T> shfl_xor_c(cplx<T> v) {
  return {lane_xor<MASK>(v.re), lane_xor<MASK>(v.im)};
}

template <typename T, int N, int TL>
struct LineFFT {
  static constexpr int M = N / TL;
  static_assert(M * TL == N, "line length must be a multiple of the lanes per line");

  // frequency held in register k by lane t after forward()
  __device__ static __forceinline__ int freq(int k, int t) { return k + M * bitrev_lane<TL>(t); }

  // v *= W_N^{DIR t k} for k = 0..M-1 (t = lane within the group, runtime)
  template <int DIR>
  __device__ static __forceinline__ void lane_twiddle(cplx<T> (&v)[M], int t) {
    if constexpr (TL == 8) {
      // W_N^{t k} = (W_N^t)^k: the lane's root is selected once among eight
      // compile-time values, its powers follow by complex products (a few ulps, k < 8)
      T r1 = T(1), i1 = T(0);
      sfor<1, 8>([&](auto j) {
        constexpr T rj = Tw<T, N, DIR>::re(CV(j)), ij = Tw<T, N, DIR>::im(CV(j));
        if (t == CV(j)) {
          r1 = rj;
          i1 = ij;
        }
      });
      T wr = r1, wi = i1;
      sfor<1, M>([&](auto k) {
        v[CV(k)] = cmul(v[CV(k)], wr, wi);
        if constexpr (CV(k) + 1 < M) {
          const T nr = wr * r1 - wi * i1;
          wi = wr * i1 + wi * r1;
          wr = nr;
        }
      });
    } else if constexpr (TL > 1) {
      sfor<1, M>([&](auto k) {
        constexpr int kk = CV(k);
        T wr, wi;
        if constexpr (TL == 2) {
          constexpr T r1 = Tw<T, N, DIR>::re(kk), i1 = Tw<T, N, DIR>::im(kk);
          wr = t ? r1 : T(1);
          wi = t ? i1 : T(0);
        } else {
          constexpr T r1 = Tw<T, N, DIR>::re(kk), i1 = Tw<T, N, DIR>::im(kk);
          constexpr T r2 = Tw<T, N, DIR>::re(2 * kk), i2 = Tw<T, N, DIR>::im(2 * kk);
          constexpr T r3 = Tw<T, N, DIR>::re(3 * kk), i3 = Tw<T, N, DIR>::im(3 * kk);
          wr = (t == 0) ? T(1) : (t == 1) ? r1 : (t == 2) ? r2 : r3;
          wi = (t == 0) ? T(0) : (t == 1) ? i1 : (t == 2) ? i2 : i3;
        }
        v[kk] = cmul(v[kk], wr, wi);
      });
    }
  }

  // the lane's root W_N^t of the forward direction (8 lanes per line), for kernels that
  // select it once and pass it to forward() and inverse() (the inverse conjugates it)
  __device__ static __forceinline__ cplx<T> root(int t) {
    T r1 = T(1), i1 = T(0);
    if constexpr (TL == 8) {
      sfor<1, 8>([&](auto j) {
        constexpr T rj = Tw<T, N, -1>::re(CV(j)), ij = Tw<T, N, -1>::im(CV(j));
        if (t == CV(j)) {
          r1 = rj;
          i1 = ij;
        }
      });
    }
    return {r1, i1};
  }

  template <int DIR>
  __device__ static __forceinline__ void lane_twiddle(cplx<T> (&v)[M], int t, cplx<T> w1) {
    if constexpr (TL == 8) {
      const T r1 = w1.re, i1 = DIR < 0 ? w1.im : -w1.im;
      T wr = r1, wi = i1;
      sfor<1, M>([&](auto k) {
        v[CV(k)] = cmul(v[CV(k)], wr, wi);
        if constexpr (CV(k) + 1 < M) {
          const T nr = wr * r1 - wi * i1;
          wi = wr * i1 + wi * r1;
          wr = nr;
        }
      });
    } else {
      lane_twiddle<DIR>(v, t);
    }
  }

  // radix-2 butterfly across lanes (xor mask): lower lane gets own+other, upper other-own,
  // both as other + sign * own (one fused multiply-add per component)
  template <int MASK>
  __device__ static __forceinline__ void xbfly(cplx<T> (&v)[M], bool upper) {
    const T sg = upper ? T(-1) : T(1);
    sfor<0, M>([&](auto k) {
      cplx<T> o = shfl_xor_c<MASK>(v[CV(k)]);
      v[CV(k)] = {T(fma(sg, v[CV(k)].re, o.re)), T(fma(sg, v[CV(k)].im, o.im))};
    });
  }

  // v *= W_8^{DIR j} on lanes whose xor-4 partner is lower (t >= 4), j = t - 4
  __device__ static __forceinline__ void w8_upper(cplx<T> (&v)[M], int t, int dir) {
    if (t < 4) return;
    const int j = t - 4;
    // W_8^{dir j}: 1, (1 + dir i)/sqrt2, dir i, (-1 + dir i)/sqrt2
    const T h = T(0.70710678118654752440);
    const T wr = j == 0 ? T(1) : j == 1 ? h : j == 2 ? T(0) : -h;
    const T wi = T(dir) * (j == 0 ? T(0) : j == 1 ? h : j == 2 ? T(1) : h);
    sfor<0, M>([&](auto k) { v[CV(k)] = cmul(v[CV(k)], wr, wi); });
  }

  template <int DIR>
  __device__ static __forceinline__ void cross_lane(cplx<T> (&v)[M], int t) {
    if constexpr (TL == 2) {
      xbfly<1>(v, t & 1);
    } else if constexpr (TL == 8) {
      // radix-2 network over the three lane bits (decimation in frequency forward,
      // its transpose with conjugate twiddles inverse); lane t holds index bitrev(t)
      if constexpr (DIR < 0) {
        xbfly<4>(v, t & 4);
        w8_upper(v, t, -1);
        xbfly<2>(v, t & 2);
        if ((t & 3) == 3) sfor<0, M>([&](auto k) { v[CV(k)] = cmul_i<-1>(v[CV(k)]); });
        xbfly<1>(v, t & 1);
      } else {
        xbfly<1>(v, t & 1);
        if ((t & 3) == 3) sfor<0, M>([&](auto k) { v[CV(k)] = cmul_i<+1>(v[CV(k)]); });
        xbfly<2>(v, t & 2);
        w8_upper(v, t, +1);
        xbfly<4>(v, t & 4);
      }
    } else if constexpr (TL == 4) {
      if constexpr (DIR < 0) {
        xbfly<2>(v, t & 2);
        if (t == 3) sfor<0, M>([&](auto k) { v[CV(k)] = cmul_i<-1>(v[CV(k)]); });
        xbfly<1>(v, t & 1);
      } else {
        // mirror of the forward network
        xbfly<1>(v, t & 1);
        if (t == 3) sfor<0, M>([&](auto k) { v[CV(k)] = cmul_i<+1>(v[CV(k)]); });
        xbfly<2>(v, t & 2);
      }
    }
  }

  __device__ static __forceinline__ void forward(cplx<T> (&v)[M], int t) {
    dft_reg<T, M, -1>(v);
    lane_twiddle<-1>(v, t);
    cross_lane<-1>(v, t);
  }

  // unnormalised inverse: inverse(forward(x)) = N x
  __device__ static __forceinline__ void inverse(cplx<T> (&v)[M], int t) {
    cross_lane<+1>(v, t);
    lane_twiddle<+1>(v, t);
    dft_reg<T, M, +1>(v);
  }

  // the same with the lane's root w1 = root(t) selected once by the caller
  __device__ static __forceinline__ void forward(cplx<T> (&v)[M], int t, cplx<T> w1) {
    dft_reg<T, M, -1>(v);
    lane_twiddle<-1>(v, t, w1);
    cross_lane<-1>(v, t);
  }
  __device__ static __forceinline__ void inverse(cplx<T> (&v)[M], int t, cplx<T> w1) {
    cross_lane<+1>(v, t);
    lane_twiddle<+1>(v, t, w1);
    dft_reg<T, M, +1>(v);
  }
};

}  // namespace dg
