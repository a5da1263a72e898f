// The DG Hamiltonian H^DG (Eq. (7), DGHamiltonian) in the ALB basis of the last
// solve.  Per element group (on the group's stream):
//   1. the ALBs extended to Q_k: the restriction's orthonormalisation (eigen-
//      decomposition of its Gram, then one Cholesky-QR pass) applied to all rows of
//      X, so that R_E F = the ALB values and F is a trigonometric polynomial on Q_k;
//   2. face traces of F: value and outward normal derivative of the interpolant half
//      a grid step beyond E_k's outer points (weights computed on the host);
//   3. spectral gradients of F (line-FFT kernels), restricted to E_k;
//   4. the kinetic + local-potential block 1/2 sum_a (d_a Phi)^T (d_a Phi) +
//      Phi^T diag(V) Phi (FP64 MFMA Grams over E_k's rows);
//   5. projector overlaps O[p, j] = <b_p, phi_j> over E_k.
// Then, on the caller's stream, one workgroup per nonzero block (k, nb) -- k itself,
// its four face neighbours and every element sharing a projector with it (projector
// supports can reach past the face neighbours) -- sums the local block, the nonlocal
// couplings of the projectors the two elements share, and the interior-penalty terms
// of their common face (or, for nb = k, of the element's four faces), in a fixed
// order (deterministic).
#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "dg_internal.h"

namespace dg {

int launch_gradient(Ctx& c, int in_blk, const int out_blk[3]);

constexpr int KC_Jc = -1;   // column code: E.J
static long long small_slot(int which) { return -1 - which; }

static int sync_read_dg(Ctx& c, void* dst, const void* src, size_t bytes) {
  DG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.stream));
  DG_HIP(hipStreamSynchronize(c.stream));
  return DG_OK;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// traces of the first J columns of block blk on the four faces of E_k:
// out[tr_off + face_base(f) + (v * J + j) * npts_f + pt], v = 0 value, 1 outward derivative
__global__ void __launch_bounds__(256) k_dg_trace(const ElemDev* elems, const DgElem* del, int elem_base, int blk,
                                                   double* work) {
  const int e = blockIdx.z;
  const ElemDev& E = elems[e];
  const DgElem& D = del[e + elem_base];
  const int f = blockIdx.y;                 // 0 x-, 1 x+, 2 y-, 3 y+
  const int npts = D.npts[f];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= npts * D.J) return;
  const int pt = i % npts, j = i / npts;
  const bool xf = f < 2;
  // face point: (tangential index t, z); the line runs along the face normal
  const int ntan = xf ? E.en[1] : E.en[0];
  const int t = pt % ntan, z = pt / ntan;
  const int n = xf ? E.nx : E.ny;
  const long long stride = xf ? 1 : E.nx;
  const long long base = xf ? (long long)E.nx * (E.elo[1] + t + (long long)E.ny * z)
                            : (long long)(E.elo[0] + t) + (long long)E.nx * E.ny * z;
  const double* col = reinterpret_cast<const double*>(E.blk[blk]) + (size_t)j * E.ld + base;
  const double* w = work + D.w_off + (size_t)f * 2 * 64;
  double v = 0.0, d = 0.0;
  for (int q = 0; q < n; ++q) {
    const double x = col[q * stride];
    v += w[q] * x;
    d += w[64 + q] * x;
  }
  long long fb = D.tr_off;
  for (int g = 0; g < f; ++g) fb += 2LL * D.J * D.npts[g];
  work[fb + (size_t)j * npts + pt] = v;
  work[fb + (size_t)(D.J + j) * npts + pt] = d;
}

// out[r, j] = V[q(r)] phi[r, j] over E_k's rows (gathered order), first J columns
__global__ void __launch_bounds__(256) k_dg_vphi(const ElemDev* elems, int phi_blk, int out_blk) {
  const int e = blockIdx.z;
  const ElemDev& E = elems[e];
  const int j = blockIdx.y;
  if (j >= E.J) return;
  const int ne = E.en[0] * E.en[1] * E.en[2];
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= ne) return;
  const int x = r % E.en[0], y = (r / E.en[0]) % E.en[1], z = r / (E.en[0] * E.en[1]);
  const int q = (x + E.elo[0]) + E.nx * ((y + E.elo[1]) + E.ny * (z + E.elo[2]));
  const size_t o = (size_t)j * E.ld + r;
  reinterpret_cast<double*>(E.blk[out_blk])[o] = E.v64[q] * reinterpret_cast<const double*>(E.blk[phi_blk])[o];
}

// local block L = 1/2 (G_xx + G_yy + G_zz) + (A + A^T) / 2 into the work buffer
// (G: the 3J x 3J Gram of [d_x Phi, d_y Phi, d_z Phi] in slot G, A = Phi^T V Phi in slot A)
__global__ void __launch_bounds__(256) k_dg_local(const ElemDev* elems, const DgElem* del, int elem_base,
                                                   double* work) {
  const int e = blockIdx.y;
  const ElemDev& E = elems[e];
  const DgElem& D = del[e + elem_base];
  const int J = E.J;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= J * J) return;
  const int i = idx % J, j = idx / J;
  const int KP = E.kmax3 + 2;
  const double* G = E.small + SmallLayout::G(KP);
  const double* Am = E.small + SmallLayout::A(KP);
  const int n3 = 3 * J;
  double kin = 0.0;
  for (int a = 0; a < 3; ++a) kin += G[(size_t)(a * J + i) * n3 + a * J + j];
  work[D.l_off + (size_t)j * J + i] = 0.5 * kin + 0.5 * (Am[(size_t)i * J + j] + Am[(size_t)j * J + i]);
}

// projector overlaps O[p * J + j] = sum_s b_p(s) phi[s, j] over E_k (phi: gathered rows)
__global__ void __launch_bounds__(256) k_dg_overlap(const ElemDev* elems, const DgElem* del, int elem_base,
                                                     int phi_blk, double* work) {
  const int e = blockIdx.z;
  const ElemDev& E = elems[e];
  const DgElem& D = del[e + elem_base];
  const int p = blockIdx.x;
  if (p >= D.np) return;
  const int j0 = blockIdx.y * 16;
  if (j0 >= D.J) return;
  const long long* ptr = reinterpret_cast<const long long*>(work + D.pj_off);
  const int* idx = reinterpret_cast<const int*>(work + D.pidx_off);
  const double* val = work + D.pval_off;
  const double* phi = reinterpret_cast<const double*>(E.blk[phi_blk]);
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (long long s = ptr[p] + threadIdx.x; s < ptr[p + 1]; s += 256) {
    const int r = idx[s];
    const double b = val[s];
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (j0 + q < D.J) acc[q] += b * phi[(size_t)(j0 + q) * E.ld + r];
  }
  __shared__ double red[4][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    double v = acc[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[w][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < 16 && j0 + threadIdx.x < D.J) {
    const double s = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    work[D.ovl_off + (size_t)p * D.J + j0 + threadIdx.x] = s;
  }
}

constexpr int kAsmThreads = 256;
constexpr int kAsmEntries = (88 * 88 + kAsmThreads - 1) / kAsmThreads;   // entries per thread
constexpr int kAsmChunk = 16;                                             // face points per LDS stage

// block b of H^DG: local block (nb = k), shared projectors, interior-penalty terms
__global__ void __launch_bounds__(kAsmThreads) k_dg_assemble(const DgElem* del, const DgBlock* blocks,
                                                             const int* pairs, const double* work, double* H,
                                                             double alpha) {
  const DgBlock& bk = blocks[blockIdx.x];
  const DgElem& A = del[bk.k];
  const DgElem& B = del[bk.nb];
  const int Ja = A.J, Jb = B.J, nent = Ja * Jb;
  double acc[kAsmEntries];
#pragma unroll
  for (int u = 0; u < kAsmEntries; ++u) {
    const int ent = threadIdx.x + u * kAsmThreads;
    acc[u] = 0.0;
    if (bk.face == 4 && ent < nent) acc[u] = work[A.l_off + ent];   // ent = i + Ja j
  }
  // nonlocal couplings through shared projectors
  for (int m = bk.pair_lo; m < bk.pair_hi; ++m) {
    const int p = pairs[2 * m], q = pairs[2 * m + 1];
    const double g = work[A.pval_off - A.np + p];   // gamma stored just before the values
    const double* oa = work + A.ovl_off + (size_t)p * Ja;
    const double* ob = work + B.ovl_off + (size_t)q * Jb;
#pragma unroll
    for (int u = 0; u < kAsmEntries; ++u) {
      const int ent = threadIdx.x + u * kAsmThreads;
      if (ent < nent) acc[u] += g * oa[ent % Ja] * ob[ent / Ja];
    }
  }
  // interior-penalty face terms: (face of k, face of nb, c1, c2); outward derivatives.
  // Same element on both sides (its four faces): -1/4 (v d' + d v') + alpha v v';
  // across a face: +1/4 (v d' + d v') - alpha v v'; each over the face sum / h_normal
  int nf = 0, fa[4], fb[4];
  double c1[4], c2[4];
  if (bk.face == 4) {
    for (int f = 0; f < 4; ++f) {
      fa[nf] = f;
      fb[nf] = f;
      c1[nf] = -0.25 * A.inv_h[f >> 1];
      c2[nf] = alpha * A.inv_h[f >> 1];
      ++nf;
    }
  } else if (bk.face >= 0) {
    const int f = bk.face;
    fa[0] = f;
    fb[0] = f ^ 1;
    c1[0] = 0.25 * A.inv_h[f >> 1];
    c2[0] = -alpha * A.inv_h[f >> 1];
    nf = 1;
  }
  __shared__ double va[kAsmChunk][88], da[kAsmChunk][88], vb[kAsmChunk][88], db[kAsmChunk][88];
  for (int t = 0; t < nf; ++t) {
    const int npts = A.npts[fa[t]];
    long long ba = A.tr_off, bb = B.tr_off;
    for (int g = 0; g < fa[t]; ++g) ba += 2LL * Ja * A.npts[g];
    for (int g = 0; g < fb[t]; ++g) bb += 2LL * Jb * B.npts[g];
    const double* tva = work + ba;
    const double* tda = work + ba + (size_t)Ja * npts;
    const double* tvb = work + bb;
    const double* tdb = work + bb + (size_t)Jb * npts;
    for (int p0 = 0; p0 < npts; p0 += kAsmChunk) {
      __syncthreads();
      for (int x = threadIdx.x; x < kAsmChunk * 88; x += kAsmThreads) {
        const int c = x % kAsmChunk, j = x / kAsmChunk;
        const bool in = p0 + c < npts;
        va[c][j] = (in && j < Ja) ? tva[(size_t)j * npts + p0 + c] : 0.0;
        da[c][j] = (in && j < Ja) ? tda[(size_t)j * npts + p0 + c] : 0.0;
        vb[c][j] = (in && j < Jb) ? tvb[(size_t)j * npts + p0 + c] : 0.0;
        db[c][j] = (in && j < Jb) ? tdb[(size_t)j * npts + p0 + c] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kAsmEntries; ++u) {
        const int ent = threadIdx.x + u * kAsmThreads;
        if (ent >= nent) continue;
        const int i = ent % Ja, j = ent / Ja;
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int c = 0; c < kAsmChunk; ++c) {
          s1 += va[c][i] * db[c][j] + da[c][i] * vb[c][j];
          s2 += va[c][i] * vb[c][j];
        }
        acc[u] += c1[t] * s1 + c2[t] * s2;
      }
    }
  }
  double* out = H + bk.off;
#pragma unroll
  for (int u = 0; u < kAsmEntries; ++u) {
    const int ent = threadIdx.x + u * kAsmThreads;
    if (ent < nent) out[ent] = acc[u];
  }
}

// ---------------------------------------------------------------------------
// host: plan of the work buffer
// ---------------------------------------------------------------------------
static inline long long up32(long long x) { return (x + 31) / 32 * 32; }

int dg_plan(const DgMeshInfo& mi, const std::vector<DgElemShape>& sh, DgPlan& P) {
  const int M = (int)sh.size();
  if (mi.n_mesh[0] < 3 || mi.n_mesh[1] < 3 || (long long)mi.n_mesh[0] * mi.n_mesh[1] != M) {
    set_error("the mesh must be n_mesh[0] x n_mesh[1] = n_elem elements, at least 3 along each axis");
    return DG_ERR_SHAPE;
  }
  P = DgPlan();
  P.el.resize(M);
  const int mx = mi.n_mesh[0], my = mi.n_mesh[1];
  auto at = [&](int k, int dx, int dy) { return ((k % mx + dx + mx) % mx) + mx * ((k / mx + dy + my) % my); };
  // face points must match across every face
  for (int k = 0; k < M; ++k) {
    const DgElemShape& a = sh[k];
    const DgElemShape& xp = sh[at(k, 1, 0)];
    const DgElemShape& yp = sh[at(k, 0, 1)];
    if (a.en[1] != xp.en[1] || a.en[2] != xp.en[2] || a.en[0] != yp.en[0] || a.en[2] != yp.en[2] ||
        a.en[2] != a.n[2] || a.elo[2] != 0 || a.n[0] > 64 || a.n[1] > 64) {
      set_error("element " + std::to_string(k) + ": E_k must span z and match its neighbours along each face");
      return DG_ERR_SHAPE;
    }
    if (a.J > 88) {
      set_error("element " + std::to_string(k) + ": more than 88 ALBs");
      return DG_ERR_SHAPE;
    }
  }
  // blocks: k itself, its four face neighbours, and every element sharing a projector
  std::map<int, std::vector<int>> by_gid;   // global projector id -> elements holding it
  for (int k = 0; k < M; ++k)
    for (int p = 0; p < mi.count[k]; ++p) by_gid[mi.gid[mi.pbase[k] + p]].push_back(k);
  P.row_ptr.assign(M + 1, 0);
  for (int k = 0; k < M; ++k) {
    std::map<int, int> cols;   // nb -> face (-1 none, 0..3, 4 self)
    cols[k] = 4;
    const int fn[4] = {at(k, -1, 0), at(k, 1, 0), at(k, 0, -1), at(k, 0, 1)};
    for (int f = 0; f < 4; ++f) cols.emplace(fn[f], f);
    for (int p = 0; p < mi.count[k]; ++p)
      for (int nb : by_gid[mi.gid[mi.pbase[k] + p]]) cols.emplace(nb, -1);
    std::map<int, int> at_k;
    for (int p = 0; p < mi.count[k]; ++p) at_k[mi.gid[mi.pbase[k] + p]] = p;
    for (const auto& cf : cols) {
      DgBlock bk{};
      bk.k = k;
      bk.nb = cf.first;
      bk.face = cf.second;
      bk.pair_lo = (int)(P.pairs.size() / 2);
      for (int q = 0; q < mi.count[bk.nb]; ++q) {
        auto it = at_k.find(mi.gid[mi.pbase[bk.nb] + q]);
        if (it == at_k.end()) continue;
        P.pairs.push_back(it->second);
        P.pairs.push_back(q);
      }
      bk.pair_hi = (int)(P.pairs.size() / 2);
      bk.off = P.total_values;
      P.total_values += (long long)sh[k].J * sh[bk.nb].J;
      P.blk.push_back(bk);
    }
    P.row_ptr[k + 1] = (long long)P.blk.size();
  }
  long long off = 0;
  P.off_del = off;
  off += up32((long long)(sizeof(DgElem) * M + 7) / 8);
  P.off_blk = off;
  off += up32((long long)(sizeof(DgBlock) * P.blk.size() + 7) / 8);
  P.off_pairs = off;
  off += up32((long long)(P.pairs.size() + 1) / 2);
  long long sumJ = 0;
  for (const DgElemShape& a : sh) sumJ += a.J;
  P.off_sval = off;
  off += up32(sumJ);
  for (int k = 0; k < M; ++k) {
    const DgElemShape& a = sh[k];
    DgElem& D = P.el[k];
    D.J = a.J;
    D.np = mi.count[k];
    for (int q = 0; q < 3; ++q) D.en[q] = a.en[q];
    D.npts[0] = D.npts[1] = a.en[1] * a.en[2];
    D.npts[2] = D.npts[3] = a.en[0] * a.en[2];
    D.inv_h[0] = a.n[0] / a.len[0];
    D.inv_h[1] = a.n[1] / a.len[1];
    D.l_off = off;
    off += up32((long long)a.J * a.J);
    D.tr_off = off;
    off += up32(2LL * a.J * (2LL * D.npts[0] + 2LL * D.npts[2]));
    D.ovl_off = off;
    off += up32((long long)std::max(1, D.np) * a.J);
    D.w_off = off;
    off += up32(4LL * 2 * 64);
    const long long nnz = mi.ptr[mi.pbase[k] + D.np] - mi.ptr[mi.pbase[k]];
    D.pj_off = off;
    off += up32(D.np + 1);
    D.pidx_off = off;
    off += up32((nnz + 1) / 2);
    // gamma (np values) immediately followed by the projector values
    const long long gam = off;
    off += D.np;
    D.pval_off = off;
    off += up32(std::max(1LL, nnz));
    (void)gam;
  }
  P.total_doubles = off + 32;
  return DG_OK;
}

// face interpolation weights (value, derivative along +axis) of the real trigonometric
// interpolant of n samples on a period L at position x: the k = -n/2 term of the sum is
// the Nyquist cosine
static void trig_weights(int n, double L, double x, double* w, double* wd) {
  const double two_pi = 2.0 * M_PI;
  const double theta = two_pi * x / L;
  for (int i = 0; i < n; ++i) {
    double a = 0.0, b = 0.0;
    for (int k = -n / 2; k < n - n / 2; ++k) {
      const double ph = k * (theta - two_pi * i / n);
      a += std::cos(ph);
      b -= (two_pi * k / L) * std::sin(ph);
    }
    w[i] = a / n;
    wd[i] = b / n;
  }
}

int dg_upload(hipStream_t s, const DgMeshInfo& mi, const std::vector<DgElemShape>& sh, const DgPlan& P,
              double* work, std::vector<std::vector<char>>& keep) {
  const int M = (int)sh.size();
  auto put = [&](long long off_doubles, const void* src, size_t bytes) -> int {
    if (!bytes) return DG_OK;
    keep.emplace_back((const char*)src, (const char*)src + bytes);
    DG_HIP(hipMemcpyAsync(work + off_doubles, keep.back().data(), bytes, hipMemcpyHostToDevice, s));
    return DG_OK;
  };
  int st;
  if ((st = put(P.off_del, P.el.data(), sizeof(DgElem) * M))) return st;
  if ((st = put(P.off_blk, P.blk.data(), sizeof(DgBlock) * P.blk.size()))) return st;
  if ((st = put(P.off_pairs, P.pairs.data(), sizeof(int) * P.pairs.size()))) return st;
  for (int k = 0; k < M; ++k) {
    const DgElemShape& a = sh[k];
    const DgElem& D = P.el[k];
    // weights: faces x-, x+ (axis 0), y-, y+ (axis 1); outward derivative sign folded in
    std::vector<double> wt(4 * 2 * 64, 0.0);
    for (int f = 0; f < 4; ++f) {
      const int ax = f >> 1;
      const int n = a.n[ax];
      const double h = a.len[ax] / n;
      const bool plus = f & 1;
      const double x = plus ? (a.elo[ax] + a.en[ax] - 0.5) * h : (a.elo[ax] - 0.5) * h;
      trig_weights(n, a.len[ax], x, &wt[f * 128], &wt[f * 128 + 64]);
      if (!plus)
        for (int i = 0; i < n; ++i) wt[f * 128 + 64 + i] = -wt[f * 128 + 64 + i];
    }
    if ((st = put(D.w_off, wt.data(), sizeof(double) * wt.size()))) return st;
    // projectors on E_k: CSR pointer (rebased), indices, gamma, values
    const int pb = mi.pbase[k];
    const long long p0 = mi.ptr[pb];
    std::vector<long long> ptr(D.np + 1);
    for (int p = 0; p <= D.np; ++p) ptr[p] = mi.ptr[pb + p] - p0;
    if ((st = put(D.pj_off, ptr.data(), sizeof(long long) * ptr.size()))) return st;
    const long long nnz = ptr[D.np];
    for (long long t = 0; t < nnz; ++t)
      if (mi.idx[p0 + t] < 0 || mi.idx[p0 + t] >= a.en[0] * a.en[1] * a.en[2]) {
        set_error("element " + std::to_string(k) + ": projector index outside E_k");
        return DG_ERR_ARG;
      }
    if ((st = put(D.pidx_off, mi.idx + p0, sizeof(int) * nnz))) return st;
    if ((st = put(D.pval_off - D.np, mi.gamma + pb, sizeof(double) * D.np))) return st;
    if ((st = put(D.pval_off, mi.val + p0, sizeof(double) * nnz))) return st;
  }
  return DG_OK;
}

// ---------------------------------------------------------------------------
// host: the element terms of one group
// ---------------------------------------------------------------------------
static int rotate_all_rows(Ctx& c, int src, int dst) {
  RotArgs ra{};
  ra.S = ColSet{1, {src, 0, 0}};
  ra.kS = KC_Jc;
  ra.nout = 1;
  ra.out_blk[0] = dst;
  ra.c0[0] = 0;
  ra.c1[0] = 1;
  ra.alpha = 1.0;
  ra.c_off = small_slot(4);
  ra.ncol = KC_Jc;
  ra.c_blockrows = 1;
  ra.rows_e = 0;
  return launch_rotate(c, DG_FP64, ra);
}

int dg_element_terms(Ctx& c, double* work, const DgElem* del_dev) {
  if (!c.solved) {
    set_error("no solve has completed on this context");
    return DG_ERR_STATE;
  }
  int st;
  ColSet S0{1, {B_T0, 0, 0}};
  // 1. F = X C1 C2 on all rows, with R_E F the orthonormal ALBs
  if ((st = launch_gather_e(c, B_X, B_T0))) return st;
  if ((st = launch_gram_rows(c, DG_FP64, S0, KC_Jc, S0, KC_Jc, small_slot(0), 1, 1))) return st;
  DG_HIP(hipMemsetAsync(c.dev_status, 0, sizeof(int) * c.n_elem, c.stream));
  if ((st = launch_rr(c, 0, KC_Jc, KC_Jc, RR_SVD, nullptr))) return st;
  {
    std::vector<double> sv((size_t)c.off_eig[c.n_elem]);
    double* dsv = work + c.dg_sval_off;
    if ((st = launch_extract_theta(c, dsv))) return st;
    if ((st = sync_read_dg(c, sv.data(), dsv, sizeof(double) * sv.size()))) return st;
    for (int e = 0; e < c.n_elem; ++e) {
      const double smax = sv[c.off_eig[e]], smin = sv[c.off_eig[e + 1] - 1];
      if (!(smin > 1e-10 * smax)) {
        set_error("element " + std::to_string(e + c.elem_base) + ": restriction to E_k is rank deficient");
        return DG_ERR_NUMERIC;
      }
    }
  }
  if ((st = rotate_all_rows(c, B_X, B_T1))) return st;
  if ((st = launch_gather_e(c, B_T1, B_T0))) return st;
  if ((st = launch_gram_rows(c, DG_FP64, S0, KC_Jc, S0, KC_Jc, small_slot(0), 1, 1))) return st;
  if ((st = launch_rr(c, 0, KC_Jc, KC_Jc, RR_CHOLQR, nullptr))) return st;
  {
    std::vector<int> stv(c.n_elem);
    if ((st = sync_read_dg(c, stv.data(), c.dev_status, sizeof(int) * c.n_elem))) return st;
    for (int e = 0; e < c.n_elem; ++e)
      if (stv[e]) {
        set_error("element " + std::to_string(e + c.elem_base) + ": ALB orthonormalisation broke down");
        return DG_ERR_NUMERIC;
      }
  }
  if ((st = rotate_all_rows(c, B_T1, B_W))) return st;   // W = F on Q_k
  int maxJ = 0, maxE = 0, maxnp = 0, maxpts = 0;
  for (int e = 0; e < c.n_elem; ++e) {
    maxJ = std::max(maxJ, c.J[e]);
    maxE = std::max(maxE, c.en[0][e] * c.en[1][e] * c.en[2][e]);
    maxpts = std::max({maxpts, c.en[1][e] * c.en[2][e], c.en[0][e] * c.en[2][e]});
  }
  maxnp = c.dg_max_np;
  // 2. traces of F
  hipLaunchKernelGGL(k_dg_trace, dim3((maxpts * maxJ + 255) / 256, 4, c.n_elem), dim3(256), 0, c.stream,
                     c.elems_dev, del_dev, c.elem_base, (int)B_W, work);
  DG_HIP(hipGetLastError());
  // 3. gradients of F, then E_k's rows of F and of its gradients
  const int gblk[3] = {B_P, B_HW, B_HP};
  if ((st = launch_gradient(c, B_W, gblk))) return st;
  if ((st = launch_gather_e(c, B_W, B_T1))) return st;    // Phi
  if ((st = launch_gather_e(c, B_P, B_T0))) return st;    // d_x Phi
  if ((st = launch_gather_e(c, B_HW, B_HX))) return st;   // d_y Phi
  if ((st = launch_gather_e(c, B_HP, B_W))) return st;    // d_z Phi
  // 4. kinetic Gram of [d_x Phi, d_y Phi, d_z Phi] (slot G) and Phi^T V Phi (slot A)
  ColSet SG{3, {B_T0, B_HX, B_W}};
  if ((st = launch_gram_rows(c, DG_FP64, SG, KC_Jc, SG, KC_Jc, small_slot(0), 1, 1))) return st;
  hipLaunchKernelGGL(k_dg_vphi, dim3((maxE + 255) / 256, maxJ, c.n_elem), dim3(256), 0, c.stream, c.elems_dev,
                     (int)B_T1, (int)B_P);
  DG_HIP(hipGetLastError());
  ColSet SP{1, {B_T1, 0, 0}}, TP{1, {B_P, 0, 0}};
  if ((st = launch_gram_rows(c, DG_FP64, SP, KC_Jc, TP, KC_Jc, small_slot(1), 1, 0))) return st;
  hipLaunchKernelGGL(k_dg_local, dim3((maxJ * maxJ + 255) / 256, c.n_elem), dim3(256), 0, c.stream, c.elems_dev,
                     del_dev, c.elem_base, work);
  DG_HIP(hipGetLastError());
  // 5. projector overlaps over E_k
  if (maxnp > 0) {
    hipLaunchKernelGGL(k_dg_overlap, dim3(maxnp, (maxJ + 15) / 16, c.n_elem), dim3(256), 0, c.stream, c.elems_dev,
                       del_dev, c.elem_base, (int)B_T1, work);
    DG_HIP(hipGetLastError());
  }
  // the work blocks now hold DG data: no solution to take ALBs or vectors from
  c.solved = false;
  return DG_OK;
}

int dg_assemble(hipStream_t s, const DgPlan& P, double* work, double* hdg, double alpha) {
  const DgElem* del = reinterpret_cast<const DgElem*>(work + P.off_del);
  hipLaunchKernelGGL(k_dg_assemble, dim3((unsigned)P.blk.size()), dim3(kAsmThreads), 0, s, del,
                     reinterpret_cast<const DgBlock*>(work + P.off_blk),
                     reinterpret_cast<const int*>(work + P.off_pairs), work, hdg, alpha);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace dg
