// Chebyshev-filtered subspace iteration on H^{Q_k} (Algorithm 2) and the band
// energy through the filter with its adjoint (gradient w.r.t. Psi_0 and V_eff).
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "dg_internal.h"

namespace dg {

int launch_cheb_step(Ctx& c, int prec, int y_blk, int hy_blk, int prev_blk, int k, int ncols, const int* active,
                     const double* bounds);
int launch_adj_step(Ctx& c, int prec, int a1_blk, int t_blk, int a2_blk, int k, int m, int ncols,
                    const double* bounds);
int launch_weighted_dot(Ctx& c, int prec, int u_blk, int w_blk, int ncols, const double* f, double scale,
                        double* E);
int launch_vbar(Ctx& c, int prec, int u_blk, int y_blk, int ncols, const double* f, const double* scale, int k,
                int m, const double* bounds, double beta, double* vbar);
int launch_scale_cols(Ctx& c, int prec, int in_blk, int out_blk, int ncols, const double* f, const double* scale,
                      double mult);
int launch_copy_cols(Ctx& c, int prec, const void* const* src_tab, void* const* dst_tab, int src_blk, int dst_blk,
                     int ncols);

static long long small_code_c(int which) { return -1 - which; }

static int sync_read_c(Ctx& c, void* dst, const void* src, size_t bytes) {
  DG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.stream));
  DG_HIP(hipStreamSynchronize(c.stream));
  return DG_OK;
}

// pick a block from the pool that is none of the excluded ones
static int pick(const std::vector<int>& pool, int x1, int x2, int x3 = -1) {
  for (int b : pool)
    if (b != x1 && b != x2 && b != x3) return b;
  return -1;
}

// ---------------------------------------------------------------------------
// ChFSI: filter X (bounds from the current Ritz values and the upper bound),
// Rayleigh-Ritz on the filtered block (Cholesky of Y^T Y, eigen-solve of the
// projected H), rotation back into X, HX.
// ---------------------------------------------------------------------------
int run_chfsi(Ctx& c, int prec, double tol, int max_iter, int degree, int* iters, int* n_done) {
  if (degree < 1 || degree > 64) {
    set_error("cheb_degree must be in [1, 64]");
    return DG_ERR_ARG;
  }
  int st;
  int* active = c.dev_active;
  c.host_ints.assign(c.n_elem, 1);
  DG_HIP(hipMemcpyAsync(active, c.host_ints.data(), sizeof(int) * c.n_elem, hipMemcpyHostToDevice, c.stream));
  c.active_host.assign(c.n_elem, 1);
  c.rr_pivot_tol = (prec == DG_FP64) ? 1e-13 : 1e-6;
  DG_HIP(hipMemsetAsync(c.dev_count + 2, 0, sizeof(int), c.stream));
  const std::vector<int> pool = {B_W, B_P, B_HW, B_HP, B_T0, B_T1};
  // start: Rayleigh-Ritz on span(X0) gives the first Ritz values (lower bounds)
  auto rr_into_x = [&](int y, int hy) -> int {
    ColSet SY{1, {y, 0, 0}}, SH{1, {hy, 0, 0}};
    int s2;
    if ((s2 = launch_gram(c, prec, SY, 0, SY, 0, small_code_c(0), active, 1))) return s2;
    if ((s2 = launch_gram(c, prec, SY, 0, SH, 0, small_code_c(1), active, 1))) return s2;
    if ((s2 = launch_rr(c, 1, 0, 0, RR_GEN, active))) return s2;
    RotArgs ra{};
    ra.active = active;
    ra.S = SY;
    ra.kS = 0;
    ra.nout = 1;
    ra.out_blk[0] = B_X;
    ra.c0[0] = 0;
    ra.c1[0] = 1;
    ra.alpha = 1.0;
    ra.c_off = small_code_c(4);
    ra.ncol = 0;
    ra.c_blockrows = 1;
    if ((s2 = launch_rotate(c, prec, ra))) return s2;
    ra.S = SH;
    ra.out_blk[0] = B_HX;
    return launch_rotate(c, prec, ra);
  };
  // first RR: copy X0 to a pool block, H it, RR back into X, HX
  if ((st = launch_copy_cols(c, prec, nullptr, nullptr, B_X, B_W, 0))) return st;
  if ((st = launch_hpsi(c, -1, 0, prec, B_W, B_HW, active))) return st;
  if ((st = rr_into_x(B_W, B_HW))) return st;
  std::vector<int> it_elem(c.n_elem, 0);
  int it;
  for (it = 1; it <= max_iter; ++it) {
    if ((st = launch_residual(c, prec, B_X, B_HX, 0, active))) return st;
    if ((st = launch_check(c, active, tol))) return st;
    int cnt[4];
    if ((st = sync_read_c(c, cnt, c.dev_count, sizeof(cnt)))) return st;
    if (cnt[1] > 0) {
      set_error("non-finite residual");
      return DG_ERR_NUMERIC;
    }
    if (it == 1 && cnt[2] > 0) {
      set_error("the start block is rank deficient in " + std::to_string(cnt[2]) +
                " element(s): the Cholesky factorisation of X0^T X0 broke down");
      return DG_ERR_NUMERIC;
    }
    std::vector<int> act(c.n_elem);
    if ((st = sync_read_c(c, act.data(), active, sizeof(int) * c.n_elem))) return st;
    for (int e = 0; e < c.n_elem; ++e)
      if (act[e] > 0) it_elem[e] = it;
    c.active_host = act;
    if (c.log_level > 0) {
      std::vector<double> mr(c.n_elem);
      if ((st = sync_read_c(c, mr.data(), c.dev_maxres, sizeof(double) * c.n_elem))) return st;
      fprintf(stderr, "[dg] chfsi prec=%d it=%d active=%d max_res=%.3e\n", prec, it, cnt[0],
              *std::max_element(mr.begin(), mr.end()));
    }
    if (cnt[0] == 0) break;
    // filter Y_m = p_m(H) X  (Algorithm 2 step 2)
    int prev = -1, cur = B_X;
    for (int k = 0; k < degree; ++k) {
      const int t = pick(pool, prev, cur);
      if ((st = launch_hpsi(c, -1, 0, prec, cur, t, active))) return st;
      if ((st = launch_cheb_step(c, prec, cur, t, prev, k, 0, active, nullptr))) return st;
      prev = cur;
      cur = t;
    }
    // steps 3-5: Rayleigh-Ritz on span(Y_m), rotated into X, HX
    const int h = pick(pool, prev, cur);
    if ((st = launch_hpsi(c, -1, 0, prec, cur, h, active))) return st;
    if ((st = rr_into_x(cur, h))) return st;
  }
  c.active_host.clear();
  c.host_ints.assign(c.n_elem, 1);
  DG_HIP(hipMemcpyAsync(active, c.host_ints.data(), sizeof(int) * c.n_elem, hipMemcpyHostToDevice, c.stream));
  if ((st = launch_residual(c, prec, B_X, B_HX, 0, active))) return st;
  if ((st = launch_check(c, active, tol))) return st;
  int cnt[4];
  if ((st = sync_read_c(c, cnt, c.dev_count, sizeof(cnt)))) return st;
  if (iters)
    for (int e = 0; e < c.n_elem; ++e) iters[e] = it_elem[e];
  *n_done = c.n_elem - cnt[0];
  c.last_breakdowns = cnt[2];
  if (cnt[1] > 0) {
    set_error("non-finite residual");
    return DG_ERR_NUMERIC;
  }
  return DG_OK;
}

// ---------------------------------------------------------------------------
// band energy E = sum_i f_i psi_i^T H psi_i, Psi = p_m(H) Psi_0, and its adjoint
// ---------------------------------------------------------------------------
struct BELayout {
  int nseg, s, m;
  int ck_prev(int j) const { return kMaxBlocks + 2 * j; }      // Y_{js-1}
  int ck_cur(int j) const { return kMaxBlocks + 2 * j + 1; }   // Y_{js}
  int ym() const { return kMaxBlocks + 2 * nseg; }
  int hym() const { return ym() + 1; }
  int seg(int i) const { return hym() + 1 + i; }
};

int band_energy(Ctx& c, int prec, int degree, const double* bounds_host, int n_vec, const void* psi0,
                const double* f, double* E) {
  if (!bounds_host || !psi0 || !f || !E) {
    set_error("bounds, psi0, f and E must be non-NULL");
    return DG_ERR_ARG;
  }
  if (prec != DG_FP64 && prec != DG_FP32) {
    set_error("prec must be DG_FP64 or DG_FP32");
    return DG_ERR_ARG;
  }
  if (degree < 1 || degree > c.max_cheb) {
    set_error("degree must be in [1, max_cheb_degree given at create] (" + std::to_string(c.max_cheb) + ")");
    return DG_ERR_ARG;
  }
  for (int e = 0; e < c.n_elem; ++e)
    if (n_vec <= 0 || n_vec > c.K[e] + (c.K[e] & 1)) {
      set_error("n_vec must be in [1, J_k + guards]");
      return DG_ERR_ARG;
    }
  for (int e = 0; e < c.n_elem; ++e) {
    const double a = bounds_host[3 * e], b = bounds_host[3 * e + 1], a0 = bounds_host[3 * e + 2];
    if (!(b > a) || !(a0 < a)) {
      set_error("bounds must satisfy a0 < a < b for every element");
      return DG_ERR_ARG;
    }
  }
  int st;
  BELayout L{(degree + c.ckpt_stride - 1) / c.ckpt_stride, c.ckpt_stride, degree};
  c.be_bounds_host.assign(bounds_host, bounds_host + 3 * c.n_elem);
  DG_HIP(hipMemcpyAsync(c.dev_bounds, c.be_bounds_host.data(), sizeof(double) * 3 * c.n_elem,
                        hipMemcpyHostToDevice, c.stream));
  const double* bd = c.dev_bounds;
  // Y_0 = Psi_0 into X
  if ((st = launch_copy_ext(c, prec, B_X, psi0, -1, n_vec, 0))) return st;
  if ((st = launch_copy_cols(c, prec, nullptr, nullptr, B_X, L.ck_cur(0), n_vec))) return st;
  const std::vector<int> ypool = {B_X, B_W, B_P};
  int prev = -1, cur = B_X;
  for (int k = 0; k < degree; ++k) {
    const int t = pick(ypool, prev, cur);
    if ((st = launch_hpsi(c, -1, n_vec, prec, cur, t, nullptr))) return st;
    if ((st = launch_cheb_step(c, prec, cur, t, prev, k, n_vec, nullptr, bd))) return st;
    prev = cur;
    cur = t;
    if ((k + 1) % L.s == 0 && k + 1 < degree) {
      const int j = (k + 1) / L.s;
      if ((st = launch_copy_cols(c, prec, nullptr, nullptr, prev, L.ck_prev(j), n_vec))) return st;
      if ((st = launch_copy_cols(c, prec, nullptr, nullptr, cur, L.ck_cur(j), n_vec))) return st;
    }
  }
  if ((st = launch_copy_cols(c, prec, nullptr, nullptr, cur, L.ym(), n_vec))) return st;
  if ((st = launch_hpsi(c, -1, n_vec, prec, L.ym(), L.hym(), nullptr))) return st;
  // f lives on the device (caller buffer)
  if ((st = launch_weighted_dot(c, prec, L.ym(), L.hym(), n_vec, f, 1.0, E))) return st;
  c.be_valid = true;
  c.solved = false;   // the solver blocks now hold filter iterates
  c.have_x = false;
  c.be_degree = degree;
  c.be_prec = prec;
  c.be_nvec = n_vec;
  c.be_f = f;
  return DG_OK;
}

int band_energy_backward(Ctx& c, const double* dE_host, void* dpsi0, void* dv) {
  if (!c.be_valid) {
    set_error("no band energy has been computed on this context");
    return DG_ERR_STATE;
  }
  if (!dE_host || !dpsi0 || !dv) {
    set_error("dE, dpsi0 and dv must be non-NULL");
    return DG_ERR_ARG;
  }
  int st;
  const int prec = c.be_prec, n_vec = c.be_nvec, m = c.be_degree;
  BELayout L{(m + c.ckpt_stride - 1) / c.ckpt_stride, c.ckpt_stride, m};
  const double* bd = c.dev_bounds;
  c.be_de_host.assign(dE_host, dE_host + c.n_elem);
  DG_HIP(hipMemcpyAsync(c.dev_de, c.be_de_host.data(), sizeof(double) * c.n_elem, hipMemcpyHostToDevice,
                        c.stream));
  double* vbar = reinterpret_cast<double*>(dv);
  // A_m = 2 dE H Y_m F ;  Vbar = dE sum_i f_i y_{m,i}^2
  int a1 = B_X, a2 = -1;
  if ((st = launch_scale_cols(c, prec, L.hym(), a1, n_vec, c.be_f, c.dev_de, 2.0))) return st;
  if ((st = launch_vbar(c, prec, L.ym(), L.ym(), n_vec, c.be_f, c.dev_de, -1, m, bd, 0.0, vbar))) return st;
  const std::vector<int> apool = {B_X, B_W, B_P};
  for (int j = L.nseg - 1; j >= 0; --j) {
    const int k0 = j * L.s, k1 = std::min(k0 + L.s, m);
    // recompute Y_{k0} .. Y_{k1-1} from the checkpoint pair of segment j
    if ((st = launch_copy_cols(c, prec, nullptr, nullptr, L.ck_cur(j), L.seg(0), n_vec))) return st;
    for (int i = 1; i < k1 - k0; ++i) {
      const int k = k0 + i - 1;
      const int prv = (i == 1) ? (j == 0 ? -1 : L.ck_prev(j)) : L.seg(i - 2);
      if ((st = launch_hpsi(c, -1, n_vec, prec, L.seg(i - 1), L.seg(i), nullptr))) return st;
      if ((st = launch_cheb_step(c, prec, L.seg(i - 1), L.seg(i), prv, k, n_vec, nullptr, bd))) return st;
    }
    for (int k = k1 - 1; k >= k0; --k) {
      // Vbar += alpha_k sum_i a_{k+1,i} y_{k,i}
      if ((st = launch_vbar(c, prec, a1, L.seg(k - k0), n_vec, nullptr, nullptr, k, m, bd, 1.0, vbar))) return st;
      const int t = pick(apool, a1, a2);
      if ((st = launch_hpsi(c, -1, n_vec, prec, a1, t, nullptr))) return st;
      if ((st = launch_adj_step(c, prec, a1, t, a2, k, m, n_vec, bd))) return st;
      a2 = a1;
      a1 = t;
    }
  }
  // dE/dPsi_0 = A_0 (packed like psi0); the solver blocks hold adjoint iterates now
  c.solved = false;
  c.have_x = false;
  if ((st = launch_copy_ext(c, prec, a1, dpsi0, -1, n_vec, 1))) return st;
  DG_HIP(hipStreamSynchronize(c.stream));
  return DG_OK;
}

}  // namespace dg
