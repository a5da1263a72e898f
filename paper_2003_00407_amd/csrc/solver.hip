// Solver drivers: H*psi on caller buffers, LOBPCG (Algorithm 1), Chebyshev-
// filtered subspace iteration (Algorithm 2 on H^{Q_k}), ALB construction.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include <cstdio>
#include <cstdlib>

#include "dg_internal.h"

namespace dg {

// column-count codes understood by the dense kernels
constexpr int KC_K = 0;    // E.K
constexpr int KC_J = -1;   // E.J

static int sync_read(Ctx& c, void* dst, const void* src, size_t bytes) {
  DG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.stream));
  DG_HIP(hipStreamSynchronize(c.stream));
  return DG_OK;
}

// Small-matrix offsets differ per element (they scale with the element's own
// K), so one launch for all elements passes a slot code that each kernel
// resolves with its element's layout: 0 G, 1 A, 2 U, 3 V, 4 C.
static long long small_code(int which) { return -1 - which; }

int apply_h(Ctx& c, int elem, int n_vec, int prec, const void* x, long long ldx, void* y, long long ldy) {
  if (!x || !y) {
    set_error("x or y is NULL");
    return DG_ERR_ARG;
  }
  if (ldx < 0 || ldy < 0) {
    set_error("ldx and ldy must be >= 0");
    return DG_ERR_ARG;
  }
  for (int e = 0; e < c.n_elem; ++e) {
    if (elem >= 0 && e != elem) continue;
    if ((ldx > 0 && ldx < c.N[e]) || (ldy > 0 && ldy < c.N[e])) {
      set_error("ldx / ldy below the grid size N_k of element " + std::to_string(e + c.elem_base));
      return DG_ERR_ARG;
    }
  }
  if (elem < -1 || elem >= c.n_elem) {
    set_error("elem out of range");
    return DG_ERR_ARG;
  }
  if (prec != DG_FP64 && prec != DG_FP32) {
    set_error("prec must be DG_FP64 or DG_FP32");
    return DG_ERR_ARG;
  }
  for (int e = 0; e < c.n_elem; ++e) {
    if (elem >= 0 && e != elem) continue;
    if (n_vec <= 0 || n_vec > c.K[e] + (c.K[e] & 1)) {
      set_error("n_vec must be in [1, J_k + guards] for every element applied");
      return DG_ERR_ARG;
    }
  }
  int st;
  // copy in (caller layout -> block W), apply W -> HW, copy out; X and the solver's
  // outputs are not touched
  if ((st = launch_copy_ext(c, prec, B_W, x, elem, n_vec, 0, ldx))) return st;
  if ((st = launch_hpsi(c, elem, n_vec, prec, B_W, B_HW, nullptr))) return st;
  if ((st = launch_copy_ext(c, prec, B_HW, y, elem, n_vec, 1, ldy))) return st;
  return DG_OK;
}

// ---------------------------------------------------------------------------
// LOBPCG (Algorithm 1) for every element at once
// ---------------------------------------------------------------------------
// HP' = H P' (P' in p_blk, into hp_blk) for the elements the last Rayleigh-Ritz step
// flagged as nearly dependent (every active element with DG_FRESH_HP=1); the others
// keep the rotated HP' already in hp_blk
static int launch_hp_afresh(Ctx& c, int prec, int p_blk, int hp_blk, const int* active) {
  const int* mask = (c.fresh_hp_all || !c.dev_hpflag) ? active : c.dev_hpflag;
  std::vector<int> saved;
  const bool account = mask == c.dev_hpflag && c.timing && !c.capturing;
  if (account) {
    // per-kernel byte accounting counts the flagged elements only
    std::vector<int> fl(c.n_elem);
    if (int st = sync_read(c, fl.data(), c.dev_hpflag, sizeof(int) * c.n_elem)) return st;
    saved = c.active_host;
    c.active_host = fl;
  }
  const int st = launch_hpsi(c, -1, 0, prec, p_blk, hp_blk, mask);
  if (account) c.active_host = saved;
  return st;
}

static int rr_and_rotate(Ctx& c, int prec, int nb, const int* active, bool lobpcg) {
  int st;
  ColSet S{nb, {B_X, B_W, B_P}};
  ColSet HS{nb, {B_HX, B_HW, B_HP}};
  // S^T S and S^T H S are symmetric (the latter in exact arithmetic): upper tiles, mirrored
  if ((st = launch_gram_pair(c, prec, S, KC_K, HS, KC_K, small_code(1), small_code(0), active))) return st;
  if ((st = launch_rr(c, nb, 0, 0, RR_GEN, active))) return st;
  // X' = S C (-> T0), P' = [W P] C_WP (-> T1); HX' = HS C, HP' = [HW HP] C_WP
  RotArgs ra{};
  ra.active = active;
  ra.S = S;
  ra.kS = KC_K;
  ra.nout = (lobpcg && nb > 1) ? 2 : 1;
  ra.out_blk[0] = B_T0;
  ra.out_blk[1] = B_T1;
  ra.c0[0] = 0;
  ra.c1[0] = nb;
  ra.c0[1] = 1;
  ra.c1[1] = nb;
  ra.beta[0] = ra.beta[1] = 0.0;
  ra.alpha = 1.0;
  ra.c_off = small_code(4);
  ra.c_ld = 0;
  ra.ncol = KC_K;
  ra.c_blockrows = 1;
  if ((st = launch_rotate(c, prec, ra))) return st;
  // X, P are free now: HX' = HS C goes to X and HP' = [HW HP] C_WP to P.  Where the
  // basis was nearly dependent (a scaled overlap pivot below hp_tol), C_WP combines
  // large coefficients that cancel, and the rotated HP' drifts from H P' by the
  // rounding of that cancellation; for those elements (flagged by the Rayleigh-Ritz
  // kernel) HP' = H P' is applied afresh, so that S^T H S stays consistent with S
  const bool two = ra.nout == 2;
  ra.S = HS;
  ra.out_blk[0] = B_X;
  ra.out_blk[1] = B_P;
  if ((st = launch_rotate(c, prec, ra))) return st;
  if (two && (st = launch_hp_afresh(c, prec, B_T1, B_P, active))) return st;
  // new X = T0, P = T1, HX = X, HP = P, T0 = HX, T1 = HP
  int perm[kMaxBlocks] = {B_T0, B_W, B_T1, B_X, B_HW, B_P, B_HX, B_HP};
  return launch_permute(c, perm, active);
}

// reads [active, NaN, Rayleigh-Ritz breakdowns, -] of the last check
static int read_counts(Ctx& c, int* cnt) { return sync_read(c, cnt, c.dev_count, 4 * sizeof(int)); }

// zero the breakdown counter before a stage (outside any captured graph)
static int reset_breakdowns(Ctx& c) {
  DG_HIP(hipMemsetAsync(c.dev_count + 2, 0, sizeof(int), c.stream));
  return DG_OK;
}

// first_stage: the start block is the caller's (or the seeded one); a breakdown of
// its Rayleigh-Ritz step (X_0^T X_0 not positive definite) is an error
static int run_lobpcg(Ctx& c, int prec, double tol, int max_iter, int* iters, int* n_done, bool carry_p = false,
                      int graph_iters = 0, bool first_stage = true) {
  int st;
  int* active = c.dev_active;
  // an FP32 stage stops an element once its residual stops improving (FP32 floor)
  const bool stagnation_exit = (prec != DG_FP64);
  std::vector<double> best(c.n_elem, 1e300);
  std::vector<int> stall(c.n_elem, 0);
  // start: H X, then Rayleigh-Ritz on span(X) (orthonormalises X, step 1)
  {
    std::vector<int> ones(c.n_elem, 1);
    c.host_ints = ones;
    DG_HIP(hipMemcpyAsync(active, c.host_ints.data(), sizeof(int) * c.n_elem, hipMemcpyHostToDevice, c.stream));
  }
  c.active_host.assign(c.n_elem, 1);
  {
    std::vector<int> zeros(c.n_elem, 0);
    c.host_ints2 = zeros;
    DG_HIP(hipMemcpyAsync(c.dev_iters, c.host_ints2.data(), sizeof(int) * c.n_elem, hipMemcpyHostToDevice,
                          c.stream));
  }
  // Gram matrices of FP32 blocks are accurate to ~1e-7: treat smaller scaled pivots as breakdown.
  // W/P columns whose scaled pivot is below drop_tol leave the basis: the projected
  // matrix is then accurate to about eps * ||H|| / drop_tol in the worst kept direction.
  c.rr_pivot_tol = (prec == DG_FP64) ? 1e-13 : 1e-6;
  c.rr_drop_tol = c.rr_drop_env >= 0.0 ? c.rr_drop_env : (prec == DG_FP64 ? 1e-8 : 1e-4);
  c.hp_tol = c.hp_tol_env >= 0.0 ? c.hp_tol_env : (prec == DG_FP64 ? 1e-6 : 1e-3);
  if ((st = reset_breakdowns(c))) return st;
  if ((st = launch_hpsi(c, -1, 0, prec, B_X, B_HX, active))) return st;
  // (the start rotation leaves the block in T1 as P: a carried search direction)
  if ((st = rr_and_rotate(c, prec, 1, active, false))) return st;
  bool have_p = false;
  if (carry_p) {
    if ((st = launch_hpsi(c, -1, 0, prec, B_P, B_HP, active))) return st;
    have_p = true;
  }
  int it = 0;
  // one LOBPCG step after a convergence check: W = T(R), W -= X (X^T W), H W, then the
  // projected problem on S = [X W P] and the rotations (Eqs. (2)-(4), steps 3-7)
  auto step = [&](int nb) -> int {
    int s2;
    // W = T(HX - X Theta)  (Eq. (3), step 3)
    if ((s2 = launch_teter(c, prec, B_X, B_HX, B_W, 0, active))) return s2;
    // W <- W - X (X^T W): optional; the projected problem on [X W P] with its overlap
    // matrix spans the same subspace, and nearly dependent columns leave the basis there
    if (c.orth_w) {
      ColSet SX{1, {B_X, 0, 0}}, SW{1, {B_W, 0, 0}};
      if ((s2 = launch_gram(c, prec, SX, KC_K, SW, KC_K, small_code(2), active, 0))) return s2;
      RotArgs ra{};
      ra.active = active;
      ra.S = SX;
      ra.kS = KC_K;
      ra.nout = 1;
      ra.out_blk[0] = B_W;
      ra.c0[0] = 0;
      ra.c1[0] = 1;
      ra.beta[0] = 1.0;
      ra.alpha = -1.0;
      ra.c_off = small_code(2);
      ra.ncol = KC_K;
      ra.c_blockrows = 1;
      if ((s2 = launch_rotate(c, prec, ra))) return s2;
    }
    // H W
    if ((s2 = launch_hpsi(c, -1, 0, prec, B_W, B_HW, active))) return s2;
    // S = [X, W, P], projected problem (Eq. (4)), rotations (Eq. (2))
    return rr_and_rotate(c, prec, nb, active, true);
  };
  // captured mode: after the first step, graph_iters steps (each followed by the
  // residual and convergence check, which retires converged elements on the device)
  // are one graph; the host reads the counts once per replay
  struct GraphHold {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    void release() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
    }
    ~GraphHold() { release(); }
  } gh;
  hipGraphExec_t& gexec = gh.exec;
  hipGraph_t& graph = gh.graph;
  auto release_graph = [&]() { gh.release(); };
  const bool use_graph = graph_iters > 0 && !stagnation_exit && c.log_level == 0;
  bool checked = false;   // a graph replay ended with the residual and check
  for (it = 1; it <= max_iter; ++it) {
    if (!checked) {
      if ((st = launch_residual(c, prec, B_X, B_HX, 0, active))) return st;
      if ((st = launch_check(c, active, tol))) return st;
    }
    checked = false;
    int cnt[4];
    if ((st = read_counts(c, cnt))) return st;
    if (cnt[1] > 0) {
      set_error("non-finite residual in " + std::to_string(cnt[1]) + " element(s)");
      return DG_ERR_NUMERIC;
    }
    if (it == 1 && first_stage && cnt[2] > 0) {
      set_error("the start block is rank deficient in " + std::to_string(cnt[2]) +
                " element(s): the Cholesky factorisation of X0^T X0 broke down");
      return DG_ERR_NUMERIC;
    }
    {
      std::vector<int> act(c.n_elem);
      if ((st = sync_read(c, act.data(), active, sizeof(int) * c.n_elem))) return st;
      if (stagnation_exit) {
        std::vector<double> mr(c.n_elem);
        if ((st = sync_read(c, mr.data(), c.dev_maxres, sizeof(double) * c.n_elem))) return st;
        bool changed = false;
        for (int e = 0; e < c.n_elem; ++e) {
          if (act[e] <= 0) continue;
          if (mr[e] < 0.8 * best[e]) {
            best[e] = mr[e];
            stall[e] = 0;
          } else if (++stall[e] >= 6) {
            act[e] = 0;
            changed = true;
            --cnt[0];
          }
        }
        if (changed) {
          c.host_ints = act;
          DG_HIP(hipMemcpyAsync(active, c.host_ints.data(), sizeof(int) * c.n_elem, hipMemcpyHostToDevice,
                                c.stream));
        }
      }
      c.active_host = act;
    }
    if (c.log_level > 0) {
      std::vector<double> mr(c.n_elem);
      std::vector<int> stv(c.n_elem);
      if ((st = sync_read(c, mr.data(), c.dev_maxres, sizeof(double) * c.n_elem))) return st;
      if ((st = sync_read(c, stv.data(), c.dev_status, sizeof(int) * c.n_elem))) return st;
      double m = 0.0;
      int brk = 0;
      for (int e = 0; e < c.n_elem; ++e) {
        m = std::max(m, mr[e]);
        brk += stv[e] != 0;
      }
      fprintf(stderr, "[dg] lobpcg prec=%d it=%d active=%d max_res=%.3e rr_fallbacks=%d\n", prec, it, cnt[0], m, brk);
      if (c.log_level >= 3) {
        std::vector<double> pv(3 * c.n_elem);
        if ((st = sync_read(c, pv.data(), c.dev_minpiv, 3 * sizeof(double) * c.n_elem))) return st;
        for (int e = 0; e < c.n_elem; ++e)
          fprintf(stderr, " %.1e/%d/%.0e@%d-%d", mr[e], stv[e], pv[3 * e], (int)pv[3 * e + 1], (int)pv[3 * e + 2]);
        fprintf(stderr, "\n");
      }
      if (c.log_level >= 2 && it % 10 == 1) {
        std::vector<long long> ph(16 * c.n_elem);
        if ((st = sync_read(c, ph.data(), c.dev_phase, sizeof(long long) * 16 * c.n_elem))) return st;
        // wall clock at 100 MHz; the element whose step took longest
        static const char* names[9] = {"chol", "zinv", "matmul", "tridiag", "bisect", "invit", "mgs", "back",
                                       "coeff"};
        int es = 0;
        for (int e = 1; e < c.n_elem; ++e)
          if (ph[16 * e + 9] - ph[16 * e] > ph[16 * es + 9] - ph[16 * es]) es = e;
        fprintf(stderr, "[dg] rr phases (us), element %d of order %d:", es, 3 * c.K[es]);
        for (int k = 0; k < 9; ++k) fprintf(stderr, " %s %.0f", names[k], (ph[16 * es + k + 1] - ph[16 * es + k]) / 100.0);
        fprintf(stderr, "\n");
      }
    }
    if (cnt[0] == 0) break;
    if (use_graph && have_p) {
      if (!gexec) {
        c.capturing = true;
        hipError_t ce = hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal);
        int s3 = ce == hipSuccess ? DG_OK : DG_ERR_HIP;
        for (int g = 0; g < graph_iters && s3 == DG_OK; ++g) {
          s3 = step(3);
          if (s3 == DG_OK) s3 = launch_residual(c, prec, B_X, B_HX, 0, active);
          if (s3 == DG_OK) s3 = launch_check(c, active, tol);
        }
        hipError_t ee = ce == hipSuccess ? hipStreamEndCapture(c.stream, &graph) : ce;
        c.capturing = false;
        if (s3 != DG_OK) return s3;
        if (ee != hipSuccess) {
          set_error(std::string("stream capture: ") + hipGetErrorString(ee));
          return DG_ERR_HIP;
        }
        if (hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
          release_graph();
          set_error("hipGraphInstantiate failed");
          return DG_ERR_HIP;
        }
      }
      {
        TimedScope ts(c, TC_OTHER);
        if (hipGraphLaunch(gexec, c.stream) != hipSuccess) {
          release_graph();
          set_error("hipGraphLaunch failed");
          return DG_ERR_HIP;
        }
      }
      it += graph_iters - 1;
      checked = true;
      continue;
    }
    if ((st = step(have_p ? 3 : 2))) return st;
    have_p = true;
  }
  c.active_host.clear();
  // final residuals for reporting (every element)
  {
    std::vector<int> ones(c.n_elem, 1);
    c.host_ints = ones;
    DG_HIP(hipMemcpyAsync(active, c.host_ints.data(), sizeof(int) * c.n_elem, hipMemcpyHostToDevice, c.stream));
  }
  release_graph();
  // iterations per element (counted by the check kernel before the final check)
  if (iters && (st = sync_read(c, iters, c.dev_iters, sizeof(int) * c.n_elem))) return st;
  if ((st = launch_residual(c, prec, B_X, B_HX, 0, active))) return st;
  if ((st = launch_check(c, active, tol))) return st;
  int cnt[4];
  if ((st = read_counts(c, cnt))) return st;
  *n_done = c.n_elem - cnt[0];
  if (cnt[1] > 0) {
    set_error("non-finite residual in " + std::to_string(cnt[1]) + " element(s)");
    return DG_ERR_NUMERIC;
  }
  // a breakdown mid-run keeps X for that iteration (C = [I; 0; 0]); it is an error
  // only when the element then fails to converge (checked by the caller's last stage)
  c.last_breakdowns = cnt[2];
  return DG_OK;
}

// Mixed refinement after the FP32 stage (LOBPCG).  X and HX stay FP64; the search
// blocks W, P and their images HW, HP are FP32 (FP32 H*psi and preconditioner, Grams
// and rotations on FP32 matrix cores).  The projected problem takes the FP64
// residual R = HX - X Theta, rounded to FP32, in place of HX (k_mixed_fix), so FP32
// rounding perturbs each correction only relative to its own size; X' = X C_X + P'
// is an FP64 rotation plus the FP32 P', and HX' = H X' is applied in FP64.  At the
// end an FP64 Rayleigh-Ritz step on span(X) restores an orthonormal FP64 Ritz basis;
// elements whose residual is then above tol continue.
static int run_mixed_refine(Ctx& c, double tol, int max_iter, int* iters, int* n_done) {
  int st;
  int* active = c.dev_active;
  auto activate_all = [&]() -> int {
    std::vector<int> ones(c.n_elem, 1);
    c.host_ints = ones;
    DG_HIP(hipMemcpyAsync(active, c.host_ints.data(), sizeof(int) * c.n_elem, hipMemcpyHostToDevice, c.stream));
    c.active_host.assign(c.n_elem, 1);
    return DG_OK;
  };
  if ((st = activate_all())) return st;
  {
    std::vector<int> zeros(c.n_elem, 0);
    c.host_ints2 = zeros;
    DG_HIP(hipMemcpyAsync(c.dev_iters, c.host_ints2.data(), sizeof(int) * c.n_elem, hipMemcpyHostToDevice,
                          c.stream));
  }
  // X columns have an exact unit overlap here.  W/P columns carry FP32 Gram rounding,
  // which shifts the Rayleigh quotient of a direction with scaled pivot p by about
  // eps_32 ||H|| / p: below p = 1e-3 such a direction can pose as a wanted eigenpair
  // (measured on C4: 1e-5 and 1e-4 let single elements diverge), so it leaves the basis
  c.rr_pivot_tol = 1e-13;
  c.rr_drop_tol = c.rr_drop_refine_env >= 0.0 ? c.rr_drop_refine_env : 1e-3;
  c.hp_tol = c.hp_tol_env >= 0.0 ? c.hp_tol_env : 1e-3;
  if ((st = reset_breakdowns(c))) return st;
  // start: H X in FP64, Rayleigh-Ritz on span(X); the carried FP32 P (in T1) becomes P
  if ((st = launch_hpsi(c, -1, 0, DG_FP64, B_X, B_HX, active))) return st;
  if ((st = rr_and_rotate(c, DG_FP64, 1, active, false))) return st;
  if ((st = launch_hpsi(c, -1, 0, DG_FP32, B_P, B_HP, active))) return st;
  bool have_p = true;
  auto step = [&](int nb) -> int {
    int s2;
    // R = HX - X Theta (into T0) and X (into T1), FP32
    if ((s2 = launch_mixed_split(c, B_X, B_HX, B_T0, B_T1, active))) return s2;
    // W = T(R), H W
    if ((s2 = launch_teter(c, DG_FP32, B_T0, B_T0, B_W, 0, active, true))) return s2;
    if ((s2 = launch_hpsi(c, -1, 0, DG_FP32, B_W, B_HW, active))) return s2;
    // FP32 Grams of S' = [W P X] with [S' | T'], T' = [HW HP R], then the projected matrices
    ColSet S = nb == 3 ? ColSet{3, {B_W, B_P, B_T1}} : ColSet{2, {B_W, B_T1, 0}};
    ColSet T = nb == 3 ? ColSet{3, {B_HW, B_HP, B_T0}} : ColSet{2, {B_HW, B_T0, 0}};
    if ((s2 = launch_gram_pair(c, DG_FP32, S, KC_K, T, KC_K, small_code(2), small_code(3), active))) return s2;
    if ((s2 = launch_mixed_fix(c, nb, active))) return s2;
    if ((s2 = launch_rr(c, nb, 0, 0, RR_GEN, active))) return s2;
    // P' = [W P] C_WP into T1, HP' = [HW HP] C_WP into T0 (FP32)
    RotArgs ra{};
    ra.active = active;
    ra.kS = KC_K;
    ra.nout = 1;
    ra.c0[0] = 1;
    ra.c1[0] = nb;
    ra.alpha = 1.0;
    ra.c_off = small_code(4);
    ra.ncol = KC_K;
    ra.c_blockrows = 1;
    ra.S = ColSet{nb, {B_X, B_W, B_P}};
    ra.out_blk[0] = B_T1;
    if ((s2 = launch_rotate(c, DG_FP32, ra))) return s2;
    ra.S = ColSet{nb, {B_HX, B_HW, B_HP}};
    ra.out_blk[0] = B_T0;
    if ((s2 = launch_rotate(c, DG_FP32, ra))) return s2;
    // H P' afresh (FP32) where the basis was nearly dependent
    if ((s2 = launch_hp_afresh(c, DG_FP32, B_T1, B_T0, active))) return s2;
    // X' = X C_X + P' into W (FP64)
    RotArgs rx{};
    rx.active = active;
    rx.kS = KC_K;
    rx.nout = 1;
    rx.c0[0] = 0;
    rx.c1[0] = 1;
    rx.beta[0] = 1.0;
    rx.alpha = 1.0;
    rx.c_off = small_code(4);
    rx.ncol = KC_K;
    rx.c_blockrows = 1;
    rx.add32 = 1;
    rx.S = ColSet{1, {B_X, 0, 0}};
    rx.out_blk[0] = B_W;
    rx.add32_blk[0] = B_T1;
    if ((s2 = launch_rotate(c, DG_FP64, rx))) return s2;
    // HX' = H X' applied afresh in FP64, so HX stays exact and FP32 rounding stays in
    // the search blocks (measured on C4: a rotated HX' = HX C_X + HP' gathers the FP32
    // rounding of HP' step after step and stalls hard elements near 5e-8, and even with
    // a refresh whenever the residual fell tenfold single elements diverged)
    if ((s2 = launch_hpsi(c, -1, 0, DG_FP64, B_W, B_HW, active))) return s2;
    // new X = W, HX = HW, P = T1, HP = T0; the other blocks are free
    int perm[kMaxBlocks] = {B_W, B_P, B_T1, B_HW, B_HP, B_T0, B_X, B_HX};
    return launch_permute(c, perm, active);
  };
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    if ((st = launch_residual(c, DG_FP64, B_X, B_HX, 0, active))) return st;
    if ((st = launch_check(c, active, tol))) return st;
    int cnt[4];
    if ((st = read_counts(c, cnt))) return st;
    if (cnt[1] > 0) {
      set_error("non-finite residual in " + std::to_string(cnt[1]) + " element(s)");
      return DG_ERR_NUMERIC;
    }
    if (cnt[0] == 0) {
      // every element converged: an FP64 Rayleigh-Ritz step on span(X) (HX = H X is
      // exact) gives the orthonormal Ritz basis, whose residuals are checked again
      if ((st = activate_all())) return st;
      if ((st = rr_and_rotate(c, DG_FP64, 1, active, false))) return st;
      have_p = false;   // the Rayleigh-Ritz step on span(X) leaves no search direction
      if ((st = launch_residual(c, DG_FP64, B_X, B_HX, 0, active))) return st;
      if ((st = launch_check(c, active, tol))) return st;
      if ((st = read_counts(c, cnt))) return st;
      if (c.log_level > 0) fprintf(stderr, "[dg] mixed refine it=%d: %d element(s) above tol after the FP64 Rayleigh-Ritz step\n", it, cnt[0]);
      if (cnt[0] == 0) break;
    }
    {
      std::vector<int> act(c.n_elem);
      if ((st = sync_read(c, act.data(), active, sizeof(int) * c.n_elem))) return st;
      c.active_host = act;
    }
    if (c.log_level > 0) {
      std::vector<double> mr(c.n_elem);
      if ((st = sync_read(c, mr.data(), c.dev_maxres, sizeof(double) * c.n_elem))) return st;
      double m = 0.0;
      for (int e = 0; e < c.n_elem; ++e) m = std::max(m, c.active_host[e] ? mr[e] : 0.0);
      fprintf(stderr, "[dg] mixed refine it=%d active=%d max_res=%.3e\n", it, cnt[0], m);
    }
    if ((st = step(have_p ? 3 : 2))) return st;
    have_p = true;
  }
  c.active_host.clear();
  if ((st = activate_all())) return st;
  c.active_host.clear();
  if (iters && (st = sync_read(c, iters, c.dev_iters, sizeof(int) * c.n_elem))) return st;
  if ((st = launch_residual(c, DG_FP64, B_X, B_HX, 0, active))) return st;
  if ((st = launch_check(c, active, tol))) return st;
  int cnt[4];
  if ((st = read_counts(c, cnt))) return st;
  *n_done = c.n_elem - cnt[0];
  if (cnt[1] > 0) {
    set_error("non-finite residual in " + std::to_string(cnt[1]) + " element(s)");
    return DG_ERR_NUMERIC;
  }
  c.last_breakdowns = cnt[2];
  return DG_OK;
}

int run_chfsi(Ctx& c, int prec, double tol, int max_iter, int degree, int* iters, int* n_done);

int solve(Ctx& c, const dg_solve_params* p, double* eig, double* resid, int* iters) {
  if (!p || !eig || !resid) {
    set_error("params, eig_dev and resid_dev must be non-NULL");
    return DG_ERR_ARG;
  }
  if (p->method != DG_LOBPCG && p->method != DG_CHFSI) {
    set_error("unknown method");
    return DG_ERR_ARG;
  }
  if (p->precision != DG_FP64 && p->precision != DG_MIXED) {
    set_error("precision must be DG_FP64 or DG_MIXED");
    return DG_ERR_ARG;
  }
  if (!(p->tol > 0.0) || p->max_iter <= 0) {
    set_error("tol must be > 0 and max_iter > 0");
    return DG_ERR_ARG;
  }
  if (p->warm_start && !c.have_x) {
    set_error("warm_start needs the vectors of an earlier solve on this context (none, or overwritten by a "
              "band-energy call)");
    return DG_ERR_STATE;
  }
  int st;
  std::vector<int> it1(c.n_elem, 0), it2(c.n_elem, 0);
  int done = 0;
  // the band energy's checkpoints are overwritten from here on
  c.be_valid = false;
  c.solved = false;
  const bool warm = p->warm_start != 0;
  // start block into X in the precision of the first stage: the caller's x0, the
  // seeded device draw, or (warm) the FP64 X of the last solve
  const int prec0 = p->precision == DG_FP64 ? DG_FP64 : DG_FP32;
  c.have_x = false;
  if (warm) {
    if (prec0 == DG_FP32) {
      if ((st = launch_convert(c, B_X, DG_FP64, B_W, DG_FP32, KC_K))) return st;
      int perm[kMaxBlocks] = {B_W, B_X, B_P, B_HX, B_HW, B_HP, B_T0, B_T1};
      if ((st = launch_permute(c, perm, nullptr))) return st;
    }
  } else if (p->x0_dev) {
    if ((st = launch_copy_packed(c, prec0, B_X, p->x0_dev, c.dev_off_x0, KC_K, 0))) return st;
  } else {
    if ((st = launch_random_block(c, prec0, B_X, (unsigned long long)p->seed))) return st;
  }
  c.last_breakdowns = 0;
  if (p->precision == DG_FP64) {
    st = p->method == DG_LOBPCG ? run_lobpcg(c, DG_FP64, p->tol, p->max_iter, it1.data(), &done, false,
                                             std::max(0, p->graph_iters))
                                : run_chfsi(c, DG_FP64, p->tol, p->max_iter, p->cheb_degree, it1.data(), &done);
    if (st < 0) return st;
  } else {
    const double tmp = p->tol_mixed > 0.0 ? p->tol_mixed : 3e-5;
    st = p->method == DG_LOBPCG ? run_lobpcg(c, DG_FP32, std::max(tmp, p->tol), p->max_iter, it1.data(), &done)
                                : run_chfsi(c, DG_FP32, std::max(tmp, p->tol), p->max_iter, p->cheb_degree,
                                            it1.data(), &done);
    if (st < 0) return st;
    // promote X (into W's storage) to FP64
    if ((st = launch_convert(c, B_X, DG_FP32, B_W, DG_FP64, KC_K))) return st;
    const bool carry = p->method == DG_LOBPCG;
    if (carry && c.mixed_refine) {
      // the FP32 search direction P moves to T1 (the start rotation turns T1 into P)
      int perm[kMaxBlocks] = {B_W, B_X, B_T1, B_HX, B_HW, B_HP, B_T0, B_P};
      if ((st = launch_permute(c, perm, nullptr))) return st;
      st = run_mixed_refine(c, p->tol, p->max_iter, it2.data(), &done);
      if (st < 0) return st;
    } else {
      // and, for LOBPCG, the last search direction P (into T1, which the start rotation
      // turns into P), then FP64 refinement sweeps
      if (carry && (st = launch_convert(c, B_P, DG_FP32, B_T1, DG_FP64, KC_K))) return st;
      int perm[kMaxBlocks] = {B_W, B_X, B_P, B_HX, B_HW, B_HP, B_T0, B_T1};
      if ((st = launch_permute(c, perm, nullptr))) return st;
      st = run_lobpcg(c, DG_FP64, p->tol, p->max_iter, it2.data(), &done, carry, std::max(0, p->graph_iters),
                      false);
      if (st < 0) return st;
    }
  }
  if (done < c.n_elem && c.last_breakdowns > 0) {
    set_error(std::to_string(c.n_elem - done) + " element(s) did not converge after " +
              std::to_string(c.last_breakdowns) + " Rayleigh-Ritz breakdown(s) of the X block");
    return DG_ERR_NUMERIC;
  }
  c.solved = true;
  c.have_x = true;
  // outputs: theta, residuals of the J wanted states
  if ((st = launch_extract_eig(c, eig, resid))) return st;
  if (iters)
    for (int e = 0; e < c.n_elem; ++e) iters[e] = it1[e] + it2[e];
  DG_HIP(hipStreamSynchronize(c.stream));
  return done == c.n_elem ? DG_OK : DG_WARN_NOT_CONVERGED;
}

int get_ritz(Ctx& c, double* theta, double* resid) {
  if (!c.solved) {
    set_error("no solve has completed on this context");
    return DG_ERR_STATE;
  }
  if (!theta || !resid) {
    set_error("theta_dev and resid_dev must be non-NULL");
    return DG_ERR_ARG;
  }
  return launch_extract_kall(c, theta, resid);
}

int get_vectors(Ctx& c, double* x) {
  if (!c.solved) {
    set_error("no solve has completed on this context");
    return DG_ERR_STATE;
  }
  if (!x) {
    set_error("x_dev is NULL");
    return DG_ERR_ARG;
  }
  return launch_copy_packed(c, DG_FP64, B_X, x, c.dev_off_vec, KC_J, 1);
}

// ALB: gather E_k rows, SVD by eigen-decomposition of the Gram (twice)
int make_alb(Ctx& c, double* alb, double* sval) {
  if (!c.solved) {
    set_error("no solve has completed on this context");
    return DG_ERR_STATE;
  }
  if (!alb || !sval) {
    set_error("alb_dev and sval_dev must be non-NULL");
    return DG_ERR_ARG;
  }
  int st;
  const int X = B_X, t0 = B_T0, t1 = B_T1;
  if ((st = launch_gather_e(c, X, t0))) return st;
  ColSet S0{1, {t0, 0, 0}}, S1{1, {t1, 0, 0}};
  if ((st = launch_gram_rows(c, DG_FP64, S0, KC_J, S0, KC_J, small_code(0), 1, 1))) return st;
  DG_HIP(hipMemsetAsync(c.dev_status, 0, sizeof(int) * c.n_elem, c.stream));
  if ((st = launch_rr(c, 0, KC_J, KC_J, RR_SVD, nullptr))) return st;
  if ((st = launch_extract_theta(c, sval))) return st;
  // rank of the restriction: sigma_min <= 1e-10 sigma_max leaves no orthonormal
  // basis of the restricted span at working precision
  {
    std::vector<double> sv((size_t)c.off_eig[c.n_elem]);
    if ((st = sync_read(c, sv.data(), sval, sizeof(double) * sv.size()))) return st;
    for (int e = 0; e < c.n_elem; ++e) {
      const double smax = sv[c.off_eig[e]], smin = sv[c.off_eig[e + 1] - 1];
      if (!(smin > 1e-10 * smax)) {
        char buf[160];
        snprintf(buf, sizeof(buf), "element %d: restriction to E_k is rank deficient (sigma_min %.3e, sigma_max %.3e)",
                 e + c.elem_base, smin, smax);
        set_error(buf);
        return DG_ERR_NUMERIC;
      }
    }
  }
  RotArgs ra{};
  ra.S = S0;
  ra.kS = KC_J;
  ra.nout = 1;
  ra.out_blk[0] = t1;
  ra.c0[0] = 0;
  ra.c1[0] = 1;
  ra.alpha = 1.0;
  ra.c_off = small_code(4);
  ra.ncol = KC_J;
  ra.c_blockrows = 1;
  ra.rows_e = 1;
  if ((st = launch_rotate(c, DG_FP64, ra))) return st;
  // second pass (Cholesky QR) restores orthonormality to working precision
  if ((st = launch_gram_rows(c, DG_FP64, S1, KC_J, S1, KC_J, small_code(0), 1, 1))) return st;
  if ((st = launch_rr(c, 0, KC_J, KC_J, RR_CHOLQR, nullptr))) return st;
  {
    std::vector<int> stv(c.n_elem);
    if ((st = sync_read(c, stv.data(), c.dev_status, sizeof(int) * c.n_elem))) return st;
    for (int e = 0; e < c.n_elem; ++e)
      if (stv[e] != 0) {
        set_error("element " + std::to_string(e + c.elem_base) +
                  ": the Cholesky-QR pass of the ALB orthonormalisation broke down");
        return DG_ERR_NUMERIC;
      }
  }
  ra.S = S1;
  ra.out_blk[0] = t0;
  if ((st = launch_rotate(c, DG_FP64, ra))) return st;
  if ((st = launch_copy_rows_out(c, t0, alb))) return st;
  DG_HIP(hipStreamSynchronize(c.stream));
  return DG_OK;
}

}  // namespace dg

