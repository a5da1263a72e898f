// Host runtime: arena plan, element staging, solver drivers.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "dg_internal.h"

namespace dg {

static thread_local std::string g_err;
void set_error(const std::string& s) { g_err = s; }
const char* get_error() { return g_err.c_str(); }

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static hipEvent_t get_event(Ctx& c) {
  if (!c.event_pool.empty()) {
    hipEvent_t e = c.event_pool.back();
    c.event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

TimedScope::TimedScope(Ctx& ctx, int k, double w) : c(ctx), cls(k), work(w) {
  if (!c.timing || c.capturing) return;
  a = get_event(c);
  b = get_event(c);
  if (a) hipEventRecord(a, c.stream);
}

TimedScope::~TimedScope() {
  if (!c.timing || c.capturing || !a || !b) return;
  hipEventRecord(b, c.stream);
  c.pending.push_back({cls, a, b});
  c.tacc.work[cls] += work;
  if (c.pending.size() > 20000) resolve_timing(c);
}

int resolve_timing(Ctx& c) {
  if (c.pending.empty()) return DG_OK;
  DG_HIP(hipStreamSynchronize(c.stream));
  for (const PendingTime& p : c.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c.tacc.ms[p.cls] += ms;
      c.tacc.launches[p.cls] += 1;
    }
    c.event_pool.push_back(p.a);
    c.event_pool.push_back(p.b);
  }
  c.pending.clear();
  return DG_OK;
}

// ---------------------------------------------------------------------------
// host-side projector preprocessing: groups of projectors with one support,
// and the transposed (grid-point-major) entry lists.
// ---------------------------------------------------------------------------
struct ProjPlan {
  std::vector<int> sptr, pbase, idx;
  std::vector<double> val;          // group-major: for group g, q*len + s
  std::vector<long long> vbase;
  std::vector<int> act_idx, act_ptr, ent_proj;
  std::vector<double> ent_val;
};

static int build_proj_plan(const dg_element_desc& d, int N, ProjPlan& P) {
  P = ProjPlan();
  P.sptr.push_back(0);
  P.pbase.push_back(0);
  int p = 0;
  while (p < d.n_proj) {
    const int64_t a = d.proj_ptr[p], b = d.proj_ptr[p + 1];
    const int len = int(b - a);
    int q = p + 1;
    while (q < d.n_proj && q - p < 4) {
      const int64_t a2 = d.proj_ptr[q], b2 = d.proj_ptr[q + 1];
      if (b2 - a2 != len || std::memcmp(d.proj_idx + a, d.proj_idx + a2, sizeof(int32_t) * len) != 0)
        break;
      ++q;
    }
    P.vbase.push_back((long long)P.val.size());
    for (int s = 0; s < len; ++s) P.idx.push_back(d.proj_idx[a + s]);
    for (int r = p; r < q; ++r)
      for (int s = 0; s < len; ++s) P.val.push_back(d.proj_val[d.proj_ptr[r] + s]);
    P.sptr.push_back((int)P.idx.size());
    P.pbase.push_back(q);
    p = q;
  }
  // transposed lists
  std::vector<int> cnt(N, 0);
  for (int r = 0; r < d.n_proj; ++r)
    for (int64_t t = d.proj_ptr[r]; t < d.proj_ptr[r + 1]; ++t) cnt[d.proj_idx[t]]++;
  std::vector<int> slot(N, -1);
  P.act_ptr.push_back(0);
  for (int i = 0; i < N; ++i)
    if (cnt[i]) {
      slot[i] = (int)P.act_idx.size();
      P.act_idx.push_back(i);
      P.act_ptr.push_back(P.act_ptr.back() + cnt[i]);
    }
  P.ent_proj.assign(P.act_ptr.back(), 0);
  P.ent_val.assign(P.act_ptr.back(), 0.0);
  std::vector<int> fill(P.act_idx.size(), 0);
  for (int r = 0; r < d.n_proj; ++r)
    for (int64_t t = d.proj_ptr[r]; t < d.proj_ptr[r + 1]; ++t) {
      const int a = slot[d.proj_idx[t]];
      const int o = P.act_ptr[a] + fill[a]++;
      P.ent_proj[o] = r;
      P.ent_val[o] = d.proj_val[t];
    }
  return DG_OK;
}

// ---------------------------------------------------------------------------
// arena plan (CPU only)
// ---------------------------------------------------------------------------
struct ElemPlan {
  int J, G, K, Kpad, N, ld, kmax3, KP;
  size_t off_v64, off_v32, off_sptr, off_pbase, off_idx, off_val64, off_val32, off_vbase, off_gamma;
  size_t off_act_idx, off_act_ptr, off_ent_proj, off_ent_v64, off_ent_v32;
  size_t off_blk[kTotalBlocks];
  int n_blocks;
  size_t off_small, off_nlc;
  int ngrp, nact, nent;
};

struct Plan {
  std::vector<ElemPlan> el;
  size_t off_elems, off_iota, off_active, off_status, off_count, off_iters, off_maxres, off_phase, off_bounds,
      off_de,
      off_minpiv, off_hpflag;
  int n_extra;
  size_t off_offx0, off_offvec, off_offalb, off_offgrid, off_offeig, off_offkall, off_offelem, off_offjj,
      off_nprojoff, off_lists;
  size_t off_ckpt, off_part;
  size_t ckpt_block_bytes;
  int n_ckpt;
  int part_ld, nsplit_max;
  size_t part_stride;
  size_t total;
  std::vector<ProjPlan> proj;
};

static int validate(int n_elem, const dg_element_desc* d) {
  if (n_elem <= 0 || !d) {
    set_error("n_elem must be positive and elems non-NULL");
    return DG_ERR_ARG;
  }
  for (int e = 0; e < n_elem; ++e) {
    const dg_element_desc& x = d[e];
    if (!grid_supported(x.n[0], x.n[1], x.n[2])) {
      set_error("element " + std::to_string(e) + ": unsupported grid " + std::to_string(x.n[0]) + "x" +
                std::to_string(x.n[1]) + "x" + std::to_string(x.n[2]) +
                " (need nx == ny, each of 8,12,16,24,32,48,64)");
      return DG_ERR_SHAPE;
    }
    for (int a = 0; a < 3; ++a) {
      if (!(x.len[a] > 0.0)) {
        set_error("element " + std::to_string(e) + ": box length must be positive");
        return DG_ERR_ARG;
      }
      if (x.elem_n[a] <= 0 || x.elem_lo[a] < 0 || x.elem_lo[a] + x.elem_n[a] > x.n[a]) {
        set_error("element " + std::to_string(e) + ": E_k box outside Q_k");
        return DG_ERR_ARG;
      }
    }
    const int N = x.n[0] * x.n[1] * x.n[2];
    if (x.n_states <= 0 || x.n_states > N / 2) {
      set_error("element " + std::to_string(e) + ": n_states out of range");
      return DG_ERR_ARG;
    }
    // J_k ALBs on E_k need at least J_k grid points there: the restriction of J_k
    // eigenvectors to fewer points is rank deficient by construction
    const long long ne = (long long)x.elem_n[0] * x.elem_n[1] * x.elem_n[2];
    if (x.n_states > ne) {
      set_error("element " + std::to_string(e) + ": n_states " + std::to_string(x.n_states) +
                " exceeds the " + std::to_string(ne) + " grid points of E_k (the ALBs would be rank deficient)");
      return DG_ERR_SHAPE;
    }
    if (!x.v_eff) {
      set_error("element " + std::to_string(e) + ": v_eff is NULL");
      return DG_ERR_ARG;
    }
    for (int i = 0; i < N; ++i)
      if (!std::isfinite(x.v_eff[i])) {
        set_error("element " + std::to_string(e) + ": v_eff[" + std::to_string(i) + "] is not finite");
        return DG_ERR_NUMERIC;
      }
    if (x.n_proj < 0 || (x.n_proj > 0 && (!x.proj_ptr || !x.proj_idx || !x.proj_val || !x.gamma))) {
      set_error("element " + std::to_string(e) + ": projector arrays missing");
      return DG_ERR_ARG;
    }
    if (x.n_proj > kMaxProjectors) {
      set_error("element " + std::to_string(e) + ": " + std::to_string(x.n_proj) + " projectors, above the " +
                std::to_string(kMaxProjectors) + " one element may carry");
      return DG_ERR_SHAPE;
    }
    if (x.n_proj > 0) {
      if (x.proj_ptr[0] != 0) {
        set_error("element " + std::to_string(e) + ": proj_ptr[0] must be 0");
        return DG_ERR_ARG;
      }
      for (int p = 0; p < x.n_proj; ++p) {
        if (x.proj_ptr[p + 1] < x.proj_ptr[p]) {
          set_error("element " + std::to_string(e) + ": proj_ptr not monotone");
          return DG_ERR_ARG;
        }
        if (!std::isfinite(x.gamma[p])) {
          set_error("element " + std::to_string(e) + ": gamma is not finite");
          return DG_ERR_NUMERIC;
        }
        for (int64_t t = x.proj_ptr[p]; t < x.proj_ptr[p + 1]; ++t) {
          if (!std::isfinite(x.proj_val[t])) {
            set_error("element " + std::to_string(e) + ": projector value is not finite");
            return DG_ERR_NUMERIC;
          }
          if (x.proj_idx[t] < 0 || x.proj_idx[t] >= N ||
              (t > x.proj_ptr[p] && x.proj_idx[t] <= x.proj_idx[t - 1])) {
            set_error("element " + std::to_string(e) + ": projector indices must be ascending and in range");
            return DG_ERR_ARG;
          }
        }
      }
    }
  }
  return DG_OK;
}

static int make_plan(int n_elem, const dg_element_desc* d, const dg_options* opt, Plan& P) {
  int st = validate(n_elem, d);
  if (st) return st;
  const int guard_opt = opt ? opt->n_guard : -1;
  const int max_cheb = opt ? std::max(0, opt->max_cheb_degree) : 0;
  const int stride = opt ? std::max(1, opt->ckpt_stride) : 1;
  P = Plan();
  P.el.resize(n_elem);
  P.proj.resize(n_elem);
  int kmax = 0;
  for (int e = 0; e < n_elem; ++e) {
    ElemPlan& p = P.el[e];
    p.J = d[e].n_states;
    // default: a fifth of J (at least 4), fewer where J + guards would pass 88
    p.G = guard_opt >= 0 ? guard_opt : std::max(4, (int)std::ceil(0.2 * p.J));
    if (guard_opt < 0 && p.J + p.G > 88) p.G = std::max(4, 88 - p.J);
    p.K = p.J + p.G;
    p.N = d[e].n[0] * d[e].n[1] * d[e].n[2];
    if (p.K > 88 || p.K > p.N / 2) {
      set_error("element " + std::to_string(e) + ": J + guards must be <= 88");
      return DG_ERR_SHAPE;
    }
    p.Kpad = p.K + (p.K & 1);
    p.ld = (p.N + 63) / 64 * 64;
    p.kmax3 = 3 * p.K;
    p.KP = p.kmax3 + 2;
    kmax = std::max(kmax, p.K);
    build_proj_plan(d[e], p.N, P.proj[e]);
  }
  // band energy: checkpoint pairs every ckpt_stride steps, Y_m, H Y_m, one segment
  P.n_extra = max_cheb > 0 ? 2 * ((max_cheb + stride - 1) / stride) + 2 + stride : 0;
  if (P.n_extra > kExtraBlocks) {
    set_error("max_cheb_degree / ckpt_stride need " + std::to_string(P.n_extra) +
              " checkpoint blocks (limit " + std::to_string(kExtraBlocks) + "); raise ckpt_stride");
    return DG_ERR_ARG;
  }
  P.part_ld = 3 * kmax;
  P.nsplit_max = std::max(1, std::min(64, 4096 / n_elem));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  P.off_elems = take(sizeof(ElemDev) * n_elem);
  P.off_iota = take(sizeof(int) * n_elem);
  P.off_active = take(sizeof(int) * n_elem);
  P.off_status = take(sizeof(int) * n_elem);
  P.off_count = take(sizeof(int) * 4);
  P.off_iters = take(sizeof(int) * n_elem);
  P.off_phase = take(sizeof(long long) * 16 * n_elem);
  P.off_maxres = take(sizeof(double) * n_elem);
  P.off_bounds = take(sizeof(double) * 3 * n_elem);
  P.off_de = take(sizeof(double) * n_elem);
  P.off_minpiv = take(3 * sizeof(double) * n_elem);
  P.off_hpflag = take(sizeof(int) * n_elem);
  P.off_offx0 = take(sizeof(long long) * (n_elem + 1));
  P.off_offvec = take(sizeof(long long) * (n_elem + 1));
  P.off_offalb = take(sizeof(long long) * (n_elem + 1));
  P.off_offgrid = take(sizeof(long long) * (n_elem + 1));
  P.off_offeig = take(sizeof(long long) * (n_elem + 1));
  P.off_offkall = take(sizeof(long long) * (n_elem + 1));
  P.off_offelem = take(sizeof(long long) * (n_elem + 1));
  P.off_offjj = take(sizeof(long long) * (n_elem + 1));
  P.off_nprojoff = take(sizeof(long long) * (n_elem + 1));
  P.off_lists = take(sizeof(int) * n_elem);
  size_t ckpt_block = 0;
  for (int e = 0; e < n_elem; ++e) {
    ElemPlan& p = P.el[e];
    const ProjPlan& pp = P.proj[e];
    p.ngrp = (int)pp.sptr.size() - 1;
    p.nact = (int)pp.act_idx.size();
    p.nent = (int)pp.ent_proj.size();
    p.off_v64 = take(sizeof(double) * p.N);
    p.off_v32 = take(sizeof(float) * p.N);
    p.off_sptr = take(sizeof(int) * pp.sptr.size());
    p.off_pbase = take(sizeof(int) * pp.pbase.size());
    p.off_idx = take(sizeof(int) * std::max<size_t>(1, pp.idx.size()));
    p.off_val64 = take(sizeof(double) * std::max<size_t>(1, pp.val.size()));
    p.off_val32 = take(sizeof(float) * std::max<size_t>(1, pp.val.size()));
    p.off_vbase = take(sizeof(long long) * std::max<size_t>(1, pp.vbase.size()));
    p.off_gamma = take(sizeof(double) * std::max(1, d[e].n_proj));
    p.off_act_idx = take(sizeof(int) * std::max<size_t>(1, pp.act_idx.size()));
    p.off_act_ptr = take(sizeof(int) * pp.act_ptr.size());
    p.off_ent_proj = take(sizeof(int) * std::max<size_t>(1, pp.ent_proj.size()));
    p.off_ent_v64 = take(sizeof(double) * std::max<size_t>(1, pp.ent_val.size()));
    p.off_ent_v32 = take(sizeof(float) * std::max<size_t>(1, pp.ent_val.size()));
    p.n_blocks = kMaxBlocks + P.n_extra;
    for (int b = 0; b < p.n_blocks; ++b) p.off_blk[b] = take(sizeof(double) * (size_t)p.ld * p.Kpad);
    p.off_small = take(sizeof(double) * SmallLayout::total(p.KP));
    p.off_nlc = take(sizeof(double) * (size_t)std::max(1, d[e].n_proj) * p.kmax3);
    ckpt_block += align256(sizeof(double) * (size_t)p.ld * p.Kpad);
  }
  P.ckpt_block_bytes = ckpt_block;
  P.n_ckpt = max_cheb > 0 ? (max_cheb / stride + 2) : 0;
  P.off_ckpt = take(P.ckpt_block_bytes * P.n_ckpt + 256);
  // split-N Gram partials; the same region is the Rayleigh-Ritz inverse-iteration workspace
  P.part_stride = std::max((size_t)P.nsplit_max * P.part_ld * P.part_ld, (size_t)6 * (P.part_ld + 2) * 512);
  P.off_part = take(sizeof(double) * (size_t)n_elem * P.part_stride);
  P.total = off + 256;
  return DG_OK;
}

int query_workspace(int n_elem, const dg_element_desc* d, const dg_options* opt, size_t* bytes) {
  if (!bytes) {
    set_error("bytes is NULL");
    return DG_ERR_ARG;
  }
  Plan P;
  int st = make_plan(n_elem, d, opt, P);
  if (st) return st;
  *bytes = P.total;
  return DG_OK;
}

// ---------------------------------------------------------------------------
// create
// ---------------------------------------------------------------------------
int create(Ctx** out, int n_elem, const dg_element_desc* d, const dg_options* opt, void* arena,
           size_t arena_bytes, void* stream) {
  if (!out || !arena) {
    set_error("ctx or arena is NULL");
    return DG_ERR_ARG;
  }
  if (((uintptr_t)arena) & 255) {
    set_error("arena must be 256-byte aligned");
    return DG_ERR_ARG;
  }
  Plan P;
  int st = make_plan(n_elem, d, opt, P);
  if (st) return st;
  if (arena_bytes < P.total) {
    set_error("arena too small: need " + std::to_string(P.total) + " bytes");
    return DG_ERR_OOM;
  }
  init_kernel_attributes();
  // owned here until every staging step has succeeded (no leak on an early return)
  std::unique_ptr<Ctx> owner(new Ctx());
  Ctx* c = owner.get();
  c->stream = (hipStream_t)stream;
  c->n_elem = n_elem;
  c->arena = (char*)arena;
  c->arena_bytes = arena_bytes;
  c->arena_used = P.total;
  c->max_cheb = opt ? std::max(0, opt->max_cheb_degree) : 0;
  c->ckpt_stride = opt ? std::max(1, opt->ckpt_stride) : 1;
  if (const char* lv = std::getenv("DG_LOG")) c->log_level = std::atoi(lv);
  if (const char* ot = std::getenv("DG_RR_ORTOL")) c->rr_ortol = std::atof(ot);
  if (const char* dt = std::getenv("DG_RR_DROP")) c->rr_drop_env = std::atof(dt);
  if (const char* dr = std::getenv("DG_RR_DROP_REFINE")) c->rr_drop_refine_env = std::atof(dr);
  if (const char* tu = std::getenv("DG_TUNE")) c->autotune = std::atoi(tu) != 0;
  if (const char* ow = std::getenv("DG_ORTH_W")) c->orth_w = std::atoi(ow) != 0;
  if (const char* fh = std::getenv("DG_FRESH_HP")) c->fresh_hp_all = std::atoi(fh) != 0;
  if (const char* ht = std::getenv("DG_HP_TOL")) c->hp_tol_env = std::atof(ht);
  if (const char* bf = std::getenv("DG_BF16")) c->bf16 = std::atoi(bf) != 0;
  if (const char* mr = std::getenv("DG_MIXED_REFINE")) c->mixed_refine = std::atoi(mr) != 0;
  char* A = c->arena;
  hipStream_t s = c->stream;
  auto cpy = [&](size_t off, const void* src, size_t bytes) -> int {
    if (bytes == 0) return DG_OK;
    hipError_t e = hipMemcpyAsync(A + off, src, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      set_error(std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
      return DG_ERR_HIP;
    }
    return DG_OK;
  };
  c->elems_host.resize(n_elem);
  c->J.resize(n_elem);
  c->G.resize(n_elem);
  c->K.resize(n_elem);
  c->N.resize(n_elem);
  c->ld.resize(n_elem);
  for (int a = 0; a < 3; ++a) {
    c->elo[a].resize(n_elem);
    c->en[a].resize(n_elem);
    c->nxyz[a].resize(n_elem);
    c->lens[a].resize(n_elem);
  }
  // host staging buffers kept alive until the stream synchronises below
  std::vector<std::vector<float>> keep32;
  std::vector<std::vector<long long>> keep64;
  std::vector<std::vector<int>> keepi;
  for (int e = 0; e < n_elem; ++e) {
    const ElemPlan& p = P.el[e];
    const ProjPlan& pp = P.proj[e];
    const dg_element_desc& x = d[e];
    ElemDev& E = c->elems_host[e];
    std::memset(&E, 0, sizeof(E));
    E.nx = x.n[0];
    E.ny = x.n[1];
    E.nz = x.n[2];
    E.N = p.N;
    E.ld = p.ld;
    E.K = p.K;
    E.J = p.J;
    for (int a = 0; a < 3; ++a) {
      E.elo[a] = x.elem_lo[a];
      E.en[a] = x.elem_n[a];
      c->elo[a][e] = x.elem_lo[a];
      c->en[a][e] = x.elem_n[a];
      c->nxyz[a][e] = x.n[a];
      c->lens[a][e] = x.len[a];
    }
    const double tp = 2.0 * M_PI;
    E.kx = 0.5 * (tp / x.len[0]) * (tp / x.len[0]);
    E.ky = 0.5 * (tp / x.len[1]) * (tp / x.len[1]);
    E.kz = 0.5 * (tp / x.len[2]) * (tp / x.len[2]);
    double vmin = x.v_eff[0], vmax = x.v_eff[0];
    for (int i = 0; i < p.N; ++i) {
      vmin = std::min(vmin, x.v_eff[i]);
      vmax = std::max(vmax, x.v_eff[i]);
    }
    E.vmin = vmin;
    // Upper bound of the spectrum: max kinetic symbol + max V + a Gershgorin bound
    // of sum_{gamma>0} gamma |b><b| through the projector overlaps |b_p . b_q|
    {
      const double kin = E.kx * (double)(x.n[0] / 2) * (x.n[0] / 2) + E.ky * (double)(x.n[1] / 2) * (x.n[1] / 2) +
                         E.kz * (double)(x.n[2] / 2) * (x.n[2] / 2);
      double nl = 0.0;
      if (x.n_proj > 0) {
        std::vector<double> rowsum(x.n_proj, 0.0);
        for (size_t a2 = 0; a2 < pp.act_idx.size(); ++a2)
          for (int q1 = pp.act_ptr[a2]; q1 < pp.act_ptr[a2 + 1]; ++q1)
            for (int q2 = pp.act_ptr[a2]; q2 < pp.act_ptr[a2 + 1]; ++q2) {
              const int p1 = pp.ent_proj[q1], p2 = pp.ent_proj[q2];
              if (x.gamma[p1] > 0.0 && x.gamma[p2] > 0.0)
                rowsum[p1] += std::sqrt(x.gamma[p1] * x.gamma[p2]) * std::fabs(pp.ent_val[q1] * pp.ent_val[q2]);
            }
        for (double r : rowsum) nl = std::max(nl, r);
      }
      E.bup_base = kin + nl + 1e-6;
      E.bup = E.bup_base + std::max(vmax, 0.0);
    }
    E.v64 = (const double*)(A + p.off_v64);
    E.v32 = (const float*)(A + p.off_v32);
    E.ngrp = p.ngrp;
    E.nproj = x.n_proj;
    E.grp_sptr = (const int*)(A + p.off_sptr);
    E.grp_pbase = (const int*)(A + p.off_pbase);
    E.grp_idx = (const int*)(A + p.off_idx);
    E.grp_val64 = (const double*)(A + p.off_val64);
    E.grp_val32 = (const float*)(A + p.off_val32);
    E.grp_vbase = (const long long*)(A + p.off_vbase);
    E.gamma = (const double*)(A + p.off_gamma);
    E.nact = p.nact;
    E.act_idx = (const int*)(A + p.off_act_idx);
    E.act_ptr = (const int*)(A + p.off_act_ptr);
    E.ent_proj = (const int*)(A + p.off_ent_proj);
    E.ent_val64 = (const double*)(A + p.off_ent_v64);
    E.ent_val32 = (const float*)(A + p.off_ent_v32);
    for (int b = 0; b < kTotalBlocks; ++b) E.blk[b] = b < p.n_blocks ? A + p.off_blk[b] : nullptr;
    E.small = (double*)(A + p.off_small);
    E.nlc = (double*)(A + p.off_nlc);
    E.kmax3 = p.kmax3;
    c->J[e] = p.J;
    c->G[e] = p.G;
    c->K[e] = p.K;
    c->N[e] = p.N;
    c->ld[e] = p.ld;
    c->kmax = std::max(c->kmax, p.K);
    c->nnz.push_back(x.n_proj > 0 ? (double)x.proj_ptr[x.n_proj] : 0.0);
    if ((st = cpy(p.off_v64, x.v_eff, sizeof(double) * p.N))) return st;
    keep32.emplace_back(x.v_eff, x.v_eff + p.N);
    if ((st = cpy(p.off_v32, keep32.back().data(), sizeof(float) * p.N))) return st;
    if ((st = cpy(p.off_sptr, pp.sptr.data(), sizeof(int) * pp.sptr.size()))) return st;
    if ((st = cpy(p.off_pbase, pp.pbase.data(), sizeof(int) * pp.pbase.size()))) return st;
    if ((st = cpy(p.off_idx, pp.idx.data(), sizeof(int) * pp.idx.size()))) return st;
    if ((st = cpy(p.off_val64, pp.val.data(), sizeof(double) * pp.val.size()))) return st;
    keep32.emplace_back(pp.val.begin(), pp.val.end());
    if ((st = cpy(p.off_val32, keep32.back().data(), sizeof(float) * pp.val.size()))) return st;
    if ((st = cpy(p.off_vbase, pp.vbase.data(), sizeof(long long) * pp.vbase.size()))) return st;
    if ((st = cpy(p.off_gamma, x.gamma, sizeof(double) * x.n_proj))) return st;
    if ((st = cpy(p.off_act_idx, pp.act_idx.data(), sizeof(int) * pp.act_idx.size()))) return st;
    if ((st = cpy(p.off_act_ptr, pp.act_ptr.data(), sizeof(int) * pp.act_ptr.size()))) return st;
    if ((st = cpy(p.off_ent_proj, pp.ent_proj.data(), sizeof(int) * pp.ent_proj.size()))) return st;
    if ((st = cpy(p.off_ent_v64, pp.ent_val.data(), sizeof(double) * pp.ent_val.size()))) return st;
    keep32.emplace_back(pp.ent_val.begin(), pp.ent_val.end());
    if ((st = cpy(p.off_ent_v32, keep32.back().data(), sizeof(float) * pp.ent_val.size()))) return st;
  }
  // packed offsets
  c->off_x0.assign(n_elem + 1, 0);
  c->off_vec.assign(n_elem + 1, 0);
  c->off_eig.assign(n_elem + 1, 0);
  c->off_alb.assign(n_elem + 1, 0);
  c->off_grid.assign(n_elem + 1, 0);
  c->off_kall.assign(n_elem + 1, 0);
  c->off_elem.assign(n_elem + 1, 0);
  c->off_jj.assign(n_elem + 1, 0);
  for (int e = 0; e < n_elem; ++e) {
    const int en = c->en[0][e] * c->en[1][e] * c->en[2][e];
    c->off_x0[e + 1] = c->off_x0[e] + (int64_t)c->N[e] * c->K[e];
    c->off_vec[e + 1] = c->off_vec[e] + (int64_t)c->N[e] * c->J[e];
    c->off_eig[e + 1] = c->off_eig[e] + c->J[e];
    c->off_alb[e + 1] = c->off_alb[e] + (int64_t)en * c->J[e];
    c->off_grid[e + 1] = c->off_grid[e] + c->N[e];
    c->off_kall[e + 1] = c->off_kall[e] + c->K[e];
    c->off_elem[e + 1] = c->off_elem[e] + en;
    c->off_jj[e + 1] = c->off_jj[e] + (int64_t)c->J[e] * c->J[e];
  }
  keep64.emplace_back(c->off_x0.begin(), c->off_x0.end());
  if ((st = cpy(P.off_offx0, keep64.back().data(), sizeof(long long) * (n_elem + 1)))) return st;
  keep64.emplace_back(c->off_vec.begin(), c->off_vec.end());
  if ((st = cpy(P.off_offvec, keep64.back().data(), sizeof(long long) * (n_elem + 1)))) return st;
  keep64.emplace_back(c->off_alb.begin(), c->off_alb.end());
  if ((st = cpy(P.off_offalb, keep64.back().data(), sizeof(long long) * (n_elem + 1)))) return st;
  keep64.emplace_back(c->off_grid.begin(), c->off_grid.end());
  if ((st = cpy(P.off_offgrid, keep64.back().data(), sizeof(long long) * (n_elem + 1)))) return st;
  c->dev_off_x0 = (long long*)(A + P.off_offx0);
  c->dev_off_vec = (long long*)(A + P.off_offvec);
  c->dev_off_alb = (long long*)(A + P.off_offalb);
  c->dev_off_grid = (long long*)(A + P.off_offgrid);
  keep64.emplace_back(c->off_eig.begin(), c->off_eig.end());
  if ((st = cpy(P.off_offeig, keep64.back().data(), sizeof(long long) * (n_elem + 1)))) return st;
  c->dev_off_eig = (long long*)(A + P.off_offeig);
  keep64.emplace_back(c->off_kall.begin(), c->off_kall.end());
  if ((st = cpy(P.off_offkall, keep64.back().data(), sizeof(long long) * (n_elem + 1)))) return st;
  c->dev_off_kall = (long long*)(A + P.off_offkall);
  keep64.emplace_back(c->off_elem.begin(), c->off_elem.end());
  if ((st = cpy(P.off_offelem, keep64.back().data(), sizeof(long long) * (n_elem + 1)))) return st;
  c->dev_off_elem = (long long*)(A + P.off_offelem);
  keep64.emplace_back(c->off_jj.begin(), c->off_jj.end());
  if ((st = cpy(P.off_offjj, keep64.back().data(), sizeof(long long) * (n_elem + 1)))) return st;
  c->dev_off_jj = (long long*)(A + P.off_offjj);
  c->nproj_off.assign(n_elem + 1, 0);
  for (int e = 0; e < n_elem; ++e) c->nproj_off[e + 1] = c->nproj_off[e] + d[e].n_proj;
  keep64.emplace_back(c->nproj_off.begin(), c->nproj_off.end());
  if ((st = cpy(P.off_nprojoff, keep64.back().data(), sizeof(long long) * (n_elem + 1)))) return st;
  c->dev_nproj_off = (long long*)(A + P.off_nprojoff);
  // shape classes
  std::map<std::tuple<int, int, int>, std::vector<int>> cls;
  for (int e = 0; e < n_elem; ++e) cls[{d[e].n[0], d[e].n[1], d[e].n[2]}].push_back(e);
  std::vector<int> lists;
  for (auto& kv : cls) {
    ShapeClass sc;
    sc.nx = std::get<0>(kv.first);
    sc.ny = std::get<1>(kv.first);
    sc.nz = std::get<2>(kv.first);
    sc.nelem = (int)kv.second.size();
    sc.max_k = 0;
    for (int e : kv.second) sc.max_k = std::max(sc.max_k, c->K[e]);
    sc.elem_list_host = kv.second;
    sc.elem_list_dev = (int*)(A + P.off_lists) + lists.size();
    lists.insert(lists.end(), kv.second.begin(), kv.second.end());
    c->classes.push_back(sc);
  }
  keepi.push_back(lists);
  if ((st = cpy(P.off_lists, keepi.back().data(), sizeof(int) * lists.size()))) return st;
  std::vector<int> iota(n_elem);
  for (int e = 0; e < n_elem; ++e) iota[e] = e;
  keepi.push_back(iota);
  if ((st = cpy(P.off_iota, keepi.back().data(), sizeof(int) * n_elem))) return st;
  c->iota_dev = (int*)(A + P.off_iota);
  c->dev_active = (int*)(A + P.off_active);
  c->dev_status = (int*)(A + P.off_status);
  c->dev_count = (int*)(A + P.off_count);
  c->dev_iters = (int*)(A + P.off_iters);
  c->dev_bounds = (double*)(A + P.off_bounds);
  c->dev_de = (double*)(A + P.off_de);
  c->dev_minpiv = (double*)(A + P.off_minpiv);
  c->dev_hpflag = (int*)(A + P.off_hpflag);
  c->n_extra_blocks = P.n_extra;
  c->dev_phase = (long long*)(A + P.off_phase);
  c->dev_maxres = (double*)(A + P.off_maxres);
  c->gram_part_ld = P.part_ld;
  c->gram_max_split = P.nsplit_max;
  c->gram_part = (double*)(A + P.off_part);
  c->gram_part_stride = (long long)P.part_stride;
  c->ckpt_base = A + P.off_ckpt;
  c->ckpt_bytes_per_block = P.ckpt_block_bytes;
  c->ckpt_off.assign(n_elem, 0);
  {
    size_t o = 0;
    for (int e = 0; e < n_elem; ++e) {
      c->ckpt_off[e] = (int64_t)o;
      o += align256(sizeof(double) * (size_t)P.el[e].ld * P.el[e].Kpad);
    }
  }
  c->elems_dev = (ElemDev*)(A + P.off_elems);
  if ((st = cpy(P.off_elems, c->elems_host.data(), sizeof(ElemDev) * n_elem))) return st;
  // zero the blocks so padded columns and unused tails are defined
  for (int e = 0; e < n_elem; ++e)
    for (int b = 0; b < P.el[e].n_blocks; ++b) {
      hipError_t he = hipMemsetAsync(A + P.el[e].off_blk[b], 0, sizeof(double) * (size_t)P.el[e].ld * P.el[e].Kpad, s);
      if (he != hipSuccess) {
        set_error(std::string("hipMemsetAsync: ") + hipGetErrorString(he));
        return DG_ERR_HIP;
      }
    }
  hipError_t se = hipStreamSynchronize(s);
  if (se != hipSuccess) {
    set_error(std::string("hipStreamSynchronize: ") + hipGetErrorString(se));
    return DG_ERR_HIP;
  }
  *out = owner.release();
  return DG_OK;
}

}  // namespace dg
