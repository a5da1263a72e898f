// extern "C" entry points declared in include/dg_alb.h: argument checks and
// dispatch only; no exception crosses this boundary.
//
// A context is a batch of element groups.  Each group is an independent
// solver context (its own arena slice, scratch and HIP stream) over a
// contiguous range of elements; with several groups, dg_solve_elements drives
// them from one host thread each, so that one group's latency-bound steps
// (the per-element Rayleigh-Ritz workgroups, host convergence checks) overlap
// another group's bandwidth- and MFMA-bound kernels.  Work is forked from and
// joined back into the caller's stream with events.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <exception>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "dg_internal.h"

using dg::Ctx;

#define DG_GUARD(body)                                  \
  try {                                                 \
    body                                                \
  } catch (const std::exception& ex) {                  \
    dg::set_error(std::string("internal: ") + ex.what()); \
    return DG_ERR_ARG;                                  \
  } catch (...) {                                       \
    dg::set_error("internal error");                    \
    return DG_ERR_ARG;                                  \
  }

namespace {

constexpr int kMaxGroups = 8;

// contiguous element ranges of roughly equal cost (N_k (J_k + g)^2, the subspace GEMMs)
std::vector<int> split_groups(int n_elem, const dg_element_desc* d, const dg_options* opt) {
  int ng = opt ? opt->n_streams : 0;
  if (ng <= 0) {
    // one group per four elements, at most four (the hardware queues of a process)
    ng = std::max(1, std::min(4, n_elem / 4));
    if (const char* s = std::getenv("DG_STREAMS")) ng = std::max(1, std::atoi(s));
  }
  ng = std::max(1, std::min({ng, n_elem, kMaxGroups}));
  std::vector<double> cost(n_elem);
  double total = 0.0;
  for (int e = 0; e < n_elem; ++e) {
    const double N = (double)d[e].n[0] * d[e].n[1] * d[e].n[2];
    const double k = d[e].n_states + std::max(4.0, std::ceil(0.1 * d[e].n_states));
    cost[e] = N * k * k;
    total += cost[e];
  }
  std::vector<int> lo(1, 0);
  double acc = 0.0;
  for (int e = 0; e < n_elem; ++e) {
    acc += cost[e];
    const int g = (int)lo.size();   // groups closed so far + 1
    const int left_elems = n_elem - 1 - e, left_groups = ng - g;
    if (g < ng && (acc >= total * g / ng || left_elems == left_groups) && left_elems >= left_groups)
      lo.push_back(e + 1);
  }
  lo.push_back(n_elem);
  return lo;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct dg_ctx {
  std::vector<Ctx> g;            // one solver context per group
  std::vector<int> lo;           // group element ranges [lo[i], lo[i+1])
  hipStream_t user = nullptr;    // the caller's stream
  std::vector<hipStream_t> own;  // library streams, one per group
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  std::vector<int64_t> off[8];   // batch-wide packed offsets per dg_offset_kind
  int be_prec = -1, be_nvec = 0; // last band-energy call (layout of dpsi0)
  int device = 0;
  double* scratch = nullptr;     // this device's static scratch (no-allocation H*psi)

  int groups() const { return (int)g.size(); }
  int fork() {
    if (own.empty()) return DG_OK;
    DG_HIP(hipEventRecord(fork_ev, user));
    for (hipStream_t s : own) DG_HIP(hipStreamWaitEvent(s, fork_ev, 0));
    return DG_OK;
  }
  int join() {
    if (own.empty()) return DG_OK;
    for (size_t i = 0; i < own.size(); ++i) {
      DG_HIP(hipEventRecord(join_ev[i], own[i]));
      DG_HIP(hipStreamWaitEvent(user, join_ev[i], 0));
    }
    return DG_OK;
  }
  ~dg_ctx() {
    for (Ctx& c : g) {
      for (const dg::PendingTime& p : c.pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
      }
      for (hipEvent_t e : c.event_pool) (void)hipEventDestroy(e);
    }
    for (hipEvent_t e : join_ev) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    for (hipStream_t s : own) (void)hipStreamDestroy(s);
  }
};

namespace {

const std::vector<int64_t>& group_off(const Ctx& c, int kind) {
  switch (kind) {
    case DG_OFF_X0: return c.off_x0;
    case DG_OFF_VEC: return c.off_vec;
    case DG_OFF_EIG: return c.off_eig;
    case DG_OFF_ALB: return c.off_alb;
    case DG_OFF_GRID: return c.off_grid;
    case DG_OFF_ELEM: return c.off_elem;
    case DG_OFF_JJ: return c.off_jj;
    default: return c.off_kall;
  }
}

template <typename P>
P* shift(P* p, int64_t elems, size_t elem_bytes) {
  return p ? reinterpret_cast<P*>(reinterpret_cast<char*>(const_cast<void*>((const void*)p)) + elems * elem_bytes)
           : nullptr;
}

// run f(group index) for every group, concurrently from one host thread each
template <typename F>
int run_groups(dg_ctx* b, F f) {
  const int ng = b->groups();
  if (ng == 1) return f(0);
  std::vector<int> st(ng, DG_OK);
  std::vector<std::string> err(ng);
  std::vector<std::thread> th;
  for (int i = 0; i < ng; ++i)
    th.emplace_back([&, i]() {
      (void)hipSetDevice(b->device);
      try {
        st[i] = f(i);
      } catch (const std::exception& ex) {
        dg::set_error(std::string("internal: ") + ex.what());
        st[i] = DG_ERR_ARG;
      } catch (...) {
        dg::set_error("internal error");
        st[i] = DG_ERR_ARG;
      }
      if (st[i] < 0) err[i] = dg::get_error();
    });
  for (auto& t : th) t.join();
  int worst = DG_OK;
  for (int i = 0; i < ng; ++i) {
    if (st[i] < 0) {
      dg::set_error("element group " + std::to_string(i) + ": " + err[i]);
      return st[i];
    }
    worst = std::max(worst, st[i]);
  }
  return worst;
}

// run f(group index) for every group in turn (asynchronous work on the group streams)
template <typename F>
int each_group(dg_ctx* b, F f) {
  int worst = DG_OK;
  for (int i = 0; i < b->groups(); ++i) {
    const int st = f(i);
    if (st < 0) return st;
    worst = std::max(worst, st);
  }
  return worst;
}

}  // namespace

extern "C" {

const char* dg_status_string(int32_t s) {
  switch (s) {
    case DG_OK: return "DG_OK";
    case DG_WARN_NOT_CONVERGED: return "DG_WARN_NOT_CONVERGED";
    case DG_ERR_ARG: return "DG_ERR_ARG";
    case DG_ERR_SHAPE: return "DG_ERR_SHAPE";
    case DG_ERR_OOM: return "DG_ERR_OOM";
    case DG_ERR_HIP: return "DG_ERR_HIP";
    case DG_ERR_NUMERIC: return "DG_ERR_NUMERIC";
    case DG_ERR_STATE: return "DG_ERR_STATE";
    default: return "DG_UNKNOWN_STATUS";
  }
}

const char* dg_last_error(const dg_ctx*) { return dg::get_error(); }

int32_t dg_query_workspace(int32_t n_elem, const dg_element_desc* elems, const dg_options* opt,
                           size_t* bytes) {
  DG_GUARD({
    if (!bytes || !elems || n_elem <= 0) {
      dg::set_error("bytes or elems is NULL, or n_elem <= 0");
      return DG_ERR_ARG;
    }
    const std::vector<int> lo = split_groups(n_elem, elems, opt);
    size_t total = 0;
    for (size_t i = 0; i + 1 < lo.size(); ++i) {
      size_t b = 0;
      const int st = dg::query_workspace(lo[i + 1] - lo[i], elems + lo[i], opt, &b);
      if (st) return st;
      total += round256(b);
    }
    *bytes = total;
    return DG_OK;
  })
}

int32_t dg_create_elements(dg_ctx** ctx, int32_t n_elem, const dg_element_desc* elems,
                           const dg_options* opt, void* dev_arena, size_t arena_bytes, void* hip_stream) {
  DG_GUARD({
    if (!ctx) {
      dg::set_error("ctx is NULL");
      return DG_ERR_ARG;
    }
    *ctx = nullptr;
    if (!elems || n_elem <= 0) {
      dg::set_error("n_elem must be positive and elems non-NULL");
      return DG_ERR_ARG;
    }
    std::unique_ptr<dg_ctx> b(new dg_ctx());
    b->lo = split_groups(n_elem, elems, opt);
    b->user = (hipStream_t)hip_stream;
    DG_HIP(hipGetDevice(&b->device));
    // set-up of the no-allocation entry point: the static scratch's address on this device
    if (int st = dg::noalloc_scratch(b->device, &b->scratch)) return st;
    const int ng = (int)b->lo.size() - 1;
    {
      // every group runs on a library stream (a capturable one even when the caller
      // passes the legacy default stream)
      DG_HIP(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
      for (int i = 0; i < ng; ++i) {
        hipStream_t s;
        DG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        b->own.push_back(s);
        hipEvent_t ev;
        DG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        b->join_ev.push_back(ev);
      }
      // the arena may still be written by work queued on the caller's stream
      if (int st = b->fork()) return st;
    }
    size_t used = 0;
    int worst = DG_OK;
    b->g.reserve(ng);
    for (int i = 0; i < ng; ++i) {
      const int n = b->lo[i + 1] - b->lo[i];
      size_t need = 0;
      int st = dg::query_workspace(n, elems + b->lo[i], opt, &need);
      if (st) return st;
      if (used + need > arena_bytes) {
        dg::set_error("arena too small for element group " + std::to_string(i));
        return DG_ERR_OOM;
      }
      Ctx* c = nullptr;
      st = dg::create(&c, n, elems + b->lo[i], opt, (char*)dev_arena + used, arena_bytes - used,
                      (void*)b->own[i]);
      if (st < 0) return st;
      worst = std::max(worst, st);
      c->elem_base = b->lo[i];
      b->g.push_back(std::move(*c));
      delete c;
      used += round256(need);
    }
    // batch-wide offsets: the groups' packed buffers follow each other
    for (int kind = 0; kind < 8; ++kind) {
      std::vector<int64_t>& o = b->off[kind];
      o.assign(1, 0);
      for (int i = 0; i < ng; ++i) {
        const std::vector<int64_t>& go = group_off(b->g[i], kind);
        const int64_t base = o.back();
        for (size_t e = 1; e < go.size(); ++e) o.push_back(base + go[e]);
      }
    }
    if (int st = b->join()) return st;
    *ctx = b.release();
    return worst;
  })
}

void dg_destroy(dg_ctx* ctx) { delete ctx; }

int32_t dg_query_offsets(const dg_ctx* ctx, int32_t kind, int64_t* offsets) {
  if (!ctx || !offsets) {
    dg::set_error("ctx or offsets is NULL");
    return DG_ERR_ARG;
  }
  if (kind < 0 || kind > 7) {
    dg::set_error("unknown offset kind");
    return DG_ERR_ARG;
  }
  const std::vector<int64_t>& v = ctx->off[kind];
  for (size_t i = 0; i < v.size(); ++i) offsets[i] = v[i];
  return DG_OK;
}

int32_t dg_apply_H(dg_ctx* ctx, int32_t elem, int32_t n_vec, int32_t prec, const void* x_dev, int64_t ldx,
                   void* y_dev, int64_t ldy) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    const int n_elem = ctx->lo.back();
    if (elem < -1 || elem >= n_elem) {
      dg::set_error("elem out of range");
      return DG_ERR_ARG;
    }
    if (ldx < 0 || ldy < 0) {
      dg::set_error("ldx and ldy must be >= 0");
      return DG_ERR_ARG;
    }
    const size_t sz = prec == DG_FP32 ? sizeof(float) : sizeof(double);
    if (int st = ctx->fork()) return st;
    int st = each_group(ctx, [&](int i) {
      const int a = ctx->lo[i], z = ctx->lo[i + 1];
      if (elem >= 0) {
        if (elem < a || elem >= z) return (int)DG_OK;
        return dg::apply_h(ctx->g[i], elem - a, n_vec, prec, x_dev, ldx, y_dev, ldy);
      }
      // this group's first element block: packed offsets, or a elements of ld * n_vec
      const int64_t nv = std::max(n_vec, 0);
      const int64_t ox = ldx > 0 ? (int64_t)a * ldx * nv : ctx->off[DG_OFF_GRID][a] * nv;
      const int64_t oy = ldy > 0 ? (int64_t)a * ldy * nv : ctx->off[DG_OFF_GRID][a] * nv;
      return dg::apply_h(ctx->g[i], -1, n_vec, prec, shift(x_dev, ox, sz), ldx, shift(y_dev, oy, sz), ldy);
    });
    if (st < 0) return st;
    if (int s2 = ctx->join()) return s2;
    return st;
  })
}

int32_t dg_solve_elements(dg_ctx* ctx, const dg_solve_params* params, double* eig_dev,
                          double* resid_dev, int32_t* iters_host) {
  if (!ctx || !params) {
    dg::set_error("ctx or params is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    if (int st = ctx->fork()) return st;
    int st = run_groups(ctx, [&](int i) {
      const int a = ctx->lo[i];
      dg_solve_params p = *params;
      p.x0_dev = shift(params->x0_dev, ctx->off[DG_OFF_X0][a], sizeof(double));
      return dg::solve(ctx->g[i], &p, shift(eig_dev, ctx->off[DG_OFF_EIG][a], sizeof(double)),
                       shift(resid_dev, ctx->off[DG_OFF_EIG][a], sizeof(double)),
                       iters_host ? iters_host + a : nullptr);
    });
    if (st < 0) return st;
    if (int s2 = ctx->join()) return s2;
    return st;
  })
}

int32_t dg_apply_H_noalloc(dg_ctx* ctx, int32_t elem, int32_t n_vec, int32_t prec, const void* x_dev,
                           int64_t ldx, void* y_dev, int64_t ldy) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    const int n_elem = ctx->lo.back();
    if (elem < -1 || elem >= n_elem) {
      dg::set_error("elem out of range");
      return DG_ERR_ARG;
    }
    if (ldx < 0 || ldy < 0 || n_vec <= 0) {
      dg::set_error("ldx and ldy must be >= 0 and n_vec > 0");
      return DG_ERR_ARG;
    }
    // scratch: nproj x n_vec doubles per applied element, groups in disjoint parts
    std::vector<long long> base(ctx->groups() + 1, 0);
    for (int i = 0; i < ctx->groups(); ++i) {
      const Ctx& c = ctx->g[i];
      long long need = 0;
      if (elem < 0) need = c.nproj_off[c.n_elem] * n_vec;
      else if (elem >= ctx->lo[i] && elem < ctx->lo[i + 1])
        need = (c.nproj_off[elem - ctx->lo[i] + 1] - c.nproj_off[elem - ctx->lo[i]]) * n_vec;
      base[i + 1] = base[i] + (need + 31) / 32 * 32;
    }
    if (base.back() > dg::noalloc_scratch_doubles()) {
      dg::set_error("the projector overlaps of this call need " + std::to_string(base.back() * 8) +
                    " bytes, above the static scratch of " + std::to_string(dg::noalloc_scratch_doubles() * 8) +
                    " bytes: apply fewer vectors or one element per call");
      return DG_ERR_ARG;
    }
    const size_t sz = prec == DG_FP32 ? sizeof(float) : sizeof(double);
    if (int st = ctx->fork()) return st;
    int st = each_group(ctx, [&](int i) {
      const int a = ctx->lo[i], z = ctx->lo[i + 1];
      double* nlc = ctx->scratch + base[i];
      if (elem >= 0) {
        if (elem < a || elem >= z) return (int)DG_OK;
        return dg::apply_h_noalloc(ctx->g[i], elem - a, n_vec, prec, x_dev, ldx, y_dev, ldy, nlc);
      }
      const int64_t nv = n_vec;
      const int64_t ox = ldx > 0 ? (int64_t)a * ldx * nv : ctx->off[DG_OFF_GRID][a] * nv;
      const int64_t oy = ldy > 0 ? (int64_t)a * ldy * nv : ctx->off[DG_OFF_GRID][a] * nv;
      return dg::apply_h_noalloc(ctx->g[i], -1, n_vec, prec, shift(x_dev, ox, sz), ldx, shift(y_dev, oy, sz),
                                 ldy, nlc);
    });
    if (st < 0) return st;
    if (int s2 = ctx->join()) return s2;
    return st;
  })
}

}  // extern "C"

namespace {

int dg_mesh_info(const dg_ctx* ctx, const dg_mesh_desc* m, dg::DgMeshInfo& mi, std::vector<dg::DgElemShape>& sh) {
  if (!ctx || !m || !m->proj_count || (!m->proj_ptr)) {
    dg::set_error("ctx or mesh (or its projector arrays) is NULL");
    return DG_ERR_ARG;
  }
  const int M = ctx->lo.back();
  mi.n_mesh[0] = m->n_mesh[0];
  mi.n_mesh[1] = m->n_mesh[1];
  mi.alpha = m->alpha;
  mi.count = m->proj_count;
  mi.gid = m->proj_gid;
  mi.ptr = reinterpret_cast<const long long*>(m->proj_ptr);
  mi.idx = m->proj_idx;
  mi.val = m->proj_val;
  mi.gamma = m->gamma;
  mi.pbase.assign(M + 1, 0);
  for (int k = 0; k < M; ++k) {
    if (m->proj_count[k] < 0) {
      dg::set_error("negative projector count");
      return DG_ERR_ARG;
    }
    mi.pbase[k + 1] = mi.pbase[k] + m->proj_count[k];
  }
  if (mi.pbase[M] > 0 && (!m->proj_gid || !m->proj_idx || !m->proj_val || !m->gamma)) {
    dg::set_error("projector arrays missing");
    return DG_ERR_ARG;
  }
  for (int p = 0; p < mi.pbase[M]; ++p)
    if (mi.ptr[p + 1] < mi.ptr[p]) {
      dg::set_error("proj_ptr not monotone");
      return DG_ERR_ARG;
    }
  if (!(m->alpha >= 0.0)) {
    dg::set_error("alpha must be >= 0");
    return DG_ERR_ARG;
  }
  sh.resize(M);
  for (int i = 0; i < ctx->groups(); ++i) {
    const Ctx& c = ctx->g[i];
    for (int e = 0; e < c.n_elem; ++e) {
      dg::DgElemShape& a = sh[ctx->lo[i] + e];
      a.J = c.J[e];
      for (int q = 0; q < 3; ++q) {
        a.n[q] = c.nxyz[q][e];
        a.len[q] = c.lens[q][e];
        a.elo[q] = c.elo[q][e];
        a.en[q] = c.en[q][e];
      }
    }
  }
  return DG_OK;
}

}  // namespace

extern "C" {

int32_t dg_query_hamiltonian(const dg_ctx* ctx, const dg_mesh_desc* mesh, int32_t* n_blocks, int64_t* row_ptr,
                             int32_t* col_idx, int64_t* block_off, size_t* work_bytes) {
  DG_GUARD({
    dg::DgMeshInfo mi;
    std::vector<dg::DgElemShape> sh;
    if (int st = dg_mesh_info(ctx, mesh, mi, sh)) return st;
    dg::DgPlan P;
    if (int st = dg::dg_plan(mi, sh, P)) return st;
    if (n_blocks) *n_blocks = (int32_t)P.blk.size();
    if (row_ptr)
      for (size_t i = 0; i < P.row_ptr.size(); ++i) row_ptr[i] = P.row_ptr[i];
    if (col_idx)
      for (size_t b = 0; b < P.blk.size(); ++b) col_idx[b] = P.blk[b].nb;
    if (block_off) {
      for (size_t b = 0; b < P.blk.size(); ++b) block_off[b] = P.blk[b].off;
      block_off[P.blk.size()] = P.total_values;
    }
    if (work_bytes) *work_bytes = (size_t)P.total_doubles * sizeof(double);
    return DG_OK;
  })
}

int32_t dg_build_hamiltonian(dg_ctx* ctx, const dg_mesh_desc* mesh, double* hdg_dev, void* work_dev,
                             size_t work_bytes) {
  DG_GUARD({
    dg::DgMeshInfo mi;
    std::vector<dg::DgElemShape> sh;
    if (int st = dg_mesh_info(ctx, mesh, mi, sh)) return st;
    if (!hdg_dev || !work_dev || ((uintptr_t)work_dev & 255)) {
      dg::set_error("hdg_dev and work_dev must be non-NULL, work_dev 256-byte aligned");
      return DG_ERR_ARG;
    }
    dg::DgPlan P;
    if (int st = dg::dg_plan(mi, sh, P)) return st;
    if (work_bytes < (size_t)P.total_doubles * sizeof(double)) {
      dg::set_error("work buffer too small: need " + std::to_string(P.total_doubles * 8) + " bytes");
      return DG_ERR_OOM;
    }
    for (const Ctx& c : ctx->g)
      if (!c.solved) {
        dg::set_error("no solve has completed on this context");
        return DG_ERR_STATE;
      }
    double* work = static_cast<double*>(work_dev);
    std::vector<std::vector<char>> keep;
    if (int st = dg::dg_upload(ctx->user, mi, sh, P, work, keep)) return st;
    if (int st = ctx->fork()) return st;
    const dg::DgElem* del = reinterpret_cast<const dg::DgElem*>(work + P.off_del);
    int st = each_group(ctx, [&](int i) {
      Ctx& c = ctx->g[i];
      c.dg_sval_off = P.off_sval + ctx->off[DG_OFF_EIG][ctx->lo[i]];
      c.dg_max_np = 0;
      for (int k = ctx->lo[i]; k < ctx->lo[i + 1]; ++k) c.dg_max_np = std::max(c.dg_max_np, mi.count[k]);
      return dg::dg_element_terms(c, work, del);
    });
    if (st < 0) return st;
    if (int s2 = ctx->join()) return s2;
    if (int s3 = dg::dg_assemble(ctx->user, P, work, hdg_dev, mi.alpha)) return s3;
    DG_HIP(hipStreamSynchronize(ctx->user));
    return DG_OK;
  })
}

int32_t dg_get_ritz(dg_ctx* ctx, double* theta_dev, double* resid_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    if (int st = ctx->fork()) return st;
    int st = each_group(ctx, [&](int i) {
      const int64_t o = ctx->off[DG_OFF_KALL][ctx->lo[i]];
      return dg::get_ritz(ctx->g[i], shift(theta_dev, o, sizeof(double)), shift(resid_dev, o, sizeof(double)));
    });
    if (st < 0) return st;
    if (int s2 = ctx->join()) return s2;
    return st;
  })
}

int32_t dg_get_vectors(dg_ctx* ctx, double* x_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    if (int st = ctx->fork()) return st;
    int st = each_group(ctx, [&](int i) {
      return dg::get_vectors(ctx->g[i], shift(x_dev, ctx->off[DG_OFF_VEC][ctx->lo[i]], sizeof(double)));
    });
    if (st < 0) return st;
    if (int s2 = ctx->join()) return s2;
    return st;
  })
}

int32_t dg_make_alb(dg_ctx* ctx, double* alb_dev, double* sval_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    if (int st = ctx->fork()) return st;
    int st = each_group(ctx, [&](int i) {
      const int a = ctx->lo[i];
      return dg::make_alb(ctx->g[i], shift(alb_dev, ctx->off[DG_OFF_ALB][a], sizeof(double)),
                          shift(sval_dev, ctx->off[DG_OFF_EIG][a], sizeof(double)));
    });
    if (st < 0) return st;
    if (int s2 = ctx->join()) return s2;
    return st;
  })
}

namespace {
std::vector<int> batch_J(const dg_ctx* ctx) {
  std::vector<int> Js;
  for (const Ctx& c : ctx->g) Js.insert(Js.end(), c.J.begin(), c.J.end());
  return Js;
}
}  // namespace

int32_t dg_query_chefsi(const dg_ctx* ctx, int32_t n_blocks, int32_t n_vec, size_t* work_bytes) {
  if (!ctx || !work_bytes || n_blocks < 0 || n_vec < 1) {
    dg::set_error("ctx and work_bytes must be non-NULL, n_blocks >= 0, n_vec >= 1");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    const std::vector<int> Js = batch_J(ctx);
    long long nb = 0;
    for (int j : Js) nb += j;
    *work_bytes = dg::chefsi_work_bytes((int)Js.size(), (int)nb, n_vec, n_blocks);
    return DG_OK;
  })
}

int32_t dg_chefsi(dg_ctx* ctx, const dg_chefsi_params* params, int32_t n_blocks, const int64_t* row_ptr,
                  const int32_t* col_idx, const int64_t* block_off, const double* hdg_dev, double* x_dev,
                  double* eig_dev, double* resid_dev, void* work_dev, size_t work_bytes, int32_t* iters_host) {
  if (!ctx || !params || !row_ptr || !block_off || (n_blocks > 0 && !col_idx) || !hdg_dev || !x_dev || !eig_dev ||
      !resid_dev || !work_dev || n_blocks < 0) {
    dg::set_error("NULL argument or n_blocks < 0");
    return DG_ERR_ARG;
  }
  if (((uintptr_t)work_dev & 255) != 0) {
    dg::set_error("work_dev must be 256-byte aligned");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    int it = 0;
    const int st = dg::chefsi(ctx->user, batch_J(ctx), *params, n_blocks, row_ptr, col_idx, block_off, hdg_dev,
                              x_dev, eig_dev, resid_dev, work_dev, work_bytes, &it);
    if (iters_host) *iters_host = it;
    return st;
  })
}

int32_t dg_density(dg_ctx* ctx, const double* alb_dev, const double* c_dev, int64_t ldc, int32_t n_e,
                   double* p_dev, double* rho_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    const int64_t rows = ctx->off[DG_OFF_EIG].back();
    if (!alb_dev || !p_dev || !rho_dev || (n_e > 0 && !c_dev)) {
      dg::set_error("alb_dev, p_dev, rho_dev (and c_dev when n_e > 0) must be non-NULL");
      return DG_ERR_ARG;
    }
    if (n_e < 0 || (n_e > 0 && ldc < rows)) {
      dg::set_error("n_e must be >= 0 and ldc >= " + std::to_string(rows) + " (the ALBs of all elements)");
      return DG_ERR_ARG;
    }
    if (int st = ctx->fork()) return st;
    int st = each_group(ctx, [&](int i) {
      const int a = ctx->lo[i];
      return dg::density(ctx->g[i], shift(alb_dev, ctx->off[DG_OFF_ALB][a], sizeof(double)),
                         shift(c_dev, ctx->off[DG_OFF_EIG][a], sizeof(double)), n_e > 0 ? ldc : 1, n_e,
                         shift(p_dev, ctx->off[DG_OFF_JJ][a], sizeof(double)),
                         shift(rho_dev, ctx->off[DG_OFF_ELEM][a], sizeof(double)));
    });
    if (st < 0) return st;
    if (int s2 = ctx->join()) return s2;
    return st;
  })
}

int32_t dg_band_energy(dg_ctx* ctx, int32_t prec, int32_t degree, const double* bounds_host,
                       int32_t n_vec, const void* psi0_dev, const double* f_dev, double* E_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    const size_t sz = prec == DG_FP32 ? sizeof(float) : sizeof(double);
    if (int st = ctx->fork()) return st;
    int st = each_group(ctx, [&](int i) {
      const int a = ctx->lo[i];
      const int64_t o = ctx->off[DG_OFF_GRID][a] * (int64_t)std::max(n_vec, 0);
      return dg::band_energy(ctx->g[i], prec, degree, bounds_host ? bounds_host + 3 * a : nullptr, n_vec,
                             shift(psi0_dev, o, sz), f_dev, E_dev ? E_dev + a : nullptr);
    });
    if (st < 0) return st;
    ctx->be_prec = prec;
    ctx->be_nvec = n_vec;
    if (int s2 = ctx->join()) return s2;
    return st;
  })
}

int32_t dg_band_energy_backward(dg_ctx* ctx, const double* dE_host, void* dpsi0_dev, void* dv_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    const size_t sz = ctx->be_prec == DG_FP32 ? sizeof(float) : sizeof(double);
    if (int st = ctx->fork()) return st;
    int st = each_group(ctx, [&](int i) {
      const int a = ctx->lo[i];
      const int64_t og = ctx->off[DG_OFF_GRID][a];
      return dg::band_energy_backward(ctx->g[i], dE_host ? dE_host + a : nullptr,
                                      shift(dpsi0_dev, og * (int64_t)ctx->be_nvec, sz),
                                      shift(dv_dev, og, sizeof(double)));
    });
    if (st < 0) return st;
    if (int s2 = ctx->join()) return s2;
    return st;
  })
}

int32_t dg_set_potential(dg_ctx* ctx, const double* v_dev) {
  if (!ctx || !v_dev) {
    dg::set_error("ctx or v_dev is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD({
    if (int st = ctx->fork()) return st;
    int st = each_group(ctx, [&](int i) {
      return dg::set_potential(ctx->g[i], shift(v_dev, ctx->off[DG_OFF_GRID][ctx->lo[i]], sizeof(double)));
    });
    if (st < 0) return st;
    if (int s2 = ctx->join()) return s2;
    return st;
  })
}

int32_t dg_timing_work(dg_ctx* ctx, double* work_host) {
  if (!ctx || !work_host) {
    dg::set_error("ctx or work_host is NULL");
    return DG_ERR_ARG;
  }
  for (int i = 0; i < dg::TC_N; ++i) {
    work_host[i] = 0.0;
    for (const Ctx& c : ctx->g) work_host[i] += c.tacc.work[i];
  }
  work_host[dg::TC_N] = 0.0;
  for (const Ctx& c : ctx->g) work_host[dg::TC_N] += c.tacc.hpsi_alg;
  return DG_OK;
}

int32_t dg_timing(dg_ctx* ctx, int32_t enable, int32_t reset, double* ms_host, int64_t* launches_host) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  for (Ctx& c : ctx->g) {
    const int st = dg::resolve_timing(c);
    if (st < 0) return st;
  }
  for (int i = 0; i < dg::TC_N; ++i) {
    double ms = 0.0;
    int64_t n = 0;
    for (const Ctx& c : ctx->g) {
      ms += c.tacc.ms[i];
      n += c.tacc.launches[i];
    }
    if (ms_host) ms_host[i] = ms;
    if (launches_host) launches_host[i] = n;
  }
  for (Ctx& c : ctx->g) {
    if (reset) c.tacc = dg::TimingAcc();
    c.timing = enable != 0;
  }
  return DG_OK;
}

}  // extern "C"
