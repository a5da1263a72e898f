// extern "C" entry points declared in include/dg_alb.h: argument checks and
// dispatch only; no exception crosses this boundary.
#include <exception>
#include <string>

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

struct dg_ctx {
  Ctx impl;
};

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
  DG_GUARD(return dg::query_workspace(n_elem, elems, opt, bytes);)
}

int32_t dg_create_elements(dg_ctx** ctx, int32_t n_elem, const dg_element_desc* elems,
                           const dg_options* opt, void* dev_arena, size_t arena_bytes, void* hip_stream) {
  DG_GUARD({
    if (!ctx) {
      dg::set_error("ctx is NULL");
      return DG_ERR_ARG;
    }
    *ctx = nullptr;
    Ctx* c = nullptr;
    int st = dg::create(&c, n_elem, elems, opt, dev_arena, arena_bytes, hip_stream);
    if (st < 0) return st;
    dg_ctx* h = new dg_ctx();
    h->impl = std::move(*c);
    delete c;
    *ctx = h;
    return st;
  })
}

void dg_destroy(dg_ctx* ctx) { delete ctx; }

int32_t dg_query_offsets(const dg_ctx* ctx, int32_t kind, int64_t* offsets) {
  if (!ctx || !offsets) {
    dg::set_error("ctx or offsets is NULL");
    return DG_ERR_ARG;
  }
  const Ctx& c = ctx->impl;
  const std::vector<int64_t>* v = nullptr;
  switch (kind) {
    case DG_OFF_X0: v = &c.off_x0; break;
    case DG_OFF_VEC: v = &c.off_vec; break;
    case DG_OFF_EIG: v = &c.off_eig; break;
    case DG_OFF_ALB: v = &c.off_alb; break;
    case DG_OFF_GRID: v = &c.off_grid; break;
    case DG_OFF_KALL: v = &c.off_kall; break;
    default: dg::set_error("unknown offset kind"); return DG_ERR_ARG;
  }
  for (size_t i = 0; i < v->size(); ++i) offsets[i] = (*v)[i];
  return DG_OK;
}

int32_t dg_apply_H(dg_ctx* ctx, int32_t elem, int32_t n_vec, int32_t prec, const void* x_dev,
                   void* y_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD(return dg::apply_h(ctx->impl, elem, n_vec, prec, x_dev, y_dev);)
}

int32_t dg_solve_elements(dg_ctx* ctx, const dg_solve_params* params, double* eig_dev,
                          double* resid_dev, int32_t* iters_host) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD(return dg::solve(ctx->impl, params, eig_dev, resid_dev, iters_host);)
}

int32_t dg_get_vectors(dg_ctx* ctx, double* x_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD(return dg::get_vectors(ctx->impl, x_dev);)
}

int32_t dg_make_alb(dg_ctx* ctx, double* alb_dev, double* sval_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD(return dg::make_alb(ctx->impl, alb_dev, sval_dev);)
}

int32_t dg_band_energy(dg_ctx* ctx, int32_t prec, int32_t degree, const double* bounds_host,
                       int32_t n_vec, const void* psi0_dev, const double* f_dev, double* E_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD(return dg::band_energy(ctx->impl, prec, degree, bounds_host, n_vec, psi0_dev, f_dev, E_dev);)
}

int32_t dg_band_energy_backward(dg_ctx* ctx, const double* dE_host, void* dpsi0_dev, void* dv_dev) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD(return dg::band_energy_backward(ctx->impl, dE_host, dpsi0_dev, dv_dev);)
}

int32_t dg_set_potential(dg_ctx* ctx, const double* v_dev) {
  if (!ctx || !v_dev) {
    dg::set_error("ctx or v_dev is NULL");
    return DG_ERR_ARG;
  }
  DG_GUARD(return dg::set_potential(ctx->impl, v_dev);)
}

int32_t dg_timing_work(dg_ctx* ctx, double* work_host) {
  if (!ctx || !work_host) {
    dg::set_error("ctx or work_host is NULL");
    return DG_ERR_ARG;
  }
  for (int i = 0; i < dg::TC_N; ++i) work_host[i] = ctx->impl.tacc.work[i];
  return DG_OK;
}

int32_t dg_timing(dg_ctx* ctx, int32_t enable, int32_t reset, double* ms_host, int64_t* launches_host) {
  if (!ctx) {
    dg::set_error("ctx is NULL");
    return DG_ERR_ARG;
  }
  Ctx& c = ctx->impl;
  int st = dg::resolve_timing(c);
  if (st < 0) return st;
  if (ms_host)
    for (int i = 0; i < dg::TC_N; ++i) ms_host[i] = c.tacc.ms[i];
  if (launches_host)
    for (int i = 0; i < dg::TC_N; ++i) launches_host[i] = c.tacc.launches[i];
  if (reset) c.tacc = dg::TimingAcc();
  c.timing = enable != 0;
  return DG_OK;
}

}  // extern "C"
