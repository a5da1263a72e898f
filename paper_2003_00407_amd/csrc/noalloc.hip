// H*psi without device allocation or workspace: the caller's x and y are used in
// place, and the only scratch, the projector overlaps C = B^T x of every applied
// element, lives in a file-scope device array of fixed size.  For callers that
// cannot allocate device memory (stream capture, serving loops).
#include <map>
#include <mutex>
#include <string>

#include "dg_internal.h"

namespace dg {

// 16 MiB of FP64 projector overlaps: nproj x n_vec doubles per applied element
constexpr long long kNoAllocScratchDoubles = 2LL * 1024 * 1024;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

long long noalloc_scratch_doubles() { return kNoAllocScratchDoubles; }

// Device address of `scratch` on `device` (which must be current), resolved once
// per device: every GPU holds its own copy of the array at its own address.
int noalloc_scratch(int device, double** ptr) {
  static std::mutex mu;
  static std::map<int, double*> table;
  std::lock_guard<std::mutex> lock(mu);
  auto it = table.find(device);
  if (it != table.end()) {
    *ptr = it->second;
    return DG_OK;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    return DG_ERR_HIP;
  }
  table[device] = static_cast<double*>(p);
  *ptr = static_cast<double*>(p);
  return DG_OK;
}

// y = H x on caller buffers for one element group; nlc: this group's part of the
// scratch (nproj_off[n_elem] * n_vec doubles, checked by the caller)
int apply_h_noalloc(Ctx& c, int elem, int n_vec, int prec, const void* x, long long ldx, void* y, long long ldy,
                    double* nlc) {
  if (!x || !y || !nlc) {
    set_error("x, y or the scratch is NULL");
    return DG_ERR_ARG;
  }
  if (elem < -1 || elem >= c.n_elem) {
    set_error("elem out of range");
    return DG_ERR_ARG;
  }
  if (prec != DG_FP64 && prec != DG_FP32) {
    set_error("prec must be DG_FP64 or DG_FP32");
    return DG_ERR_ARG;
  }
  if (ldx < 0 || ldy < 0) {
    set_error("ldx and ldy must be >= 0");
    return DG_ERR_ARG;
  }
  for (int e = 0; e < c.n_elem; ++e) {
    if (elem >= 0 && e != elem) continue;
    if (n_vec <= 0 || n_vec > c.K[e] + (c.K[e] & 1)) {
      set_error("n_vec must be in [1, J_k + guards] for every element applied");
      return DG_ERR_ARG;
    }
    if ((ldx > 0 && ldx < c.N[e]) || (ldy > 0 && ldy < c.N[e])) {
      set_error("ldx / ldy below the grid size N_k of element " + std::to_string(e + c.elem_base));
      return DG_ERR_ARG;
    }
  }
  ExtBufs ext;
  ext.x = x;
  ext.y = y;
  ext.ldx = ldx;
  ext.ldy = ldy;
  ext.nvec = n_vec;
  ext.elem_only = elem;
  ext.off_grid = c.dev_off_grid;
  ext.nlc = nlc;
  ext.nproj_off = c.dev_nproj_off;
  return launch_hpsi_ext(c, elem, n_vec, prec, ext);
}

}  // namespace dg
