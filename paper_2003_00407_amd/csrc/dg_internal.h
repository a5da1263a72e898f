// Internal types shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <map>
#include <vector>

#include "../../include/dg_alb.h"

namespace dg {

constexpr int kMaxBlocks = 8;     // solver blocks per element (roles permuted per element)
// projectors per element: the nonlocal apply stages gamma C (17 doubles per projector)
// in 64 KB of dynamic LDS
constexpr int kMaxProjectors = 480;
constexpr int kExtraBlocks = 40;  // band-energy checkpoint / segment blocks (allocated on demand)
constexpr int kTotalBlocks = kMaxBlocks + kExtraBlocks;
enum BlockId { B_X = 0, B_W = 1, B_P = 2, B_HX = 3, B_HW = 4, B_HP = 5, B_T0 = 6, B_T1 = 7 };

// Per-element data resident on the device (read-only in kernels).
struct ElemDev {
  int nx, ny, nz, N;       // Q_k grid
  int ld;                  // leading dimension of N x K blocks (elements)
  int K;                   // block width J + guards
  int J;                   // wanted states
  int elo[3], en[3];       // E_k box inside Q_k
  double kx, ky, kz;       // (2 pi / L_axis)^2 / 2: g_axis(f) = k_axis * f^2
  double vmin;             // min V_eff (preconditioner energy scale)
  const double* v64;       // V_eff, N values
  const float* v32;
  // nonlocal projectors, grouped by shared support (one group per atom)
  int ngrp, nproj;
  const int* grp_sptr;     // ngrp+1 offsets into grp_idx
  const int* grp_pbase;    // ngrp+1: first projector of each group (group g has pbase[g+1]-pbase[g])
  const int* grp_idx;      // support grid indices
  const double* grp_val64; // values, for group g projector q: grp_val[vbase + q*len + s]
  const float* grp_val32;
  const long long* grp_vbase;  // ngrp offsets into grp_val
  const double* gamma;     // nproj
  // transposed projectors over the active grid points (union of supports)
  int nact;
  const int* act_idx;      // nact grid indices
  const int* act_ptr;      // nact+1 offsets into ent_*
  const int* ent_proj;     // projector ids, ascending per point
  const double* ent_val64;
  const float* ent_val32;
  // per-element block bases (FP64 view; the FP32 view uses the same bytes);
  // blocks kMaxBlocks.. exist only when the context was created for band energies
  void* blk[kTotalBlocks];
  double bup;              // upper bound of the spectrum of H^{Q_k} (Chebyshev filter)
  double bup_base;         // its V-independent part: kinetic maximum + nonlocal Gershgorin bound
  // per-element small-matrix workspace (FP64)
  double* small;           // see SmallLayout
  double* nlc;             // projector overlaps C = B^T X: nproj x Kmax3 (FP64)
  int kmax3;               // 3 * K
};

struct SmallLayout {
  // offsets (doubles) inside ElemDev::small; sizes for K3 = 3K
  static __host__ __device__ inline long long G(int) { return 0; }
  static __host__ __device__ inline long long A(int K3) { return (long long)K3 * K3; }
  static __host__ __device__ inline long long U(int K3) { return 2LL * K3 * K3; }
  static __host__ __device__ inline long long V(int K3) { return 3LL * K3 * K3; }
  static __host__ __device__ inline long long C(int K3) { return 4LL * K3 * K3; }
  static __host__ __device__ inline long long vec(int K3) { return 5LL * K3 * K3; }  // 8 K3-vectors
  static __host__ __device__ inline long long total(int K3) { return 5LL * K3 * K3 + 8LL * K3 + 64; }
};

// vec slots inside SmallLayout::vec
enum VecSlot { VS_THETA = 0, VS_RES = 1, VS_EKIN = 2, VS_D = 3, VS_T0 = 4, VS_T1 = 5, VS_T2 = 6, VS_FLAGS = 7 };

// Shape class: elements with identical grid dims launch together.
struct ShapeClass {
  int nx, ny, nz;
  int nelem;
  int max_k;
  int* elem_list_dev;              // nelem element ids
  std::vector<int> elem_list_host;
};

// Caller buffers standing in for blocks in H*psi (block ids kExtX, kExtY): the
// no-allocation H*psi reads x and writes y in place, with the projector overlaps in
// a caller-independent scratch array instead of the element's arena slice.
constexpr int kExtX = -2, kExtY = -3;
struct ExtBufs {
  const void* x = nullptr;
  void* y = nullptr;
  long long ldx = 0, ldy = 0;          // > 0: element blocks ld x nvec; 0: packed (ld = N_k)
  int nvec = 0;
  int elem_only = -1;                  // >= 0: the buffers hold only this element's block
  const long long* off_grid = nullptr; // per element offset of its N_k values in a packed vector
  double* nlc = nullptr;               // projector overlaps, nproj_k x nvec per element
  const long long* nproj_off = nullptr;  // per element prefix of nproj (its nlc block at nproj_off * nvec)
};

// DG Hamiltonian (dg.hip): per element data in the caller's work buffer (offsets in
// doubles), indexed by the element's position in the whole batch
struct DgElem {
  int J, np;              // ALBs, projectors with support on E_k
  int en[3];              // E_k extent
  int npts[4];            // points of the faces x-, x+, y-, y+
  double inv_h[2];        // 1 / h_x, 1 / h_y
  long long l_off;        // local block (kinetic + V), J x J column-major
  long long tr_off;       // traces: per face, J values then J outward derivatives, npts each
  long long ovl_off;      // projector overlaps, np x J
  long long w_off;        // face weights: 4 faces x {value, derivative} x 64
  long long pj_off;       // projector CSR pointer (np + 1, int64)
  long long pidx_off;     // E_k-local indices (int32)
  long long pval_off;     // values (gamma: the np doubles just before)
};
struct DgMeshInfo {
  int n_mesh[2];
  double alpha;
  const int* count;
  const int* gid;
  const long long* ptr;
  const int* idx;
  const double* val;
  const double* gamma;
  std::vector<int> pbase;  // prefix of count (n_elem + 1)
};
struct DgElemShape {
  int J;
  int n[3], elo[3], en[3];
  double len[3];
};
// one block (k, nb) of H^DG: its place in the output and what contributes to it
struct DgBlock {
  int k, nb;
  int face;               // -1: no common face; 0..3: the face of k shared with nb; 4: nb = k
  int pair_lo, pair_hi;   // shared projectors (pairs of local indices) in the pair list
  long long off;          // first value in the output (doubles)
};
struct DgPlan {
  std::vector<DgElem> el;
  std::vector<DgBlock> blk;
  std::vector<long long> row_ptr;
  std::vector<int> pairs;
  long long off_del = 0, off_blk = 0, off_pairs = 0, off_sval = 0;
  long long total_doubles = 0, total_values = 0;
};
int dg_plan(const DgMeshInfo& mi, const std::vector<DgElemShape>& sh, DgPlan& P);
int dg_upload(hipStream_t s, const DgMeshInfo& mi, const std::vector<DgElemShape>& sh, const DgPlan& P,
              double* work, std::vector<std::vector<char>>& keep);

// kernel classes timed with HIP events when timing is enabled
enum TimeClass { TC_PLANE = 0, TC_ZCOL = 1, TC_NL = 2, TC_TETER = 3, TC_GRAM = 4, TC_ROT = 5, TC_RR = 6,
                 TC_OTHER = 7, TC_N = 8 };

struct TimingAcc {
  double ms[TC_N] = {0};
  int64_t launches[TC_N] = {0};
  double work[TC_N] = {0};   // algorithmic bytes (passes 0-3) or flops (4-5) of the timed launches
  double hpsi_alg = 0;       // H*psi bytes by the per-state formula 2Ns + Ns/J + nnz(s+4)/J
};

struct PendingTime {
  int cls;
  hipEvent_t a, b;
};

// H^DG as a block-sparse operator for the CheFSI on the global problem (device tables):
// element row k holds blocks row_ptr[k]..row_ptr[k+1] (column element col_idx[b],
// J_k x J_col column-major at H + boff[b]); roff: first row of each element
struct DgOp {
  int M = 0;
  bool active = false;      // the context's "H" is this operator (one pseudo-element)
  const double* H = nullptr;
  const long long* row_ptr = nullptr;
  const int* col_idx = nullptr;
  const long long* boff = nullptr;
  const long long* roff = nullptr;
  const int* J = nullptr;
};

struct Ctx {
  hipStream_t stream = nullptr;
  int n_elem = 0;
  std::vector<ElemDev> elems_host;   // host copy (device pointers inside)
  ElemDev* elems_dev = nullptr;
  std::vector<ShapeClass> classes;
  std::vector<int> J, G, K, N, ld;
  std::vector<int> elo[3], en[3];
  std::vector<int64_t> off_x0, off_vec, off_eig, off_alb, off_grid, off_kall, off_elem, off_jj;
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  bool solved = false;             // the blocks hold a solution (ALBs, vectors may be taken)
  bool have_x = false;             // X (with guards) of the last solve is intact: warm start possible
  int elem_base = 0;               // index of this group's first element in the whole batch
  int last_breakdowns = 0;         // Rayleigh-Ritz breakdowns of the X block in the last stage
  std::vector<int> nxyz[3];        // Q_k grid per element
  std::vector<double> lens[3];     // Q_k box lengths per element
  long long dg_sval_off = 0;       // DG build: this group's singular-value scratch in the work buffer
  int dg_max_np = 0;               // DG build: most projectors on one E_k of this group
  int solved_K3 = 0;
  // band-energy state
  int be_degree = 0, be_prec = 0, be_nvec = 0, be_stride = 1, be_nckpt = 0;
  std::vector<double> be_bounds;
  std::vector<double> be_alpha, be_beta, be_c;   // per element coefficient arrays
  const void* be_psi0 = nullptr;
  const double* be_f = nullptr;
  bool be_valid = false;
  void* ckpt_base = nullptr;       // checkpoint region
  size_t ckpt_bytes_per_block = 0; // sum over elements of ld*K*8
  std::vector<int64_t> ckpt_off;   // per element offset (bytes) inside one checkpoint block
  int max_cheb = 0, ckpt_stride = 1;
  // timing
  bool timing = false;
  TimingAcc tacc;
  std::vector<PendingTime> pending;
  std::vector<hipEvent_t> event_pool;
  // misc device scratch
  int* iota_dev = nullptr;         // 0..n_elem-1
  int* dev_active = nullptr;       // per element solver flags
  int* dev_status = nullptr;       // per element RR status
  int* dev_count = nullptr;        // [active count, NaN count, Rayleigh-Ritz breakdowns, -]
  int* dev_iters = nullptr;        // per element iterations performed (counted by the check kernel)
  bool capturing = false;          // a stream capture is open: no timing events
  double* dev_maxres = nullptr;    // per element max residual
  double* dev_bounds = nullptr;    // band energy: (a, b, a0) per element
  double* dev_de = nullptr;        // band energy backward: dE per element
  double* dev_minpiv = nullptr;    // diagnostics: smallest scaled overlap pivot of the last RR
  int* dev_hpflag = nullptr;       // per element: the last RR's basis is ill-conditioned (H P afresh)
  std::vector<double> be_bounds_host, be_de_host;
  int n_extra_blocks = 0;
  long long* dev_off_x0 = nullptr; // packed offsets (doubles), per element
  long long* dev_off_vec = nullptr;
  long long* dev_off_alb = nullptr;
  long long* dev_off_grid = nullptr;
  long long* dev_off_eig = nullptr;
  long long* dev_off_kall = nullptr;
  long long* dev_off_elem = nullptr;
  long long* dev_off_jj = nullptr;
  long long* dev_nproj_off = nullptr;  // per element prefix of the projector counts (n_elem + 1)
  std::vector<long long> nproj_off;    // host copy
  std::vector<int> host_ints;      // staging for small async uploads
  std::vector<int> host_ints2;      // staging of the iteration-counter reset
  std::vector<int> active_host;    // host mirror of the solver's active flags (work accounting)
  std::vector<double> nnz;         // projector nonzeros per element
  int roles_x = 0;                 // physical block holding the converged X
  double* gram_part = nullptr;
  long long gram_part_stride = 0;
  int gram_part_ld = 0;
  int gram_max_split = 16;
  std::map<long long, int> gram_split_table;   // autotuned row splits per Gram shape
  bool autotune = true;
  bool mixed_refine = false;                   // DG_MIXED_REFINE=1: refinement with FP32 search blocks after
                                               // the FP32 stage (default: FP64 LOBPCG refinement)
  bool bf16 = false;                           // DG_BF16=1: FP32 blocks' Grams and rotations as BF16x3
  bool fresh_hp_all = false;                   // DG_FRESH_HP=1: HP = H P for every element each LOBPCG step
  bool orth_w = false;                         // W <- W - X (X^T W) before the projected problem
                                               // (DG_ORTH_W=1); by default the overlap S^T S carries it                        // DG_TUNE=0 keeps the default splits
  int nl_pending_np = 0, nl_pending_kk = 0;
  DgOp dg_op;                      // set: H*psi is the block-sparse H^DG product
  int kmax = 0;                    // max K over elements
  int log_level = 0;               // DG_LOG environment variable
  double rr_pivot_tol = 1e-13;     // overlap-Cholesky breakdown threshold (FP64 data)
  double rr_drop_tol = 1e-8;       // W/P columns with smaller scaled overlap pivots leave the basis
  double rr_drop_env = -1.0;       // DG_RR_DROP override (diagnostics)
  double rr_drop_refine_env = -1.0;  // DG_RR_DROP_REFINE: the mixed refinement's drop threshold
  double hp_tol = 1e-6;            // scaled overlap pivots below this: H P applied afresh, not rotated
  double hp_tol_env = -1.0;        // DG_HP_TOL override
  double rr_ortol = 1e-5;          // cluster tolerance of the inverse iteration (relative to ||T||)
  long long* dev_phase = nullptr;  // diagnostics: RR phase timestamps (16 per element)
};

// RAII: records a HIP event pair around the launches of one kernel class
struct TimedScope {
  Ctx& c;
  int cls;
  double work;
  hipEvent_t a = nullptr, b = nullptr;
  TimedScope(Ctx& ctx, int k, double w = 0.0);
  ~TimedScope();
};
int resolve_timing(Ctx& c);

// thread-local error message
void set_error(const std::string& s);
const char* get_error();

#define DG_HIP(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::dg::set_error(std::string(#call " failed: ") + hipGetErrorString(e_));     \
      return DG_ERR_HIP;                                                           \
    }                                                                              \
  } while (0)

// ---- kernel launchers (k_hpsi.hip) ----
bool grid_supported(int nx, int ny, int nz);
int launch_hpsi(Ctx& c, int elem, int ncols, int prec, int in_blk, int out_blk, const int* active);
// H*psi on caller buffers (ext.x -> ext.y), projector overlaps in ext.nlc
int launch_hpsi_ext(Ctx& c, int elem, int ncols, int prec, const ExtBufs& ext);
int launch_teter(Ctx& c, int prec, int x_blk, int hx_blk, int w_blk, int k3, const int* active,
                 bool r_given = false);
// mixed refinement: R = HX - X theta and X in FP32 (FP64 X, HX in), and the projected
// matrices of [X W P] from the FP32 Grams of [W P X32] with [HW HP R]
int launch_mixed_split(Ctx& c, int x_blk, int hx_blk, int r_blk, int x32_blk, const int* active);
int launch_mixed_fix(Ctx& c, int nb, const int* active);

// ---- dense launchers (k_dense.hip) ----
struct ColSet {
  int nb;
  int blk[3];
};
enum RRMode { RR_GEN = 0, RR_SVD = 1, RR_CHOLQR = 2 };
struct RotArgs {
  const ElemDev* elems;
  const int* active;
  ColSet S;
  int kS;              // columns per S block (<= 0: E.K)
  int nout;            // 1 or 2
  int out_blk[2];
  int c0[2], c1[2];    // C row ranges
  double beta[2];
  double alpha;
  long long c_off;     // C matrix offset in E.small (doubles)
  int c_ld;            // <= 0: ncol
  int ncol;            // output columns (<= 0: E.K)
  int c_blockrows;     // if > 0: c0/c1 are in units of S blocks (multiplied by kS)
  int rows_e;          // 1: the first |E_k| rows only
  int add32;           // FP64 rotation, 1: the beta term reads FP32 block add32_blk[o], not the output
  int add32_blk[2];
};
int launch_gram(Ctx& c, int prec, const ColSet& S, int kS, const ColSet& T, int kT,
                long long out_off, const int* active, int sym);
int launch_rr(Ctx& c, int nb, int kfix, int nkeep, int mode, const int* active);
int launch_rotate(Ctx& c, int prec, const RotArgs& a);
int launch_residual(Ctx& c, int prec, int x_blk, int hx_blk, int ncol, const int* active);
int launch_check(Ctx& c, int* active, double tol);
void init_kernel_attributes();
int launch_gram_rows(Ctx& c, int prec, const ColSet& S, int kS, const ColSet& T, int kT,
                     long long out_off, int rows_e, int sym);
// symmetric S^T T (to out_off_st) and S^T S (to out_off_ss) from one staging of [S | T]
// where the shapes allow it, else as two Grams
int launch_gram_pair(Ctx& c, int prec, const ColSet& S, int kS, const ColSet& T, int kT, long long out_off_st,
                     long long out_off_ss, const int* active);
// caller buffer <-> block: ld == 0 packed (N_k per element), ld > 0 every element's
// block ld x ncol, element blocks ld * ncol apart
int launch_copy_ext(Ctx& c, int prec, int blk, const void* ptr, int elem, int ncol, int to_packed,
                    long long ld = 0);
// seeded Gaussian start block (counter-based: element index + elem_base, column, row)
int launch_random_block(Ctx& c, int prec, int blk, unsigned long long seed);
// per element: bup = bup_base + max(max V, 0) (after a potential update)
int launch_update_bounds(Ctx& c);
// J+g Ritz values and residuals per element into packed outputs (DG_OFF_KALL)
int launch_extract_kall(Ctx& c, double* theta, double* resid);
int launch_copy_packed(Ctx& c, int prec, int blk, const double* ptr, const long long* off, int ncol,
                       int to_packed);
int launch_gather_e(Ctx& c, int src_blk, int dst_blk);
int launch_copy_rows_out(Ctx& c, int blk, double* out);
int launch_convert(Ctx& c, int src_blk, int src_prec, int dst_blk, int dst_prec, int ncol);
int launch_extract_eig(Ctx& c, double* eig, double* resid);
int launch_extract_theta(Ctx& c, double* out);
int launch_permute(Ctx& c, const int* perm, const int* active);

// ---- drivers (solver.hip, runtime.hip) ----
int query_workspace(int n_elem, const dg_element_desc* d, const dg_options* opt, size_t* bytes);
int create(Ctx** out, int n_elem, const dg_element_desc* d, const dg_options* opt, void* arena,
           size_t arena_bytes, void* stream);
int apply_h(Ctx& c, int elem, int n_vec, int prec, const void* x, long long ldx, void* y, long long ldy);
int solve(Ctx& c, const dg_solve_params* p, double* eig, double* resid, int* iters);
int get_vectors(Ctx& c, double* x);
int make_alb(Ctx& c, double* alb, double* sval);
int density(Ctx& c, const double* alb, const double* C, long long ldc, int n_e, double* P, double* rho);
int launch_dg_bsr(Ctx& c, int in_blk, int out_blk, int ncols, const int* active);
size_t chefsi_work_bytes(int M, int Nb, int K, int n_blocks);
int chefsi(hipStream_t stream, const std::vector<int>& Js, const dg_chefsi_params& p, int n_blocks,
           const int64_t* row_ptr, const int32_t* col_idx, const int64_t* block_off, const double* hdg,
           double* x, double* eig, double* resid, void* work, size_t work_bytes, int* iters_out);
int band_energy(Ctx& c, int prec, int degree, const double* bounds_host, int n_vec, const void* psi0,
                const double* f, double* E);
int band_energy_backward(Ctx& c, const double* dE_host, void* dpsi0, void* dv);
int set_potential(Ctx& c, const double* v);
int get_ritz(Ctx& c, double* theta, double* resid);
int dg_element_terms(Ctx& c, double* work, const DgElem* del_dev);
int dg_assemble(hipStream_t s, const DgPlan& P, double* work, double* hdg, double alpha);
// no-allocation H*psi (noalloc.hip): the static scratch array and its per-device address
long long noalloc_scratch_doubles();
int noalloc_scratch(int device, double** ptr);
int apply_h_noalloc(Ctx& c, int elem, int n_vec, int prec, const void* x, long long ldx, void* y, long long ldy,
                    double* nlc);

}  // namespace dg
