/*
 * dg_alb.h -- batched adaptive-local-basis (ALB) generation on one AMD MI355X.
 *
 * The library solves, for a batch of extended elements Q_k, the local
 * Kohn-Sham eigenproblem of Eq. (1) (LocalKS)
 *
 *     H^{Q_k} phi = (-1/2 Laplacian + V_eff + sum_{I,l} gamma_{I,l} |b_{I,l}><b_{I,l}|) phi
 *                 = lambda phi
 *
 * in the plane-wave basis of the periodic box Q_k (every grid plane wave,
 * Nyquist mode included), for the lowest J_k eigenpairs ("Generating ALB
 * functions" subsection), by LOBPCG (Algorithm 1, Eqs. (2)-(4)) or by
 * Chebyshev-filtered subspace iteration (Algorithm 2 and Eqs. (8)-(9),
 * applied to H^{Q_k}), then restricts the eigenvectors to the element E_k and
 * orthonormalises them there into ALBs.
 *
 * Conventions (all entry points):
 *  - Grid vectors are real FP64 or FP32 arrays of N = n[0]*n[1]*n[2] values,
 *    x fastest: index = x + n[0]*(y + n[1]*z).  Vectors are Euclidean
 *    normalised on the grid (x^T x = 1).
 *  - "Packed" blocks hold, element after element, an N_k x m_k column-major
 *    matrix with leading dimension N_k (one state per contiguous column).
 *    dg_query_offsets gives the start of each element's block.
 *  - Pointers named *_dev are device pointers (HBM), *_host are host
 *    pointers.  Device buffers are owned by the caller and must stay alive
 *    until the work queued on the context's stream has completed.
 *  - Every function returns a dg_status.  Negative = error, no output is
 *    valid.  Positive = warning, outputs are valid.  No exception or abort
 *    crosses the interface.  dg_last_error() describes the last failure on
 *    the calling thread.
 *  - A context is bound to one HIP stream (the caller's) and is not
 *    thread-safe.  Internally the elements may be split into groups that run
 *    on library-owned streams (dg_options.n_streams); their work is ordered
 *    after the work already queued on the caller's stream and the caller's
 *    stream waits for it, so the caller sees one stream.  The library never
 *    allocates device memory: the caller provides one arena of the size
 *    dg_query_workspace reports.
 *  - Environment variables read by dg_create_elements (tuning and
 *    diagnostics): DG_STREAMS (element groups when n_streams <= 0);
 *    DG_TUNE=0 (no timing of the Gram row split, the size heuristic is
 *    used); DG_LOG (progress on stderr: 1 residuals per iteration and the
 *    tuner's choices, 2 Rayleigh-Ritz phase times, 3 Cholesky pivots; any
 *    level > 0 turns graph capture off); DG_RR_ORTOL (inverse-iteration
 *    cluster tolerance relative to ||T||, default 1e-5); DG_RR_DROP
 *    (threshold on the scaled-overlap pivot below which a W or P column
 *    leaves the basis; default 1e-8 in FP64, 1e-4 in the FP32 stage);
 *    DG_ORTH_W=1 (W is made orthogonal to X before the projected problem).
 */
#ifndef DG_ALB_H
#define DG_ALB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

enum dg_status {
  DG_OK = 0,
  DG_WARN_NOT_CONVERGED = 1, /* outputs valid; residuals above tolerance */
  DG_ERR_ARG = -1,           /* invalid argument (NULL, out of range)   */
  DG_ERR_SHAPE = -2,         /* unsupported grid / sizes                */
  DG_ERR_OOM = -3,           /* arena too small                         */
  DG_ERR_HIP = -4,           /* HIP runtime error (see dg_last_error)   */
  DG_ERR_NUMERIC = -5,       /* NaN/Inf or unrecoverable breakdown      */
  DG_ERR_STATE = -6          /* call out of order (e.g. ALB before solve) */
};

enum dg_prec {
  DG_FP64 = 0,  /* every step in FP64                                            */
  DG_MIXED = 1, /* FP32 H*psi and subspace GEMMs, FP64 small dense; then FP64    */
                /* refinement sweeps to the requested tolerance                  */
  DG_FP32 = 2   /* FP32 H*psi (dg_apply_H, dg_band_energy only)                  */
};

enum dg_method {
  DG_LOBPCG = 0, /* Algorithm 1 */
  DG_CHFSI = 1   /* Algorithm 2 applied to H^{Q_k} */
};

/* One extended element Q_k (Eq. (1)); host pointers, copied by dg_create_elements. */
typedef struct {
  int32_t n[3];        /* grid points of Q_k along x, y, z                         */
  double len[3];       /* box lengths (bohr); grid spacing len[i]/n[i]             */
  int32_t elem_lo[3];  /* first grid point of E_k inside Q_k                       */
  int32_t elem_n[3];   /* grid points of E_k                                       */
  int32_t n_states;    /* J_k wanted eigenpairs                                    */
  const double *v_eff; /* N values of V_eff on Q_k (Ha)                            */
  int32_t n_proj;      /* number of projectors b_{I,l} with support in Q_k (<= 480) */
  const int64_t *proj_ptr; /* n_proj+1 offsets into proj_idx / proj_val (CSC of B) */
  const int32_t *proj_idx; /* grid indices, strictly ascending within a projector  */
  const double *proj_val;  /* b_{I,l} values                                       */
  const double *gamma;     /* n_proj weights gamma_{I,l} (Ha)                      */
} dg_element_desc;

typedef struct {
  int32_t n_guard;        /* guard states carried above J_k; < 0: max(4, ceil(J_k/5)),  */
                          /* reduced (not below 4) where J_k + guards would pass 88     */
  int32_t max_cheb_degree;/* largest Chebyshev degree used by dg_band_energy (0: none)  */
  int32_t ckpt_stride;    /* checkpoint every ckpt_stride filter steps (>= 1)           */
  int32_t n_streams;      /* element groups solved concurrently, each on its own HIP     */
                          /* stream and host thread (<= 0: n_elem / 4 clamped to 1..4,  */
                          /* or the DG_STREAMS value)                                   */
} dg_options;

typedef struct {
  int32_t method;      /* dg_method                                                   */
  int32_t precision;   /* DG_FP64 or DG_MIXED                                         */
  double tol;          /* converged when max_i ||H x_i - theta_i x_i||_2 <= tol (Ha)  */
                       /* over the J_k wanted states of every element                */
  double tol_mixed;    /* DG_MIXED: residual at which the FP32 stage hands over to    */
                       /* FP64 refinement (<= 0: 3e-5)                                */
  int32_t max_iter;    /* iteration cap per stage                                     */
  int32_t cheb_degree; /* DG_CHFSI filter degree m                                    */
  const double *x0_dev;/* packed initial blocks, N_k x (J_k + guards) per element     */
                       /* (dg_query_offsets(DG_OFF_X0)); need not be orthonormal.     */
                       /* NULL: a seeded Gaussian start drawn on the device from      */
                       /* seed (counter-based, so one seed gives one start for every  */
                       /* element, independent of the element groups)                 */
  int32_t graph_iters; /* FP64 LOBPCG: > 0 captures this many iterations of every     */
                       /* element group as one HIP graph, replayed with one host      */
                       /* convergence check per replay (the count may then overshoot */
                       /* max_iter by less than graph_iters); 0: launch per kernel     */
  int64_t seed;        /* seed of the device-drawn start (x0_dev == NULL)             */
  int32_t warm_start;  /* nonzero: start from the eigenvectors and guard vectors of   */
                       /* the last solve on this context (x0_dev and seed ignored),   */
                       /* e.g. after dg_set_potential in an inner SCF step, where the */
                       /* ALBs adapt to the updated V_eff; DG_ERR_STATE if no solve   */
                       /* has left vectors on the context since the last band-energy */
                       /* call                                                        */
} dg_solve_params;

enum dg_offset_kind {
  DG_OFF_X0 = 0,   /* packed N_k x (J_k+g_k) blocks (x0_dev)            */
  DG_OFF_VEC = 1,  /* packed N_k x J_k blocks (dg_get_vectors)           */
  DG_OFF_EIG = 2,  /* J_k values per element (eigenvalues, residuals)    */
  DG_OFF_ALB = 3,  /* packed |E_k| x J_k blocks (dg_make_alb)            */
  DG_OFF_GRID = 4, /* N_k values per element (V, dE/dV)                  */
  DG_OFF_KALL = 5, /* J_k+g_k values per element                         */
  DG_OFF_ELEM = 6, /* |E_k| values per element (density)                 */
  DG_OFF_JJ = 7    /* J_k x J_k blocks (density-matrix diagonal blocks)   */
};

/* Human-readable name of a status code (static string). */
const char *dg_status_string(int32_t status);

/* Description of the last error on the calling thread (ctx may be NULL). */
const char *dg_last_error(const dg_ctx *ctx);

/* Arena bytes needed for these elements and options.  CPU only: validates the
 * descriptors and never touches the GPU.  Errors: DG_ERR_ARG, DG_ERR_SHAPE. */
int32_t dg_query_workspace(int32_t n_elem, const dg_element_desc *elems,
                           const dg_options *opt, size_t *bytes);

/* Create a context: copies the element data (Eq. (1)'s V_eff, b, gamma and the
 * E_k boxes) into the caller's device arena on hip_stream, and builds the
 * batch plan.  dev_arena must hold arena_bytes >= dg_query_workspace's value,
 * 256-byte aligned.  *ctx is set on success and must be released with
 * dg_destroy.  Errors: DG_ERR_ARG, DG_ERR_SHAPE, DG_ERR_OOM, DG_ERR_HIP. */
int32_t dg_create_elements(dg_ctx **ctx, int32_t n_elem, const dg_element_desc *elems,
                           const dg_options *opt, void *dev_arena, size_t arena_bytes,
                           void *hip_stream);

/* Release the context (host memory only; the arena stays the caller's). */
void dg_destroy(dg_ctx *ctx);

/* Offsets (in elements of the block's value type) of each element's part of a
 * packed buffer, n_elem + 1 values (last = total).  CPU only. */
int32_t dg_query_offsets(const dg_ctx *ctx, int32_t kind, int64_t *offsets);

/* y = H^{Q_k} x (Eq. (1)) for n_vec vectors per element: kinetic term by line
 * FFTs, local potential, nonlocal projectors.  elem = -1 applies every element,
 * elem >= 0 element elem only.  Layout of x_dev (and likewise y_dev with ldy):
 * ldx == 0: packed, N_k x n_vec column-major per element (leading dimension
 * N_k), the elements' blocks concatenated (for elem >= 0 the one block);
 * ldx > 0: every element's block is ldx x n_vec column-major (ldx >= N_k of
 * every element applied), element blocks ldx * n_vec values apart (elem >= 0:
 * the one block at x_dev).  prec = DG_FP64: double buffers; DG_FP32: float
 * buffers.  x and y must not overlap.  n_vec must not exceed J_k + g_k of any
 * element applied.  Errors: DG_ERR_ARG (NULL, ranges, ld too small), DG_ERR_HIP. */
int32_t dg_apply_H(dg_ctx *ctx, int32_t elem, int32_t n_vec, int32_t prec,
                   const void *x_dev, int64_t ldx, void *y_dev, int64_t ldy);

/* dg_apply_H for callers that cannot allocate device memory (code under HIP
 * stream capture, tight serving loops): the same y = H x, arguments and layouts
 * as dg_apply_H, but x is read and y written in place, without staging through
 * the context's workspace, and the only scratch, the projector overlaps
 * C = B^T x (nproj_k x n_vec FP64 values per applied element), lives in a
 * library-owned static device array of 16 MiB per GPU, resolved when the
 * context is created.  No device memory is allocated by the call.  Calls that
 * overlap in time on one GPU (any context, any stream) share that array and
 * race; the array keeps the last call's contents.  The solver's vectors are left
 * untouched.  Errors: DG_ERR_ARG (as dg_apply_H, and when the overlaps of the
 * call exceed the array: apply fewer vectors or one element per call),
 * DG_ERR_HIP. */
int32_t dg_apply_H_noalloc(dg_ctx *ctx, int32_t elem, int32_t n_vec, int32_t prec,
                           const void *x_dev, int64_t ldx, void *y_dev, int64_t ldy);

/* Lowest J_k eigenpairs of every H^{Q_k} ("Generating ALB functions";
 * Algorithm 1 or 2).  eig_dev, resid_dev: J_k FP64 values per element
 * (DG_OFF_EIG); iters_host: n_elem iteration counts (may be NULL).  The
 * eigenvectors stay in the context for dg_make_alb / dg_get_vectors and for a
 * warm-started solve.  Returns DG_WARN_NOT_CONVERGED when some element missed
 * tol after max_iter.  Errors: DG_ERR_ARG; DG_ERR_STATE (warm_start without
 * vectors); DG_ERR_NUMERIC: a non-finite residual (NaN/Inf in V_eff or the
 * start), a rank-deficient start block (the Cholesky of X_0^T X_0 breaks
 * down, e.g. repeated columns), or an element that did not converge after a
 * Rayleigh-Ritz breakdown of its X block; DG_ERR_HIP. */
int32_t dg_solve_elements(dg_ctx *ctx, const dg_solve_params *params, double *eig_dev,
                          double *resid_dev, int32_t *iters_host);

/* All J_k + g_k Ritz values of the last solve (the J_k wanted states, then the
 * guard states) and their residual norms, FP64, packed per element
 * (DG_OFF_KALL).  The guards bound the gap lambda_{J+1} - lambda_J that
 * conditions the ALB subspace: theta_{J+1} - theta_J near zero means the cut at
 * J_k splits a (nearly) degenerate cluster and the ALB span is not unique.
 * Errors: DG_ERR_STATE before a solve, DG_ERR_ARG. */
int32_t dg_get_ritz(dg_ctx *ctx, double *theta_dev, double *resid_dev);

/* Copy the converged eigenvectors (first J_k columns, FP64) to x_dev, packed
 * N_k x J_k per element (DG_OFF_VEC).  Errors: DG_ERR_STATE before a solve. */
int32_t dg_get_vectors(dg_ctx *ctx, double *x_dev);

/* ALBs: restrict the J_k eigenvectors to E_k and orthonormalise them there
 * ("Generating ALB functions": truncated to E_k, orthonormal on E_k).
 * alb_dev: packed |E_k| x J_k FP64 (DG_OFF_ALB), columns orthonormal, spanning
 * the restricted eigenvectors; sval_dev: J_k singular values of the
 * restriction, descending (DG_OFF_EIG).  Errors: DG_ERR_STATE before a solve,
 * DG_ERR_NUMERIC if the restriction is rank deficient for some element
 * (sigma_min <= 1e-10 sigma_max, or the orthonormalisation breaks down): the
 * outputs are then not valid. */
int32_t dg_make_alb(dg_ctx *ctx, double *alb_dev, double *sval_dev);

/* The element mesh of the global problem, for the DG Hamiltonian (Eq. (7),
 * DGHamiltonian).  The context's elements, in order, are the elements E_k of an
 * n_mesh[0] x n_mesh[1] periodic 2D mesh (element k at (k % n_mesh[0],
 * k / n_mesh[0])); each spans the whole periodic z range and shares its x and y
 * faces with its neighbours, which must have the same E_k extent along the face.
 * Projectors: every projector b_{I,l} with support on E_k, restricted to E_k,
 * with a global id that identifies the same projector in other elements. */
typedef struct {
  int32_t n_mesh[2];         /* elements along x and y, >= 3 each                        */
  double alpha;              /* interior-penalty parameter (Ha bohr)                     */
  const int32_t *proj_count; /* per element: projectors with support on E_k               */
  const int32_t *proj_gid;   /* their global ids, the elements' lists concatenated        */
  const int64_t *proj_ptr;   /* sum(proj_count) + 1 offsets into proj_idx / proj_val       */
  const int32_t *proj_idx;   /* E_k-local grid indices (x fastest inside E_k), ascending   */
  const double *proj_val;    /* values on E_k (the global projector's, unnormalised)       */
  const double *gamma;       /* per projector weight (Ha)                                 */
} dg_mesh_desc;

/* Block-sparse layout of H^DG for dg_build_hamiltonian: row k holds the blocks
 * (k, col_idx[b]) for b in [row_ptr[k], row_ptr[k+1]), the distinct elements that
 * are k itself, share a face with it, or share a projector with it, in ascending
 * order; block b is J_k x J_col column-major (ld J_k) at block_off[b] doubles
 * (n_blocks + 1 values, last = total).  Call with row_ptr = col_idx = block_off =
 * NULL to get *n_blocks and *work_bytes (the device workspace of the build), then
 * with arrays of n_elem + 1, n_blocks and n_blocks + 1 values.  CPU only (host mesh
 * data is read).  Errors: DG_ERR_ARG, DG_ERR_SHAPE. */
int32_t dg_query_hamiltonian(const dg_ctx *ctx, const dg_mesh_desc *mesh, int32_t *n_blocks, int64_t *row_ptr,
                             int32_t *col_idx, int64_t *block_off, size_t *work_bytes);

/* The DG Hamiltonian H^DG (Eq. (7)) in the ALB basis of the last solve: per
 * element the kinetic and local-potential block 1/2 <grad phi, grad phi'> +
 * <phi, V phi'> over E_k; the nonlocal coupling sum gamma <phi, b><b, phi'> of
 * every pair of elements sharing a projector; and the interior-penalty face terms
 * -1/2 <[[phi]], {{grad phi'}}> - 1/2 <{{grad phi}}, [[phi']]> + alpha <[[phi]],
 * [[phi']]> of the four faces of every element.  ALBs are the orthonormal bases
 * of dg_make_alb; inside E_k and on its faces they are evaluated as the
 * trigonometric polynomials on Q_k whose restriction they are (gradients by the
 * spectral derivative on Q_k, traces by trigonometric interpolation half a grid
 * step beyond E_k's outer points); element and face integrals are rectangle sums
 * of the Euclidean-normalised grid functions (a face sum carries 1 / h_normal).
 * hdg_dev: the blocks (dg_query_hamiltonian); work_dev: work_bytes of device
 * scratch (256-byte aligned).  Uses the solver's work blocks (call dg_make_alb or
 * dg_get_vectors before it if needed; X stays for warm starts).  Errors:
 * DG_ERR_STATE before a solve, DG_ERR_ARG, DG_ERR_SHAPE (mesh does not match the
 * elements), DG_ERR_NUMERIC (rank-deficient restriction), DG_ERR_HIP. */
int32_t dg_build_hamiltonian(dg_ctx *ctx, const dg_mesh_desc *mesh, double *hdg_dev, void *work_dev,
                             size_t work_bytes);

/* CheFSI on the DG Hamiltonian (Algorithm 2; H^DG X by the block-row product of
 * Eq. (8)). */
typedef struct {
  int32_t n_want;        /* wanted lowest eigenpairs N_e (the residual test)          */
  int32_t n_vec;         /* block width N_e + guards, <= 88 and <= N_b / 2            */
  int32_t degree;        /* Chebyshev filter degree m (1..64; the paper uses 10-40)   */
  int32_t max_iter;      /* filter passes (each: filter, Cholesky-QR, projected eig)   */
  double tol;            /* max ||H x_i - theta_i x_i|| over the wanted pairs          */
  int32_t lanczos_steps; /* steps of the Lanczos run for b_up (0: 10)                  */
  int32_t reserved;      /* 0                                                          */
  int64_t seed;          /* Lanczos start vector (counter-based Gaussian draw)         */
} dg_chefsi_params;

/* Device workspace bytes of dg_chefsi for a block-sparse H^DG with n_blocks blocks
 * over this context's elements (N_b = sum_k J_k rows) and n_vec columns.  CPU only.
 * Errors: DG_ERR_ARG. */
int32_t dg_query_chefsi(const dg_ctx *ctx, int32_t n_blocks, int32_t n_vec, size_t *work_bytes);

/* Lowest eigenpairs of H^DG by CheFSI (Algorithm 2): b_up from a Lanczos run, b_low
 * and the lowest-eigenvalue estimate from the previous Ritz values (the first from a
 * Rayleigh-Ritz step on the start block), then per pass the degree-m filter, Cholesky
 * orthonormalisation, projected eigenproblem and rotation, until the n_want residuals
 * are below tol.  The matrix is given as dg_build_hamiltonian writes it: hdg_dev on
 * the device with the host layout row_ptr (n_elem + 1), col_idx (n_blocks), block_off
 * (n_blocks + 1), rows of element k being its J_k ALBs (DG_OFF_EIG offsets).
 * x_dev: in: the start block, column-major N_b x n_vec (ld N_b), full rank; out: the
 * Ritz vectors, ascending.  eig_dev, resid_dev: n_vec Ritz values and residual norms.
 * work_dev: dg_query_chefsi bytes, 256-byte aligned.  Runs on the caller's stream and
 * returns after it.  Returns DG_WARN_NOT_CONVERGED when tol was missed after max_iter.
 * Errors: DG_ERR_ARG (NULL, layout that does not match the elements' J_k, parameters
 * out of range), DG_ERR_SHAPE (n_vec above 88 or N_b / 2), DG_ERR_OOM (work too small),
 * DG_ERR_NUMERIC (non-finite residual, rank-deficient start block), DG_ERR_HIP. */
int32_t dg_chefsi(dg_ctx *ctx, const dg_chefsi_params *params, int32_t n_blocks, const int64_t *row_ptr,
                  const int32_t *col_idx, const int64_t *block_off, const double *hdg_dev, double *x_dev,
                  double *eig_dev, double *resid_dev, void *work_dev, size_t work_bytes, int32_t *iters_host);

/* Electron density from the DG eigenvectors (Eq. (10)) through the diagonal blocks of
 * the density matrix (Eq. (11)): every ALB lives on its own element, so on E_k
 * rho(r) = sum_{j,l} phi_{k,j}(r) P_kk[j, l] phi_{k,l}(r) with P_kk = C_k C_k^T, C_k the
 * J_k rows of C that belong to element k.  alb_dev: the ALB values (dg_make_alb layout,
 * DG_OFF_ALB: |E_k| x J_k column-major per element, Euclidean-normalised);
 * c_dev: FP64 column-major (sum_k J_k) x n_e with leading dimension ldc >= sum_k J_k,
 * element k's rows starting at its DG_OFF_EIG offset, one column per state with unit
 * weight (fold occupations into the columns as sqrt(f_i)); p_dev: out, P_kk per
 * element, J_k x J_k column-major (DG_OFF_JJ); rho_dev: out, rho on E_k's points
 * (DG_OFF_ELEM), per grid point (sum over all points = trace C^T C; the physical
 * density is rho / dV).  n_e = 0 gives zeros.  Needs no solve (pure function of its
 * inputs and the element shapes); asynchronous on the caller's stream.  Errors:
 * DG_ERR_ARG (NULL, n_e < 0, ldc too small), DG_ERR_HIP. */
int32_t dg_density(dg_ctx *ctx, const double *alb_dev, const double *c_dev, int64_t ldc, int32_t n_e,
                   double *p_dev, double *rho_dev);

/* Band energy E = sum_i f_i psi_i^T H psi_i with Psi = p_m(H) Psi_0, p_m the
 * degree-m scaled Chebyshev filter of Algorithm 2 / Eq. (8) with bounds
 * (a, b, a0) per element (bounds_host: 3 host values per element, a0 < a < b;
 * the coefficients are held fixed, not differentiated), for n_vec columns per
 * element.  psi0_dev: packed N_k x n_vec (FP64 for DG_FP64, FP32 for DG_FP32);
 * f_dev: n_vec FP64 weights (device, same for every element, kept alive until
 * the backward call); E_dev: one FP64 energy per element.  Every ckpt_stride-th
 * pair of filter iterates is kept for dg_band_energy_backward.  The context
 * must have been created with max_cheb_degree >= degree.  Overwrites the
 * solver's blocks (call dg_solve_elements again before dg_make_alb).
 * Errors: DG_ERR_ARG. */
int32_t dg_band_energy(dg_ctx *ctx, int32_t prec, int32_t degree, const double *bounds_host,
                       int32_t n_vec, const void *psi0_dev, const double *f_dev, double *E_dev);

/* Gradient of the last dg_band_energy call, scaled per element by dE_host[k]
 * (the upstream gradient): dpsi0_dev = dE dE/dPsi_0 (packed like psi0, its
 * precision) by the adjoint three-term recurrence, recomputing each
 * checkpointed segment of the filter; dv_dev = dE dE/dV_eff (FP64, N_k per
 * element, DG_OFF_GRID).  Errors: DG_ERR_STATE without a preceding
 * dg_band_energy. */
int32_t dg_band_energy_backward(dg_ctx *ctx, const double *dE_host, void *dpsi0_dev,
                                void *dv_dev);

/* Replace V_eff of every element (v_dev: FP64 device buffer, packed N_k per
 * element, DG_OFF_GRID), e.g. for an inner SCF step ("Generating ALB
 * functions": the ALBs adapt as V_eff changes) or for finite differences in V.
 * The spectral upper bound used by the Chebyshev filter is recomputed from the
 * new maximum of V_eff.  The eigenvectors of the last solve are kept as a
 * warm start (dg_solve_params.warm_start) but no longer count as a solution:
 * dg_make_alb and dg_get_vectors need a new solve.  A pending band energy is
 * invalidated (its backward returns DG_ERR_STATE).  Errors: DG_ERR_ARG. */
int32_t dg_set_potential(dg_ctx *ctx, const double *v_dev);

/* Algorithmic work of the launches timed since the last reset (9 values):
 * [0..7] per class of dg_timing: bytes for classes 0-3 (each pass's own minimal
 * reads and writes), flops for classes 4-5 (2 r n_i n_j per product, r n (n+1)
 * for a symmetric n x n Gram), 0 for 6-7; [8] the bytes of the H*psi state
 * applications (classes 0-2 together) by the per-state count 2 N s + N s / J +
 * nnz (s + 4) / J (read psi, write H psi, V and the projectors amortised over
 * the J wanted states; s = 8 or 4 bytes).  Call before a resetting dg_timing.
 * Errors: DG_ERR_ARG. */
int32_t dg_timing_work(dg_ctx *ctx, double *work_host);

/* Per-kernel-class GPU time accumulated since the last reset, measured with
 * HIP events recorded on the context's stream around each launch group.
 * Classes (8): 0 plane pass of H*psi (x/y line FFTs + V), 1 z-column pass,
 * 2 nonlocal overlap/apply, 3 Teter preconditioner (three passes), 4 Gram
 * GEMMs (+ split reduction), 5 rotations, 6 Rayleigh-Ritz small dense,
 * 7 other.  ms_host[8], launches_host[8] (may be NULL) receive the totals,
 * then reset != 0 clears them and enable sets timing on or off (default off).
 * Synchronises the stream.  Errors: DG_ERR_ARG, DG_ERR_HIP. */
int32_t dg_timing(dg_ctx *ctx, int32_t enable, int32_t reset, double *ms_host,
                  int64_t *launches_host);

#ifdef __cplusplus
}
#endif

#endif /* DG_ALB_H */
