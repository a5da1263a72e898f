// Electron density from the DG eigenvectors (Eq. (10) with the density matrix of
// Eq. (11)).  Every ALB lives on one element only, so the density on E_k needs only
// the diagonal block P_kk = C_k C_k^T of the density matrix, C_k being the J_k rows of
// the coefficients that belong to element k:
//   1. k_dens_p: P_kk, one workgroup per (element, 32 x 32 tile of the upper
//      triangle); the states are staged through LDS 64 at a time and each tile is
//      written to both triangles;
//   2. k_dens_rho: rho(r) = sum_{j,l} U[r, j] P_kk[j, l] U[r, l] with one thread per
//      point of E_k.  U is read column by column (coalesced across the wave) in
//      chunks of 16 ALBs held in registers; every pair of chunks (a <= b) takes one
//      16 x 16 block of P from LDS, off-diagonal pairs counted twice (P symmetric).
//      U is read from HBM once per chunk pair (about J / 16 times per point in
//      total, mostly from L2), P from LDS as broadcasts.
#include <algorithm>
#include <string>

#include "dg_internal.h"

namespace dg {

constexpr int kDpTile = 32;     // P tile edge
constexpr int kDpStates = 64;   // states staged per LDS round
constexpr int kDrChunk = 16;    // ALBs per register chunk

// P_kk tile (ti, tj), ti <= tj, of element e: rows ti*32.., columns tj*32..
__global__ void __launch_bounds__(256) k_dens_p(const ElemDev* elems, const long long* off_eig,
                                                 const long long* off_jj, const double* C, long long ldc, int n_e,
                                                 double* P) {
  const int e = blockIdx.y;
  const int J = elems[e].J;
  const int nt = (J + kDpTile - 1) / kDpTile;
  // upper-triangle tile index -> (ti, tj)
  int t = blockIdx.x, ti = 0;
  while (ti < nt && t >= nt - ti) {
    t -= nt - ti;
    ++ti;
  }
  if (ti >= nt) return;   // more tiles launched than this element has (uniform per workgroup)
  const int tj = ti + t;
  const double* Ck = C + off_eig[e];
  __shared__ double a[kDpStates][kDpTile + 1], b[kDpStates][kDpTile + 1];
  const int r = threadIdx.x % kDpTile, c0 = threadIdx.x / kDpTile;   // 8 column groups of 4
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s0 = 0; s0 < n_e; s0 += kDpStates) {
    __syncthreads();
    for (int x = threadIdx.x; x < kDpStates * kDpTile; x += 256) {
      const int row = x % kDpTile, s = x / kDpTile;
      const int gi = ti * kDpTile + row, gj = tj * kDpTile + row;
      const bool in = s0 + s < n_e;
      a[s][row] = (in && gi < J) ? Ck[(long long)(s0 + s) * ldc + gi] : 0.0;
      b[s][row] = (in && gj < J) ? Ck[(long long)(s0 + s) * ldc + gj] : 0.0;
    }
    __syncthreads();
    for (int s = 0; s < kDpStates; ++s) {
      const double av = a[s][r];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += av * b[s][c0 + 8 * q];
    }
  }
  double* Pk = P + off_jj[e];
  const int gi = ti * kDpTile + r;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gj = tj * kDpTile + c0 + 8 * q;
    if (gi < J && gj < J) {
      Pk[(long long)gj * J + gi] = acc[q];
      Pk[(long long)gi * J + gj] = acc[q];
    }
  }
}

__device__ inline void load_chunk(const double* U, long long nE, int r, int j0, int J, bool in, double* u) {
#pragma unroll
  for (int a = 0; a < kDrChunk; ++a) u[a] = (in && j0 + a < J) ? U[(long long)(j0 + a) * nE + r] : 0.0;
}

__global__ void __launch_bounds__(256) k_dens_rho(const ElemDev* elems, const long long* off_alb,
                                                   const long long* off_jj, const long long* off_elem,
                                                   const double* alb, const double* P, double* rho) {
  const int e = blockIdx.y;
  const ElemDev& E = elems[e];
  const int J = E.J;
  const long long nE = (long long)E.en[0] * E.en[1] * E.en[2];
  const long long r0 = (long long)blockIdx.x * 256;
  if (r0 >= nE) return;   // uniform per workgroup
  const int r = (int)(r0 + threadIdx.x);
  const bool in = r < nE;
  const double* U = alb + off_alb[e];
  const double* Pk = P + off_jj[e];
  __shared__ double pb[kDrChunk][kDrChunk + 1];
  double uj[kDrChunk], ul[kDrChunk];
  double acc = 0.0;
  for (int j0 = 0; j0 < J; j0 += kDrChunk) {
    load_chunk(U, nE, r, j0, J, in, uj);
    for (int l0 = j0; l0 < J; l0 += kDrChunk) {
      if (l0 != j0) load_chunk(U, nE, r, l0, J, in, ul);
      __syncthreads();
      {
        const int a = threadIdx.x % kDrChunk, b = threadIdx.x / kDrChunk;   // 256 = 16 x 16
        pb[a][b] = (j0 + a < J && l0 + b < J) ? Pk[(long long)(l0 + b) * J + j0 + a] : 0.0;
      }
      __syncthreads();
      double s = 0.0;
      if (l0 == j0) {
#pragma unroll
        for (int a = 0; a < kDrChunk; ++a) {
          double t = 0.0;
#pragma unroll
          for (int b = 0; b < kDrChunk; ++b) t += pb[a][b] * uj[b];
          s += uj[a] * t;
        }
      } else {
#pragma unroll
        for (int a = 0; a < kDrChunk; ++a) {
          double t = 0.0;
#pragma unroll
          for (int b = 0; b < kDrChunk; ++b) t += pb[a][b] * ul[b];
          s += 2.0 * uj[a] * t;
        }
      }
      acc += s;
    }
  }
  if (in) rho[off_elem[e] + r] = acc;
}

int density(Ctx& c, const double* alb, const double* C, long long ldc, int n_e, double* P, double* rho) {
  int jmax = 0;
  long long emax = 0;
  for (int e = 0; e < c.n_elem; ++e) {
    jmax = std::max(jmax, c.J[e]);
    emax = std::max(emax, (long long)c.en[0][e] * c.en[1][e] * c.en[2][e]);
  }
  const int nt = (jmax + kDpTile - 1) / kDpTile;
  hipLaunchKernelGGL(k_dens_p, dim3(nt * (nt + 1) / 2, c.n_elem), dim3(256), 0, c.stream, c.elems_dev,
                     c.dev_off_eig, c.dev_off_jj, C, ldc, n_e, P);
  DG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_dens_rho, dim3((unsigned)((emax + 255) / 256), c.n_elem), dim3(256), 0, c.stream,
                     c.elems_dev, c.dev_off_alb, c.dev_off_jj, c.dev_off_elem, alb, P, rho);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace dg
