"""Electron density from the DG eigenvectors (oracle, FP64, test infrastructure).

Only the tests, the smoke check and the benchmark's CPU leg use this module.

The Kohn-Sham orbitals are expanded in the ALBs, psi_i = sum_{k,j} C_{i;k,j}
phi_{k,j} (Eq. (6)), and the density is the sum of their squares (Eq. (10), first
line).  Every ALB vanishes outside its own element, so on E_k only element k's terms
survive and the density there is sum_{j,j'} phi_{k,j} phi_{k,j'} P_{k,j;k,j'} (Eq.
(10), last line) with P the density matrix of Eq. (11): only its diagonal blocks
P_kk = C_k C_k^T enter, and each element needs only its own.

Readings (where the paper leaves the discretisation open):
  R1  Grid functions are Euclidean-normalised as in the DG Hamiltonian (an ALB has
      unit 2-norm over E_k's points), so rho is a value per grid point: its sum over
      all points is trace(C^T C) (N_e for orthonormal C); the physical density is
      rho / dV.
  R2  The sum over states runs over the N_e columns of C with unit weight, as
      printed; occupations or a spin factor are folded into C's columns (scale
      column i by sqrt(f_i)).
  R3  C is stored with one row per ALB, element-major (element k's J_k rows follow
      element k-1's), and one column per state.
"""
from __future__ import annotations

import numpy as np

__all__ = ["row_offsets", "density_matrix_blocks", "density", "density_from_orbitals"]


def row_offsets(Js) -> np.ndarray:
    """First row of each element's ALB coefficients in C (R3)."""
    return np.concatenate([[0], np.cumsum(Js)]).astype(np.int64)


def density_matrix_blocks(C: np.ndarray, Js) -> list:
    """Diagonal blocks P_kk = sum_i C_{i;k,.} C_{i;k,.}^T of Eq. (11)."""
    off = row_offsets(Js)
    return [C[off[k]:off[k + 1], :] @ C[off[k]:off[k + 1], :].T for k in range(len(Js))]


def density(U: list, C: np.ndarray, Js) -> list:
    """rho on every element's points from the diagonal blocks of P (Eq. (10), last
    line): rho_k(r) = sum_{j,j'} U_k[r, j] P_kk[j, j'] U_k[r, j']; U_k holds the ALB
    values of element k on E_k (|E_k| x J_k)."""
    P = density_matrix_blocks(C, Js)
    return [np.einsum("rj,jl,rl->r", U[k], P[k], U[k]) for k in range(len(Js))]


def density_from_orbitals(U: list, C: np.ndarray, Js, elem_global_indices, n_global: int) -> np.ndarray:
    """rho on the global grid from the orbitals themselves (Eq. (10), first line):
    each psi_i is assembled point by point over the whole domain from every element's
    ALB values (Eq. (6)), then squared and summed over the states."""
    off = row_offsets(Js)
    psi = np.zeros((n_global, C.shape[1]))
    for k in range(len(Js)):
        psi[elem_global_indices(k), :] += U[k] @ C[off[k]:off[k + 1], :]
    return np.sum(psi * psi, axis=1)
