"""ALB construction and subspace comparison (oracle, FP64, test infrastructure).

"Generating ALB functions" subsection: the lowest J_k eigenfunctions on Q_k are
restricted and truncated to the element E_k and orthonormalised there.  The
orthonormalisation is an SVD of the restricted block (all J_k columns kept):
Phi_E = X[E_k rows, :J] = U Sigma V^T, ALBs = U, singular values Sigma.
ALBs are defined by their span; signs and rotations inside the span are free.
"""
from __future__ import annotations

import numpy as np

__all__ = ["make_alb", "max_principal_angle", "restrict"]


def restrict(el, X: np.ndarray) -> np.ndarray:
    """Rows of X on E_k's grid points, in E_k's own x-fastest order."""
    return X[el.elem_indices(), :]


def make_alb(el, X: np.ndarray, n_want: int):
    """(U, sigma) for the first n_want columns of X restricted to E_k."""
    phi = restrict(el, X[:, :n_want])
    U, s, _ = np.linalg.svd(phi, full_matrices=False)
    return U, s


def max_principal_angle(A: np.ndarray, B: np.ndarray) -> float:
    """Largest principal angle between span(A) and span(B) (orthonormal columns).

    arcsin ||(I - A A^T) B||_2, accurate for small angles.
    """
    D = B - A @ (A.T @ B)
    s = np.linalg.norm(D, 2) if D.size else 0.0
    return float(np.arcsin(min(1.0, s)))
