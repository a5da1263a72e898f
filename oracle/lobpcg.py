"""LOBPCG eigensolver for H^{Q_k} (oracle, FP64, test infrastructure).

Follows Algorithm 1 (LOBPCG) and Eqs. (2)-(4):
  * X is orthonormalised at the start (step 1);
  * W = T(HX - X(X^T H X)), T the Teter preconditioner (Eq. (3), step 3);
  * S = [X, W, P] (step 4); the projected problem S^T H S C = S^T S C Lambda
    (Eq. (4), step 5) is solved for its lowest eigenpairs;
  * P <- W C_W + P C_P (step 6); X <- X C_X + P (step 7, Eq. (2)).

Readings where the paper is silent (all affect convergence only, not the
fixed point): seeded Gaussian start; W and P are orthonormalised (SVD, with
directions below 1e-10 relative dropped) before the projected problem, so
S^T S = I and step 5 becomes a standard symmetric eigenproblem; guard states
are carried above the J wanted ones; convergence is max_i ||r_i||_2 over the
wanted states, in Ha, with ||x_i|| = 1.

Teter preconditioner (Teter, Payne & Allan 1989): per state i,
  K(t) = (27 + 18 t + 12 t^2 + 8 t^3) / (27 + 18 t + 12 t^2 + 8 t^3 + 16 t^4),
  t = (|G|^2/2) / E_i, applied in G-space to r_i; E_i = <x_i|T|x_i> (kinetic
  energy of the state).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

from .planewave import apply_kinetic, hpsi, kinetic_symbol

__all__ = ["teter_factor", "teter_apply", "lobpcg", "LobpcgResult", "orth_svd", "rayleigh_ritz"]


def teter_factor(t: np.ndarray) -> np.ndarray:
    num = 27.0 + t * (18.0 + t * (12.0 + 8.0 * t))
    return num / (num + 16.0 * t ** 4)


def teter_apply(el, R: np.ndarray, ekin: np.ndarray) -> np.ndarray:
    """Columns r_i -> F^{-1} K(g / E_i) F r_i."""
    g = kinetic_symbol(el.n, el.length)
    out = np.empty_like(R)
    for i in range(R.shape[1]):
        out[:, i] = apply_kinetic(el.n, el.length, R[:, i], symbol=teter_factor(g / ekin[i]))
    return out


def orth_svd(A: np.ndarray, scale: float, rel_drop: float = 1e-10) -> np.ndarray:
    """Orthonormal basis of range(A) by SVD, dropping sigma < rel_drop * scale.

    ``scale`` is the norm of the block before it was projected against the rest
    of the subspace, so a block that projection has reduced to rounding noise
    is dropped entirely.
    """
    if A.shape[1] == 0 or scale == 0.0:
        return A[:, :0]
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    return U[:, s > rel_drop * scale]


def rayleigh_ritz(el, X0: np.ndarray):
    """Ritz pairs of H^{Q_k} on span(X0) (the start of Algorithm 1, step 1): an
    orthonormal basis Q of span(X0) (Householder QR), the projected matrix Q^T H Q and
    its eigendecomposition; returns (Ritz values ascending, Ritz vectors Q V)."""
    Q, _ = np.linalg.qr(X0)
    A = Q.T @ hpsi(el, Q)
    theta, V = np.linalg.eigh(0.5 * (A + A.T))
    return theta, Q @ V


@dataclasses.dataclass
class LobpcgResult:
    eigvals: np.ndarray      # wanted + guard Ritz values, ascending
    X: np.ndarray            # N x (J+g) Ritz vectors, orthonormal
    resid: np.ndarray        # ||H x_i - theta_i x_i|| for all columns
    iters: int
    converged: bool
    history: list


def lobpcg(el, x0: np.ndarray, n_want: int, tol: float = 1e-10, max_iter: int = 400,
           apply_h=None, precondition: bool = True) -> LobpcgResult:
    """Lowest eigenpairs of H^{Q_k}; x0 is N x (J+g), n_want = J."""
    H = (lambda V: hpsi(el, V)) if apply_h is None else apply_h
    # step 1: orthonormalise X, and Rayleigh-Ritz on span(X)
    X, _ = np.linalg.qr(x0)
    HX = H(X)
    theta, V = np.linalg.eigh(0.5 * (X.T @ HX + HX.T @ X))
    X, HX = X @ V, HX @ V
    P = None
    k = X.shape[1]
    history = []
    it = 0
    for it in range(1, max_iter + 1):
        # step 3: residual and preconditioned residual
        lam = 0.5 * (X.T @ HX + HX.T @ X)
        R = HX - X @ lam
        res = np.linalg.norm(R, axis=0)
        history.append(float(res[:n_want].max()))
        if res[:n_want].max() <= tol:
            # H X has been carried by rotations; confirm with a fresh application
            X, _ = np.linalg.qr(X)
            HX = H(X)
            theta, V = np.linalg.eigh(0.5 * (X.T @ HX + HX.T @ X))
            X, HX = X @ V, HX @ V
            res = np.linalg.norm(HX - X * theta[None, :], axis=0)
            if res[:n_want].max() <= tol:
                break
            P = None
            continue
        if precondition:
            ekin = np.einsum("ij,ij->j", X, apply_kinetic(el.n, el.length, X))
            W = teter_apply(el, R, np.maximum(ekin, 1e-3))
        else:
            W = R.copy()
        # step 4: S = [X, W, P], with W and P orthonormalised against X and each other
        wscale = np.linalg.norm(W)
        W = W - X @ (X.T @ W)
        W = W - X @ (X.T @ W)
        W = orth_svd(W, wscale)
        blocks = [X, W]
        hblocks = [HX, H(W)]
        if P is not None:
            # P made orthogonal to X and W (twice, for numerical orthogonality)
            pscale = np.linalg.norm(P)
            for _ in range(2):
                P = P - X @ (X.T @ P) - W @ (W.T @ P)
            Po = orth_svd(P, pscale)
            if Po.shape[1]:
                blocks.append(Po)
                hblocks.append(H(Po))
        S = np.hstack(blocks)
        HS = np.hstack(hblocks)
        # step 5: projected eigenproblem (S^T S = I here)
        A = 0.5 * (S.T @ HS + HS.T @ S)
        w, C = scipy.linalg.eigh(A)
        C = C[:, :k]
        theta = w[:k]
        # steps 6-7
        P = S[:, k:] @ C[k:, :]
        X = X @ C[:k, :] + P
        HX = HX @ C[:k, :] + HS[:, k:] @ C[k:, :]
    lam = 0.5 * (X.T @ HX + HX.T @ X)
    theta, V = np.linalg.eigh(lam)
    X, HX = X @ V, HX @ V
    res = np.linalg.norm(HX - X * theta[None, :], axis=0)
    return LobpcgResult(theta, X, res, it, bool(res[:n_want].max() <= tol), history)
