"""Chebyshev-filtered subspace iteration on H^{Q_k} (oracle, FP64, test infrastructure).

Algorithm 2 (CheFSI) is stated for H^DG; the same steps are applied here to the
local Hamiltonian H^{Q_k}:
  1. lower bound b_low from the previous Ritz values, upper bound b_up by Lanczos;
  2. filter Y~ = p_m(H) X with [b_low, b_up] mapped to [-1, 1] (Eq. (8)'s
     three-term recurrence);
  3. S = Y~^T Y~ = U^T U (Cholesky), Y^ = Y~ U^{-1} (reading of the garbled
     "Y^ U = Y~");
  4. H^ = Y^^T H Y^ (Eq. (9)), H^ V = V D;
  5. X <- Y^ V.

Filter (Zhou & Saad 2007, scaled recurrence), with e = (b-a)/2, c = (b+a)/2 and
sigma_1 = e / (a0 - c), a0 an estimate of the lowest eigenvalue:
  Y_1 = (sigma_1 / e)(H - c) Y_0,
  sigma_{k+1} = 1 / (2/sigma_1 - sigma_k),
  Y_{k+1} = (2 sigma_{k+1} / e)(H - c) Y_k - sigma_k sigma_{k+1} Y_{k-1}.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

from .planewave import hpsi

__all__ = ["filter_coefficients", "cheb_filter", "lanczos_upper_bound", "chfsi", "ChfsiResult"]


def filter_coefficients(degree: int, a: float, b: float, a0: float):
    """Per-step (alpha_k, beta_k) with Y_{k+1} = alpha_k (H - c) Y_k - beta_k Y_{k-1}.

    Step 0 has beta_0 = 0 (no Y_{-1}).  Returns (c, alphas, betas).
    """
    e = 0.5 * (b - a)
    c = 0.5 * (b + a)
    s1 = e / (a0 - c)
    alphas = [s1 / e]
    betas = [0.0]
    s = s1
    for _ in range(1, degree):
        s_new = 1.0 / (2.0 / s1 - s)
        alphas.append(2.0 * s_new / e)
        betas.append(s * s_new)
        s = s_new
    return c, np.array(alphas), np.array(betas)


def cheb_filter(apply_h, Y0: np.ndarray, degree: int, a: float, b: float, a0: float,
                keep_all: bool = False):
    """p_m(H) Y0 by the scaled three-term recurrence; optionally returns all Y_k."""
    c, al, be = filter_coefficients(degree, a, b, a0)
    Yprev = None
    Y = Y0
    hist = [Y0]
    for k in range(degree):
        Z = al[k] * (apply_h(Y) - c * Y)
        if k > 0:
            Z -= be[k] * Yprev
        Yprev, Y = Y, Z
        if keep_all:
            hist.append(Y)
    return (Y, hist) if keep_all else Y


def lanczos_upper_bound(apply_h, n: int, steps: int = 10, seed: int = 7) -> float:
    """Upper bound on the spectrum: largest Ritz value of a k-step Lanczos plus ||f||."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    alphas, betas = [], []
    v_prev = np.zeros(n)
    beta = 0.0
    f = None
    for _ in range(steps):
        w = apply_h(v.reshape(-1, 1))[:, 0]
        alpha = float(v @ w)
        f = w - alpha * v - beta * v_prev
        alphas.append(alpha)
        beta = float(np.linalg.norm(f))
        betas.append(beta)
        if beta == 0.0:
            break
        v_prev, v = v, f / beta
    T = np.diag(alphas) + np.diag(betas[:-1], 1) + np.diag(betas[:-1], -1)
    return float(np.linalg.eigvalsh(T).max() + np.linalg.norm(f))


@dataclasses.dataclass
class ChfsiResult:
    eigvals: np.ndarray
    X: np.ndarray
    resid: np.ndarray
    iters: int
    converged: bool
    history: list


def chfsi(el, x0: np.ndarray, n_want: int, degree: int = 16, tol: float = 1e-10,
          max_iter: int = 200, apply_h=None) -> ChfsiResult:
    """Lowest eigenpairs of H^{Q_k} by Chebyshev-filtered subspace iteration."""
    H = (lambda V: hpsi(el, V)) if apply_h is None else apply_h
    N = x0.shape[0]
    b = lanczos_upper_bound(H, N)
    # initial Rayleigh-Ritz gives the first Ritz values for the lower bound
    X, _ = np.linalg.qr(x0)
    HX = H(X)
    d, V = np.linalg.eigh(0.5 * (X.T @ HX + HX.T @ X))
    X, HX = X @ V, HX @ V
    history = []
    it = 0
    res = np.linalg.norm(HX - X * d[None, :], axis=0)
    for it in range(1, max_iter + 1):
        a, a0 = float(d[-1]), float(d[0])
        Y = cheb_filter(H, X, degree, a, b, a0)
        S = Y.T @ Y
        U = scipy.linalg.cholesky(0.5 * (S + S.T), lower=False)
        Yh = scipy.linalg.solve_triangular(U, Y.T, trans="T", lower=False).T
        HY = H(Yh)
        d, V = np.linalg.eigh(0.5 * (Yh.T @ HY + HY.T @ Yh))
        X, HX = Yh @ V, HY @ V
        res = np.linalg.norm(HX - X * d[None, :], axis=0)
        history.append(float(res[:n_want].max()))
        if res[:n_want].max() <= tol:
            break
    return ChfsiResult(d, X, res, it, bool(res[:n_want].max() <= tol), history)
