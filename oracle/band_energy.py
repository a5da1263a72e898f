"""Band energy through the Chebyshev filter and its gradient (oracle, FP64, test infrastructure).

E(V, Psi_0) = sum_i f_i psi_i^T H[V] psi_i,   Psi = p_m(H[V]) Psi_0,

with p_m the scaled Chebyshev filter of Algorithm 2 / Eq. (8) (coefficients
held fixed, not differentiated).  H[V] = T + diag(V) + V_nl (Eq. (1)) depends
on the local potential V only through its diagonal.  The gradient is the
adjoint of the three-term recurrence, with every intermediate Y_k stored:

  Ybar_m = 2 H Y_m F,   Vbar += sum_i f_i y_{m,i}^2,
  for k = m-1 .. 0 (Y_{k+1} = alpha_k (H - c) Y_k - beta_k Y_{k-1}):
      Ybar_k     += alpha_k (H - c) Ybar_{k+1}
      Vbar       += alpha_k sum_i ybar_{k+1,i} * y_{k,i}
      Ybar_{k-1} -= beta_k Ybar_{k+1}        (k >= 1)

The Euclidean gradient dE/dPsi_0 = Ybar_0 and dE/dV = Vbar are returned.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .chebyshev import filter_coefficients
from .planewave import hpsi

__all__ = ["band_energy", "band_energy_grad"]


def _with_v(el, v):
    return dataclasses.replace(el, v_eff=np.asarray(v, dtype=np.float64))


def band_energy(el, v, psi0, f, degree, a, b, a0):
    """E(V, Psi_0) (scalar)."""
    e2 = _with_v(el, v)
    H = lambda Y: hpsi(e2, Y)
    c, al, be = filter_coefficients(degree, a, b, a0)
    Yp, Y = None, psi0
    for k in range(degree):
        Z = al[k] * (H(Y) - c * Y)
        if k > 0:
            Z -= be[k] * Yp
        Yp, Y = Y, Z
    return float(np.sum(f * np.einsum("ij,ij->j", Y, H(Y))))


def band_energy_grad(el, v, psi0, f, degree, a, b, a0):
    """(E, dE/dPsi_0, dE/dV) by the stored-intermediate adjoint recurrence."""
    e2 = _with_v(el, v)
    H = lambda Y: hpsi(e2, Y)
    c, al, be = filter_coefficients(degree, a, b, a0)
    Ys = [psi0]
    for k in range(degree):
        Z = al[k] * (H(Ys[k]) - c * Ys[k])
        if k > 0:
            Z -= be[k] * Ys[k - 1]
        Ys.append(Z)
    Ym = Ys[-1]
    HYm = H(Ym)
    E = float(np.sum(f * np.einsum("ij,ij->j", Ym, HYm)))
    Ybar = [np.zeros_like(psi0) for _ in range(degree + 1)]
    Ybar[degree] = 2.0 * HYm * f[None, :]
    vbar = (Ym * Ym) @ f
    for k in range(degree - 1, -1, -1):
        Ybar[k] += al[k] * (H(Ybar[k + 1]) - c * Ybar[k + 1])
        vbar += al[k] * np.sum(Ybar[k + 1] * Ys[k], axis=1)
        if k >= 1:
            Ybar[k - 1] -= be[k] * Ybar[k + 1]
    return E, Ybar[0], vbar
