"""Local Kohn-Sham Hamiltonian on an extended element (oracle, FP64, test infrastructure).

Eq. (1) (LocalKS): H^{Q_k} = -1/2 Laplacian + V_eff + V_nl, with
V_nl = sum_{I,l} gamma_{I,l} |b_{I,l}><b_{I,l}|, discretised in the plane-wave
basis of the periodic box Q_k (the PWDFT discretisation described right after
Eq. (1)).  With all N grid plane waves kept (reading: full FFT box, Nyquist
mode included) the kinetic operator on real grid vectors is

    T = F^{-1} diag(|G|^2 / 2) F,

F the N-point 3D DFT, and the full operator is H = T + diag(v) + B diag(gamma) B^T.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft
import scipy.sparse

__all__ = ["kinetic_symbol", "apply_kinetic", "hpsi", "dense_kinetic", "dense_H",
           "n_workers"]


def n_workers() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _freq(n: int, length: float) -> np.ndarray:
    """Reciprocal vectors G = 2 pi k / L, k = 0..n/2-1, -n/2..-1 (Nyquist as -n/2)."""
    k = np.fft.fftfreq(n) * n
    return 2.0 * np.pi * k / length


def kinetic_symbol(n, length) -> np.ndarray:
    """|G|^2 / 2 on the full FFT grid, shape (nz, ny, nx)."""
    gx, gy, gz = (_freq(n[a], length[a]) for a in range(3))
    return 0.5 * (gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2)


def _half(g: np.ndarray) -> np.ndarray:
    return g[:, :, : g.shape[2] // 2 + 1]


def apply_kinetic(n, length, x: np.ndarray, symbol: np.ndarray | None = None) -> np.ndarray:
    """T x for real x of shape (N,) or (N, m): irfftn(symbol * rfftn(x)).

    ``symbol`` (default |G|^2/2) is any real multiplier with symbol(G) = symbol(-G).
    """
    nx, ny, nz = n
    g = kinetic_symbol(n, length) if symbol is None else symbol
    vec = x.ndim == 1
    xs = x.reshape(-1, 1) if vec else x
    m = xs.shape[1]
    cube = np.ascontiguousarray(xs.T).reshape(m, nz, ny, nx)
    spec = scipy.fft.rfftn(cube, axes=(1, 2, 3), workers=n_workers())
    spec *= _half(g)[None]
    out = scipy.fft.irfftn(spec, s=(nz, ny, nx), axes=(1, 2, 3), workers=n_workers())
    out = out.reshape(m, nz * ny * nx).T
    return out[:, 0] if vec else out


def hpsi(el, x: np.ndarray) -> np.ndarray:
    """y = H^{Q_k} x (Eq. (1)); x is (N,) or (N, m), FP64."""
    xs = x.reshape(-1, 1) if x.ndim == 1 else x
    y = apply_kinetic(el.n, el.length, xs)
    y += el.v_eff[:, None] * xs
    if el.n_proj:
        B = el.projector_matrix()
        y += B @ (el.gamma[:, None] * (B.T @ xs))
    return y[:, 0] if x.ndim == 1 else y


def _dft_matrix(n: int) -> np.ndarray:
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def dense_kinetic(n, length) -> np.ndarray:
    """Dense T = Re(F^H diag(g) F) / N with F the explicit Kronecker DFT matrix.

    Brute force for tiny grids (N <= ~2000): the definition written out with
    no FFT, F = F_z (x) F_y (x) F_x for x-fastest flattening.
    """
    nx, ny, nz = n
    F = np.kron(_dft_matrix(nz), np.kron(_dft_matrix(ny), _dft_matrix(nx)))
    g = kinetic_symbol(n, length).ravel()
    T = (F.conj().T * g[None, :]) @ F / F.shape[0]
    return np.ascontiguousarray(T.real)


def dense_H(el, kinetic: np.ndarray | None = None) -> np.ndarray:
    """Explicit N x N matrix of H^{Q_k} (tiny grids only)."""
    T = dense_kinetic(el.n, el.length) if kinetic is None else kinetic
    H = T + np.diag(el.v_eff)
    if el.n_proj:
        B = el.projector_matrix().toarray()
        H = H + (B * el.gamma[None, :]) @ B.T
    return 0.5 * (H + H.T)
