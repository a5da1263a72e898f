"""DG Hamiltonian from adaptive local basis functions (oracle, FP64, test infrastructure).

Follows the DG discretisation of the global Kohn-Sham problem: the wavefunctions
are expanded in the ALBs of every element (Eq. (6), PsiALB) and the Hamiltonian
matrix is Eq. (7) (DGHamiltonian):

  H_{k'j'; kj} = ( 1/2 <grad phi_{k,j'}, grad phi_{k,j}>_T + <phi_{k,j'}, V phi_{k,j}>_T ) delta_{kk'}
               + sum_{I,l} gamma_{I,l} <phi_{k',j'}, b_{I,l}>_T <b_{I,l}, phi_{k,j}>_T
               - 1/2 <[[phi_{k',j'}]], {{grad phi_{k,j}}}>_S - 1/2 <{{grad phi_{k',j'}}}, [[phi_{k,j}]]>_S
               + alpha <[[phi_{k',j'}]], [[phi_{k,j}]]>_S

with <.,.>_T the sum of element integrals, <.,.>_S the sum of face integrals, and
[[.]], {{.}} the jump and average across a face.  Only blocks of an element with
itself and with the elements it shares a face or a projector with are nonzero.

Readings (where the paper leaves the discretisation open):
  D1  An ALB phi_{k,j} is the restriction to E_k of the trigonometric polynomial
      (X_k W_k)_j on the periodic box Q_k, where X_k are the element's eigenvectors
      and W_k = V S^{-1} from the SVD R_E X_k = U S V^T (so U = R_E X_k W_k are the
      ALB values).  Its gradient inside E_k, and its value and normal derivative on
      E_k's faces, are those of that polynomial (spectral derivative on Q_k; the
      Nyquist mode's odd derivative is zero).
  D2  Grid functions are Euclidean-normalised (sum phi^2 = 1 on E_k's points); the
      physical function is phi / sqrt(dV).  Element integrals are rectangle sums over
      E_k's grid points (the cell centres; dV cancels); faces lie half a grid step
      beyond E_k's outer points, and a face integral is the rectangle sum over the
      face's grid points times dA / dV = 1 / h_normal.
  D3  The mesh is 2D (elements are columns spanning the periodic z direction), so
      every element has four faces, x-, x+, y-, y+; [[u]] = u^- n^- + u^+ n^+ and
      {{v}} = (v^- + v^+) / 2 on each face.
  D4  alpha (the interior-penalty parameter) is an input; the tests use 40 Ha bohr.
  D5  The projectors in the nonlocal term are the global ones restricted to E_k
      (workloads.Mesh.elem_projectors), matched across elements by global id.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .planewave import n_workers

__all__ = ["alb_coefficients", "spectral_gradient", "face_traces", "dg_hamiltonian", "dense_from_blocks",
           "apply_blocks", "dg_chefsi"]


def alb_coefficients(el, X: np.ndarray, J: int):
    """(U, sigma, W): ALB values on E_k and the coefficients with U = R_E X[:, :J] W (D1)."""
    phi = X[el.elem_indices(), :J]
    U, s, Vt = np.linalg.svd(phi, full_matrices=False)
    return U, s, Vt.T / s[None, :]


def _wavenumbers(n: int, length: float) -> np.ndarray:
    """2 pi k / L with the Nyquist wavenumber set to zero (odd derivatives)."""
    k = np.fft.fftfreq(n) * n
    if n % 2 == 0:
        k[n // 2] = 0.0
    return 2.0 * np.pi * k / length


def spectral_gradient(el, F: np.ndarray) -> np.ndarray:
    """(3, N, m): d/dx, d/dy, d/dz of the columns of F (N x m) on Q_k's periodic grid."""
    nx, ny, nz = el.n
    m = F.shape[1]
    cube = np.ascontiguousarray(F.T).reshape(m, nz, ny, nx)
    out = np.empty((3, F.shape[0], m))
    for a, (axis, n, L) in enumerate(((3, nx, el.length[0]), (2, ny, el.length[1]), (1, nz, el.length[2]))):
        spec = scipy.fft.fft(cube, axis=axis, workers=n_workers())
        shape = [1, 1, 1, 1]
        shape[axis] = n
        spec *= 1j * _wavenumbers(n, L).reshape(shape)
        d = scipy.fft.ifft(spec, axis=axis, workers=n_workers()).real
        out[a] = d.reshape(m, -1).T
    return out


def _trig_eval_weights(n: int, length: float, x: float):
    """Weights w, w' with f(x) = sum_i w_i f(i h) and f'(x) = sum_i w'_i f(i h) for the
    real trigonometric interpolant of the n samples (Nyquist term as cos)."""
    k = np.fft.fftfreq(n) * n
    theta = 2.0 * np.pi * x / length
    # f(x) = (1/n) sum_k F_k exp(i k theta) with F = fft(f): w_i = (1/n) sum_k exp(i k (theta - 2 pi i / n))
    i = np.arange(n)
    phase = k[:, None] * (theta - 2.0 * np.pi * i[None, :] / n)
    c = np.cos(phase)
    s = np.sin(phase)
    kk = 2.0 * np.pi * k / length
    # the real parts of exp(i k (theta - 2 pi i / n)): with k = -n/2 the Nyquist term is
    # (-1)^i cos(n theta / 2), the cosine interpolant, and its derivative follows alike
    w = c.sum(axis=0) / n
    wd = (-kk[:, None] * s).sum(axis=0) / n
    return w, wd


def face_traces(el, F: np.ndarray):
    """Values and outward normal derivatives of the columns of F (trigonometric
    polynomials on Q_k) on E_k's four faces (D1, D2): a dict face -> (values,
    derivatives), each (n_face_points, m), face points in the face's own (tangential,
    z) order with the tangential index fastest."""
    nx, ny, nz = el.n
    m = F.shape[1]
    h = [el.length[a] / el.n[a] for a in range(3)]
    lo, en = el.elem_lo, el.elem_n
    cube = F.reshape(nz, ny, nx, m)
    out = {}
    for face, axis, sign in (("x-", 0, -1), ("x+", 0, 1), ("y-", 1, -1), ("y+", 1, 1)):
        n = el.n[axis]
        pos = (lo[axis] - 0.5) * h[axis] if sign < 0 else (lo[axis] + en[axis] - 0.5) * h[axis]
        w, wd = _trig_eval_weights(n, el.length[axis], pos)
        if axis == 0:
            sub = cube[:, lo[1]:lo[1] + en[1], :, :]           # (nz, ny_E, nx, m)
            val = np.einsum("zyxm,x->zym", sub, w)
            der = np.einsum("zyxm,x->zym", sub, wd)
        else:
            sub = cube[:, :, lo[0]:lo[0] + en[0], :]           # (nz, ny, nx_E, m)
            val = np.einsum("zyxm,y->zxm", sub, w)
            der = np.einsum("zyxm,y->zxm", sub, wd)
        out[face] = (val.reshape(-1, m), sign * der.reshape(-1, m))
    return out


def dg_hamiltonian(mesh, els, Xs, alpha: float):
    """Nonzero blocks {(k', k): J_k' x J_k} of Eq. (7) for the elements els (mesh
    layout), their eigenvectors Xs (N_k x >= J_k) and the penalty alpha."""
    M = mesh.n_elem
    assert len(els) == M
    h = [mesh.length[a] / mesh.global_n[a] for a in range(3)]
    data = []
    for k, el in enumerate(els):
        J = el.n_states
        U, s, W = alb_coefficients(el, Xs[k], J)
        F = Xs[k][:, :J] @ W                                   # ALBs extended to Q_k (D1)
        G = spectral_gradient(el, F)
        ei = el.elem_indices()
        data.append({"U": U, "grad": G[:, ei, :], "v": el.v_eff[ei], "traces": face_traces(el, F), "J": J})
    blocks = {}

    def add(kp, k, B):
        blocks[(kp, k)] = blocks.get((kp, k), 0.0) + B

    # element terms: kinetic + local potential (diagonal blocks)
    for k, d in enumerate(data):
        Gr = d["grad"]
        add(k, k, 0.5 * sum(Gr[a].T @ Gr[a] for a in range(3)) + d["U"].T @ (d["v"][:, None] * d["U"]))
    # nonlocal: O_k[p, j] = <b_p, phi_{k,j}> over E_k for every projector touching E_k
    ovl = []
    for k, d in enumerate(data):
        gid, ptr, idx, val, gam = mesh.elem_projectors(k)
        O = np.zeros((len(gid), d["J"]))
        for p in range(len(gid)):
            O[p] = val[ptr[p]:ptr[p + 1]] @ d["U"][idx[ptr[p]:ptr[p + 1]], :]
        ovl.append({int(g): (O[p], gam[p]) for p, g in enumerate(gid)})
    for kp in range(M):
        for k in range(M):
            common = sorted(set(ovl[kp]) & set(ovl[k]))
            if not common:
                continue
            A = np.array([ovl[kp][g][0] for g in common])      # n_c x J_k'
            B = np.array([ovl[k][g][0] for g in common])       # n_c x J_k
            gm = np.array([ovl[k][g][1] for g in common])
            add(kp, k, A.T @ (gm[:, None] * B))
    # faces: each x+ face of k is the x- face of its x+ neighbour (same for y)
    for k in range(M):
        nb = mesh.neighbours(k)
        for face, other, oface, axis in (("x+", nb[1], "x-", 0), ("y+", nb[3], "y-", 1)):
            # minus side: element k (outward normal +e_axis); plus side: the neighbour
            vm, dm = data[k]["traces"][face]                  # outward derivative on k: +d/d axis
            vp, dp = data[other]["traces"][oface]             # outward derivative on other: -d/d axis
            dmn, dpn = dm, -dp                                 # derivatives along +e_axis
            inv_h = 1.0 / h[axis]
            sides = ((k, vm, dmn, 1.0), (other, vp, dpn, -1.0))
            for (a, va, da, sa) in sides:
                for (b, vb, db, sb) in sides:
                    # H_ab += int [ -1/4 s_a v_a db - 1/4 s_b da vb + alpha s_a s_b v_a vb ] dA
                    B = (-0.25 * sa * (va.T @ db) - 0.25 * sb * (da.T @ vb) + alpha * sa * sb * (va.T @ vb)) * inv_h
                    add(a, b, B)
    return blocks


def dense_from_blocks(blocks, Js):
    """The dense (sum J) x (sum J) matrix of a block dict."""
    off = np.concatenate([[0], np.cumsum(Js)])
    H = np.zeros((off[-1], off[-1]))
    for (kp, k), B in blocks.items():
        H[off[kp]:off[kp + 1], off[k]:off[k + 1]] += B
    return H


def apply_blocks(blocks, Js, X: np.ndarray) -> np.ndarray:
    """H^DG X one element row at a time (Eq. (8)): the rows of element k are
    sum over the nonzero blocks (k, k') of H_{k,k'} X_{k'}, X_{k'} the rows of element
    k' (element-major rows, J_k per element)."""
    off = np.concatenate([[0], np.cumsum(Js)]).astype(np.int64)
    Y = np.zeros((off[-1], X.shape[1]))
    for (k, kp), B in blocks.items():
        Y[off[k]:off[k + 1], :] += B @ X[off[kp]:off[kp + 1], :]
    return Y


def dg_chefsi(blocks, Js, x0: np.ndarray, n_want: int, degree: int = 16, tol: float = 1e-10,
              max_iter: int = 200):
    """Lowest eigenpairs of H^DG by Algorithm 2 (CheFSI) with the block-sparse product
    of Eq. (8): the Chebyshev-filtered subspace iteration of ``oracle.chebyshev.chfsi``
    (Lanczos upper bound, lower bound from the previous Ritz values, Cholesky
    orthonormalisation, projected eigenproblem, rotation) applied to H^DG."""
    from .chebyshev import chfsi
    return chfsi(None, x0, n_want, degree=degree, tol=tol, max_iter=max_iter,
                 apply_h=lambda V: apply_blocks(blocks, Js, V))
