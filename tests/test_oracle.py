"""Pins of the CPU oracle against closed forms, brute force, invariants and library routines.

Every oracle function is checked here by something other than itself, so that a
dropped term, a wrong sign or index, or a transposed operand fails a test.
"""
import dataclasses
import itertools
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg

import workloads as W
from oracle import alb, band_energy, chebyshev, lobpcg, planewave

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_element(n=(8, 8, 8), length=(6.0, 6.4, 7.2), n_sites=2, n_proj=3, seed=1,
                 n_states=6, supp=40):
    """Small element with wells and random sparse projectors (generic B, gamma)."""
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0, 1, size=(n_sites, 3)) * np.array(length)
    el = W._box_element(n, length, sites, n_states)
    N = el.npts
    ptr, idx, val = [0], [], []
    for _ in range(n_proj):
        s = np.sort(rng.choice(N, size=supp, replace=False))
        b = rng.standard_normal(supp)
        b /= np.linalg.norm(b)
        idx.append(s.astype(np.int32))
        val.append(b)
        ptr.append(ptr[-1] + supp)
    gam = rng.uniform(0.2, 1.0, size=n_proj)
    return dataclasses.replace(el, proj_ptr=np.array(ptr, np.int64),
                               proj_idx=np.concatenate(idx), proj_val=np.concatenate(val),
                               gamma=gam)


def load_shells():
    rows = np.loadtxt(os.path.join(GOLDEN, "free_electron_10bohr_16cubed.txt"))
    return rows


# ---------------------------------------------------------------- kinetic / FFT

def test_golden_shells_are_the_integer_lattice():
    """The golden fixture itself: count integer vectors by brute force."""
    rows = load_shells()
    rng = range(-8, 8)
    counts = {}
    for k in itertools.product(rng, rng, rng):
        n2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
        counts[n2] = counts.get(n2, 0) + 1
    for n2, val, mult, cum in rows:
        assert counts[int(n2)] == int(mult)
        assert abs(val - 0.5 * (2 * np.pi / 10.0) ** 2 * n2) < 1e-9


def test_free_electron_symbol_matches_closed_form():
    g = np.sort(planewave.kinetic_symbol((16, 16, 16), (10.0, 10.0, 10.0)).ravel())
    rows = load_shells()
    pos = 0
    for n2, val, mult, cum in rows:
        seg = g[pos:pos + int(mult)]
        assert np.allclose(seg, val, atol=1e-9)
        pos += int(mult)
        assert pos == int(cum)


def test_kinetic_fft_equals_dense_definition():
    """FFT-based T x equals the explicit Kronecker-DFT definition (no FFT)."""
    for n, L in [((8, 8, 8), (6.0, 6.4, 7.2)), ((6, 8, 4), (5.0, 7.0, 3.0)), ((9, 6, 4), (5.0, 4.0, 3.0))]:
        T = planewave.dense_kinetic(n, L)
        x = np.random.default_rng(3).standard_normal((T.shape[0], 3))
        assert np.allclose(planewave.apply_kinetic(n, L, x), T @ x, rtol=0, atol=1e-12 * np.abs(T).max() * 10)
        assert np.allclose(T, T.T, atol=1e-12)


def test_kinetic_parseval_and_roundtrip():
    n, L = (12, 10, 8), (7.0, 6.0, 5.0)
    x = np.random.default_rng(4).standard_normal(np.prod(n))
    g = planewave.kinetic_symbol(n, L)
    xh = np.fft.fftn(x.reshape(n[2], n[1], n[0]))
    # <x, T x> = (1/N) sum_G g |x^(G)|^2 over the full grid
    assert np.isclose(x @ planewave.apply_kinetic(n, L, x), np.sum(g * np.abs(xh) ** 2) / x.size, rtol=1e-13)
    # Parseval itself and the identity multiplier round trip
    assert np.isclose(x @ x, np.sum(np.abs(xh) ** 2) / x.size, rtol=1e-13)
    y = planewave.apply_kinetic(n, L, x, symbol=np.ones_like(g))
    assert np.max(np.abs(y - x)) < 1e-14


def test_free_electron_eigenvalues_lobpcg():
    el = W.free_electron_element(n_states=19)
    rows = load_shells()
    expect = np.concatenate([np.full(int(m), v) for _, v, m, _ in rows])
    for J in (7, 19):
        x0 = W.initial_block(el.npts, J + 4, seed=100 + J).T
        r = lobpcg.lobpcg(el, x0, J, tol=1e-9, max_iter=300)
        assert r.converged
        assert np.max(np.abs(r.eigvals[:J] - expect[:J])) < 1e-9


# ---------------------------------------------------------------- full H

def test_hpsi_equals_dense_H_matvec():
    el = tiny_element()
    H = planewave.dense_H(el)
    x = np.random.default_rng(5).standard_normal((el.npts, 4))
    assert np.max(np.abs(planewave.hpsi(el, x) - H @ x)) < 1e-11


def test_hpsi_terms_separately():
    """Potential and projector terms against their definitions, elementwise."""
    el = tiny_element()
    x = np.random.default_rng(6).standard_normal(el.npts)
    T = planewave.dense_kinetic(el.n, el.length)
    B = np.zeros((el.npts, el.n_proj))
    for p in range(el.n_proj):
        for t in range(el.proj_ptr[p], el.proj_ptr[p + 1]):
            B[el.proj_idx[t], p] = el.proj_val[t]
    manual = T @ x + el.v_eff * x + sum(el.gamma[p] * B[:, p] * (B[:, p] @ x) for p in range(el.n_proj))
    assert np.max(np.abs(planewave.hpsi(el, x) - manual)) < 1e-11


def test_hermiticity():
    el = W.small_slab()[1]
    rng = np.random.default_rng(7)
    x, y = rng.standard_normal(el.npts), rng.standard_normal(el.npts)
    a = y @ planewave.hpsi(el, x)
    b = planewave.hpsi(el, y) @ x
    assert abs(a - b) <= 1e-13 * max(abs(a), 1.0) * 10


@pytest.mark.parametrize("n", [(8, 8, 8), (12, 12, 12)])
def test_lobpcg_matches_dense_brute_force(n):
    el = tiny_element(n=n, length=(6.0, 6.4, 7.2), n_states=6)
    ev = scipy.linalg.eigh(planewave.dense_H(el), eigvals_only=True)
    J = 6
    x0 = W.initial_block(el.npts, J + 4, seed=11).T
    r = lobpcg.lobpcg(el, x0, J, tol=1e-10)
    assert r.converged
    assert np.max(np.abs(r.eigvals[:J] - ev[:J])) < 1e-10
    # orthonormality of the returned block
    assert np.max(np.abs(r.X.T @ r.X - np.eye(r.X.shape[1]))) < 1e-12


def test_c1_lobpcg_dense_16cubed():
    """C1 itself (4 wells, 16^3): dense H from separable 1D circulants equals the 3D definition."""
    el = W.make_config("c1").elements[0]
    # separable dense T (sum of 1D spectral operators) -- checked against the
    # Kronecker definition on a smaller grid in test_separable_equals_kron
    T = _separable_dense_T(el.n, el.length)
    H = T + np.diag(el.v_eff)
    ev = scipy.linalg.eigh(H, eigvals_only=True, subset_by_index=[0, 11])
    J = 8
    x0 = W.initial_block(el.npts, J + 4, seed=100).T
    r = lobpcg.lobpcg(el, x0, J, tol=1e-10)
    assert r.converged
    assert np.max(np.abs(r.eigvals[:J] - ev[:J])) < 1e-10


def _separable_dense_T(n, L):
    mats = []
    for a in range(3):
        k = np.fft.fftfreq(n[a]) * n[a]
        g = 0.5 * (2 * np.pi * k / L[a]) ** 2
        F = np.exp(-2j * np.pi * np.outer(np.arange(n[a]), np.arange(n[a])) / n[a])
        mats.append(((F.conj().T * g) @ F / n[a]).real)
    Ix, Iy, Iz = (np.eye(n[a]) for a in range(3))
    return (np.kron(Iz, np.kron(Iy, mats[0])) + np.kron(Iz, np.kron(mats[1], Ix))
            + np.kron(mats[2], np.kron(Iy, Ix)))


def test_separable_equals_kron():
    n, L = (6, 8, 4), (5.0, 7.0, 3.0)
    assert np.max(np.abs(_separable_dense_T(n, L) - planewave.dense_kinetic(n, L))) < 1e-12


def test_constant_shift():
    el = tiny_element()
    ev0 = scipy.linalg.eigh(planewave.dense_H(el), eigvals_only=True)[:6]
    el2 = dataclasses.replace(el, v_eff=el.v_eff + 0.37)
    x0 = W.initial_block(el.npts, 10, seed=12).T
    r = lobpcg.lobpcg(el2, x0, 6, tol=1e-10)
    assert np.max(np.abs(r.eigvals[:6] - (ev0 + 0.37))) < 1e-10


def test_translation_invariance():
    el = tiny_element()
    nx, ny, nz = el.n
    shift = (3, 5, 2)
    v3 = el.v_eff.reshape(nz, ny, nx)
    v_s = np.roll(v3, shift=(shift[2], shift[1], shift[0]), axis=(0, 1, 2)).ravel()
    ix = el.proj_idx % nx
    iy = (el.proj_idx // nx) % ny
    iz = el.proj_idx // (nx * ny)
    new = ((ix + shift[0]) % nx) + nx * (((iy + shift[1]) % ny) + ny * ((iz + shift[2]) % nz))
    ptr, idx, val = [0], [], []
    for p in range(el.n_proj):
        a, b = el.proj_ptr[p], el.proj_ptr[p + 1]
        o = np.argsort(new[a:b])
        idx.append(new[a:b][o].astype(np.int32))
        val.append(el.proj_val[a:b][o])
        ptr.append(b)
    el2 = dataclasses.replace(el, v_eff=v_s, proj_idx=np.concatenate(idx), proj_val=np.concatenate(val))
    x0 = W.initial_block(el.npts, 10, seed=13).T
    r1 = lobpcg.lobpcg(el, x0, 6, tol=1e-10)
    r2 = lobpcg.lobpcg(el2, x0, 6, tol=1e-10)
    assert np.max(np.abs(r1.eigvals[:6] - r2.eigvals[:6])) < 1e-10


def test_rank_one_projector_closed_form():
    """v = 0, b = unit cos(G0 . r) mode: eigenvalue |G0|^2/2 + gamma appears, rest unchanged."""
    n, L = (8, 8, 8), (6.0, 6.0, 6.0)
    el = W._box_element(n, L, [], 8)
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    k0 = (1, 0, 0)
    b = np.cos(2 * np.pi * (k0[0] * x / nx + k0[1] * y / ny + k0[2] * z / nz)).ravel()
    b /= np.linalg.norm(b)
    gam = 0.9
    el = dataclasses.replace(el, proj_ptr=np.array([0, el.npts], np.int64),
                             proj_idx=np.arange(el.npts, dtype=np.int32), proj_val=b,
                             gamma=np.array([gam]))
    g = np.sort(planewave.kinetic_symbol(n, L).ravel())
    g0 = 0.5 * (2 * np.pi / 6.0) ** 2
    expect = g.copy()
    expect[np.argmin(np.abs(expect - g0))] = g0 + gam
    expect = np.sort(expect)
    ev = scipy.linalg.eigh(planewave.dense_H(el), eigvals_only=True)
    assert np.max(np.abs(ev - expect)) < 1e-10
    x0 = W.initial_block(el.npts, 12, seed=14).T
    r = lobpcg.lobpcg(el, x0, 8, tol=1e-10)
    assert np.max(np.abs(r.eigvals[:8] - expect[:8])) < 1e-9


def test_weyl_interlacing_rank_one():
    el = tiny_element(n_proj=1)
    el0 = dataclasses.replace(el, proj_ptr=np.zeros(1, np.int64), proj_idx=np.zeros(0, np.int32),
                              proj_val=np.zeros(0), gamma=np.zeros(0))
    e0 = scipy.linalg.eigh(planewave.dense_H(el0), eigvals_only=True)
    e1 = scipy.linalg.eigh(planewave.dense_H(el), eigvals_only=True)
    assert np.all(e1 >= e0 - 1e-12)
    assert np.all(e1[:-1] <= e0[1:] + 1e-12)


def test_lobpcg_vs_arpack_slab():
    """Two independent iterations (LOBPCG, ARPACK Lanczos) on a small slab element."""
    el = W.small_slab(n_states=8)[0]
    J = 8
    x0 = W.initial_block(el.npts, J + 4, seed=15).T
    r = lobpcg.lobpcg(el, x0, J, tol=1e-10)
    op = scipy.sparse.linalg.LinearOperator((el.npts, el.npts), matvec=lambda v: planewave.hpsi(el, v),
                                            dtype=np.float64)
    ev = np.sort(scipy.sparse.linalg.eigsh(op, k=J + 4, which="SA", tol=1e-13,
                                           v0=np.ones(el.npts), return_eigenvectors=False))
    assert r.converged
    assert np.max(np.abs(r.eigvals[:J] - ev[:J])) < 1e-10


# ---------------------------------------------------------------- Chebyshev

def test_chebyshev_filter_is_scaled_chebyshev_polynomial():
    el = tiny_element()
    H = planewave.dense_H(el)
    lam, V = np.linalg.eigh(H)
    a, b, a0, m = lam[8], lam[-1] + 0.1, lam[0], 9
    Y0 = np.random.default_rng(16).standard_normal((el.npts, 3))
    Y = chebyshev.cheb_filter(lambda X: H @ X, Y0, m, a, b, a0)
    e, c = (b - a) / 2, (b + a) / 2
    coef = np.zeros(m + 1)
    coef[m] = 1.0
    p = np.polynomial.chebyshev.chebval((lam - c) / e, coef) / np.polynomial.chebyshev.chebval((a0 - c) / e, coef)
    ref = V @ (p[:, None] * (V.T @ Y0))
    assert np.max(np.abs(Y - ref)) < 1e-10 * np.max(np.abs(ref))


def test_lanczos_upper_bound_is_an_upper_bound():
    el = tiny_element()
    H = planewave.dense_H(el)
    ub = chebyshev.lanczos_upper_bound(lambda X: H @ X, el.npts)
    lmax = np.linalg.eigvalsh(H)[-1]
    assert ub >= lmax
    assert ub <= lmax * 1.5 + 1.0


def test_chfsi_matches_dense():
    el = tiny_element(n=(8, 8, 8))
    ev = scipy.linalg.eigh(planewave.dense_H(el), eigvals_only=True)
    x0 = W.initial_block(el.npts, 10, seed=17).T
    r = chebyshev.chfsi(el, x0, 6, degree=10, tol=1e-10)
    assert r.converged
    assert np.max(np.abs(r.eigvals[:6] - ev[:6])) < 1e-10


# ---------------------------------------------------------------- ALB

def test_alb_properties_and_lapack_gesvd():
    el = W.small_slab(n_states=8)[2]
    x0 = W.initial_block(el.npts, 12, seed=18).T
    r = lobpcg.lobpcg(el, x0, 8, tol=1e-9)
    U, s = alb.make_alb(el, r.X, 8)
    phi = alb.restrict(el, r.X[:, :8])
    assert U.shape == (np.prod(el.elem_n), 8)
    assert np.max(np.abs(U.T @ U - np.eye(8))) < 1e-13
    assert np.linalg.norm(phi - U @ (U.T @ phi), 2) < 1e-12
    # independent LAPACK driver (dgesvd instead of dgesdd)
    U2, s2, _ = scipy.linalg.svd(phi, full_matrices=False, lapack_driver="gesvd")
    assert np.max(np.abs(s - s2)) < 1e-13
    assert alb.max_principal_angle(U, U2) < 1e-12
    # restriction picks E_k's rows in order
    nx, ny, _ = el.n
    lo = el.elem_lo
    assert phi[1, 0] == r.X[(lo[0] + 1) + nx * (lo[1] + ny * lo[2]), 0]


def test_alb_whole_element_is_identity():
    el = W.make_config("c1").elements[0]
    x0 = W.initial_block(el.npts, 12, seed=19).T
    r = lobpcg.lobpcg(el, x0, 8, tol=1e-9)
    U, s = alb.make_alb(el, r.X, 8)
    assert np.max(np.abs(s - 1.0)) < 1e-13
    assert alb.max_principal_angle(U, r.X[:, :8]) < 1e-12


def test_principal_angle_known_rotation():
    e = np.eye(6)
    t = 1e-4
    A = e[:, :2]
    B = np.column_stack([e[:, 0], np.cos(t) * e[:, 1] + np.sin(t) * e[:, 2]])
    assert abs(alb.max_principal_angle(A, B) - t) < 1e-15


# ---------------------------------------------------------------- band energy gradient

def _be_setup(seed=20, m=4):
    el = tiny_element(n=(6, 6, 8), length=(4.5, 4.5, 6.0), supp=20)
    H = planewave.dense_H(el)
    lam = np.linalg.eigvalsh(H)
    rng = np.random.default_rng(seed)
    psi0 = rng.standard_normal((el.npts, 3))
    f = rng.uniform(0, 2, size=3)
    return el, psi0, f, m, lam[5], lam[-1] + 0.5, lam[0]


def test_band_energy_degree_zero_closed_forms():
    el, psi0, f, _, a, b, a0 = _be_setup()
    E, gpsi, gv = band_energy.band_energy_grad(el, el.v_eff, psi0, f, 0, a, b, a0)
    Hpsi = planewave.hpsi(el, psi0)
    assert np.isclose(E, np.sum(f * np.sum(psi0 * Hpsi, axis=0)), rtol=1e-14)
    assert np.max(np.abs(gpsi - 2 * Hpsi * f)) < 1e-12
    assert np.max(np.abs(gv - (psi0 ** 2) @ f)) < 1e-14


def test_band_energy_grad_fd_psi():
    el, psi0, f, m, a, b, a0 = _be_setup()
    E, gpsi, _ = band_energy.band_energy_grad(el, el.v_eff, psi0, f, m, a, b, a0)
    rng = np.random.default_rng(21)
    for _ in range(3):
        d = rng.standard_normal(psi0.shape)
        d /= np.linalg.norm(d)
        h = 1e-4
        fd = (band_energy.band_energy(el, el.v_eff, psi0 + h * d, f, m, a, b, a0)
              - band_energy.band_energy(el, el.v_eff, psi0 - h * d, f, m, a, b, a0)) / (2 * h)
        an = np.sum(gpsi * d)
        assert abs(fd - an) <= 1e-8 * max(abs(an), 1.0)


def test_band_energy_grad_fd_v():
    el, psi0, f, m, a, b, a0 = _be_setup()
    E, _, gv = band_energy.band_energy_grad(el, el.v_eff, psi0, f, m, a, b, a0)
    rng = np.random.default_rng(22)
    for _ in range(3):
        d = rng.standard_normal(el.npts)
        d /= np.linalg.norm(d)
        h = 1e-4
        fd = (band_energy.band_energy(el, el.v_eff + h * d, psi0, f, m, a, b, a0)
              - band_energy.band_energy(el, el.v_eff - h * d, psi0, f, m, a, b, a0)) / (2 * h)
        an = gv @ d
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0)


def test_rayleigh_ritz_full_span_and_interlacing():
    """On a tiny element: Ritz values of a full-rank start are the eigenvalues of the
    dense Hamiltonian; for a smaller start they lie above the lowest eigenvalues
    (Cauchy interlacing: theta_i >= lambda_i) and each Ritz pair's residual is
    orthogonal to the span."""
    el = tiny_element(n=(8, 8, 8), length=(6.0, 6.4, 7.2), n_states=6)
    lam = np.linalg.eigvalsh(planewave.dense_H(el))
    x0 = W.initial_block(el.npts, el.npts, 4).T
    theta, X = lobpcg.rayleigh_ritz(el, x0)
    assert np.max(np.abs(theta - lam)) < 1e-10 * np.max(np.abs(lam))
    x0 = W.initial_block(el.npts, 9, 5).T
    theta, X = lobpcg.rayleigh_ritz(el, x0)
    assert np.all(theta >= lam[:9] - 1e-12)
    R = planewave.hpsi(el, X) - X * theta
    assert np.max(np.abs(X.T @ R)) < 1e-11 * np.max(np.abs(lam))
    assert np.max(np.abs(X.T @ X - np.eye(9))) < 1e-13
