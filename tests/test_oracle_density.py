"""Pins of the density oracle (Eqs. (10) and (11)) against the orbital definition, the
sum rule and closed-shell free electrons (CPU only)."""
import os

import numpy as np

import workloads as W
from oracle import density as odens
from oracle import dg as odg
from oracle import lobpcg as olob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "free_electron_10bohr_16cubed.txt")


def _random_orthonormal(rng, n, J):
    q, _ = np.linalg.qr(rng.standard_normal((n, J)))
    return q


def test_density_matrix_route_equals_orbitals_on_the_mesh():
    """The diagonal blocks of P (Eq. (10), last line) against the orbitals assembled
    point by point over the whole 3x3 slab and squared (Eq. (10), first line): a wrong
    element's rows of C, a missing symmetrisation or a dropped state breaks it.  The
    ALBs are random orthonormal bases of unequal size per element; N_e differs from
    every J_k so a transposed product cannot go through."""
    _, mesh = W.small_slab_with_mesh(n_states=8)
    rng = np.random.default_rng(3)
    n_e_pts = [len(mesh.elem_global_indices(k)) for k in range(mesh.n_elem)]
    Js = [5 + (k % 4) for k in range(mesh.n_elem)]
    U = [_random_orthonormal(rng, n_e_pts[k], Js[k]) for k in range(mesh.n_elem)]
    n_e = 11
    C = rng.standard_normal((sum(Js), n_e))
    rho = odens.density(U, C, Js)
    ref = odens.density_from_orbitals(U, C, Js, mesh.elem_global_indices, int(np.prod(mesh.global_n)))
    got = np.zeros_like(ref)
    for k in range(mesh.n_elem):
        got[mesh.elem_global_indices(k)] = rho[k]
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(ref)
    # sum rule: orthonormal ALBs carry the norm of every state
    assert abs(got.sum() - np.trace(C.T @ C)) < 1e-11 * np.trace(C.T @ C)


def test_density_matrix_blocks_are_symmetric_positive_semidefinite():
    rng = np.random.default_rng(5)
    Js = [4, 7, 3]
    C = rng.standard_normal((sum(Js), 2))           # rank 2 < every J_k
    for P in odens.density_matrix_blocks(C, Js):
        w = np.linalg.eigvalsh(P)
        assert np.allclose(P, P.T, atol=0)
        assert w.min() > -1e-13 and np.sum(w > 1e-12) <= 2


def test_closed_shell_free_electrons_give_a_uniform_density():
    """v = 0, one element covering the periodic box: the DG eigenvectors of the lowest
    J states fill whole |G|^2 shells (J = 7, 19), and a filled shell's squared
    orbitals sum to the same value at every point, J / N per grid point."""
    rows = np.loadtxt(GOLDEN)
    sizes = np.cumsum([int(m) for _, _, m, _ in rows])
    for J in (7, 19):
        assert J in sizes
        el = W.free_electron_element(n_states=J)
        mesh = W.Mesh(1, 16, (16, 16, 16), (10.0, 10.0, 10.0), np.zeros(16 ** 3), [])
        X = olob.lobpcg(el, W.initial_block(el.npts, J + W.guard_count(J), 3).T, J, tol=1e-11).X
        H = odg.dense_from_blocks(odg.dg_hamiltonian(mesh, [el], [X], alpha=40.0), [J])
        _, Cdg = np.linalg.eigh(H)
        Uo, _, _ = odg.alb_coefficients(el, X, J)
        rho = odens.density([Uo], Cdg, [J])[0]
        # X holds the shell to its residual 1e-11 (over the gap 0.197 Ha)
        assert np.max(np.abs(rho - J / el.npts)) < 1e-9 * (J / el.npts)
        # a partly filled shell is not uniform
        rho_part = odens.density([Uo], Cdg[:, :J - 1], [J])[0]
        assert np.max(rho_part) - np.min(rho_part) > 1e-3 / el.npts
