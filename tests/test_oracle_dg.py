"""Pins of the DG Hamiltonian oracle (Eq. (7)) against closed forms, the plane-wave
Hamiltonian and the global spectrum (CPU only)."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import dg as odg
from oracle import lobpcg as olob
from oracle import planewave

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "free_electron_10bohr_16cubed.txt")


def test_trig_interpolation_closed_form():
    """Value and derivative of the trigonometric interpolant off the grid equal the
    analytic function for a band-limited f, the Nyquist cosine included."""
    n, L = 16, 7.3
    h = L / n
    x = np.arange(n) * h
    G1, G2 = 2 * np.pi * 3 / L, 2 * np.pi * 5 / L
    f = np.cos(G1 * x + 0.7) + 0.3 * np.sin(G2 * x) + 0.2 * np.cos(np.pi * x / h)
    for xf in (2.35 * h, (n - 0.5) * h, -0.5 * h, 0.0):
        w, wd = odg._trig_eval_weights(n, L, xf)
        val = np.cos(G1 * xf + 0.7) + 0.3 * np.sin(G2 * xf) + 0.2 * np.cos(np.pi * xf / h)
        der = -G1 * np.sin(G1 * xf + 0.7) + 0.3 * G2 * np.cos(G2 * xf) - 0.2 * (np.pi / h) * np.sin(np.pi * xf / h)
        assert abs(w @ f - val) < 1e-13
        assert abs(wd @ f - der) < 1e-12


def test_spectral_gradient_closed_form():
    el = W.free_electron_element(n=(16, 12, 24), length=(7.0, 5.0, 9.0))
    nx, ny, nz = el.n
    z, y, x = np.meshgrid(*(np.arange(el.n[a]) * el.length[a] / el.n[a] for a in (2, 1, 0)), indexing="ij")
    G = np.array([2 * np.pi * 2 / 7.0, -2 * np.pi * 1 / 5.0, 2 * np.pi * 3 / 9.0])
    f = np.cos(G[0] * x + G[1] * y + G[2] * z + 0.4).ravel()
    g = -np.sin(G[0] * x + G[1] * y + G[2] * z + 0.4).ravel()
    D = odg.spectral_gradient(el, f[:, None])
    for a in range(3):
        assert np.max(np.abs(D[a, :, 0] - G[a] * g)) < 1e-12


def _one_element_case():
    els, mesh = W.small_slab_with_mesh(n_mesh=1, elem_pts=24, nz=32, buffer=0, n_states=8)
    el = els[0]
    x0 = W.initial_block(el.npts, 12, 11).T
    X = olob.lobpcg(el, x0, 8, tol=1e-11).X
    return el, mesh, X


def test_single_element_domain_is_the_projected_hamiltonian():
    """One element covering the periodic domain: the ALB traces on its two x faces (and
    two y faces) are the same periodic function, every jump vanishes, and Eq. (7)
    reduces to Phi^T H Phi with H the plane-wave Hamiltonian of Eq. (1)."""
    el, mesh, X = _one_element_case()
    blocks = odg.dg_hamiltonian(mesh, [el], [X], alpha=40.0)
    assert list(blocks) == [(0, 0)]
    U, s, Wc = odg.alb_coefficients(el, X, 8)
    ref = U.T @ planewave.hpsi(el, U)
    assert np.max(np.abs(blocks[(0, 0)] - 0.5 * (ref + ref.T))) < 1e-9
    # and the traces do match across the periodic seam
    tr = odg.face_traces(el, X[:, :8] @ Wc)
    assert np.max(np.abs(tr["x+"][0] - tr["x-"][0])) < 1e-12
    assert np.max(np.abs(tr["x+"][1] + tr["x-"][1])) < 1e-11      # outward derivatives opposite


def test_single_element_free_electrons_closed_form():
    """v = 0, no projectors, one element: the eigenvalues of H^DG are the lowest
    |G|^2/2 shells (J on a shell closure)."""
    rows = np.loadtxt(GOLDEN)
    expect = np.concatenate([np.full(int(m), v) for _, v, m, _ in rows])
    for J in (7, 19):
        el = W.free_electron_element(n_states=J)
        mesh = W.Mesh(1, 16, (16, 16, 16), (10.0, 10.0, 10.0), np.zeros(16 ** 3), [])
        X = olob.lobpcg(el, W.initial_block(el.npts, J + W.guard_count(J), 3).T, J, tol=1e-11).X
        H = odg.dense_from_blocks(odg.dg_hamiltonian(mesh, [el], [X], alpha=40.0), [J])
        assert np.max(np.abs(np.linalg.eigvalsh(H) - expect[:J])) < 1e-10


@pytest.fixture(scope="module")
def slab_dg():
    """DG Hamiltonians of the 3x3 small slab from 8 and from 16 ALBs per element."""
    out = {}
    for J in (8, 16):
        els, mesh = W.small_slab_with_mesh(n_states=J)
        Xs = [olob.lobpcg(el, W.initial_block(el.npts, J + W.guard_count(J), 600 + k).T, J, tol=1e-9).X
              for k, el in enumerate(els)]
        out[J] = (els, mesh, odg.dg_hamiltonian(mesh, els, Xs, alpha=40.0))
    return out


def test_slab_dg_hamiltonian_is_symmetric_and_block_sparse(slab_dg):
    els, mesh, blocks = slab_dg[8]
    H = odg.dense_from_blocks(blocks, [8] * len(els))
    assert np.max(np.abs(H - H.T)) < 1e-12 * np.max(np.abs(H))
    for k in range(len(els)):
        for nb in mesh.neighbours(k):
            assert (k, nb) in blocks and (nb, k) in blocks
            assert np.max(np.abs(blocks[(k, nb)] - blocks[(nb, k)].T)) < 1e-13


def test_slab_dg_spectrum_converges_to_the_global_problem(slab_dg):
    """The DG eigenvalues against the global plane-wave problem on the whole 24x24x32
    slab (every atom): they lie above it, and doubling the ALBs per element (8 -> 16)
    cuts the error of the lowest eight states at least in half (measured: 0.51 ->
    0.17 Ha).  A sign error in a face term or a missing nonlocal coupling breaks one
    of the two."""
    els, mesh, _ = slab_dg[8]
    gel = W.Element(n=mesh.global_n, length=mesh.length, elem_lo=(0, 0, 0), elem_n=mesh.global_n, n_states=8,
                    v_eff=mesh.v_global, proj_ptr=None, proj_idx=None, proj_val=None, gamma=None)
    gid, ptr, idx, val, gam = _global_projectors(mesh)
    gel.proj_ptr, gel.proj_idx, gel.proj_val, gel.gamma = ptr, idx, val, gam
    ref = olob.lobpcg(gel, W.initial_block(gel.npts, 12, 5).T, 8, tol=1e-9).eigvals[:8]
    errs = {}
    for J, (els_j, _, blocks) in slab_dg.items():
        ev = np.linalg.eigvalsh(odg.dense_from_blocks(blocks, [J] * len(els_j)))[:8]
        errs[J] = ev - ref
        print(f"J = {J}: DG - global (Ha):", np.array2string(errs[J], precision=4))
        assert np.all(errs[J] >= -1e-3)
    assert np.max(errs[16]) <= 0.5 * np.max(errs[8])


def _global_projectors(mesh):
    ptr, idx, val, gam, gid = [0], [], [], [], []
    for a, (ai, av) in enumerate(mesh.atoms):
        for p in range(4):
            idx.append(ai.astype(np.int32))
            val.append(av[p])
            gam.append(W.GAMMA_S if p == 0 else W.GAMMA_P)
            gid.append(4 * a + p)
            ptr.append(ptr[-1] + len(ai))
    return (np.array(gid), np.array(ptr, dtype=np.int64), np.concatenate(idx), np.concatenate(val),
            np.array(gam))


def test_block_product_and_chefsi_on_the_dg_hamiltonian(slab_dg):
    """Eq. (8)'s block-row product equals the dense product, and CheFSI (Algorithm 2)
    on H^DG reaches the lowest eigenpairs of the dense matrix (brute force)."""
    els, mesh, blocks = slab_dg[8]
    Js = [8] * len(els)
    H = odg.dense_from_blocks(blocks, Js)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((H.shape[0], 5))
    assert np.max(np.abs(odg.apply_blocks(blocks, Js, X) - H @ X)) < 1e-12 * np.max(np.abs(H))
    lam, V = np.linalg.eigh(H)
    n_want = 20
    r = odg.dg_chefsi(blocks, Js, W.initial_block(H.shape[0], n_want + 4, 21).T, n_want, degree=12, tol=1e-9)
    assert r.converged
    assert np.max(np.abs(r.eigvals[:n_want] - lam[:n_want])) < 1e-9
    # same invariant subspace (lam[n_want] - lam[n_want - 1] is well above the residual)
    P = r.X[:, :n_want] @ r.X[:, :n_want].T - V[:, :n_want] @ V[:, :n_want].T
    assert np.linalg.norm(P, 2) < 1e-7
