"""The DG Hamiltonian (Eq. (7)) and the density (Eqs. (10), (11)) on the GPU against
the oracle.

Both sides start from the same seeded blocks X0 (one per element, J_k + g_k columns)
and take the Ritz vectors of span(X0) (the GPU through a solve that stops after its
first Rayleigh-Ritz step, the oracle by that step's definition); each then forms its
own orthonormal ALB basis of span(R_E X), so the two Hamiltonians differ by a
block-diagonal rotation Q_k = U_oracle^T U_gpu, applied only in the comparison.
Two starts: the oracle's converged LOBPCG eigenvectors of the 3x3 small slab (the
physical case; its X0 is an oracle output, the GPU's Ritz step leaves it in place),
and seeded Gaussian blocks on the 4x4 slab at full size (48x48x64, 40 ALBs).

The density is compared on basis-independent inputs: each side's own lowest DG
eigenvectors below a gap of its spectrum, and coefficients C_k = U_k^T Y_k of seeded
real-space blocks Y_k (so U_k C_k = U_k U_k^T Y_k is the projection of Y_k on the ALB
span, the same on both sides)."""
import numpy as np
import pytest

import workloads as W
from oracle import density as odens
from oracle import dg as odg
from oracle import lobpcg as olob
from tests.gpu_util import need_torch_cuda, unpack

pytestmark = pytest.mark.gpu

ALPHA = 40.0


class Case:
    pass


def _run(els, mesh, X0):
    """GPU: Ritz step on X0, ALBs, H^DG.  Oracle: Ritz step on X0, H^DG."""
    torch = need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    print(f"[dg] {len(els)} elements grid {els[0].n} J {els[0].n_states}", flush=True)
    c = Case()
    c.els, c.mesh, c.X0 = els, mesh, X0
    c.Js = [e.n_states for e in els]
    E = D.Elements(els)
    x0 = torch.tensor(np.concatenate([x.T.ravel() for x in X0]), dtype=torch.float64, device="cuda")
    eig, res, iters, st = E.solve(x0, tol=1e30, max_iter=1)
    assert st == 0
    alb, sv = E.make_alb()
    c.U = unpack(alb.cpu().numpy(), E.offsets(D.DG_OFF_ALB), [int(np.prod(e.elem_n)) for e in els], c.Js)
    hm = D.HostMesh((mesh.n_mesh, mesh.n_mesh), ALPHA, [mesh.elem_projectors(k) for k in range(len(els))])
    H, layout = E.build_hamiltonian(hm)
    c.blocks = E.hamiltonian_blocks(H, layout)
    c.H, c.layout = H, layout
    c.E, c.alb, c.D = E, alb, D
    # oracle
    c.X = [olob.rayleigh_ritz(el, X0[k])[1] for k, el in enumerate(els)]
    c.ref = odg.dg_hamiltonian(mesh, els, c.X, ALPHA)
    c.Uo = [odg.alb_coefficients(el, c.X[k], el.n_states)[0] for k, el in enumerate(els)]
    return c


@pytest.fixture(scope="module")
def small_slab():
    els, mesh = W.small_slab_with_mesh(n_states=8)
    X0 = [olob.lobpcg(el, W.initial_block(el.npts, 8 + W.guard_count(8), 600 + k).T, 8, tol=1e-10).X
          for k, el in enumerate(els)]
    return _run(els, mesh, X0)


@pytest.fixture(scope="module")
def c2_slab():
    cfg = W.make_config("c2")
    els = cfg.elements
    X0 = [W.initial_block(el.npts, el.n_states + W.guard_count(el.n_states), cfg.x0_seed_base + k).T
          for k, el in enumerate(els)]
    return _run(els, cfg.mesh, X0)


def _rotations(c, U):
    Q = []
    for k in range(len(c.els)):
        Q.append(c.Uo[k].T @ U[k])
        assert np.max(np.abs(Q[-1].T @ Q[-1] - np.eye(c.Js[k]))) < 1e-10   # same span
    return Q


def _block_distance(blocks, ref, Q, Js, scale):
    worst = 0.0
    for (k, nb), G in blocks.items():
        R = ref.get((k, nb), np.zeros((Js[k], Js[nb])))
        worst = max(worst, np.max(np.abs(G - Q[k].T @ R @ Q[nb])) / scale)
    return worst


def _perturbed_oracle(c):
    """The oracle on X0 perturbed entrywise by relative sqrt(N_k) eps with random signs
    (the error model of a length-N_k dot product, as in every Gram of the GPU path);
    computed once per case."""
    if getattr(c, "pert", None) is None:
        c.pert = _perturbed_oracle_run(c)
    return c.pert


def _perturbed_oracle_run(c):
    rng = np.random.default_rng(7)
    eps = np.finfo(np.float64).eps
    X0p = [x * (1.0 + np.sqrt(x.shape[0]) * eps * rng.standard_normal(x.shape)) for x in c.X0]
    Xp = [olob.rayleigh_ritz(el, X0p[k])[1] for k, el in enumerate(c.els)]
    Up = [odg.alb_coefficients(el, Xp[k], el.n_states)[0] for k, el in enumerate(c.els)]
    return Up, odg.dg_hamiltonian(c.mesh, c.els, Xp, ALPHA)


def _check_hamiltonian(c):
    """Blocks and spectrum against the oracle, to within 10x the oracle's own response to
    a rounding-level change of X0.  The ALBs extend to Q_k through W = V S^-1, so a
    rounding error in the restriction is amplified by up to sigma_max / sigma_min; the
    bound is measured, not assumed."""
    for key in c.ref:
        assert key in c.blocks, f"oracle block {key} missing on the GPU"
    scale = max(np.max(np.abs(b)) for b in c.ref.values())
    worst = _block_distance(c.blocks, c.ref, _rotations(c, c.U), c.Js, scale)
    Up, ref_p = _perturbed_oracle(c)
    sens = _block_distance(ref_p, c.ref, _rotations(c, Up), c.Js, scale)
    Hg = odg.dense_from_blocks(c.blocks, c.Js)
    Ho = odg.dense_from_blocks(c.ref, c.Js)
    ev_g, ev_o = np.linalg.eigvalsh(0.5 * (Hg + Hg.T)), np.linalg.eigvalsh(Ho)
    ev_sens = np.max(np.abs(np.linalg.eigvalsh(odg.dense_from_blocks(ref_p, c.Js)) - ev_o))
    print(f"[dg] max block difference {worst:.1e} (relative to max |H| {scale:.2f}; oracle's own response to "
          f"rounding {sens:.1e}); asymmetry {np.max(np.abs(Hg - Hg.T)) / scale:.1e}; lowest DG eigenvalues "
          f"{ev_g[:4]}, max eigenvalue difference {np.max(np.abs(ev_g - ev_o)):.1e} (oracle's response "
          f"{ev_sens:.1e})", flush=True)
    assert worst <= 10.0 * max(sens, 1e-14)
    assert np.max(np.abs(Hg - Hg.T)) <= 1e-14 * scale
    assert np.max(np.abs(ev_g - ev_o)) <= 10.0 * max(ev_sens, 1e-14 * scale)


def _gpu_density(c, C):
    torch = need_torch_cuda()
    Ct = torch.tensor(np.ascontiguousarray(C.T), dtype=torch.float64, device="cuda")
    P, rho = c.E.density(c.alb, Ct)
    D = c.D
    rho_k = unpack(rho.cpu().numpy(), c.E.offsets(D.DG_OFF_ELEM), [len(c.U[k]) for k in range(len(c.els))],
                   [1] * len(c.els))
    P_k = unpack(P.cpu().numpy(), c.E.offsets(D.DG_OFF_JJ), c.Js, c.Js)
    return [r[:, 0] for r in rho_k], P_k


def _projected_density(c, U, Uo, Y, rho_o, P_o, rho, P):
    """(max rho difference / max rho, max P-block difference / max |P_kk|) of a density
    (rho, P in the basis U) against the oracle's (rho_o, P_o in the basis Uo)."""
    Q = _rotations(c, U)
    scale = max(np.max(r) for r in rho_o)
    err = max(np.max(np.abs(rho[k] - rho_o[k])) for k in range(len(c.els))) / scale
    perr = max(np.max(np.abs(P[k] - Q[k].T @ P_o[k] @ Q[k])) / np.max(np.abs(P_o[k])) for k in range(len(c.els)))
    return err, perr, scale


def _check_density_projection(c, n_e):
    """rho of C_k = U_k^T Y_k (seeded Y_k on E_k): the same function on both sides; the
    bound is 10x the oracle's response to the rounding-level change of X0."""
    rng = np.random.default_rng(11)
    nk = range(len(c.els))
    Y = [rng.standard_normal((len(c.U[k]), n_e)) for k in nk]
    Cg = np.concatenate([c.U[k].T @ Y[k] for k in nk])
    Co = np.concatenate([c.Uo[k].T @ Y[k] for k in nk])
    rho_g, P_g = _gpu_density(c, Cg)
    rho_o = odens.density(c.Uo, Co, c.Js)
    P_o = odens.density_matrix_blocks(Co, c.Js)
    err, perr, scale = _projected_density(c, c.U, c.Uo, Y, rho_o, P_o, rho_g, P_g)
    Up, _ = _perturbed_oracle(c)
    Cp = np.concatenate([Up[k].T @ Y[k] for k in nk])
    serr, sperr, _ = _projected_density(c, Up, c.Uo, Y, rho_o, P_o, odens.density(Up, Cp, c.Js),
                                        odens.density_matrix_blocks(Cp, c.Js))
    print(f"[density] projected Y ({n_e} states): max rho difference {err:.1e} of max rho {scale:.3e} (oracle's "
          f"response to rounding {serr:.1e}); P blocks {perr:.1e} (oracle's response {sperr:.1e})", flush=True)
    return err, perr, serr, sperr


def _check_density_eigenvectors(c):
    """rho of the lowest DG eigenvectors of each side's own H^DG, up to the widest gap
    between J and 2 J states of the oracle's spectrum (a basis-independent projector)."""
    Hg = odg.dense_from_blocks(c.blocks, c.Js)
    Ho = odg.dense_from_blocks(c.ref, c.Js)
    ev_o, Vo = np.linalg.eigh(Ho)
    ev_g, Vg = np.linalg.eigh(0.5 * (Hg + Hg.T))
    J = c.Js[0]
    gaps = ev_o[J:2 * J] - ev_o[J - 1:2 * J - 1]
    n_e = J + int(np.argmax(gaps))
    rho_g, _ = _gpu_density(c, Vg[:, :n_e])
    rho_o = odens.density(c.Uo, Vo[:, :n_e], c.Js)
    scale = max(np.max(r) for r in rho_o)
    err = max(np.max(np.abs(rho_g[k] - rho_o[k])) for k in range(len(c.els))) / scale
    total = sum(r.sum() for r in rho_g)
    # ||H_gpu - Q^T H_oracle Q||_2 with Q the block-diagonal basis rotation
    Q = _rotations(c, c.U)
    off = np.concatenate([[0], np.cumsum(c.Js)])
    Qd = np.zeros_like(Ho)
    for k in range(len(c.els)):
        Qd[off[k]:off[k + 1], off[k]:off[k + 1]] = Q[k]
    dev = np.linalg.norm(0.5 * (Hg + Hg.T) - Qd.T @ Ho @ Qd, 2)
    print(f"[density] lowest {n_e} DG states (gap {np.max(gaps):.3f} Ha, ||dH|| {dev:.1e}): max rho difference "
          f"{err:.1e} of max rho {scale:.3e}; sum rho {total:.12f}", flush=True)
    return err, total, n_e, np.max(gaps), dev


def test_dg_hamiltonian_small_slab_vs_oracle(small_slab):
    _check_hamiltonian(small_slab)


def test_dg_hamiltonian_c2_vs_oracle(c2_slab):
    """The 4x4 slab at full size: 16 elements of 48x48x64, 40 ALBs each."""
    _check_hamiltonian(c2_slab)


@pytest.mark.parametrize("case", ["small_slab", "c2_slab"])
def test_density_of_projected_blocks_vs_oracle(case, request):
    c = request.getfixturevalue(case)
    for n_e in (1, 13, 3 * c.Js[0] + 5):
        err, perr, serr, sperr = _check_density_projection(c, n_e)
        assert err <= 10.0 * max(serr, 1e-14) and perr <= 10.0 * max(sperr, 1e-14)


@pytest.mark.parametrize("case", ["small_slab", "c2_slab"])
def test_density_of_dg_eigenvectors_vs_oracle(case, request):
    """The occupied subspace moves by at most ||dH|| / gap (Davis-Kahan), and rho, a
    quadratic form in it, by about twice that relative to its maximum: the bound is
    10 x ||dH|| / gap + rounding."""
    c = request.getfixturevalue(case)
    err, total, n_e, gap, dev = _check_density_eigenvectors(c)
    assert abs(total - n_e) <= 1e-10 * n_e
    assert err <= 10.0 * dev / gap + 1e-12


def test_density_edge_cases(small_slab):
    """No states gives zeros; ldc larger than the row count reads only the first rows."""
    torch = need_torch_cuda()
    c = small_slab
    n_rows = sum(c.Js)
    P, rho = c.E.density(c.alb, None, n_e=0)
    assert float(rho.abs().max()) == 0.0 and float(P.abs().max()) == 0.0
    rng = np.random.default_rng(2)
    C = rng.standard_normal((n_rows, 5))
    wide = np.zeros((5, n_rows + 7))
    wide[:, :n_rows] = C.T
    wide[:, n_rows:] = np.nan       # never read
    Ct = torch.tensor(wide, dtype=torch.float64, device="cuda")
    P1, rho1 = c.E.density(c.alb, Ct, n_e=5, ldc=n_rows + 7)
    rho2, _ = _gpu_density(c, C)
    assert np.array_equal(rho1.cpu().numpy(), np.concatenate(rho2))


# ---------------------------------------------------------------------------
# CheFSI on H^DG (Algorithm 2)
# ---------------------------------------------------------------------------
def _pack_blocks(c, blocks):
    """A block dict in the device layout of build_hamiltonian (absent blocks zero)."""
    torch = need_torch_cuda()
    row_ptr, col, off = c.layout
    flat = np.zeros(int(off[-1]))
    for k in range(len(c.els)):
        for b in range(int(row_ptr[k]), int(row_ptr[k + 1])):
            B = blocks.get((k, int(col[b])))
            if B is not None:
                flat[off[b]:off[b + 1]] = B.T.ravel()      # column-major J_k x J_col
    return torch.tensor(flat, dtype=torch.float64, device="cuda")


def _chefsi_case(c, n_want, n_vec, degree, tol, seed=31, max_iter=200):
    """GPU CheFSI on the oracle's H^DG against the dense eigendecomposition of the same
    matrix and against the oracle's CheFSI (Algorithm 2) from the same start."""
    torch = need_torch_cuda()
    Ho = odg.dense_from_blocks(c.ref, c.Js)
    Nb = Ho.shape[0]
    x0 = W.initial_block(Nb, n_vec, seed)                 # (n_vec, N_b): column-major N_b x n_vec
    X, eig, res, it, st = c.E.chefsi(_pack_blocks(c, c.ref), c.layout,
                                     torch.tensor(x0, dtype=torch.float64, device="cuda"), n_want,
                                     degree=degree, tol=tol, max_iter=max_iter)
    lam, V = np.linalg.eigh(Ho)
    Xg = X.cpu().numpy().T
    th = eig.cpu().numpy()
    r = res.cpu().numpy()
    orc = odg.dg_chefsi(c.ref, c.Js, x0.T, n_want, degree=degree, tol=tol, max_iter=max_iter)
    gap = lam[n_want] - lam[n_want - 1]
    Pd = Xg[:, :n_want] @ Xg[:, :n_want].T - V[:, :n_want] @ V[:, :n_want].T
    true_res = np.linalg.norm(Ho @ Xg[:, :n_want] - Xg[:, :n_want] * th[:n_want], axis=0)
    print(f"[chefsi] N_b {Nb} n_want {n_want} n_vec {n_vec} m {degree}: status {st}, {it} passes (oracle "
          f"{orc.iters}); max |theta - lambda| {np.max(np.abs(th[:n_want] - lam[:n_want])):.1e}, reported "
          f"residual {r[:n_want].max():.1e}, recomputed {true_res.max():.1e}, subspace {np.linalg.norm(Pd, 2):.1e} "
          f"(gap {gap:.3f})", flush=True)
    return st, it, th, r, true_res, lam, Pd, gap, orc


@pytest.mark.parametrize("case,n_want,n_vec,degree", [("small_slab", 20, 24, 12), ("c2_slab", 60, 72, 16)])
def test_chefsi_on_dg_hamiltonian_vs_dense_and_oracle(case, n_want, n_vec, degree, request):
    """Ritz values within the residual bound |theta_i - lambda_i| <= ||r_i||, the wanted
    subspace within ||r|| / gap (Davis-Kahan), residuals recomputed on the host agree
    with the reported ones, and the oracle's CheFSI from the same start converges to the
    same pairs."""
    c = request.getfixturevalue(case)
    tol = 1e-9
    st, it, th, r, true_res, lam, Pd, gap, orc = _chefsi_case(c, n_want, n_vec, degree, tol)
    assert st == 0 and orc.converged
    assert r[:n_want].max() <= tol and true_res.max() <= 2 * tol
    assert np.max(np.abs(th[:n_want] - lam[:n_want])) <= 2 * tol
    assert np.linalg.norm(Pd, 2) <= 10 * tol * np.sqrt(n_want) / gap
    assert np.max(np.abs(th[:n_want] - orc.eigvals[:n_want])) <= 4 * tol


def test_chefsi_edge_cases(small_slab):
    """One pass cannot reach 1e-12 (a warning with finite output); a start block with a
    repeated column is rank deficient (a numeric error); a block wider than N_b / 2 is a
    shape error; a layout whose block sizes do not match the elements is an argument
    error."""
    torch = need_torch_cuda()
    c = small_slab
    D = c.D
    Ho = odg.dense_from_blocks(c.ref, c.Js)
    Nb = Ho.shape[0]
    Hdev = _pack_blocks(c, c.ref)
    x0 = torch.tensor(W.initial_block(Nb, 24, 5), dtype=torch.float64, device="cuda")
    X, eig, res, it, st = c.E.chefsi(Hdev, c.layout, x0, 20, degree=8, tol=1e-12, max_iter=1)
    assert st == D.DG_WARN_NOT_CONVERGED and it == 1
    assert np.all(np.isfinite(eig.cpu().numpy())) and np.all(np.isfinite(X.cpu().numpy()))
    xd = x0.clone()
    xd[3] = xd[2]
    with pytest.raises(D.DGError) as e:
        c.E.chefsi(Hdev, c.layout, xd, 20, degree=8, tol=1e-9)
    assert e.value.status == D.DG_ERR_NUMERIC
    with pytest.raises(D.DGError) as e:
        c.E.chefsi(Hdev, c.layout, torch.zeros((37, Nb), dtype=torch.float64, device="cuda"), 20)
    assert e.value.status == D.DG_ERR_SHAPE
    row_ptr, col, off = c.layout
    bad = (row_ptr, col, off.copy())
    bad[2][1:] += 1
    with pytest.raises(D.DGError) as e:
        c.E.chefsi(Hdev, bad, x0, 20)
    assert e.value.status == D.DG_ERR_ARG


def test_chefsi_on_the_gpu_built_hamiltonian(c2_slab):
    """The pipeline as it runs: the GPU's H^DG into the GPU's CheFSI.  Its Ritz values
    match the oracle H^DG's eigenvalues to the Hamiltonians' own difference (the
    basis rotation leaves the spectrum unchanged)."""
    torch = need_torch_cuda()
    c = c2_slab
    Ho = odg.dense_from_blocks(c.ref, c.Js)
    lam = np.linalg.eigvalsh(Ho)
    Hg = odg.dense_from_blocks(c.blocks, c.Js)
    dev = np.max(np.abs(np.linalg.eigvalsh(0.5 * (Hg + Hg.T)) - lam))
    x0 = torch.tensor(W.initial_block(Ho.shape[0], 72, 8), dtype=torch.float64, device="cuda")
    X, eig, res, it, st = c.E.chefsi(c.H, c.layout, x0, 60, degree=16, tol=1e-9)
    th = eig.cpu().numpy()[:60]
    print(f"[chefsi] GPU-built H^DG: {it} passes, max |theta - lambda_oracle| {np.max(np.abs(th - lam[:60])):.1e} "
          f"(H difference {dev:.1e})", flush=True)
    assert st == 0
    assert np.max(np.abs(th - lam[:60])) <= 2e-9 + 10 * dev
