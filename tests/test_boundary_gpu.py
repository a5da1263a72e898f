"""The C-ABI's promises on the GPU: error paths forced from host arguments, the
seeded device start, strided H*psi buffers, the Ritz values that expose the gap at
the cut, and warm-started re-solves after a potential update (the inner SCF loop
in which the ALBs adapt to V_eff, "Generating ALB functions" subsection; Fig. 2).

Every kernel in these tests runs to completion: failures are provoked through the
inputs (a NaN potential, a rank-deficient start block or restriction, one
iteration), and the library reports them as status codes.
"""
import dataclasses
import os

import numpy as np
import pytest

import workloads as W
from oracle import alb as oalb
from oracle import chebyshev as ocheb
from oracle import lobpcg as olobpcg
from oracle import planewave
from tests.gpu_util import need_torch_cuda, unpack

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "free_electron_10bohr_16cubed.txt")


def _D():
    from paper_2003_00407_amd import dgalb as D
    return D


def _x0(els, seed_base):
    torch = need_torch_cuda()
    return torch.tensor(_D().pack_initial(els, seed_base), dtype=torch.float64, device="cuda")


def _per_elem(t, off):
    a = t.cpu().numpy()
    return [a[off[k]:off[k + 1]] for k in range(len(off) - 1)]


def test_one_iteration_warns_not_converged():
    D = _D()
    els = W.small_slab(n_states=8)[:3]
    print("[boundary] max_iter = 1", flush=True)
    E = D.Elements(els)
    eig, res, iters, st = E.solve(_x0(els, 100), max_iter=1, tol=1e-9)
    assert st == D.DG_WARN_NOT_CONVERGED
    assert np.all(np.isfinite(eig.cpu().numpy())) and res.max().item() > 1e-9
    assert np.all(iters == 1)
    # the outputs are valid: orthonormal vectors, ALBs can be formed
    X = unpack(E.vectors().cpu().numpy(), E.offsets(D.DG_OFF_VEC), [e.npts for e in els],
               [e.n_states for e in els])
    assert max(np.max(np.abs(x.T @ x - np.eye(8))) for x in X) < 1e-10


def test_nan_potential_is_numeric_error_and_context_recovers():
    torch = need_torch_cuda()
    D = _D()
    els = W.small_slab(n_states=8)[:2]
    print("[boundary] NaN in V_eff via set_potential", flush=True)
    E = D.Elements(els)
    v = np.concatenate([e.v_eff for e in els])
    bad = v.copy()
    bad[els[0].npts + 777] = np.nan
    E.set_potential(torch.tensor(bad, dtype=torch.float64, device="cuda"))
    with pytest.raises(D.DGError) as ex:
        E.solve(_x0(els, 100), tol=1e-9)
    assert ex.value.status == D.DG_ERR_NUMERIC
    assert "non-finite" in str(ex.value)
    # a valid potential again: the same context solves normally
    E.set_potential(torch.tensor(v, dtype=torch.float64, device="cuda"))
    eig, res, iters, st = E.solve(_x0(els, 100), tol=1e-9)
    assert st == 0 and res.max().item() <= 1e-9


@pytest.mark.parametrize("method", [0, 1])
def test_repeated_start_columns_are_rank_deficient(method):
    """X0 with two equal columns: the Cholesky of X0^T X0 breaks down (DG_ERR_NUMERIC)."""
    torch = need_torch_cuda()
    D = _D()
    els = W.small_slab(n_states=8)[:2]
    print(f"[boundary] repeated start columns, method {method}", flush=True)
    E = D.Elements(els)
    x0 = _x0(els, 100)
    off = E.offsets(D.DG_OFF_X0)
    n1 = els[1].npts
    b = x0[off[1]:off[2]].view(-1, n1)
    b[3].copy_(b[5])
    with pytest.raises(D.DGError) as ex:
        E.solve(x0, method=method, tol=1e-9, cheb_degree=10)
    assert ex.value.status == D.DG_ERR_NUMERIC
    assert "rank deficient" in str(ex.value)


def test_rank_deficient_restriction_is_numeric_error():
    """Free electrons, J = 7 (two closed shells: 1, cos/sin along x, y, z): on a line
    of E_k points along z the x and y modes are constants, so the restriction has
    rank 3 < 7 and no ALB basis exists."""
    D = _D()
    el = dataclasses.replace(W.free_electron_element(n_states=7), elem_lo=(3, 5, 0), elem_n=(1, 1, 16))
    print("[boundary] rank-deficient restriction", flush=True)
    E = D.Elements([el])
    eig, res, iters, st = E.solve(_x0([el], 57), tol=1e-9)
    assert st == 0
    with pytest.raises(D.DGError) as ex:
        E.make_alb()
    assert ex.value.status == D.DG_ERR_NUMERIC
    assert "rank deficient" in str(ex.value)


def test_degenerate_cut_reports_zero_gap():
    """J = 8 cuts the 12-fold third free-electron shell: the Ritz values of the
    wanted and guard states show a zero gap at the cut (the ALB span is not unique),
    while the eigenvalues are the closed-form shells."""
    D = _D()
    rows = np.loadtxt(GOLDEN)
    expect = np.concatenate([np.full(int(m), v) for _, v, m, _ in rows])
    el = W.free_electron_element(n_states=8)
    print("[boundary] degenerate cut J = 8", flush=True)
    E = D.Elements([el])
    eig, res, iters, st = E.solve(_x0([el], 58), tol=1e-9)
    assert st == 0
    th, rs = E.ritz()
    th = th.cpu().numpy()
    K = 8 + W.guard_count(8)
    assert th.size == K
    gap = th[8] - th[7]
    print(f"Ritz values {th}, gap at the cut {gap:.2e}, guard residuals {rs.cpu().numpy()[8:]}")
    assert np.max(np.abs(eig.cpu().numpy() - expect[:8])) < 1e-8
    assert abs(gap) < 1e-7
    # guards converge more slowly: bounded by their own residuals
    assert np.all(np.abs(th[8:] - expect[8:K]) <= rs.cpu().numpy()[8:] + 1e-8)


def test_seeded_device_start():
    """x0 = NULL: a counter-based seeded start drawn on the device; any seed reaches
    the same eigenvalues, and the start does not depend on the element groups."""
    D = _D()
    els = W.small_slab(n_states=8)
    print("[boundary] seeded device start", flush=True)
    E1 = D.Elements(els, n_streams=1)
    e1, r1, i1, s1 = E1.solve(None, seed=7, tol=1e-10)
    e2, r2, i2, s2 = E1.solve(None, seed=8, tol=1e-10)
    E3 = D.Elements(els, n_streams=3)
    e3, r3, i3, s3 = E3.solve(None, seed=7, tol=1e-10)
    assert s1 == 0 and s2 == 0 and s3 == 0
    assert (e1 - e2).abs().max().item() < 1e-9
    assert (e1 - e3).abs().max().item() < 1e-10
    # same seed, same start with one group or three (only the Gram row splits, and so
    # the rounding, may differ)
    assert np.max(np.abs(i1 - i3)) <= 2
    ref = olobpcg.lobpcg(els[4], W.initial_block(els[4].npts, 12, 4).T, 8, tol=1e-10)
    off = E1.offsets(D.DG_OFF_EIG)
    assert np.max(np.abs(e1.cpu().numpy()[off[4]:off[5]] - ref.eigvals[:8])) < 1e-8


def test_apply_h_leading_dimensions():
    """Strided caller buffers (ldx, ldy > N_k) give the packed result, all elements
    and one element."""
    torch = need_torch_cuda()
    D = _D()
    els = W.small_slab(n_states=8)[:4]
    E = D.Elements(els)
    n_vec, N = 5, els[0].npts
    rng = np.random.default_rng(3)
    x = torch.tensor(rng.standard_normal(N * n_vec * len(els)), dtype=torch.float64, device="cuda")
    y = E.apply_H(x, n_vec)
    ldx, ldy = N + 96, N + 160
    xs = torch.full((len(els) * ldx * n_vec,), float("nan"), dtype=torch.float64, device="cuda")
    xs.view(len(els), n_vec, ldx)[:, :, :N] = x.view(len(els), n_vec, N)
    ys = torch.zeros(len(els) * ldy * n_vec, dtype=torch.float64, device="cuda")
    E.apply_H(xs, n_vec, ldx=ldx, ldy=ldy, y=ys)
    got = ys.view(len(els), n_vec, ldy)
    assert torch.equal(got[:, :, :N], y.view(len(els), n_vec, N))
    assert torch.count_nonzero(got[:, :, N:]).item() == 0       # padding untouched
    # one element, strided
    y2 = torch.zeros(ldy * n_vec, dtype=torch.float64, device="cuda")
    E.apply_H(xs[2 * ldx * n_vec:3 * ldx * n_vec].contiguous(), n_vec, elem=2, ldx=ldx, ldy=ldy, y=y2)
    assert torch.equal(y2.view(n_vec, ldy)[:, :N], y.view(len(els), n_vec, N)[2])
    with pytest.raises(D.DGError) as ex:
        E.apply_H(xs, n_vec, ldx=N - 1, ldy=ldy, y=ys)
    assert ex.value.status == D.DG_ERR_ARG


def _bump(el, centre, height, width):
    """A periodic Gaussian bump on el's grid (added to V_eff in the tests below)."""
    nx, ny, nz = el.n
    h = [el.length[a] / el.n[a] for a in range(3)]
    z, y, x = np.meshgrid(np.arange(nz) * h[2], np.arange(ny) * h[1], np.arange(nx) * h[0], indexing="ij")
    d2 = 0.0
    for coord, c, L in ((x, centre[0], el.length[0]), (y, centre[1], el.length[1]), (z, centre[2], el.length[2])):
        d = coord - c
        d -= L * np.round(d / L)
        d2 = d2 + d * d
    return (height * np.exp(-d2 / (2.0 * width * width))).ravel()


@pytest.mark.parametrize("precision", [0, 1])
def test_warm_start_after_potential_update(precision):
    """Inner SCF step: V_eff changes, the solve restarts from the previous vectors
    (with guards), reaches the oracle's eigenpairs for the new potential in fewer
    iterations than a cold start, and the ALBs follow."""
    torch = need_torch_cuda()
    D = _D()
    els = W.small_slab(n_states=8)[:4]
    print(f"[boundary] warm start, precision {precision}", flush=True)
    E = D.Elements(els)
    x0 = _x0(els, 100)
    eig0, res0, it_cold, st = E.solve(x0, precision=precision, tol=1e-9)
    assert st == 0
    rng = np.random.default_rng(21)
    new = []
    for el in els:
        c = rng.uniform(0, 1, 3) * np.array(el.length)
        new.append(dataclasses.replace(el, v_eff=el.v_eff + _bump(el, c, 0.3, 1.5)))
    v = torch.tensor(np.concatenate([e.v_eff for e in new]), dtype=torch.float64, device="cuda")
    E.set_potential(v)
    with pytest.raises(D.DGError) as ex:      # the old vectors are no solution of the new H
        E.make_alb()
    assert ex.value.status == D.DG_ERR_STATE
    eig1, res1, it_warm, st = E.solve(None, precision=precision, tol=1e-9, warm_start=True)
    assert st == 0 and res1.max().item() <= 1e-9
    E2 = D.Elements(new)
    _, _, it_cold2, st2 = E2.solve(x0, precision=precision, tol=1e-9)
    print(f"iterations: cold (old V) {it_cold.tolist()}, warm (new V) {it_warm.tolist()}, "
          f"cold (new V) {it_cold2.tolist()}")
    assert st2 == 0 and it_warm.sum() < it_cold2.sum()
    alb, sv = E.make_alb()
    off_e, off_a = E.offsets(D.DG_OFF_EIG), E.offsets(D.DG_OFF_ALB)
    A = unpack(alb.cpu().numpy(), off_a, [int(np.prod(e.elem_n)) for e in new], [8] * len(new))
    for k, el in enumerate(new):
        ref = olobpcg.lobpcg(el, W.initial_block(el.npts, 12, 7300 + k).T, 8, tol=1e-10)
        err = np.max(np.abs(eig1.cpu().numpy()[off_e[k]:off_e[k + 1]] - ref.eigvals[:8]))
        gap = ref.eigvals[8] - ref.eigvals[7]
        U_ref, s_ref = oalb.make_alb(el, ref.X, 8)
        ang = oalb.max_principal_angle(U_ref, A[k])
        print(f"elem {k}: eig err {err:.1e}, gap {gap:.2e}, ALB angle {ang:.1e}")
        assert err < 1e-8
        if gap > 1e-2:
            assert ang < 1e-6


def test_chfsi_after_raising_the_potential_maximum():
    """set_potential recomputes the filter's upper spectral bound: a potential whose
    maximum rises by 20 Ha still gets a filter interval covering the spectrum, and
    ChFSI reaches the oracle's eigenvalues (an interval ending 20 Ha below the top
    would amplify the unwanted end by ~1e3 per filter)."""
    torch = need_torch_cuda()
    D = _D()
    els = W.small_slab(n_states=8)[:2]
    new = [dataclasses.replace(el, v_eff=el.v_eff + _bump(el, (1.0, 1.0, 1.0), 20.0, 0.8)) for el in els]
    print("[boundary] ChFSI after raising max V by 20 Ha", flush=True)
    E = D.Elements(els)
    E.set_potential(torch.tensor(np.concatenate([e.v_eff for e in new]), dtype=torch.float64, device="cuda"))
    eig, res, iters, st = E.solve(_x0(els, 500), method=D.DG_CHFSI, tol=1e-9, cheb_degree=10, max_iter=200)
    assert st == 0
    off = E.offsets(D.DG_OFF_EIG)
    for k, el in enumerate(new):
        ub = ocheb.lanczos_upper_bound(lambda Y: planewave.hpsi(el, Y), el.npts)
        ref = olobpcg.lobpcg(el, W.initial_block(el.npts, 12, 7400 + k).T, 8, tol=1e-10)
        err = np.max(np.abs(eig.cpu().numpy()[off[k]:off[k + 1]] - ref.eigvals[:8]))
        print(f"elem {k}: top of spectrum (Lanczos) {ub:.2f} Ha, max V {el.v_eff.max():.2f}, "
              f"iterations {iters[k]}, eig err {err:.1e}")
        assert err < 1e-8


def test_band_energy_state_is_invalidated():
    """A backward needs its own forward: a solve or potential update in between, or a
    second forward, leaves no adjoint state for the first."""
    torch = need_torch_cuda()
    D = _D()
    els = W.small_slab(n_states=8)[:2]
    E = D.Elements(els, max_cheb_degree=4, ckpt_stride=2)
    rng = np.random.default_rng(2)
    n_vec = 3
    psi = torch.tensor(rng.standard_normal(sum(e.npts for e in els) * n_vec) * 0.01, dtype=torch.float64,
                       device="cuda")
    f = torch.ones(n_vec, dtype=torch.float64, device="cuda")
    bounds = np.array([(0.4, 95.0, -1.0)] * len(els))
    E.band_energy(psi, f, 4, bounds)
    E.solve(_x0(els, 100), tol=1e-8)
    with pytest.raises(D.DGError) as ex:
        E.band_energy_backward(np.ones(len(els)))
    assert ex.value.status == D.DG_ERR_STATE
    # a backward leaves adjoint data in the blocks: no vectors, ALBs or warm start after it
    E.band_energy(psi, f, 4, bounds)
    E.band_energy_backward(np.ones(len(els)))
    for call in (E.make_alb, E.vectors):
        with pytest.raises(D.DGError) as ex:
            call()
        assert ex.value.status == D.DG_ERR_STATE
    with pytest.raises(D.DGError) as ex:
        E.solve(None, warm_start=True)
    assert ex.value.status == D.DG_ERR_STATE
    # autograd: two forwards, then the first one's backward
    x = psi.clone().requires_grad_(True)
    out1 = D.BandEnergy.apply(None, x, E, f, 4, bounds, D.DG_FP64)
    out2 = D.BandEnergy.apply(None, x, E, f, 4, bounds, D.DG_FP64)
    with pytest.raises(RuntimeError, match="another band energy"):
        out1.sum().backward()
    out2.sum().backward()
    assert torch.isfinite(x.grad).all()
