"""Chebyshev filter on the GPU: ChFSI solves, band energy and its adjoint gradient."""
import numpy as np
import pytest

import workloads as W
from oracle import band_energy as obe
from oracle import chebyshev as ocheb
from oracle import lobpcg as olobpcg
from tests.gpu_util import need_torch_cuda, rel_err, unpack

pytestmark = pytest.mark.gpu


def test_chfsi_slab_vs_oracle():
    torch = need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    els = W.small_slab(n_states=8)[:4]
    print(f"[chfsi] n_elem={len(els)} grid={els[0].n}", flush=True)
    E = D.Elements(els)
    x0 = torch.tensor(D.pack_initial(els, 500), dtype=torch.float64, device="cuda")
    eig, res, iters, st = E.solve(x0, method=D.DG_CHFSI, tol=1e-9, cheb_degree=10, max_iter=200)
    assert st == 0
    off = E.offsets(D.DG_OFF_EIG)
    eig = eig.cpu().numpy()
    for k, el in enumerate(els):
        ref = olobpcg.lobpcg(el, W.initial_block(el.npts, 12, 7200 + k).T, 8, tol=1e-10)
        err = np.max(np.abs(eig[off[k]:off[k + 1]] - ref.eigvals[:8]))
        print(f"chfsi elem {k}: iters {iters[k]} err {err:.2e}")
        assert err < 1e-8


def _be_case(els, seed=0):
    """psi0 blocks, weights and filter bounds (a, b, a0) per element."""
    rng = np.random.default_rng(seed)
    n_vec = 6
    psi = [rng.standard_normal((e.npts, n_vec)) / np.sqrt(e.npts) for e in els]
    f = rng.uniform(0.0, 2.0, n_vec)
    bounds = []
    for e in els:
        from oracle.planewave import hpsi
        b = ocheb.lanczos_upper_bound(lambda Y: hpsi(e, Y), e.npts)
        bounds.append((0.4, b, float(e.v_eff.min())))
    return psi, f, bounds


def _gpu_be(E, psi, f, degree, bounds, prec, dE=None):
    torch = need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    dt = torch.float64 if prec == D.DG_FP64 else torch.float32
    x = torch.tensor(np.concatenate([p.T.ravel() for p in psi]), dtype=dt, device="cuda")
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    Ev = E.band_energy(x, ft, degree, np.array(bounds), prec).cpu().numpy()
    if dE is None:
        return Ev
    dpsi, dv = E.band_energy_backward(dE)
    return Ev, dpsi.double().cpu().numpy(), dv.cpu().numpy()


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (2, 2e-4)])
def test_band_energy_and_gradient_vs_oracle(prec, tol):
    need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    els = W.small_slab(n_states=8)[:2]
    degree = 6
    print(f"[band energy] prec={prec} degree={degree}", flush=True)
    E = D.Elements(els, max_cheb_degree=degree, ckpt_stride=2)
    psi, f, bounds = _be_case(els)
    Ev, dpsi, dv = _gpu_be(E, psi, f, degree, bounds, prec, dE=np.ones(len(els)))
    offg = E.offsets(D.DG_OFF_GRID)
    off = 0
    for k, el in enumerate(els):
        a, b, a0 = bounds[k]
        Er, gp, gv = obe.band_energy_grad(el, el.v_eff, psi[k], f, degree, a, b, a0)
        n = el.npts * len(f)
        gp_gpu = dpsi[off:off + n].reshape(len(f), el.npts).T
        off += n
        e1, e2, e3 = abs(Ev[k] - Er) / abs(Er), rel_err(gp_gpu, gp), rel_err(dv[offg[k]:offg[k + 1]], gv)
        print(f"elem {k}: E rel {e1:.1e} dpsi rel {e2:.1e} dV rel {e3:.1e}")
        assert e1 < tol and e2 < tol * 10 and e3 < tol * 10


def test_checkpointed_equals_stored():
    """Segment recomputation (stride 4) gives the gradient of the stride-1 (all stored) run."""
    need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    els = W.small_slab(n_states=8)[:2]
    degree = 9
    psi, f, bounds = _be_case(els, seed=3)
    outs = []
    for stride in (1, 4):
        E = D.Elements(els, max_cheb_degree=degree, ckpt_stride=stride)
        outs.append(_gpu_be(E, psi, f, degree, bounds, 0, dE=np.array([1.0, -0.5])))
    assert rel_err(outs[1][0], outs[0][0]) < 1e-14
    assert rel_err(outs[1][1], outs[0][1]) < 1e-12
    assert rel_err(outs[1][2], outs[0][2]) < 1e-12


def test_c5_finite_differences_and_oracle_gradient():
    """C5: the 4x4 slab, degree-16 filter: oracle gradient at full size, and central
    differences (h = 1e-4) on 32 seeded directions each for Psi_0 and V."""
    torch = need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    cfg = W.make_config("c5")
    els = cfg.elements
    degree, n_dir = 16, 32
    E = D.Elements(els, max_cheb_degree=degree, ckpt_stride=4)
    rng = np.random.default_rng(5)
    n_vec = 6
    psi = [rng.standard_normal((e.npts, n_vec)) / np.sqrt(e.npts) for e in els]
    f = rng.uniform(0.0, 2.0, n_vec)
    # a above the wanted states, b above the top of the spectrum (kinetic maximum ~92.5 Ha)
    bounds = [(0.2, 95.0, float(e.v_eff.min())) for e in els]
    print("[c5] forward + backward", flush=True)
    E0, dpsi, dv = _gpu_be(E, psi, f, degree, bounds, 0, dE=np.ones(len(els)))
    # the oracle's stored-intermediate adjoint on one full-size element
    a, b, a0 = bounds[0]
    Er, gp, gv = obe.band_energy_grad(els[0], els[0].v_eff, psi[0], f, degree, a, b, a0)
    n0 = els[0].npts
    e1 = abs(E0[0] - Er) / abs(Er)
    e2 = rel_err(dpsi[:n0 * n_vec].reshape(n_vec, n0).T, gp)
    e3 = rel_err(dv[:n0], gv)
    print(f"C5 element 0 vs oracle: E {e1:.1e} dPsi {e2:.1e} dV {e3:.1e}")
    assert e1 < 1e-12 and e2 < 1e-11 and e3 < 1e-11
    h = 1e-4
    x = np.concatenate([p.T.ravel() for p in psi])
    v0 = np.concatenate([e.v_eff for e in els])
    worst_psi = worst_v = 0.0          # |FD - <grad, d>| / ||grad||  (unit d)
    proj_psi = proj_v = 0.0            # |FD - <grad, d>| / |<grad, d>| (reported)
    gn_psi, gn_v = np.linalg.norm(dpsi), np.linalg.norm(dv)
    for _ in range(n_dir):
        d = rng.standard_normal(x.size)
        d /= np.linalg.norm(d)
        ep = _gpu_be(E, _split(x + h * d, els, n_vec), f, degree, bounds, 0)
        em = _gpu_be(E, _split(x - h * d, els, n_vec), f, degree, bounds, 0)
        an = float(dpsi @ d)
        err = abs((ep.sum() - em.sum()) / (2 * h) - an)
        worst_psi = max(worst_psi, err / gn_psi)
        proj_psi = max(proj_psi, err / max(abs(an), 1e-30))
    for _ in range(n_dir):
        d = rng.standard_normal(v0.size)
        d /= np.linalg.norm(d)
        E.set_potential(torch.tensor(v0 + h * d, dtype=torch.float64, device="cuda"))
        ep = _gpu_be(E, psi, f, degree, bounds, 0)
        E.set_potential(torch.tensor(v0 - h * d, dtype=torch.float64, device="cuda"))
        em = _gpu_be(E, psi, f, degree, bounds, 0)
        an = float(dv @ d)
        err = abs((ep.sum() - em.sum()) / (2 * h) - an)
        worst_v = max(worst_v, err / gn_v)
        proj_v = max(proj_v, err / max(abs(an), 1e-30))
    E.set_potential(torch.tensor(v0, dtype=torch.float64, device="cuda"))
    print(f"C5 FD over {n_dir} directions: |FD-<g,d>|/||g||: Psi_0 {worst_psi:.1e}, V {worst_v:.1e}; "
          f"relative to |<g,d>|: Psi_0 {proj_psi:.1e}, V {proj_v:.1e}")
    # E is quadratic in Psi_0 (central differences exact up to rounding); in V a unit
    # direction moves each grid value by ~1e-4/sqrt(2.4e6), near the FP64 rounding of
    # 16 H*psi applications, which bounds how well FD can resolve <g, d>
    assert worst_psi < 1e-9
    assert worst_v < 1e-6


def _split(x, els, n_vec):
    out, o = [], 0
    for e in els:
        out.append(x[o:o + e.npts * n_vec].reshape(n_vec, e.npts).T)
        o += e.npts * n_vec
    return out


def test_autograd_function():
    torch = need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    els = W.small_slab(n_states=8)[:2]
    degree = 5
    E = D.Elements(els, max_cheb_degree=degree, ckpt_stride=2)
    psi, f, bounds = _be_case(els, seed=9)
    x = torch.tensor(np.concatenate([p.T.ravel() for p in psi]), dtype=torch.float64, device="cuda",
                     requires_grad=True)
    v = torch.tensor(np.concatenate([e.v_eff for e in els]), dtype=torch.float64, device="cuda",
                     requires_grad=True)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    out = D.BandEnergy.apply(v, x, E, ft, degree, np.array(bounds), D.DG_FP64)
    (out * torch.tensor([1.0, 2.0], dtype=torch.float64, device="cuda")).sum().backward()
    Ev, dpsi, dv = _gpu_be(E, psi, f, degree, bounds, 0, dE=np.array([1.0, 2.0]))
    assert rel_err(x.grad.cpu().numpy(), dpsi) < 1e-13
    assert rel_err(v.grad.cpu().numpy(), dv) < 1e-13
