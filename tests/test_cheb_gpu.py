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


def _gpu_be_packed(E, x, f, degree, bounds):
    """FP64 band energies for a packed device Psi_0 (no host copies)."""
    torch = need_torch_cuda()
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    return E.band_energy(x.contiguous(), ft, degree, np.array(bounds), 0).cpu().numpy()


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


def _atom_bump(el, centre, width=1.2):
    """Unit-norm Gaussian bump on el's grid around centre (a direction in V)."""
    nx, ny, nz = el.n
    h = [el.length[a] / el.n[a] for a in range(3)]
    z, y, x = np.meshgrid(np.arange(nz) * h[2], np.arange(ny) * h[1], np.arange(nx) * h[0], indexing="ij")
    d2 = 0.0
    for coord, c, L in ((x, centre[0], el.length[0]), (y, centre[1], el.length[1]), (z, centre[2], el.length[2])):
        dd = coord - c
        dd -= L * np.round(dd / L)
        d2 = d2 + dd * dd
    v = np.exp(-d2 / (2.0 * width * width)).ravel()
    return v / np.linalg.norm(v)


def test_c5_as_configured():
    """C5: the 4x4 slab; Psi_0 = the converged C2 eigenvectors (J = 40 per element),
    degree-16 filter with bounds from the Ritz values (a = highest kept Ritz value,
    a0 = lowest) and the spectral upper bound b (Lanczos); f = 1 and f ~ U[0, 2].
    The GPU band energy and both gradients against the oracle's stored-intermediate
    adjoint on a full-size element (FP64, and FP32 at the tolerance its rounding
    allows), then central differences on 32 seeded directions each for Psi_0 and V
    in FP64, relative to <g, d>."""
    torch = need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    from oracle.planewave import hpsi
    cfg = W.make_config("c5")
    els = cfg.elements
    degree, n_dir, J = 16, 32, 40
    E = D.Elements(els, max_cheb_degree=degree, ckpt_stride=4)
    x0 = torch.tensor(D.pack_initial(els, cfg.x0_seed_base), dtype=torch.float64, device="cuda")
    eig, res, iters, st = E.solve(x0, tol=1e-8)
    assert st == 0
    th, _ = E.ritz()
    th = th.cpu().numpy()
    offk = E.offsets(D.DG_OFF_KALL)
    psi_t = E.vectors()                                       # packed N x J per element, FP64
    psi = [psi_t[o0:o1].cpu().numpy().reshape(J, e.npts).T
           for e, o0, o1 in zip(els, E.offsets(D.DG_OFF_VEC)[:-1], E.offsets(D.DG_OFF_VEC)[1:])]
    bounds = []
    for k, el in enumerate(els):
        b = ocheb.lanczos_upper_bound(lambda Y: hpsi(el, Y), el.npts)
        bounds.append((float(th[offk[k + 1] - 1]), b, float(th[offk[k]])))
    print(f"[c5] bounds element 0: a {bounds[0][0]:.4f} b {bounds[0][1]:.2f} a0 {bounds[0][2]:.4f}", flush=True)
    rng = np.random.default_rng(5)
    fs = {"ones": np.ones(J), "U[0,2]": rng.uniform(0.0, 2.0, J)}
    n0 = els[0].npts
    for name, f in fs.items():
        a, b, a0 = bounds[0]
        Er, gp, gv = obe.band_energy_grad(els[0], els[0].v_eff, psi[0], f, degree, a, b, a0)
        for prec, tol in ((0, 1e-11), (2, 2e-6)):
            Ev, dpsi, dv = _gpu_be(E, psi, f, degree, bounds, prec, dE=np.ones(len(els)))
            e1 = abs(Ev[0] - Er) / abs(Er)
            e2 = rel_err(dpsi[:n0 * J].reshape(J, n0).T, gp)
            e3 = rel_err(dv[:n0], gv)
            print(f"[c5] f={name} prec={prec}: element 0 vs oracle: E {e1:.1e} dPsi {e2:.1e} dV {e3:.1e}",
                  flush=True)
            assert e1 < tol and e2 < tol and e3 < tol
    # central differences, FP64, f ~ U[0, 2]
    f = fs["U[0,2]"]
    E0, dpsi, dv = _gpu_be(E, psi, f, degree, bounds, 0, dE=np.ones(len(els)))
    # Psi_0: E is quadratic in Psi_0, so a central difference is exact up to rounding
    # for any step; h = 0.05 keeps the rounding of E / h small
    h = 0.05
    x = psi_t                                                 # packed device Psi_0
    dpsi_t = torch.tensor(dpsi, dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(5)
    worst_psi = 0.0
    for _ in range(n_dir):
        d = torch.randn(x.numel(), dtype=torch.float64, device="cuda", generator=gen)
        d /= torch.linalg.norm(d)
        ep = _gpu_be_packed(E, x + h * d, f, degree, bounds)
        em = _gpu_be_packed(E, x - h * d, f, degree, bounds)
        an = float(torch.dot(dpsi_t, d).item())
        worst_psi = max(worst_psi, abs((ep.sum() - em.sum()) / (2 * h) - an) / abs(an))
    # V: unit Gaussian bumps (width 1.2 bohr) centred on seeded atom sites of seeded
    # elements, where the gradient (a density) is large; E is a polynomial in V, so
    # Richardson extrapolation of steps h and h/2 removes the O(h^2) term
    v0 = np.concatenate([e.v_eff for e in els])
    offg = E.offsets(D.DG_OFF_GRID)
    worst_v = 0.0

    def e_at(vv):
        E.set_potential(torch.tensor(vv, dtype=torch.float64, device="cuda"))
        return _gpu_be(E, psi, f, degree, bounds, 0).sum()

    for _ in range(n_dir):
        k = int(rng.integers(len(els)))
        el = els[k]
        # atom centres of element k are not stored; centre the bump on its strongest well
        # (a grid point of lowest V) shifted by a seeded offset of up to 1 bohr
        i = int(np.argmin(el.v_eff + 1e-3 * rng.standard_normal(el.npts)))
        ix, iy, iz = i % el.n[0], (i // el.n[0]) % el.n[1], i // (el.n[0] * el.n[1])
        hx = [el.length[a] / el.n[a] for a in range(3)]
        c = np.array([ix * hx[0], iy * hx[1], iz * hx[2]]) + rng.uniform(-1.0, 1.0, 3)
        d = np.zeros_like(v0)
        d[offg[k]:offg[k + 1]] = _atom_bump(el, c)
        hv = 2e-4
        fd1 = (e_at(v0 + hv * d) - e_at(v0 - hv * d)) / (2 * hv)
        fd2 = (e_at(v0 + 0.5 * hv * d) - e_at(v0 - 0.5 * hv * d)) / hv
        fd = (4.0 * fd2 - fd1) / 3.0
        an = float(dv @ d)
        worst_v = max(worst_v, abs(fd - an) / abs(an))
    E.set_potential(torch.tensor(v0, dtype=torch.float64, device="cuda"))
    print(f"[c5] central differences over {n_dir} directions, |FD - <g,d>| / |<g,d>|: "
          f"Psi_0 {worst_psi:.1e}, V {worst_v:.1e}", flush=True)
    assert worst_psi < 1e-6
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
