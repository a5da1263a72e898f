"""dg_apply_H_noalloc (the entry point for callers that cannot allocate device
memory) against dg_apply_H, through the C ABI: two calls in a row, the second one
smaller, FP64 and FP32; the solver's vectors are left untouched; a call whose
projector overlaps exceed the static scratch is refused."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import need_torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 2])
def test_noalloc_matches_apply_h_on_two_calls(prec):
    torch = need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    els = W.make_config("c2").elements[:3]           # full-size elements with projectors
    print(f"[noalloc] prec {prec}: three 48x48x64 elements", flush=True)
    E = D.Elements(els)
    dt = torch.float64 if prec == D.DG_FP64 else torch.float32
    N = els[0].npts
    gen = torch.Generator(device="cuda").manual_seed(17)
    # first call: every element, 7 vectors, packed
    x1 = torch.randn(3 * N * 7, dtype=torch.float64, device="cuda", generator=gen).to(dt)
    ref1 = E.apply_H(x1, 7, prec)
    y1 = torch.full_like(x1, float("nan"))
    E.apply_H_noalloc(x1, y1, 7, prec)
    # second call, smaller: element 1 only, 3 vectors, strided buffers
    ldx, ldy = N + 64, N + 128
    x2 = torch.randn(ldx * 3, dtype=torch.float64, device="cuda", generator=gen).to(dt)
    y2 = torch.full((ldy * 3,), float("nan"), dtype=dt, device="cuda")
    ref2 = torch.zeros(ldy * 3, dtype=dt, device="cuda")
    E.apply_H(x2, 3, prec, elem=1, ldx=ldx, ldy=ldy, y=ref2)
    E.apply_H_noalloc(x2, y2, 3, prec, elem=1, ldx=ldx, ldy=ldy)
    torch.cuda.synchronize()
    tol = 1e-14 if prec == D.DG_FP64 else 1e-6
    for got, ref, tag in ((y1, ref1, "first"), (y2.view(3, ldy)[:, :N], ref2.view(3, ldy)[:, :N], "second")):
        err = ((got.double() - ref.double()).abs().max() / ref.double().abs().max()).item()
        print(f"[noalloc] prec {prec} {tag} call: max relative difference {err:.1e}", flush=True)
        assert err <= tol
    assert torch.isnan(y2.view(3, ldy)[:, N:]).all()        # padding untouched


def test_noalloc_leaves_the_solver_state():
    torch = need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    els = W.small_slab(n_states=8)[:3]
    E = D.Elements(els)
    x0 = torch.tensor(D.pack_initial(els, 100), dtype=torch.float64, device="cuda")
    eig, res, iters, st = E.solve(x0, tol=1e-9)
    assert st == 0
    X0 = E.vectors()
    x = torch.randn(sum(e.npts for e in els) * 5, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    E.apply_H_noalloc(x, y, 5)
    assert torch.equal(E.vectors(), X0)
    alb, sv = E.make_alb()                   # the solution is still there
    assert torch.isfinite(sv).all()


def test_noalloc_refuses_scratch_overflow():
    """Sixty 16^3 elements with J = 80 (88 vectors) and 480 one-point projectors each:
    60 x 480 x 88 overlaps exceed the 2^21 FP64 values of the static scratch; one
    element per call fits and matches dg_apply_H."""
    torch = need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    base = W.make_config("c1").elements[0]
    n_p = 480
    idx = np.sort((np.arange(n_p) * 7919) % base.npts)
    el = dataclasses.replace(base, n_states=80, proj_ptr=np.arange(n_p + 1, dtype=np.int64),
                             proj_idx=idx.astype(np.int32), proj_val=np.full(n_p, 0.1), gamma=np.full(n_p, 0.01))
    els = [el] * 60
    print("[noalloc] 60 elements x 480 projectors x 88 vectors", flush=True)
    E = D.Elements(els, n_streams=1)
    K = 80 + W.guard_count(80)
    x = torch.randn(60 * base.npts * K, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(D.DGError) as ex:
        E.apply_H_noalloc(x, y, K)
    assert ex.value.status == D.DG_ERR_ARG and "static scratch" in str(ex.value)
    xe = x[:base.npts * K].contiguous()
    ye = torch.empty_like(xe)
    E.apply_H_noalloc(xe, ye, K, elem=4)
    ref = E.apply_H(xe, K, elem=4)
    assert ((ye - ref).abs().max() / ref.abs().max()).item() <= 1e-14
