"""H*psi on the GPU (dg_apply_H) against the oracle's plane-wave H (Eq. (1)), element by element."""
import dataclasses
import sys

import numpy as np
import pytest

import workloads as W
from oracle import planewave
from tests.gpu_util import need_torch_cuda, rel_err

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12   # relative to max |H x|; FFT rounding ~ eps log N
FP32_TOL = 5e-6


def _run(els, n_vec, prec, seed=1, elem=-1):
    torch = need_torch_cuda()
    from paper_2003_00407_amd import dgalb as D
    print(f"[hpsi] grids={[e.n for e in els]} n_vec={n_vec} prec={prec} elem={elem}", flush=True)
    E = D.Elements(els)
    rng = np.random.default_rng(seed)
    use = [k for k in range(len(els)) if elem < 0 or k == elem]
    xs = [rng.standard_normal((n_vec, els[k].npts)) for k in use]
    dt = torch.float64 if prec == D.DG_FP64 else torch.float32
    x = torch.tensor(np.concatenate([a.ravel() for a in xs]), dtype=dt, device="cuda")
    y = E.apply_H(x, n_vec, prec, elem=elem)
    torch.cuda.synchronize()
    yh = y.double().cpu().numpy()
    errs = []
    off = 0
    for i, k in enumerate(use):
        n = els[k].npts
        X = xs[i].T
        if prec == D.DG_FP32:
            X = X.astype(np.float32).astype(np.float64)
        ref = planewave.hpsi(els[k], X)
        got = yh[off:off + n * n_vec].reshape(n_vec, n).T
        off += n * n_vec
        errs.append(rel_err(got, ref))
    return max(errs)


def test_hpsi_c1_fp64_odd_ncols():
    assert _run(W.make_config("c1").elements, 5, 0) < FP64_TOL


def test_hpsi_slab_batch_fp64():
    assert _run(W.small_slab(), 12, 0) < FP64_TOL


def test_hpsi_slab_batch_fp32():
    assert _run(W.small_slab(), 12, 2) < FP32_TOL


def test_hpsi_single_element_mode():
    assert _run(W.small_slab(), 7, 0, elem=4) < FP64_TOL


@pytest.mark.parametrize("n", [(8, 8, 64), (12, 12, 24), (24, 24, 12), (32, 32, 48), (64, 64, 16)])
def test_hpsi_line_lengths(n):
    """Every supported line length (radix 2, 3, 4 paths), with wells, FP64 and FP32."""
    L = tuple(0.45 * x for x in n)
    rng = np.random.default_rng(sum(n))
    el = W._box_element(n, L, rng.uniform(0, 1, (3, 3)) * np.array(L), 4)
    assert _run([el], 3, 0) < FP64_TOL
    assert _run([el], 3, 2) < FP32_TOL


def test_hpsi_c2_full_size_elements_fp64():
    """Two elements of the 4x4 slab at full size (48x48x64, projectors)."""
    els = W.make_config("c2").elements[:2]
    assert _run(els, 4, 0) < FP64_TOL
    assert _run(els, 4, 2) < FP32_TOL
