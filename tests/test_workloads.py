"""Seeded input generator: determinism, geometry and projector sanity."""
import numpy as np

import workloads as W


def test_c1_deterministic():
    a = W.make_config("c1").elements[0]
    b = W.make_config("c1").elements[0]
    assert np.array_equal(a.v_eff, b.v_eff)
    assert a.n == (16, 16, 16) and a.n_proj == 0 and a.n_states == 8
    assert a.v_eff.min() < -2.0 and a.v_eff.max() < 0.0


def test_honeycomb_bond_lengths():
    s = W.honeycomb_sites(25.6, 25.6, 12.8)
    assert 60 <= len(s) <= 90
    d = s[:, None, :2] - s[None, :, :2]
    d -= 25.6 * np.round(d / 25.6)
    r = np.sqrt((d ** 2).sum(-1)) + np.eye(len(s)) * 1e9
    assert r.min() >= 1.0
    # bulk sites have three neighbours at the C-C distance
    nn = (np.abs(r - W.CC_BOND) < 1e-9).sum(1)
    assert np.median(nn) == 3


def test_slab_elements_geometry_and_projectors():
    els = W.small_slab()
    assert len(els) == 9
    for el in els:
        assert el.n == (16, 16, 32)
        assert el.elem_lo == (4, 4, 0) and el.elem_n == (8, 8, 32)
        assert el.v_eff.shape == (el.npts,)
        assert el.proj_ptr[0] == 0 and el.proj_ptr[-1] == el.proj_idx.size
        assert el.n_proj == 4 * el.n_atoms
        for p in range(el.n_proj):
            idx = el.proj_idx[el.proj_ptr[p]:el.proj_ptr[p + 1]]
            assert np.all(np.diff(idx) > 0)
            assert idx.min() >= 0 and idx.max() < el.npts
        assert np.all(el.gamma > 0)
    # element restriction indices cover E_k exactly once
    idx = els[0].elem_indices()
    assert len(np.unique(idx)) == 8 * 8 * 32


def test_projectors_unit_norm_on_global_grid_and_restricted():
    els = W.small_slab()
    norms = []
    for el in els:
        for p in range(el.n_proj):
            v = el.proj_val[el.proj_ptr[p]:el.proj_ptr[p + 1]]
            norms.append(np.linalg.norm(v))
    norms = np.array(norms)
    assert norms.max() <= 1.0 + 1e-12
    assert np.isclose(norms.max(), 1.0)


def test_c4_uneven_shapes_and_vacancies():
    rng = np.random.default_rng(4)
    q = rng.choice([32, 48, 64], size=256)
    js = rng.integers(20, 81, size=256)
    assert set(q.tolist()) == {32, 48, 64}
    assert js.min() >= 20 and js.max() <= 80


def test_initial_block_seeded():
    a = W.initial_block(100, 5, seed=3)
    b = W.initial_block(100, 5, seed=3)
    assert a.shape == (5, 100) and np.array_equal(a, b)
    assert W.guard_count(40) == 8 and W.guard_count(60) == 12 and W.guard_count(8) == 4
    assert W.guard_count(80) == 8 and W.guard_count(84) == 4   # J + guards <= 88
