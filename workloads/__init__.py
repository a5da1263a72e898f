"""Seeded synthetic inputs for the batched adaptive-local-basis (ALB) eigensolves.

This module builds *inputs only*: grids, a local potential on each extended
element, nonlocal projector vectors, element sub-boxes and seeded initial
blocks.  It contains none of the solver's arithmetic (no Hamiltonian
application, no eigensolver, no orthonormalisation) and is imported by both
the CPU oracle and the GPU binding, which otherwise share no code.

Physical model (stand-in for the paper's graphene systems, whose coordinates
and pseudopotential tables are not available):

* Global periodic domain split into a 2D mesh of elements E_k; each extended
  element Q_k is E_k plus a buffer of neighbouring elements (paper Sec. 2.A and
  the ALB-generation subsection, Fig. 1: a 3x3 block of elements around E_k).
* Local potential V_eff = sum of Gaussian wells, one per site, depth -2 Ha,
  width sigma = 1 bohr, summed over periodic images (the restriction of the
  global periodic array to Q_k, as in Eq. (1)'s V_eff^{Q_k}).
* Nonlocal part V_nl = sum_{I,l} gamma_{I,l} |b_{I,l}><b_{I,l}| (Eq. (1)):
  four projectors per site, one s-like exp(-r^2/2 s^2) and three p-like
  r_a exp(-r^2/2 s^2), s = 0.7 bohr, truncated at r_c = 4 bohr, normalised to
  unit Euclidean norm on the global grid, then restricted to Q_k.
  gamma_s = 1.0 Ha, gamma_p = 0.5 Ha.
* Honeycomb sites with C-C distance 2.68 bohr in the plane z = L_z / 2.
* Grid spacing 0.4 bohr (E_cut = pi^2 / (2 h^2) ~ 30.8 Ha by the paper's grid
  rule (N_r)_i = sqrt(2 E_cut) L_i / pi, Sec. 3 before Table 1).

Grid vectors are flattened with x fastest: index = x + nx * (y + ny * z);
numpy arrays are shaped (nz, ny, nx).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Element", "Config", "make_config", "initial_block", "CONFIG_NAMES",
    "guard_count", "honeycomb_sites", "free_electron_element", "Mesh", "small_slab_with_mesh",
]

CC_BOND = 2.68          # bohr
H_SPACING = 0.4         # bohr
WELL_DEPTH = -2.0       # Ha
WELL_WIDTH = 1.0        # bohr (Gaussian sigma)
PROJ_SIGMA = 0.7        # bohr
PROJ_RCUT = 4.0         # bohr
GAMMA_S = 1.0           # Ha
GAMMA_P = 0.5           # Ha
WELL_RCUT = 9.0         # bohr; exp(-81/2) ~ 2.6e-18 relative truncation


@dataclasses.dataclass
class Element:
    """One extended element Q_k with its central element E_k (host arrays).

    v_eff      float64[N]      local potential on Q_k's grid (Ha), x fastest
    proj_ptr   int64[n_proj+1] CSR-by-projector offsets into proj_idx/proj_val
    proj_idx   int32[nnz]      grid indices (ascending within a projector)
    proj_val   float64[nnz]    projector values b_{I,l}(r)
    gamma      float64[n_proj] projector weights (Ha)
    """
    n: Tuple[int, int, int]
    length: Tuple[float, float, float]
    elem_lo: Tuple[int, int, int]
    elem_n: Tuple[int, int, int]
    n_states: int
    v_eff: np.ndarray
    proj_ptr: np.ndarray
    proj_idx: np.ndarray
    proj_val: np.ndarray
    gamma: np.ndarray
    n_atoms: int = 0
    # global layout (slab workloads): Q_k's first grid point in the global grid (may be
    # negative: the global grid is periodic) and a global id per projector (the same
    # projector restricted to several extended elements carries the same id)
    q_lo: Tuple[int, int, int] = (0, 0, 0)
    proj_gid: Optional[np.ndarray] = None

    @property
    def npts(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def n_proj(self) -> int:
        return int(self.gamma.shape[0])

    def elem_indices(self) -> np.ndarray:
        """Flat Q_k grid indices of E_k's points, in E_k's own x-fastest order."""
        nx, ny, _ = self.n
        lo, en = self.elem_lo, self.elem_n
        z, y, x = np.meshgrid(np.arange(lo[2], lo[2] + en[2]),
                              np.arange(lo[1], lo[1] + en[1]),
                              np.arange(lo[0], lo[0] + en[0]), indexing="ij")
        return (x + nx * (y + ny * z)).ravel().astype(np.int64)

    def projector_matrix(self):
        """Projectors as a scipy.sparse CSC matrix B (N x n_proj)."""
        import scipy.sparse as sp
        return sp.csc_matrix((self.proj_val, self.proj_idx.astype(np.int64), self.proj_ptr),
                             shape=(self.npts, self.n_proj))


@dataclasses.dataclass
class Mesh:
    """The 2D element mesh of a slab: element k = (k % n_mesh, k // n_mesh) covers the
    global grid points [ex*elem_pts, (ex+1)*elem_pts) x [ey*elem_pts, ...) x all of z
    (DG elements E_k; each has four faces, shared with its x and y neighbours)."""
    n_mesh: int
    elem_pts: int
    global_n: Tuple[int, int, int]
    length: Tuple[float, float, float]
    v_global: Optional[np.ndarray] = None     # V_eff on the global grid (flat, x fastest)
    atoms: Optional[list] = None              # per site: (ascending global flat indices, 4 x len values)

    @property
    def n_elem(self) -> int:
        return self.n_mesh * self.n_mesh

    @property
    def elem_npts(self) -> int:
        return self.elem_pts * self.elem_pts * self.global_n[2]

    def elem_global_indices(self, k: int) -> np.ndarray:
        """Global flat indices of E_k's points in E_k's own x-fastest order."""
        gx, gy, gz = self.global_n
        ox, oy, _ = self.origin(k)
        z, y, x = np.meshgrid(np.arange(gz), np.arange(oy, oy + self.elem_pts),
                              np.arange(ox, ox + self.elem_pts), indexing="ij")
        return (x + gx * (y + gy * z)).ravel().astype(np.int64)

    def elem_projectors(self, k: int):
        """Every projector with support on E_k, restricted to E_k: (global ids int32,
        CSR pointer int64, E_k-local indices int32, values float64, gamma float64).
        Projector 4a + p is site a's s (p = 0) or p_x, p_y, p_z (p = 1, 2, 3) function."""
        gidx = self.elem_global_indices(k)
        loc = {int(g): i for i, g in enumerate(gidx)}
        gids, ptr, idx, val, gam = [], [0], [], [], []
        for a, (ai, av) in enumerate(self.atoms):
            hit = [(loc[int(g)], t) for t, g in enumerate(ai) if int(g) in loc]
            if not hit:
                continue
            hit.sort()
            li = np.array([h[0] for h in hit], dtype=np.int32)
            ti = np.array([h[1] for h in hit], dtype=np.int64)
            for p in range(4):
                gids.append(4 * a + p)
                idx.append(li)
                val.append(av[p][ti])
                gam.append(GAMMA_S if p == 0 else GAMMA_P)
                ptr.append(ptr[-1] + len(li))
        return (np.array(gids, dtype=np.int32), np.array(ptr, dtype=np.int64),
                np.concatenate(idx).astype(np.int32) if idx else np.zeros(0, np.int32),
                np.concatenate(val) if val else np.zeros(0), np.array(gam, dtype=np.float64))

    def origin(self, k: int) -> Tuple[int, int, int]:
        return ((k % self.n_mesh) * self.elem_pts, (k // self.n_mesh) * self.elem_pts, 0)

    def neighbours(self, k: int) -> Tuple[int, int, int, int]:
        """Elements across the x-, x+, y-, y+ faces (periodic)."""
        m = self.n_mesh
        ex, ey = k % m, k // m
        return (((ex - 1) % m) + m * ey, ((ex + 1) % m) + m * ey,
                ex + m * ((ey - 1) % m), ex + m * ((ey + 1) % m))


@dataclasses.dataclass
class Config:
    name: str
    elements: List[Element]
    description: str
    x0_seed_base: int
    method: str = "lobpcg"
    precision: str = "fp64"
    mesh: Optional[Mesh] = None

    @property
    def n_elem(self) -> int:
        return len(self.elements)


def guard_count(j: int) -> int:
    """Number of guard states carried above the J wanted ones: a fifth of J (at least
    4), fewer where J + guards would pass the solver's 88 columns."""
    g = max(4, int(math.ceil(0.2 * j)))
    return g if j + g <= 88 else max(4, 88 - j)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def honeycomb_sites(lx: float, ly: float, z0: float, bond: float = CC_BOND,
                    min_sep: float = 1.0) -> np.ndarray:
    """Honeycomb lattice points wrapped into [0,lx) x [0,ly), seam duplicates removed.

    a = sqrt(3) * bond; a1 = (a, 0); a2 = (a/2, a sqrt(3)/2); basis (0,0) and
    (a/2, bond/2).  The lattice is generally incommensurate with the box: sites
    are wrapped modulo the box and any site closer than ``min_sep`` (minimum
    image) to an earlier one is dropped, deterministically.
    """
    a = math.sqrt(3.0) * bond
    a1 = np.array([a, 0.0])
    a2 = np.array([a / 2.0, a * math.sqrt(3.0) / 2.0])
    basis = [np.array([0.0, 0.0]), np.array([a / 2.0, bond / 2.0])]
    nmax = int(math.ceil(2 * max(lx, ly) / a)) + 2
    pts = []
    for j in range(-nmax, nmax + 1):
        for i in range(-nmax, nmax + 1):
            for b in basis:
                p = i * a1 + j * a2 + b
                if 0.0 <= p[0] < lx and 0.0 <= p[1] < ly:
                    pts.append(p)
    pts = np.array(pts)
    order = np.lexsort((pts[:, 0], pts[:, 1]))
    pts = pts[order]
    kept: List[np.ndarray] = []
    for p in pts:
        ok = True
        for q in kept:
            d = p - q
            d[0] -= lx * round(d[0] / lx)
            d[1] -= ly * round(d[1] / ly)
            if math.hypot(d[0], d[1]) < min_sep:
                ok = False
                break
        if ok:
            kept.append(p)
    xy = np.array(kept)
    return np.column_stack([xy, np.full(len(xy), z0)])


def _local_box(center: np.ndarray, h: Sequence[float], ng: Sequence[int], rcut: float):
    """Grid offsets (unwrapped ints per axis) of the box of half-width rcut around center."""
    rng_axes = []
    for a in range(3):
        lo = int(math.ceil((center[a] - rcut) / h[a]))
        hi = int(math.floor((center[a] + rcut) / h[a]))
        rng_axes.append(np.arange(lo, hi + 1))
    return rng_axes


def _gaussian_wells(ng: Tuple[int, int, int], length: Tuple[float, float, float],
                    sites: np.ndarray, depth: float, width: float,
                    rcut: float = WELL_RCUT) -> np.ndarray:
    """Sum of Gaussian wells over all periodic images within rcut; returns (nz,ny,nx)."""
    nx, ny, nz = ng
    h = [length[0] / nx, length[1] / ny, length[2] / nz]
    out = np.zeros(nx * ny * nz)
    for c in sites:
        ax, ay, az = _local_box(c, h, ng, rcut)
        dx = ax * h[0] - c[0]
        dy = ay * h[1] - c[1]
        dz = az * h[2] - c[2]
        r2 = (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
        val = depth * np.exp(-r2 / (2.0 * width * width))
        idx = ((ax % nx)[None, None, :] + nx * ((ay % ny)[None, :, None]
               + ny * (az % nz)[:, None, None]))
        out += np.bincount(idx.ravel(), weights=val.ravel(), minlength=out.size)
    return out.reshape(nz, ny, nx)


def _atom_projectors(ng, length, center, sigma=PROJ_SIGMA, rcut=PROJ_RCUT):
    """Global flat indices (ascending) and the 4 normalised projector values for one site."""
    nx, ny, nz = ng
    h = [length[0] / nx, length[1] / ny, length[2] / nz]
    ax, ay, az = _local_box(center, h, ng, rcut)
    dx = ax * h[0] - center[0]
    dy = ay * h[1] - center[1]
    dz = az * h[2] - center[2]
    DZ, DY, DX = np.meshgrid(dz, dy, dx, indexing="ij")
    r2 = DX ** 2 + DY ** 2 + DZ ** 2
    mask = r2 <= rcut * rcut
    IZ, IY, IX = np.meshgrid(az % nz, ay % ny, ax % nx, indexing="ij")
    idx = (IX + nx * (IY + ny * IZ))[mask]
    g = np.exp(-r2[mask] / (2.0 * sigma * sigma))
    vals = np.stack([g, DX[mask] * g, DY[mask] * g, DZ[mask] * g])
    if len(np.unique(idx)) != len(idx):
        raise ValueError("projector support wraps onto itself: box too small for r_c")
    order = np.argsort(idx)
    idx = idx[order]
    vals = vals[:, order]
    vals /= np.linalg.norm(vals, axis=1, keepdims=True)
    return idx.astype(np.int64), vals


def _restrict(global_flat_idx: np.ndarray, ng, q_lo, q_n):
    """Map global flat indices into Q's local flat indices; returns (keep_mask, local_idx)."""
    nx, ny, nz = ng
    gx = global_flat_idx % nx
    gy = (global_flat_idx // nx) % ny
    gz = global_flat_idx // (nx * ny)
    lx = (gx - q_lo[0]) % nx
    ly = (gy - q_lo[1]) % ny
    lz = (gz - q_lo[2]) % nz
    keep = (lx < q_n[0]) & (ly < q_n[1]) & (lz < q_n[2])
    loc = lx + q_n[0] * (ly + q_n[1] * lz)
    return keep, loc


def _slab_elements(n_mesh: int, elem_pts: int, nz: int, buffers: Sequence[int],
                   n_states: Sequence[int], vacancy_frac: float = 0.0,
                   vacancy_seed: Optional[int] = None, mesh_out: Optional[list] = None) -> List[Element]:
    """Elements of a graphene-like slab on an n_mesh x n_mesh element mesh (the
    global mesh data is appended to mesh_out when given)."""
    h = H_SPACING
    ngx = n_mesh * elem_pts
    ng = (ngx, ngx, nz)
    length = (ngx * h, ngx * h, nz * h)
    sites = honeycomb_sites(length[0], length[1], length[2] / 2.0)
    if vacancy_frac > 0.0:
        rng = np.random.default_rng(vacancy_seed)
        n_vac = int(round(vacancy_frac * len(sites)))
        drop = rng.choice(len(sites), size=n_vac, replace=False)
        sites = np.delete(sites, drop, axis=0)
    vglob = _gaussian_wells(ng, length, sites, WELL_DEPTH, WELL_WIDTH).ravel()
    atoms = [_atom_projectors(ng, length, c) for c in sites]
    if mesh_out is not None:
        mesh_out.append(Mesh(n_mesh, elem_pts, ng, length, vglob, atoms))
    elements = []
    for k in range(n_mesh * n_mesh):
        ex, ey = k % n_mesh, k // n_mesh
        buf = int(buffers[k])
        nq = elem_pts + 2 * buf
        q_lo = (ex * elem_pts - buf, ey * elem_pts - buf, 0)
        q_n = (nq, nq, nz)
        # restriction of the global potential to Q_k
        zz, yy, xx = np.meshgrid(np.arange(nz), (np.arange(nq) + q_lo[1]) % ngx,
                                 (np.arange(nq) + q_lo[0]) % ngx, indexing="ij")
        v = vglob[(xx + ngx * (yy + ngx * zz)).ravel()]
        # atoms whose minimum-image centre lies in Q_k
        ptr = [0]
        idx_l, val_l, gam_l, gid_l = [], [], [], []
        n_at = 0
        for a_id, (c, (gidx, gval)) in enumerate(zip(sites, atoms)):
            fx = (c[0] / h - q_lo[0]) % ngx
            fy = (c[1] / h - q_lo[1]) % ngx
            if not (fx < nq and fy < nq):
                continue
            keep, loc = _restrict(gidx, ng, q_lo, q_n)
            loc = loc[keep]
            order = np.argsort(loc)
            loc = loc[order]
            n_at += 1
            for p in range(4):
                idx_l.append(loc.astype(np.int32))
                val_l.append(gval[p][keep][order])
                gam_l.append(GAMMA_S if p == 0 else GAMMA_P)
                gid_l.append(4 * a_id + p)
                ptr.append(ptr[-1] + len(loc))
        elements.append(Element(
            n=(nq, nq, nz), length=(nq * h, nq * h, nz * h),
            elem_lo=(buf, buf, 0), elem_n=(elem_pts, elem_pts, nz),
            n_states=int(n_states[k]), v_eff=v.astype(np.float64),
            proj_ptr=np.array(ptr, dtype=np.int64),
            proj_idx=(np.concatenate(idx_l) if idx_l else np.zeros(0, np.int32)).astype(np.int32),
            proj_val=(np.concatenate(val_l) if val_l else np.zeros(0)).astype(np.float64),
            gamma=np.array(gam_l, dtype=np.float64), n_atoms=n_at,
            q_lo=q_lo, proj_gid=np.array(gid_l, dtype=np.int32)))
    return elements





def _box_element(n: Tuple[int, int, int], length: Tuple[float, float, float], sites,
                 n_states: int, elem_lo=None, elem_n=None) -> Element:
    v = (_gaussian_wells(n, length, np.asarray(sites, float), WELL_DEPTH, WELL_WIDTH).ravel()
         if len(sites) else np.zeros(n[0] * n[1] * n[2]))
    return Element(n=tuple(n), length=tuple(length),
                   elem_lo=tuple(elem_lo or (0, 0, 0)), elem_n=tuple(elem_n or n),
                   n_states=n_states, v_eff=v,
                   proj_ptr=np.zeros(1, np.int64), proj_idx=np.zeros(0, np.int32),
                   proj_val=np.zeros(0), gamma=np.zeros(0), n_atoms=len(sites))


def free_electron_element(n=(16, 16, 16), length=(10.0, 10.0, 10.0), n_states=7) -> Element:
    """V = 0, no projectors: the spectrum is the multiset of |G|^2 / 2."""
    return _box_element(n, length, [], n_states)


def small_slab(n_mesh=3, elem_pts=8, nz=32, buffer=4, n_states=8) -> List[Element]:
    """A reduced slab (same physics, smaller grids) for tests the oracle finishes in seconds."""
    return _slab_elements(n_mesh, elem_pts, nz, [buffer] * (n_mesh * n_mesh),
                          [n_states] * (n_mesh * n_mesh))


def small_slab_with_mesh(n_mesh=3, elem_pts=8, nz=32, buffer=4, n_states=8):
    """small_slab's elements and their global mesh (DG element layout, V, projectors)."""
    out: list = []
    els = _slab_elements(n_mesh, elem_pts, nz, [buffer] * (n_mesh * n_mesh), [n_states] * (n_mesh * n_mesh),
                         mesh_out=out)
    return els, out[0]


CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")


def make_config(name: str) -> Config:
    """The five workloads (sizes as stated in each description)."""
    name = name.lower()
    if name == "c1":
        rng = np.random.default_rng(0)
        sites = rng.uniform(0.0, 10.0, size=(4, 3))
        el = _box_element((16, 16, 16), (10.0, 10.0, 10.0), sites, 8)
        return Config("c1", [el], "single 10 bohr cubic element, 16^3 grid, 4 Gaussian wells, "
                      "no projectors, 8 states, FP64 LOBPCG", 100, "lobpcg", "fp64")
    mo: list = []
    if name in ("c2", "c5"):
        els = _slab_elements(4, 16, 64, [16] * 16, [40] * 16, mesh_out=mo)
        desc = ("graphene-like slab, 4x4 elements of 16x16x64, extended elements 48x48x64 "
                "(h = 0.4 bohr), Gaussian wells + 4 projectors per site, 40 states per element")
        if name == "c2":
            return Config("c2", els, desc + ", FP64", 1000, "lobpcg", "fp64", mo[0])
        return Config("c5", els, desc + ", band energy through a degree-16 Chebyshev filter",
                      1000, "chfsi", "fp64", mo[0])
    if name == "c3":
        els = _slab_elements(8, 16, 64, [16] * 64, [60] * 64, mesh_out=mo)
        return Config("c3", els, "graphene-like slab, 8x8 elements, extended 48x48x64, "
                      "60 states per element, mixed precision", 3000, "lobpcg", "mixed", mo[0])
    if name == "c4":
        rng = np.random.default_rng(4)
        q = rng.choice([32, 48, 64], size=256)
        js = rng.integers(20, 81, size=256)
        els = _slab_elements(16, 16, 64, [(int(x) - 16) // 2 for x in q], js,
                             vacancy_frac=0.02, vacancy_seed=44, mesh_out=mo)
        return Config("c4", els, "uneven batch: 256 elements, extended in-plane 32/48/64 x 64, "
                      "20-80 states, 2% vacancies, mixed precision", 4000, "lobpcg", "mixed", mo[0])
    raise ValueError(f"unknown config {name!r}")


def initial_block(n_points: int, n_cols: int, seed: int) -> np.ndarray:
    """Seeded Gaussian initial block, column-major (shape (n_cols, n_points) = one state per row)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_cols, n_points))
