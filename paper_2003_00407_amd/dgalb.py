"""ctypes binding of the C ABI in include/dg_alb.h (argument marshalling only).

Every computation runs in the HIP library ``libdgalb.so``; PyTorch provides
device memory (the arena and the caller buffers) and the HIP stream.  If the
library has not been built, importing this module raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgalb.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2003_00407_amd/build.py "
                      "(or __graft_entry__.build())")
# PyTorch's HIP runtime is loaded before the library, so that the library binds to
# it (same soname) and the caller's tensors, streams and the library share one
# runtime instance; loaded the other way round, the process would hold two.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

DG_OK, DG_WARN_NOT_CONVERGED = 0, 1
DG_ERR_ARG, DG_ERR_SHAPE, DG_ERR_OOM, DG_ERR_HIP, DG_ERR_NUMERIC, DG_ERR_STATE = -1, -2, -3, -4, -5, -6
DG_FP64, DG_MIXED, DG_FP32 = 0, 1, 2
DG_LOBPCG, DG_CHFSI = 0, 1
DG_OFF_X0, DG_OFF_VEC, DG_OFF_EIG, DG_OFF_ALB, DG_OFF_GRID, DG_OFF_KALL, DG_OFF_ELEM, DG_OFF_JJ = range(8)

EXPORTED = [
    "dg_status_string", "dg_last_error", "dg_query_workspace", "dg_create_elements", "dg_destroy",
    "dg_query_offsets", "dg_apply_H", "dg_apply_H_noalloc", "dg_solve_elements", "dg_get_ritz", "dg_get_vectors", "dg_make_alb",
    "dg_band_energy", "dg_band_energy_backward", "dg_set_potential", "dg_timing", "dg_timing_work",
    "dg_query_hamiltonian", "dg_build_hamiltonian", "dg_density", "dg_query_chefsi", "dg_chefsi",
]


class ElementDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3), ("len", C.c_double * 3), ("elem_lo", C.c_int32 * 3),
        ("elem_n", C.c_int32 * 3), ("n_states", C.c_int32), ("v_eff", C.POINTER(C.c_double)),
        ("n_proj", C.c_int32), ("proj_ptr", C.POINTER(C.c_int64)), ("proj_idx", C.POINTER(C.c_int32)),
        ("proj_val", C.POINTER(C.c_double)), ("gamma", C.POINTER(C.c_double)),
    ]


class Options(C.Structure):
    _fields_ = [("n_guard", C.c_int32), ("max_cheb_degree", C.c_int32), ("ckpt_stride", C.c_int32),
                ("n_streams", C.c_int32)]


class SolveParams(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32), ("tol", C.c_double),
                ("tol_mixed", C.c_double), ("max_iter", C.c_int32), ("cheb_degree", C.c_int32),
                ("x0_dev", C.c_void_p), ("graph_iters", C.c_int32), ("seed", C.c_int64),
                ("warm_start", C.c_int32)]


class ChefsiParams(C.Structure):
    _fields_ = [("n_want", C.c_int32), ("n_vec", C.c_int32), ("degree", C.c_int32), ("max_iter", C.c_int32),
                ("tol", C.c_double), ("lanczos_steps", C.c_int32), ("reserved", C.c_int32), ("seed", C.c_int64)]


class MeshDesc(C.Structure):
    _fields_ = [("n_mesh", C.c_int32 * 2), ("alpha", C.c_double), ("proj_count", C.POINTER(C.c_int32)),
                ("proj_gid", C.POINTER(C.c_int32)), ("proj_ptr", C.POINTER(C.c_int64)),
                ("proj_idx", C.POINTER(C.c_int32)), ("proj_val", C.POINTER(C.c_double)),
                ("gamma", C.POINTER(C.c_double))]


_lib.dg_status_string.restype = C.c_char_p
_lib.dg_status_string.argtypes = [C.c_int32]
_lib.dg_last_error.restype = C.c_char_p
_lib.dg_last_error.argtypes = [C.c_void_p]
_lib.dg_query_workspace.argtypes = [C.c_int32, C.POINTER(ElementDesc), C.POINTER(Options), C.POINTER(C.c_size_t)]
_lib.dg_create_elements.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(ElementDesc), C.POINTER(Options),
                                    C.c_void_p, C.c_size_t, C.c_void_p]
_lib.dg_destroy.argtypes = [C.c_void_p]
_lib.dg_destroy.restype = None
_lib.dg_query_offsets.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]
_lib.dg_apply_H.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                            C.c_int64]
_lib.dg_apply_H_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int64,
                                    C.c_void_p, C.c_int64]
_lib.dg_get_ritz.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
_lib.dg_solve_elements.argtypes = [C.c_void_p, C.POINTER(SolveParams), C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_int32)]
_lib.dg_get_vectors.argtypes = [C.c_void_p, C.c_void_p]
_lib.dg_make_alb.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
_lib.dg_band_energy.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                C.c_void_p, C.c_void_p, C.c_void_p]
_lib.dg_band_energy_backward.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.c_void_p]
_lib.dg_set_potential.argtypes = [C.c_void_p, C.c_void_p]
_lib.dg_timing.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
_lib.dg_timing_work.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
_lib.dg_query_hamiltonian.argtypes = [C.c_void_p, C.POINTER(MeshDesc), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]
_lib.dg_build_hamiltonian.argtypes = [C.c_void_p, C.POINTER(MeshDesc), C.c_void_p, C.c_void_p, C.c_size_t]
_lib.dg_query_chefsi.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
_lib.dg_chefsi.argtypes = [C.c_void_p, C.POINTER(ChefsiParams), C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                           C.POINTER(C.c_int64), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_size_t, C.POINTER(C.c_int32)]
_lib.dg_density.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p]


class DGError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.dg_last_error(None).decode(errors="replace")
        super().__init__(f"{where}: {_lib.dg_status_string(status).decode()} ({msg})")


def _check(st: int, where: str) -> int:
    if st < 0:
        raise DGError(st, where)
    return st


def status_string(st: int) -> str:
    return _lib.dg_status_string(st).decode()


def last_error() -> str:
    return _lib.dg_last_error(None).decode(errors="replace")


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class HostDescs:
    """ctypes descriptors for a list of workloads.Element (keeps the arrays alive)."""

    def __init__(self, elements: Sequence):
        self.keep: List[np.ndarray] = []
        arr = (ElementDesc * len(elements))()
        for i, el in enumerate(elements):
            d = arr[i]
            d.n[:] = list(el.n)
            d.len[:] = list(el.length)
            d.elem_lo[:] = list(el.elem_lo)
            d.elem_n[:] = list(el.elem_n)
            d.n_states = int(el.n_states)
            v = np.ascontiguousarray(el.v_eff, dtype=np.float64)
            pp = np.ascontiguousarray(el.proj_ptr, dtype=np.int64)
            pi = np.ascontiguousarray(el.proj_idx, dtype=np.int32)
            pv = np.ascontiguousarray(el.proj_val, dtype=np.float64)
            g = np.ascontiguousarray(el.gamma, dtype=np.float64)
            self.keep += [v, pp, pi, pv, g]
            d.v_eff = _ptr(v, C.c_double)
            d.n_proj = int(g.size)
            d.proj_ptr = _ptr(pp, C.c_int64)
            d.proj_idx = _ptr(pi, C.c_int32)
            d.proj_val = _ptr(pv, C.c_double)
            d.gamma = _ptr(g, C.c_double)
        self.arr = arr
        self.n = len(elements)


def query_workspace(elements: Sequence, n_guard: int = -1, max_cheb_degree: int = 0,
                    ckpt_stride: int = 1, n_streams: int = 0) -> int:
    """Arena bytes for these elements (CPU only, never touches the GPU)."""
    hd = HostDescs(elements)
    opt = Options(n_guard, max_cheb_degree, ckpt_stride, n_streams)
    out = C.c_size_t(0)
    _check(_lib.dg_query_workspace(hd.n, hd.arr, C.byref(opt), C.byref(out)), "dg_query_workspace")
    return int(out.value)


class HostMesh:
    """ctypes mesh descriptor (dg_mesh_desc) from per-element projector lists on E_k
    [(global ids, CSR pointer, E_k-local indices, values, gamma), ...] (keeps the arrays)."""

    def __init__(self, n_mesh, alpha: float, projectors):
        counts = np.array([len(p[0]) for p in projectors], dtype=np.int32)
        gid = np.ascontiguousarray(np.concatenate([p[0] for p in projectors]).astype(np.int32))
        ptr, base = [np.zeros(1, np.int64)], 0
        for p in projectors:
            ptr.append(p[1][1:].astype(np.int64) + base)
            base += int(p[1][-1])
        ptr = np.ascontiguousarray(np.concatenate(ptr))
        idx = np.ascontiguousarray(np.concatenate([p[2] for p in projectors]).astype(np.int32))
        val = np.ascontiguousarray(np.concatenate([p[3] for p in projectors]).astype(np.float64))
        gam = np.ascontiguousarray(np.concatenate([p[4] for p in projectors]).astype(np.float64))
        self.keep = [counts, gid, ptr, idx, val, gam]
        d = MeshDesc()
        d.n_mesh[:] = [int(n_mesh[0]), int(n_mesh[1])]
        d.alpha = float(alpha)
        d.proj_count = _ptr(counts, C.c_int32)
        d.proj_gid = _ptr(gid, C.c_int32)
        d.proj_ptr = _ptr(ptr, C.c_int64)
        d.proj_idx = _ptr(idx, C.c_int32)
        d.proj_val = _ptr(val, C.c_double)
        d.gamma = _ptr(gam, C.c_double)
        self.desc = d


class Elements:
    """A batch of extended elements resident on one GPU (the dg_ctx)."""

    def __init__(self, elements: Sequence, n_guard: int = -1, max_cheb_degree: int = 0,
                 ckpt_stride: int = 1, n_streams: int = 0, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.elements = list(elements)
        self.hd = HostDescs(self.elements)
        self.opt = Options(n_guard, max_cheb_degree, ckpt_stride, n_streams)
        nbytes = C.c_size_t(0)
        _check(_lib.dg_query_workspace(self.hd.n, self.hd.arr, C.byref(self.opt), C.byref(nbytes)),
               "dg_query_workspace")
        self.arena = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        self._arena_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p(0)
        # held by the instance: module globals may already be cleared when the
        # destructor runs at interpreter exit
        self._destroy = _lib.dg_destroy
        _check(_lib.dg_create_elements(C.byref(self.ctx), self.hd.n, self.hd.arr, C.byref(self.opt),
                                       C.c_void_p(self._arena_ptr), C.c_size_t(int(nbytes.value)),
                                       C.c_void_p(self.stream.cuda_stream)), "dg_create_elements")
        self.n_elem = self.hd.n
        # bumped by every call that replaces the context's band-energy state, so a
        # backward can tell whether its forward is still the last one
        self.generation = 0

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self._destroy(ctx)
            self.ctx = C.c_void_p(0)

    # ---- layout helpers
    def offsets(self, kind: int) -> np.ndarray:
        out = np.zeros(self.n_elem + 1, dtype=np.int64)
        _check(_lib.dg_query_offsets(self.ctx, kind, _ptr(out, C.c_int64)), "dg_query_offsets")
        return out

    def _dev(self, n, dtype):
        return self.torch.empty(int(n), dtype=dtype, device=self.device)

    # ---- entry points
    def apply_H(self, x, n_vec: int, prec: int = DG_FP64, elem: int = -1, ldx: int = 0, ldy: int = 0, y=None):
        """y = H x; x packed N_k x n_vec per element (ldx = 0) or ldx x n_vec blocks (ldx > 0)."""
        torch = self.torch
        dt = torch.float64 if prec == DG_FP64 else torch.float32
        if x.dtype != dt or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous CUDA tensor of the precision's dtype")
        if y is None:
            if ldy != ldx:
                raise ValueError("pass y when ldy differs from ldx")
            y = torch.empty_like(x)
        _check(_lib.dg_apply_H(self.ctx, elem, n_vec, prec, C.c_void_p(x.data_ptr()), int(ldx),
                               C.c_void_p(y.data_ptr()), int(ldy)), "dg_apply_H")
        return y

    def apply_H_noalloc(self, x, y, n_vec: int, prec: int = DG_FP64, elem: int = -1, ldx: int = 0, ldy: int = 0):
        """y = H x in place on caller buffers, scratch in the library's static array."""
        _check(_lib.dg_apply_H_noalloc(self.ctx, elem, n_vec, prec, C.c_void_p(x.data_ptr()), int(ldx),
                                       C.c_void_p(y.data_ptr()), int(ldy)), "dg_apply_H_noalloc")
        return y

    def solve(self, x0=None, method: int = DG_LOBPCG, precision: int = DG_FP64, tol: float = 1e-8,
              tol_mixed: float = 3e-5, max_iter: int = 300, cheb_degree: int = 16, graph_iters: int = 0,
              seed: int = 0, warm_start: bool = False):
        """Lowest J_k eigenpairs of every element; returns (eig, resid, iters, status).

        x0: packed N_k x (J_k+g_k) FP64 start blocks, or None for the seeded device draw
        (``seed``); warm_start=True starts from the vectors of the last solve."""
        torch = self.torch
        if x0 is not None and (x0.dtype != torch.float64 or not x0.is_cuda or not x0.is_contiguous()):
            raise ValueError("x0 must be a contiguous CUDA float64 tensor (packed N_k x (J_k+g_k))")
        n_eig = int(self.offsets(DG_OFF_EIG)[-1])
        eig = self._dev(n_eig, torch.float64)
        res = self._dev(n_eig, torch.float64)
        iters = (C.c_int32 * self.n_elem)()
        p = SolveParams(method, precision, tol, tol_mixed, max_iter, cheb_degree,
                        C.c_void_p(x0.data_ptr() if x0 is not None else 0), graph_iters, int(seed),
                        int(bool(warm_start)))
        self.generation += 1
        st = _check(_lib.dg_solve_elements(self.ctx, C.byref(p), C.c_void_p(eig.data_ptr()),
                                           C.c_void_p(res.data_ptr()), iters), "dg_solve_elements")
        return eig, res, np.array(list(iters), dtype=np.int32), st

    def ritz(self):
        """All J_k + g_k Ritz values and residuals of the last solve (packed, DG_OFF_KALL)."""
        n = int(self.offsets(DG_OFF_KALL)[-1])
        th = self._dev(n, self.torch.float64)
        rs = self._dev(n, self.torch.float64)
        _check(_lib.dg_get_ritz(self.ctx, C.c_void_p(th.data_ptr()), C.c_void_p(rs.data_ptr())), "dg_get_ritz")
        return th, rs

    def vectors(self):
        n = int(self.offsets(DG_OFF_VEC)[-1])
        out = self._dev(n, self.torch.float64)
        _check(_lib.dg_get_vectors(self.ctx, C.c_void_p(out.data_ptr())), "dg_get_vectors")
        return out

    def make_alb(self):
        torch = self.torch
        alb = self._dev(int(self.offsets(DG_OFF_ALB)[-1]), torch.float64)
        sv = self._dev(int(self.offsets(DG_OFF_EIG)[-1]), torch.float64)
        _check(_lib.dg_make_alb(self.ctx, C.c_void_p(alb.data_ptr()), C.c_void_p(sv.data_ptr())),
               "dg_make_alb")
        return alb, sv

    def set_potential(self, v):
        """Replace V_eff (packed FP64 CUDA tensor, N_k per element)."""
        if v.dtype != self.torch.float64 or not v.is_cuda or not v.is_contiguous():
            raise ValueError("v must be a contiguous CUDA float64 tensor")
        self.generation += 1
        _check(_lib.dg_set_potential(self.ctx, C.c_void_p(v.data_ptr())), "dg_set_potential")

    def band_energy(self, psi0, f, degree: int, bounds, prec: int = DG_FP64):
        """E per element for Psi = p_m(H) Psi_0 (packed psi0, n_vec columns per element)."""
        torch = self.torch
        n_vec = int(f.numel())
        bnd = np.ascontiguousarray(np.asarray(bounds, dtype=np.float64).reshape(-1))
        if bnd.size != 3 * self.n_elem:
            raise ValueError("bounds needs 3 values per element")
        E = self._dev(self.n_elem, torch.float64)
        self._be_f = f          # must outlive the backward
        self.generation += 1
        _check(_lib.dg_band_energy(self.ctx, prec, degree, _ptr(bnd, C.c_double), n_vec,
                                   C.c_void_p(psi0.data_ptr()), C.c_void_p(f.data_ptr()),
                                   C.c_void_p(E.data_ptr())), "dg_band_energy")
        self._be_shape = (psi0.numel(), psi0.dtype)
        return E

    def band_energy_backward(self, dE):
        """(dE/dPsi_0 packed like psi0, dE/dV packed FP64) scaled by dE (per element)."""
        torch = self.torch
        n, dt = self._be_shape
        dpsi = self._dev(n, dt)
        dv = self._dev(int(self.offsets(DG_OFF_GRID)[-1]), torch.float64)
        de = np.ascontiguousarray(np.asarray(dE, dtype=np.float64).reshape(-1))
        _check(_lib.dg_band_energy_backward(self.ctx, _ptr(de, C.c_double), C.c_void_p(dpsi.data_ptr()),
                                            C.c_void_p(dv.data_ptr())), "dg_band_energy_backward")
        return dpsi, dv

    def hamiltonian_layout(self, hmesh: "HostMesh"):
        """Block-sparse layout of the DG Hamiltonian for this mesh: (row_ptr (n_elem + 1),
        col_idx (n_blocks), block_off (n_blocks + 1), work bytes)."""
        nb = C.c_int32(0)
        wb = C.c_size_t(0)
        _check(_lib.dg_query_hamiltonian(self.ctx, C.byref(hmesh.desc), C.byref(nb), None, None, None, C.byref(wb)),
               "dg_query_hamiltonian")
        row_ptr = np.zeros(self.n_elem + 1, dtype=np.int64)
        col = np.zeros(nb.value, dtype=np.int32)
        off = np.zeros(nb.value + 1, dtype=np.int64)
        _check(_lib.dg_query_hamiltonian(self.ctx, C.byref(hmesh.desc), C.byref(nb), _ptr(row_ptr, C.c_int64),
                                         _ptr(col, C.c_int32), _ptr(off, C.c_int64), C.byref(wb)),
               "dg_query_hamiltonian")
        return row_ptr, col, off, int(wb.value)

    def build_hamiltonian(self, hmesh: "HostMesh"):
        """H^DG (packed FP64 device tensor of blocks) and its layout (row_ptr, col_idx,
        block_off); block b of row k is J_k x J_col column-major; see dg_build_hamiltonian."""
        torch = self.torch
        row_ptr, col, off, wb = self.hamiltonian_layout(hmesh)
        H = self._dev(int(off[-1]), torch.float64)
        work = torch.empty(wb + 256, dtype=torch.uint8, device=self.device)
        wp = (work.data_ptr() + 255) // 256 * 256
        self.generation += 1
        _check(_lib.dg_build_hamiltonian(self.ctx, C.byref(hmesh.desc), C.c_void_p(H.data_ptr()), C.c_void_p(wp),
                                         C.c_size_t(wb)), "dg_build_hamiltonian")
        return H, (row_ptr, col, off)

    def hamiltonian_blocks(self, H, layout) -> dict:
        """{(k, nb): J_k x J_nb numpy block} from build_hamiltonian's output (host copy)."""
        row_ptr, col, off = layout
        Hh = H.cpu().numpy()
        Js = [e.n_states for e in self.elements]
        out = {}
        for k in range(self.n_elem):
            for b in range(int(row_ptr[k]), int(row_ptr[k + 1])):
                nb = int(col[b])
                out[(k, nb)] = Hh[off[b]:off[b + 1]].reshape(Js[nb], Js[k]).T
        return out

    def chefsi(self, H, layout, x0, n_want: int, degree: int = 16, tol: float = 1e-9, max_iter: int = 100,
               lanczos_steps: int = 10, seed: int = 0):
        """Lowest eigenpairs of H^DG (build_hamiltonian's H and layout) by CheFSI from the
        start block x0 (a (n_vec, N_b) row-major CUDA float64 tensor = column-major
        N_b x n_vec); returns (X like x0, Ritz values, residuals, iterations, status)."""
        torch = self.torch
        row_ptr, col, off = layout
        n_vec, nb = int(x0.shape[0]), int(x0.shape[1])
        if x0.dtype != torch.float64 or not x0.is_cuda or not x0.is_contiguous():
            raise ValueError("x0 must be a contiguous CUDA float64 tensor")
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        off = np.ascontiguousarray(off, dtype=np.int64)
        wb = C.c_size_t(0)
        _check(_lib.dg_query_chefsi(self.ctx, len(col), n_vec, C.byref(wb)), "dg_query_chefsi")
        work = torch.empty(wb.value + 256, dtype=torch.uint8, device=self.device)
        wp = (work.data_ptr() + 255) // 256 * 256
        X = x0.clone()
        eig = self._dev(n_vec, torch.float64)
        res = self._dev(n_vec, torch.float64)
        it = C.c_int32(0)
        p = ChefsiParams(n_want, n_vec, degree, max_iter, tol, lanczos_steps, 0, int(seed))
        st = _check(_lib.dg_chefsi(self.ctx, C.byref(p), len(col), _ptr(row_ptr, C.c_int64), _ptr(col, C.c_int32),
                                   _ptr(off, C.c_int64), C.c_void_p(H.data_ptr()), C.c_void_p(X.data_ptr()),
                                   C.c_void_p(eig.data_ptr()), C.c_void_p(res.data_ptr()), C.c_void_p(wp),
                                   C.c_size_t(wb.value), C.byref(it)), "dg_chefsi")
        return X, eig, res, int(it.value), st

    def density(self, alb, C_coef, n_e: int = -1, ldc: int = 0):
        """(P diagonal blocks, rho) from the ALB values (make_alb) and the FP64 DG
        coefficients C_coef: a column-major (sum J_k) x n_e device tensor given as
        its transpose, i.e. a row-major (n_e, ldc) tensor; see dg_density."""
        torch = self.torch
        if n_e < 0:
            n_e = int(C_coef.shape[0]) if C_coef is not None else 0
        if C_coef is not None:
            if C_coef.dtype != torch.float64 or not C_coef.is_cuda or C_coef.dim() != 2 or \
                    (C_coef.shape[1] > 1 and C_coef.stride(1) != 1):
                raise ValueError("C_coef must be a 2-D CUDA float64 tensor with unit column stride")
            if ldc == 0:
                # a single state's row stride is not meaningful (torch may report any value)
                ldc = int(C_coef.shape[1]) if C_coef.shape[0] <= 1 else int(C_coef.stride(0))
        P = self._dev(int(self.offsets(DG_OFF_JJ)[-1]), torch.float64)
        rho = self._dev(int(self.offsets(DG_OFF_ELEM)[-1]), torch.float64)
        cp = C.c_void_p(C_coef.data_ptr()) if C_coef is not None else None
        _check(_lib.dg_density(self.ctx, C.c_void_p(alb.data_ptr()), cp, C.c_int64(ldc), C.c_int32(n_e),
                               C.c_void_p(P.data_ptr()), C.c_void_p(rho.data_ptr())), "dg_density")
        return P, rho

    TIMING_CLASSES = ("plane", "zcol", "nonlocal", "teter", "gram", "rotate", "rayleigh_ritz", "other")

    def timing(self, enable: bool = True, reset: bool = False):
        """(ms, launches, algorithmic work) per class since the last reset; then reset/enable.

        work has 9 entries: the 8 classes, then the H*psi bytes by the per-state count."""
        ms = (C.c_double * 8)()
        n = (C.c_int64 * 8)()
        w = (C.c_double * 9)()
        _check(_lib.dg_timing_work(self.ctx, w), "dg_timing_work")
        _check(_lib.dg_timing(self.ctx, int(enable), int(reset), ms, n), "dg_timing")
        return list(ms), list(n), list(w)


def pack_initial(elements: Sequence, seed_base: int, n_guard: int = -1):
    """Seeded initial blocks, packed N_k x (J_k + g_k) per element (host float64)."""
    import workloads as W
    parts = []
    for k, el in enumerate(elements):
        g = W.guard_count(el.n_states) if n_guard < 0 else n_guard
        parts.append(W.initial_block(el.npts, el.n_states + g, seed=seed_base + k).ravel())
    return np.concatenate(parts)


def _band_energy_function():
    import torch

    class BandEnergy(torch.autograd.Function):
        """E_k(V, Psi_0) = sum_i f_i psi_i^T H[V] psi_i through the degree-m Chebyshev filter.

        forward(v, psi0, elements, f, degree, bounds, prec): v packed FP64 (N_k per
        element) or None to keep the context's potential; psi0 packed (n_vec = f.numel()
        columns per element).  Returns E (one FP64 value per element).  The backward
        runs the checkpointed adjoint recurrence in the HIP library.
        """

        @staticmethod
        def forward(ctx, v, psi0, elements, f, degree, bounds, prec=DG_FP64):
            if v is not None:
                elements.set_potential(v.detach().contiguous())
            E = elements.band_energy(psi0.detach().contiguous(), f, degree, bounds, prec)
            ctx.elements = elements
            ctx.has_v = v is not None
            ctx.generation = elements.generation
            return E

        @staticmethod
        def backward(ctx, gE):
            if ctx.elements.generation != ctx.generation:
                raise RuntimeError("BandEnergy.backward: the context ran another band energy, solve or "
                                   "potential update after this forward; its adjoint state is gone "
                                   "(run backward before the next forward on the same Elements)")
            dpsi, dv = ctx.elements.band_energy_backward(gE.detach().double().cpu().numpy())
            return (dv if ctx.has_v else None), dpsi, None, None, None, None, None

    return BandEnergy


def __getattr__(name):
    if name == "BandEnergy":
        return _band_energy_function()
    raise AttributeError(name)
