"""ctypes binding of libhgeo.so (the C ABI of include/hgeo.h).

Argument marshalling only: every step of the geodesic pipeline runs in the
library's HIP kernels.  torch supplies device memory and streams.  The
binding refuses to run when the compiled library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgeo.so")

HG_OK, HG_E_INVALID_ARG, HG_E_BAD_MESH, HG_E_OOM, HG_E_NOT_CONVERGED, HG_E_DEVICE = range(6)
FORM_FACE, FORM_EDGE = 0, 1
_STATUS = {0: "HG_OK", 1: "HG_E_INVALID_ARG", 2: "HG_E_BAD_MESH", 3: "HG_E_OOM",
           4: "HG_E_NOT_CONVERGED", 5: "HG_E_DEVICE"}


class HgeoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status
        self.msg = msg


class NotConverged(HgeoError):
    pass


class Opts(C.Structure):
    _fields_ = [
        ("formulation", C.c_int32), ("m", C.c_double), ("tol_u", C.c_double),
        ("tol_admm", C.c_double), ("max_sweeps", C.c_int32), ("max_admm", C.c_int32),
        ("mu", C.c_double), ("check_every", C.c_int32), ("diffusion_schedule", C.c_int32),
        ("inner_sweeps", C.c_int32), ("relax", C.c_double), ("source_paths", C.c_int32),
        ("t_per_component", C.c_int32), ("use_graphs", C.c_int32), ("cycle_constraints", C.c_int32),
        ("tol_seam", C.c_double), ("admm_block", C.c_int32), ("overlap_rings", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("bfs_depth", C.c_int32), ("sweeps", C.c_int32), ("passes", C.c_int32),
        ("admm_iters", C.c_int32), ("res_u", C.c_double), ("res_primal", C.c_double),
        ("res_dual", C.c_double), ("t", C.c_double),
        ("ms_bfs", C.c_float), ("ms_diffusion", C.c_float), ("ms_normalize", C.c_float),
        ("ms_admm", C.c_float), ("ms_integrate", C.c_float), ("ms_total", C.c_float),
        ("bytes_alg", C.c_uint64), ("workspace_bytes", C.c_uint64),
        ("converged_u", C.c_int32), ("converged_admm", C.c_int32),
        ("ms_pass_kernel", C.c_float), ("ms_admm_kernel", C.c_float),
        ("bytes_pass_kernel", C.c_uint64), ("bytes_admm_kernel", C.c_uint64),
        ("n_paths", C.c_int32), ("path_edges", C.c_int32), ("n_cycles", C.c_int32), ("cycle_slots", C.c_int32),
        ("seam", C.c_float), ("admm_launches", C.c_int32), ("admm_block", C.c_int32),
        ("reserved", C.c_int32 * 1),
    ]

    def as_dict(self):
        return {k: (getattr(self, k) if k != "reserved" else None) for k, _ in self._fields_ if k != "reserved"}


class MeshStats(C.Structure):
    _fields_ = [
        ("nv", C.c_int64), ("nf", C.c_int64), ("ne", C.c_int64), ("n_boundary_edges", C.c_int64),
        ("hbar", C.c_double), ("total_area", C.c_double), ("max_valence", C.c_int32),
        ("n_patches", C.c_int32), ("mesh_bytes", C.c_uint64), ("n_components", C.c_int32),
        ("n_colors", C.c_int32), ("n_cycles", C.c_int32), ("cycle_edges", C.c_int32), ("cycle_faces", C.c_int32),
        ("intrinsic", C.c_int32), ("n_flips", C.c_int32), ("n_nondelaunay", C.c_int32), ("reserved", C.c_int32 * 4),
    ]


class Result(C.Structure):
    _fields_ = [
        ("ticket", C.c_int64), ("status", C.c_int32), ("reserved0", C.c_int32),
        ("t_submit", C.c_double), ("t_start", C.c_double), ("t_end", C.c_double), ("info", Info),
    ]


class ServerStats(C.Structure):
    _fields_ = [
        ("n_slots", C.c_int32), ("pending", C.c_int32), ("running", C.c_int32),
        ("completed_unread", C.c_int32), ("workspaces_idle", C.c_int32), ("reserved0", C.c_int32),
        ("workspace_bytes_held", C.c_uint64), ("workspace_bytes_idle", C.c_uint64),
        ("workspace_budget", C.c_uint64), ("reserved", C.c_int32 * 8),
    ]


class TuneReport(C.Structure):
    _fields_ = [
        ("n_candidates", C.c_int32), ("chosen", C.c_int32), ("schedule", C.c_int32 * 8),
        ("inner_sweeps", C.c_int32 * 8), ("ms", C.c_float * 8), ("passes", C.c_int32 * 8),
        ("overlap_rings", C.c_int32 * 8), ("n_admm", C.c_int32), ("admm_chosen", C.c_int32),
        ("admm_block", C.c_int32 * 4), ("admm_us_per_iteration", C.c_float * 4),
    ]


class CgInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("res_rel", C.c_double), ("res_abs", C.c_double),
                ("res_abs0", C.c_double), ("ms", C.c_float), ("reserved", C.c_int32 * 3)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


# (name, argtypes)
_P = C.c_void_p
_API = {
    "hg_opts_default": [C.POINTER(Opts)],
    "hg_mesh_create": [_P, C.c_int64, _P, C.c_int64, _P, C.POINTER(_P)],
    "hg_mesh_create_intrinsic": [_P, C.c_int64, _P, C.c_int64, _P, C.POINTER(_P)],
    "hg_mesh_intrinsic": [_P, _P, _P],
    "hg_mesh_destroy": [_P],
    "hg_mesh_get_stats": [_P, C.POINTER(MeshStats)],
    "hg_geodesic_solve": [_P, _P, C.c_int32, C.c_double, C.POINTER(Opts), _P, _P, C.POINTER(Info)],
    "hg_geodesic_solve_batch": [_P, C.c_int32, _P, _P, C.c_double, C.POINTER(Opts), _P, _P, C.POINTER(Info)],
    "hg_mesh_bytes": [_P],
    "hg_cg_diffuse": [_P, _P, C.c_int32, C.c_double, C.c_int32, C.c_double, _P, _P, C.POINTER(CgInfo)],
    "hg_cg_poisson": [_P, C.c_int32, _P, _P, C.c_int32, C.c_int32, C.c_double, _P, _P, C.POINTER(CgInfo)],
    "hg_heat_residual": [_P, _P, C.c_int32, C.c_double, _P, C.c_int32, C.POINTER(C.c_double), _P],
    "hg_query_bytes": [_P, C.c_int32, C.POINTER(Opts)],
    "hg_bfs": [_P, _P, C.c_int32, _P, _P, _P, C.POINTER(C.c_int32)],
    "hg_bfs_noalloc": [_P, _P, C.c_int32, _P, _P, _P, C.POINTER(C.c_int32)],
    "hg_diffuse": [_P, _P, C.c_int32, C.c_double, C.POINTER(Opts), _P, _P, C.POINTER(Info)],
    "hg_normalize": [_P, _P, _P, _P],
    "hg_admm_edge": [_P, _P, _P, C.c_int32, C.c_int32, C.POINTER(Opts), _P, _P, C.POINTER(Info)],
    "hg_admm_face": [_P, _P, _P, C.c_int32, C.c_int32, C.POINTER(Opts), _P, _P, C.POINTER(Info)],
    "hg_integrate_edge": [_P, _P, C.c_int32, _P, _P, _P],
    "hg_integrate_face": [_P, _P, C.c_int32, _P, _P, _P],
    "hg_mesh_edges": [_P, _P, _P],
    "hg_mesh_weights": [_P, _P, _P, _P],
    "hg_mesh_cycles": [_P, C.c_int32, _P, _P, _P, C.c_int64],
    "hg_mesh_autotune": [_P, _P, C.c_int32, C.c_double, C.POINTER(Opts), _P, C.POINTER(TuneReport)],
    "hg_server_create": [C.c_int32, C.c_uint64, C.POINTER(_P)],
    "hg_server_submit": [_P, _P, _P, C.c_int32, C.c_double, C.POINTER(Opts), _P, C.POINTER(C.c_int64)],
    "hg_server_wait": [_P, C.POINTER(Result), C.c_int32],
    "hg_server_stats": [_P, C.POINTER(ServerStats)],
    "hg_server_clock": [],
    "hg_server_destroy": [_P],
    "hg_last_error": [],
}
EXPORTED = tuple(_API)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhgeo.so and declare its prototypes (no GPU needed)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1812_06060_amd.build`")
    lib = C.CDLL(path)
    for name, args in _API.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        if name == "hg_last_error":
            fn.restype = C.c_char_p
        elif name in ("hg_mesh_destroy", "hg_server_destroy"):
            fn.restype = None
        elif name == "hg_server_clock":
            fn.restype = C.c_double
        elif name in ("hg_mesh_bytes", "hg_query_bytes"):
            fn.restype = C.c_uint64
        else:
            fn.restype = C.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def _check(st: int):
    if st == HG_OK:
        return
    msg = _lib.hg_last_error().decode()
    if st == HG_E_NOT_CONVERGED:
        raise NotConverged(st, msg)
    raise HgeoError(st, msg)


def default_opts(**kw) -> Opts:
    lib = load_library()
    o = Opts()
    lib.hg_opts_default(C.byref(o))
    form = kw.pop("formulation", None)
    if form is not None:
        o.formulation = {"face": FORM_FACE, "edge": FORM_EDGE}.get(form, form)
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def paper_opts(formulation="edge", **kw) -> Opts:
    """The paper's own ADMM setting (Sec. 6): ten iterations, penalty
    mu = 100, no over-relaxation (alpha = 1).  Ten iterations stop far short
    of the discrete optimum on meshes of many rings, so solves with these
    options end at the cap (HG_E_NOT_CONVERGED, results written)."""
    base = dict(formulation=formulation, max_admm=10, mu=100.0, relax=1.0)
    base.update(kw)
    return default_opts(**base)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("hgeo needs a ROCm GPU (torch.cuda is not available)")
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _src_array(sources):
    a = np.ascontiguousarray(np.atleast_1d(np.asarray(sources, dtype=np.int32)))
    return a, a.ctypes.data_as(C.c_void_p), C.c_int32(a.size)


def _dptr(t, dtype, numel):
    torch = _torch()
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"expected a contiguous CUDA {dtype} tensor with {numel} elements")
    return C.c_void_p(t.data_ptr())


@dataclass
class SolveInfo:
    raw: dict

    def __getattr__(self, k):
        try:
            return self.raw[k]
        except KeyError:
            raise AttributeError(k)


class Mesh:
    """A resident device mesh (hg_mesh_create; with intrinsic=True
    hg_mesh_create_intrinsic, the intrinsic Delaunay triangulation)."""

    def __init__(self, verts, tris, stream=None, intrinsic: bool = False):
        load_library()
        _torch()
        v = np.ascontiguousarray(np.asarray(verts, dtype=np.float64))
        f = np.ascontiguousarray(np.asarray(tris, dtype=np.int32))
        if v.ndim != 2 or v.shape[1] != 3 or f.ndim != 2 or f.shape[1] != 3:
            raise ValueError("verts must be [V,3] and tris [F,3]")
        h = C.c_void_p()
        create = _lib.hg_mesh_create_intrinsic if intrinsic else _lib.hg_mesh_create
        _check(create(v.ctypes.data_as(C.c_void_p), v.shape[0], f.ctypes.data_as(C.c_void_p), f.shape[0],
                      _stream(stream), C.byref(h)))
        self._h = h
        st = MeshStats()
        _check(_lib.hg_mesh_get_stats(self._h, C.byref(st)))
        self.nv, self.nf, self.ne = st.nv, st.nf, st.ne
        self.hbar = st.hbar
        self.total_area = st.total_area

    @property
    def stats(self) -> dict:
        """hg_mesh_get_stats, read now (mesh_bytes grows when a query first
        builds the face form's slot records or the blocked ADMM's tiles)."""
        st = MeshStats()
        _check(_lib.hg_mesh_get_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_ if k != "reserved"}

    def close(self):
        if getattr(self, "_h", None):
            _lib.hg_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ whole solve
    def solve(self, sources, t: float = 0.0, opts: Opts | None = None, out=None, stream=None,
              raise_on_nonconvergence: bool = True):
        torch = _torch()
        if out is None:
            out = torch.empty(self.nv, dtype=torch.float32, device="cuda")
        a, p, n = _src_array(sources)
        info = Info()
        st = _lib.hg_geodesic_solve(self._h, p, n, float(t), C.byref(opts) if opts else None,
                                    _dptr(out, torch.float32, self.nv), _stream(stream), C.byref(info))
        if st != HG_E_NOT_CONVERGED or raise_on_nonconvergence:
            _check(st)
        return out, SolveInfo(info.as_dict())

    # ------------------------------------------- Sec. 6.4 comparator (CG)
    def cg_diffuse(self, sources, t: float = 0.0, max_iters: int = 100000, tol: float = 1e-12, stream=None,
                   raise_on_nonconvergence: bool = True):
        """Jacobi-preconditioned CG on Eq. 4 (hg_cg_diffuse): (float64 u, info)."""
        torch = _torch()
        u = torch.empty(self.nv, dtype=torch.float64, device="cuda")
        a, p, n = _src_array(sources)
        info = CgInfo()
        st = _lib.hg_cg_diffuse(self._h, p, n, float(t), int(max_iters), float(tol),
                                _dptr(u, torch.float64, self.nv), _stream(stream), C.byref(info))
        if st != HG_E_NOT_CONVERGED or raise_on_nonconvergence:
            _check(st)
        return u, info.as_dict()

    def cg_poisson(self, h, sources, form: str = "face", max_iters: int = 100000, tol: float = 1e-12,
                   stream=None, raise_on_nonconvergence: bool = True):
        """Jacobi-preconditioned CG on the Poisson step with d = 0 at the
        sources (hg_cg_poisson), from float32 h [nf*3]: (float64 d, info)."""
        torch = _torch()
        d = torch.empty(self.nv, dtype=torch.float64, device="cuda")
        a, p, n = _src_array(sources)
        fm = {"face": FORM_FACE, "edge": FORM_EDGE}[form]
        info = CgInfo()
        st = _lib.hg_cg_poisson(self._h, fm, _dptr(h, torch.float32, 3 * self.nf), p, n, int(max_iters),
                                float(tol), _dptr(d, torch.float64, self.nv), _stream(stream), C.byref(info))
        if st != HG_E_NOT_CONVERGED or raise_on_nonconvergence:
            _check(st)
        return d, info.as_dict()

    def heat_residual(self, sources, u, t: float = 0.0, is_log: bool = False, stream=None) -> float:
        """E_1 = |(A - t L_c) u - u_0|_2 of Eq. 29 (hg_heat_residual)."""
        torch = _torch()
        a, p, n = _src_array(sources)
        e1 = C.c_double()
        _check(_lib.hg_heat_residual(self._h, p, n, float(t), _dptr(u, torch.float64, self.nv),
                                     1 if is_log else 0, C.byref(e1), _stream(stream)))
        return e1.value

    def mesh_bytes(self) -> int:
        return int(_lib.hg_mesh_bytes(self._h))

    def query_bytes(self, nsrc: int, opts: Opts | None = None) -> int:
        """Upper estimate of one query's workspace bytes (hg_query_bytes)."""
        return int(_lib.hg_query_bytes(self._h, int(nsrc), C.byref(opts) if opts else None))

    def autotune(self, sources, t: float = 0.0, opts: Opts | None = None, stream=None) -> dict:
        """Pick the fastest diffusion schedule for this mesh on a probe query
        (hg_mesh_autotune); later solves with automatic options use it."""
        a, p, n = _src_array(sources)
        rep = TuneReport()
        _check(_lib.hg_mesh_autotune(self._h, p, n, float(t), C.byref(opts) if opts else None, _stream(stream),
                                     C.byref(rep)))
        k = rep.n_candidates
        return {"chosen": rep.chosen,
                "candidates": [{"schedule": rep.schedule[i], "inner_sweeps": rep.inner_sweeps[i],
                                "overlap_rings": rep.overlap_rings[i], "ms": rep.ms[i], "passes": rep.passes[i]}
                               for i in range(k)],
                "admm_chosen": rep.admm_chosen,
                "admm": [{"block": rep.admm_block[i], "us_per_iteration": rep.admm_us_per_iteration[i]}
                         for i in range(rep.n_admm)]}

    def intrinsic_triangulation(self):
        """(flipped triangles int32[F, 3], edge lengths float64[E] in
        canonical edge order) of an intrinsic mesh (hg_mesh_intrinsic)."""
        tri = np.zeros((self.nf, 3), dtype=np.int32)
        length = np.zeros(self.ne, dtype=np.float64)
        _check(_lib.hg_mesh_intrinsic(self._h, tri.ctypes.data, length.ctypes.data))
        return tri, length

    def cycles(self, form: str = "edge"):
        """The generator loops of the cycle constraints (hg_mesh_cycles), as a
        list of (ids, coef): edge form canonical edge ids and signs, face form
        caller face ids and [n, 3] polyline segments."""
        fm = {"face": FORM_FACE, "edge": FORM_EDGE}[form]
        n = self.stats["n_cycles"]
        cap = self.stats["cycle_edges" if fm == FORM_EDGE else "cycle_faces"]
        ptr = np.zeros(n + 1, dtype=np.int32)
        ids = np.zeros(max(cap, 1), dtype=np.int32)
        coef = np.zeros(max(cap, 1) * (1 if fm == FORM_EDGE else 3), dtype=np.float32)
        _check(_lib.hg_mesh_cycles(self._h, fm, ptr.ctypes.data, ids.ctypes.data, coef.ctypes.data, cap))
        out = []
        for i in range(n):
            a, b = int(ptr[i]), int(ptr[i + 1])
            c = coef[a:b].copy() if fm == FORM_EDGE else coef[3 * a:3 * b].reshape(-1, 3).copy()
            out.append((ids[a:b].copy(), c))
        return out

    # ---------------------------------------------------------------- stages
    def edges(self, stream=None):
        torch = _torch()
        out = torch.empty((self.ne, 2), dtype=torch.int32, device="cuda")
        _check(_lib.hg_mesh_edges(self._h, _dptr(out, torch.int32, 2 * self.ne), _stream(stream)))
        return out

    def weights(self, stream=None):
        """(theta per canonical edge, lumped area per vertex), float64 on the device."""
        torch = _torch()
        th = torch.empty(self.ne, dtype=torch.float64, device="cuda")
        ar = torch.empty(self.nv, dtype=torch.float64, device="cuda")
        _check(_lib.hg_mesh_weights(self._h, _dptr(th, torch.float64, self.ne), _dptr(ar, torch.float64, self.nv),
                                    _stream(stream)))
        return th, ar

    def bfs(self, sources, stream=None):
        torch = _torch()
        lev = torch.empty(self.nv, dtype=torch.int32, device="cuda")
        par = torch.empty(self.nv, dtype=torch.int32, device="cuda")
        a, p, n = _src_array(sources)
        depth = C.c_int32()
        _check(_lib.hg_bfs(self._h, p, n, _dptr(lev, torch.int32, self.nv), _dptr(par, torch.int32, self.nv),
                           _stream(stream), C.byref(depth)))
        return lev, par, depth.value

    def bfs_noalloc(self, sources, level=None, parent=None, stream=None):
        """hg_bfs on the library's fixed device array (no device allocation
        inside the call); level/parent: optional caller-owned int32[nv]."""
        torch = _torch()
        lev = torch.empty(self.nv, dtype=torch.int32, device="cuda") if level is None else level
        par = torch.empty(self.nv, dtype=torch.int32, device="cuda") if parent is None else parent
        a, p, n = _src_array(sources)
        depth = C.c_int32()
        _check(_lib.hg_bfs_noalloc(self._h, p, n, _dptr(lev, torch.int32, self.nv),
                                   _dptr(par, torch.int32, self.nv), _stream(stream), C.byref(depth)))
        return lev, par, depth.value

    def diffuse(self, sources, t: float = 0.0, opts: Opts | None = None, stream=None,
                raise_on_nonconvergence: bool = True):
        torch = _torch()
        out = torch.empty(self.nv, dtype=torch.float64, device="cuda")
        a, p, n = _src_array(sources)
        info = Info()
        st = _lib.hg_diffuse(self._h, p, n, float(t), C.byref(opts) if opts else None,
                             _dptr(out, torch.float64, self.nv), _stream(stream), C.byref(info))
        if st != HG_E_NOT_CONVERGED or raise_on_nonconvergence:
            _check(st)
        return out, SolveInfo(info.as_dict())

    def normalize(self, logu, stream=None):
        torch = _torch()
        h = torch.empty((self.nf, 3), dtype=torch.float32, device="cuda")
        _check(_lib.hg_normalize(self._h, _dptr(logu, torch.float64, self.nv),
                                 _dptr(h, torch.float32, 3 * self.nf), _stream(stream)))
        return h

    def admm_edge(self, h, iters: int = 0, opts: Opts | None = None, stream=None, sources=None):
        """Edge-form ADMM; `sources` (two or more) adds the path constraints
        of Eq. 25."""
        torch = _torch()
        x = torch.empty(self.ne, dtype=torch.float32, device="cuda")
        info = Info()
        a, p, n = _src_array(sources) if sources is not None else (None, None, 0)
        st = _lib.hg_admm_edge(self._h, _dptr(h, torch.float32, 3 * self.nf), p, n, int(iters),
                               C.byref(opts) if opts else None, _dptr(x, torch.float32, self.ne),
                               _stream(stream), C.byref(info))
        _check(st)
        return x, SolveInfo(info.as_dict())

    def admm_face(self, h, iters: int = 0, opts: Opts | None = None, stream=None, sources=None):
        """Face-form ADMM; `sources` (two or more) adds the path constraints
        of Eq. 24."""
        torch = _torch()
        g = torch.empty((self.nf, 3), dtype=torch.float32, device="cuda")
        info = Info()
        a, p, n = _src_array(sources) if sources is not None else (None, None, 0)
        st = _lib.hg_admm_face(self._h, _dptr(h, torch.float32, 3 * self.nf), p, n, int(iters),
                               C.byref(opts) if opts else None, _dptr(g, torch.float32, 3 * self.nf),
                               _stream(stream), C.byref(info))
        _check(st)
        return g, SolveInfo(info.as_dict())

    def integrate_edge(self, sources, x, stream=None):
        torch = _torch()
        d = torch.empty(self.nv, dtype=torch.float32, device="cuda")
        a, p, n = _src_array(sources)
        _check(_lib.hg_integrate_edge(self._h, p, n, _dptr(x, torch.float32, self.ne),
                                      _dptr(d, torch.float32, self.nv), _stream(stream)))
        return d

    def integrate_face(self, sources, g, stream=None):
        torch = _torch()
        d = torch.empty(self.nv, dtype=torch.float32, device="cuda")
        a, p, n = _src_array(sources)
        _check(_lib.hg_integrate_face(self._h, p, n, _dptr(g, torch.float32, 3 * self.nf),
                                      _dptr(d, torch.float32, self.nv), _stream(stream)))
        return d


def solve_batch(meshes, sources, t: float = 0.0, opts: Opts | None = None, outs=None, stream=None,
                raise_on_nonconvergence: bool = True):
    """One solve over several resident meshes (hg_geodesic_solve_batch):
    query i on meshes[i] from sources[i] (its own vertex ids).  Returns (list
    of float32 device tensors, one per mesh, SolveInfo of the batch)."""
    torch = _torch()
    n = len(meshes)
    if n == 0 or len(sources) != n:
        raise ValueError("one source list per mesh expected")
    if outs is None:
        outs = [torch.empty(m.nv, dtype=torch.float32, device="cuda") for m in meshes]
    arrs = [np.ascontiguousarray(np.atleast_1d(np.asarray(s, dtype=np.int32))) for s in sources]
    hs = (C.c_void_p * n)(*[m._h for m in meshes])
    sp = (C.c_void_p * n)(*[a.ctypes.data for a in arrs])
    ns = (C.c_int32 * n)(*[a.size for a in arrs])
    dp = (C.c_void_p * n)(*[_dptr(o, torch.float32, m.nv).value for o, m in zip(outs, meshes)])
    info = Info()
    st = _lib.hg_geodesic_solve_batch(hs, n, sp, ns, float(t), C.byref(opts) if opts else None, dp,
                                      _stream(stream), C.byref(info))
    if st != HG_E_NOT_CONVERGED or raise_on_nonconvergence:
        _check(st)
    return outs, SolveInfo(info.as_dict())


class Server:
    """Concurrent query runtime (hg_server_*): n_slots worker slots, each on
    its own stream; queries are admitted as slots and memory free up."""

    def __init__(self, n_slots: int = 4, workspace_budget: int = 0):
        load_library()
        _torch()
        h = C.c_void_p()
        _check(_lib.hg_server_create(int(n_slots), int(workspace_budget), C.byref(h)))
        self._h = h
        self._keep = {}   # ticket -> (mesh, out tensor) kept alive until taken

    def submit(self, mesh: "Mesh", sources, out=None, t: float = 0.0, opts: Opts | None = None) -> tuple:
        torch = _torch()
        if out is None:
            out = torch.empty(mesh.nv, dtype=torch.float32, device="cuda")
        a, p, n = _src_array(sources)
        tk = C.c_int64()
        _check(_lib.hg_server_submit(self._h, mesh._h, p, n, float(t), C.byref(opts) if opts else None,
                                     _dptr(out, torch.float32, mesh.nv), C.byref(tk)))
        self._keep[tk.value] = (mesh, out)
        return tk.value, out

    def wait(self, timeout_ms: int = -1):
        """The next completed query as a dict (None on timeout)."""
        r = Result()
        _check(_lib.hg_server_wait(self._h, C.byref(r), int(timeout_ms)))
        if r.ticket < 0:
            return None
        mesh, out = self._keep.pop(r.ticket)
        return {"ticket": r.ticket, "status": r.status, "t_submit": r.t_submit, "t_start": r.t_start,
                "t_end": r.t_end, "info": SolveInfo(r.info.as_dict()), "out": out}

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib.hg_server_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_ if not k.startswith("reserved")}

    @staticmethod
    def clock() -> float:
        load_library()
        return _lib.hg_server_clock()

    def close(self):
        if getattr(self, "_h", None):
            _lib.hg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
