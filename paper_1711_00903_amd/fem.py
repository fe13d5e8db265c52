"""Python binding of libfem (``include/fem.h``): argument marshalling only.

Every function has the name and argument order of its C entry point.  Array
arguments may be torch tensors (their ``data_ptr()`` is passed) or raw integer
addresses; ``stream`` may be a ``torch.cuda.Stream``, a raw ``hipStream_t``
integer, or None for torch's current stream.  All compute runs in the HIP
kernels of libfem; there is no fallback: if the library is missing, importing
:func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from functools import lru_cache

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfem.so")

FEM_OK = 0
FEM_ERR_ARG = 1
FEM_ERR_UNSUPPORTED = 2
FEM_ERR_ALIGN = 3
FEM_ERR_HIP = 4
FEM_ERR_NOT_CONVERGED = 5
FEM_ERR_BREAKDOWN = 6
FEM_ERR_WORKSPACE = 7
FEM_ERR_GEOMETRY = 8

FEM_F64, FEM_F32, FEM_BF16, FEM_F16, FEM_BF16G, FEM_F16G = 0, 1, 2, 3, 4, 5
FEM_F32G64, FEM_BF16G64, FEM_F16G64 = 6, 7, 8
FEM_OP_BP10, FEM_OP_BP35, FEM_OP_BP30 = 0, 1, 2
FEM_QUAD_GLL, FEM_QUAD_GL = 0, 1
FEM_CG_FUSE_AUTO, FEM_CG_FUSE_NONE, FEM_CG_FUSE_ONEPASS = 0, 1, 2
FUSION_NAMES = {"auto": FEM_CG_FUSE_AUTO, "none": FEM_CG_FUSE_NONE, "onepass": FEM_CG_FUSE_ONEPASS}

PREC_NAMES = {"f64": FEM_F64, "f32": FEM_F32, "bf16": FEM_BF16, "f16": FEM_F16,
              "bf16g": FEM_BF16G, "f16g": FEM_F16G, "f32g64": FEM_F32G64,
              "bf16g64": FEM_BF16G64, "f16g64": FEM_F16G64}
OP_NAMES = {"BP10": FEM_OP_BP10, "BP35": FEM_OP_BP35, "BP30": FEM_OP_BP30}


class FemError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} (status {status})")


_vp = C.c_void_p
_i64 = C.c_int64
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)

class CgOperator(C.Structure):
    _fields_ = [("N", C.c_int), ("E", C.c_int64), ("I1d", C.c_void_p), ("D1d", C.c_void_p),
                ("G", C.c_void_p), ("wJ", C.c_void_p), ("lam", C.c_double), ("inner_prec", C.c_int),
                ("G_lo", C.c_void_p), ("wJ_lo", C.c_void_p), ("geo_scale_G", C.c_float),
                ("geo_scale_wJ", C.c_float)]


class CgOptions(C.Structure):
    _fields_ = [("mode", C.c_int), ("rtol", C.c_double), ("max_iters", C.c_int),
                ("delta", C.c_double), ("check_every", C.c_int), ("fusion", C.c_int),
                ("history", C.POINTER(C.c_double)), ("history_len", C.c_int)]


class CgReport(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("reliable_updates", C.c_int),
                ("hi_matvecs", C.c_int), ("history_count", C.c_int), ("rel_res", C.c_double),
                ("ms", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Assembly(C.Structure):
    _fields_ = [("n_global", C.c_int64), ("gather", C.c_void_p), ("offsets", C.c_void_p), ("locals", C.c_void_p)]


class ApplyDesc(C.Structure):
    _fields_ = [("op", C.c_int), ("N", C.c_int), ("E", C.c_int64), ("prec", C.c_int),
                ("I1d", C.c_void_p), ("D1d", C.c_void_p), ("Dgl", C.c_void_p), ("G", C.c_void_p),
                ("wJ", C.c_void_p), ("lam", C.c_double), ("beta", C.c_double), ("geo_scale", C.c_float),
                ("u", C.c_void_p), ("y", C.c_void_p)]


_SIGS = {
    "fem_status_str": ([C.c_int], C.c_char_p),
    "fem_version": ([], C.c_int),
    "fem_build_id": ([], C.c_char_p),
    "fem_max_degree": ([], C.c_int),
    "fem_max_elements": ([], _i64),
    "fem_basis_tables": ([C.c_int] + [_dp] * 7, C.c_int),
    "fem_geometric_factors": ([C.c_int, _i64, C.c_int, _vp, _vp, _vp, C.c_int, C.c_float, _vp, _vp],
                              C.c_int),
    "fem_node_coords": ([C.c_int, _i64, C.c_int, _vp, _vp, _vp], C.c_int),
    "fem_geo_vector_width": ([C.c_int, C.c_int, C.c_int], C.c_int),
    "fem_mass_apply": ([C.c_int, _i64, _vp, _vp, _vp, _vp, C.c_double, C.c_int, C.c_float, _vp],
                       C.c_int),
    "fem_stiff_collocated_apply": ([C.c_int, _i64, _vp, _vp, _vp, C.c_double, _vp, _vp, C.c_double,
                                    C.c_int, C.c_float, _vp], C.c_int),
    "fem_stiff_collocated_vertex_apply": ([C.c_int, _i64, _vp, _vp, C.c_double, _vp, _vp, C.c_double, _vp],
                                          C.c_int),
    "fem_stiff_dealiased_vertex_apply": ([C.c_int, _i64, _vp, _vp, _vp, C.c_double, _vp, _vp, C.c_double,
                                          _vp], C.c_int),
    "fem_stiff_dealiased_apply": ([C.c_int, _i64, _vp, _vp, _vp, _vp, C.c_double, _vp, _vp,
                                   C.c_double, C.c_int, C.c_float, _vp], C.c_int),
    "fem_stream_copy": ([_vp, _vp, C.c_size_t, _vp], C.c_int),
    "fem_lds_bandwidth": ([C.c_int, _i64, C.c_int, _vp, _vp], C.c_int),
    "fem_cg_workspace_bytes": ([C.POINTER(CgOperator), C.POINTER(CgOptions)], C.c_size_t),
    "fem_cg_solve": ([C.POINTER(CgOperator), C.POINTER(CgOptions), _vp, _vp, _vp, C.c_size_t,
                      C.POINTER(CgReport), _vp], C.c_int),
    "fem_cg_solve_noalloc": ([C.POINTER(CgOperator), C.POINTER(CgOptions), _vp, _vp, C.POINTER(CgReport), _vp],
                             C.c_int),
    "fem_assembly_inverse_map": ([_i64, _vp, _i64, _vp, _vp], C.c_int),
    "fem_gather": ([_i64, _i64, _vp, _vp, _vp, _vp], C.c_int),
    "fem_scatter": ([_i64, _i64, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "fem_assembled_workspace_bytes": ([C.POINTER(CgOperator), C.POINTER(Assembly)], C.c_size_t),
    "fem_assembled_apply": ([C.POINTER(CgOperator), C.POINTER(Assembly), _vp, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "fem_assembled_diagonal": ([C.POINTER(CgOperator), C.POINTER(Assembly), _vp, _vp, C.c_size_t, _vp], C.c_int),
    "fem_pcg_solve": ([C.POINTER(CgOperator), C.POINTER(Assembly), C.POINTER(CgOptions), _vp, _vp, _vp, _vp,
                       C.c_size_t, C.POINTER(CgReport), _vp], C.c_int),
    "fem_batch_apply": ([C.POINTER(ApplyDesc), C.c_int, _vp], C.c_int),
    "fem_batch_graph_create": ([C.POINTER(ApplyDesc), C.c_int, C.c_int, _vp, C.POINTER(C.c_void_p)], C.c_int),
    "fem_batch_graph_launch": ([_vp, _vp], C.c_int),
    "fem_batch_graph_destroy": ([_vp], C.c_int),
    "fem_tune_load": ([C.c_char_p], C.c_int),
    "fem_tune_set": ([C.c_int] * 5, C.c_int),
    "fem_tune_get": ([C.c_int, C.c_int, C.c_int, _ip, _ip], C.c_int),
    "fem_kernel_info": ([C.c_int] * 4 + [_ip, _ip], C.c_int),
    "fem_supported_epb": ([C.c_int] * 3 + [_ip, C.c_int], C.c_int),
}


@lru_cache(maxsize=1)
def lib() -> C.CDLL:
    """Load libfem.so (built in-tree by ``__graft_entry__.build()``)."""
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libfem.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


def symbols() -> list[str]:
    return list(_SIGS)


def status_str(status: int) -> str:
    return lib().fem_status_str(int(status)).decode()


def _check(status: int, where: str) -> None:
    if status != FEM_OK:
        raise FemError(status, where)


def _ptr(x):
    """Device/host address of a tensor, or an integer address, or NULL."""
    if x is None:
        return None
    if isinstance(x, int):
        return x or None
    return x.data_ptr() or None


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(s, int):
        return s or None
    return s.cuda_stream or None


# ---------------------------------------------------------------- host entry points

def fem_version() -> int:
    return lib().fem_version()


def fem_build_id() -> str:
    return lib().fem_build_id().decode()


def fem_max_degree() -> int:
    return lib().fem_max_degree()


def fem_basis_tables(N: int) -> dict:
    """Quadrature rules and 1-D tables of degree N as host float64 arrays."""
    nq, ng = N + 1, N + 2
    out = dict(r_gll=np.zeros(nq), w_gll=np.zeros(nq), r_gl=np.zeros(ng), w_gl=np.zeros(ng),
               I1d=np.zeros((ng, nq)), D1d=np.zeros((nq, nq)), Dgl=np.zeros((ng, ng)))
    args = [out[k].ctypes.data_as(_dp) for k in ("r_gll", "w_gll", "r_gl", "w_gl", "I1d", "D1d", "Dgl")]
    _check(lib().fem_basis_tables(N, *args), "fem_basis_tables")
    return out


def fem_tune_set(op: int, N: int, prec: int, epb: int = 0, grid_cap: int = 0) -> None:
    _check(lib().fem_tune_set(op, N, prec, epb, grid_cap), "fem_tune_set")


def fem_tune_get(op: int, N: int, prec: int) -> tuple[int, int]:
    e, c = C.c_int(), C.c_int()
    _check(lib().fem_tune_get(op, N, prec, C.byref(e), C.byref(c)), "fem_tune_get")
    return e.value, c.value


def fem_kernel_info(op: int, N: int, prec: int, epb: int = 0) -> tuple[int, int]:
    th, lds = C.c_int(), C.c_int()
    _check(lib().fem_kernel_info(op, N, prec, epb, C.byref(th), C.byref(lds)), "fem_kernel_info")
    return th.value, lds.value


def fem_supported_epb(op: int, N: int, prec: int) -> list[int]:
    buf = (C.c_int * 8)()
    n = lib().fem_supported_epb(op, N, prec, buf, 8)
    if n < 0:
        raise FemError(-n, "fem_supported_epb")
    return list(buf[:n])


def fem_geo_vector_width(N: int, quad: int, prec: int) -> int:
    w = lib().fem_geo_vector_width(N, quad, prec)
    if w <= 0:
        raise FemError(FEM_ERR_ARG, "fem_geo_vector_width")
    return w


def geo_layout_offsets(n: int, W: int) -> np.ndarray:
    """Stored offset of each node (natural order i + n j + n^2 k) inside one
    factor block of the interleaved geometric-data layout of fem.h."""
    k, col = np.divmod(np.arange(n ** 3), n * n)
    return ((k // W) * n * n + col) * W + k % W


# ---------------------------------------------------------------- device entry points

def fem_geometric_factors(N, E, quad, X, G, wJ, prec=FEM_F64, geo_scale=1.0, bad_count=None,
                          stream=None) -> None:
    _check(lib().fem_geometric_factors(N, E, quad, _ptr(X), _ptr(G), _ptr(wJ), prec, geo_scale,
                                       _ptr(bad_count), _stream(stream)), "fem_geometric_factors")


def fem_node_coords(N, E, quad, X, xyz, stream=None) -> None:
    _check(lib().fem_node_coords(N, E, quad, _ptr(X), _ptr(xyz), _stream(stream)), "fem_node_coords")


def fem_mass_apply(N, E, I1d, wJ, u, y, beta=0.0, prec=FEM_F64, geo_scale=1.0, stream=None) -> None:
    _check(lib().fem_mass_apply(N, E, _ptr(I1d), _ptr(wJ), _ptr(u), _ptr(y), beta, prec, geo_scale,
                                _stream(stream)), "fem_mass_apply")


def fem_stiff_collocated_apply(N, E, D1d, G, wJ, lam, u, y, beta=0.0, prec=FEM_F64, geo_scale=1.0,
                               stream=None) -> None:
    _check(lib().fem_stiff_collocated_apply(N, E, _ptr(D1d), _ptr(G), _ptr(wJ), lam, _ptr(u), _ptr(y),
                                            beta, prec, geo_scale, _stream(stream)),
           "fem_stiff_collocated_apply")


def fem_stiff_collocated_vertex_apply(N, E, D1d, X, lam, u, y, beta=0.0, stream=None) -> None:
    _check(lib().fem_stiff_collocated_vertex_apply(N, E, _ptr(D1d), _ptr(X), lam, _ptr(u), _ptr(y), beta,
                                                   _stream(stream)), "fem_stiff_collocated_vertex_apply")


def fem_stiff_dealiased_vertex_apply(N, E, I1d, Dgl, X, lam, u, y, beta=0.0, stream=None) -> None:
    _check(lib().fem_stiff_dealiased_vertex_apply(N, E, _ptr(I1d), _ptr(Dgl), _ptr(X), lam, _ptr(u), _ptr(y),
                                                  beta, _stream(stream)), "fem_stiff_dealiased_vertex_apply")


def fem_stiff_dealiased_apply(N, E, I1d, Dgl, G, wJ, lam, u, y, beta=0.0, prec=FEM_F64,
                              geo_scale=1.0, stream=None) -> None:
    _check(lib().fem_stiff_dealiased_apply(N, E, _ptr(I1d), _ptr(Dgl), _ptr(G), _ptr(wJ), lam,
                                           _ptr(u), _ptr(y), beta, prec, geo_scale, _stream(stream)),
           "fem_stiff_dealiased_apply")


def fem_stream_copy(src, dst, nbytes: int, stream=None) -> None:
    _check(lib().fem_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)), "fem_stream_copy")


def fem_lds_bandwidth(mode: int, workgroups: int, iters: int, sink, stream=None) -> None:
    _check(lib().fem_lds_bandwidth(mode, workgroups, iters, _ptr(sink), _stream(stream)), "fem_lds_bandwidth")


def fem_cg_workspace_bytes(op: CgOperator, opt: CgOptions) -> int:
    return int(lib().fem_cg_workspace_bytes(C.byref(op), C.byref(opt)))


def fem_cg_solve(op: CgOperator, opt: CgOptions, b, x, workspace, workspace_bytes: int,
                 stream=None, raise_on_error: bool = True) -> CgReport:
    """Blocking CG solve; returns the report.  FEM_ERR_NOT_CONVERGED and
    FEM_ERR_BREAKDOWN are returned in the report (not raised) unless
    raise_on_error and the status is an argument / runtime error."""
    rep = CgReport()
    st = lib().fem_cg_solve(C.byref(op), C.byref(opt), _ptr(b), _ptr(x), _ptr(workspace),
                            workspace_bytes, C.byref(rep), _stream(stream))
    if raise_on_error and st not in (FEM_OK, FEM_ERR_NOT_CONVERGED, FEM_ERR_BREAKDOWN):
        raise FemError(st, "fem_cg_solve")
    return rep


# FEM_CG_NOALLOC_BYTES of include/fem.h: the device array fem_cg_solve_noalloc works in
FEM_CG_NOALLOC_BYTES = 64 << 20


def fem_cg_solve_noalloc(op: CgOperator, opt: CgOptions, b, x, stream=None,
                         raise_on_error: bool = True) -> CgReport:
    """fem_cg_solve with the library's own device workspace (no allocation);
    statuses as for fem_cg_solve."""
    rep = CgReport()
    st = lib().fem_cg_solve_noalloc(C.byref(op), C.byref(opt), _ptr(b), _ptr(x), C.byref(rep), _stream(stream))
    if raise_on_error and st not in (FEM_OK, FEM_ERR_NOT_CONVERGED, FEM_ERR_BREAKDOWN):
        raise FemError(st, "fem_cg_solve_noalloc")
    return rep


def fem_assembly_inverse_map(gather: np.ndarray, n_global: int) -> tuple[np.ndarray, np.ndarray]:
    """(offsets [n_global + 1], locals [n_local]) int32 host arrays of a host
    int32 gather map."""
    g = np.ascontiguousarray(gather, dtype=np.int32).ravel()
    off = np.zeros(n_global + 1, dtype=np.int32)
    loc = np.zeros(g.size, dtype=np.int32)
    _check(lib().fem_assembly_inverse_map(g.size, g.ctypes.data, n_global, off.ctypes.data, loc.ctypes.data),
           "fem_assembly_inverse_map")
    return off, loc


def fem_gather(n_local, n_global, gather, ug, ul, stream=None) -> None:
    _check(lib().fem_gather(n_local, n_global, _ptr(gather), _ptr(ug), _ptr(ul), _stream(stream)), "fem_gather")


def fem_scatter(n_local, n_global, offsets, locals_, ul, ug, stream=None) -> None:
    _check(lib().fem_scatter(n_local, n_global, _ptr(offsets), _ptr(locals_), _ptr(ul), _ptr(ug), _stream(stream)),
           "fem_scatter")


def fem_assembled_workspace_bytes(op: CgOperator, asm: Assembly) -> int:
    return int(lib().fem_assembled_workspace_bytes(C.byref(op), C.byref(asm)))


def fem_assembled_apply(op: CgOperator, asm: Assembly, ug, yg, workspace, workspace_bytes: int,
                        stream=None) -> None:
    _check(lib().fem_assembled_apply(C.byref(op), C.byref(asm), _ptr(ug), _ptr(yg), _ptr(workspace),
                                     workspace_bytes, _stream(stream)), "fem_assembled_apply")


def fem_assembled_diagonal(op: CgOperator, asm: Assembly, diag, workspace, workspace_bytes: int,
                           stream=None) -> None:
    _check(lib().fem_assembled_diagonal(C.byref(op), C.byref(asm), _ptr(diag), _ptr(workspace), workspace_bytes,
                                        _stream(stream)), "fem_assembled_diagonal")


def fem_pcg_solve(op: CgOperator, asm: Assembly, opt: CgOptions, diag, b, x, workspace, workspace_bytes: int,
                  stream=None, raise_on_error: bool = True) -> CgReport:
    """Blocking Jacobi-PCG solve on the assembled operator; returns the report
    (FEM_ERR_NOT_CONVERGED / FEM_ERR_BREAKDOWN in the report, as for
    fem_cg_solve)."""
    rep = CgReport()
    st = lib().fem_pcg_solve(C.byref(op), C.byref(asm), C.byref(opt), _ptr(diag), _ptr(b), _ptr(x),
                             _ptr(workspace), workspace_bytes, C.byref(rep), _stream(stream))
    if raise_on_error and st not in (FEM_OK, FEM_ERR_NOT_CONVERGED, FEM_ERR_BREAKDOWN):
        raise FemError(st, "fem_pcg_solve")
    return rep


def fem_tune_load(text: str) -> None:
    _check(lib().fem_tune_load(text.encode()), "fem_tune_load")


def _desc_array(descs):
    arr = (ApplyDesc * max(1, len(descs)))()
    for i, d in enumerate(descs):
        arr[i] = d
    return arr


def fem_batch_apply(descs: list, stream=None) -> None:
    arr = _desc_array(descs)
    _check(lib().fem_batch_apply(arr, len(descs), _stream(stream)), "fem_batch_apply")


class BatchGraph:
    """A captured ragged batch (fem_batch_graph_*); keeps its descriptors alive."""

    def __init__(self, descs: list, lanes: int = 4, stream=None):
        self._arr = _desc_array(descs)
        self._descs = descs
        h = C.c_void_p()
        _check(lib().fem_batch_graph_create(self._arr, len(descs), lanes, _stream(stream), C.byref(h)),
               "fem_batch_graph_create")
        self.handle = h

    def launch(self, stream=None) -> None:
        _check(lib().fem_batch_graph_launch(self.handle, _stream(stream)), "fem_batch_graph_launch")

    def destroy(self) -> None:
        if self.handle:
            _check(lib().fem_batch_graph_destroy(self.handle), "fem_batch_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
