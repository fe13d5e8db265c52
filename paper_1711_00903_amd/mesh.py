"""Device-resident operator data of one hex mesh at degree N.

Plumbing over the C ABI: torch supplies device memory and the stream; the 1-D
tables come from ``fem_basis_tables`` (host) and the geometric factors from the
``fem_geometric_factors`` kernel.  Every operator call is one libfem launch.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import fem

# storage dtype of the geometric data (G, wJ) and of the field vectors (u) per precision mode
GEO_DTYPE = {fem.FEM_F64: torch.float64, fem.FEM_F32: torch.float32,
             fem.FEM_BF16: torch.bfloat16, fem.FEM_F16: torch.float16,
             fem.FEM_BF16G: torch.bfloat16, fem.FEM_F16G: torch.float16,
             fem.FEM_F32G64: torch.float32, fem.FEM_BF16G64: torch.bfloat16,
             fem.FEM_F16G64: torch.float16}
FIELD_DTYPE = {fem.FEM_F64: torch.float64, fem.FEM_F32: torch.float32,
               fem.FEM_BF16: torch.bfloat16, fem.FEM_F16: torch.float16,
               fem.FEM_BF16G: torch.float32, fem.FEM_F16G: torch.float32,
               fem.FEM_F32G64: torch.float64, fem.FEM_BF16G64: torch.float64,
               fem.FEM_F16G64: torch.float64}
TORCH_DTYPE = FIELD_DTYPE


def out_dtype(prec: int) -> torch.dtype:
    return torch.float64 if FIELD_DTYPE[prec] == torch.float64 else torch.float32


def is_f16(prec: int) -> bool:
    return prec in (fem.FEM_F16, fem.FEM_F16G, fem.FEM_F16G64)


def default_geo_scale(h: float, kind: str) -> float:
    """Power-of-two factor that lifts FP16-stored geometric data of a mesh of
    spacing h into FP16's normal range: metric factors scale like h, scaled
    Jacobians like h^3 (largest entries about 2^10 h resp. 2^10 h^3 before
    scaling)."""
    p = 1 if kind == "G" else 3
    return float(2.0 ** round(np.log2(2.0 ** 10 / max(h, 1e-30) ** p)))


_TUNED = [False]


class DeviceMesh:
    """Element vertices, 1-D tables and lazily built geometric data on one GPU.

    The first instance applies the packaged MI355X tune table (if present)."""

    def __init__(self, N: int, X, device: str | torch.device = "cuda", h: float | None = None):
        if not _TUNED[0]:
            from . import tune
            tune.load()
            _TUNED[0] = True
        self.N = N
        self.nq, self.ng = N + 1, N + 2
        self.np, self.npg = self.nq ** 3, self.ng ** 3
        self.device = torch.device(device)
        Xt = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float64)) if not torch.is_tensor(X) else X
        self.X = Xt.to(self.device, torch.float64).contiguous()
        self.E = int(self.X.shape[0])
        T = fem.fem_basis_tables(N)
        self.host_tables = T
        self.I1d = torch.from_numpy(T["I1d"]).to(self.device)
        self.D1d = torch.from_numpy(T["D1d"]).to(self.device)
        self.Dgl = torch.from_numpy(T["Dgl"]).to(self.device)
        self.h = h if h is not None else 1.0 / max(1.0, round(self.E ** (1.0 / 3.0)))
        self._geo: dict = {}

    # ---------------------------------------------------------------- geometry
    def geo_scale(self, prec: int, kind: str = "G") -> float:
        return default_geo_scale(self.h, kind) if is_f16(prec) else 1.0

    def geometry(self, quad: int, prec: int = fem.FEM_F64, want_G: bool = True,
                 want_wJ: bool = True, kind: str = "G", stream=None):
        """(G [E,6,npq] or None, wJ [E,npq] or None) in storage precision ``prec``
        (FP16 data multiplied by ``geo_scale(prec, kind)``)."""
        key = (quad, prec, want_G, want_wJ, self.geo_scale(prec, kind))
        if key in self._geo:
            return self._geo[key]
        npq = self.np if quad == fem.FEM_QUAD_GLL else self.npg
        dt = GEO_DTYPE[prec]
        G = torch.empty((self.E, 6, npq), dtype=dt, device=self.device) if want_G else None
        wJ = torch.empty((self.E, npq), dtype=dt, device=self.device) if want_wJ else None
        bad = torch.zeros(1, dtype=torch.int64, device=self.device)
        fem.fem_geometric_factors(self.N, self.E, quad, self.X, G, wJ, prec,
                                  self.geo_scale(prec, kind), bad, stream)
        nbad = int(bad.item())
        if nbad:
            raise fem.FemError(fem.FEM_ERR_GEOMETRY, f"fem_geometric_factors ({nbad} nodes)")
        self._geo[key] = (G, wJ)
        return G, wJ

    def drop_geometry(self) -> None:
        self._geo.clear()

    def node_coords(self, quad: int = fem.FEM_QUAD_GLL, stream=None) -> torch.Tensor:
        npq = self.np if quad == fem.FEM_QUAD_GLL else self.npg
        xyz = torch.empty((self.E, npq, 3), dtype=torch.float64, device=self.device)
        fem.fem_node_coords(self.N, self.E, quad, self.X, xyz, stream)
        return xyz

    # ---------------------------------------------------------------- operators
    def _y(self, y, prec):
        if y is None:
            return torch.empty((self.E, self.np), dtype=out_dtype(prec), device=self.device)
        return y

    def mass(self, u, y=None, beta=0.0, prec=fem.FEM_F64, stream=None):
        _, wJ = self.geometry(fem.FEM_QUAD_GL, prec, want_G=False, kind="wJ")
        y = self._y(y, prec)
        fem.fem_mass_apply(self.N, self.E, self.I1d, wJ, u, y, beta, prec,
                           self.geo_scale(prec, "wJ"), stream)
        return y

    def stiff35(self, u, y=None, lam=0.0, beta=0.0, prec=fem.FEM_F64, stream=None):
        G, _ = self.geometry(fem.FEM_QUAD_GLL, prec, want_wJ=False)
        wJ = self.geometry(fem.FEM_QUAD_GLL, prec, want_G=False)[1] if lam else None
        y = self._y(y, prec)
        fem.fem_stiff_collocated_apply(self.N, self.E, self.D1d, G, wJ, lam, u, y, beta, prec,
                                       self.geo_scale(prec), stream)
        return y

    def stiff35_vertices(self, u, y=None, lam=0.0, beta=0.0, stream=None):
        """BP3.5 in FP64 with the geometric factors formed in the kernel from
        the element vertices (no G or wJ in memory)."""
        y = self._y(y, fem.FEM_F64)
        fem.fem_stiff_collocated_vertex_apply(self.N, self.E, self.D1d, self.X, lam, u, y, beta, stream)
        return y

    def stiff30_vertices(self, u, y=None, lam=0.0, beta=0.0, stream=None):
        """BP3.0 in FP64 with the geometric factors formed in the kernel from
        the element vertices (no G or wJ in memory)."""
        y = self._y(y, fem.FEM_F64)
        fem.fem_stiff_dealiased_vertex_apply(self.N, self.E, self.I1d, self.Dgl, self.X, lam, u, y, beta, stream)
        return y

    def stiff30(self, u, y=None, lam=0.0, beta=0.0, prec=fem.FEM_F64, stream=None):
        G, _ = self.geometry(fem.FEM_QUAD_GL, prec, want_wJ=False)
        wJ = self.geometry(fem.FEM_QUAD_GL, prec, want_G=False)[1] if lam else None
        y = self._y(y, prec)
        fem.fem_stiff_dealiased_apply(self.N, self.E, self.I1d, self.Dgl, G, wJ, lam, u, y, beta,
                                      prec, self.geo_scale(prec), stream)
        return y

    # ---------------------------------------------------------------- CG
    def cg_structs(self, lam: float = 1.0, mode: int = 0, inner_prec: int = fem.FEM_F32,
                   rtol: float = 1e-10, max_iters: int = 20000, delta: float = 0.1,
                   check_every: int = 1, fusion: int = fem.FEM_CG_FUSE_AUTO, history: int = 0):
        """(fem_cg_operator, fem_cg_options, history buffer) of a solve of
        (S + lam M) x = b on this mesh, with the geometric data it needs built."""
        G64, _ = self.geometry(fem.FEM_QUAD_GLL, fem.FEM_F64, want_wJ=False)
        _, wJ64 = self.geometry(fem.FEM_QUAD_GL, fem.FEM_F64, want_G=False, kind="wJ")
        op = fem.CgOperator(N=self.N, E=self.E, I1d=self.I1d.data_ptr(), D1d=self.D1d.data_ptr(),
                            G=G64.data_ptr(), wJ=wJ64.data_ptr() if lam else None, lam=lam,
                            inner_prec=inner_prec)
        if mode != 0:
            Glo, _ = self.geometry(fem.FEM_QUAD_GLL, inner_prec, want_wJ=False)
            _, wJlo = self.geometry(fem.FEM_QUAD_GL, inner_prec, want_G=False, kind="wJ")
            op.G_lo = Glo.data_ptr()
            op.wJ_lo = wJlo.data_ptr() if lam else None
            op.geo_scale_G = self.geo_scale(inner_prec, "G")
            op.geo_scale_wJ = self.geo_scale(inner_prec, "wJ")
        hist = (ctypes.c_double * max(1, history))()
        opt = fem.CgOptions(mode=mode, rtol=rtol, max_iters=max_iters, delta=delta,
                            check_every=check_every, fusion=int(fusion),
                            history=ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)) if history else None,
                            history_len=history)
        return op, opt, hist

    def cg_solve(self, b, x, lam: float = 1.0, mode: int = 0, inner_prec: int = fem.FEM_F32,
                 rtol: float = 1e-10, max_iters: int = 20000, delta: float = 0.1,
                 check_every: int = 1, fusion: int = fem.FEM_CG_FUSE_AUTO, history: int = 0,
                 stream=None, noalloc: bool = False) -> dict:
        """Solve (S + lam M) x = b with libfem's CG; b, x FP64 [E, Np] device tensors.
        With noalloc, through fem_cg_solve_noalloc (the library's own workspace)."""
        op, opt, hist = self.cg_structs(lam, mode, inner_prec, rtol, max_iters, delta, check_every, fusion,
                                        history)
        if noalloc:
            rep = fem.fem_cg_solve_noalloc(op, opt, b, x, stream)
        else:
            nbytes = fem.fem_cg_workspace_bytes(op, opt)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            rep = fem.fem_cg_solve(op, opt, b, x, ws, nbytes, stream)
            del ws
        out = rep.as_dict()
        if history:
            out["history"] = list(hist[:rep.history_count])
        return out

    # ---------------------------------------------------------------- assembled operator
    def set_assembly(self, gather: np.ndarray, n_global: int) -> None:
        """The global numbering of this mesh's nodes (gather [E, Np] int32 host
        array): the device gather map and its inverse (fem_assembly_inverse_map)."""
        off, loc = fem.fem_assembly_inverse_map(gather, n_global)
        self.n_global = int(n_global)
        self._gather = torch.from_numpy(np.ascontiguousarray(gather, dtype=np.int32)).to(self.device)
        self._offsets = torch.from_numpy(off).to(self.device)
        self._locals = torch.from_numpy(loc).to(self.device)
        self.asm = fem.Assembly(n_global=self.n_global, gather=self._gather.data_ptr(),
                                offsets=self._offsets.data_ptr(), locals=self._locals.data_ptr())

    def _assembled_ws(self, op):
        nbytes = fem.fem_assembled_workspace_bytes(op, self.asm)
        if nbytes == 0:
            raise fem.FemError(fem.FEM_ERR_ARG, "fem_assembled_workspace_bytes")
        return torch.empty(nbytes, dtype=torch.uint8, device=self.device), nbytes

    def assembled_apply(self, ug, lam: float = 1.0, yg=None, stream=None):
        """yg = Z^T (S + lam M) Z ug on the global nodes (FP64)."""
        op, _, _ = self.cg_structs(lam)
        yg = torch.empty(self.n_global, dtype=torch.float64, device=self.device) if yg is None else yg
        ws, nbytes = self._assembled_ws(op)
        fem.fem_assembled_apply(op, self.asm, ug, yg, ws, nbytes, stream)
        return yg

    def assembled_diagonal(self, lam: float = 1.0, stream=None):
        op, _, _ = self.cg_structs(lam)
        d = torch.empty(self.n_global, dtype=torch.float64, device=self.device)
        ws, nbytes = self._assembled_ws(op)
        fem.fem_assembled_diagonal(op, self.asm, d, ws, nbytes, stream)
        return d

    def pcg_solve(self, b, x, lam: float = 1.0, jacobi: bool = True, rtol: float = 1e-10,
                  max_iters: int = 20000, check_every: int = 1, history: int = 0, stream=None) -> dict:
        """Jacobi-PCG (or plain CG with jacobi=False) on the assembled system;
        b, x FP64 [n_global] device tensors."""
        op, opt, hist = self.cg_structs(lam, 0, 0, rtol, max_iters, 0.1, check_every, 0, history)
        ws, nbytes = self._assembled_ws(op)
        diag = None
        if jacobi:
            diag = torch.empty(self.n_global, dtype=torch.float64, device=self.device)
            fem.fem_assembled_diagonal(op, self.asm, diag, ws, nbytes, stream)
        rep = fem.fem_pcg_solve(op, self.asm, opt, diag, b, x, ws, nbytes, stream)
        del ws
        out = rep.as_dict()
        if history:
            out["history"] = list(hist[:rep.history_count])
        return out

    # ---------------------------------------------------------------- batches
    def desc(self, op: str, u, y, prec: int = fem.FEM_F64, lam: float = 0.0, beta: float = 0.0):
        """Descriptor (fem_apply_desc) of one apply on this mesh, for fem_batch_*."""
        d = fem.ApplyDesc(op=fem.OP_NAMES[op], N=self.N, E=self.E, prec=prec, lam=lam, beta=beta,
                          u=u.data_ptr(), y=y.data_ptr())
        if op == "BP10":
            _, wJ = self.geometry(fem.FEM_QUAD_GL, prec, want_G=False, kind="wJ")
            d.I1d, d.wJ, d.geo_scale = self.I1d.data_ptr(), wJ.data_ptr(), self.geo_scale(prec, "wJ")
        else:
            quad = fem.FEM_QUAD_GLL if op == "BP35" else fem.FEM_QUAD_GL
            G, _ = self.geometry(quad, prec, want_wJ=False)
            d.G, d.geo_scale = G.data_ptr(), self.geo_scale(prec)
            if lam:
                d.wJ = self.geometry(quad, prec, want_G=False)[1].data_ptr()
            if op == "BP35":
                d.D1d = self.D1d.data_ptr()
            else:
                d.I1d, d.Dgl = self.I1d.data_ptr(), self.Dgl.data_ptr()
        return d
