"""FP64 CPU oracle for the BP1.0 / BP3.5 / BP3.0 tensor-product operators.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library (``paper_1711_00903_amd``) and neither imports the other; the
only common module is :mod:`workloads`, which draws seeded random inputs and
holds none of the method's arithmetic.

Two tiers, both written from the paper (arXiv 1711.00903):

* ``fem_oracle.c`` (O2): the sum-factorised element loops of Alg. 1-5 in plain
  C with OpenMP over elements, plus the quadrature rules, 1-D tables and
  trilinear geometric factors.
* :mod:`oracle.dense` (O1): the element matrices of eqs. (massQuad),
  (stiffQuad) and (stiffQuad2) assembled explicitly as Kronecker products
  (``M^e = I^T J^e I``, ``S^e = D^T G^e D``) and applied as dense products.

What pins each function to something other than itself is listed in the
test-suite (``tests/test_oracle_*.py``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAXN = 15

_dp = C.POINTER(C.c_double)


def build(force: bool = False) -> str:
    """Compile ``fem_oracle.c`` into ``liboracle.so`` with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                        "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


@lru_cache(maxsize=1)
def lib() -> C.CDLL:
    build()
    L = C.CDLL(_LIB)
    i64 = C.c_int64
    L.ora_gl.argtypes = [C.c_int, _dp, _dp]
    L.ora_gll.argtypes = [C.c_int, _dp, _dp]
    L.ora_tables.argtypes = [C.c_int] + [_dp] * 7
    L.ora_geometry.argtypes = [C.c_int, i64, C.c_int, _dp, _dp, _dp]
    L.ora_geometry.restype = i64
    L.ora_node_coords.argtypes = [C.c_int, i64, C.c_int, _dp, _dp]
    L.ora_bp10.argtypes = [C.c_int, i64, _dp, _dp, _dp, _dp, C.c_int]
    L.ora_bp35.argtypes = [C.c_int, i64, _dp, _dp, _dp, C.c_double, _dp, _dp, C.c_int]
    L.ora_bp30.argtypes = [C.c_int, i64, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp, C.c_int]
    L.ora_set_threads.argtypes = [C.c_int]
    L.ora_cg_residual_ld.argtypes = [C.c_int, i64, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp, _dp]
    L.ora_set_threads.restype = C.c_int
    return L


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "oracle wants C-contiguous float64"
    return a.ctypes.data_as(_dp)


def set_threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count of the oracle."""
    return int(lib().ora_set_threads(n))


def gl(n: int):
    """n-point Gauss-Legendre nodes and weights (ascending)."""
    r, w = np.zeros(n), np.zeros(n)
    if lib().ora_gl(n, _p(r), _p(w)):
        raise ValueError(n)
    return r, w


def gll(N: int):
    """(N+1)-point Gauss-Lobatto-Legendre nodes and weights (ascending)."""
    r, w = np.zeros(N + 1), np.zeros(N + 1)
    if lib().ora_gll(N, _p(r), _p(w)):
        raise ValueError(N)
    return r, w


class Tables:
    """1-D nodes, weights and operator tables for degree N."""

    def __init__(self, N: int):
        nq, ng = N + 1, N + 2
        self.N, self.nq, self.ng = N, nq, ng
        self.rgll, self.wgll = np.zeros(nq), np.zeros(nq)
        self.rgl, self.wgl = np.zeros(ng), np.zeros(ng)
        self.I = np.zeros((ng, nq))
        self.D = np.zeros((nq, nq))
        self.Dgl = np.zeros((ng, ng))
        if lib().ora_tables(N, _p(self.rgll), _p(self.wgll), _p(self.rgl), _p(self.wgl),
                            _p(self.I), _p(self.D), _p(self.Dgl)):
            raise ValueError(N)


@lru_cache(maxsize=32)
def tables(N: int) -> Tables:
    return Tables(N)


def geometry(N: int, X: np.ndarray, quad: str, want_G: bool = True, want_wJ: bool = True):
    """Geometric factors at GLL (quad='gll') or GL (quad='gl') nodes.

    X: (E, 8, 3) element vertices.  Returns (G (E, 6, npq) or None, wJ (E, npq) or None).
    Raises if any node has detJ <= 0.
    """
    X = np.ascontiguousarray(X, dtype=np.float64)
    E = X.shape[0]
    q = {"gll": 0, "gl": 1}[quad]
    nq = N + 1 + q
    npq = nq ** 3
    G = np.zeros((E, 6, npq)) if want_G else None
    wJ = np.zeros((E, npq)) if want_wJ else None
    bad = lib().ora_geometry(N, E, q, _p(X), _p(G), _p(wJ))
    if bad != 0:
        raise ValueError(f"geometry: {bad} nodes with non-positive Jacobian")
    return G, wJ


def node_coords(N: int, X: np.ndarray, quad: str = "gll") -> np.ndarray:
    """Physical coordinates (E, npq, 3) of the tensor nodes under the trilinear map."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    q = {"gll": 0, "gl": 1}[quad]
    nq = N + 1 + q
    out = np.zeros((X.shape[0], nq ** 3, 3))
    lib().ora_node_coords(N, X.shape[0], q, _p(X), _p(out))
    return out


def _out(y, shape, accumulate):
    if y is None:
        if accumulate:
            raise ValueError("accumulate needs y")
        return np.zeros(shape)
    return y


def bp10(N: int, wJ: np.ndarray, u: np.ndarray, y: np.ndarray | None = None,
         accumulate: bool = False) -> np.ndarray:
    """Mass operator BP1.0 (Alg. 3), wJ at GL nodes."""
    T = tables(N)
    u = np.ascontiguousarray(u, dtype=np.float64)
    wJ = np.ascontiguousarray(wJ, dtype=np.float64)
    E = u.shape[0]
    y = _out(y, u.shape, accumulate)
    lib().ora_bp10(N, E, _p(T.I), _p(wJ), _p(u), _p(y), int(accumulate))
    return y


def bp35(N: int, G: np.ndarray, u: np.ndarray, wJ: np.ndarray | None = None,
         lam: float = 0.0, y: np.ndarray | None = None, accumulate: bool = False) -> np.ndarray:
    """Collocated stiffness BP3.5 (Alg. 4), G and wJ at GLL nodes."""
    T = tables(N)
    u = np.ascontiguousarray(u, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    if wJ is not None:
        wJ = np.ascontiguousarray(wJ, dtype=np.float64)
    y = _out(y, u.shape, accumulate)
    if lib().ora_bp35(N, u.shape[0], _p(T.D), _p(G), _p(wJ), float(lam), _p(u), _p(y),
                      int(accumulate)):
        raise ValueError("ora_bp35 arguments")
    return y


def bp30(N: int, G: np.ndarray, u: np.ndarray, wJ: np.ndarray | None = None,
         lam: float = 0.0, y: np.ndarray | None = None, accumulate: bool = False) -> np.ndarray:
    """De-aliased stiffness BP3.0 (Alg. 5), G and wJ at GL nodes."""
    T = tables(N)
    u = np.ascontiguousarray(u, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    if wJ is not None:
        wJ = np.ascontiguousarray(wJ, dtype=np.float64)
    y = _out(y, u.shape, accumulate)
    if lib().ora_bp30(N, u.shape[0], _p(T.I), _p(T.Dgl), _p(G), _p(wJ), float(lam), _p(u),
                      _p(y), int(accumulate)):
        raise ValueError("ora_bp30 arguments")
    return y


class Problem:
    """Oracle-side operators of one mesh (element vertices X) at degree N.

    Builds the geometric data it needs lazily, with the oracle's own geometry.
    """

    def __init__(self, N: int, X: np.ndarray):
        self.N = N
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.E = self.X.shape[0]
        self._g = {}

    def _geo(self, quad):
        if quad not in self._g:
            self._g[quad] = geometry(self.N, self.X, quad)
        return self._g[quad]

    def G_gll(self):
        return self._geo("gll")[0]

    def wJ_gll(self):
        return self._geo("gll")[1]

    def G_gl(self):
        return self._geo("gl")[0]

    def wJ_gl(self):
        return self._geo("gl")[1]

    def mass(self, u):
        return bp10(self.N, self.wJ_gl(), u)

    def stiff35(self, u, lam=0.0):
        return bp35(self.N, self.G_gll(), u, self.wJ_gll() if lam else None, lam)

    def stiff30(self, u, lam=0.0):
        return bp30(self.N, self.G_gl(), u, self.wJ_gl() if lam else None, lam)

    def cg_residual_ld(self, x, b, lam=1.0) -> tuple[float, float]:
        """(||b - (S + lam M) x||^2, ||b||^2) with every operation in long double
        (fem_oracle.c: ora_cg_residual_ld)."""
        T = tables(self.N)
        x = np.ascontiguousarray(x, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        E = x.shape[0]
        out = np.zeros(2)
        wJ = self.wJ_gl() if lam else np.zeros(1)
        st = lib().ora_cg_residual_ld(self.N, E, _p(np.ascontiguousarray(T.I)), _p(np.ascontiguousarray(T.D)),
                                      _p(self.G_gll()), _p(wJ), float(lam), _p(x), _p(b), _p(out))
        if st:
            raise ValueError("ora_cg_residual_ld: bad arguments")
        return float(out[0]), float(out[1])

    def cg_operator(self, u, lam=1.0):
        """A u = S3.5 u + lam * M1.0 u (the operator of the CG workload)."""
        y = self.stiff35(u)
        return bp10(self.N, self.wJ_gl(), u * lam, y=y, accumulate=True) if lam else y
