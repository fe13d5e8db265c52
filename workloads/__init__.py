"""Seeded synthetic inputs for the hexahedral tensor-product operators.

This module is shared by the oracle-side checks and by the GPU-side tests and
benchmark.  It holds none of the method's arithmetic: no quadrature nodes, no
basis tables, no geometric factors and no operator.  It produces only

* the vertices of a structured ``n^3`` hex grid of the unit cube whose interior
  vertices are displaced at random (every element is then the trilinear image of
  the reference cube through its 8 vertices, Problem description section);
* the element-to-vertex gathering of that grid (element vertex order
  ``a + 2 b + 4 c`` for the corner at ``r = +-1, s = +-1, t = +-1``);
* the global numbering of the degree-N tensor nodes of that grid: local node
  ``(i, j, k)`` of element ``(ex, ey, ez)`` is lattice point
  ``(N ex + i, N ey + j, N ez + k)``, so nodes on shared faces, edges and
  corners get one global number (connectivity only);
* uniform random fields ``u`` over the local nodes of each element;
* the random noise and the random mesh descriptors of the batched workload.

Everything is drawn from ``numpy.random.default_rng(seed)`` (PCG64), so the same
seed gives the same arrays on every machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# seeds of the named workloads
SEED_MESH = 1711
SEED_FIELD = 903
SEED_RHS_NOISE = 2017
SEED_BATCH = 355


def grid_vertices(n: int, seed: int = SEED_MESH, amp: float = 0.1) -> np.ndarray:
    """Vertices of an ``n^3`` grid of the unit cube, interior ones perturbed.

    Returns a ``((n+1)^3, 3)`` float64 array; vertex ``(ix, iy, iz)`` sits at row
    ``ix + (n+1) (iy + (n+1) iz)``.  Each coordinate of an interior vertex
    (``0 < ix, iy, iz < n``) is moved by ``h * U[-amp, amp]`` with ``h = 1/n``;
    boundary vertices stay on the cube's faces, so the elements tile the unit
    cube exactly.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    idx = np.arange(n + 1, dtype=np.float64)
    iz, iy, ix = np.meshgrid(idx, idx, idx, indexing="ij")
    V = np.stack([ix, iy, iz], axis=-1).reshape(-1, 3) * h
    rng = np.random.default_rng(seed)
    P = rng.uniform(-amp, amp, size=((n + 1) ** 3, 3)) * h
    ii = np.stack([ix, iy, iz], axis=-1).reshape(-1, 3)
    interior = np.all((ii > 0) & (ii < n), axis=1)
    P[~interior] = 0.0
    return V + P


def element_vertices(n: int, V: np.ndarray | None = None, E: int | None = None,
                     seed: int = SEED_MESH, amp: float = 0.1) -> np.ndarray:
    """Per-element vertex coordinates, shape ``(E, 8, 3)``, float64, C-contiguous.

    Element ``e = ex + n (ey + n ez)``; its local vertex ``a + 2 b + 4 c``
    (``a, b, c`` in {0, 1}) is grid vertex ``(ex + a, ey + b, ez + c)``.  With
    ``E`` given, only the first ``E`` elements in this lexicographic order are
    returned.
    """
    if V is None:
        V = grid_vertices(n, seed=seed, amp=amp)
    Etot = n ** 3
    if E is None:
        E = Etot
    if not (0 <= E <= Etot):
        raise ValueError("E out of range")
    e = np.arange(E, dtype=np.int64)
    ex, ey, ez = e % n, (e // n) % n, e // (n * n)
    out = np.empty((E, 8, 3), dtype=np.float64)
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                vid = (ex + a) + (n + 1) * ((ey + b) + (n + 1) * (ez + c))
                out[:, a + 2 * b + 4 * c, :] = V[vid]
    return out


def element_vertices_subset(n: int, elems: np.ndarray, V: np.ndarray | None = None,
                            seed: int = SEED_MESH, amp: float = 0.1) -> np.ndarray:
    """Vertices ``(len(elems), 8, 3)`` of the listed elements of the ``n^3`` grid."""
    if V is None:
        V = grid_vertices(n, seed=seed, amp=amp)
    e = np.asarray(elems, dtype=np.int64)
    ex, ey, ez = e % n, (e // n) % n, e // (n * n)
    out = np.empty((e.size, 8, 3), dtype=np.float64)
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                vid = (ex + a) + (n + 1) * ((ey + b) + (n + 1) * (ez + c))
                out[:, a + 2 * b + 4 * c, :] = V[vid]
    return out


def global_numbering(n: int, N: int, E: int | None = None) -> tuple[np.ndarray, int]:
    """Global node numbers of the first ``E`` elements of the ``n^3`` grid at
    degree N: ``(gids (E, (N+1)^3) int32, n_global)``.

    Local node ``i + Nq j + Nq^2 k`` of element ``e = ex + n (ey + n ez)`` is
    the lattice point ``(N ex + i, N ey + j, N ez + k)`` of the
    ``(N n + 1)^3`` node lattice; the lattice points the elements touch are
    numbered 0.. in lexicographic order (z slowest), so a partial grid has no
    unused numbers.
    """
    if E is None:
        E = n ** 3
    Nq = N + 1
    L = N * n + 1
    e = np.arange(E, dtype=np.int64)
    ex, ey, ez = e % n, (e // n) % n, e // (n * n)
    k, j, i = np.meshgrid(np.arange(Nq), np.arange(Nq), np.arange(Nq), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()              # local node i + Nq j + Nq^2 k
    lat = ((N * ex[:, None] + i) + L * ((N * ey[:, None] + j) + L * (N * ez[:, None] + k)))
    used = np.zeros(L ** 3, dtype=bool)
    used[lat.ravel()] = True
    rank = np.cumsum(used, dtype=np.int64) - 1              # number of each used lattice point
    ng = int(rank[-1]) + 1
    if ng >= 2 ** 31:
        raise ValueError("more global nodes than int32 numbers")
    return rank[lat].astype(np.int32), ng


def global_lattice_coords(n: int, N: int, E: int | None = None) -> np.ndarray:
    """Integer lattice coordinates ``(n_global, 3)`` (x, y, z index on the
    ``(N n + 1)^3`` lattice) of each global node of :func:`global_numbering`."""
    if E is None:
        E = n ** 3
    gids, ng = global_numbering(n, N, E)
    Nq = N + 1
    e = np.arange(E, dtype=np.int64)
    ex, ey, ez = e % n, (e // n) % n, e // (n * n)
    k, j, i = np.meshgrid(np.arange(Nq), np.arange(Nq), np.arange(Nq), indexing="ij")
    out = np.empty((ng, 3), dtype=np.int64)
    out[gids, 0] = N * ex[:, None] + i.ravel()
    out[gids, 1] = N * ey[:, None] + j.ravel()
    out[gids, 2] = N * ez[:, None] + k.ravel()
    return out


def field(E: int, Nq: int, seed: int = SEED_FIELD) -> np.ndarray:
    """``u ~ U[-1, 1]`` per local node, shape ``(E, Nq^3)``, node ``i + Nq j + Nq^2 k``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(E, Nq ** 3))


def field_rows(E: int, Nq: int, rows: np.ndarray, seed: int = SEED_FIELD,
               chunk: int = 4096) -> np.ndarray:
    """Rows ``rows`` of :func:`field` (same values) without materialising all of it."""
    rows = np.asarray(rows, dtype=np.int64)
    out = np.empty((rows.size, Nq ** 3))
    rng = np.random.default_rng(seed)
    order = np.argsort(rows)
    srt = rows[order]
    pos = 0
    for start in range(0, E, chunk):
        stop = min(E, start + chunk)
        blk = rng.uniform(-1.0, 1.0, size=(stop - start, Nq ** 3))
        while pos < srt.size and srt[pos] < stop:
            out[order[pos]] = blk[srt[pos] - start]
            pos += 1
        if pos == srt.size:
            break
    return out


def field_chunked(E: int, Nq: int, seed: int = SEED_FIELD, chunk: int = 4096):
    """Yield ``(start, block)`` pieces of :func:`field`, identical values, bounded memory."""
    rng = np.random.default_rng(seed)
    for start in range(0, E, chunk):
        stop = min(E, start + chunk)
        yield start, rng.uniform(-1.0, 1.0, size=(stop - start, Nq ** 3))


def global_noise(n_global: int, seed: int = SEED_RHS_NOISE) -> np.ndarray:
    """Noise ``U[-1, 1]`` per global node, shape ``(n_global,)`` (scaled by the caller)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n_global)


def rhs_noise(E: int, Nq: int, seed: int = SEED_RHS_NOISE) -> np.ndarray:
    """Noise ``U[-1, 1]`` per local node, shape ``(E, Nq^3)`` (scaled by the caller)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(E, Nq ** 3))


OPS = ("BP10", "BP35", "BP30")


@dataclass(frozen=True)
class BatchMesh:
    """One mesh of a ragged batch: operator, degree and element count."""
    op: str
    N: int
    E: int
    n: int          # grid edge: the mesh is the first E elements of an n^3 grid
    mesh_seed: int
    field_seed: int


def ragged_batch(count: int = 64, seed: int = SEED_BATCH, e_min: int = 64,
                 e_max: int = 32768, n_min: int = 1, n_max: int = 15) -> list[BatchMesh]:
    """Ragged batch descriptors: ``N ~ U{n_min..n_max}``, ``E`` log-uniform in
    ``[e_min, e_max]``, operator uniform over BP1.0 / BP3.5 / BP3.0."""
    rng = np.random.default_rng(seed)
    out = []
    for m in range(count):
        N = int(rng.integers(n_min, n_max + 1))
        E = int(math.floor(math.exp(rng.uniform(math.log(e_min), math.log(e_max)))))
        op = OPS[int(rng.integers(0, 3))]
        n = int(math.ceil(round(E ** (1.0 / 3.0), 9)))
        while n ** 3 < E:
            n += 1
        out.append(BatchMesh(op=op, N=N, E=E, n=n, mesh_seed=SEED_MESH + m,
                             field_seed=SEED_FIELD + m))
    return out


# Named workloads (degree N, grid edge n, E = n^3).
WORKLOADS = {
    "bp10_n3_e512": dict(op="BP10", N=3, n=8),
    "bp35_n7_e32768": dict(op="BP35", N=7, n=32),
    "bp30_n7_e262144": dict(op="BP30", N=7, n=64),
    "cg_n7_e262144": dict(op="CG", N=7, n=64),
}
