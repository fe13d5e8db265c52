"""Pins of the oracle's assembled operators (oracle/assembly.py) and its
preconditioned CG, against values the finite-element method fixes:

* the multiplicity of each global node on a structured grid (closed form);
* gather / scatter against the dense Boolean Z and Z^T A_L Z built as
  matrices (brute force, small meshes);
* at N = 1 on an undistorted grid, the textbook Q1 stencils: the exact Q1
  stiffness (BP3.0: Gauss quadrature is exact on affine elements), the
  seven-point stencil of the vertex-quadrature Q1 stiffness (BP3.5: the
  2-point GLL rule), and the Q1 mass (BP1.0);
* the Neumann null space (the assembled stiffness annihilates constants),
  the domain's volume and first moments from the assembled mass;
* the element diagonals against the dense element matrices' diagonals and
  against e_n^T A e_n through the sum-factorised operator;
* Jacobi-preconditioned CG against numpy.linalg.solve.
"""
import numpy as np
import pytest

import oracle
from oracle import assembly, dense
from oracle.cg import cg, pcg
import workloads


def lattice_multiplicity(n, N):
    """Closed form: a lattice coordinate that is a multiple of N strictly
    inside (0, N n) lies on an element interface in that direction (2 elements
    share it), otherwise in one element; multiplicities multiply."""
    g = np.arange(N * n + 1)
    m1 = np.where((g % N == 0) & (g > 0) & (g < N * n), 2.0, 1.0)
    return np.einsum("k,j,i->kji", m1, m1, m1).ravel()


@pytest.mark.parametrize("n,N", [(2, 1), (3, 2), (2, 4), (4, 3)])
def test_multiplicity_closed_form(n, N):
    gids, ng = workloads.global_numbering(n, N)
    assert ng == (N * n + 1) ** 3
    np.testing.assert_array_equal(assembly.multiplicity(gids, ng), lattice_multiplicity(n, N))
    # every element's local nodes are distinct global nodes
    assert all(len(set(r)) == gids.shape[1] for r in gids)


def test_partial_grid_numbering_is_dense():
    gids, ng = workloads.global_numbering(3, 2, E=5)
    assert sorted(set(gids.ravel())) == list(range(ng))
    lat = workloads.global_lattice_coords(3, 2, E=5)
    assert len({tuple(p) for p in lat}) == ng


def _elem_matrices(op, N, X, lam=0.0):
    Gll, wJll = oracle.geometry(N, X, "gll")
    Ggl, wJgl = oracle.geometry(N, X, "gl")
    out = []
    for e in range(X.shape[0]):
        if op == "BP10":
            out.append(dense.mass_matrix(N, wJgl[e]))
        elif op == "BP35":
            out.append(dense.stiff35_matrix(N, Gll[e], wJll[e], lam))
        else:
            out.append(dense.stiff30_matrix(N, Ggl[e], wJgl[e], lam))
    return out


def _local(op, N, X, lam=0.0):
    pb = oracle.Problem(N, X)
    return {"BP10": pb.mass, "BP35": lambda u: pb.stiff35(u, lam), "BP30": lambda u: pb.stiff30(u, lam)}[op]


@pytest.mark.parametrize("op", ["BP10", "BP35", "BP30"])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_gather_scatter_equals_dense(op, N):
    n = 2
    X = workloads.element_vertices(n)
    gids, ng = workloads.global_numbering(n, N)
    Ad = assembly.dense_assembled(_elem_matrices(op, N, X, 0.5), gids, ng)
    ug = np.random.default_rng(N).uniform(-1, 1, ng)
    y = assembly.assembled_apply(_local(op, N, X, 0.5), gids, ng, ug)
    np.testing.assert_allclose(y, Ad @ ug, rtol=0, atol=1e-13 * np.abs(Ad).max() * ng)
    np.testing.assert_allclose(Ad, Ad.T, atol=1e-14 * np.abs(Ad).max())


def _interior_row(op, N, n, h):
    """Row of the interior lattice point (1,1,1) of the assembled operator on
    an undistorted n^3 grid, as a 3x3x3 stencil [dz][dy][dx]."""
    X = workloads.element_vertices(n, amp=0.0)
    gids, ng = workloads.global_numbering(n, N)
    A = assembly.dense_assembled(_elem_matrices(op, N, X), gids, ng)
    L = N * n + 1
    c = 1 + L * (1 + L)
    st = np.zeros((3, 3, 3))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                st[dz + 1, dy + 1, dx + 1] = A[c, c + dx + L * (dy + L * dz)]
    return st, A[c]


def test_q1_stencils():
    n = 2
    h = 1.0 / n
    kinds = lambda st: (st[1, 1, 1], st[1, 1, 0], st[1, 0, 0], st[0, 0, 0])   # centre, face, edge, corner
    # exact Q1 stiffness (Gauss quadrature, affine elements)
    st, row = _interior_row("BP30", 1, n, h)
    np.testing.assert_allclose(kinds(st), (8 * h / 3, 0.0, -h / 6, -h / 12), atol=1e-15)
    assert abs(row.sum()) < 1e-15 and np.count_nonzero(np.abs(row) > 1e-15) == 27 - 6
    # vertex (2-point GLL) quadrature: the seven-point stencil
    st, row = _interior_row("BP35", 1, n, h)
    np.testing.assert_allclose(kinds(st), (6 * h, -h, 0.0, 0.0), atol=1e-15)
    assert np.count_nonzero(np.abs(row) > 1e-15) == 7
    # Q1 mass: tensor product of the 1-D [h/6, 2h/3, h/6]
    st, row = _interior_row("BP10", 1, n, h)
    a, b = 2 / 3, 1 / 6
    np.testing.assert_allclose(kinds(st), (a ** 3 * h ** 3, a * a * b * h ** 3, a * b * b * h ** 3, b ** 3 * h ** 3),
                               atol=1e-16)
    assert abs(row.sum() - h ** 3) < 1e-16


@pytest.mark.parametrize("op", ["BP35", "BP30"])
@pytest.mark.parametrize("N", [2, 5])
def test_neumann_null_space(op, N):
    n = 3
    X = workloads.element_vertices(n)
    gids, ng = workloads.global_numbering(n, N)
    one = np.ones(ng)
    y = assembly.assembled_apply(_local(op, N, X), gids, ng, one)
    scale = np.abs(assembly.assembled_apply(_local(op, N, X), gids, ng,
                                            np.random.default_rng(1).uniform(-1, 1, ng))).max()
    assert np.abs(y).max() < 1e-13 * scale


@pytest.mark.parametrize("N", [1, 3, 6])
def test_assembled_mass_moments(N):
    n = 3
    X = workloads.element_vertices(n)
    gids, ng = workloads.global_numbering(n, N)
    xg = np.zeros((ng, 3))
    xg[gids] = oracle.node_coords(N, X, "gll")           # the coordinate fields, continuous
    M1 = assembly.assembled_apply(_local("BP10", N, X), gids, ng, np.ones(ng))
    assert abs(M1.sum() - 1.0) < 1e-13                     # volume of the unit cube
    np.testing.assert_allclose(xg.T @ M1, [0.5, 0.5, 0.5], atol=1e-13)    # first moments


@pytest.mark.parametrize("N", [1, 2, 3])
def test_element_diagonals_dense(N):
    X = workloads.element_vertices(2)
    Gll, wJll = oracle.geometry(N, X, "gll")
    _, wJgl = oracle.geometry(N, X, "gl")
    ds = assembly.stiff35_diag(N, Gll, wJll, 0.75)
    dm = assembly.mass_diag(N, wJgl)
    for e in range(X.shape[0]):
        np.testing.assert_allclose(ds[e], np.diag(dense.stiff35_matrix(N, Gll[e], wJll[e], 0.75)), rtol=1e-13,
                                   atol=1e-16)
        np.testing.assert_allclose(dm[e], np.diag(dense.mass_matrix(N, wJgl[e])), rtol=1e-13, atol=1e-18)


def test_element_diagonals_unit_vectors_n7():
    N = 7
    X = workloads.element_vertices(2, E=2)
    pb = oracle.Problem(N, X)
    ds = assembly.stiff35_diag(N, pb.G_gll())
    dm = assembly.mass_diag(N, pb.wJ_gl())
    Np = (N + 1) ** 3
    for node in (0, 9, 73, 300, Np - 1):
        u = np.zeros((2, Np))
        u[:, node] = 1.0
        np.testing.assert_allclose(pb.stiff35(u)[:, node], ds[:, node], rtol=1e-12)
        np.testing.assert_allclose(pb.mass(u)[:, node], dm[:, node], rtol=1e-12)


def test_jacobi_pcg_matches_direct_solve():
    rng = np.random.default_rng(7)
    n = 50
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = (Q * np.logspace(0, 2, n)) @ Q.T
    s = np.logspace(-3, 3, n)                               # a badly scaled SPD matrix
    A = s[:, None] * B * s[None, :]
    b = rng.standard_normal(n)
    x, it, hist = pcg(lambda v: A @ v, b, lambda r: r / np.diag(A), rtol=1e-12)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-7)
    _, it_plain, _ = cg(lambda v: A @ v, b, rtol=1e-12, max_iters=5000)
    assert it < it_plain
    # identity preconditioner: the plain CG iterates
    x1, it1, h1 = pcg(lambda v: A @ v, b, lambda r: r.copy(), rtol=1e-6)
    x2, it2, h2 = cg(lambda v: A @ v, b, rtol=1e-6)
    assert it1 == it2 and np.allclose(x1, x2, rtol=1e-10)
