"""Pins of the oracle's trilinear geometry (scaled Jacobians and metric tensor).

Closed forms for boxes, NumPy's matrix inverse for affine (sheared) elements,
rigid-motion invariance, and whole-mesh volume sums over the unit cube, which
the perturbed grid tiles exactly.
"""
import numpy as np
import pytest

import oracle
import workloads


def box_vertices(x0, h):
    X = np.zeros((1, 8, 3))
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                X[0, a + 2 * b + 4 * c] = np.asarray(x0) + np.array([a, b, c]) * np.asarray(h)
    return X


def affine_vertices(A, x0):
    """Vertices of the parallelepiped x = x0 + A (r + 1) / 2."""
    X = np.zeros((1, 8, 3))
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                X[0, a + 2 * b + 4 * c] = x0 + A @ np.array([a, b, c], dtype=float)
    return X


@pytest.mark.parametrize("N", [1, 2, 5])
@pytest.mark.parametrize("quad", ["gll", "gl"])
def test_box_closed_form(N, quad):
    h = np.array([0.3, 0.7, 1.9])
    G, wJ = oracle.geometry(N, box_vertices([0.1, -2.0, 5.0], h), quad)
    r, w = oracle.gll(N) if quad == "gll" else oracle.gl(N + 2)
    nq = r.size
    W = np.einsum("c,b,a->cba", w, w, w).reshape(-1)
    det = h.prod() / 8
    np.testing.assert_allclose(wJ[0], W * det, rtol=1e-14)
    diag = (2.0 / h) ** 2
    expect = [diag[0], 0, 0, diag[1], 0, diag[2]]
    for f in range(6):
        np.testing.assert_allclose(G[0, f], W * det * expect[f], rtol=1e-13, atol=1e-15)
    assert G.shape == (1, 6, nq ** 3)


@pytest.mark.parametrize("quad", ["gll", "gl"])
def test_affine_against_numpy_inverse(quad):
    rng = np.random.default_rng(5)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    assert np.linalg.det(A) > 0
    N = 3
    G, wJ = oracle.geometry(N, affine_vertices(A, np.array([0.2, 0.3, -0.1])), quad)
    r, w = oracle.gll(N) if quad == "gll" else oracle.gl(N + 2)
    W = np.einsum("c,b,a->cba", w, w, w).reshape(-1)
    J = A / 2.0                        # dx/dr of the affine map
    Ji = np.linalg.inv(J)
    det = np.linalg.det(J)
    g = det * Ji @ Ji.T                # reference-space metric: dr_a/dx . dr_b/dx
    idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for f, (p, q) in enumerate(idx):
        np.testing.assert_allclose(G[0, f], W * g[p, q], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(wJ[0], W * det, rtol=1e-13)


@pytest.mark.parametrize("N", [1, 2, 3, 7])
def test_mesh_volume_is_one(N):
    """The perturbed n^3 grid tiles the unit cube: sum of w detJ over all GL nodes
    is 1 (GL with N+2 points integrates the degree-2 detJ exactly); so is the
    GLL sum for N >= 2."""
    X = workloads.element_vertices(4)
    _, wJ = oracle.geometry(N, X, "gl", want_G=False)
    assert abs(wJ.sum() - 1.0) < 1e-13
    _, wJl = oracle.geometry(N, X, "gll", want_G=False)
    if N >= 2:
        assert abs(wJl.sum() - 1.0) < 1e-13
    assert np.all(wJ > 0) and np.all(wJl > 0)


def test_rigid_motion_invariance():
    rng = np.random.default_rng(11)
    X = workloads.element_vertices(3)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    Xr = X @ Q.T + np.array([3.0, -1.0, 0.5])
    for quad in ("gll", "gl"):
        G, wJ = oracle.geometry(4, X, quad)
        Gr, wJr = oracle.geometry(4, Xr, quad)
        np.testing.assert_allclose(Gr, G, rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(wJr, wJ, rtol=1e-12)


def test_node_coords_hit_vertices():
    X = workloads.element_vertices(2)
    N = 3
    xyz = oracle.node_coords(N, X, "gll")
    nq = N + 1
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                n = a * N + nq * (b * N) + nq * nq * (c * N)
                np.testing.assert_allclose(xyz[:, n], X[:, a + 2 * b + 4 * c], atol=1e-15)


def test_inverted_element_is_reported():
    X = box_vertices([0, 0, 0], [1, 1, 1])
    X[0, [0, 1]] = X[0, [1, 0]]       # swap two vertices: the map folds
    with pytest.raises(ValueError):
        oracle.geometry(2, X, "gl")


def test_perturbed_grid_keeps_boundary():
    n = 5
    V = workloads.grid_vertices(n)
    h = 1.0 / n
    idx = np.arange(n + 1)
    iz, iy, ix = np.meshgrid(idx, idx, idx, indexing="ij")
    grid = np.stack([ix, iy, iz], -1).reshape(-1, 3) * h
    d = V - grid
    assert np.max(np.abs(d)) <= 0.1 * h + 1e-15
    onb = np.any((np.stack([ix, iy, iz], -1).reshape(-1, 3) % n) == 0, axis=1)
    assert np.all(d[onb] == 0) and np.all(np.abs(d[~onb]).max(axis=1) > 0)


def test_chunked_fields_reproduce_single_draw():
    a = workloads.field(3000, 4)
    b = np.concatenate([blk for _, blk in workloads.field_chunked(3000, 4, chunk=701)])
    assert np.array_equal(a, b)
    rows = np.array([2999, 0, 700, 701, 1500])
    assert np.array_equal(workloads.field_rows(3000, 4, rows, chunk=250), a[rows])
