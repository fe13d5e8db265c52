"""Pins of the oracle's operators BP1.0, BP3.5 and BP3.0.

* O1 (dense element matrices) against O2 (sum-factorised loops), N <= 3.
* Reference cube: closed Kronecker forms built from 1-D mass and stiffness
  matrices that NumPy's polynomial routines integrate exactly.
* Whole perturbed mesh of the unit cube (tiled exactly): integrals of
  polynomial fields that the quadrature must reproduce exactly --
  mass moments (1, 1/2, 1/3, 1/4, 1/8) and gradient energies (1, 0, 4/3, 2/3).
* Affine elements: Gauss quadrature is exact, so the operators equal the
  Galerkin integrals computed with a high-order NumPy Gauss rule.
* Symmetry, annihilation of constants, positivity, rigid-motion invariance,
  and the lambda terms.

A dropped term, a wrong sign, a wrong index or a transposed table in either
tier fails at least one of these.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as P

import oracle
from oracle import dense
import workloads


def mesh(n, N):
    X = workloads.element_vertices(n)
    return oracle.Problem(N, X)


def ref_cube_vertices():
    X = np.zeros((1, 8, 3))
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                X[0, a + 2 * b + 4 * c] = [2 * a - 1, 2 * b - 1, 2 * c - 1]
    return X


def lagrange_polys(r):
    out = []
    for i in range(r.size):
        others = np.delete(r, i)
        c = P.polyfromroots(others)
        out.append(c / np.prod(r[i] - others))
    return out


def exact_1d(r):
    """Exact 1-D mass and stiffness matrices of the Lagrange basis on nodes r."""
    L = lagrange_polys(r)
    n = r.size
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            m = P.polyint(P.polymul(L[i], L[j]))
            M[i, j] = P.polyval(1, m) - P.polyval(-1, m)
            k = P.polyint(P.polymul(P.polyder(L[i]), P.polyder(L[j])))
            K[i, j] = P.polyval(1, k) - P.polyval(-1, k)
    return M, K


def k3(t, s, r):
    return np.kron(t, np.kron(s, r))


def as_matrix(apply, np_):
    Id = np.eye(np_)
    return np.stack([apply(Id[c][None, :])[0] for c in range(np_)], axis=1)


# ---------------------------------------------------------------- O1 vs O2

@pytest.mark.parametrize("N", [1, 2, 3])
@pytest.mark.parametrize("lam", [0.0, 0.7])
def test_dense_vs_sumfactorised(N, lam):
    pb = mesh(2, N)
    u = workloads.field(pb.E, N + 1, seed=3)
    y1 = dense.apply_mass(N, pb.wJ_gl(), u)
    y2 = pb.mass(u)
    np.testing.assert_allclose(y2, y1, rtol=0, atol=1e-14 * np.abs(y1).max())
    y1 = dense.apply_stiff35(N, pb.G_gll(), u, pb.wJ_gll(), lam)
    y2 = pb.stiff35(u, lam)
    np.testing.assert_allclose(y2, y1, rtol=0, atol=1e-13 * np.abs(y1).max())
    y1 = dense.apply_stiff30(N, pb.G_gl(), u, pb.wJ_gl(), lam)
    y2 = pb.stiff30(u, lam)
    np.testing.assert_allclose(y2, y1, rtol=0, atol=1e-13 * np.abs(y1).max())


# ---------------------------------------------------------------- reference cube

@pytest.mark.parametrize("N", [1, 2, 3, 6])
def test_reference_cube_closed_forms(N):
    X = ref_cube_vertices()
    pb = oracle.Problem(N, X)
    nq = N + 1
    rgll, wgll = oracle.gll(N)
    M1, K1 = exact_1d(rgll)
    W = np.diag(wgll)
    Mex = k3(M1, M1, M1)
    S30ex = k3(M1, M1, K1) + k3(M1, K1, M1) + k3(K1, M1, M1)
    S35ex = k3(W, W, K1) + k3(W, K1, W) + k3(K1, W, W)
    Mo = as_matrix(pb.mass, nq ** 3)
    S30 = as_matrix(pb.stiff30, nq ** 3)
    S35 = as_matrix(pb.stiff35, nq ** 3)
    np.testing.assert_allclose(Mo, Mex, atol=1e-14)
    np.testing.assert_allclose(S30, S30ex, atol=1e-12 * N * N)
    np.testing.assert_allclose(S35, S35ex, atol=1e-12 * N * N)
    # the GLL-collocated mass of BP3.5 is W (x) W (x) W
    np.testing.assert_allclose(pb.wJ_gll()[0], np.diag(k3(W, W, W)), rtol=1e-14)


def test_reference_cube_N1_textbook():
    pb = oracle.Problem(1, ref_cube_vertices())
    M1 = np.array([[2 / 3, 1 / 3], [1 / 3, 2 / 3]])
    K1 = np.array([[0.5, -0.5], [-0.5, 0.5]])
    W = np.eye(2)
    np.testing.assert_allclose(as_matrix(pb.mass, 8), k3(M1, M1, M1), atol=1e-15)
    np.testing.assert_allclose(as_matrix(pb.stiff35, 8),
                               k3(W, W, K1) + k3(W, K1, W) + k3(K1, W, W), atol=1e-15)
    np.testing.assert_allclose(as_matrix(pb.stiff30, 8),
                               k3(M1, M1, K1) + k3(M1, K1, M1) + k3(K1, M1, M1), atol=1e-15)


# ---------------------------------------------------------------- whole-mesh integrals

def fields(pb):
    xyz = oracle.node_coords(pb.N, pb.X, "gll")
    return xyz[..., 0], xyz[..., 1], xyz[..., 2]


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_mass_moments_over_unit_cube(N):
    pb = mesh(3, N)
    x, y, z = fields(pb)
    one = np.ones_like(x)
    dot = lambda a, b: float(np.sum(a * pb.mass(b)))
    assert abs(dot(one, one) - 1.0) < 1e-14
    assert abs(dot(x, one) - 0.5) < 1e-14
    assert abs(dot(x, x) - 1 / 3) < 1e-14
    assert abs(dot(x, y) - 1 / 4) < 1e-14
    if N >= 2:
        assert abs(dot(x * y, z) - 1 / 8) < 1e-14
        assert abs(dot(x * x, y * y) - 1 / 9) < 1e-14


@pytest.mark.parametrize("op,N", [("stiff30", 1), ("stiff30", 2), ("stiff30", 4),
                                  ("stiff35", 2), ("stiff35", 3), ("stiff35", 6)])
def test_gradient_energies_over_unit_cube(op, N):
    pb = mesh(3, N)
    A = getattr(pb, op)
    x, y, z = fields(pb)
    one = np.ones_like(x)
    dot = lambda a, b: float(np.sum(a * A(b)))
    scale = np.abs(A(x)).max()
    assert np.abs(A(one)).max() < 1e-13 * max(1.0, scale)
    assert abs(dot(x, x) - 1.0) < 1e-13
    assert abs(dot(y, y) - 1.0) < 1e-13
    assert abs(dot(z, z) - 1.0) < 1e-13
    assert abs(dot(x, y)) < 1e-13 and abs(dot(y, z)) < 1e-13 and abs(dot(x, z)) < 1e-13
    quad_ok = (op == "stiff30" and N >= 2) or (op == "stiff35" and N >= 3)
    if quad_ok:
        assert abs(dot(x * x, x * x) - 4 / 3) < 1e-12
        assert abs(dot(x * y, x * y) - 2 / 3) < 1e-12
        assert abs(dot(x * x, y * y)) < 1e-12


def test_bp35_N1_not_exact_on_perturbed_mesh():
    """GLL with 2 points integrates only degree 1: the energy identity must fail
    at N = 1 on perturbed elements (and hold on the unperturbed grid)."""
    pb = mesh(3, 1)
    x, _, _ = fields(pb)
    assert abs(float(np.sum(x * pb.stiff35(x))) - 1.0) > 1e-6
    pb0 = oracle.Problem(1, workloads.element_vertices(3, amp=0.0))
    x0, _, _ = fields(pb0)
    assert abs(float(np.sum(x0 * pb0.stiff35(x0))) - 1.0) < 1e-13


# ---------------------------------------------------------------- affine elements

def affine_element(seed=5):
    rng = np.random.default_rng(seed)
    A = 0.5 * (np.eye(3) + 0.3 * rng.standard_normal((3, 3)))
    x0 = np.array([0.2, 0.3, -0.1])
    X = np.zeros((1, 8, 3))
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                X[0, a + 2 * b + 4 * c] = x0 + A @ np.array([a, b, c], dtype=float)
    return X, A, x0


def random_poly(deg, rng):
    terms = [(a, b, c) for a in range(deg + 1) for b in range(deg + 1) for c in range(deg + 1)
             if a + b + c <= deg]
    return [(rng.standard_normal(), t) for t in terms]


def peval(p, x):
    return sum(c * x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** cc for c, (a, b, cc) in p)


def pgrad(p, x):
    g = np.zeros(x.shape)
    for c, (a, b, cc) in p:
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        if a:
            g[..., 0] += c * a * X ** (a - 1) * Y ** b * Z ** cc
        if b:
            g[..., 1] += c * b * X ** a * Y ** (b - 1) * Z ** cc
        if cc:
            g[..., 2] += c * cc * X ** a * Y ** b * Z ** (cc - 1)
    return g


def galerkin(f, A, x0, npts=16):
    """int over the parallelepiped x0 + A (r+1)/2 of f(x) dx, NumPy Gauss rule."""
    r, w = npleg.leggauss(npts)
    R = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    W = np.einsum("a,b,c->abc", w, w, w).reshape(-1)
    x = x0 + ((R + 1.0) / 2.0) @ A.T
    return float(np.sum(W * f(x))) * abs(np.linalg.det(A / 2.0))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_affine_exactness(N):
    X, A, x0 = affine_element()
    pb = oracle.Problem(N, X)
    xyz = oracle.node_coords(N, X, "gll")[0]
    rng = np.random.default_rng(N)
    p, q = random_poly(N, rng), random_poly(N, rng)
    up, uq = peval(p, xyz)[None], peval(q, xyz)[None]
    mass_ex = galerkin(lambda x: peval(p, x) * peval(q, x), A, x0)
    stiff_ex = galerkin(lambda x: np.sum(pgrad(p, x) * pgrad(q, x), -1), A, x0)
    assert abs(float(np.sum(up * pb.mass(uq))) - mass_ex) < 1e-13 * max(1, abs(mass_ex))
    assert abs(float(np.sum(up * pb.stiff30(uq))) - stiff_ex) < 1e-12 * max(1, abs(stiff_ex))
    assert abs(float(np.sum(up * pb.stiff35(uq))) - stiff_ex) < 1e-12 * max(1, abs(stiff_ex))


# ---------------------------------------------------------------- structure

@pytest.mark.parametrize("N", [2, 4, 7])
def test_symmetry_and_definiteness(N):
    pb = mesh(2, N)
    u = workloads.field(pb.E, N + 1, seed=1)
    v = workloads.field(pb.E, N + 1, seed=2)
    for A in (pb.mass, pb.stiff35, pb.stiff30, lambda w: pb.stiff35(w, 2.0),
              lambda w: pb.stiff30(w, 2.0), lambda w: pb.cg_operator(w, 1.0)):
        Au, Av = A(u), A(v)
        asym = abs(float(np.sum(v * Au) - np.sum(u * Av)))
        assert asym <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(Av)
        assert float(np.sum(u * Au)) > 0
    # per element positivity of the mass, non-negativity of the stiffness
    assert np.all(np.einsum("en,en->e", u, pb.mass(u)) > 0)
    assert np.all(np.einsum("en,en->e", u, pb.stiff30(u)) > -1e-14)


@pytest.mark.parametrize("N", [2, 5])
def test_lambda_terms(N):
    pb = mesh(2, N)
    u = workloads.field(pb.E, N + 1, seed=4)
    lam = 3.25
    d35 = pb.stiff35(u, lam) - pb.stiff35(u)
    np.testing.assert_allclose(d35, lam * pb.wJ_gll() * u, rtol=1e-10, atol=1e-15)
    d30 = pb.stiff30(u, lam) - pb.stiff30(u)
    np.testing.assert_allclose(d30, lam * pb.mass(u), rtol=1e-9, atol=1e-14)
    y = pb.cg_operator(u, 1.0)
    np.testing.assert_allclose(y, pb.stiff35(u) + pb.mass(u), rtol=1e-13, atol=1e-16)


def test_rigid_motion_invariance():
    rng = np.random.default_rng(9)
    N = 3
    X = workloads.element_vertices(2)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    Xr = X @ Q.T + np.array([1.0, 2.0, -3.0])
    a, b = oracle.Problem(N, X), oracle.Problem(N, Xr)
    u = workloads.field(a.E, N + 1, seed=7)
    for op in ("mass", "stiff35", "stiff30"):
        ya, yb = getattr(a, op)(u), getattr(b, op)(u)
        np.testing.assert_allclose(yb, ya, rtol=0, atol=1e-12 * np.abs(ya).max())


def test_scaling_with_element_size():
    """On a box of side h: M scales as h^3, S as h."""
    N = 3
    X = workloads.element_vertices(1, amp=0.0)
    u = workloads.field(1, N + 1, seed=8)
    a, b = oracle.Problem(N, X), oracle.Problem(N, X * 0.25)
    np.testing.assert_allclose(b.mass(u), a.mass(u) * 0.25 ** 3, rtol=1e-13)
    np.testing.assert_allclose(b.stiff30(u), a.stiff30(u) * 0.25, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(b.stiff35(u), a.stiff35(u) * 0.25, rtol=1e-12, atol=1e-15)


def test_empty_mesh():
    N = 3
    u = np.zeros((0, 64))
    for f in (lambda: oracle.bp10(N, np.zeros((0, 125)), u),
              lambda: oracle.bp35(N, np.zeros((0, 6, 64)), u),
              lambda: oracle.bp30(N, np.zeros((0, 6, 125)), u)):
        assert f().shape == (0, 64)


def test_accumulate():
    pb = mesh(2, 3)
    u = workloads.field(pb.E, 4, seed=4)
    y0 = workloads.field(pb.E, 4, seed=5)
    y = oracle.bp35(3, pb.G_gll(), u, y=y0.copy(), accumulate=True)
    np.testing.assert_allclose(y, y0 + pb.stiff35(u), rtol=1e-14, atol=1e-15)
