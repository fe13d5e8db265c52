"""Pins of the oracle's quadrature rules and 1-D tables.

Each check is independent of the oracle's own code: textbook closed forms,
NumPy's Legendre routines, exact monomial integrals, and exact differentiation
/ interpolation of polynomials that the tables must reproduce.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle

NS = list(range(1, 16))


def test_gll_closed_forms():
    s5, s37 = math.sqrt(1 / 5), math.sqrt(3 / 7)
    cases = {
        1: ([-1, 1], [1, 1]),
        2: ([-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
        3: ([-1, -s5, s5, 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
        4: ([-1, -s37, 0, s37, 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
    }
    for N, (r, w) in cases.items():
        rr, ww = oracle.gll(N)
        np.testing.assert_allclose(rr, r, atol=1e-15)
        np.testing.assert_allclose(ww, w, rtol=1e-14)


def test_gl_closed_forms():
    s3, s35 = math.sqrt(1 / 3), math.sqrt(3 / 5)
    cases = {1: ([0.0], [2.0]), 2: ([-s3, s3], [1, 1]), 3: ([-s35, 0, s35], [5 / 9, 8 / 9, 5 / 9])}
    for n, (r, w) in cases.items():
        rr, ww = oracle.gl(n)
        np.testing.assert_allclose(rr, r, atol=1e-15)
        np.testing.assert_allclose(ww, w, rtol=1e-14)


@pytest.mark.parametrize("n", range(1, 18))
def test_gl_matches_numpy_leggauss(n):
    r, w = oracle.gl(n)
    rr, ww = npleg.leggauss(n)
    np.testing.assert_allclose(r, rr, atol=2e-15)
    np.testing.assert_allclose(w, ww, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("N", NS)
def test_gll_nodes_are_roots_of_dPN(N):
    r, w = oracle.gll(N)
    interior = np.sort(npleg.Legendre.basis(N).deriv().roots().real)
    np.testing.assert_allclose(r[1:-1], interior, atol=1e-13)
    assert r[0] == -1.0 and r[-1] == 1.0
    # weights 2/(N(N+1) P_N(r)^2) from NumPy's P_N
    PN = npleg.Legendre.basis(N)(r)
    np.testing.assert_allclose(w, 2.0 / (N * (N + 1) * PN ** 2), rtol=1e-13)


def _exact_moment(k):
    return 0.0 if k % 2 else 2.0 / (k + 1)


@pytest.mark.parametrize("N", NS)
def test_quadrature_exactness(N):
    r, w = oracle.gll(N)
    for k in range(0, 2 * N):          # GLL: exact to degree 2N-1
        assert abs(np.dot(w, r ** k) - _exact_moment(k)) < 1e-14
    rg, wg = oracle.gl(N + 2)
    for k in range(0, 2 * (N + 2)):    # GL with N+2 points: exact to degree 2N+3
        assert abs(np.dot(wg, rg ** k) - _exact_moment(k)) < 1e-14
    # and the GLL rule is NOT exact at degree 2N (the reason BP3.5 under-integrates)
    assert abs(np.dot(w, r ** (2 * N)) - _exact_moment(2 * N)) > 1e-11


def test_D_closed_forms():
    T1 = oracle.tables(1)
    np.testing.assert_allclose(T1.D, [[-0.5, 0.5], [-0.5, 0.5]], atol=1e-15)
    for N in NS:
        D = oracle.tables(N).D
        assert abs(D[0, 0] + N * (N + 1) / 4) < 1e-12 * N * N
        assert abs(D[N, N] - N * (N + 1) / 4) < 1e-12 * N * N


@pytest.mark.parametrize("N", NS)
def test_tables_on_polynomials(N):
    """D differentiates, I interpolates and Dgl differentiates polynomials of
    the right degree exactly (definitions of eqs. interpolationOps and
    derivativeOps: rows are basis values / derivatives at the nodes)."""
    T = oracle.tables(N)
    scale = max(1.0, N * N)
    for k in range(0, N + 1):
        f = T.rgll ** k
        df = k * T.rgll ** (k - 1) if k else np.zeros_like(T.rgll)
        assert np.max(np.abs(T.D @ f - df)) < 1e-12 * scale * max(1, k)
        assert np.max(np.abs(T.I @ f - T.rgl ** k)) < 1e-13
    for k in range(0, N + 2):
        g = T.rgl ** k
        dg = k * T.rgl ** (k - 1) if k else np.zeros_like(T.rgl)
        assert np.max(np.abs(T.Dgl @ g - dg)) < 1e-12 * scale * max(1, k)


@pytest.mark.parametrize("N", NS)
def test_centro_symmetry(N):
    """Each interpolation entry appears twice, I[n][m] = I[ng-1-n][nq-1-m]
    (BP1.0 optimisation section, Kernel 8); D and Dgl are centro-antisymmetric."""
    T = oracle.tables(N)
    np.testing.assert_allclose(T.I, T.I[::-1, ::-1], atol=1e-14)
    np.testing.assert_allclose(T.D, -T.D[::-1, ::-1], atol=1e-12 * N * N)
    np.testing.assert_allclose(T.Dgl, -T.Dgl[::-1, ::-1], atol=1e-12 * N * N)


def test_bad_degree_rejected():
    with pytest.raises(ValueError):
        oracle.Tables(0)
    with pytest.raises(ValueError):
        oracle.Tables(16)
