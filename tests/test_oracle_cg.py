"""Pins of the oracle's conjugate gradients: against numpy.linalg.solve on small
SPD systems, finite termination on distinct spectra, and the textbook bound
for an operator with few distinct eigenvalues."""
import numpy as np

import oracle
from oracle.cg import cg, true_relative_residual
import workloads


def spd(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.logspace(0, np.log10(cond), n)
    return (Q * ev) @ Q.T, ev


def test_cg_matches_direct_solve():
    A, _ = spd(40, 1)
    b = np.random.default_rng(2).standard_normal(40)
    x, it, hist = cg(lambda v: A @ v, b, rtol=1e-13)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)
    assert hist[-1] <= 1e-13 and it <= 200


def test_cg_finite_termination_few_eigenvalues():
    # k distinct eigenvalues: exact CG terminates in k steps
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    ev = np.repeat([1.0, 3.0, 10.0, 30.0], 15)
    A = (Q * ev) @ Q.T
    b = rng.standard_normal(60)
    x, it, _ = cg(lambda v: A @ v, b, rtol=1e-12)
    assert it <= 6
    assert true_relative_residual(lambda v: A @ v, b, x) < 1e-11


def test_cg_on_screened_poisson():
    N = 3
    X = workloads.element_vertices(3)
    pb = oracle.Problem(N, X)
    b = workloads.field(pb.E, N + 1, seed=4)
    x, it, hist = cg(lambda v: pb.cg_operator(v, 1.0), b, rtol=1e-10)
    assert true_relative_residual(lambda v: pb.cg_operator(v, 1.0), b, x) < 1e-9
    assert it < 2000
