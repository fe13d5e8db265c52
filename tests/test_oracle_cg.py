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


def _exact_residual_sq(pb, N, x, b, lam):
    """||b - (S + lam M) x||^2 in exact rational arithmetic on the FP64 inputs
    (fractions.Fraction), from the operators' definitions: S = sum_ab D_a^T
    diag(G_ab) D_b with D_r = I x I x D etc., M = I^T diag(wJ) I."""
    from fractions import Fraction as F
    T = oracle.tables(N)
    nq, ng = N + 1, N + 2
    D = [[F(float(T.D[i, m])) for m in range(nq)] for i in range(nq)]
    I = [[F(float(T.I[a, i])) for i in range(nq)] for a in range(ng)]
    G, wJ = pb.G_gll(), pb.wJ_gl()
    tot = F(0)
    for e in range(x.shape[0]):
        u = {(i, j, k): F(float(x[e, i + nq * j + nq * nq * k])) for i in range(nq) for j in range(nq) for k in range(nq)}
        g = lambda f, i, j, k: F(float(G[e, f, i + nq * j + nq * nq * k]))
        w = {}
        for (i, j, k) in u:
            qr = sum(D[i][m] * u[(m, j, k)] for m in range(nq))
            qs = sum(D[j][m] * u[(i, m, k)] for m in range(nq))
            qt = sum(D[k][m] * u[(i, j, m)] for m in range(nq))
            w[(i, j, k)] = (g(0, i, j, k) * qr + g(1, i, j, k) * qs + g(2, i, j, k) * qt,
                            g(1, i, j, k) * qr + g(3, i, j, k) * qs + g(4, i, j, k) * qt,
                            g(2, i, j, k) * qr + g(4, i, j, k) * qs + g(5, i, j, k) * qt)
        if lam:
            ut = {}
            for a in range(ng):
                for bb in range(ng):
                    for c in range(ng):
                        ut[(a, bb, c)] = F(float(wJ[e, a + ng * bb + ng * ng * c])) * sum(
                            I[a][i] * I[bb][j] * I[c][k] * u[(i, j, k)] for (i, j, k) in u)
        for (i, j, k) in u:
            y = sum(D[m][i] * w[(m, j, k)][0] + D[m][j] * w[(i, m, k)][1] + D[m][k] * w[(i, j, m)][2]
                    for m in range(nq))
            if lam:
                y += F(lam) * sum(I[a][i] * I[bb][j] * I[c][k] * v for (a, bb, c), v in ut.items())
            r = F(float(b[e, i + nq * j + nq * nq * k])) - y
            tot += r * r
    return tot


def test_extended_precision_residual():
    """ora_cg_residual_ld against what fixes it: (1) x = 0 gives ||b||^2 for
    both sums; (2) on a residual far above rounding it agrees with the FP64
    operator; (3) with b = the FP64 oracle's A x, the residual is that
    operator's own rounding (about 1e-16 relative), which exact rational
    arithmetic gives; the long-double evaluation must match it to 1%, where an
    evaluation in FP64 arithmetic is off by its own rounding, i.e. by 100%."""
    for N, lam in ((3, 1.0), (7, 1.0), (7, 4096.0), (5, 0.0)):
        X = workloads.element_vertices(4, E=37)
        pb = oracle.Problem(N, X)
        rng = np.random.default_rng(N)
        x = rng.uniform(-1, 1, (37, (N + 1) ** 3))
        b = rng.uniform(-1, 1, x.shape)
        rr, bb = pb.cg_residual_ld(np.zeros_like(x), b, lam)
        assert rr == bb and abs(bb - float(np.vdot(b, b))) <= 1e-12 * bb
        rr, bb = pb.cg_residual_ld(x, b, lam)
        r64 = b - pb.cg_operator(x, lam)
        assert abs(np.sqrt(rr) - np.linalg.norm(r64)) <= 1e-13 * np.linalg.norm(r64)
    for N, lam in ((1, 1.0), (2, 4096.0), (1, 0.0)):
        X = workloads.element_vertices(3, E=2)
        pb = oracle.Problem(N, X)
        x = np.random.default_rng(10 + N).uniform(-1, 1, (2, (N + 1) ** 3))
        ax = pb.cg_operator(x, lam)
        rr, bb = pb.cg_residual_ld(x, ax, lam)
        exact = float(_exact_residual_sq(pb, N, x, ax, lam))
        assert exact > 0.0 and np.sqrt(exact / bb) < 1e-14
        assert abs(rr - exact) <= 0.02 * exact, (N, lam, rr, exact)
