"""Assembled (continuous) operators: Z^T A Z (TEST INFRASTRUCTURE ONLY).

The paper applies the element operators as one block-diagonal matrix, each
element on its own copy of its nodes (Problem description section); the
global finite-element operator of a conforming mesh is the same blocks summed
into shared nodes.  With Z the Boolean matrix that copies global node values
to the element-local nodes (Z[l, g] = 1 iff local node l is global node g),
the assembled operator is Z^T A_L Z, A_L the block-diagonal matrix of element
matrices.  Here Z is applied as an index gather and Z^T as a sum over the
local copies of each global node, in ascending local-node order; the dense
forms build Z and A_L as matrices (small meshes only).

The Jacobi preconditioner needs diag(Z^T A_L Z) = Z^T diag(A_L).  The diagonal
of one element's matrix, written out from its definition:

* stiffness, S = sum_ab D_a^T diag(G_ab) D_b with D_r = Id x Id x D,
  D_s = Id x D x Id, D_t = D x Id x Id: for node n = (i, j, k),
    S_nn = sum_a D[a,i]^2 G_rr(a,j,k) + sum_b D[b,j]^2 G_ss(i,b,k)
         + sum_c D[c,k]^2 G_tt(i,j,c)
         + 2 D[i,i] D[j,j] G_rs(n) + 2 D[i,i] D[k,k] G_rt(n) + 2 D[j,j] D[k,k] G_st(n)
  (a mixed term D_a^T diag(G) D_b with a != b touches node n only through
  the point n itself); plus lambda wJ(n) for the collocated mass;
* mass, M = I^T diag(wJ) I with I = I1 x I1 x I1:
    M_nn = sum_abc wJ(a,b,c) I1[a,i]^2 I1[b,j]^2 I1[c,k]^2.
"""
from __future__ import annotations

import numpy as np

from . import tables

# factor order rr, rs, rt, ss, st, tt
RR, RS, RT, SS, ST, TT = range(6)


def gather(ug: np.ndarray, gids: np.ndarray) -> np.ndarray:
    """Z u: the local copies (E, Np) of the global vector ug."""
    return np.asarray(ug, dtype=np.float64)[gids]


def scatter(ul: np.ndarray, gids: np.ndarray, n_global: int) -> np.ndarray:
    """Z^T u: each global node receives the sum of its local copies, added in
    ascending local-node order (element-major)."""
    out = np.zeros(n_global)
    np.add.at(out, gids.ravel(), np.asarray(ul, dtype=np.float64).ravel())
    return out


def multiplicity(gids: np.ndarray, n_global: int) -> np.ndarray:
    """Z^T 1: the number of local copies of each global node."""
    return np.bincount(gids.ravel(), minlength=n_global).astype(np.float64)


def assembled_apply(apply_local, gids: np.ndarray, n_global: int, ug: np.ndarray) -> np.ndarray:
    """Z^T A_L Z ug for a local operator apply_local((E, Np) -> (E, Np))."""
    return scatter(apply_local(gather(ug, gids)), gids, n_global)


def stiff35_diag(N: int, G: np.ndarray, wJ: np.ndarray | None = None, lam: float = 0.0) -> np.ndarray:
    """Diagonal (E, Np) of the collocated stiffness (+ lam * GLL mass) of each
    element, from the formula in the module docstring; G (E, 6, Np) in the
    natural node order."""
    T = tables(N)
    D = T.D
    q = N + 1
    E = G.shape[0]
    g = G.reshape(E, 6, q, q, q)           # [e][f][k][j][i]
    D2 = D * D
    dd = np.diag(D)
    out = np.zeros((E, q, q, q))
    for k in range(q):
        for j in range(q):
            for i in range(q):
                s = np.zeros(E)
                for a in range(q):
                    s += D2[a, i] * g[:, RR, k, j, a]
                    s += D2[a, j] * g[:, SS, k, a, i]
                    s += D2[a, k] * g[:, TT, a, j, i]
                s += 2 * dd[i] * dd[j] * g[:, RS, k, j, i]
                s += 2 * dd[i] * dd[k] * g[:, RT, k, j, i]
                s += 2 * dd[j] * dd[k] * g[:, ST, k, j, i]
                out[:, k, j, i] = s
    out = out.reshape(E, q ** 3)
    if lam:
        out += lam * wJ
    return out


def mass_diag(N: int, wJ: np.ndarray) -> np.ndarray:
    """Diagonal (E, Np) of the mass matrix of each element, wJ (E, Ng^3) at
    the Gauss points (natural order), from the formula in the module
    docstring."""
    T = tables(N)
    I2 = T.I * T.I                         # [a][i]
    g, q = N + 2, N + 1
    w = wJ.reshape(-1, g, g, g)            # [e][c][b][a]
    out = np.zeros((w.shape[0], q, q, q))
    for k in range(q):
        for j in range(q):
            for i in range(q):
                s = np.zeros(w.shape[0])
                for c in range(g):
                    for b in range(g):
                        for a in range(g):
                            s += w[:, c, b, a] * I2[a, i] * I2[b, j] * I2[c, k]
                out[:, k, j, i] = s
    return out.reshape(w.shape[0], q ** 3)


def dense_Z(gids: np.ndarray, n_global: int) -> np.ndarray:
    """Z as a dense (E Np, n_global) 0/1 matrix."""
    Z = np.zeros((gids.size, n_global))
    Z[np.arange(gids.size), gids.ravel()] = 1.0
    return Z


def dense_assembled(element_matrices: list[np.ndarray], gids: np.ndarray, n_global: int) -> np.ndarray:
    """Z^T blockdiag(A_e) Z as a dense matrix."""
    Z = dense_Z(gids, n_global)
    Np = gids.shape[1]
    A = np.zeros((gids.size, gids.size))
    for e, Ae in enumerate(element_matrices):
        A[e * Np:(e + 1) * Np, e * Np:(e + 1) * Np] = Ae
    return Z.T @ A @ Z
