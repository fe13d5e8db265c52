"""O1: dense brute-force element matrices (TEST INFRASTRUCTURE ONLY).

Builds, for each element, the explicit matrices of the paper's definitions and
applies them as dense products:

* ``M^e = I^T J^e I`` with ``I = I1d (x) I1d (x) I1d`` (eq. massQuad and the
  matrix form that follows it);
* ``S^e = sum_{ab} D_a^T diag(G_ab) D_b`` with ``D_r = Id (x) Id (x) D1d``,
  ``D_s = Id (x) D1d (x) Id``, ``D_t = D1d (x) Id (x) Id`` (eq. stiffQuad and the
  Kronecker form of D^r, D^s, D^t), plus ``lambda J^e`` for the GLL mass;
* ``S^e = I^T (sum_{ab} D~_a^T diag(G~_ab) D~_b + lambda J~^e) I`` for the
  de-aliased form (eq. stiffQuad2).

Kronecker order: node ``i + Nq j + Nq^2 k`` has k slowest, so the 3-D operator
is ``kron(A_t, kron(A_s, A_r))``.  Sizes are small (N <= 3 or a handful of
elements); the O(Np^2) work per element is the point: no sum factorisation.
"""
from __future__ import annotations

import numpy as np

from . import tables

# index of the symmetric factor (a, b) in the rr, rs, rt, ss, st, tt order
SYM = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 0): 1, (1, 1): 3, (1, 2): 4,
       (2, 0): 2, (2, 1): 4, (2, 2): 5}


def kron3(At, As, Ar):
    return np.kron(At, np.kron(As, Ar))


def grad_ops(D):
    Id = np.eye(D.shape[0])
    return (kron3(Id, Id, D), kron3(Id, D, Id), kron3(D, Id, Id))


def mass_matrix(N, wJ_e):
    T = tables(N)
    I3 = kron3(T.I, T.I, T.I)
    return I3.T @ (wJ_e[:, None] * I3)


def stiff35_matrix(N, G_e, wJ_e=None, lam=0.0):
    T = tables(N)
    Ds = grad_ops(T.D)
    S = np.zeros((Ds[0].shape[1],) * 2)
    for a in range(3):
        for b in range(3):
            S += Ds[a].T @ (G_e[SYM[a, b]][:, None] * Ds[b])
    if lam:
        S += lam * np.diag(wJ_e)
    return S


def stiff30_matrix(N, G_e, wJ_e=None, lam=0.0):
    T = tables(N)
    I3 = kron3(T.I, T.I, T.I)
    Ds = grad_ops(T.Dgl)
    A = np.zeros((Ds[0].shape[1],) * 2)
    for a in range(3):
        for b in range(3):
            A += Ds[a].T @ (G_e[SYM[a, b]][:, None] * Ds[b])
    if lam:
        A += lam * np.diag(wJ_e)
    return I3.T @ A @ I3


def apply_mass(N, wJ, u):
    return np.stack([mass_matrix(N, wJ[e]) @ u[e] for e in range(u.shape[0])])


def apply_stiff35(N, G, u, wJ=None, lam=0.0):
    return np.stack([stiff35_matrix(N, G[e], None if wJ is None else wJ[e], lam) @ u[e]
                     for e in range(u.shape[0])])


def apply_stiff30(N, G, u, wJ=None, lam=0.0):
    return np.stack([stiff30_matrix(N, G[e], None if wJ is None else wJ[e], lam) @ u[e]
                     for e in range(u.shape[0])])
