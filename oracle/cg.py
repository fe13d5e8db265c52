"""Plain conjugate gradients (Hestenes & Stiefel 1952) for the oracle.

TEST INFRASTRUCTURE ONLY.  FP64 NumPy, textbook recurrences, no restarts, no
residual replacement; the operator is any callable ``A(v) -> A v`` on arrays
of the shape of ``b``.  Used to check the GPU solver's iteration counts and to
evaluate true residuals of its solutions with the oracle's own operator.
"""
from __future__ import annotations

import numpy as np


def cg(A, b: np.ndarray, x0: np.ndarray | None = None, rtol: float = 1e-10,
       max_iters: int = 100000) -> tuple[np.ndarray, int, list[float]]:
    """Return (x, iterations, recursive residual norms / ||b||)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = float(np.vdot(r, r))
    bn = float(np.sqrt(np.vdot(b, b)))
    hist = [np.sqrt(rr) / bn]
    it = 0
    while hist[-1] > rtol and it < max_iters:
        Ap = A(p)
        alpha = rr / float(np.vdot(p, Ap))
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(np.vdot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr) / bn)
    return x, it, hist


def true_relative_residual(A, b: np.ndarray, x: np.ndarray) -> float:
    r = b - A(x)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def pcg(A, b: np.ndarray, Minv, x0: np.ndarray | None = None, rtol: float = 1e-10,
        max_iters: int = 100000) -> tuple[np.ndarray, int, list[float]]:
    """Preconditioned CG (the same recurrences with z = Minv(r) in place of r
    in the direction and step length).  Stops on the unpreconditioned
    recursive residual ||r|| <= rtol ||b||.  Return (x, iterations, ||r|| /
    ||b|| per iteration)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A(x) if x0 is not None else b.copy()
    z = Minv(r)
    p = z.copy()
    rz = float(np.vdot(r, z))
    bn = float(np.sqrt(np.vdot(b, b)))
    hist = [float(np.sqrt(np.vdot(r, r))) / bn]
    it = 0
    while hist[-1] > rtol and it < max_iters:
        Ap = A(p)
        alpha = rz / float(np.vdot(p, Ap))
        x += alpha * p
        r -= alpha * Ap
        z = Minv(r)
        rz_new = float(np.vdot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        hist.append(float(np.sqrt(np.vdot(r, r))) / bn)
    return x, it, hist
