"""Conjugate gradients on the normal equations G y = b, G = Z^T Z.

Test infrastructure only (see the package docstring).

Textbook preconditioned CG (Hestenes & Stiefel 1952) with an optional
block-Jacobi preconditioner built from the K diagonal M x M blocks G_kk of
the Gram (one block per ensemble member), or from its consecutive nb x nb
diagonal blocks (`block_jacobi_tiles`).  Iteration counts depend on the
inputs; the converged answer is pinned against the direct solve.
"""
from __future__ import annotations

import numpy as np


def block_jacobi(G: np.ndarray, K: int, M: int):
    """Return a function applying blockdiag(G_kk)^{-1} via per-block Cholesky."""
    facs = [np.linalg.cholesky(G[k * M:(k + 1) * M, k * M:(k + 1) * M]) for k in range(K)]

    def apply(r):
        out = np.empty_like(r)
        for k, L in enumerate(facs):
            s = slice(k * M, (k + 1) * M)
            t = np.linalg.solve(L, r[s])
            out[s] = np.linalg.solve(L.T, t)
        return out
    return apply


def block_jacobi_tiles(G: np.ndarray, nb: int):
    """Block-Jacobi with the consecutive nb x nb diagonal blocks of G (the last
    one smaller when nb does not divide the order): applies the inverse of
    blockdiag(G[s, s]) via per-block Cholesky."""
    n = G.shape[0]
    blocks = [slice(s, min(s + nb, n)) for s in range(0, n, nb)]
    facs = [np.linalg.cholesky(G[s, s]) for s in blocks]

    def apply(r):
        out = np.empty_like(r)
        for s, L in zip(blocks, facs):
            out[s] = np.linalg.solve(L.T, np.linalg.solve(L, r[s]))
        return out
    return apply


def pcg(G: np.ndarray, b: np.ndarray, y0=None, precond=None, tol=1e-10, maxiter=10000):
    """Solve G y = b for one right-hand side.  Stops when ||b - G y|| <= tol ||b||.
    Returns (y, iterations)."""
    y = np.zeros_like(b) if y0 is None else np.array(y0, dtype=np.float64)
    r = b - G @ y
    z = precond(r) if precond else r
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    if np.linalg.norm(r) <= tol * bn:
        return y, 0
    for it in range(1, maxiter + 1):
        Gp = G @ p
        alpha = rz / (p @ Gp)
        y += alpha * p
        r -= alpha * Gp
        if np.linalg.norm(r) <= tol * bn:
            return y, it
        z = precond(r) if precond else r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return y, maxiter
