"""The paper's own left inverse for the square case n_w = K (Sec. 3.9-3.10).

Test infrastructure only (see the package docstring).

Inputs follow the paper's statement of the problem: the n x K matrix of
scaled members (its columns z_k, eq. zkDefinition), the n_h x L eigenvectors
V_b of the localization block and its L non-zero eigenvalues delta_b
(Sec. 3.9, the economical eigendecomposition C_b = V_b Delta_b V_b^T).

With n_w = K the matrix A of eq. ADef is square; its per-grid-column blocks
A_m (n_w x K: the rows of the member matrix that belong to grid column m,
Sec. 3.9) are factored by SVD independently, and
    left inverse = Delta^{-1/2} V^T F Lambda^{-1} E^T     (eq. InverseSquareRootSwift)
whose action on a vector is computed column by column (step V1), regrouped by
member (V2-V3), projected on the localization modes (V4) and concatenated (V5).

Readings (the printed text is inconsistent in places):
  * V1 uses the factorization of eq. svdOfAm, A_m = E_m Lambda_m F_m^T, so
    w^(m) = A_m^{-1} x^(m) = F_m Lambda_m^{-1} E_m^T x^(m);
  * V4 applies Delta_b^{-1/2} V_b^T (V_b is n_h x L, eq. InverseSquareRootAlmost);
  * the segments w_l of V3-V4 are indexed by the member k (the block-diagonal V
    has one block per member, and the paper writes n_w blocks only because
    n_w = K there).
"""
from __future__ import annotations

import numpy as np


def column_blocks(Zm: np.ndarray, n_h: int, n_w: int) -> np.ndarray:
    """A_m for every grid column m: array (n_h, n_w, K) with A[m][l, k] = z_k[l*n_h + m]."""
    n, K = Zm.shape
    return np.transpose(Zm.reshape(n_w, n_h, K), (1, 0, 2))


def swift_apply(Zm: np.ndarray, Vb: np.ndarray, delta_b: np.ndarray, n_w: int,
                x: np.ndarray) -> np.ndarray:
    """x~ = (P^c)^{-1/2} x by steps V1-V5 (one vector or the columns of a matrix)."""
    n, K = Zm.shape
    n_h, L = Vb.shape
    if n_w != K:
        raise ValueError("the paper's algorithm needs n_w = K")
    vec = x.ndim == 1
    X = x[:, None] if vec else x
    R = X.shape[1]
    A = column_blocks(Zm, n_h, n_w)
    Xc = np.transpose(X.reshape(n_w, n_h, R), (1, 0, 2))      # x^(m): (n_h, n_w, R)
    w = np.empty((n_h, K, R))
    for m in range(n_h):                                       # V1: one task per column
        Em, lam, FmT = np.linalg.svd(A[m])                     # A_m = E_m Lambda_m F_m^T
        w[m] = FmT.T @ ((Em.T @ Xc[m]) / lam[:, None])
    # V2-V3: the n-vector w, split in member segments w_k (n_h each)
    wk = np.transpose(w, (1, 0, 2))                            # (K, n_h, R)
    # V4: x~_k = Delta_b^{-1/2} V_b^T w_k
    out = np.einsum("jl,kjr->klr", Vb, wk) / np.sqrt(delta_b)[None, :, None]
    Y = out.reshape(K * L, R)                                  # V5: concatenate
    return Y[:, 0] if vec else Y


def swift_matrix(Zm: np.ndarray, Vb: np.ndarray, delta_b: np.ndarray, n_w: int) -> np.ndarray:
    """The full left inverse Delta^{-1/2} V^T F Lambda^{-1} E^T (K*L x n), eq.
    InverseSquareRootSwift, assembled from the per-column SVDs (eqs. LambdaBlocks,
    EBlocks, FBlocks) for tiny problems."""
    n, K = Zm.shape
    n_h, L = Vb.shape
    A = column_blocks(Zm, n_h, n_w)
    Ainv = np.zeros((K * n_h, n))                  # columns index (k, m); rows of x index (l, m)
    for m in range(n_h):
        Em, lam, FmT = np.linalg.svd(A[m])
        Am_inv = FmT.T @ np.diag(1.0 / lam) @ Em.T                 # K x n_w
        rows = np.arange(K) * n_h + m
        cols = np.arange(n_w) * n_h + m
        Ainv[np.ix_(rows, cols)] = Am_inv
    V = np.kron(np.eye(K), Vb)                     # eq. VBlocks (one block per member)
    Dm = np.kron(np.ones(K), 1.0 / np.sqrt(delta_b))
    return Dm[:, None] * (V.T @ Ainv)
