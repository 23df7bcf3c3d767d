"""The Hybrid covariance model in standardized variables (Sec. 2.2).

Test infrastructure only (see the package docstring).

Written out from the two forms the paper gives, with explicit n~ x n~
matrices (small inputs only):
  * the unsimplified form (eq. svCBKHybridBeforeSimplification), the
    climatologically unbiased Hybrid of the motivation (eq. CBKHybrid) in
    standardized variables, where the climatological covariance is I:
        P~h = (U - beta_e C~) o I + beta_e C~ o P~e,
    U the all-ones matrix;
  * the simplified form (eq. svCBKHybrid), valid when every diagonal entry
    of C~ is 1:
        P~h = (1 - beta_e) I + beta_e C~ o P~e.
P~e = E~ E~^T is the ensemble covariance of the standardized members
(Sec. 2.2: P~e = (P^c)^{-1/2} P^e ((P^c)^{-1/2})^T, so its factor is the
left inverse applied to the scaled forecast members).  The localization is
given by its modes W~ on the horizontal grid, C~ = (1 1^T) (x) (W~ W~^T)
over n_w levels (the same horizontal structure as in Sec. 3.6).
"""
from __future__ import annotations

import numpy as np


def localization(Wt: np.ndarray, n_w: int) -> np.ndarray:
    """C~ = (1_{n_w} 1_{n_w}^T) kron (W~ W~^T): entry (l n_h + j, l' n_h + j') = (W~ W~^T)[j, j']."""
    Ch = Wt @ Wt.T
    return np.kron(np.ones((n_w, n_w)), Ch)


def hybrid_unsimplified(Et: np.ndarray, Ct: np.ndarray, beta_e: float) -> np.ndarray:
    """(U - beta_e C~) o I + beta_e C~ o (E~ E~^T)   (eq. svCBKHybridBeforeSimplification)."""
    n = Ct.shape[0]
    U = np.ones((n, n))
    return (U - beta_e * Ct) * np.eye(n) + beta_e * Ct * (Et @ Et.T)


def hybrid_matrix(Et: np.ndarray, Ct: np.ndarray, beta_e: float) -> np.ndarray:
    """(1 - beta_e) I + beta_e C~ o (E~ E~^T)   (eq. svCBKHybrid)."""
    n = Ct.shape[0]
    return (1.0 - beta_e) * np.eye(n) + beta_e * Ct * (Et @ Et.T)


def hybrid_apply(Et: np.ndarray, Wt: np.ndarray, n_w: int, beta_e: float, V: np.ndarray) -> np.ndarray:
    """P~h V with the simplified form, by the explicit matrix."""
    return hybrid_matrix(Et, localization(Wt, n_w), beta_e) @ V
