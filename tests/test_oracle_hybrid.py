"""Pins of the Hybrid oracle (Sec. 2.2) against what the paper and the
mathematics fix: the paper's two forms agree exactly when the localization
has a unit diagonal (and differ by beta_e (1 - c_ii) on the diagonal
otherwise); the localized ensemble covariance is Z~ Z~^T of the modulated
columns (the Schur product identity of Sec. 3.7, checked by brute force
against the explicit modulated matrix); a standardized ensemble covariance
equal to I gives P~h = I (the climatological unbiasedness the paper claims);
the smallest eigenvalue is at least 1 - beta_e (Schur product theorem: the
paper's positive definiteness)."""
import numpy as np
import pytest

from oracle import hybrid, lsq


def _factors(n_h, n_w, K, L, seed, unit_diag=True):
    rng = np.random.default_rng(seed)
    Et = rng.standard_normal((n_h * n_w, K)) / np.sqrt(K - 1)
    Wt = rng.standard_normal((n_h, L))
    if unit_diag:
        Wt /= np.linalg.norm(Wt, axis=1, keepdims=True)
    return Et, Wt


@pytest.mark.parametrize("shape", [(6, 1, 4, 3), (5, 2, 3, 4), (8, 3, 6, 2)])
def test_two_forms_agree_with_unit_diagonal(shape):
    n_h, n_w, K, L = shape
    Et, Wt = _factors(n_h, n_w, K, L, 7)
    Ct = hybrid.localization(Wt, n_w)
    assert np.allclose(np.diag(Ct), 1.0, atol=1e-15)
    for beta in (0.0, 0.3, 0.75, 1.0):
        a = hybrid.hybrid_unsimplified(Et, Ct, beta)
        b = hybrid.hybrid_matrix(Et, Ct, beta)
        assert np.abs(a - b).max() <= 4e-16 * np.abs(b).max()


def test_forms_differ_on_the_diagonal_without_unit_diagonal():
    Et, Wt = _factors(7, 2, 4, 3, 8, unit_diag=False)
    Ct = hybrid.localization(Wt, 2)
    beta = 0.4
    d = hybrid.hybrid_unsimplified(Et, Ct, beta) - hybrid.hybrid_matrix(Et, Ct, beta)
    assert np.allclose(d, np.diag(beta * (1.0 - np.diag(Ct))), atol=1e-14)
    assert np.abs(np.diag(d)).max() > 1e-3


@pytest.mark.parametrize("shape", [(6, 1, 4, 3), (5, 2, 3, 4), (4, 3, 5, 4)])
def test_localized_covariance_is_modulated_product(shape):
    """C~ o (E~ E~^T) = Z~ Z~^T with Z~ the columns e~_k o w~_m, formed by
    the least-squares oracle's explicit modulation (brute force)."""
    n_h, n_w, K, L = shape
    Et, Wt = _factors(n_h, n_w, K, L, 9, unit_diag=False)
    Zt = lsq.form_z(Et, Wt, n_w)
    beta = 0.6
    H = hybrid.hybrid_matrix(Et, hybrid.localization(Wt, n_w), beta)
    assert np.abs(H - ((1 - beta) * np.eye(n_h * n_w) + beta * Zt @ Zt.T)).max() <= 1e-14 * np.abs(H).max()
    V = np.random.default_rng(3).standard_normal((n_h * n_w, 5))
    assert np.allclose(hybrid.hybrid_apply(Et, Wt, n_w, beta, V), H @ V, rtol=0, atol=1e-13)


def test_identity_ensemble_covariance_gives_identity():
    """With P~e = I (orthogonal standardized members) and a unit-diagonal
    localization the Hybrid is I for every beta_e."""
    n = 12
    Q, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((n, n)))
    _, Wt = _factors(n, 1, 2, 5, 10)
    Ct = hybrid.localization(Wt, 1)
    for beta in (0.2, 0.5, 0.9):
        assert np.abs(hybrid.hybrid_matrix(Q, Ct, beta) - np.eye(n)).max() <= 1e-14
        assert np.abs(hybrid.hybrid_unsimplified(Q, Ct, beta) - np.eye(n)).max() <= 1e-14


@pytest.mark.parametrize("beta", [0.1, 0.5, 0.95])
def test_positive_definite_with_margin(beta):
    """Rank-deficient ensemble (K << n~) and localization: still every
    eigenvalue >= 1 - beta_e."""
    Et, Wt = _factors(10, 2, 3, 2, 11)
    H = hybrid.hybrid_matrix(Et, hybrid.localization(Wt, 2), beta)
    assert np.linalg.eigvalsh(H).min() >= (1 - beta) - 1e-13
