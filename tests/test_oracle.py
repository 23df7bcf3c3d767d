"""Pins for the FP64 CPU oracle: library routines, closed forms, invariants,
brute force and hand-derived cases.  No GPU needed."""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import cg, lsq, mlp, swift

HERE = os.path.dirname(os.path.abspath(__file__))


def small_instance(n_lat=4, n_lon=8, n_w=1, K=3, M=5, R=4, seed=7, centring="none"):
    return wl.make_instance(n_lat, n_lon, K, M, R, 0.3, 0.6, seed, n_w=n_w, centring=centring)


SHAPES = [(4, 8, 1, 3, 5), (4, 8, 2, 4, 6), (3, 6, 3, 2, 9), (4, 8, 4, 8, 7), (2, 4, 1, 1, 8)]


# ---------------------------------------------------------------- Z itself
@pytest.mark.parametrize("shape", SHAPES)
def test_modulation_identity(shape):
    """Z Z^T = C o P^s with P^s = E E^T and C built from equal blocks W W^T
    (the Bishop-Hodyss modulation identity used in Sec. 3.7)."""
    n_lat, n_lon, n_w, K, M = shape
    inst = small_instance(n_lat, n_lon, n_w, K, M)
    Z = lsq.form_z(inst.E, inst.W, n_w)
    assert Z.shape == (inst.n, K * M)
    P = lsq.localized_covariance(inst.E, inst.W, n_w)
    assert np.abs(Z @ Z.T - P).max() <= 1e-13 * np.abs(P).max()


def test_column_order_and_segments():
    """Column k*M+m of Z is diag(z_k) applied to the stacked mode w_m (eq. DiagZC):
    checked on unit vectors so a transposed or shifted index cannot pass."""
    n_h, n_w, K, M = 3, 2, 2, 3
    E = np.arange(1.0, n_h * n_w * K + 1).reshape(n_h * n_w, K, order="F")
    W = np.arange(1.0, n_h * M + 1).reshape(n_h, M, order="F") * 10
    Z = lsq.form_z(E, W, n_w)
    for k in range(K):
        for m in range(M):
            e = np.zeros(K * M)
            e[k * M + m] = 1.0
            col = Z @ e
            expect = E[:, k] * np.concatenate([W[:, m]] * n_w)
            assert np.array_equal(col, expect)


# ------------------------------------------------------------ least squares
@pytest.mark.parametrize("shape", SHAPES)
def test_lstsq_matches_pinv(shape):
    """QR least squares equals the SVD pseudo-inverse (LAPACK gesdd via numpy)."""
    n_lat, n_lon, n_w, K, M = shape
    inst = small_instance(n_lat, n_lon, n_w, K, M, R=5)
    Z = lsq.form_z(inst.E, inst.W, n_w)
    Y, _ = lsq.lstsq_qr(Z, inst.X)
    Yp = np.linalg.pinv(Z) @ inst.X
    kappa = np.linalg.cond(Z)
    assert np.abs(Y - Yp).max() <= 1e-12 * kappa * max(1.0, np.abs(Yp).max())
    Yl = np.linalg.lstsq(Z, inst.X, rcond=None)[0]
    assert np.abs(Y - Yl).max() <= 1e-12 * kappa * max(1.0, np.abs(Yl).max())


@pytest.mark.parametrize("shape", SHAPES[:3])
def test_own_householder_matches_lapack(shape):
    n_lat, n_lon, n_w, K, M = shape
    inst = small_instance(n_lat, n_lon, n_w, K, M, R=3)
    Z = lsq.form_z(inst.E, inst.W, n_w)
    Y1, i1 = lsq.lstsq_qr(Z, inst.X, own=False)
    Y2, i2 = lsq.lstsq_qr(Z, inst.X, own=True)
    assert np.abs(Y1 - Y2).max() <= 1e-11 * max(1.0, np.abs(Y1).max())
    assert np.allclose(np.abs(i1["rdiag"]), np.abs(i2["rdiag"]), rtol=1e-12, atol=0)
    np.testing.assert_allclose(i1["residual_norm"], i2["residual_norm"], rtol=1e-10, atol=1e-13)
    # reconstruct Z from the own reflectors: Q^T Z = [R; 0]
    V, tau, R = lsq.householder_qr(Z)
    QtZ = lsq.apply_qt(V, tau, Z)
    assert np.abs(QtZ[: Z.shape[1]] - R).max() <= 1e-12 * np.abs(R).max()
    assert np.abs(QtZ[Z.shape[1]:]).max() <= 1e-12 * np.abs(R).max()


@pytest.mark.parametrize("shape", SHAPES)
def test_left_inverse_invariants(shape):
    """Z^+ Z = I (the defining left-inverse property, Sec. 2.1), least-squares
    orthogonality Z^T (x - Z y) = 0, and Z (Z^+ x) = x for x in range(Z)."""
    n_lat, n_lon, n_w, K, M = shape
    inst = small_instance(n_lat, n_lon, n_w, K, M, R=4)
    Z = lsq.form_z(inst.E, inst.W, n_w)
    kappa = np.linalg.cond(Z)
    ZpZ, _ = lsq.lstsq_qr(Z, Z)
    assert np.abs(ZpZ - np.eye(K * M)).max() <= 1e-13 * kappa
    Y, info = lsq.lstsq_qr(Z, inst.X)
    r = inst.X - Z @ Y
    g = Z.T @ r
    assert np.abs(g).max() <= 1e-13 * kappa * np.abs(Z).max() * np.abs(inst.X).sum(0).max()
    np.testing.assert_allclose(np.linalg.norm(r, axis=0), info["residual_norm"], rtol=1e-9, atol=1e-12)
    t = np.random.default_rng(1).standard_normal((K * M, 3))
    x = Z @ t
    assert np.abs(lsq.lstsq_qr(Z, x)[0] - t).max() <= 1e-13 * kappa * np.abs(t).max() * 10
    xp = lsq.project_range(inst.E, inst.W, n_w, inst.X)
    yp = lsq.lstsq_qr(Z, xp)[0]
    assert np.abs(Z @ yp - xp).max() <= 1e-12 * kappa
    assert np.abs(yp - Y).max() <= 1e-12 * kappa * max(1, np.abs(Y).max())


def test_closed_form_single_member_orthogonal_modes():
    """K=1, e_1 = 1: Z = W with orthogonal columns W = V_b Delta_b^{1/2}, so
    Z^+ x = Delta_b^{-1} W^T x exactly."""
    n_lat, n_lon, M = 4, 8, 9
    W, info = wl.localization_modes(n_lat, n_lon, M, 0.5)
    n_h = n_lat * n_lon
    E = np.ones((n_h, 1))
    x = np.random.default_rng(3).standard_normal((n_h, 2))
    delta = np.sum(W * W, axis=0)
    y = lsq.left_inverse_apply(E, W, 1, x)
    assert np.abs(y - (W.T @ x) / delta[:, None]).max() <= 1e-12


def test_closed_form_diagonal():
    """M = n_h, n_w = 1, K = 1, W = I: Z = diag(e_1), so Z^+ x = x / e_1."""
    n_h = 12
    rng = np.random.default_rng(4)
    e = rng.uniform(0.5, 2.0, n_h) * rng.choice([-1, 1], n_h)
    x = rng.standard_normal((n_h, 3))
    y = lsq.left_inverse_apply(e[:, None], np.eye(n_h), 1, x)
    assert np.abs(y - x / e[:, None]).max() <= 1e-14


def test_closed_form_constant_mode():
    """M = 1, w_1 = c: Z = c E, so Z^+ = E^+ / c (E^+ by SVD)."""
    n_h, n_w, K, c = 10, 2, 4, 0.37
    rng = np.random.default_rng(5)
    E = rng.standard_normal((n_h * n_w, K))
    x = rng.standard_normal((n_h * n_w, 2))
    y = lsq.left_inverse_apply(E, np.full((n_h, 1), c), n_w, x)
    assert np.abs(y - np.linalg.pinv(E) @ x / c).max() <= 1e-12


def test_hand_cases():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as f:
        cases = json.load(f)["cases"]
    for cs in cases:
        E = np.array(cs["E"], dtype=float)
        W = np.array(cs["W"], dtype=float)
        x = np.array(cs["x"], dtype=float)
        if cs.get("error") == "shape":
            with pytest.raises(ValueError):
                lsq.left_inverse_apply(E, W, cs["n_w"], x)
            continue
        y, info = lsq.lstsq_qr(lsq.form_z(E, W, cs["n_w"]), x)
        np.testing.assert_allclose(y, cs["y"], rtol=0, atol=1e-14)
        assert abs(info["residual_norm"][0] ** 2 - cs["residual_norm2"]) <= 1e-12


def test_rank_deficiency_detected():
    """Sample-mean centring makes the members sum to zero, so A (and Z) lose
    rank (Sec. 4.2 and the rank statement of the supporting information)."""
    inst = small_instance(4, 8, 1, 4, 6, centring="sample")
    with pytest.raises(lsq.RankDeficient):
        lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    ok = small_instance(4, 8, 1, 4, 6, centring="discard")
    lsq.left_inverse_apply(ok.E, ok.W, 1, ok.X)


# --------------------------------------------------- Gram structure / rounding
@pytest.mark.parametrize("shape", SHAPES)
def test_gram_structure(shape):
    """Z^T Z has the doubly symmetric block form G_{(k,m),(k',m')} =
    sum_j S_j[k,k'] W[j,m] W[j,m'] with S_j = A_j^T A_j the per-column Gram."""
    n_lat, n_lon, n_w, K, M = shape
    inst = small_instance(n_lat, n_lon, n_w, K, M)
    G = lsq.gram(inst.E, inst.W, n_w)
    S = lsq.column_grams(inst.E, inst.n_h, n_w)
    G2 = np.einsum("jab,jm,jq->ambq", S, inst.W, inst.W).reshape(K * M, K * M)
    assert np.abs(G - G2).max() <= 1e-13 * np.abs(G).max()
    G4 = G.reshape(K, M, K, M)
    assert np.abs(G4 - G4.transpose(2, 1, 0, 3)).max() <= 1e-13 * np.abs(G).max()
    assert np.abs(G4 - G4.transpose(0, 3, 2, 1)).max() <= 1e-13 * np.abs(G).max()


def test_round_bf16_matches_torch_on_float32_values():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    x32 = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lsq.round_bf16(x32.astype(np.float64)), ref)


def test_round_bf16_ties_and_specials():
    one = 1.0
    ulp = 2.0 ** -7                               # bfloat16 spacing in [1, 2)
    assert lsq.round_bf16(np.array([one + ulp / 2]))[0] == one           # tie -> even
    assert lsq.round_bf16(np.array([one + 3 * ulp / 2]))[0] == one + 2 * ulp
    assert lsq.round_bf16(np.array([one + ulp / 2 + 2.0 ** -40]))[0] == one + ulp
    assert lsq.round_bf16(np.array([-(one + ulp / 2)]))[0] == -one
    assert lsq.round_bf16(np.array([2.0 - ulp / 4]))[0] == 2.0            # carry into exponent
    assert lsq.round_bf16(np.array([0.0, 1e-40]))[1] == 0.0                # below normal range


def test_gram_lowprec_close_and_psd():
    inst = small_instance(4, 8, 1, 4, 6)
    G = lsq.gram(inst.E, inst.W, 1)
    for fmt, u in (("bf16", 2.0 ** -8), ("fp32", 2.0 ** -24)):
        Gt = lsq.gram_lowprec(inst.E, inst.W, 1, fmt)
        assert np.abs(Gt - G).max() <= 4 * u * np.abs(G).max() * 2
        assert np.linalg.eigvalsh(Gt).min() > 0


# -------------------------------------------------------- the paper's algorithm
def _square_problem(n_lat=3, n_lon=6, K=4, seed=11, M=None):
    """n_w = K (the paper's assumption).  M = n_h gives a square, invertible Z."""
    n_h = n_lat * n_lon
    M = n_h if M is None else M
    spec = wl.circulant_spectrum(n_lat, n_lon, 0.7)
    rng = np.random.Generator(np.random.PCG64(seed))
    E = np.concatenate([wl.grf_draws(n_lat, n_lon, K, 0.5, rng) for _ in range(K)], axis=0)
    E /= math.sqrt(K - 1)
    W, info = wl.localization_modes(n_lat, n_lon, M, 0.7)
    delta = np.sum(W * W, axis=0)
    Vb = W / np.sqrt(delta)[None, :]
    return E, W, Vb, delta


def test_swift_equals_qr_in_square_case():
    """With n_w = K and all n_h localization modes, Z is square and invertible:
    the paper's left inverse (steps V1-V5) is the inverse, hence equal to the
    QR least-squares answer."""
    K = 4
    E, W, Vb, delta = _square_problem(K=K)
    n = E.shape[0]
    x = np.random.default_rng(8).standard_normal((n, 5))
    y_qr = lsq.left_inverse_apply(E, W, K, x)
    y_sw = swift.swift_apply(E, Vb, delta, K, x)
    Z = lsq.form_z(E, W, K)
    assert Z.shape[0] == Z.shape[1]
    kappa = np.linalg.cond(Z)
    assert np.abs(y_qr - y_sw).max() <= 1e-13 * kappa * np.abs(y_qr).max()
    Lp = swift.swift_matrix(E, Vb, delta, K)
    assert np.abs(Lp @ x - y_sw).max() <= 1e-12 * kappa * np.abs(y_sw).max()


def test_swift_on_range_and_paper_accuracy_tests():
    """M < n_h: the paper's left inverse is not Moore-Penrose, but both agree on
    range(Z).  Also the paper's two accuracy indicators: Xi = I - Z^-1 P Z^-T
    (Sec. 4.9) and delta = x~ - Z^-1 Z x~ (Sec. 4.10), both ~ 0."""
    K = 4
    E, W, Vb, delta = _square_problem(K=K, M=7)
    Z = lsq.form_z(E, W, K)
    t = np.random.default_rng(9).standard_normal((Z.shape[1], 6))
    x = Z @ t
    y_sw = swift.swift_apply(E, Vb, delta, K, x)
    y_qr = lsq.left_inverse_apply(E, W, K, x)
    assert np.abs(y_sw - t).max() <= 1e-10
    assert np.abs(y_qr - t).max() <= 1e-10
    Lp = swift.swift_matrix(E, Vb, delta, K)
    P = lsq.localized_covariance(E, W, K)
    Xi = np.eye(Z.shape[1]) - Lp @ P @ Lp.T
    assert math.sqrt(np.sum(Xi ** 2)) <= 1e-9 and np.abs(Xi).max() <= 1e-9
    # off range(Z) the two left inverses differ (the paper's is not Moore-Penrose)
    xr = np.random.default_rng(10).standard_normal((Z.shape[0], 1))
    assert np.abs(swift.swift_apply(E, Vb, delta, K, xr) - lsq.left_inverse_apply(E, W, K, xr)).max() > 1e-6


# ---------------------------------------------------------------- MLP and Adam
def _tiny_net(rng, d_in=7, h=5, d_out=6):
    return [rng.standard_normal((h, d_in)) * 0.4, rng.standard_normal(h) * 0.1,
            rng.standard_normal((d_out, h)) * 0.4, rng.standard_normal(d_out) * 0.1]


def test_mlp_backward_finite_differences():
    rng = np.random.default_rng(12)
    params = _tiny_net(rng)
    X = rng.standard_normal((4, 7))
    T = rng.standard_normal((4, 6))
    Y, cache = mlp.forward(params, X)
    grads = mlp.backward(params, cache, Y, T)
    for p, g in zip(params, grads):
        flat = p.reshape(-1)
        gflat = g.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[idx]
            h = 1e-6 * max(1.0, abs(old))
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(params, X)[0], T)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(params, X)[0], T)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[idx]) <= 1e-7 * max(1.0, abs(fd))


def test_gelu_special_values():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([10.0]))[0] - 10.0) < 1e-12
    assert abs(mlp.gelu(np.array([-10.0]))[0]) < 1e-12
    assert abs(mlp.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    # gelu(1) = Phi(1) = 0.841344746068543 (standard normal CDF table value)
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.841344746068543) < 1e-12


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so the step is
    lr * g / (|g| + eps)."""
    rng = np.random.default_rng(13)
    p = rng.standard_normal(10)
    g = rng.standard_normal(10)
    p1, m, v = mlp.adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=0.01)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-15)


# ------------------------------------------------------------------------- CG
def test_cg_matches_direct_solve():
    inst = small_instance(4, 8, 1, 3, 5)
    G = lsq.gram(inst.E, inst.W, 1)
    b = lsq.zt_apply(inst.E, inst.W, 1, inst.X[:, :1])[:, 0]
    y_direct = lsq.tri_solves(lsq.cholesky(G), b)
    y_cg, it = cg.pcg(G, b, tol=1e-13, maxiter=1000)
    assert np.abs(y_cg - y_direct).max() <= 1e-9 * np.abs(y_direct).max()
    pre = cg.block_jacobi(G, 3, 5)
    y_p, it_p = cg.pcg(G, b, precond=pre, tol=1e-13, maxiter=1000)
    assert np.abs(y_p - y_direct).max() <= 1e-9 * np.abs(y_direct).max()
    y0, it0 = cg.pcg(G, b, y0=y_direct, tol=1e-8)
    assert it0 == 0
    # the direct solve is the least-squares answer of the oracle
    y_ls = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X[:, :1])[:, 0]
    assert np.abs(y_direct - y_ls).max() <= 1e-9 * np.abs(y_ls).max()


def test_block_jacobi_tiles_inverts_its_blocks():
    """Applied to a column of G, the tile preconditioner returns the unit
    vector inside that column's block (it inverts G's diagonal blocks), for a
    block size that leaves a ragged last block; with one block it is G^{-1}."""
    inst = small_instance(4, 8, 1, 3, 5)
    G = lsq.gram(inst.E, inst.W, 1)
    n = G.shape[0]
    pre = cg.block_jacobi_tiles(G, 4)
    for j in range(n):
        z = pre(G[:, j].copy())
        s = slice(4 * (j // 4), min(4 * (j // 4) + 4, n))
        e = np.zeros(n)
        e[j] = 1.0
        assert np.abs(z[s] - e[s]).max() <= 1e-10
    full = cg.block_jacobi_tiles(G, n)
    b = np.arange(1.0, n + 1)
    assert np.abs(G @ full(b) - b).max() <= 1e-9 * np.abs(b).max()
    y, it = cg.pcg(G, b, precond=pre, tol=1e-13, maxiter=200)
    assert np.abs(G @ y - b).max() <= 1e-10 * np.abs(b).max()


# ------------------------------------------------ large-problem QR and condition
@pytest.mark.parametrize("m,n,panel", [(700, 300, 64), (500, 500, 128), (900, 130, 512), (257, 129, 32)])
def test_inplace_panel_qr_matches_lapack(m, n, panel):
    """The panel-by-panel in-place Householder QR (used for the stored values
    of the largest workload) gives LAPACK's factorization: same |R_ii|, same
    least-squares solution and residual norms, including ragged last panels
    (the trailing products are written in place by the BLAS), on a matrix
    with condition number 1e3."""
    rng = np.random.Generator(np.random.PCG64(m + n))
    Z = rng.standard_normal((m, n)) @ np.diag(np.logspace(0, 3, n))
    X = rng.standard_normal((m, 3))
    Y0, i0 = lsq.lstsq_qr(Z, X)
    Zc = np.asfortranarray(Z.copy())
    Y1, i1 = lsq.lstsq_qr_inplace(Zc, X, panel=panel)
    assert np.abs(Y1 - Y0).max() <= 1e-12 * np.abs(Y0).max()
    np.testing.assert_allclose(np.abs(i1["rdiag"]), np.abs(i0["rdiag"]), rtol=1e-12)
    np.testing.assert_allclose(i1["residual_norm"], i0["residual_norm"], rtol=1e-10)
    # Z now holds R on and above the diagonal: R^T R = Z^T Z
    R = np.triu(Zc[:n, :n])
    assert np.abs(R.T @ R - Z.T @ Z).max() <= 1e-12 * np.abs(Z.T @ Z).max()


def test_inplace_panel_qr_without_blas_handle(monkeypatch):
    """The same factorization when the BLAS cannot be reached directly
    (numpy's matmul on column chunks instead)."""
    monkeypatch.setattr(lsq, "_blas_gemm", lambda: None)
    rng = np.random.Generator(np.random.PCG64(3))
    Z = rng.standard_normal((600, 250)) @ np.diag(np.logspace(0, 3, 250))
    X = rng.standard_normal((600, 2))
    Y0, _ = lsq.lstsq_qr(Z, X)
    Y1, _ = lsq.lstsq_qr_inplace(np.asfortranarray(Z.copy()), X, panel=96)
    assert np.abs(Y1 - Y0).max() <= 1e-12 * np.abs(Y0).max()


def test_triu_cond_estimate_against_svd_and_diagonal():
    """Power / inverse iteration on R^T R: exact for a diagonal R (kappa =
    max|d| / min|d|), and within 1e-6 of the SVD value for a dense R with
    well-separated extreme singular values."""
    d = np.array([3.0, -0.5, 7.0, 0.02, 1.0])
    k, smax, smin = lsq.triu_cond_estimate(np.diag(d), iters=80)
    assert abs(k - 350.0) <= 1e-9 * 350 and abs(smax - 7.0) <= 1e-12 and abs(smin - 0.02) <= 1e-14
    rng = np.random.Generator(np.random.PCG64(5))
    A = rng.standard_normal((400, 300)) @ np.diag(np.logspace(0, 4, 300))
    R = np.linalg.qr(A, mode="r")
    k, _, _ = lsq.triu_cond_estimate(np.asfortranarray(R), iters=200)
    assert abs(k / np.linalg.cond(R) - 1) <= 1e-6


def test_cond_closed_form_single_member():
    """K = 1 with e = 1: Z = W, whose columns are orthogonal with squared norms
    the localization eigenvalues, so kappa(Z) = sqrt(lambda_1 / lambda_M)."""
    W, info = wl.localization_modes(6, 12, 9, 0.5)
    E = np.ones((72, 1))
    lam = info["eigvals"][:9]
    assert abs(lsq.cond(E, W, 1) / math.sqrt(lam[0] / lam[8]) - 1) <= 1e-10


def test_gram_lowprec_rounds_the_product_once():
    """Hand case: e = w = 1 + 2^-8.  The product 1 + 2^-7 + 2^-16 rounds to
    1 + 2^-7 in bfloat16 (8 significant bits), while rounding the factors
    first (1 + 2^-8 is a tie, to even: 1) would give 1.  So the Gram of the
    once-rounded Z is (1 + 2^-7)^2, not 1.  In float32 the product is exact."""
    E = np.array([[1.0 + 2.0 ** -8]])
    W = np.array([[1.0 + 2.0 ** -8]])
    G = lsq.gram_lowprec(E, W, 1, "bf16")
    assert G.shape == (1, 1) and G[0, 0] == (1.0 + 2.0 ** -7) ** 2
    G32 = lsq.gram_lowprec(E, W, 1, "fp32")
    assert G32[0, 0] == (1.0 + 2.0 ** -8) ** 4


def test_bf16_forms_round_the_fp32_product():
    """The bf16 forms round the float32 product of float32 copies of E and W:
    e = 1 + 2^-8 + 2^-30 has the float32 copy 1 + 2^-8 (2^-30 is below its 24
    bits), an exact tie for bfloat16 that rounds to even, 1; the float64
    product rounded once would have given 1 + 2^-7.  Split bf16 then has
    Hi = 1 and Lo = 2^-8 (the float32 value is recovered exactly).  The fp32
    form keeps the float64 product: fp32(1 + 2^-8 + 2^-30) = 1 + 2^-8."""
    E = np.array([[1.0 + 2.0 ** -8 + 2.0 ** -30]])
    W = np.array([[1.0]])
    assert lsq.form_z32(E, W, 1)[0, 0] == 1.0 + 2.0 ** -8
    assert lsq.gram_lowprec(E, W, 1, "bf16")[0, 0] == 1.0
    Hi, Lo = lsq.lowprec_operands(E, W, 1, "bf16x3")
    assert Hi[0, 0] == 1.0 and Lo[0, 0] == 2.0 ** -8
    assert lsq.lowprec_operands(E, W, 1, "fp32")[0][0, 0] == 1.0 + 2.0 ** -8
    # the float32 product is rounded to nearest even: (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24 is a tie
    # (half an ulp of 2^-23), to even: 1 + 2^-11; (1 + 2^-12 + 2^-23)(1 + 2^-12) =
    # 1 + 2^-11 + 2^-23 + 2^-24 + 2^-35 lies above the next tie and rounds up to 1 + 2^-11 + 2^-22
    a = np.array([[1.0 + 2.0 ** -12], [1.0 + 2.0 ** -12 + 2.0 ** -23]])
    z = lsq.form_z32(a, np.array([[1.0 + 2.0 ** -12], [1.0 + 2.0 ** -12]]), 1)
    assert z[0, 0] == 1.0 + 2.0 ** -11
    assert z[1, 0] == 1.0 + 2.0 ** -11 + 2.0 ** -22


def test_split_bf16_hand_cases_and_bound():
    """Split bfloat16: a value with at most 8 significant bits has Lo = 0; the
    hand value 1 + 2^-8 + 2^-20 gives Hi = 1 + 2^-7 (above the tie) and
    Lo = bf16(-2^-8 + 2^-20) = -2^-8; and in general |Z - Hi - Lo| <= 2^-16 |Z|
    (two roundings of 8 significant bits each)."""
    Hi, Lo = lsq.split_bf16(np.array([1.5, -3.0 * 2.0 ** -10, 1.0 + 2.0 ** -8 + 2.0 ** -20]))
    assert Hi[0] == 1.5 and Lo[0] == 0.0 and Hi[1] == -3.0 * 2.0 ** -10 and Lo[1] == 0.0
    assert Hi[2] == 1.0 + 2.0 ** -7 and Lo[2] == -(2.0 ** -8)
    rng = np.random.Generator(np.random.PCG64(11))
    Z = rng.standard_normal((300, 20)) * np.exp(rng.uniform(-5, 5, (300, 20)))
    Hi, Lo = lsq.split_bf16(Z)
    assert np.all(np.abs(Z - Hi - Lo) <= 2.0 ** -16 * np.abs(Z))


def test_gram_lowprec_split_bf16():
    """The three-product Gram equals (Hi + Lo)^T (Hi + Lo) - Lo^T Lo, is exact
    when Z has no more than 8 significant bits (Lo = 0), and lies within
    3 * 2^-16 |Z|^T |Z| of the exact Gram."""
    inst = small_instance(4, 8, 1, 3, 5)
    Z = lsq.form_z(inst.E, inst.W, 1)
    G3 = lsq.gram_lowprec(inst.E, inst.W, 1, "bf16x3")
    Hi, Lo = lsq.split_bf16(lsq.form_z32(inst.E, inst.W, 1))
    S = Hi + Lo
    assert np.abs(G3 - (S.T @ S - Lo.T @ Lo)).max() <= 1e-14 * np.abs(G3).max()
    assert np.all(np.abs(G3 - Z.T @ Z) <= 3 * 2.0 ** -16 * (np.abs(Z).T @ np.abs(Z)))
    Eb, Wb = lsq.round_bf16(inst.E), np.ones((inst.n_h, 1))
    Zb = lsq.form_z(Eb, Wb, 1)
    assert np.array_equal(lsq.gram_lowprec(Eb, Wb, 1, "bf16x3"), Zb.T @ Zb)


def test_separable_modes_match_the_generator():
    """The separable form of the generator's modes: the oracle's product
    U[a, m] Phi[i, m] at grid column a n_lon + i equals localization_modes'
    W to rounding (same modes, products in another order), and its columns
    are orthogonal with squared norms the eigenvalues (unit Fourier columns
    times orthonormal latitude vectors)."""
    for n_lat, n_lon, M, ell in ((6, 12, 20, 0.5), (8, 16, 37, 0.3)):
        U, Phi, info = wl.localization_factors(n_lat, n_lon, M, ell)
        W, info2 = wl.localization_modes(n_lat, n_lon, M, ell)
        Ws = lsq.separable_modes(U, Phi)
        assert np.abs(Ws - W).max() <= 8 * 2.0 ** -53 * np.abs(W).max()
        assert np.array_equal(info["eigvals"], info2["eigvals"])
        Gm = Ws.T @ Ws
        lam = info["eigvals"][:M]
        assert np.abs(np.diag(Gm) - lam).max() <= 1e-13 * lam.max()
        assert np.abs(Gm - np.diag(np.diag(Gm))).max() <= 1e-13 * lam.max()
        # lat-major: row a n_lon + i of W is U[a] * Phi[i]
        a, i, m = n_lat - 2, 3, M - 1
        assert Ws[a * n_lon + i, m] == U[a, m] * Phi[i, m]


def test_zt_apply_lowprec_hand_cases():
    """Reduced-precision Z^T x, hand values.  One row: x = 1 + 2^-8 + 2^-30
    has the float32 copy 1 + 2^-8, a bfloat16 tie that rounds to even, 1
    (rounding x straight to bfloat16 would give 1 + 2^-7); with e = w = 1 the
    bf16 product is 1 and the fp32 one 1 + 2^-8.  Two rows (n_h = 2):
    z = (1 + 2^-8)^2 = 1 + 2^-7 + 2^-16 rounds to 1 + 2^-7 in bfloat16 and
    2 * 0.5 = 1 stays; x = (3, 1 + 2^-9) rounds to (3, 1), so the bf16 value
    is 3 (1 + 2^-7) + 1; in fp32 every operand is exact and the value is the
    plain 3 (1 + 2^-8)^2 + (1 + 2^-9)."""
    one = np.array([[1.0]])
    x = np.array([[1.0 + 2.0 ** -8 + 2.0 ** -30]])
    assert lsq.zt_apply_lowprec(one, one, 1, x, "bf16")[0, 0] == 1.0
    assert lsq.round_bf16(x)[0, 0] == 1.0 + 2.0 ** -7
    assert lsq.zt_apply_lowprec(one, one, 1, x, "fp32")[0, 0] == 1.0 + 2.0 ** -8
    E = np.array([[1.0 + 2.0 ** -8], [2.0]])
    W = np.array([[1.0 + 2.0 ** -8], [0.5]])
    X = np.array([[3.0], [1.0 + 2.0 ** -9]])
    assert lsq.zt_apply_lowprec(E, W, 1, X, "bf16")[0, 0] == 3.0 * (1.0 + 2.0 ** -7) + 1.0
    assert lsq.zt_apply_lowprec(E, W, 1, X, "fp32")[0, 0] == 3.0 * (1.0 + 2.0 ** -8) ** 2 + (1.0 + 2.0 ** -9)
    with pytest.raises(ValueError):
        lsq.zt_apply_lowprec(E, W, 1, X, "bf16x3")


def test_zt_apply_lowprec_bound_and_layout():
    """On a random multi-level instance: the rounded product lies within the
    operand rounding bound of the exact Z^T X (bf16: |z~ - z| <= (2^-9 +
    2^-22)|z|, |x~ - x| <= (2^-9 + 2^-23)|x|; fp32: 2^-23 each, products
    included), differs from it (the rounding is there), and its column block
    of member k equals W^T (e_k o X) summed over levels up to that bound --
    the column order (k, m) and the row order (l, j) of Z."""
    inst = small_instance(3, 5, 2, 4, 6)
    rng = np.random.Generator(np.random.PCG64(17))
    X = rng.standard_normal((inst.n, 7))
    Z = lsq.form_z(inst.E, inst.W, inst.n_w)
    exact = Z.T @ X
    mag = np.abs(Z).T @ np.abs(X)
    for fmt, u in (("bf16", 2.0 ** -8 + 2.0 ** -20), ("fp32", 2.0 ** -22)):
        B = lsq.zt_apply_lowprec(inst.E, inst.W, inst.n_w, X, fmt)
        assert np.all(np.abs(B - exact) <= u * mag), fmt
        assert not np.array_equal(B, exact)
        for k in range(inst.K):
            blk = sum(inst.W.T @ (inst.E[l * inst.n_h:(l + 1) * inst.n_h, k:k + 1]
                                  * X[l * inst.n_h:(l + 1) * inst.n_h]) for l in range(inst.n_w))
            assert np.all(np.abs(B[k * inst.M:(k + 1) * inst.M] - blk) <= u * mag[k * inst.M:(k + 1) * inst.M])
