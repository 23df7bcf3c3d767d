"""Least-squares oracle: y = Z^+ x with Z formed explicitly and Householder QR.

Test infrastructure only (see the package docstring).

Z is the modulated square root of the horizontally localized covariance:
its column (k, m), at position k*M + m, is the element-wise product of the
scaled member z_k with the localization mode w_m repeated over the n_w levels
(eqs. SqrtOfC, SQRTofPCModulation and DiagZC of the paper).  Rows are in the
paper's segment order i = l*n_h + j (Sec. 3.4): level/kind l, grid column j.

Reading used for the operation itself: the paper's left inverse (eq.
InverseSquareRootSwift) needs n_w = K; for the general tall Z the library
computes the Moore-Penrose left inverse, i.e. the least-squares solution
argmin_y ||Z y - x||_2, which coincides with the paper's left inverse on
range(Z) (and everywhere when Z is square).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
import scipy.linalg.lapack as lapack

U64 = 2.0 ** -53


def form_z(E: np.ndarray, W: np.ndarray, n_w: int) -> np.ndarray:
    """Explicit Z (n x K*M): Z[l*n_h + j, k*M + m] = E[l*n_h + j, k] * W[j, m].

    Follows eq. SQRTofPCModulation: Z = [diag(z_1) C^{1/2}, ..., diag(z_K) C^{1/2}]
    with C^{1/2} the n_w-fold vertical stack of C_b^{1/2} = W (eq. SqrtOfC).
    """
    n, K = E.shape
    n_h, M = W.shape
    assert n == n_h * n_w
    C_half = np.tile(W, (n_w, 1))                      # eq. SqrtOfC
    return np.concatenate([E[:, k:k + 1] * C_half for k in range(K)], axis=1)


def separable_modes(U: np.ndarray, Phi: np.ndarray) -> np.ndarray:
    """Dense modes from separable factors on an n_lat x n_lon grid (grid column
    j = a*n_lon + i): W[a*n_lon + i, m] = U[a, m] * Phi[i, m], each product
    formed once in float64 (modes defined analytically need not be stored,
    Sec. 3.11; this is their value at each grid column)."""
    n_lat, M = U.shape
    n_lon = Phi.shape[0]
    return (U[:, None, :] * Phi[None, :, :]).reshape(n_lat * n_lon, M)


def localized_covariance(E: np.ndarray, W: np.ndarray, n_w: int) -> np.ndarray:
    """P^c = C o P^s (eq. HLocalizedPc) with P^s = E E^T and C = 1 (x) (W W^T) blocks."""
    Ps = E @ E.T                                       # eq. PsAndItsSquareRoot
    Cb = W @ W.T
    C = np.tile(Cb, (n_w, n_w))                        # eq. blockStructureCEqualBlocks
    return C * Ps


# ---------------------------------------------------------------- Householder QR
def householder_qr(A: np.ndarray):
    """Unblocked Householder QR of a tall matrix (for tiny inputs).

    Standard reflectors H_j = I - tau_j v_j v_j^T with v_j[0] = 1 and
    beta_j = -sign(alpha_j) ||x_j||, so that R[j, j] = beta_j.
    Returns (V, tau, R): V holds the reflectors below the diagonal.
    """
    A = np.array(A, dtype=np.float64, copy=True)
    m, n = A.shape
    tau = np.zeros(n)
    for j in range(n):
        x = A[j:, j]
        alpha = x[0]
        xnorm = np.linalg.norm(x[1:])
        if xnorm == 0.0:
            tau[j] = 0.0
            continue
        beta = -np.copysign(np.hypot(alpha, xnorm), alpha)
        tau[j] = (beta - alpha) / beta
        v = x.copy()
        v[0] = 1.0
        v[1:] = x[1:] / (alpha - beta)
        A[j:, j + 1:] -= tau[j] * np.outer(v, v @ A[j:, j + 1:])
        A[j, j] = beta
        A[j + 1:, j] = v[1:]
    R = np.triu(A[:n, :n])
    return A, tau, R


def apply_qt(V: np.ndarray, tau: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Q^T X for the reflectors of `householder_qr`."""
    X = np.array(X, dtype=np.float64, copy=True)
    n = V.shape[1]
    for j in range(n):
        v = np.concatenate([[1.0], V[j + 1:, j]])
        X[j:] -= tau[j] * np.outer(v, v @ X[j:])
    return X


# ----------------------------------------------------------- least squares
class RankDeficient(Exception):
    """Z has no left inverse: the QR diagonal has an (almost) zero entry."""


def lstsq_qr(Z: np.ndarray, X: np.ndarray, own: bool = False, check_rank: bool = True):
    """Least-squares solve min ||Z y - x|| for every column of X by Householder QR.

    Steps: Z = QR (LAPACK dgeqrf, or the unblocked `householder_qr` when own=True);
    rank check on diag(R); c = Q^T x (dormqr); y = R^{-1} c[:ncols] (dtrtrs).
    Returns (Y, info) with info = {"residual_norm": ||c[ncols:]|| per column,
    "rdiag": diag(R)}.
    """
    Z = np.asarray(Z, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    m, n = Z.shape
    if n > m:
        raise ValueError("Z must be tall (K*M <= n)")
    if own:
        V, tau, R = householder_qr(Z)
        C = apply_qt(V, tau, X)
    else:
        qr, tau, _, info = lapack.dgeqrf(np.array(Z, order="F", copy=True), overwrite_a=1)
        if info != 0:
            raise RuntimeError("dgeqrf failed")
        R = np.triu(qr[:n, :n])
        lwork = max(1, X.shape[1] * 64)
        C, _, info = lapack.dormqr("L", "T", qr, tau, np.asfortranarray(X.copy()), lwork)
        if info != 0:
            raise RuntimeError("dormqr failed")
    rd = np.abs(np.diag(R))
    if check_rank and (rd.size == 0 or rd.min() <= m * U64 * rd.max()):
        raise RankDeficient(f"min |R_ii| = {rd.min():.3e}, max = {rd.max():.3e}")
    Y = scipy.linalg.solve_triangular(R, C[:n], lower=False)
    info = {"residual_norm": np.linalg.norm(C[n:], axis=0), "rdiag": np.diag(R).copy()}
    return (Y[:, 0] if vec else Y), info


def form_z_fortran(E: np.ndarray, W: np.ndarray, n_w: int) -> np.ndarray:
    """`form_z` written column by column into one column-major array (no
    intermediate copies: the largest workload's Z is 34 GB)."""
    n, K = E.shape
    n_h, M = W.shape
    assert n == n_h * n_w
    Z = np.empty((n, K * M), order="F")
    for k in range(K):
        for l in range(n_w):
            Z[l * n_h:(l + 1) * n_h, k * M:(k + 1) * M] = E[l * n_h:(l + 1) * n_h, k:k + 1] * W
    return Z


def _larft(V: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Upper-triangular T of the compact WY form H_1 H_2 ... H_b = I - V T V^T
    (Schreiber and Van Loan), built column by column:
    T[j, j] = tau_j,  T[:j, j] = -tau_j T[:j, :j] (V[:, :j]^T v_j)."""
    b = V.shape[1]
    T = np.zeros((b, b))
    VtV = V.T @ V
    for j in range(b):
        T[j, j] = tau[j]
        if j:
            T[:j, j] = -tau[j] * (T[:j, :j] @ VtV[:j, j])
    return T


def _blas_gemm():
    """cblas_dgemm of the BLAS numpy itself links (located through
    threadpoolctl), for products written in place into strided column-major
    views; None if it cannot be found (numpy's matmul is used instead)."""
    import ctypes
    try:
        from threadpoolctl import threadpool_info
        for d in threadpool_info():
            if d.get("internal_api") != "openblas" or "numpy" not in d.get("filepath", ""):
                continue
            lib = ctypes.CDLL(d["filepath"])
            for name in ("scipy_cblas_dgemm64_", "cblas_dgemm64_", "cblas_dgemm"):
                if hasattr(lib, name):
                    f = getattr(lib, name)
                    i64 = ctypes.c_int64 if "64" in name else ctypes.c_int32
                    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i64, i64, i64, ctypes.c_double,
                                  ctypes.c_void_p, i64, ctypes.c_void_p, i64, ctypes.c_double, ctypes.c_void_p, i64]
                    f.restype = None
                    return f
    except Exception:
        return None
    return None


def _col_major(a):
    """(pointer, leading dimension) of a column-major (possibly strided) 2-D view."""
    assert a.dtype == np.float64 and a.strides[0] == 8 and a.strides[1] % 8 == 0
    return a.ctypes.data, max(a.strides[1] // 8, a.shape[0], 1)


def lstsq_qr_inplace(Z: np.ndarray, X: np.ndarray, panel: int = 512, progress=None):
    """Least squares by Householder QR, computed in place on a column-major Z.

    The same factorization as `lstsq_qr` (LAPACK's reflector convention),
    organized by panels so that a Z too large to copy can be factored and so
    that progress can be reported: each panel of `panel` columns is factored
    by LAPACK dgeqrf (numpy, mode "raw"), its reflectors are written back below
    the diagonal, and its Q_p^T = I - V T^T V^T (compact WY form) is applied
    to the trailing columns, C <- C - V (T^T (V^T C)), with the products
    written in place by the BLAS, and to X.  Afterwards
    y = R^{-1} (Q^T x)[:ncols] by block back substitution.
    Z is overwritten (R on and above the diagonal).  Returns (Y, info) as
    `lstsq_qr` does, info also holding "rdiag".
    """
    if not (Z.flags.f_contiguous and Z.dtype == np.float64):
        raise ValueError("Z must be a column-major float64 array")
    m, n = Z.shape
    if n > m:
        raise ValueError("Z must be tall (K*M <= n)")
    gemm = _blas_gemm()
    COL, NT, TR = 102, 111, 112
    C = np.array(X, dtype=np.float64, order="F", copy=True)
    if C.ndim == 1:
        C = C[:, None]
    for j0 in range(0, n, panel):
        j1 = min(n, j0 + panel)
        b = j1 - j0
        h, tau = np.linalg.qr(np.asfortranarray(Z[j0:, j0:j1]), mode="raw")
        A = h.T                                        # (m - j0) x b, R above, reflectors below
        Z[j0:, j0:j1] = A
        V = np.asfortranarray(np.tril(A, -1))
        V[np.arange(b), np.arange(b)] = 1.0
        Tt = np.asfortranarray(_larft(V, tau).T)
        if j1 < n:
            Cv = Z[j0:, j1:]                           # trailing columns, a strided view
            if gemm is not None:
                Wm = np.empty((b, n - j1), order="F")
                pc_, ldc = _col_major(Cv)
                gemm(COL, TR, NT, b, n - j1, m - j0, 1.0, V.ctypes.data, m - j0, pc_, ldc, 0.0,
                     Wm.ctypes.data, b)                # W = V^T C
                Wm = np.asfortranarray(Tt @ Wm)        # T^T W
                gemm(COL, NT, NT, m - j0, n - j1, b, -1.0, V.ctypes.data, m - j0, Wm.ctypes.data, b, 1.0,
                     pc_, ldc)                         # C <- C - V (T^T W)
            else:
                for c0 in range(j1, n, 2048):
                    blk = Z[j0:, c0:min(n, c0 + 2048)]
                    blk -= V @ (Tt @ (V.T @ blk))
        C[j0:] -= V @ (Tt @ (V.T @ C[j0:]))
        if progress is not None:
            progress(j1, n)
    rdiag = np.array([Z[i, i] for i in range(n)])
    Y = C[:n].copy()
    for i1 in range(n, 0, -panel):                     # back substitution by diagonal blocks
        i0 = max(0, i1 - panel)
        if i1 < n:
            Y[i0:i1] -= Z[i0:i1, i1:n] @ Y[i1:n]
        Y[i0:i1] = scipy.linalg.solve_triangular(np.triu(Z[i0:i1, i0:i1]), Y[i0:i1], lower=False)
    info = {"residual_norm": np.linalg.norm(C[n:], axis=0), "rdiag": rdiag}
    return Y, info


def triu_cond_estimate(R: np.ndarray, iters: int = 60, seed: int = 0):
    """2-norm condition number of an upper-triangular R (only its upper
    triangle is read; R may be a view into a larger array) by power
    iteration on R^T R for sigma_max and inverse iteration (two triangular
    solves by diagonal blocks) for sigma_min.  Returns (kappa, sigma_max,
    sigma_min); both iterations approach their singular value from the
    inside, so kappa is a lower bound that tightens with `iters`."""
    n = R.shape[0]
    blk = 1024

    def rmul(v):                                       # R v
        out = np.empty_like(v)
        for i0 in range(0, n, blk):
            i1 = min(n, i0 + blk)
            out[i0:i1] = np.triu(R[i0:i1, i0:i1]) @ v[i0:i1] + R[i0:i1, i1:n] @ v[i1:n]
        return out

    def rtmul(v):                                      # R^T v
        out = np.empty_like(v)
        for i0 in range(0, n, blk):
            i1 = min(n, i0 + blk)
            out[i0:i1] = np.triu(R[i0:i1, i0:i1]).T @ v[i0:i1] + R[:i0, i0:i1].T @ v[:i0]
        return out

    def rsolve(v):                                     # R^{-1} v
        y = v.copy()
        for i1 in range(n, 0, -blk):
            i0 = max(0, i1 - blk)
            if i1 < n:
                y[i0:i1] -= R[i0:i1, i1:n] @ y[i1:n]
            y[i0:i1] = scipy.linalg.solve_triangular(np.triu(R[i0:i1, i0:i1]), y[i0:i1], lower=False)
        return y

    def rtsolve(v):                                    # R^{-T} v
        y = v.copy()
        for i0 in range(0, n, blk):
            i1 = min(n, i0 + blk)
            if i0:
                y[i0:i1] -= R[:i0, i0:i1].T @ y[:i0]
            y[i0:i1] = scipy.linalg.solve_triangular(np.triu(R[i0:i1, i0:i1]), y[i0:i1], lower=False,
                                                     trans="T")
        return y

    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(n)
    w = rng.standard_normal(n)
    smax = smin_inv = 0.0
    for _ in range(iters):
        v /= np.linalg.norm(v)
        v = rtmul(rmul(v))
        smax = math.sqrt(np.linalg.norm(v))
        w /= np.linalg.norm(w)
        w = rsolve(rtsolve(w))
        smin_inv = math.sqrt(np.linalg.norm(w))
    smin = 1.0 / smin_inv
    return smax / smin, smax, smin


def left_inverse_apply(E: np.ndarray, W: np.ndarray, n_w: int, X: np.ndarray,
                       own: bool = False):
    """The operation the library performs: Y = Z^+ X (eq. svTransform with the
    Moore-Penrose left inverse), by explicit Z and Householder QR."""
    return lstsq_qr(form_z(E, W, n_w), X, own=own)[0]


def project_range(E: np.ndarray, W: np.ndarray, n_w: int, X: np.ndarray) -> np.ndarray:
    """Orthogonal projection Q Q^T X onto range(Z) (Q from the QR of Z)."""
    Z = form_z(E, W, n_w)
    Q, _ = np.linalg.qr(Z, mode="reduced")
    return Q @ (Q.T @ X)


def cond(E: np.ndarray, W: np.ndarray, n_w: int) -> float:
    """2-norm condition number of Z from its singular values."""
    s = np.linalg.svd(form_z(E, W, n_w), compute_uv=False)
    return float(s[0] / s[-1])


# ------------------------------------------------ reference sub-steps (explicit)
def zt_apply(E, W, n_w, X):
    """Z^T X with Z explicit."""
    return form_z(E, W, n_w).T @ X


def z_apply(E, W, n_w, Y):
    """Z Y with Z explicit (the forward square root x = Z x~)."""
    return form_z(E, W, n_w) @ Y


def gram(E, W, n_w):
    """Z^T Z with Z explicit."""
    Z = form_z(E, W, n_w)
    return Z.T @ Z


def column_grams(E: np.ndarray, n_h: int, n_w: int) -> np.ndarray:
    """Per-grid-column Grams S[j] = A_j^T A_j (K x K), A_j the n_w x K rows of
    the members that belong to grid column j (the paper's A_m, Sec. 3.9)."""
    n, K = E.shape
    A = E.reshape(n_w, n_h, K)                          # A[l, j, k]
    return np.einsum("ljk,ljq->jkq", A, A)


def cholesky(G):
    """Lower Cholesky factor (LAPACK dpotrf through numpy)."""
    return np.linalg.cholesky(G)


def tri_solves(L, B):
    """Y = L^{-T} (L^{-1} B)."""
    Z = scipy.linalg.solve_triangular(L, B, lower=True)
    return scipy.linalg.solve_triangular(L.T, Z, lower=False)


# --------------------------------------------------- low-precision copies of Z
def round_fp32(x: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest float32 (ties to even), returned as float64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (8 significant bits, ties to
    even), returned as float64.  Written from the format's definition: keep the
    sign, the 8 exponent bits and the top 7 fraction bits of the float32 layout,
    i.e. round the binary64 significand to 8 bits.  Magnitudes below the
    smallest normal bfloat16 (2**-126) are flushed to a signed zero; magnitudes
    that would overflow raise (they never occur for these inputs)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = np.abs(x) >= 2.0 ** -126
    out[~nz] = np.copysign(0.0, x[~nz])
    m, e = np.frexp(x[nz])            # x = m * 2**e, 0.5 <= |m| < 1
    if np.any(e > 128):
        raise ValueError("value outside the bfloat16 range")
    scaled = np.ldexp(m, 8)           # |scaled| in [128, 256): integer part has 8 bits
    r = np.round(scaled)              # numpy rounds half to even
    out[nz] = np.ldexp(r, e - 8)
    return out


def split_bf16(Z: np.ndarray):
    """Split bfloat16 representation Z ~ Hi + Lo: Hi = bf16(Z), Lo = bf16(Z - Hi)
    (the difference is exact in float64).  Returned as float64 arrays."""
    Hi = round_bf16(Z)
    return Hi, round_bf16(Z - Hi)


def form_z32(E: np.ndarray, W: np.ndarray, n_w: int) -> np.ndarray:
    """Z32[l*n_h + j, k*M + m] = fl32(fp32(E[l*n_h + j, k]) * fp32(W[j, m])): Z formed
    in float32 arithmetic from float32 copies of E and W (each value rounded to
    nearest even once, the product rounded once), returned as float64."""
    E32 = np.asarray(E, dtype=np.float64).astype(np.float32)
    C32 = np.tile(np.asarray(W, dtype=np.float64).astype(np.float32), (n_w, 1))
    return np.concatenate([E32[:, k:k + 1] * C32 for k in range(E32.shape[1])], axis=1).astype(np.float64)


def lowprec_operands(E, W, n_w, fmt: str):
    """The rounded square root whose Gram the reduced-precision modes form:
    "fp32": [fp32(Z)], each FP64 product E[i,k]*W[j,m] rounded once to float32;
    "bf16": [bf16(Z32)];  "bf16x3": [Hi, Lo] = split_bf16(Z32),
    with Z32 the float32 product of float32 copies of E and W (form_z32)."""
    if fmt == "fp32":
        return [round_fp32(form_z(E, W, n_w))]
    Z32 = form_z32(E, W, n_w)
    if fmt == "bf16":
        return [round_bf16(Z32)]
    if fmt == "bf16x3":
        return list(split_bf16(Z32))
    raise ValueError(fmt)


def round_rhs(X: np.ndarray, fmt: str) -> np.ndarray:
    """The right-hand sides as the reduced-precision Z^T x reads them:
    "fp32": fp32(x); "bf16": bf16(fp32(x)) -- rounded to float32 first, then
    to bfloat16, both to nearest even (the two roundings can differ from one
    direct rounding to bfloat16 at a float32 tie).  Returned as float64."""
    if fmt == "fp32":
        return round_fp32(X)
    if fmt == "bf16":
        return round_bf16(round_fp32(X))
    raise ValueError(fmt)


def zt_apply_lowprec(E, W, n_w, X, fmt: str):
    """Exact (float64) product Zt^T Xt of the reduced-precision Z^T x: Zt the
    rounded square root of `lowprec_operands` ("fp32" or "bf16") and Xt the
    rounded right-hand sides of `round_rhs`.  The GPU accumulates these
    products in float32; this is the value that accumulation approximates."""
    Zt = lowprec_operands(E, W, n_w, fmt)[0]
    return Zt.T @ round_rhs(X, fmt)


def gram_lowprec(E, W, n_w, fmt: str):
    """Exact (float64) Gram of the rounded square root of `lowprec_operands`:
    Zt^T Zt for "bf16" and "fp32"; for "bf16x3" the three-product split-bf16
    Gram Hi^T Hi + Hi^T Lo + Lo^T Hi (the Lo^T Lo term is left out)."""
    ops = lowprec_operands(E, W, n_w, fmt)
    if fmt == "bf16x3":
        Hi, Lo = ops
        return Hi.T @ Hi + Hi.T @ Lo + Lo.T @ Hi
    Zt = ops[0]
    return Zt.T @ Zt
