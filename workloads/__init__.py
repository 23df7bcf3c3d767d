"""Seeded synthetic workloads shared by the oracle-side tests, the GPU tests and the bench.

This module generates inputs only; it holds none of the left-inverse
arithmetic.  Everything here is a statement of the workload:

* a regular latitude-longitude grid on the unit sphere (the paper's experiment
  uses such a grid, Sec. 4.1; cell-centred latitudes are used here);
* Gaussian random fields (GRFs) with a chordal-Gaussian correlation
  exp(-d^2 / (2 l^2)), drawn exactly through the block-circulant (in
  longitude) structure of an isotropic kernel on a regular lat-lon grid;
* localization square-root modes W = V_b Delta_b^{1/2}, the leading M
  eigenpairs of a chordal-Gaussian localization block C_b (the paper's choice
  of square root, Sec. 3.7, truncated to M modes);
* right-hand sides x ~ N(0, 1).

Layouts (all float64, column-major as the library expects):
  E : n x K, rows in segment order i = l * n_h + j (level l, grid column j),
      already scaled by 1/sqrt(K-1) (the paper's z_k, eq. zkDefinition);
  W : n_h x M;
  X : n x R.
Grid columns are flattened latitude-major: j = lat * n_lon + lon.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from threadpoolctl import threadpool_limits

__all__ = [
    "latlon_points", "circulant_spectrum", "grf_draws", "localization_modes",
    "Instance", "make_instance", "config", "batched_config", "CONFIG_NAMES", "mlp_init",
    "multilevel_config", "MULTILEVEL", "MULTILEVEL_NAME",
]


def latlon_points(n_lat: int, n_lon: int) -> np.ndarray:
    """Unit vectors of a cell-centred lat-lon grid, latitude-major, shape (n_lat*n_lon, 3)."""
    lat = -0.5 * math.pi + (np.arange(n_lat) + 0.5) * math.pi / n_lat
    lon = 2.0 * math.pi * np.arange(n_lon) / n_lon
    cl, sl = np.cos(lat)[:, None], np.sin(lat)[:, None]
    p = np.stack([np.broadcast_to(cl * np.cos(lon)[None, :], (n_lat, n_lon)),
                  np.broadcast_to(cl * np.sin(lon)[None, :], (n_lat, n_lon)),
                  np.broadcast_to(sl, (n_lat, n_lon))], axis=-1)
    return p.reshape(n_lat * n_lon, 3)


def _one_thread(fn):
    """Run fn with single-threaded BLAS: LAPACK's eigensolvers give slightly
    different bits for different thread counts, and the near-degenerate
    eigenpairs of these kernels turn those bits into different fields, so the
    generated workload would depend on the host's thread count."""
    def wrapped(*a, **k):
        with threadpool_limits(limits=1):
            return fn(*a, **k)
    wrapped.__name__, wrapped.__doc__ = fn.__name__, fn.__doc__
    return wrapped


@_one_thread
def circulant_spectrum(n_lat: int, n_lon: int, length: float):
    """Eigen-decomposition of the chordal-Gaussian correlation on the grid.

    The correlation between (a, i) and (b, i') depends on (a, b, i - i' mod n_lon)
    only, so Fourier modes in longitude decouple it into n_lon//2 + 1 real
    symmetric n_lat x n_lat problems.  Returns a list of (q, eigvals, eigvecs),
    eigvals descending, one entry per longitudinal wavenumber q.
    """
    lat = -0.5 * math.pi + (np.arange(n_lat) + 0.5) * math.pi / n_lat
    dlon = 2.0 * math.pi * np.arange(n_lon) / n_lon
    ca, sa = np.cos(lat), np.sin(lat)
    # squared chordal distance 2 - 2 cos(angle)
    cosang = (ca[:, None, None] * ca[None, :, None] * np.cos(dlon)[None, None, :]
              + sa[:, None, None] * sa[None, :, None])
    f = np.exp(-(2.0 - 2.0 * cosang) / (2.0 * length * length))
    # f is even in the longitude offset, so its DFT is real: C_hat_q = sum_d f_d cos(2 pi q d / N)
    fh = np.fft.rfft(f, axis=2).real
    out = []
    for q in range(n_lon // 2 + 1):
        ch = 0.5 * (fh[:, :, q] + fh[:, :, q].T)
        lam, u = np.linalg.eigh(ch)
        order = np.argsort(-lam, kind="stable")
        out.append((q, lam[order], u[:, order]))
    return out


def _mode_columns(q: int, n_lon: int):
    """Real longitudinal basis vectors for wavenumber q: list of (kind, vector) with unit norm."""
    i = np.arange(n_lon)
    if q == 0:
        return [("cos", np.full(n_lon, 1.0 / math.sqrt(n_lon)))]
    if 2 * q == n_lon:
        return [("cos", np.cos(math.pi * i) / math.sqrt(n_lon))]
    s = math.sqrt(2.0 / n_lon)
    ang = 2.0 * math.pi * q * i / n_lon
    return [("cos", s * np.cos(ang)), ("sin", s * np.sin(ang))]


@_one_thread
def grf_draws(n_lat: int, n_lon: int, count: int, length: float,
              rng: np.random.Generator, spectrum=None) -> np.ndarray:
    """`count` independent zero-mean unit-variance GRF draws, shape (n_h, count).

    Exact sampling through the spectral square root of the correlation matrix
    (tiny negative eigenvalues clipped to zero).
    """
    if spectrum is None:
        spectrum = circulant_spectrum(n_lat, n_lon, length)
    n_h = n_lat * n_lon
    out = np.zeros((n_lat, n_lon, count))
    for q, lam, u in spectrum:
        amp = np.sqrt(np.clip(lam, 0.0, None))
        for _, col in _mode_columns(q, n_lon):
            xi = rng.standard_normal((lam.shape[0], count))
            lat_part = u @ (amp[:, None] * xi)                   # n_lat x count
            out += lat_part[:, None, :] * col[None, :, None]
    return out.reshape(n_h, count)


@_one_thread
def localization_factors(n_lat: int, n_lon: int, M: int, length: float):
    """The M leading localization modes of `localization_modes` in separable
    form: mode m is sqrt(lambda_m) u_m (a latitude eigenvector, n_lat values)
    times a real Fourier mode in longitude (n_lon values), same order.
    Returns (U, Phi, info): U (n_lat x M) = sqrt(lambda_m) u_m, Phi (n_lon x M)
    the unit-norm cos/sin columns; the mode at grid column j = a n_lon + i is
    U[a, m] Phi[i, m]."""
    spec = circulant_spectrum(n_lat, n_lon, length)
    cands = []
    for q, lam, u in spec:
        for kind_idx, (kind, _) in enumerate(_mode_columns(q, n_lon)):
            for r in range(lam.shape[0]):
                cands.append((-lam[r], q, kind_idx, r))
    cands.sort()
    if M > len(cands):
        raise ValueError("M exceeds the number of grid columns")
    by_q = {q: (lam, u) for q, lam, u in spec}
    U = np.empty((n_lat, M))
    Phi = np.empty((n_lon, M))
    for c in range(M):
        _, q, kind_idx, r = cands[c]
        lam, u = by_q[q]
        U[:, c] = math.sqrt(max(lam[r], 0.0)) * u[:, r]
        Phi[:, c] = _mode_columns(q, n_lon)[kind_idx][1]
    lead = np.array([-c[0] for c in cands[:M + 1]])
    gap = lead[M - 1] / lead[M] if M < len(cands) and lead[M] > 0 else float("inf")
    return U, Phi, {"eigvals": lead, "gap": float(gap)}


def localization_modes(n_lat: int, n_lon: int, M: int, length: float):
    """W = V_b Delta_b^{1/2} from the M leading eigenpairs of the localization block.

    Eigenvalues are sorted descending; exact ties (the cos/sin pair of one
    wavenumber) are broken by (wavenumber, cos before sin).  Returns (W, info)
    with info = {"eigvals": leading M+1 eigenvalues, "gap": lam_M / lam_{M+1}}.
    """
    spec = circulant_spectrum(n_lat, n_lon, length)
    cands = []
    for q, lam, u in spec:
        for kind_idx, (kind, _) in enumerate(_mode_columns(q, n_lon)):
            for r in range(lam.shape[0]):
                cands.append((-lam[r], q, kind_idx, r))
    cands.sort()
    if M > len(cands):
        raise ValueError("M exceeds the number of grid columns")
    by_q = {q: (lam, u) for q, lam, u in spec}
    W = np.empty((n_lat * n_lon, M))
    for c in range(M):
        neg, q, kind_idx, r = cands[c]
        lam, u = by_q[q]
        col = _mode_columns(q, n_lon)[kind_idx][1]
        v = (u[:, r][:, None] * col[None, :]).reshape(-1)
        W[:, c] = math.sqrt(max(lam[r], 0.0)) * v
    lead = np.array([-c[0] for c in cands[:M + 1]])
    gap = lead[M - 1] / lead[M] if M < len(cands) and lead[M] > 0 else float("inf")
    return W, {"eigvals": lead, "gap": float(gap)}


@dataclasses.dataclass
class Instance:
    """One problem: E (n x K, scaled members), W (n_h x M), X (n x R)."""
    n_lat: int
    n_lon: int
    n_w: int
    K: int
    M: int
    E: np.ndarray
    W: np.ndarray
    X: np.ndarray
    seed: int
    info: dict

    @property
    def n_h(self) -> int:
        return self.n_lat * self.n_lon

    @property
    def n(self) -> int:
        return self.n_h * self.n_w

    @property
    def KM(self) -> int:
        return self.K * self.M

    @property
    def R(self) -> int:
        return self.X.shape[1]


def make_instance(n_lat: int, n_lon: int, K: int, M: int, R: int, l_ens: float,
                  l_loc: float, seed: int, n_w: int = 1, centring: str = "none",
                  W: Optional[np.ndarray] = None, W_info: Optional[dict] = None) -> Instance:
    """Build one seeded instance.

    centring:
      "none"     population-mean-zero draws, no sample-mean subtraction (default);
      "discard"  the paper's remedy (Sec. 4.2): draw K+4 members, subtract their
                 mean, discard 4 chosen at random, keep K;
      "sample"   subtract the K-member sample mean (makes Z rank deficient; only
                 for failure tests).
    Members are scaled by 1/sqrt(K-1) (eq. zkDefinition).
    """
    rng_e = np.random.Generator(np.random.PCG64(seed + 1))
    rng_x = np.random.Generator(np.random.PCG64(seed + 2))
    n_h = n_lat * n_lon
    spec = circulant_spectrum(n_lat, n_lon, l_ens)
    Kd = K + 4 if centring == "discard" else K
    # each level draws independent fields (no vertical correlation is needed
    # for the left inverse; the paper's P has one, which is irrelevant here)
    E = np.empty((n_w * n_h, Kd))
    for level in range(n_w):
        E[level * n_h:(level + 1) * n_h, :] = grf_draws(n_lat, n_lon, Kd, l_ens, rng_e, spec)
    if centring == "discard":
        E = E - E.mean(axis=1, keepdims=True)
        drop = rng_e.choice(Kd, size=4, replace=False)
        E = E[:, np.setdiff1d(np.arange(Kd), drop)]
    elif centring == "sample":
        E = E - E.mean(axis=1, keepdims=True)
    elif centring != "none":
        raise ValueError(centring)
    E = np.asfortranarray(E / math.sqrt(K - 1)) if K > 1 else np.asfortranarray(E)
    if W is None:
        W, W_info = localization_modes(n_lat, n_lon, M, l_loc)
    X = np.asfortranarray(rng_x.standard_normal((n_w * n_h, R)))
    return Instance(n_lat, n_lon, n_w, K, M, E, np.asfortranarray(W), X, seed,
                    {"loc_gap": (W_info or {}).get("gap"), "l_ens": l_ens, "l_loc": l_loc,
                     "centring": centring})


# The benchmark configurations: (n_lat, n_lon, K, M, R, l_ens, l_loc, seed)
_CONFIGS = {
    1: (16, 32, 8, 32, 16, 0.08, 0.25, 1000),
    2: (64, 128, 32, 128, 256, 0.05, 0.2, 2000),
    4: (256, 512, 64, 512, 1024, 0.02, 0.1, 4000),
}
CONFIG_NAMES = {
    1: "c1_n512_K8_M32_R16",
    2: "c2_n8192_K32_M128_R256",
    3: "c3_batched64_uneven",
    4: "c4_n131072_K64_M512_R1024",
    5: "c5_learned_n131072_K64_M512",
}


# A multi-level instance (n_w levels of the same horizontal grid share the
# horizontal localization modes): 64x128 grid, 8 levels, K = 32, M = 128,
# 256 right-hand sides; Z is 65536 x 4096.
MULTILEVEL = dict(n_lat=64, n_lon=128, n_w=8, K=32, M=128, R=256, l_ens=0.05, l_loc=0.2, seed=6000)
MULTILEVEL_NAME = "ml_n65536_nw8_K32_M128_R256"


def multilevel_config() -> Instance:
    """The multi-level instance (each level draws independent members)."""
    p = MULTILEVEL
    return make_instance(p["n_lat"], p["n_lon"], p["K"], p["M"], p["R"], p["l_ens"], p["l_loc"], p["seed"],
                         n_w=p["n_w"])


def config_params(c: int) -> dict:
    """Generator parameters of single-problem configuration c (5 reuses 4's)."""
    n_lat, n_lon, K, M, R, l_ens, l_loc, seed = _CONFIGS[4 if c == 5 else c]
    return dict(n_lat=n_lat, n_lon=n_lon, K=K, M=M, R=R, l_ens=l_ens, l_loc=l_loc, seed=seed)


def config(c: int, R: Optional[int] = None) -> Instance:
    """Instance for single-problem configuration 1, 2 or 4 (5 reuses 4's shapes)."""
    if c == 5:
        c = 4
    n_lat, n_lon, K, M, R0, l_ens, l_loc, seed = _CONFIGS[c]
    return make_instance(n_lat, n_lon, K, M, R0 if R is None else R, l_ens, l_loc, seed)


def batched_params(count: int = 64, seed: int = 3000) -> List[dict]:
    """Shapes of the uneven batch: grids 32x64..96x192, K in {8,16,32,64},
    M in {32,...,256} (multiples of 32), 8..128 right-hand sides, and
    K*M <= n (resampled until it holds).  Near K*M = n the lat-lon grid, whose
    rows crowd together near the poles, makes Z ill-conditioned (condition
    numbers of 1e5-1e6 occur in this batch)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(count):
        n_lat = int(rng.choice(np.arange(32, 97, 8)))
        n_lon = 2 * n_lat
        while True:
            K = int(rng.choice([8, 16, 32, 64]))
            M = int(rng.choice(np.arange(32, 257, 32)))
            if K * M <= n_lat * n_lon:
                break
        R = int(rng.integers(8, 129))
        out.append(dict(n_lat=n_lat, n_lon=n_lon, K=K, M=M, R=R, seed=seed + 1 + b))
    return out


def batched_config(count: int = 64, seed: int = 3000, scale: float = 1.0) -> List[Instance]:
    """The uneven batch.  `scale` < 1 shrinks every grid (for quick tests),
    reducing M where needed so that K*M <= n/2 still holds."""
    insts = []
    cache = {}
    for p in batched_params(count, seed):
        n_lat = max(4, int(round(p["n_lat"] * scale)))
        n_lon = 2 * n_lat
        K, M = p["K"], p["M"]
        if scale != 1.0:
            M = max(1, min(M, (n_lat * n_lon) // (2 * K)))
        key = (n_lat, n_lon, M)
        if key not in cache:
            cache[key] = localization_modes(n_lat, n_lon, M, 0.2)
        W, info = cache[key]
        insts.append(make_instance(n_lat, n_lon, K, M, p["R"], 0.05, 0.2, p["seed"],
                                   W=W, W_info=info))
    return insts


def mlp_init(d: int, h: int, seed: int, bias_scale: float = 0.0):
    """Seeded float32 starting parameters of the warm-start network:
    W1 (h x d) ~ N(0, 1/d), b1 (h), W2 (d x h) ~ N(0, 1/h), b2 (d); biases
    N(0, bias_scale^2) (zero by default)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = (rng.standard_normal((h, d)) / math.sqrt(d)).astype(np.float32)
    b1 = (bias_scale * rng.standard_normal(h)).astype(np.float32)
    W2 = (rng.standard_normal((d, h)) / math.sqrt(h)).astype(np.float32)
    b2 = (bias_scale * rng.standard_normal(d)).astype(np.float32)
    return W1, b1, W2, b2

