"""Host-side checks of the seeded synthetic workload generators."""
import numpy as np

import workloads as wl


def _dense_corr(n_lat, n_lon, length):
    p = wl.latlon_points(n_lat, n_lon)
    d2 = ((p[:, None, :] - p[None, :, :]) ** 2).sum(-1)
    return np.exp(-d2 / (2 * length * length))


def test_circulant_spectrum_matches_dense():
    for L in (0.3, 0.08):
        C = _dense_corr(6, 12, L)
        lam = np.sort(np.linalg.eigvalsh(C))[::-1]
        got = []
        for q, l, u in wl.circulant_spectrum(6, 12, L):
            got += list(l) * (1 if q in (0, 6) else 2)
        assert np.abs(np.sort(got)[::-1] - lam).max() <= 1e-12


def test_localization_modes_are_scaled_orthogonal_eigenvectors():
    C = _dense_corr(6, 12, 0.4)
    W, info = wl.localization_modes(6, 12, 72, 0.4)
    assert np.abs(W @ W.T - C).max() <= 1e-12
    W, info = wl.localization_modes(6, 12, 10, 0.4)
    D = W.T @ W
    assert np.abs(D - np.diag(np.diag(D))).max() <= 1e-12
    assert np.abs(C @ W - W * np.diag(D)[None, :]).max() <= 1e-12
    assert info["gap"] >= 1.0


def test_grf_unit_variance_and_correlation():
    rng = np.random.default_rng(0)
    x = wl.grf_draws(4, 8, 40000, 0.3, rng)
    emp = x @ x.T / x.shape[1]
    assert np.abs(emp - _dense_corr(4, 8, 0.3)).max() < 0.05


def test_config_shapes_and_determinism():
    a = wl.config(1)
    b = wl.config(1)
    assert a.E.shape == (512, 8) and a.W.shape == (512, 32) and a.X.shape == (512, 16)
    assert np.array_equal(a.E, b.E) and np.array_equal(a.X, b.X)
    assert a.E.flags.f_contiguous and a.W.flags.f_contiguous


def test_batched_params_constraints():
    ps = wl.batched_params()
    assert len(ps) == 64
    for p in ps:
        n = p["n_lat"] * p["n_lon"]
        assert 32 <= p["n_lat"] <= 96 and p["n_lon"] == 2 * p["n_lat"]
        assert p["K"] in (8, 16, 32, 64) and p["M"] % 32 == 0 and 32 <= p["M"] <= 256
        assert p["K"] * p["M"] <= n and 8 <= p["R"] <= 128


def test_generation_independent_of_blas_threads():
    """The eigensolvers run single-threaded inside the generator, so the
    inputs are the same bytes whatever thread count the caller's BLAS has
    (stored oracle values for the largest workload depend on this)."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        a = wl.config(2, R=2)
    with threadpool_limits(limits=4):
        b = wl.config(2, R=2)
    assert np.array_equal(a.E, b.E) and np.array_equal(a.W, b.W) and np.array_equal(a.X, b.X)
