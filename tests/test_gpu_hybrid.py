"""The Hybrid covariance product in standardized variables (Sec. 2.2, eq.
svCBKHybrid) on the GPU, through the C ABI, against the oracle's explicit
matrices: element by element within the rounding bound of its two products,
in place, over several levels, and as the end of the paper's chain (the
forecast members mapped to standardized variables by the left inverse)."""
import ctypes

import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import hybrid, lsq
from tests.gpu_util import U64, dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu


def _factors(n_h, n_w, K, L, seed):
    rng = np.random.default_rng(seed)
    Et = rng.standard_normal((n_h * n_w, K)) / np.sqrt(K - 1)
    Wt = rng.standard_normal((n_h, L))
    Wt /= np.linalg.norm(Wt, axis=1, keepdims=True)
    return Et, Wt


def _bound(Et, Wt, n_w, beta, V):
    """|(1 - b) v + b Z (Z^T v)| rounding: Z^T v over n~ terms, Z b over K L
    terms, each product formed once (e * w), plus the final combination."""
    Za = np.abs(lsq.form_z(Et, Wt, n_w))
    n, KL = Za.shape
    g = (n + KL + 4) * U64
    return 2 * g * beta * (Za @ (Za.T @ np.abs(V))) + 2 * U64 * np.abs((1 - beta) * V) + 1e-300


@pytest.mark.parametrize("shape", [(40, 1, 6, 5, 3), (333, 1, 16, 24, 70), (96, 2, 5, 7, 17), (50, 3, 9, 16, 130)])
@pytest.mark.parametrize("beta", [0.35, 1.0])
def test_hybrid_matches_explicit_matrix(shape, beta):
    n_h, n_w, K, L, R = shape
    Et, Wt = _factors(n_h, n_w, K, L, 5 + n_h)
    V = np.random.default_rng(6).standard_normal((n_h * n_w, R))
    Out = empty(n_h * n_w, R)
    work = empty(K * L, R)
    pc.pc_hybrid_apply(dev(Et), dev(Wt), beta, dev(V), Out, work, n_w=n_w)
    got = host(Out)
    ref = hybrid.hybrid_apply(Et, Wt, n_w, beta, V)
    assert np.all(np.abs(got - ref) <= _bound(Et, Wt, n_w, beta, V)), np.abs(got - ref).max()


def test_hybrid_in_place_and_beta_zero():
    Et, Wt = _factors(120, 1, 8, 12, 21)
    V = np.random.default_rng(7).standard_normal((120, 9))
    Vd = dev(V)
    work = empty(96, 9)
    pc.pc_hybrid_apply(dev(Et), dev(Wt), 0.5, Vd, Vd, work)
    ref = hybrid.hybrid_apply(Et, Wt, 1, 0.5, V)
    assert np.all(np.abs(host(Vd) - ref) <= _bound(Et, Wt, 1, 0.5, V))
    Out = empty(120, 9)
    pc.pc_hybrid_apply(dev(Et), dev(Wt), 0.0, dev(V), Out, work)
    assert np.array_equal(host(Out), V)      # (1 - 0) v + 0 (...) = v exactly


def test_chain_from_forecast_members():
    """Standardized members e~ = Z^+ z^f (the left inverse of the square
    root, Sec. 2.1 eq. svTransform) from a plan, then the Hybrid over the
    n~ = K M standardized variables with a localization given by unit-norm
    modes, against the oracle's QR left inverse and explicit Hybrid."""
    clim = wl.make_instance(8, 16, 6, 12, 1, 0.15, 0.5, 81)
    fc = wl.make_instance(8, 16, 10, 12, 1, 0.15, 0.5, 82)     # 10 forecast members on the same grid
    Ef = fc.E
    plan = pc.Plan([inst_dict(clim, max_rhs=Ef.shape[1])], max_refine=2)
    plan.factor()
    Et_d = empty(clim.KM, Ef.shape[1])
    plan.apply([dev(Ef)], [Et_d])
    plan.close()
    Et_ref = lsq.left_inverse_apply(clim.E, clim.W, clim.n_w, Ef)
    assert np.abs(host(Et_d) - Et_ref).max() <= 1e-11 * np.abs(Et_ref).max()
    nt = clim.KM
    rng = np.random.default_rng(83)
    Wt = rng.standard_normal((nt, 20))
    Wt /= np.linalg.norm(Wt, axis=1, keepdims=True)
    V = rng.standard_normal((nt, 11))
    beta = 0.7
    Out = empty(nt, 11)
    pc.pc_hybrid_apply(Et_d, dev(Wt), beta, dev(V), Out, empty(Ef.shape[1] * 20, 11))
    ref = hybrid.hybrid_apply(Et_ref, Wt, 1, beta, V)
    assert np.abs(host(Out) - ref).max() <= 1e-10 * np.abs(ref).max()
    # positive definite with margin 1 - beta on these vectors: v^T P~h v >= (1 - beta) |v|^2
    q = np.sum(V * host(Out), axis=0)
    assert np.all(q >= (1 - beta) * np.sum(V * V, axis=0) * (1 - 1e-12))


def test_hybrid_argument_errors():
    lib = pc.load_library()
    Et, Wt = _factors(30, 1, 4, 5, 3)
    E, W, V, Out, work = dev(Et), dev(Wt), dev(np.ones((30, 2))), empty(30, 2), empty(20, 2)
    inst = pc.PcInstance(30, 1, 4, 5, E.data_ptr(), 30, W.data_ptr(), 30, 0)
    call = lambda beta, ldwork: lib.pc_hybrid_apply(ctypes.byref(inst), beta, V.data_ptr(), 30, 2,
                                                    Out.data_ptr(), 30, work.data_ptr(), ldwork, None)
    assert call(1.5, 20) == pc.PC_ERR_INVALID_ARG
    assert call(float("nan"), 20) == pc.PC_ERR_INVALID_ARG
    assert call(0.5, 19) == pc.PC_ERR_INVALID_ARG
    assert call(0.5, 20) == pc.PC_OK
    bad = pc.PcInstance(0, 1, 4, 5, E.data_ptr(), 30, W.data_ptr(), 30, 0)
    assert lib.pc_hybrid_apply(ctypes.byref(bad), 0.5, V.data_ptr(), 30, 2, Out.data_ptr(), 30,
                               work.data_ptr(), 20, None) == pc.PC_ERR_SHAPE
