"""The fused factor-and-apply call: Z^T x on a second stream during the
factorization, and the forward pass of the solve behind it (its tasks wait
for the L blocks the running factorization publishes).  Its results meet
the same bounds against the oracle as the separate calls; error statuses
and the paths without the overlap are checked too."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import lsq
from tests.gpu_util import dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu

SHAPES = [(16, 32, 1, 8, 32, 16), (12, 24, 2, 9, 31, 70), (3, 6, 1, 1, 1, 1), (20, 40, 1, 16, 40, 33),
          (8, 16, 1, 8, 13, 17), (24, 48, 1, 16, 36, 130)]


def _inst(shape, seed=31):
    n_lat, n_lon, n_w, K, M, R = shape
    return wl.make_instance(n_lat, n_lon, K, M, R, 0.3, 0.5, seed, n_w=n_w)


def _rel_err(got, ref):
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


def _ls_tol(inst, X, Y):
    """max(1e-10, 20 u kappa (1 + kappa eta)) per right-hand side: the
    first-order sensitivity of the least-squares solution."""
    Z = lsq.form_z(inst.E, inst.W, inst.n_w)
    s = np.linalg.svd(Z, compute_uv=False)
    kappa = s[0] / s[-1]
    eta = np.linalg.norm(X - Z @ Y, axis=0) / (s[0] * np.linalg.norm(Y, axis=0))
    return np.maximum(1e-10, 20 * 2.0 ** -53 * kappa * (1 + kappa * eta))


@pytest.mark.parametrize("shape", SHAPES)
def test_factor_apply_matches_oracle(shape):
    inst = _inst(shape)
    kappa = lsq.cond(inst.E, inst.W, inst.n_w)
    plan = pc.Plan([inst_dict(inst)], max_refine=0 if kappa <= 1e4 else 40, tol=1e-14)
    ref = lsq.left_inverse_apply(inst.E, inst.W, inst.n_w, inst.X)
    tol = _ls_tol(inst, inst.X, ref)
    X = dev(inst.X)
    for _ in range(2):                      # twice: the second call reuses every buffer
        Y = empty(inst.KM, inst.R)
        st, failed = plan.factor_apply([X], [Y])
        assert st == pc.PC_OK and failed == -1
        err = _rel_err(host(Y), ref)
        assert np.all(err <= tol), (err.max(), kappa)
    # the plan is factored: a plain apply with other, fewer right-hand sides
    rng = np.random.Generator(np.random.PCG64(7))
    R2 = max(1, inst.R // 2)
    X2 = rng.standard_normal((inst.n, R2))
    Y2 = empty(inst.KM, R2)
    plan.apply([dev(X2)], [Y2])
    ref2 = lsq.left_inverse_apply(inst.E, inst.W, inst.n_w, X2)
    assert np.all(_rel_err(host(Y2), ref2) <= _ls_tol(inst, X2, ref2))
    # and a fused call with those
    Y3 = empty(inst.KM, R2)
    plan.factor_apply([dev(X2)], [Y3])
    assert np.all(_rel_err(host(Y3), ref2) <= _ls_tol(inst, X2, ref2))
    plan.close()


def test_factor_apply_reduced_precision_with_refinement():
    inst = _inst((16, 32, 1, 8, 32, 16))
    ref = lsq.left_inverse_apply(inst.E, inst.W, inst.n_w, inst.X)
    for precision in (pc.PC_PREC_FP32_REFINE, pc.PC_PREC_BF16_REFINE):
        plan = pc.Plan([inst_dict(inst)], precision=precision, max_refine=30, tol=1e-12)
        Y = empty(inst.KM, inst.R)
        st, _ = plan.factor_apply([dev(inst.X)], [Y])
        assert st == pc.PC_OK
        assert np.all(_rel_err(host(Y), ref) <= 1e-8)
        assert pc.pc_query_info(plan.handle, 0)[0] >= 1
        plan.close()


def test_factor_apply_rank_deficient_is_reported():
    inst = wl.make_instance(6, 12, 4, 9, 3, 0.3, 0.5, 5, centring="sample")
    plan = pc.Plan([inst_dict(inst)])
    Y = empty(inst.KM, inst.R)
    st, failed = plan.factor_apply([dev(inst.X)], [Y], raise_on_error=False)
    assert st == pc.PC_ERR_NOT_SPD and failed == 0
    assert plan.apply([dev(inst.X)], [Y], raise_on_error=False) == pc.PC_ERR_NOT_FACTORED
    # a good instance afterwards on a fresh plan still works (nothing left waiting)
    good = _inst((8, 16, 1, 4, 9, 5))
    plan2 = pc.Plan([inst_dict(good)])
    Y2 = empty(good.KM, good.R)
    assert plan2.factor_apply([dev(good.X)], [Y2])[0] == pc.PC_OK
    plan2.close()
    plan.close()


def test_factor_apply_argument_errors():
    inst = _inst((4, 8, 1, 3, 5, 3))
    plan = pc.Plan([inst_dict(inst)])
    X = dev(np.ones((inst.n, 4)))
    Y = empty(inst.KM, 4)
    st, _ = plan.factor_apply([X], [Y], raise_on_error=False)
    assert st == pc.PC_ERR_TOO_MANY_RHS
    plan.close()


def test_factor_apply_batch_without_overlap():
    """Several instances take the batched path (no overlap): the same result
    as the separate calls, bit for bit."""
    insts = [_inst((8, 16, 1, 4, 9, 5), seed=41), _inst((6, 12, 1, 3, 7, 4), seed=42)]
    plan = pc.Plan([inst_dict(i) for i in insts])
    Xs = [dev(i.X) for i in insts]
    Ys = [empty(i.KM, i.R) for i in insts]
    plan.factor()
    plan.apply(Xs, Ys)
    Yf = [empty(i.KM, i.R) for i in insts]
    st, failed = plan.factor_apply(Xs, Yf)
    assert st == pc.PC_OK and failed == -1
    for a, b in zip(Ys, Yf):
        assert np.array_equal(host(a), host(b))
    plan.close()
