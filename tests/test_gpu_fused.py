"""The fused factor-and-apply call: the same result as the two separate calls
(it runs the same kernels, the products Z^T x on a second stream while the
factorization runs), its error statuses, and the paths without the overlap."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from tests.gpu_util import dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu


def _inst(shape, seed=31):
    n_lat, n_lon, n_w, K, M, R = shape
    return wl.make_instance(n_lat, n_lon, K, M, R, 0.3, 0.5, seed, n_w=n_w)


@pytest.mark.parametrize("shape", [(16, 32, 1, 8, 32, 16), (12, 24, 2, 9, 31, 70), (3, 6, 1, 1, 1, 1),
                                   (20, 40, 1, 16, 40, 33)])
def test_factor_apply_equals_separate_calls(shape):
    inst = _inst(shape)
    plan = pc.Plan([inst_dict(inst)])
    X = dev(inst.X)
    Y_sep = empty(inst.KM, inst.R)
    plan.factor()
    plan.apply([X], [Y_sep])
    Y_fused = empty(inst.KM, inst.R)
    st, failed = plan.factor_apply([X], [Y_fused])
    assert st == pc.PC_OK and failed == -1
    assert np.array_equal(host(Y_sep), host(Y_fused))
    # a second fused call with fewer, different right-hand sides
    rng = np.random.Generator(np.random.PCG64(7))
    R2 = max(1, inst.R // 2)
    X2 = dev(rng.standard_normal((inst.n, R2)))
    Y2 = empty(inst.KM, R2)
    plan.factor_apply([X2], [Y2])
    Y2_sep = empty(inst.KM, R2)
    plan.apply([X2], [Y2_sep])
    assert np.array_equal(host(Y2), host(Y2_sep))
    plan.close()


def test_factor_apply_with_refinement_equals_separate_calls():
    inst = _inst((16, 32, 1, 8, 32, 16))
    for precision in (pc.PC_PREC_FP64, pc.PC_PREC_BF16_REFINE):
        plan = pc.Plan([inst_dict(inst)], precision=precision, max_refine=30, tol=1e-13)
        X = dev(inst.X)
        Y_sep = empty(inst.KM, inst.R)
        plan.factor()
        plan.apply([X], [Y_sep])
        it_sep = pc.pc_query_info(plan.handle, 0)[0]
        Y_fused = empty(inst.KM, inst.R)
        plan.factor_apply([X], [Y_fused])
        assert pc.pc_query_info(plan.handle, 0)[0] == it_sep
        assert np.array_equal(host(Y_sep), host(Y_fused))
        plan.close()


def test_factor_apply_rank_deficient_is_reported():
    inst = wl.make_instance(6, 12, 4, 9, 3, 0.3, 0.5, 5, centring="sample")
    plan = pc.Plan([inst_dict(inst)])
    Y = empty(inst.KM, inst.R)
    st, failed = plan.factor_apply([dev(inst.X)], [Y], raise_on_error=False)
    assert st == pc.PC_ERR_NOT_SPD and failed == 0
    assert plan.apply([dev(inst.X)], [Y], raise_on_error=False) == pc.PC_ERR_NOT_FACTORED
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
    as the separate calls."""
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
