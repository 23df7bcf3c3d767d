"""Edge cases through the C ABI: instances with no right-hand sides (alone,
inside a batch, in reduced precision with refinement, in the fused call and
in the reduced-precision Z^T x), and a square Z (K M = n, the largest K M
the method admits), where the least-squares solution is the exact inverse."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import lsq
from tests.gpu_util import dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu


def _rel(got, ref):
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


@pytest.mark.parametrize("prec", [pc.PC_PREC_FP64, pc.PC_PREC_BF16_REFINE])
@pytest.mark.parametrize("fused", [False, True])
def test_batch_with_an_instance_without_rhs(prec, fused):
    """Three instances, the middle one with zero right-hand sides: the other
    two match the oracle and the middle one's output is left untouched."""
    insts = [wl.make_instance(8, 16, 4, 12, 6, 0.15, 0.5, 71), wl.make_instance(6, 12, 3, 10, 5, 0.15, 0.5, 72),
             wl.make_instance(8, 16, 5, 9, 7, 0.15, 0.5, 73)]
    refine = 0 if prec == pc.PC_PREC_FP64 else 40
    plan = pc.Plan([inst_dict(i) for i in insts], precision=prec, max_refine=refine, tol=1e-13)
    X = [dev(i.X) for i in insts]
    X[1] = X[1][:, :0]
    Y = [empty(i.KM, i.R) for i in insts]
    Y[1].fill_(7.0)
    Yarg = list(Y)
    Yarg[1] = Y[1][:, :0]
    if fused:
        plan.factor_apply(X, Yarg)
    else:
        plan.factor()
        plan.apply(X, Yarg)
    assert np.all(host(Y[1]) == 7.0)
    for k in (0, 2):
        ref = lsq.left_inverse_apply(insts[k].E, insts[k].W, 1, insts[k].X)
        err = _rel(host(Y[k]), ref)
        assert err.max() <= (1e-10 if prec == pc.PC_PREC_FP64 else 1e-8), (k, err.max())
    plan.close()


def test_single_instance_without_rhs():
    inst = wl.make_instance(8, 16, 4, 12, 6, 0.15, 0.5, 74)
    plan = pc.Plan([inst_dict(inst)], precision=pc.PC_PREC_BF16_REFINE, max_refine=10)
    X0 = dev(inst.X)[:, :0]
    Y = empty(inst.KM, 1)
    Y.fill_(3.0)
    plan.factor_apply([X0], [Y[:, :0]])
    plan.apply([X0], [Y[:, :0]])
    pc.pc_sqrt_transpose_apply(plan.handle, 0, X0, Y[:, :0])
    pc.pc_sqrt_transpose_apply_lowprec(plan.handle, 0, pc.PC_PREC_FP32_REFINE, X0, Y[:, :0])
    assert np.all(host(Y) == 3.0)
    plan.close()


@pytest.mark.parametrize("shape,refine", [((8, 8, 4, 16, 0.2, 0.2, 5), 0), ((8, 16, 8, 16, 0.1, 0.15, 7), 10)])
def test_square_z_is_inverted(shape, refine):
    """K M = n: Z is square and invertible, Z^+ = Z^{-1}, so Z (Z^+ x) = x.
    The first case (kappa(Z) = 629) in plain normal equations, the second
    (kappa(Z) = 5.1e5) with corrected semi-normal steps; tolerance
    max(1e-10, 20 u kappa) (no residual: the system is consistent)."""
    n_lat, n_lon, K, M, l_e, l_l, seed = shape
    inst = wl.make_instance(n_lat, n_lon, K, M, 6, l_e, l_l, seed)
    assert inst.KM == inst.n
    kappa = lsq.cond(inst.E, inst.W, 1)
    Z = lsq.form_z(inst.E, inst.W, 1)
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    plan = pc.Plan([inst_dict(inst)], max_refine=refine, tol=1e-12)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(inst.X)], [Y])
    y = host(Y)
    err = _rel(y, ref)
    tol = max(1e-10, 20 * 2.0 ** -53 * kappa)
    print(f"square Z: kappa {kappa:.3e}, max rel err {err.max():.3e}, tolerance {tol:.1e}")
    assert err.max() <= tol
    # x is in range(Z): Z (Z^+ x) = x up to the normal equations' kappa^2 u
    assert np.linalg.norm(Z @ y - inst.X) <= 20 * 2.0 ** -53 * kappa ** 2 * np.linalg.norm(inst.X)
    plan.close()
