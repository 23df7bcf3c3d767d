"""Reduced-precision Gram (bf16, split bf16, fp32 on MFMA, fp32 accumulation;
the rounded Z formed inside the Gram kernel) with FP64 Cholesky and FP64
refinement, against the oracle, through the C-ABI; and the precision ladder
bf16 -> split bf16 -> fp32 -> FP64."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import lsq
from tests.gpu_util import dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu

PRECS = {"bf16": pc.PC_PREC_BF16_REFINE, "fp32": pc.PC_PREC_FP32_REFINE, "bf16x3": pc.PC_PREC_BF16X3_REFINE}
SHAPES = [
    (4, 8, 1, 3, 5, 3),
    (8, 16, 1, 8, 13, 17),
    (5, 10, 3, 5, 9, 2),
    (12, 24, 2, 9, 31, 70),
    (16, 32, 1, 8, 32, 16),
]


def _inst(shape, seed=31):
    n_lat, n_lon, n_w, K, M, R = shape
    return wl.make_instance(n_lat, n_lon, K, M, R, 0.15, 0.5, seed, n_w=n_w)


@pytest.mark.parametrize("prec", sorted(PRECS))
@pytest.mark.parametrize("shape", SHAPES)
def test_lowprec_gram_is_gram_of_rounded_z(prec, shape):
    """The assembled Gram equals the exact Gram of the oracle's rounded Z
    (bf16 of the fp32 product of fp32 copies of E and W, or fp32 of the FP64
    product; float64 Gram) up to the fp32 accumulation of the MFMAs:
    |G - Gt| <= 2 n u32 (|Zt|^T |Zt|); for split bf16, of its three
    products, with 3n terms per entry."""
    inst = _inst(shape)
    plan = pc.Plan([inst_dict(inst)], precision=PRECS[prec], max_refine=1, flags=pc.PC_FLAG_FIXED_PRECISION)
    pc.pc_gram_assemble(plan.handle)
    G = dev(np.zeros((inst.KM, inst.KM)))
    pc.pc_gram_export(plan.handle, 0, G)
    got = np.tril(host(G))
    ops = lsq.lowprec_operands(inst.E, inst.W, inst.n_w, prec)
    u32 = 2.0 ** -24
    if prec == "bf16x3":
        Hi, Lo = ops
        ref = np.tril(Hi.T @ Hi + Hi.T @ Lo + Lo.T @ Hi)
        absum = np.abs(Hi).T @ np.abs(Hi) + np.abs(Hi).T @ np.abs(Lo) + np.abs(Lo).T @ np.abs(Hi)
        bound = np.tril(2 * 3 * inst.n * u32 * absum) + 1e-300
    else:
        Zt = ops[0]
        ref = np.tril(Zt.T @ Zt)
        bound = np.tril(2 * inst.n * u32 * (np.abs(Zt).T @ np.abs(Zt))) + 1e-300
    assert np.array_equal(np.tril(lsq.gram_lowprec(inst.E, inst.W, inst.n_w, prec)), ref)
    assert np.all(np.abs(got - ref) <= bound), np.abs(got - ref).max()
    plan.close()


def _rel_err(got, ref):
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


@pytest.mark.parametrize("prec", sorted(PRECS))
@pytest.mark.parametrize("shape", SHAPES)
def test_mixed_left_inverse_matches_oracle(prec, shape):
    inst = _inst(shape)
    plan = pc.Plan([inst_dict(inst)], precision=PRECS[prec], max_refine=60, tol=1e-13,
                   flags=pc.PC_FLAG_FIXED_PRECISION)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(inst.X)], [Y])
    it, rel = pc.pc_query_info(plan.handle, 0)
    ref = lsq.left_inverse_apply(inst.E, inst.W, inst.n_w, inst.X)
    err = _rel_err(host(Y), ref)
    assert err.max() <= 1e-8, (err.max(), it, rel)
    assert it >= 1
    plan.close()


@pytest.mark.parametrize("prec", sorted(PRECS))
def test_mixed_config2_full_size(prec):
    """64x128 grid, K=32, M=128, 256 right-hand sides: <= 1e-8 per RHS."""
    inst = wl.config(2)
    plan = pc.Plan([inst_dict(inst)], precision=PRECS[prec], max_refine=60, tol=1e-13,
                   flags=pc.PC_FLAG_FIXED_PRECISION)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(inst.X)], [Y])
    it, rel = pc.pc_query_info(plan.handle, 0)
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    err = _rel_err(host(Y), ref)
    print(prec, "config 2: iterations", it, "max rel err", err.max())
    assert err.max() <= 1e-8
    plan.close()


def test_mixed_rank_deficient_is_reported():
    inst = wl.make_instance(6, 12, 4, 9, 3, 0.3, 0.5, 5, centring="sample")
    for flags in (pc.PC_FLAG_FIXED_PRECISION, 0):     # the ladder ends at FP64, which fails too
        plan = pc.Plan([inst_dict(inst)], precision=pc.PC_PREC_FP32_REFINE, max_refine=5, flags=flags)
        st, failed = plan.factor(raise_on_error=False)
        assert st == pc.PC_ERR_NOT_SPD and failed == 0
        if flags == 0:
            assert pc.pc_query_instance(plan.handle, 0)[0] == pc.PC_PREC_FP64
        plan.close()


def _ls_tol(inst, Y):
    """max(1e-8, 20 u kappa (1 + kappa eta)) per right-hand side: the
    first-order sensitivity of the least-squares solution."""
    Z = lsq.form_z(inst.E, inst.W, inst.n_w)
    s = np.linalg.svd(Z, compute_uv=False)
    kappa = s[0] / s[-1]
    eta = np.linalg.norm(inst.X - Z @ Y, axis=0) / (s[0] * np.linalg.norm(Y, axis=0))
    return np.maximum(1e-8, 20 * 2.0 ** -53 * kappa * (1 + kappa * eta)), kappa


@pytest.mark.parametrize("use_fused", [False, True])
def test_precision_ladder_climbs_until_converged(use_fused):
    """kappa(Z) ~ 9e3 on a 10x20 grid (K = 8, M = 22): bf16 refinement cannot
    converge (its contraction factor ~ kappa 2^-9 > 1), so with a fixed
    precision the apply reports no convergence, while the ladder moves the
    instance to split bf16 or fp32 and meets the least-squares bound."""
    inst = wl.make_instance(10, 20, 8, 22, 4, 0.3, 0.5, 51)
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    tol, kappa = _ls_tol(inst, ref)
    assert kappa > 5e3
    X = dev(inst.X)
    plan = pc.Plan([inst_dict(inst)], precision=pc.PC_PREC_BF16_REFINE, max_refine=30, tol=1e-13,
                   flags=pc.PC_FLAG_FIXED_PRECISION)
    Y = empty(inst.KM, inst.R)
    st, _ = plan.factor(raise_on_error=False)
    if st == pc.PC_OK:
        st = plan.apply([X], [Y], raise_on_error=False)
    assert st in (pc.PC_ERR_NO_CONVERGENCE, pc.PC_ERR_NOT_SPD)
    assert pc.pc_query_instance(plan.handle, 0)[0] == pc.PC_PREC_BF16_REFINE
    plan.close()
    plan = pc.Plan([inst_dict(inst)], precision=pc.PC_PREC_BF16_REFINE, max_refine=30, tol=1e-13)
    Y = empty(inst.KM, inst.R)
    if use_fused:
        st, _ = plan.factor_apply([X], [Y], raise_on_error=False)
    else:
        plan.factor()
        st = plan.apply([X], [Y], raise_on_error=False)
    assert st == pc.PC_OK
    rung = pc.pc_query_instance(plan.handle, 0)[0]
    assert rung in (pc.PC_PREC_BF16X3_REFINE, pc.PC_PREC_FP32_REFINE, pc.PC_PREC_FP64)
    err = _rel_err(host(Y), ref)
    print("ladder: kappa %.3g, rung %d, max rel err %.3g" % (kappa, rung, err.max()))
    assert np.all(err <= tol)
    # the plan keeps the raised precision: the next factor and apply start there
    plan.factor()
    Y2 = empty(inst.KM, inst.R)
    assert plan.apply([X], [Y2]) == pc.PC_OK
    assert pc.pc_query_instance(plan.handle, 0)[0] == rung
    assert np.all(_rel_err(host(Y2), ref) <= tol)
    plan.close()
