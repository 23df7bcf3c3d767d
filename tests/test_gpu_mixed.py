"""Reduced-precision Gram (bf16 / fp32 on MFMA, fp32 accumulation) with FP64
Cholesky and FP64 refinement, against the oracle, through the C-ABI."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import lsq
from tests.gpu_util import dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu

PRECS = {"bf16": pc.PC_PREC_BF16_REFINE, "fp32": pc.PC_PREC_FP32_REFINE}
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
    """The assembled Gram equals the exact Gram of round(Z) (oracle, float64)
    up to fp32 accumulation: |G - Gt| <= 2 n u32 (|Zt|^T |Zt|)."""
    inst = _inst(shape)
    plan = pc.Plan([inst_dict(inst)], precision=PRECS[prec], max_refine=1)
    pc.pc_gram_assemble(plan.handle)
    G = dev(np.zeros((inst.KM, inst.KM)))
    pc.pc_gram_export(plan.handle, 0, G)
    got = np.tril(host(G))
    Z = lsq.form_z(inst.E, inst.W, inst.n_w)
    Zt = lsq.round_bf16(Z) if prec == "bf16" else lsq.round_fp32(Z)
    ref = np.tril(Zt.T @ Zt)
    assert np.array_equal(np.tril(lsq.gram_lowprec(inst.E, inst.W, inst.n_w, prec)), ref)
    u32 = 2.0 ** -24
    bound = np.tril(2 * inst.n * u32 * (np.abs(Zt).T @ np.abs(Zt))) + 1e-300
    assert np.all(np.abs(got - ref) <= bound), np.abs(got - ref).max()
    plan.close()


def _rel_err(got, ref):
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


@pytest.mark.parametrize("prec", sorted(PRECS))
@pytest.mark.parametrize("shape", SHAPES)
def test_mixed_left_inverse_matches_oracle(prec, shape):
    inst = _inst(shape)
    plan = pc.Plan([inst_dict(inst)], precision=PRECS[prec], max_refine=60, tol=1e-13)
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
    plan = pc.Plan([inst_dict(inst)], precision=PRECS[prec], max_refine=60, tol=1e-13)
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
    plan = pc.Plan([inst_dict(inst)], precision=pc.PC_PREC_FP32_REFINE, max_refine=5)
    st, failed = plan.factor(raise_on_error=False)
    assert st == pc.PC_ERR_NOT_SPD and failed == 0
    plan.close()
