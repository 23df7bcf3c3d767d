"""The multi-level workload at full size (64 x 128 grid, 8 levels, K = 32,
M = 128; Z is 65536 x 4096; 256 right-hand sides) in the launch
configuration the benchmark times (autotuned plan, factor and apply in one
call), against stored oracle values: the least-squares solutions of 8 fixed
right-hand sides by explicit Z and Householder QR
(tests/golden/make_ml_oracle.py), with kappa(Z) from the singular values of
Z.  Tolerance per right-hand side: max(floor, 20 u kappa (1 + kappa eta)),
floor 1e-10 for FP64 and 1e-8 for a reduced-precision Gram with FP64
refinement.  Sampled entries of Z^T x (the level sum of the multi-level
path) are checked against their defining sums."""
import hashlib
import os

import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from tests.gpu_util import dev, empty, host, inst_dict, sum_bound

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ml_oracle.npz")
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def ml():
    g = np.load(GOLD)
    inst = wl.multilevel_config()
    for name, a in (("E", inst.E), ("W", inst.W), ("X", inst.X)):
        if hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest() != str(g["digest_" + name]):
            pytest.fail(f"generated {name} differs from the inputs of the stored oracle values")
    return inst, g


def _tolerance(g, floor):
    y = g["Y"]
    kappa = float(g["kappa"])
    eta = g["residual_norm"] / (float(g["sigma_max"]) * np.linalg.norm(y, axis=0))
    return np.maximum(floor, 20 * U64 * kappa * (1 + kappa * eta))


@pytest.mark.parametrize("name,precision,refine", [("fp64", pc.PC_PREC_FP64, 0),
                                                   ("bf16", pc.PC_PREC_BF16_REFINE, 30),
                                                   ("fp32", pc.PC_PREC_FP32_REFINE, 30)])
def test_multilevel_against_oracle(ml, name, precision, refine):
    inst, g = ml
    assert inst.n_w == 8
    plan = pc.Plan([inst_dict(inst)], precision=precision, max_refine=refine, tol=1e-11 if refine else 0.0)
    pc.pc_autotune(plan.handle, None, False)
    Y = empty(inst.KM, inst.R)
    st, _ = plan.factor_apply([dev(inst.X)], [Y], raise_on_error=False)
    it, _ = pc.pc_query_info(plan.handle, 0)
    plan.close()
    assert st == pc.PC_OK
    got = host(Y)[:, g["columns"]]
    err = np.linalg.norm(got - g["Y"], axis=0) / np.linalg.norm(g["Y"], axis=0)
    tol = _tolerance(g, 1e-10 if precision == pc.PC_PREC_FP64 else 1e-8)
    print(f"{name}: kappa {float(g['kappa']):.3e}, refinement iterations {it}, max rel err {err.max():.3e}")
    assert np.all(err <= tol), (err, tol)


def test_multilevel_sampled_ztx_entries(ml):
    """b[(k, m), r] = sum_l sum_j E[l n_h + j, k] W[j, m] X[l n_h + j, r] at
    sampled (k, m, r), within the rounding bound of a float64 sum."""
    inst, _ = ml
    plan = pc.Plan([inst_dict(inst)])
    B = empty(inst.KM, inst.R)
    pc.pc_sqrt_transpose_apply(plan.handle, 0, dev(inst.X), B)
    b = host(B)
    plan.close()
    rng = np.random.default_rng(12)
    Wt = np.tile(inst.W, (inst.n_w, 1))
    for _ in range(24):
        k, m, r = int(rng.integers(inst.K)), int(rng.integers(inst.M)), int(rng.integers(inst.R))
        terms = inst.E[:, k] * Wt[:, m] * inst.X[:, r]
        ref = terms.sum()
        assert abs(b[k * inst.M + m, r] - ref) <= sum_bound(np.abs(terms).sum(), inst.n + 2), (k, m, r)
