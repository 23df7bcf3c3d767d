"""The allocation-free entry point pc_factor_apply_noalloc against the
plan-based pc_factor_apply it is a variant of (same kernels, workspace taken
from a fixed library array), through the C ABI: two calls in a row, the
second with a smaller instance and fewer right-hand sides, both within the
FP64 bound of each other and of the oracle.  Also the size limit and the
statuses that need no GPU computation."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import lsq
from tests.gpu_util import dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu


def _rel_err(got, ref):
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


def _plan_result(inst):
    plan = pc.Plan([inst_dict(inst)])
    Y = empty(inst.KM, inst.R)
    st, _ = plan.factor_apply([dev(inst.X)], [Y])
    assert st == pc.PC_OK
    out = host(Y)
    plan.close()
    return out


def test_noalloc_matches_plan_path_twice():
    big = wl.make_instance(24, 48, 16, 40, 70, 0.1, 0.3, seed=41)      # n 1152, KM 640 (ragged tiles), R 70, kappa 68
    small = wl.make_instance(12, 24, 8, 13, 9, 0.1, 0.3, seed=42)      # n 288, KM 104, R 9, kappa 9
    for inst in (big, small):
        print(f"noalloc: n={inst.n} KM={inst.KM} R={inst.R}", flush=True)
        E, W, X = dev(inst.E), dev(inst.W), dev(inst.X)
        Y = empty(inst.KM, inst.R)
        Y.fill_(np.nan)
        assert pc.pc_factor_apply_noalloc(E, W, X, Y) == pc.PC_OK
        got = host(Y)
        ref_plan = _plan_result(inst)
        ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
        assert np.all(np.isfinite(got))
        assert _rel_err(got, ref_plan).max() <= 1e-11
        assert _rel_err(got, ref).max() <= 1e-10


def test_noalloc_limits_and_statuses():
    inst = wl.make_instance(12, 24, 8, 13, 5, 0.1, 0.3, seed=43)
    E, W, X = dev(inst.E), dev(inst.W), dev(inst.X)
    Y = empty(inst.KM, inst.R)
    # K*M = 4096 on a 64x128 grid: the Gram and its factor alone exceed the workspace
    big = wl.make_instance(64, 128, 32, 128, 2, 0.05, 0.2, seed=44)
    Yb = empty(big.KM, 2)
    st = pc.pc_factor_apply_noalloc(dev(big.E), dev(big.W), dev(big.X), Yb, raise_on_error=False)
    assert st == pc.PC_ERR_WORKSPACE
    # rank deficiency: a member repeated
    E2 = inst.E.copy()
    E2[:, 1] = E2[:, 0]
    st = pc.pc_factor_apply_noalloc(dev(E2), W, X, Y, raise_on_error=False)
    assert st == pc.PC_ERR_NOT_SPD
    # a NaN in W
    W2 = inst.W.copy()
    W2[3, 2] = np.nan
    st = pc.pc_factor_apply_noalloc(E, dev(W2), X, Y, raise_on_error=False)
    assert st == pc.PC_ERR_NONFINITE
    # and the entry point still works after those failures
    assert pc.pc_factor_apply_noalloc(E, W, X, Y) == pc.PC_OK
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    assert _rel_err(host(Y), ref).max() <= 1e-10
