"""Per-right-hand-side refinement through the C-ABI: every column of Y stops
on its own stop rule, and pc_query_rhs_info reports each column's outcome.

The properties that pin it: a zero right-hand side has y = 0 and stops after
its first update (max|delta| = 0); scaling a column by a power of two scales
every product of its refinement exactly, so its iteration count equals the
unscaled column's; a column solved alone follows the same iterations as in a
batch; the instance's iteration count is the largest per column; results
still match the oracle's QR least squares."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import lsq
from tests.gpu_util import dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu

PRECS = {"fp64": pc.PC_PREC_FP64, "fp32": pc.PC_PREC_FP32_REFINE, "bf16": pc.PC_PREC_BF16_REFINE}


def _problem(R, seed=61):
    inst = wl.make_instance(12, 24, 6, 20, R, 0.15, 0.5, seed)
    X = inst.X.copy()
    X[:, 0] = 0.0                 # zero right-hand side
    X[:, 2] = 1024.0 * X[:, 1]    # exact power-of-two scaling of column 1
    return inst, X


def _solve(inst, X, prec, max_refine=40, tol=1e-13):
    plan = pc.Plan([inst_dict(inst, max_rhs=max(X.shape[1], inst.R))], precision=PRECS[prec],
                   max_refine=max_refine, tol=tol, flags=pc.PC_FLAG_FIXED_PRECISION)
    plan.factor()
    Y = empty(inst.KM, X.shape[1])
    st = plan.apply([dev(X)], [Y], raise_on_error=False)
    info = pc.pc_query_rhs_info(plan.handle, 0, X.shape[1])
    it, _ = pc.pc_query_info(plan.handle, 0)
    plan.close()
    return st, host(Y), info, it


@pytest.mark.parametrize("prec", sorted(PRECS))
def test_each_column_stops_on_its_own(prec):
    inst, X = _problem(9)
    st, Y, info, it = _solve(inst, X, prec)
    assert st == pc.PC_OK, pc.pc_status_string(st)
    ref = lsq.left_inverse_apply(inst.E, inst.W, inst.n_w, X)
    print(prec, [i[0] for i in info], it)
    assert info[0] == (1, 1, 0.0)
    assert np.all(Y[:, 0] == 0.0)
    assert all(s == 1 for _, s, _ in info)
    assert info[1][0] == info[2][0]
    assert it == max(i[0] for i in info)
    err = np.linalg.norm(Y[:, 1:] - ref[:, 1:], axis=0) / np.linalg.norm(ref[:, 1:], axis=0)
    assert err.max() <= 1e-8, err.max()
    if prec != "fp64":
        # the zero column needs one update, the others more
        assert min(i[0] for i in info[1:]) > 1


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_column_alone_matches_batch(prec):
    inst, X = _problem(9)
    _, Y, info, _ = _solve(inst, X, prec)
    for r in (1, 5):
        _, Yr, info_r, _ = _solve(inst, X[:, r:r + 1], prec)
        assert info_r[0][0] == info[r][0]
        assert np.abs(Yr[:, 0] - Y[:, r]).max() <= 1e-13 * np.abs(Y[:, r]).max()


def test_budget_spent_and_argument_errors():
    inst, X = _problem(5)
    st, Y, info, it = _solve(inst, X, "bf16", max_refine=1)
    assert st == pc.PC_ERR_NO_CONVERGENCE
    assert info[0] == (1, 1, 0.0)                                  # the zero column converged
    assert all(i[0] == 1 and i[1] == 0 for i in info[1:])          # the others ran out of budget
    assert it == 1
    plan = pc.Plan([inst_dict(inst)], max_refine=2)
    plan.factor()
    with pytest.raises(pc.PcError) as e:                            # no apply yet
        pc.pc_query_rhs_info(plan.handle, 0, 1)
    assert e.value.status == pc.PC_ERR_INVALID_ARG
    Y = empty(inst.KM, 3)
    plan.apply([dev(X[:, :3])], [Y])
    assert len(pc.pc_query_rhs_info(plan.handle, 0, 3)) == 3
    with pytest.raises(pc.PcError) as e:                            # more than the last apply's R
        pc.pc_query_rhs_info(plan.handle, 0, 4)
    assert e.value.status == pc.PC_ERR_INVALID_ARG
    plan.close()
