"""Separable localization modes generated inside the kernels (pc_sqrt_build_separable):
W[a n_lon + i, m] = U[a, m] Phi[i, m] is never stored.  Every kernel that
reads a mode generates the same FP64 value as the dense W formed by that
product, so a separable plan must reproduce the dense plan's results bit
for bit (Gram, Z^T x, Z y, solves, refinement, reduced precision, batches),
and both match the oracle's least squares with the dense W."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import lsq
from tests.gpu_util import dev, empty, host

pytestmark = pytest.mark.gpu

SHAPES = [  # n_lat, n_lon, n_w, K, M, R
    (8, 16, 1, 4, 24, 5),
    (12, 24, 1, 6, 40, 70),
    (6, 10, 3, 5, 12, 9),      # several levels, n_h = 60 (not a multiple of 8)
    (16, 32, 2, 8, 64, 33),
]


def _problem(shape, seed=91):
    n_lat, n_lon, n_w, K, M, R = shape
    inst = wl.make_instance(n_lat, n_lon, K, M, R, 0.15, 0.5, seed, n_w=n_w)
    U, Phi, _ = wl.localization_factors(n_lat, n_lon, M, 0.5)
    return inst, U, Phi, lsq.separable_modes(U, Phi)


def _plans(inst, U, Phi, W, **kw):
    E = dev(inst.E)
    dense = pc.Plan([{"E": E, "W": dev(W), "n_w": inst.n_w, "max_rhs": inst.R}], **kw)
    sep = pc.Plan([{"E": E, "U": dev(U), "Phi": dev(Phi), "n_w": inst.n_w, "max_rhs": inst.R}], **kw)
    return dense, sep


@pytest.mark.parametrize("shape", SHAPES)
def test_separable_fp64_equals_dense_bitwise_and_oracle(shape):
    inst, U, Phi, W = _problem(shape)
    dense, sep = _plans(inst, U, Phi, W, max_refine=2)
    X = dev(inst.X)
    out = []
    for plan in (dense, sep):
        pc.pc_gram_assemble(plan.handle)
        G = dev(np.zeros((inst.KM, inst.KM)))
        pc.pc_gram_export(plan.handle, 0, G)
        B = empty(inst.KM, inst.R)
        pc.pc_sqrt_transpose_apply(plan.handle, 0, X, B)
        Xb = empty(inst.n, inst.R)
        pc.pc_sqrt_apply(plan.handle, 0, B, Xb)
        Y = empty(inst.KM, inst.R)
        plan.factor_apply([X], [Y])
        out.append([host(G), host(B), host(Xb), host(Y)])
    for a, b in zip(*out):
        assert np.array_equal(a, b)
    ref = lsq.left_inverse_apply(inst.E, W, inst.n_w, inst.X)
    err = np.linalg.norm(out[1][3] - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= 1e-10, err.max()
    dense.close()
    sep.close()


@pytest.mark.parametrize("prec", [pc.PC_PREC_BF16_REFINE, pc.PC_PREC_FP32_REFINE, pc.PC_PREC_BF16X3_REFINE])
def test_separable_reduced_precision_equals_dense(prec):
    inst, U, Phi, W = _problem((12, 24, 1, 6, 40, 20))
    dense, sep = _plans(inst, U, Phi, W, precision=prec, max_refine=30, tol=1e-13)
    Ys = []
    for plan in (dense, sep):
        Y = empty(inst.KM, inst.R)
        plan.factor_apply([dev(inst.X)], [Y])
        Ys.append(host(Y))
    assert np.array_equal(Ys[0], Ys[1])
    ref = lsq.left_inverse_apply(inst.E, W, 1, inst.X)
    assert (np.linalg.norm(Ys[1] - ref, axis=0) / np.linalg.norm(ref, axis=0)).max() <= 1e-8
    dense.close()
    sep.close()


def test_separable_batch_equals_dense_batch():
    shapes = [(8, 16, 1, 4, 24, 5), (10, 20, 1, 5, 32, 12), (6, 12, 1, 3, 16, 7)]
    probs = [_problem(sh, seed=100 + i) for i, sh in enumerate(shapes)]
    res = []
    for kind in ("W", "sep"):
        descs = []
        for inst, U, Phi, W in probs:
            d = {"E": dev(inst.E), "n_w": 1, "max_rhs": inst.R}
            if kind == "W":
                d["W"] = dev(W)
            else:
                d["U"], d["Phi"] = dev(U), dev(Phi)
            descs.append(d)
        plan = pc.Plan(descs, precision=pc.PC_PREC_FP32_REFINE, max_refine=20, tol=1e-12, use_graph=1)
        Ys = [empty(p[0].KM, p[0].R) for p in probs]
        plan.factor_apply([dev(p[0].X) for p in probs], Ys)
        res.append([host(y) for y in Ys])
        plan.close()
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_separable_argument_errors():
    import ctypes
    import torch
    inst, U, Phi, W = _problem((8, 16, 1, 4, 24, 5))
    E, Ud, Pd = dev(inst.E), dev(U), dev(Phi)
    lib = pc.load_library()
    opt = pc.PcOptions(0, 0, 0.0, 0, 0)

    def build(n_lat, n_lon, ldU, Pt):
        d = pc.PcInstanceSeparable(n_lat, n_lon, 1, 4, 24, E.data_ptr(), 128, Ud.data_ptr(), ldU,
                                   Pt.data_ptr(), 16, 5)
        plan = ctypes.c_void_p()
        st = lib.pc_sqrt_build_separable(ctypes.byref(d), 1, ctypes.byref(opt), None, ctypes.byref(plan))
        if plan.value:
            pc.pc_plan_destroy(plan.value)
        return st

    assert build(8, 16, 8, Pd) == pc.PC_OK
    assert build(8, 16, 7, Pd) == pc.PC_ERR_INVALID_ARG      # ldU < n_lat
    assert build(0, 16, 8, Pd) == pc.PC_ERR_SHAPE
    bad = Phi.copy()
    bad[3, 5] = np.nan
    assert build(8, 16, 8, dev(bad)) == pc.PC_ERR_NONFINITE
    torch.cuda.synchronize()
