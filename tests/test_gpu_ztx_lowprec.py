"""Reduced-precision Z^T x (pc_sqrt_transpose_apply_lowprec and the plan
flags PC_FLAG_ZTX_FP32 / PC_FLAG_ZTX_BF16) against the oracle, through the
C ABI: element by element against the exact product of the oracle's rounded
operands (the rounded Z of the reduced-precision Grams and the rounded
right-hand sides) within the bound of fp32 accumulation; and mixed-precision
solves that start from it still meet the refinement's accuracy."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import lsq
from tests.gpu_util import dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu

FMTS = {"fp32": pc.PC_PREC_FP32_REFINE, "bf16": pc.PC_PREC_BF16_REFINE}
U32 = 2.0 ** -24
SHAPES = [  # n_lat, n_lon, n_w, K, M, R
    (16, 32, 1, 8, 32, 16),      # the 16 x 32 workload's shape
    (16, 32, 1, 5, 70, 67),      # ragged in members (4 per tile), modes and right-hand sides (64 per tile)
    (6, 10, 2, 3, 20, 10),       # two levels, n_h = 60 (rows wrap inside a 32-row chunk)
    (2, 3, 3, 2, 3, 5),          # n_h = 6 < 8, three levels
    (20, 41, 1, 9, 65, 130),     # n = 820: a ragged last chunk, three right-hand-side tiles
]


def _inst(shape, seed=61):
    n_lat, n_lon, n_w, K, M, R = shape
    return wl.make_instance(n_lat, n_lon, K, M, R, 0.15, 0.5, seed, n_w=n_w)


def _bound(Zt, Xt, n):
    """fp32 accumulation of n products (one rounding per product and per
    addition): gamma_{n+1}(u32) |Zt|^T |Xt|."""
    g = (n + 1) * U32
    return g / (1 - g) * (np.abs(Zt).T @ np.abs(Xt)) + 1e-300


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("shape", SHAPES)
def test_lowprec_ztx_matches_oracle(fmt, shape):
    inst = _inst(shape)
    plan = pc.Plan([inst_dict(inst)])
    B = empty(inst.KM, inst.R)
    B.fill_(np.nan)
    pc.pc_sqrt_transpose_apply_lowprec(plan.handle, 0, FMTS[fmt], dev(inst.X), B)
    got = host(B)
    ref = lsq.zt_apply_lowprec(inst.E, inst.W, inst.n_w, inst.X, fmt)
    Zt = lsq.lowprec_operands(inst.E, inst.W, inst.n_w, fmt)[0]
    Xt = lsq.round_rhs(inst.X, fmt)
    bound = _bound(Zt, Xt, inst.n)
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - ref) <= bound), (np.abs(got - ref) / bound).max()
    if fmt == "bf16":
        # the bf16 roundings are visible: far outside the accumulation bound of the FP64 product
        exact = lsq.zt_apply(inst.E, inst.W, inst.n_w, inst.X)
        assert (np.abs(got - exact) / bound).max() > 10
    plan.close()


@pytest.mark.parametrize("fmt", sorted(FMTS))
def test_lowprec_ztx_separable_modes_equal_dense(fmt):
    """Modes generated from separable factors give the same rounded operands,
    so the same bits as the dense modes they define."""
    n_lat, n_lon, K, M, R = 12, 24, 6, 40, 70
    inst = wl.make_instance(n_lat, n_lon, K, M, R, 0.15, 0.5, 91)
    U, Phi, _ = wl.localization_factors(n_lat, n_lon, M, 0.5)
    W = lsq.separable_modes(U, Phi)
    E, X = dev(inst.E), dev(inst.X)
    dense = pc.Plan([{"E": E, "W": dev(W), "n_w": 1, "max_rhs": R}])
    sep = pc.Plan([{"E": E, "U": dev(U), "Phi": dev(Phi), "n_w": 1, "max_rhs": R}])
    out = []
    for plan in (dense, sep):
        B = empty(inst.KM, R)
        pc.pc_sqrt_transpose_apply_lowprec(plan.handle, 0, FMTS[fmt], X, B)
        out.append(host(B))
        plan.close()
    assert np.array_equal(out[0], out[1])
    ref = lsq.zt_apply_lowprec(inst.E, W, 1, inst.X, fmt)
    Zt = lsq.lowprec_operands(inst.E, W, 1, fmt)[0]
    assert np.all(np.abs(out[0] - ref) <= _bound(Zt, lsq.round_rhs(inst.X, fmt), inst.n))


def test_lowprec_ztx_arguments():
    inst = _inst(SHAPES[0])
    plan = pc.Plan([inst_dict(inst)])
    B = empty(inst.KM, inst.R)
    X = dev(inst.X)
    for bad in (pc.PC_PREC_FP64, pc.PC_PREC_BF16X3_REFINE, 7):
        with pytest.raises(pc.PcError) as e:
            pc.pc_sqrt_transpose_apply_lowprec(plan.handle, 0, bad, X, B)
        assert e.value.status == pc.PC_ERR_INVALID_ARG
    with pytest.raises(pc.PcError) as e:
        pc.pc_sqrt_transpose_apply_lowprec(plan.handle, 1, pc.PC_PREC_FP32_REFINE, X, B)
    assert e.value.status == pc.PC_ERR_INVALID_ARG
    plan.close()
    with pytest.raises(pc.PcError) as e:
        pc.Plan([inst_dict(inst)], precision=pc.PC_PREC_BF16_REFINE, max_refine=5,
                flags=pc.PC_FLAG_ZTX_FP32 | pc.PC_FLAG_ZTX_BF16)
    assert e.value.status == pc.PC_ERR_INVALID_ARG


def _rel_err(got, ref):
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


@pytest.mark.parametrize("flag", ["ZTX_FP32", "ZTX_BF16"])
@pytest.mark.parametrize("prec", ["bf16", "bf16x3", "fp32"])
@pytest.mark.parametrize("fused", [False, True])
def test_mixed_solve_from_lowprec_ztx_matches_oracle(flag, prec, fused):
    """A reduced-precision plan whose first b = Z^T x is formed in reduced
    precision: the refined answer meets 1e-8 against the QR oracle, on the
    64 x 128 workload's shapes scaled to a 32 x 64 grid and on a ragged
    one; and its first b is exactly what pc_sqrt_transpose_apply_lowprec
    gives (no refinement)."""
    precs = {"bf16": pc.PC_PREC_BF16_REFINE, "bf16x3": pc.PC_PREC_BF16X3_REFINE, "fp32": pc.PC_PREC_FP32_REFINE}
    fl = getattr(pc, "PC_FLAG_" + flag) | pc.PC_FLAG_FIXED_PRECISION
    for shape in [(32, 64, 1, 16, 64, 40), (12, 24, 2, 9, 31, 70)]:
        inst = _inst(shape, seed=73)
        ref = lsq.left_inverse_apply(inst.E, inst.W, inst.n_w, inst.X)
        X = dev(inst.X)
        plan = pc.Plan([inst_dict(inst)], precision=precs[prec], max_refine=60, tol=1e-13, flags=fl)
        Y = empty(inst.KM, inst.R)
        if fused:
            plan.factor_apply([X], [Y])
        else:
            plan.factor()
            plan.apply([X], [Y])
        it, _ = pc.pc_query_info(plan.handle, 0)
        err = _rel_err(host(Y), ref)
        assert err.max() <= 1e-8, (shape, err.max(), it)
        plan.close()
    # no refinement: the result is the solve of the reduced-precision b with the plan's factor
    inst = _inst((16, 32, 1, 8, 32, 16), seed=73)
    X = dev(inst.X)
    fmt = pc.PC_PREC_FP32_REFINE if flag == "ZTX_FP32" else pc.PC_PREC_BF16_REFINE
    plan = pc.Plan([inst_dict(inst)], precision=precs[prec], max_refine=0, flags=fl)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([X], [Y])
    plain = pc.Plan([inst_dict(inst)], precision=precs[prec], max_refine=0, flags=pc.PC_FLAG_FIXED_PRECISION)
    plain.factor()
    Y2 = empty(inst.KM, inst.R)
    plain.apply([X], [Y2])
    B = empty(inst.KM, inst.R)
    pc.pc_sqrt_transpose_apply_lowprec(plan.handle, 0, fmt, X, B)
    Bf = empty(inst.KM, inst.R)
    pc.pc_sqrt_transpose_apply(plan.handle, 0, X, Bf)
    # G~ y = b~ and G~ y2 = b: the difference of the solutions is G~^{-1} (b~ - b)
    G = dev(np.zeros((inst.KM, inst.KM)))
    pc.pc_gram_export(plan.handle, 0, G)
    Lg = np.tril(host(G))
    d = np.linalg.solve(Lg.T, np.linalg.solve(Lg, host(B) - host(Bf)))
    got = host(Y) - host(Y2)
    assert np.linalg.norm(got - d) <= 1e-6 * np.linalg.norm(d) + 1e-10 * np.linalg.norm(host(Y2))
    plan.close()
    plain.close()


# Launches large enough for each members-per-tile choice of the two Z^T x
# kernels (64 x 128 grid): (FP64 tile, reduced-precision tile) = (2, 1), (4, 2), (4, 4)
BIG = [(64, 128, 1, 24, 256, 512), (64, 128, 1, 24, 320, 640), (64, 128, 1, 32, 256, 1024)]


@pytest.mark.parametrize("shape", BIG)
def test_ztx_tile_choices_match_oracle(shape):
    inst = _inst(shape, seed=67)
    plan = pc.Plan([inst_dict(inst)])
    X = dev(inst.X)
    B = empty(inst.KM, inst.R)
    pc.pc_sqrt_transpose_apply(plan.handle, 0, X, B)
    Z = lsq.form_z(inst.E, inst.W, 1)
    absZ = np.abs(Z)
    g = (inst.n + 2) * 2.0 ** -53
    assert np.all(np.abs(host(B) - Z.T @ inst.X) <= 2 * g / (1 - g) * (absZ.T @ np.abs(inst.X)) + 1e-300)
    del Z, absZ
    for fmt in sorted(FMTS):
        pc.pc_sqrt_transpose_apply_lowprec(plan.handle, 0, FMTS[fmt], X, B)
        Zt = lsq.lowprec_operands(inst.E, inst.W, 1, fmt)[0]
        Xt = lsq.round_rhs(inst.X, fmt)
        ref = Zt.T @ Xt
        assert np.all(np.abs(host(B) - ref) <= _bound(Zt, Xt, inst.n)), fmt
        del Zt
    plan.close()
