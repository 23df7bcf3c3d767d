"""Parity of the FP64 HIP path with the oracle, through the C-ABI."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import lsq
from tests.gpu_util import dev, empty, host, inst_dict, sum_bound

pytestmark = pytest.mark.gpu

# (n_lat, n_lon, n_w, K, M, R): several tiles, ragged tails, n_w > 1, tiny cases
SHAPES = [
    (4, 8, 1, 3, 5, 3),
    (6, 12, 2, 4, 7, 5),
    (8, 16, 1, 8, 13, 17),
    (5, 10, 3, 5, 9, 2),
    (16, 32, 1, 8, 32, 16),
    (12, 24, 2, 9, 31, 70),
    (20, 40, 1, 16, 40, 33),
    (3, 6, 1, 1, 1, 1),
    (16, 32, 1, 64, 4, 3),     # 2080 member pairs: 16 full pair tiles and a tail of 32
]


def _inst(shape, seed=21):
    n_lat, n_lon, n_w, K, M, R = shape
    return wl.make_instance(n_lat, n_lon, K, M, R, 0.3, 0.5, seed, n_w=n_w)


def _plan(inst, **kw):
    return pc.Plan([inst_dict(inst)], **kw)


@pytest.mark.parametrize("shape", SHAPES)
def test_transpose_apply_matches_explicit(shape):
    inst = _inst(shape)
    plan = _plan(inst)
    X = dev(inst.X)
    B = empty(inst.KM, inst.R)
    pc.pc_sqrt_transpose_apply(plan.handle, 0, X, B)
    got = host(B)
    Z = lsq.form_z(inst.E, inst.W, inst.n_w)
    ref = Z.T @ inst.X
    # one FP64 dot product over the n rows of Z, each term (e w) x with e w rounded once
    bound = sum_bound(np.abs(Z).T @ np.abs(inst.X), inst.n + 2)
    assert np.all(np.abs(got - ref) <= bound), np.abs(got - ref).max()
    plan.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_sqrt_apply_matches_explicit(shape):
    inst = _inst(shape)
    plan = _plan(inst)
    Yin = np.random.default_rng(3).standard_normal((inst.KM, inst.R))
    Xo = empty(inst.n, inst.R)
    pc.pc_sqrt_apply(plan.handle, 0, dev(Yin), Xo)
    Z = lsq.form_z(inst.E, inst.W, inst.n_w)
    ref = Z @ Yin
    bound = sum_bound(np.abs(Z) @ np.abs(Yin), inst.KM + 1)
    assert np.all(np.abs(host(Xo) - ref) <= bound)
    plan.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_gram_matches_explicit(shape):
    inst = _inst(shape)
    plan = _plan(inst)
    pc.pc_gram_assemble(plan.handle)
    G = dev(np.zeros((inst.KM, inst.KM)))
    pc.pc_gram_export(plan.handle, 0, G)
    got = np.tril(host(G))
    Z = lsq.form_z(inst.E, inst.W, inst.n_w)
    ref = np.tril(Z.T @ Z)
    bound = np.tril(sum_bound(np.abs(Z).T @ np.abs(Z), inst.n_h + inst.n_w))
    assert np.all(np.abs(got - ref) <= bound), np.abs(got - ref).max()
    plan.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_factor_matches_cholesky(shape):
    inst = _inst(shape)
    plan = _plan(inst)
    plan.factor()
    L = dev(np.zeros((inst.KM, inst.KM)))
    pc.pc_gram_export(plan.handle, 0, L)
    got = np.tril(host(L))
    G = lsq.gram(inst.E, inst.W, inst.n_w)
    ref = lsq.cholesky(G)
    kappa = np.linalg.cond(G)
    assert np.abs(got - ref).max() <= 1e-13 * kappa * np.abs(ref).max()
    # and it is a factor of G to working accuracy
    assert np.abs(got @ got.T - G).max() <= 1e-13 * inst.KM * np.abs(G).max()
    plan.close()


def _rel_err(got, ref):
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


def _ls_tol(inst, X, Y):
    """Per right-hand side: max(1e-10, 20 u kappa (1 + kappa eta)), eta =
    ||x - Z y|| / (sigma_max ||y||) -- the first-order sensitivity of a
    least-squares solution (Wedin), which also bounds the oracle's own
    Householder-QR error.  For well-conditioned Z it is 1e-10."""
    Z = lsq.form_z(inst.E, inst.W, inst.n_w)
    s = np.linalg.svd(Z, compute_uv=False)
    kappa = s[0] / s[-1]
    eta = np.linalg.norm(X - Z @ Y, axis=0) / (s[0] * np.linalg.norm(Y, axis=0))
    return np.maximum(1e-10, 20 * 2.0 ** -53 * kappa * (1 + kappa * eta))


@pytest.mark.parametrize("shape", SHAPES)
def test_left_inverse_matches_oracle(shape):
    """Plain normal equations lose kappa(Z)^2 u; for ill-conditioned shapes
    (kappa(Z) > 1e4) the FP64 corrected semi-normal steps are switched on."""
    inst = _inst(shape)
    kappa = lsq.cond(inst.E, inst.W, inst.n_w)
    refine = 0 if kappa <= 1e4 else 40
    plan = _plan(inst, max_refine=refine, tol=1e-14)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(inst.X)], [Y])
    ref = lsq.left_inverse_apply(inst.E, inst.W, inst.n_w, inst.X)
    err = _rel_err(host(Y), ref)
    tol = _ls_tol(inst, inst.X, ref)
    assert np.all(err <= tol), (err.max(), kappa, tol.min())
    plan.close()


def test_fp64_refinement_recovers_ill_conditioned():
    """kappa(Z) ~ 3e7: the plain solve is off by ~1e-3, the corrected
    semi-normal iteration reaches the QR answer."""
    inst = _inst((20, 40, 1, 16, 40, 33))
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    errs = []
    for refine in (0, 40):
        plan = _plan(inst, max_refine=refine, tol=1e-14)
        plan.factor()
        Y = empty(inst.KM, inst.R)
        plan.apply([dev(inst.X)], [Y])
        errs.append(_rel_err(host(Y), ref).max())
        if refine:
            it, rel = pc.pc_query_info(plan.handle, 0)
            assert 1 <= it < 40 and rel <= 1e-8   # stops once the updates stall
        plan.close()
    tol = _ls_tol(inst, inst.X, ref).min()
    assert errs[0] > 1e-6 and errs[1] <= tol and errs[1] < 1e-3 * errs[0], (errs, tol)


def test_config1_range_projected_rhs():
    """16x32 grid, K=8, M=32, 16 right-hand sides projected on range(Z): the
    answer is exact and Z (Z^+ x) = x."""
    inst = wl.config(1)
    X = lsq.project_range(inst.E, inst.W, 1, inst.X)
    plan = _plan(inst)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(X)], [Y])
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, X)
    y = host(Y)
    assert _rel_err(y, ref).max() <= 1e-10
    Z = lsq.form_z(inst.E, inst.W, 1)
    assert np.abs(Z @ y - X).max() <= 1e-10 * np.abs(X).max()
    plan.close()


def test_config2_full_size():
    """64x128 grid, K=32, M=128 (Z is 8192 x 4096), 256 right-hand sides."""
    inst = wl.config(2)
    plan = _plan(inst)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(inst.X)], [Y])
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    err = _rel_err(host(Y), ref)
    print("config 2 max/median rel err", err.max(), np.median(err))
    assert err.max() <= 1e-10
    plan.close()


def test_rank_deficient_is_reported():
    inst = wl.make_instance(6, 12, 4, 9, 3, 0.3, 0.5, 5, centring="sample")
    plan = _plan(inst)
    st, failed = plan.factor(raise_on_error=False)
    assert st == pc.PC_ERR_NOT_SPD and failed == 0
    Y = empty(inst.KM, inst.R)
    assert plan.apply([dev(inst.X)], [Y], raise_on_error=False) == pc.PC_ERR_NOT_FACTORED
    plan.close()


def test_shape_and_argument_errors():
    inst = _inst((4, 8, 1, 3, 5, 3))
    d = inst_dict(inst)
    with pytest.raises(pc.PcError) as e:
        pc.Plan([{"E": d["E"], "W": dev(np.ones((32, 20))), "n_w": 1, "max_rhs": 2}])
    assert e.value.status == pc.PC_ERR_SHAPE
    bad = inst.E.copy()
    bad[3, 1] = np.nan
    with pytest.raises(pc.PcError) as e:
        pc.Plan([{"E": dev(bad), "W": d["W"], "n_w": 1, "max_rhs": 2}])
    assert e.value.status == pc.PC_ERR_NONFINITE
    plan = pc.Plan([d])
    plan.factor()
    X = dev(np.ones((inst.n, 4)))
    Y = empty(inst.KM, 4)
    assert plan.apply([X], [Y], raise_on_error=False) == pc.PC_ERR_TOO_MANY_RHS
    plan.close()


def test_deterministic_bitwise():
    inst = _inst((16, 32, 1, 8, 32, 16))
    outs = []
    for _ in range(2):
        plan = _plan(inst)
        plan.factor()
        Y = empty(inst.KM, inst.R)
        plan.apply([dev(inst.X)], [Y])
        outs.append(host(Y))
        plan.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("shape", [(16, 32, 1, 8, 32, 16), (20, 40, 1, 16, 40, 33)])
def test_refactor_after_operand_change(shape):
    """The FP64 plan borrows E and W: after they change in place, a new
    factorization uses the new values everywhere (no tile of the previous
    factor survives in any buffer or cache).  Each result is checked like a
    fresh plan's, with refinement for the ill-conditioned shape."""
    a = _inst(shape, seed=21)
    b = _inst(shape, seed=22)
    kappa = max(lsq.cond(a.E, a.W, a.n_w), lsq.cond(b.E, b.W, b.n_w))
    d = inst_dict(a)
    plan = pc.Plan([d], max_refine=0 if kappa <= 1e4 else 40, tol=1e-14)
    for inst in (a, b, a):
        d["E"].copy_(dev(inst.E))
        d["W"].copy_(dev(inst.W))
        plan.factor()
        Y = empty(inst.KM, inst.R)
        plan.apply([dev(inst.X)], [Y])
        ref = lsq.left_inverse_apply(inst.E, inst.W, inst.n_w, inst.X)
        err = _rel_err(host(Y), ref)
        assert np.all(err <= _ls_tol(inst, inst.X, ref)), err.max()
    plan.close()
