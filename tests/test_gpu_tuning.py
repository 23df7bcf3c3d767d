"""Launch-shape autotuning through the C-ABI: every shape the tuner can pick
gives the oracle's answer, and the tuning cache round-trips."""
import itertools

import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from oracle import lsq
from tests.gpu_util import dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu


def _rel(got, ref):
    return (np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)).max()


@pytest.mark.parametrize("gram,ztx,chol", list(itertools.product([1, 2, 3, 4], [1, 2], [1, 2])))
def test_every_launch_shape_matches_oracle(gram, ztx, chol):
    inst = wl.make_instance(12, 24, 5, 24, 70, 0.2, 0.5, 21)
    plan = pc.Plan([inst_dict(inst)])
    pc.pc_set_tuning(plan.handle, 0, gram, ztx, chol)
    assert pc.pc_query_tuning(plan.handle, 0) == (gram, ztx, chol)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(inst.X)], [Y])
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    assert _rel(host(Y), ref) <= 1e-10
    plan.close()


def test_autotune_cache_round_trip(tmp_path):
    insts = wl.batched_config(count=5, scale=0.3)
    cache = str(tmp_path / "tune.txt")
    plan = pc.Plan([inst_dict(i) for i in insts])
    pc.pc_autotune(plan.handle, cache, use_cached=True)
    chosen = [pc.pc_query_tuning(plan.handle, k) for k in range(len(insts))]
    for g, z, c in chosen:
        assert g in (1, 2, 3, 4) and z in (1, 2) and c in (1, 2)
    assert len({c for _, _, c in chosen}) == 1            # one grid for the batched factorization
    plan.factor()
    Ys = [empty(i.KM, i.R) for i in insts]
    plan.apply([dev(i.X) for i in insts], Ys)
    for i, y in zip(insts, Ys):
        assert _rel(host(y), lsq.left_inverse_apply(i.E, i.W, 1, i.X)) <= 1e-10
    plan.close()
    lines = open(cache).read().split("\n")
    assert lines[0] == "pcsqrt-tune-v2"
    rows = [ln.split() for ln in lines[1:] if ln.strip()]
    assert len(rows) == len({(i.n_h, i.K, i.M, i.R) for i in insts})
    assert all(len(r) == 11 for r in rows)   # shape key, then gram, ztx, grid, block width, product tile
    plan2 = pc.Plan([inst_dict(i) for i in insts])
    pc.pc_autotune(plan2.handle, cache, use_cached=True)
    assert [pc.pc_query_tuning(plan2.handle, k) for k in range(len(insts))] == chosen
    plan2.close()


def test_set_tuning_rejects_bad_values():
    inst = wl.make_instance(6, 12, 2, 8, 4, 0.2, 0.5, 22)
    plan = pc.Plan([inst_dict(inst)])
    for bad in ((5, 1, 1), (-1, 1, 1), (1, 3, 1), (1, 1, 3)):
        with pytest.raises(pc.PcError) as e:
            pc.pc_set_tuning(plan.handle, 0, *bad)
        assert e.value.status == pc.PC_ERR_INVALID_ARG
    plan.close()


def test_gram_parts_agree():
    """The FP64 Gram in one to four contraction parts: the same Gram up to
    the rounding of the partial sums, and every part count reused after
    another."""
    inst = wl.make_instance(16, 32, 4, 20, 8, 0.2, 0.5, 23)
    plan = pc.Plan([inst_dict(inst)])
    grams = {}
    for parts in (4, 1, 3, 2, 4):
        pc.pc_set_tuning(plan.handle, 0, parts, 0, 0)
        pc.pc_gram_assemble(plan.handle)
        G = dev(np.zeros((inst.KM, inst.KM)))
        pc.pc_gram_export(plan.handle, 0, G)
        grams.setdefault(parts, []).append(np.tril(host(G)))
    ref = grams[1][0]
    scale = np.abs(ref).max()
    for parts, gs in grams.items():
        for G in gs:
            assert np.abs(G - ref).max() <= 1e-13 * scale * inst.n, parts
    assert np.array_equal(grams[4][0], grams[4][1])
    plan.close()


@pytest.mark.parametrize("block", [128, 192, -1])
def test_blocked_factorization_matches_oracle(block):
    """Block columns of 128 / 192 (with a narrower last block) and the plain
    tile DAG give the oracle's answer; K*M = 420 (7 tiles, ragged)."""
    inst = wl.make_instance(20, 40, 6, 70, 33, 0.15, 0.4, 23)
    plan = pc.Plan([inst_dict(inst)])
    pc.pc_set_tuning(plan.handle, 0, 0, 0, 0, block)
    assert pc.pc_query_tuning(plan.handle, 0, with_block=True)[3] == (block if block > 0 else 0)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(inst.X)], [Y])
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    assert _rel(host(Y), ref) <= 1e-10
    plan.close()


@pytest.mark.parametrize("tile", [1, 2])
def test_blocked_factorization_tile_shapes(tile):
    """Both tile shapes of the blocked factorization's products give the same
    answer as the oracle (block columns of 128 over K*M = 420: panel and
    trailing products with ragged edges)."""
    inst = wl.make_instance(20, 40, 6, 70, 33, 0.15, 0.4, 23)
    plan = pc.Plan([inst_dict(inst)])
    pc.pc_set_tuning(plan.handle, 0, 0, 0, 0, 128)
    pc.pc_set_tile_shape(plan.handle, 0, tile)
    assert pc.pc_query_tile_shape(plan.handle, 0) == tile
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(inst.X)], [Y])
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    assert _rel(host(Y), ref) <= 1e-10
    with pytest.raises(pc.PcError):
        pc.pc_set_tile_shape(plan.handle, 0, 3)
    plan.close()


@pytest.mark.parametrize("block,prec", [(128, "fp64"), (192, "fp64"), (128, "bf16")])
def test_blocked_solve_many_right_hand_sides(block, prec):
    """From four tiles of 64 right-hand sides on, a blocked factor is solved
    block column by block column (tile-DAG solves of the diagonal blocks,
    MFMA products for the rest).  R = 300 (ragged last tile, K*M = 420 with a
    narrower last block) against the oracle, and against the tile-DAG solve
    of the first 100 columns (one launch per pass) on the same factor; in
    BF16 the refinement's solves run the blocked path too."""
    inst = wl.make_instance(20, 40, 6, 70, 300, 0.15, 0.4, 29)
    kw = {} if prec == "fp64" else {"precision": pc.PC_PREC_BF16_REFINE, "max_refine": 30, "tol": 1e-13,
                                     "flags": pc.PC_FLAG_FIXED_PRECISION}
    plan = pc.Plan([inst_dict(inst)], **kw)
    pc.pc_set_tuning(plan.handle, 0, 0, 0, 0, block)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(inst.X)], [Y])
    Ys = empty(inst.KM, 100)
    plan.apply([dev(inst.X[:, :100])], [Ys])
    plan.close()
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    got = host(Y)
    assert _rel(got, ref) <= 1e-10
    assert _rel(got[:, :100], host(Ys)) <= 1e-12


def test_blocked_factorization_reports_rank_deficiency():
    inst = wl.make_instance(10, 20, 4, 40, 3, 0.3, 0.5, 5, centring="sample")
    plan = pc.Plan([inst_dict(inst)])
    pc.pc_set_tuning(plan.handle, 0, 0, 0, 0, 128)
    st, failed = plan.factor(raise_on_error=False)
    assert st == pc.PC_ERR_NOT_SPD and failed == 0
    plan.close()


def test_blocked_after_batch_plan_reuses_memory():
    """A blocked factorization's solves must not depend on what freed device
    memory held before the plan was built: here a batch plan (one instance
    without right-hand sides) is built and freed first, whose memory the
    blocked plan's counters then reuse."""
    batch = wl.batched_config(count=4, scale=0.3)
    bp = pc.Plan([inst_dict(i) for i in batch])
    bp.factor()
    Xs = [dev(i.X) for i in batch]
    Ys = [empty(i.KM, i.R) for i in batch]
    Xs[1] = None
    bp.apply(Xs, Ys)
    bp.close()
    inst = wl.make_instance(20, 40, 6, 70, 33, 0.15, 0.4, 23)
    plan = pc.Plan([inst_dict(inst)])
    pc.pc_set_tuning(plan.handle, 0, 0, 0, 0, 192)
    plan.factor()
    Y = empty(inst.KM, inst.R)
    plan.apply([dev(inst.X)], [Y])
    ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
    assert _rel(host(Y), ref) <= 1e-10
    plan.close()
