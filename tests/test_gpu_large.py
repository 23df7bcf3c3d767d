"""The large single instance (256 x 512 grid, n = 131072, K = 64, M = 512,
Z is 131072 x 32768, 1024 right-hand sides) at full size.  The oracle's QR
of Z is out of reach here, so the checks are properties that hold at any
size, on sampled outputs computed on the host from the factors E and W:
sampled Gram entries against their defining sums, and the least-squares
optimality of sampled solutions, ||Z^T (x - Z y)|| <= eps ||Z||_F^2 ||y||
(a relative error eps of y implies it, since Z^T (x - Z y) = G (y* - y))."""
import numpy as np
import pytest

import paper_2609_13327_amd as pc
import workloads as wl
from tests.gpu_util import dev, empty, host, inst_dict

pytestmark = pytest.mark.gpu

COLS = [0, 1, 511, 1023]


@pytest.fixture(scope="module")
def big():
    return wl.config(4)


def _zy(inst, Y):
    return sum(inst.E[:, [k]] * (inst.W @ Y[k * inst.M:(k + 1) * inst.M]) for k in range(inst.K))


def _ztr(inst, R):
    return np.concatenate([inst.W.T @ (inst.E[:, [k]] * R) for k in range(inst.K)])


def _optimality(inst, Y, cols):
    y = Y[:, cols]
    r = inst.X[:, cols] - _zy(inst, y)
    g = _ztr(inst, r)
    zf2 = float(np.sum((inst.E ** 2).sum(axis=1) * (inst.W ** 2).sum(axis=1)))
    return np.linalg.norm(g, axis=0) / (zf2 * np.linalg.norm(y, axis=0))


def test_large_instance_fp64_and_bf16(big):
    import torch
    inst = big
    d = inst_dict(inst)
    X = dev(inst.X)
    plan = pc.Plan([d])
    print("factor (FP64 Gram, blocked Cholesky)", flush=True)
    assert pc.pc_query_tuning(plan.handle, 0, with_block=True)[3] == 1024
    plan.factor()
    Y64 = empty(inst.KM, inst.R)
    plan.apply([X], [Y64])
    torch.cuda.synchronize()
    y64 = host(Y64)
    opt = _optimality(inst, y64, COLS)
    print("FP64 optimality", opt, flush=True)
    assert np.all(opt <= 1e-10)
    # sampled Gram entries against their defining sums, on a fresh assembly
    pc.pc_gram_assemble(plan.handle)
    G = torch.empty((inst.KM, inst.KM), dtype=torch.float64, device="cuda:0").t()
    pc.pc_gram_export(plan.handle, 0, G)
    rng = np.random.default_rng(4)
    for _ in range(6):
        a, b = sorted(rng.integers(0, inst.KM, 2))[::-1]
        ka, ma, kb, mb = a // inst.M, a % inst.M, b // inst.M, b % inst.M
        ref = float(np.dot(inst.E[:, ka] * inst.W[:, ma], inst.E[:, kb] * inst.W[:, mb]))
        got = float(G[a, b].item())
        scale = float(np.dot(np.abs(inst.E[:, ka] * inst.W[:, ma]), np.abs(inst.E[:, kb] * inst.W[:, mb])))
        assert abs(got - ref) <= 1e-12 * scale, (a, b, got, ref)
    del G
    plan.close()
    # BF16 Gram + FP64 refinement: agrees with the FP64 answer and is optimal
    planb = pc.Plan([d], precision=pc.PC_PREC_BF16_REFINE, max_refine=30, tol=1e-11)
    print("factor (BF16 Gram)", flush=True)
    planb.factor()
    Yb = empty(inst.KM, inst.R)
    planb.apply([X], [Yb])
    it, rel = pc.pc_query_info(planb.handle, 0)
    yb = host(Yb)
    planb.close()
    diff = np.linalg.norm(yb - y64, axis=0) / np.linalg.norm(y64, axis=0)
    print("BF16 refinement iterations", it, "max rel diff to FP64", diff.max(), flush=True)
    assert diff.max() <= 1e-8
    assert np.all(_optimality(inst, yb, COLS) <= 1e-10)
