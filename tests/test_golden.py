"""The stored oracle values (tests/golden/*.npz) against the generator and
against the definition of the least-squares solution, on the CPU:

* the generated inputs still hash to the digests the values were computed
  from (so the GPU tests compare against values of the same problem);
* every stored solution y satisfies the optimality condition of
  min ||Z y - x||, Z^T (x - Z y) = 0, up to rounding: the measure
  rho = ||Z^T r|| / (sigma_max (||r|| + sigma_max ||y||)) stays at the level
  of float64 rounding, and a relative error delta in y would raise it to
  at least delta / kappa(Z)^2.  Z is applied through its structure (column
  (k, m) = e_k o w_m, the modes repeated over the levels), independently of
  the Householder QR that produced the values;
* the stored residual norms equal ||x - Z y||.
"""
import hashlib
import os

import numpy as np
import pytest

import workloads as wl

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _z_apply(E, W, n_w, Y):
    """(Z Y)[l n_h + j] = sum_k E[l n_h + j, k] (W Y_k)[j], Y_k the rows k M .. k M + M - 1."""
    M = W.shape[1]
    out = np.zeros((E.shape[0], Y.shape[1]))
    for k in range(E.shape[1]):
        out += E[:, k:k + 1] * np.tile(W @ Y[k * M:(k + 1) * M], (n_w, 1))
    return out


def _zt_apply(E, W, n_w, R):
    """(Z^T R)[k M + m] = sum_l sum_j W[j, m] E[l n_h + j, k] R[l n_h + j]."""
    n_h, M = W.shape
    B = np.zeros((E.shape[1] * M, R.shape[1]))
    for k in range(E.shape[1]):
        B[k * M:(k + 1) * M] = W.T @ (E[:, k:k + 1] * R).reshape(n_w, n_h, -1).sum(axis=0)
    return B


def _optimality(E, W, n_w, X, Y, smax):
    R = X - _z_apply(E, W, n_w, Y)
    G = _zt_apply(E, W, n_w, R)
    rho = np.linalg.norm(G, axis=0) / (smax * (np.linalg.norm(R, axis=0) + smax * np.linalg.norm(Y, axis=0)))
    return rho, np.linalg.norm(R, axis=0)


@pytest.mark.parametrize("name", ["ml", "c4"])
def test_single_instance_values(name):
    g = np.load(os.path.join(GOLD, f"{name}_oracle.npz"))
    inst = wl.multilevel_config() if name == "ml" else wl.config(4)
    for key, a in (("E", inst.E), ("W", inst.W), ("X", inst.X)):
        assert _digest(a) == str(g["digest_" + key]), key
    X = inst.X[:, g["columns"]]
    rho, rn = _optimality(inst.E, inst.W, inst.n_w, X, g["Y"], float(g["sigma_max"]))
    assert rho.max() <= 2e-15, rho
    assert np.allclose(rn, g["residual_norm"], rtol=1e-10, atol=0)
    # the check has teeth: a stored solution off by 1e-6 (relative, in a random direction) fails it
    rng = np.random.default_rng(3)
    Yp = g["Y"] + 1e-6 * np.linalg.norm(g["Y"], axis=0) * rng.standard_normal(g["Y"].shape) / np.sqrt(inst.KM)
    rho_p, _ = _optimality(inst.E, inst.W, inst.n_w, X, Yp, float(g["sigma_max"]))
    assert rho_p.min() > 2e-15, rho_p
    assert float(g["sigma_max"]) / float(g["sigma_min"]) == pytest.approx(float(g["kappa"]), rel=1e-6)


def test_batch_values():
    """The 64-instance batch: one digest over every instance's E, W and X;
    optimality of the two stored right-hand sides of every instance the
    oracle did not find rank deficient, within rounding scaled by kappa(Z)
    for the ill-conditioned ones (their stored y is only as accurate as
    kappa(Z) u allows)."""
    g = np.load(os.path.join(GOLD, "c3_oracle.npz"))
    insts = wl.batched_config()
    h = hashlib.sha256()
    for i in insts:
        for a in (i.E, i.W, i.X):
            h.update(np.ascontiguousarray(a).tobytes())
    assert h.hexdigest() == str(g["digest"])
    offs = g["offsets"]
    checked = 0
    for k, inst in enumerate(insts):
        if g["rank_deficient"][k]:
            continue
        y = g["y"][offs[k]:offs[k + 1]].reshape(2, inst.KM).T
        X = inst.X[:, list(g["columns"][k])]
        rho, _ = _optimality(inst.E, inst.W, 1, X, y, float(g["sigma_max"][k]))
        assert rho.max() <= max(2e-15, 2e-16 * float(g["kappa"][k])), (k, rho.max(), float(g["kappa"][k]))
        checked += 1
    assert checked >= 56
