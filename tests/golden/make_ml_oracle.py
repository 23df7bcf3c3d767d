#!/usr/bin/env python3
"""Stored oracle values for the multi-level workload (64x128 grid, 8 levels,
K = 32 members, M = 128 modes; Z is 65536 x 4096; 256 right-hand sides).

Writes tests/golden/ml_oracle.npz: the least-squares solutions y = Z^+ x of 8
fixed columns of the workload's X by the FP64 oracle only (explicit Z,
LAPACK Householder QR, oracle.lsq.lstsq_qr), the residual norms, the
2-norm condition number of Z from the singular values of R, and SHA-256
digests of the generated E, W and X.

Run from the repository root:  python tests/golden/make_ml_oracle.py
(about a minute and 5 GB of host memory on 8 cores).
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl   # noqa: E402
from oracle import lsq   # noqa: E402

COLUMNS = [0, 1, 63, 64, 127, 128, 200, 255]
OUT = os.path.join(ROOT, "tests", "golden", "ml_oracle.npz")


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    t0 = time.time()
    inst = wl.multilevel_config()
    print(f"generated n={inst.n} (n_w={inst.n_w}) KM={inst.KM} R={inst.R} in {time.time() - t0:.0f} s", flush=True)
    dig = {"E": digest(inst.E), "W": digest(inst.W), "X": digest(inst.X)}
    Xs = np.asfortranarray(inst.X[:, COLUMNS])
    Z = lsq.form_z(inst.E, inst.W, inst.n_w)
    t1 = time.time()
    Y, info = lsq.lstsq_qr(Z, Xs)
    t_qr = time.time() - t1
    sv = np.linalg.svd(Z, compute_uv=False)      # as oracle.lsq.cond, keeping the extremes
    kappa, smax, smin = float(sv[0] / sv[-1]), float(sv[0]), float(sv[-1])
    print(f"QR + solve {t_qr:.0f} s; kappa(Z) = {kappa:.4e}", flush=True)
    np.savez(OUT, columns=np.array(COLUMNS), Y=Y, residual_norm=info["residual_norm"], kappa=kappa,
             sigma_max=smax, sigma_min=smin, digest_E=dig["E"], digest_W=dig["W"], digest_X=dig["X"],
             qr_seconds=t_qr)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
