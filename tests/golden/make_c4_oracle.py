#!/usr/bin/env python3
"""Stored oracle values for the 131072 x 32768 workload (256x512 grid, K = 64
members, M = 512 modes, 1024 right-hand sides).

Writes tests/golden/c4_oracle.npz: the least-squares solutions y = Z^+ x of 8
fixed columns of that workload's X, computed by the FP64 oracle only
(explicit Z, Householder QR in place, oracle.lsq.lstsq_qr_inplace), with the
estimated 2-norm condition number of Z (from R) and SHA-256 digests of the
generated E, W and X so that a test can tell whether its host generated the
same inputs.

Run from the repository root:  python tests/golden/make_c4_oracle.py
Needs about 42 GB of host memory (Z alone is 34.4 GB) and, on 8 cores, about
an hour.
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

COLUMNS = [0, 1, 127, 128, 511, 512, 1000, 1023]
OUT = os.path.join(ROOT, "tests", "golden", "c4_oracle.npz")


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    t0 = time.time()
    inst = wl.config(4)
    print(f"generated n={inst.n} KM={inst.KM} R={inst.R} in {time.time() - t0:.0f} s", flush=True)
    dig = {"E": digest(inst.E), "W": digest(inst.W), "X": digest(inst.X)}
    Xs = np.asfortranarray(inst.X[:, COLUMNS])
    E, W = inst.E, inst.W
    del inst
    t1 = time.time()
    Z = lsq.form_z_fortran(E, W, 1)
    print(f"Z formed ({Z.nbytes / 2**30:.1f} GiB) in {time.time() - t1:.0f} s", flush=True)
    t1 = time.time()

    def progress(done, total):
        print(f"  QR {done}/{total} columns, {time.time() - t1:.0f} s", flush=True)

    Y, info = lsq.lstsq_qr_inplace(Z, Xs, panel=512, progress=progress)
    t_qr = time.time() - t1
    rd = np.abs(info["rdiag"])
    print(f"QR + solve {t_qr:.0f} s; min|R_ii|/max|R_ii| = {rd.min() / rd.max():.3e}", flush=True)
    KM = Z.shape[1]
    kappa, smax, smin = lsq.triu_cond_estimate(Z[:KM, :KM], iters=60)
    print(f"kappa(Z) >= {kappa:.4e} (sigma_max {smax:.4e}, sigma_min {smin:.4e})", flush=True)
    np.savez(OUT, columns=np.array(COLUMNS), Y=Y, residual_norm=info["residual_norm"],
             kappa=kappa, sigma_max=smax, sigma_min=smin, rdiag_min=rd.min(), rdiag_max=rd.max(),
             digest_E=dig["E"], digest_W=dig["W"], digest_X=dig["X"], qr_seconds=t_qr)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
