#!/usr/bin/env python3
"""Stored oracle values for the batch of 64 uneven instances (grids 32x64 to
96x192, K in {8, 16, 32, 64}, M in {32, ..., 256}, K*M <= n, 8-128
right-hand sides each).

Writes tests/golden/c3_oracle.npz: for every instance the least-squares
solutions y = Z^+ x of its first and last right-hand side, computed by the
FP64 oracle only (explicit Z, Householder QR: oracle.lsq.lstsq_qr_inplace),
the 2-norm condition number of Z (singular values for K*M <= 4096, else the
estimate from R), the relative residual eta = ||x - Z y|| / (sigma_max ||y||)
of each stored column, the oracle's rank test (numerically rank deficient when
min |R_ii| <= n u max |R_ii|, as oracle.lsq.lstsq_qr decides; such an
instance has no meaningful least-squares solution in FP64) and the SHA-256
digest of all generated inputs.

Run from the repository root:  python tests/golden/make_c3_oracle.py
(a few minutes on 8 cores, under 4 GB of memory).
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

OUT = os.path.join(ROOT, "tests", "golden", "c3_oracle.npz")


def main():
    t0 = time.time()
    insts = wl.batched_config()
    h = hashlib.sha256()
    for i in insts:
        for a in (i.E, i.W, i.X):
            h.update(np.ascontiguousarray(a).tobytes())
    print(f"generated 64 instances in {time.time() - t0:.0f} s", flush=True)
    cols, ys, kappa, smax, eta, rankdef, offs = [], [], [], [], [], [], [0]
    for k, inst in enumerate(insts):
        t1 = time.time()
        c = [0, inst.R - 1]
        Xs = np.asfortranarray(inst.X[:, c])
        Z = lsq.form_z_fortran(inst.E, inst.W, 1)
        if inst.KM <= 4096:
            s = np.linalg.svd(Z, compute_uv=False)
            kap, sm = s[0] / s[-1], s[0]
        Zq = Z if inst.KM > 4096 else np.asfortranarray(Z.copy())
        Y, info = lsq.lstsq_qr_inplace(Zq, Xs, panel=256)
        if inst.KM > 4096:
            kap, sm, _ = lsq.triu_cond_estimate(Zq[:inst.KM, :inst.KM], iters=60)
        cols.append(c)
        ys.append(Y.T.reshape(-1))           # column 0 then column 1
        kappa.append(kap)
        smax.append(sm)
        eta.append(info["residual_norm"] / (sm * np.linalg.norm(Y, axis=0)))
        rd = np.abs(info["rdiag"])
        rankdef.append(bool(rd.min() <= inst.n * lsq.U64 * rd.max()))
        offs.append(offs[-1] + 2 * inst.KM)
        print(f"{k:2d} n={inst.n:5d} K={inst.K:2d} M={inst.M:3d} KM={inst.KM:5d} kappa={kap:.3e} "
              f"rank deficient={rankdef[-1]} {time.time() - t1:.1f} s", flush=True)
    np.savez(OUT, columns=np.array(cols), y=np.concatenate(ys), offsets=np.array(offs), kappa=np.array(kappa),
             sigma_max=np.array(smax), eta=np.array(eta), rank_deficient=np.array(rankdef), digest=h.hexdigest())
    print("wrote", OUT, f"in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
