#!/usr/bin/env python3
"""Benchmark: Z^+ x right-hand sides per second on one MI355X.

One step = the whole hot path on one batch: the Gram of the modulated square
root (per-column Grams + MFMA Gram), its FP64 Cholesky factorization, b = Z^T x
and the two triangular solves (plus FP64 refinement in the reduced-precision
modes), for the 64x128-grid workload (n = 8192, K = 32 members, M = 128 modes,
Z is 8192 x 4096, 256 right-hand sides).  The plan (validation and workspace
allocation) is built once before timing, like an FFT plan.

Prints one JSON line.  The oracle (explicit Z + Householder QR in float64) runs
on the host cores on the same arrays; it supplies the accuracy check and the
CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Z⁺x RHS/sec at rel.err≤1e-8 vs FP64 oracle; % HBM/MFMA roofline"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
HBM_PEAK_GBS = 8000.0
GRAM_SOURCES = ["paper_2609_13327_amd/csrc/k_gram.hip", "paper_2609_13327_amd/csrc/gemm_core.h",
                "paper_2609_13327_amd/csrc/pc_common.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 4])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the reduced-precision variants")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sources_sha():
    h = hashlib.sha256()
    for p in GRAM_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def gram_flops(inst):
    """Algorithmic FP64 Gram work: 2 n_h [K(K+1)/2] [M(M+1)/2] (both symmetries)."""
    return 2.0 * inst.n_h * (inst.K * (inst.K + 1) / 2) * (inst.M * (inst.M + 1) / 2)


def gram_flops_lowprec(inst):
    """Algorithmic work of the Gram of a rounded Z: n KM (KM+1) (one symmetry)."""
    return float(inst.n) * inst.KM * (inst.KM + 1)


def copy_probe():
    import torch
    n = 1 << 27  # 1 GiB of float64
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        log("bench.py: only --gpus 1 is supported (single-GPU build; see DESIGN.md for sharding)")
        return 2
    if args.copy_probe:
        copy_probe()
        return 0
    import torch
    import paper_2609_13327_amd as pc
    import workloads as wl

    pc.load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    log(f"generating config {args.config}")
    inst = wl.config(args.config)
    R = inst.R

    def to_dev(a):
        return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to(dev).t()

    dE, dW, dX = to_dev(inst.E), to_dev(inst.W), to_dev(inst.X)
    dY = torch.empty((R, inst.KM), dtype=torch.float64, device=dev).t()

    precs = {"fp64": (pc.PC_PREC_FP64, 0), "fp32": (pc.PC_PREC_FP32_REFINE, 10),
             "bf16": (pc.PC_PREC_BF16_REFINE, 30)}

    def measure(prec_name, steps, warmup, profile=True):
        code, refine = precs[prec_name]
        plan = pc.Plan([{"E": dE, "W": dW, "n_w": 1, "max_rhs": R}], precision=code,
                       max_refine=refine, tol=1e-10 if prec_name != "fp64" else 0.0)
        for _ in range(warmup):
            plan.factor()
            plan.apply([dX], [dY])
        torch.cuda.synchronize()
        pc.pc_profile_read(plan.handle)  # drop anything recorded so far
        if profile:
            pc.pc_profile_enable(plan.handle, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.factor()
            plan.apply([dX], [dY])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        phases = pc.pc_profile_read(plan.handle)
        pc.pc_profile_enable(plan.handle, False)
        # apply only (factor reused)
        plan.apply([dX], [dY])
        torch.cuda.synchronize()
        ta = time.perf_counter()
        napply = max(3, steps)
        for _ in range(napply):
            plan.apply([dX], [dY])
        torch.cuda.synchronize()
        tb = time.perf_counter()
        it, rel = pc.pc_query_info(plan.handle, 0)
        Y = dY.cpu().numpy()
        plan.close()
        ms = (t1 - t0) * 1e3 / steps
        return {"ms_per_step": ms, "rhs_per_s": R / (ms * 1e-3),
                "apply_only_rhs_per_s": R / ((tb - ta) / napply),
                "phases_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in phases.items()},
                "phase_counts": {k: v[1] for k, v in phases.items()},
                "refine_iters": it, "refine_last_rel": rel, "Y": Y}

    log(f"timing {args.precision}: {args.warmup} warmup + {args.steps} steps")
    main_res = measure(args.precision, args.steps, args.warmup)
    log(f"  {main_res['ms_per_step']:.3f} ms/step")

    # oracle on the host: accuracy reference and CPU baseline
    from oracle import lsq
    ref = None
    cpu = None
    if args.config in (1, 2) and not args.no_cpu_baseline:
        try:
            from threadpoolctl import threadpool_info
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count()])
        except Exception:
            threads = os.cpu_count()
        log("oracle (explicit Z + Householder QR) on the host")
        t0 = time.perf_counter()
        ref = lsq.left_inverse_apply(inst.E, inst.W, 1, inst.X)
        t_or = time.perf_counter() - t0
        log(f"  oracle {t_or:.2f} s")
        if True:
            cpu = {"value": R / t_or, "unit": "RHS/s", "cores": int(threads), "kind": "oracle",
                   "sample": f"the full {wl.CONFIG_NAMES[args.config]} step: form Z "
                             f"({inst.n}x{inst.KM}), LAPACK Householder QR, {R} right-hand sides"}

    def rel_err(Y):
        if ref is None:
            return None
        e = np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)
        return float(e.max()), float(np.median(e))

    err = rel_err(main_res["Y"])
    variants = {}
    if not args.no_variants:
        for name in ("bf16", "fp32", "fp64"):
            if name == args.precision:
                continue
            try:
                v = measure(name, max(3, args.steps // 4), 2)
                e = rel_err(v["Y"])
                variants[name] = {"ms_per_step": v["ms_per_step"], "rhs_per_s": v["rhs_per_s"],
                                  "apply_only_rhs_per_s": v["apply_only_rhs_per_s"],
                                  "refine_iters": v["refine_iters"],
                                  "rel_err_max": e[0] if e else None,
                                  "phases_ms": v["phases_ms"]}
            except Exception as ex:  # a variant that is not available is reported as such
                variants[name] = {"error": str(ex)}

    gram_ms = main_res["phases_ms"]["gram"]
    if args.precision == "fp64":
        flops = gram_flops(inst)
        peak = PEAK_TFLOPS["fp64"]
    else:
        flops = gram_flops_lowprec(inst)
        peak = PEAK_TFLOPS[args.precision]
    achieved = flops / (gram_ms * 1e-3) / 1e12 if gram_ms > 0 else None
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"gram_{args.precision}_c{args.config}_traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            t = json.load(f)
        if t.get("kernel_source_sha") == sources_sha():
            traffic = t.get("bytes_per_launch")
    out = {
        "metric": METRIC,
        "value": main_res["rhs_per_s"],
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": wl.CONFIG_NAMES[args.config], "n": inst.n, "K": inst.K, "M": inst.M,
                   "rhs": R, "precision": args.precision, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "kernel": "gram", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": (achieved / peak) if achieved else None,
                     "traffic": traffic, "flops_per_launch": flops,
                     "avg_launch_ms": gram_ms},
        "cpu_baseline": cpu,
        "rel_err_max": err[0] if err else None,
        "rel_err_median": err[1] if err else None,
        "apply_only_rhs_per_s": main_res["apply_only_rhs_per_s"],
        "phases_ms": main_res["phases_ms"],
        "variants": variants,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
