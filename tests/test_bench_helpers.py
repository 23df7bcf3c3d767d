"""The benchmark's roofline arithmetic (no GPU): the algorithmic work per
launch of each phase against the per-unit figures of the method (both
symmetries of the FP64 Gram, one symmetry of a reduced-precision Gram, the
Cholesky and triangular-solve counts, Z^T x as per-column modulation plus
projection), evaluated at the 131072 x 32768 and 8192 x 4096 workloads; and
the pipeline roofline as the flop-weighted time at peak over the step."""
import types

import pytest

import bench


def _inst(n_h, n_w, K, M):
    return types.SimpleNamespace(n_h=n_h, n_w=n_w, n=n_h * n_w, K=K, M=M, KM=K * M)


def test_algorithmic_flops_largest_workload():
    c4 = _inst(131072, 1, 64, 512)
    # FP64 Gram: 2 n_h [K(K+1)/2] [M(M+1)/2] = 2 * 131072 * 2080 * 131328
    assert bench.algorithmic_flops("gram", "fp64", c4, 1024) == 2 * 131072 * 2080 * 131328
    assert abs(bench.algorithmic_flops("gram", "fp64", c4, 1024) / 7.16e13 - 1) < 1e-3
    # reduced precision: the Gram of one rounded Z, n KM (KM + 1); split bf16 three times that
    assert bench.algorithmic_flops("gram", "bf16", c4, 1024) == 131072 * 32768 * 32769
    assert bench.algorithmic_flops("gram", "bf16x3", c4, 1024) == 3 * 131072 * 32768 * 32769
    assert abs(bench.algorithmic_flops("gram", "fp32", c4, 1024) / 1.41e14 - 1) < 3e-3   # a 3-digit figure
    assert bench.algorithmic_flops("cholesky", "fp64", c4, 1024) == pytest.approx(32768 ** 3 / 3)
    assert abs(bench.algorithmic_flops("cholesky", "fp64", c4, 1024) / 1.17e13 - 1) < 3e-3
    # Z^T x: 2 n_h M K R + n K R
    assert bench.algorithmic_flops("ztx", "fp64", c4, 1024) == 2 * 131072 * 512 * 64 * 1024 + 131072 * 64 * 1024
    assert abs(bench.algorithmic_flops("ztx", "fp64", c4, 1024) / 8.8e12 - 1) < 1e-3
    # one triangular solve: (KM)^2 R
    assert bench.algorithmic_flops("solve", "fp64", c4, 1024) == 32768 ** 2 * 1024


def test_algorithmic_flops_levels_and_64x128():
    c2 = _inst(8192, 1, 32, 128)
    assert abs(bench.algorithmic_flops("gram", "fp64", c2, 256) / 7.1e10 - 1) < 1e-2
    assert abs(bench.algorithmic_flops("cholesky", "fp64", c2, 256) / 2.3e10 - 1) < 1e-2
    # several levels: the FP64 Gram's level sums come first (n_h, not n), the reduced-precision one contracts n rows
    ml = _inst(8192, 8, 32, 128)
    assert bench.algorithmic_flops("gram", "fp64", ml, 256) == bench.algorithmic_flops("gram", "fp64", c2, 256)
    assert bench.algorithmic_flops("gram", "bf16", ml, 256) == 8 * bench.algorithmic_flops("gram", "bf16", c2, 256)


def test_peaks_and_pipeline_roofline():
    assert bench.PEAK_TFLOPS == {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}
    assert bench.phase_peak("gram", "bf16") == 2500.0 and bench.phase_peak("cholesky", "bf16") == 78.6
    kern = {"gram": {"flops_per_launch": 78.6e12, "launches_per_step": 1.0, "peak_tflops": 78.6},
            "solve": {"flops_per_launch": 78.6e12 / 4, "launches_per_step": 2.0, "peak_tflops": 78.6}}
    pr = bench.pipeline_roofline(kern, 3000.0)
    assert pr["t_roof_ms"] == pytest.approx(1500.0)
    assert pr["frac"] == pytest.approx(0.5)
    assert pr["phases"] == ["gram", "solve"]
