"""FP64 CPU oracle for the left inverse of the modulated ensemble square root.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's compute path may import,
call, link or execute anything in this package; it exists so that tests, the
smoke check and the benchmark's CPU baseline can judge the GPU results.  It
shares no code with the HIP path: it takes plain numpy arrays (produced by the
seeded generators in `workloads`) and computes, slowly and in float64, what the
paper defines.

Modules
  lsq     explicit square root Z (eq. SQRTofPCModulation), Householder QR least
          squares y = Z^+ x, and the reference sub-steps (Z^T x, Z y, Z^T Z,
          Cholesky, triangular solves, low-precision rounding of Z)
  swift   the paper's own left inverse for n_w = K (Sec. 3.9-3.10: per-column
          SVDs, eq. InverseSquareRootSwift and steps V1-V5)
  mlp     two-layer GELU network: forward, backward, relative-MSE loss, Adam
  cg      (block-Jacobi preconditioned) conjugate gradients on the normal equations
  hybrid  the Hybrid covariance model in standardized variables (Sec. 2.2), both
          of the paper's forms as explicit matrices

Parity status: every function here is pinned by tests in tests/test_oracle.py
against library routines, closed forms, invariants or brute force, except the
items marked "parity unpinned" in their docstrings.
"""
from . import lsq, swift, mlp, cg, hybrid  # noqa: F401
