"""Python binding of libpcsqrt (include/pcsqrt.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module turns
torch device tensors into pointers and leading dimensions and checks status
codes.  Matrices are column-major: a tensor of shape (rows, cols) must have
stride (1, ld) with ld >= rows (use `fortran()` to get one).

The functions keep the C names.  `Plan` is a small convenience owner that
keeps the borrowed E and W tensors alive for the plan's lifetime.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_void_p
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcsqrt.so")

PC_OK = 0
PC_ERR_INVALID_ARG = 1
PC_ERR_SHAPE = 2
PC_ERR_NONFINITE = 3
PC_ERR_NOT_SPD = 4
PC_ERR_NOT_FACTORED = 5
PC_ERR_NO_CONVERGENCE = 6
PC_ERR_OOM = 7
PC_ERR_DEVICE = 8
PC_ERR_TOO_MANY_RHS = 9
PC_ERR_WORKSPACE = 10

PC_PREC_FP64 = 0
PC_PREC_FP32_REFINE = 1
PC_PREC_BF16_REFINE = 2
PC_PREC_BF16X3_REFINE = 3

PC_FLAG_KEEP_GRAM = 1
PC_FLAG_CG_MEMBER_BLOCKS = 2
PC_FLAG_FIXED_PRECISION = 4
PC_FLAG_ZTX_FP32 = 8
PC_FLAG_ZTX_BF16 = 16
PC_MLP_BF16 = 0
PC_MLP_FP32 = 1

EXPORTED = [
    "pc_sqrt_build", "pc_gram_factor", "pc_left_inverse_apply", "pc_query_info",
    "pc_plan_destroy", "pc_status_string", "pc_sqrt_transpose_apply", "pc_sqrt_apply",
    "pc_gram_assemble", "pc_gram_export", "pc_profile_enable", "pc_profile_read",
    "pc_selftest_task_order", "pc_cg_solve", "pc_mlp_create", "pc_mlp_destroy", "pc_mlp_set_params",
    "pc_mlp_get_params", "pc_mlp_forward", "pc_mlp_gradients", "pc_mlp_train_step", "pc_mlp_warm_start",
    "pc_learned_apply", "pc_mlp_training_pairs", "pc_autotune", "pc_query_tuning",
    "pc_set_tuning", "pc_factor_apply", "pc_factor_apply_noalloc", "pc_query_instance", "pc_query_rhs_info", "pc_hybrid_apply",
    "pc_sqrt_build_separable", "pc_set_tile_shape", "pc_query_tile_shape",
    "pc_swift_build", "pc_swift_apply", "pc_swift_destroy", "pc_sqrt_transpose_apply_lowprec",
]

PHASES = ["column_grams", "gram", "pad", "cholesky", "ztx", "solve", "refine", "copyout", "solve_alongside"]


class PcInstance(ctypes.Structure):
    _fields_ = [("n_h", c_int64), ("n_w", c_int64), ("K", c_int64), ("M", c_int64),
                ("E", c_void_p), ("ldE", c_int64), ("W", c_void_p), ("ldW", c_int64),
                ("max_rhs", c_int64)]


class PcInstanceSeparable(ctypes.Structure):
    _fields_ = [("n_lat", c_int64), ("n_lon", c_int64), ("n_w", c_int64), ("K", c_int64), ("M", c_int64),
                ("E", c_void_p), ("ldE", c_int64), ("U", c_void_p), ("ldU", c_int64),
                ("Phi", c_void_p), ("ldPhi", c_int64), ("max_rhs", c_int64)]


class PcRhsInfo(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("state", c_int32), ("last_rel_update", c_double)]


class PcOptions(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("max_refine", c_int32), ("tol", c_double),
                ("use_graph", c_int32), ("flags", c_int32)]


class PcError(RuntimeError):
    def __init__(self, status: int, where: str = "", extra: str = ""):
        self.status = status
        msg = f"{where}: {status_string(status)} (status {status})"
        if extra:
            msg += f" {extra}"
        super().__init__(msg)


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run __graft_entry__.build() or paper_2609_13327_amd/build.py)")
    # PyTorch brings its own HIP runtime; importing it first makes the library
    # bind to that one, so that one runtime owns the device in this process
    # (a second runtime loaded before it cannot allocate device memory).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    lib.pc_sqrt_build.argtypes = [POINTER(PcInstance), c_int32, POINTER(PcOptions), c_void_p,
                                  POINTER(c_void_p)]
    lib.pc_sqrt_build_separable.argtypes = [POINTER(PcInstanceSeparable), c_int32, POINTER(PcOptions), c_void_p,
                                            POINTER(c_void_p)]
    lib.pc_gram_factor.argtypes = [c_void_p, c_void_p, POINTER(c_int32)]
    lib.pc_left_inverse_apply.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_int64),
                                          POINTER(c_int64), POINTER(c_void_p), POINTER(c_int64),
                                          c_void_p]
    lib.pc_factor_apply.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_int64), POINTER(c_int64),
                                    POINTER(c_void_p), POINTER(c_int64), c_void_p, POINTER(c_int32)]
    lib.pc_query_info.argtypes = [c_void_p, c_int32, POINTER(c_int32), POINTER(c_double)]
    lib.pc_plan_destroy.argtypes = [c_void_p]
    lib.pc_status_string.argtypes = [c_int32]
    lib.pc_status_string.restype = ctypes.c_char_p
    lib.pc_sqrt_transpose_apply.argtypes = [c_void_p, c_int32, c_void_p, c_int64, c_int64, c_void_p,
                                            c_int64, c_void_p]
    lib.pc_sqrt_apply.argtypes = [c_void_p, c_int32, c_void_p, c_int64, c_int64, c_void_p, c_int64,
                                  c_void_p]
    lib.pc_sqrt_transpose_apply_lowprec.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_int64, c_int64,
                                                    c_void_p, c_int64, c_void_p]
    lib.pc_gram_assemble.argtypes = [c_void_p, c_void_p]
    lib.pc_gram_export.argtypes = [c_void_p, c_int32, c_void_p, c_int64, c_void_p]
    lib.pc_profile_enable.argtypes = [c_void_p, c_int32]
    lib.pc_profile_read.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int64)]
    lib.pc_selftest_task_order.argtypes = [c_int32, c_int32]
    lib.pc_cg_solve.argtypes = [c_void_p, c_int32, c_void_p, c_int64, c_int64, c_void_p, c_int64, c_double,
                                c_int32, c_int32, POINTER(c_int32), c_void_p]
    lib.pc_mlp_create.argtypes = [c_int64, c_int64, c_int64, c_int32, POINTER(c_void_p)]
    lib.pc_mlp_destroy.argtypes = [c_void_p]
    lib.pc_mlp_set_params.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.pc_mlp_get_params.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.pc_mlp_forward.argtypes = [c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_int64, c_void_p]
    lib.pc_mlp_gradients.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_int64, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.pc_mlp_train_step.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_int64, ctypes.c_float,
                                      c_void_p, c_void_p]
    lib.pc_mlp_warm_start.argtypes = [c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_int64, c_void_p]
    lib.pc_mlp_training_pairs.argtypes = [c_void_p, c_int64, c_void_p, c_int64, c_int64, c_int64, c_void_p,
                                          c_int64, c_void_p, c_int64, c_void_p]
    lib.pc_autotune.argtypes = [c_void_p, ctypes.c_char_p, c_int32, c_void_p]
    lib.pc_set_tuning.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32]
    lib.pc_query_tuning.argtypes = [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                    POINTER(c_int32)]
    lib.pc_learned_apply.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_int64,
                                     c_double, c_int32, POINTER(c_int32), POINTER(c_int32), c_void_p]
    lib.pc_swift_build.argtypes = [c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                   c_int64, c_void_p, POINTER(c_void_p)]
    lib.pc_swift_apply.argtypes = [c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_int64, c_void_p]
    lib.pc_swift_destroy.argtypes = [c_void_p]
    lib.pc_query_instance.argtypes = [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32)]
    lib.pc_query_rhs_info.argtypes = [c_void_p, c_int32, c_int64, POINTER(PcRhsInfo)]
    lib.pc_set_tile_shape.argtypes = [c_void_p, c_int32, c_int32]
    lib.pc_query_tile_shape.argtypes = [c_void_p, c_int32, POINTER(c_int32)]
    lib.pc_hybrid_apply.argtypes = [POINTER(PcInstance), c_double, c_void_p, c_int64, c_int64, c_void_p,
                                    c_int64, c_void_p, c_int64, c_void_p]
    lib.pc_factor_apply_noalloc.argtypes = [POINTER(PcInstance), c_void_p, c_int64, c_int64, c_void_p, c_int64,
                                            c_void_p]
    for name in EXPORTED:
        if name != "pc_status_string":
            getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load_library().pc_status_string(int(status)).decode()


def _check(status: int, where: str, extra: str = ""):
    if status != PC_OK:
        raise PcError(status, where, extra)


# ------------------------------------------------------------ tensor helpers
def fortran(t):
    """Column-major copy (or view) of a 2-D tensor: stride (1, rows)."""
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    if t.stride(0) == 1 and t.stride(1) >= max(1, t.shape[0]):
        return t
    return t.t().contiguous().t()


def _ld(t) -> int:
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError("expected a column-major 2-D tensor (stride (1, ld)); use fortran()")
    return max(int(t.stride(1)), int(t.shape[0]), 1)


def _ptr(t) -> int:
    import torch
    if t.dtype != torch.float64 or not t.is_cuda:
        raise ValueError("expected a float64 device tensor")
    return t.data_ptr()


def _fptr(t) -> int:
    import torch
    if t.dtype != torch.float32 or not t.is_cuda:
        raise ValueError("expected a float32 device tensor")
    return t.data_ptr()


def _rows(t) -> int:
    """Row stride of a row-major 2-D tensor (stride (ld, 1))."""
    if t.dim() != 2 or (t.stride(1) != 1 and t.shape[1] > 1):
        raise ValueError("expected a row-major 2-D tensor (stride (ld, 1))")
    return max(int(t.stride(0)), int(t.shape[1]), 1)


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


# -------------------------------------------------------- C-named functions
def pc_sqrt_build(instances: Sequence[dict], precision: int = PC_PREC_FP64, max_refine: int = 0,
                  tol: float = 0.0, use_graph: int = 0, stream=None, flags: int = 0) -> int:
    """instances: dicts with E (n x K), W (n_h x M) column-major float64 device
    tensors, n_w and max_rhs -- or, for separable modes, U (n_lat x M) and
    Phi (n_lon x M) in place of W (pc_sqrt_build_separable).  Returns the plan
    handle."""
    lib = load_library()
    opt = PcOptions(int(precision), int(max_refine), float(tol), int(use_graph), int(flags))
    if instances and "U" in instances[0]:
        sep = (PcInstanceSeparable * len(instances))()
        for i, d in enumerate(instances):
            E, U, Phi = d["E"], d["U"], d["Phi"]
            n_w = int(d.get("n_w", 1))
            n_lat, n_lon = int(U.shape[0]), int(Phi.shape[0])
            if E.shape[0] != n_lat * n_lon * n_w or U.shape[1] != Phi.shape[1]:
                raise ValueError("E must have n_lat * n_lon * n_w rows; U and Phi the same mode count")
            sep[i] = PcInstanceSeparable(n_lat, n_lon, n_w, int(E.shape[1]), int(U.shape[1]), _ptr(E), _ld(E),
                                         _ptr(U), _ld(U), _ptr(Phi), _ld(Phi), int(d.get("max_rhs", 1)))
        plan = c_void_p()
        _check(lib.pc_sqrt_build_separable(sep, len(instances), ctypes.byref(opt), c_void_p(_stream(stream)),
                                           ctypes.byref(plan)), "pc_sqrt_build_separable")
        return plan.value
    arr = (PcInstance * len(instances))()
    for i, d in enumerate(instances):
        E, W = d["E"], d["W"]
        n_w = int(d.get("n_w", 1))
        n_h = int(W.shape[0])
        arr[i] = PcInstance(n_h, n_w, int(E.shape[1]), int(W.shape[1]), _ptr(E), _ld(E), _ptr(W),
                            _ld(W), int(d.get("max_rhs", 1)))
        if E.shape[0] != n_h * n_w:
            raise ValueError("E must have n_h * n_w rows")
    plan = c_void_p()
    _check(lib.pc_sqrt_build(arr, len(instances), ctypes.byref(opt), c_void_p(_stream(stream)),
                             ctypes.byref(plan)), "pc_sqrt_build")
    return plan.value


def pc_gram_factor(plan: int, stream=None, raise_on_error: bool = True):
    """Returns (status, failed_instance)."""
    lib = load_library()
    failed = c_int32(-1)
    st = lib.pc_gram_factor(c_void_p(plan), c_void_p(_stream(stream)), ctypes.byref(failed))
    if raise_on_error:
        _check(st, "pc_gram_factor", f"(instance {failed.value})")
    return st, failed.value


def pc_gram_assemble(plan: int, stream=None):
    _check(load_library().pc_gram_assemble(c_void_p(plan), c_void_p(_stream(stream))),
           "pc_gram_assemble")


def _apply_args(X: Sequence, Y: Sequence):
    n = len(X)
    xp = (c_void_p * n)()
    ldx = (c_int64 * n)()
    rr = (c_int64 * n)()
    yp = (c_void_p * n)()
    ldy = (c_int64 * n)()
    for i in range(n):
        if X[i] is None:
            xp[i], ldx[i], rr[i], yp[i], ldy[i] = None, 1, 0, None, 1
            continue
        if X[i].shape[1] != Y[i].shape[1]:
            raise ValueError("X and Y must have the same number of columns")
        xp[i], ldx[i], rr[i] = _ptr(X[i]), _ld(X[i]), int(X[i].shape[1])
        yp[i], ldy[i] = _ptr(Y[i]), _ld(Y[i])
    return xp, ldx, rr, yp, ldy


def pc_factor_apply(plan: int, X: Sequence, Y: Sequence, stream=None, raise_on_error: bool = True):
    """Factor and apply in one call (Y[i] <- Z_i^+ X[i]); returns (status, failed_instance)."""
    lib = load_library()
    xp, ldx, rr, yp, ldy = _apply_args(X, Y)
    failed = c_int32(-1)
    st = lib.pc_factor_apply(c_void_p(plan), xp, ldx, rr, yp, ldy, c_void_p(_stream(stream)),
                             ctypes.byref(failed))
    if raise_on_error:
        _check(st, "pc_factor_apply", f"(instance {failed.value})")
    return st, failed.value


def pc_factor_apply_noalloc(E, W, X, Y, n_w: int = 1, stream=None, raise_on_error: bool = True) -> int:
    """Y <- Z^+ X for one instance in FP64 without any allocation (fixed
    library workspace, no plan).  E, W, X, Y: column-major float64 device
    tensors.  Returns the status."""
    lib = load_library()
    n_h = int(W.shape[0])
    if E.shape[0] != n_h * int(n_w):
        raise ValueError("E must have n_h * n_w rows")
    if X.shape[1] != Y.shape[1]:
        raise ValueError("X and Y must have the same number of columns")
    inst = PcInstance(n_h, int(n_w), int(E.shape[1]), int(W.shape[1]), _ptr(E), _ld(E), _ptr(W), _ld(W),
                      int(X.shape[1]))
    st = lib.pc_factor_apply_noalloc(ctypes.byref(inst), _ptr(X), _ld(X), int(X.shape[1]), _ptr(Y), _ld(Y),
                                     c_void_p(_stream(stream)))
    if raise_on_error:
        _check(st, "pc_factor_apply_noalloc")
    return st


def pc_hybrid_apply(E, W, beta_e: float, V, Out, work, n_w: int = 1, stream=None) -> None:
    """Out <- (1 - beta_e) V + beta_e (C~ o P~e) V with P~e = E E^T and the
    localization C~ given by its modes W (n_h x M).  E (n~ x K), W, V, Out
    (n~ x R) and work (K*M x R, overwritten): column-major float64 device
    tensors; Out may be V."""
    lib = load_library()
    n_h = int(W.shape[0])
    if E.shape[0] != n_h * int(n_w) or V.shape[0] != E.shape[0] or Out.shape[0] != E.shape[0]:
        raise ValueError("E, V and Out must have n_h * n_w rows")
    R = int(V.shape[1])
    if Out.shape[1] != R or work.shape[1] < R or work.shape[0] < E.shape[1] * W.shape[1]:
        raise ValueError("Out must be n~ x R and work at least K*M x R")
    inst = PcInstance(n_h, int(n_w), int(E.shape[1]), int(W.shape[1]), _ptr(E), _ld(E), _ptr(W), _ld(W), 0)
    _check(lib.pc_hybrid_apply(ctypes.byref(inst), float(beta_e), _ptr(V), _ld(V), R, _ptr(Out), _ld(Out),
                               _ptr(work), _ld(work), c_void_p(_stream(stream))), "pc_hybrid_apply")


def pc_left_inverse_apply(plan: int, X: Sequence, Y: Sequence, stream=None,
                          raise_on_error: bool = True) -> int:
    """Y[i] <- Z_i^+ X[i] for every instance (None entries skip an instance)."""
    lib = load_library()
    n = len(X)
    xp = (c_void_p * n)()
    ldx = (c_int64 * n)()
    rr = (c_int64 * n)()
    yp = (c_void_p * n)()
    ldy = (c_int64 * n)()
    for i in range(n):
        if X[i] is None:
            xp[i], ldx[i], rr[i], yp[i], ldy[i] = None, 1, 0, None, 1
            continue
        if X[i].shape[1] != Y[i].shape[1]:
            raise ValueError("X and Y must have the same number of columns")
        xp[i], ldx[i], rr[i] = _ptr(X[i]), _ld(X[i]), int(X[i].shape[1])
        yp[i], ldy[i] = _ptr(Y[i]), _ld(Y[i])
    st = lib.pc_left_inverse_apply(c_void_p(plan), xp, ldx, rr, yp, ldy, c_void_p(_stream(stream)))
    if raise_on_error:
        _check(st, "pc_left_inverse_apply")
    return st


def pc_query_info(plan: int, instance: int = 0):
    it = c_int32(0)
    rel = c_double(0.0)
    _check(load_library().pc_query_info(c_void_p(plan), int(instance), ctypes.byref(it),
                                        ctypes.byref(rel)), "pc_query_info")
    return it.value, rel.value


def pc_query_instance(plan: int, instance: int = 0):
    """(precision of the instance's current Gram after the precision ladder,
    whether its factorization succeeded)."""
    pr = c_int32(0)
    fa = c_int32(0)
    _check(load_library().pc_query_instance(c_void_p(plan), int(instance), ctypes.byref(pr), ctypes.byref(fa)),
           "pc_query_instance")
    return pr.value, bool(fa.value)


def pc_query_rhs_info(plan: int, instance: int, R: int):
    """Per-right-hand-side refinement outcome of the instance's last apply:
    a list of R (iterations, state, last relative update), state 0 budget
    spent, 1 converged, 2 stalled, 3 diverging."""
    out = (PcRhsInfo * max(int(R), 1))()
    _check(load_library().pc_query_rhs_info(c_void_p(plan), int(instance), int(R), out), "pc_query_rhs_info")
    return [(out[r].iterations, out[r].state, out[r].last_rel_update) for r in range(int(R))]


def pc_set_tile_shape(plan: int, instance: int, gemm_tile: int):
    _check(load_library().pc_set_tile_shape(c_void_p(plan), int(instance), int(gemm_tile)), "pc_set_tile_shape")


def pc_query_tile_shape(plan: int, instance: int = 0) -> int:
    t = c_int32(0)
    _check(load_library().pc_query_tile_shape(c_void_p(plan), int(instance), ctypes.byref(t)), "pc_query_tile_shape")
    return t.value


def pc_plan_destroy(plan: Optional[int]):
    _check(load_library().pc_plan_destroy(c_void_p(plan)), "pc_plan_destroy")


def pc_status_string(status: int) -> str:
    return status_string(status)


def pc_sqrt_transpose_apply(plan: int, instance: int, X, B, stream=None):
    _check(load_library().pc_sqrt_transpose_apply(c_void_p(plan), int(instance), _ptr(X), _ld(X),
                                                  int(X.shape[1]), _ptr(B), _ld(B),
                                                  c_void_p(_stream(stream))), "pc_sqrt_transpose_apply")


def pc_sqrt_transpose_apply_lowprec(plan: int, instance: int, precision: int, X, B, stream=None):
    _check(load_library().pc_sqrt_transpose_apply_lowprec(c_void_p(plan), int(instance), int(precision), _ptr(X),
                                                          _ld(X), int(X.shape[1]), _ptr(B), _ld(B),
                                                          c_void_p(_stream(stream))),
           "pc_sqrt_transpose_apply_lowprec")


def pc_sqrt_apply(plan: int, instance: int, Y, X, stream=None):
    _check(load_library().pc_sqrt_apply(c_void_p(plan), int(instance), _ptr(Y), _ld(Y),
                                        int(Y.shape[1]), _ptr(X), _ld(X), c_void_p(_stream(stream))),
           "pc_sqrt_apply")


def pc_gram_export(plan: int, instance: int, G, stream=None):
    _check(load_library().pc_gram_export(c_void_p(plan), int(instance), _ptr(G), _ld(G),
                                         c_void_p(_stream(stream))), "pc_gram_export")


def pc_selftest_task_order(T: int, group: int = 0) -> int:
    """0 when the Cholesky DAG task order for T tile rows, with update tasks
    of `group` columns (0: the default), is valid (host only)."""
    return int(load_library().pc_selftest_task_order(int(T), int(group)))


def pc_profile_enable(plan: int, on: bool = True):
    _check(load_library().pc_profile_enable(c_void_p(plan), int(bool(on))), "pc_profile_enable")


def pc_profile_read(plan: int):
    """{phase: (total_ms, count)} of the intervals recorded since the last read."""
    n = len(PHASES)
    tot = (c_double * n)()
    cnt = (c_int64 * n)()
    _check(load_library().pc_profile_read(c_void_p(plan), tot, cnt), "pc_profile_read")
    return {PHASES[i]: (tot[i], cnt[i]) for i in range(n)}


def pc_cg_solve(plan: int, instance: int, B, Y, tol: float, maxiter: int, warm: bool = False, stream=None,
                raise_on_error: bool = True):
    """CG on G y = b (B, Y column-major K*M x R).  Returns (status, iterations)."""
    it = c_int32(0)
    st = load_library().pc_cg_solve(c_void_p(plan), int(instance), _ptr(B), _ld(B), int(B.shape[1]), _ptr(Y),
                                    _ld(Y), float(tol), int(maxiter), int(bool(warm)), ctypes.byref(it),
                                    c_void_p(_stream(stream)))
    if raise_on_error and st not in (PC_OK, PC_ERR_NO_CONVERGENCE):
        _check(st, "pc_cg_solve")
    return st, it.value


def pc_learned_apply(plan: int, instance: int, mlp: Optional[int], X, Y, tol: float, maxiter: int,
                     stream=None):
    """Y = Z^+ X by CG from the network's warm start.  Returns (iterations, fallback)."""
    it = c_int32(0)
    fb = c_int32(0)
    _check(load_library().pc_learned_apply(c_void_p(plan), int(instance), c_void_p(mlp), _ptr(X), _ld(X),
                                           int(X.shape[1]), _ptr(Y), _ld(Y), float(tol), int(maxiter),
                                           ctypes.byref(it), ctypes.byref(fb), c_void_p(_stream(stream))),
           "pc_learned_apply")
    return it.value, fb.value


def pc_mlp_create(d: int, h: int, max_batch: int, operand_type: int = PC_MLP_BF16) -> int:
    m = c_void_p()
    _check(load_library().pc_mlp_create(int(d), int(h), int(max_batch), int(operand_type), ctypes.byref(m)),
           "pc_mlp_create")
    return m.value


def pc_mlp_destroy(mlp: Optional[int]):
    _check(load_library().pc_mlp_destroy(c_void_p(mlp)), "pc_mlp_destroy")


def pc_mlp_set_params(mlp: int, W1, b1, W2, b2, stream=None):
    """Row-major float32 device tensors: W1 (h, d), b1 (h,), W2 (d, h), b2 (d,)."""
    for t in (W1, b1, W2, b2):
        if not t.is_contiguous():
            raise ValueError("parameters must be contiguous")
    _check(load_library().pc_mlp_set_params(c_void_p(mlp), _fptr(W1), _fptr(b1), _fptr(W2), _fptr(b2),
                                            c_void_p(_stream(stream))), "pc_mlp_set_params")


def pc_mlp_get_params(mlp: int, W1, b1, W2, b2, stream=None):
    _check(load_library().pc_mlp_get_params(c_void_p(mlp), _fptr(W1), _fptr(b1), _fptr(W2), _fptr(b2),
                                            c_void_p(_stream(stream))), "pc_mlp_get_params")


def pc_mlp_forward(mlp: int, X, Y, stream=None):
    _check(load_library().pc_mlp_forward(c_void_p(mlp), _fptr(X), _rows(X), int(X.shape[0]), _fptr(Y), _rows(Y),
                                         c_void_p(_stream(stream))), "pc_mlp_forward")


def pc_mlp_gradients(mlp: int, X, T, loss, dW1, db1, dW2, db2, stream=None):
    """Any of loss, dW1 .. db2 may be None (not computed / not written)."""
    opt = lambda t: c_void_p(_fptr(t) if t is not None else None)
    _check(load_library().pc_mlp_gradients(c_void_p(mlp), _fptr(X), _rows(X), _fptr(T), _rows(T), int(X.shape[0]),
                                           opt(loss), opt(dW1), opt(db1), opt(dW2), opt(db2),
                                           c_void_p(_stream(stream))), "pc_mlp_gradients")


def pc_mlp_train_step(mlp: int, X, T, lr: float, loss=None, stream=None):
    _check(load_library().pc_mlp_train_step(c_void_p(mlp), _fptr(X), _rows(X), _fptr(T), _rows(T),
                                            int(X.shape[0]), ctypes.c_float(lr),
                                            c_void_p(_fptr(loss) if loss is not None else None),
                                            c_void_p(_stream(stream))), "pc_mlp_train_step")


def pc_mlp_warm_start(mlp: int, B, Y0, stream=None):
    _check(load_library().pc_mlp_warm_start(c_void_p(mlp), _ptr(B), _ld(B), int(B.shape[1]), _ptr(Y0), _ld(Y0),
                                            c_void_p(_stream(stream))), "pc_mlp_warm_start")


def pc_mlp_training_pairs(B, Y, X, T, stream=None):
    """B, Y: column-major float64 (d, N); X, T: row-major float32 (N, d)."""
    _check(load_library().pc_mlp_training_pairs(_ptr(B), _ld(B), _ptr(Y), _ld(Y), int(B.shape[0]), int(B.shape[1]),
                                                _fptr(X), _rows(X), _fptr(T), _rows(T), c_void_p(_stream(stream))),
           "pc_mlp_training_pairs")


def pc_autotune(plan: int, cache_path: Optional[str] = None, use_cached: bool = True, stream=None):
    path = cache_path.encode() if cache_path else None
    _check(load_library().pc_autotune(c_void_p(plan), path, int(bool(use_cached)), c_void_p(_stream(stream))),
           "pc_autotune")


def pc_set_tuning(plan: int, instance: int, gram_split: int, ztx_split: int, chol_per_cu: int,
                  chol_block: int = 0):
    _check(load_library().pc_set_tuning(c_void_p(plan), int(instance), int(gram_split), int(ztx_split),
                                        int(chol_per_cu), int(chol_block)), "pc_set_tuning")


def pc_query_tuning(plan: int, instance: int = 0, with_block: bool = False):
    """(gram_split, ztx_split, chol_per_cu[, chol_block]) of an instance (0 = heuristic)."""
    g, z, c, b = c_int32(0), c_int32(0), c_int32(0), c_int32(0)
    _check(load_library().pc_query_tuning(c_void_p(plan), int(instance), ctypes.byref(g), ctypes.byref(z),
                                          ctypes.byref(c), ctypes.byref(b)), "pc_query_tuning")
    return (g.value, z.value, c.value, b.value) if with_block else (g.value, z.value, c.value)


# -------------------------------------------------------------- convenience
def pc_swift_build(E, Vb, delta, max_rhs: int, stream=None) -> int:
    """The paper's left inverse for n_w = K.  E: column-major float64 device
    tensor (n_h*K, K); Vb: (n_h, L); delta: float64 device vector (L,)."""
    import torch
    n_h, L = int(Vb.shape[0]), int(Vb.shape[1])
    K = int(E.shape[1])
    if E.shape[0] != n_h * K:
        raise ValueError("E must have n_h * K rows (n_w = K)")
    if delta.dtype != torch.float64 or not delta.is_cuda or delta.numel() != L or not delta.is_contiguous():
        raise ValueError("delta: contiguous float64 device vector of L eigenvalues")
    h = c_void_p()
    _check(load_library().pc_swift_build(n_h, K, L, _ptr(E), _ld(E), _ptr(Vb), _ld(Vb), delta.data_ptr(),
                                         int(max_rhs), c_void_p(_stream(stream)), ctypes.byref(h)), "pc_swift_build")
    return h.value


def pc_swift_apply(handle: int, X, Y, stream=None):
    _check(load_library().pc_swift_apply(c_void_p(handle), _ptr(X), _ld(X), int(X.shape[1]), _ptr(Y), _ld(Y),
                                         c_void_p(_stream(stream))), "pc_swift_apply")


def pc_swift_destroy(handle: Optional[int]):
    _check(load_library().pc_swift_destroy(c_void_p(handle)), "pc_swift_destroy")


class Swift:
    """Owns a pc_swift handle and keeps its borrowed V_b tensor alive (E is
    only read at build time, V_b at every apply)."""

    def __init__(self, E, Vb, delta, max_rhs: int, stream=None):
        self._keep = (E, Vb, delta)
        self.handle = pc_swift_build(E, Vb, delta, max_rhs, stream)

    def apply(self, X, Y, stream=None):
        pc_swift_apply(self.handle, X, Y, stream)

    def close(self):
        if self.handle:
            pc_swift_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Owns a plan and keeps its borrowed E/W tensors alive."""

    def __init__(self, instances: Sequence[dict], precision: int = PC_PREC_FP64, max_refine: int = 0,
                 tol: float = 0.0, use_graph: int = 0, stream=None, flags: int = 0):
        self._keep = [tuple(d[k] for k in ("E", "W", "U", "Phi") if k in d) for d in instances]
        self.instances = list(instances)
        self.handle = pc_sqrt_build(instances, precision, max_refine, tol, use_graph, stream, flags)

    def factor(self, stream=None, raise_on_error: bool = True):
        return pc_gram_factor(self.handle, stream, raise_on_error)

    def apply(self, X: Sequence, Y: Sequence, stream=None, raise_on_error: bool = True):
        return pc_left_inverse_apply(self.handle, X, Y, stream, raise_on_error)

    def factor_apply(self, X: Sequence, Y: Sequence, stream=None, raise_on_error: bool = True):
        return pc_factor_apply(self.handle, X, Y, stream, raise_on_error)

    def close(self):
        if self.handle:
            pc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """Owns a warm-start network handle."""

    def __init__(self, d: int, h: int, max_batch: int, operand_type: int = PC_MLP_BF16):
        self.d, self.h = d, h
        self.handle = pc_mlp_create(d, h, max_batch, operand_type)

    def close(self):
        if self.handle:
            pc_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

