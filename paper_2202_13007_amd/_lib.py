"""ctypes loader for libblaz.so (the C ABI declared in include/libblaz.h).

The library is built in-tree by ``paper_2202_13007_amd._build``.  Loading
fails loudly when it is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libblaz.so")

BLAZ_OK = 0
STATUS_NAMES = {
    0: "BLAZ_OK", -1: "BLAZ_ERR_NULL", -2: "BLAZ_ERR_SHAPE", -3: "BLAZ_ERR_MISMATCH",
    -4: "BLAZ_ERR_ALIGN", -5: "BLAZ_ERR_ARG", -6: "BLAZ_ERR_UNSUPPORTED",
    -7: "BLAZ_ERR_WORKSPACE", -8: "BLAZ_ERR_HIP", -9: "BLAZ_ERR_TOO_LARGE",
}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}

# Every symbol include/libblaz.h declares.
EXPORTS = (
    "blaz_block_count", "blaz_compressed_bytes", "blaz_code_stride", "blaz_compressed_bytes_lines", "blaz_compress", "blaz_compress_predicted",
    "blaz_decompress", "blaz_add",
    "blaz_sub", "blaz_scale", "blaz_dot", "blaz_dot_dense", "blaz_matmul_workspace_bytes",
    "blaz_matmul", "blaz_matmul_tiled", "blaz_matmul_static", "blaz_matmul_compressed_workspace_bytes", "blaz_matmul_compressed",
    "blaz_diagnose", "blaz_status_string", "blaz_batch_plan_bytes", "blaz_batch_plan", "blaz_batch_run",
    "blaz_batch_run_resident",
    "blaz_matmul_group_plan_bytes", "blaz_matmul_group_plan", "blaz_matmul_group_run",
)


class BlazMatrixC(ctypes.Structure):
    """Mirror of ``blaz_matrix``: shape, four device pointers, kept lines (0 = 2)."""
    _fields_ = [
        ("rows", ctypes.c_int64),
        ("cols", ctypes.c_int64),
        ("f", ctypes.c_void_p),
        ("s", ctypes.c_void_p),
        ("phi", ctypes.c_void_p),
        ("codes", ctypes.c_void_p),
        ("lines", ctypes.c_int64),
    ]


class BatchItemC(ctypes.Structure):
    """Mirror of ``blaz_batch_item``."""
    _fields_ = [
        ("op", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("x", BlazMatrixC),
        ("y", BlazMatrixC),
        ("z", BlazMatrixC),
        ("dense", ctypes.c_void_p),
        ("ld", ctypes.c_int64),
        ("c", ctypes.c_double),
        ("xrow", ctypes.c_void_p),
        ("ycol", ctypes.c_void_p),
        ("count", ctypes.c_int64),
        ("out", ctypes.c_void_p),
    ]


class BatchStateC(ctypes.Structure):
    """Mirror of ``blaz_batch_state``."""
    _fields_ = [
        ("n_plan", ctypes.c_int64),
        ("total_chunks", ctypes.c_int64),
        ("counter", ctypes.c_uint64),
        ("status", ctypes.c_int64),
    ]


class MatmulItemC(ctypes.Structure):
    """Mirror of ``blaz_matmul_item``."""
    _fields_ = [
        ("a", BlazMatrixC),
        ("b", BlazMatrixC),
        ("bdense", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("ldb", ctypes.c_int64),
        ("c", ctypes.c_void_p),
        ("ldc", ctypes.c_int64),
        ("tile", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class MatmulGroupInfoC(ctypes.Structure):
    """Mirror of ``blaz_matmul_group_info``."""
    _fields_ = [
        ("rebuild_jobs", ctypes.c_int64),
        ("rebuild_waves", ctypes.c_int64),
        ("items128", ctypes.c_int64),
        ("workgroups128", ctypes.c_int64),
        ("items64", ctypes.c_int64),
        ("workgroups64", ctypes.c_int64),
        ("plan_bytes", ctypes.c_size_t),
        ("workspace_bytes", ctypes.c_size_t),
    ]


OPS = {"compress": 0, "decompress": 1, "add": 2, "sub": 3, "scale": 4, "dot": 5, "dot_dense": 6}


class BlazError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)} ({_status_string(status)})")


_lib = None


def _status_string(status: int) -> str:
    try:
        return lib().blaz_status_string(status).decode()
    except Exception:  # pragma: no cover - only used while formatting an error
        return "?"


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libblaz.so not found at {LIB_PATH}: build it with "
                           "`python -m paper_2202_13007_amd._build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, D, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    M = ctypes.POINTER(BlazMatrixC)
    sig = {
        "blaz_block_count": ([I64, I64], I64),
        "blaz_compressed_bytes": ([I64, I64], ctypes.c_size_t),
        "blaz_code_stride": ([I64], I64),
        "blaz_compressed_bytes_lines": ([I64, I64, I64], ctypes.c_size_t),
        "blaz_compress": ([P, I64, M, I, P, P], I),
        "blaz_compress_predicted": ([P, I64, M, P, P], I),
        "blaz_decompress": ([M, P, I64, P], I),
        "blaz_add": ([M, M, M, P], I),
        "blaz_sub": ([M, M, M, P], I),
        "blaz_scale": ([M, D, M, P], I),
        "blaz_diagnose": ([M, P, P], I),
        "blaz_dot": ([M, P, M, P, I64, P, P], I),
        "blaz_dot_dense": ([M, P, P, I64, I64, P, P], I),
        "blaz_matmul_workspace_bytes": ([I64, I64, I64, I, I], ctypes.c_size_t),
        "blaz_matmul": ([M, M, P, I64, I64, P, I64, I, P, ctypes.c_size_t, P], I),
        "blaz_matmul_tiled": ([M, M, P, I64, I64, P, I64, I, P, ctypes.c_size_t, ctypes.c_int32, P], I),
        "blaz_matmul_static": ([M, M, P, I64, I64, P, I64, I, P], I),
        "blaz_matmul_compressed_workspace_bytes": ([I64, I64, I64, I, I], ctypes.c_size_t),
        "blaz_matmul_compressed": ([M, M, P, I64, I64, M, I, P, ctypes.c_size_t, ctypes.c_int32, P], I),
        "blaz_status_string": ([I], ctypes.c_char_p),
        "blaz_batch_plan_bytes": ([I64], ctypes.c_size_t),
        "blaz_batch_plan": ([P, I64, P, ctypes.c_size_t, P, P], I),
        "blaz_batch_run": ([P, I64, I64, P, I64, ctypes.c_int32, P], I),
        "blaz_batch_run_resident": ([P, I64, P, I64, ctypes.c_int32, P], I),
        "blaz_matmul_group_plan_bytes": ([I64], ctypes.c_size_t),
        "blaz_matmul_group_plan": ([P, I64, P, ctypes.c_size_t, P, ctypes.c_size_t, P], I),
        "blaz_matmul_group_run": ([P, P, P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(status: int, what: str) -> None:
    if status != BLAZ_OK:
        raise BlazError(status, what)
