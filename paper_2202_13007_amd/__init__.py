"""libblaz for MI355X: the blaz compressed-matrix method (arXiv 2202.13007) on gfx950.

The library itself is the C ABI in include/libblaz.h, implemented by the HIP
kernels under csrc/ and built into libblaz.so.  This package is its thin
Python binding (``api``) and the build script (``_build``).
"""
from .api import (DIAGNOSE_FIELDS, Batch, BatchPlan, BlazMatrix, MatmulGroup, MatmulGroupPlan, ResidentBatch, add, code_stride, compress,  # noqa: F401
                  compress_predicted, decompress,
                  diagnose, dot, dot_dense,
                  matmul, matmul_compressed, matmul_compressed_workspace_bytes, matmul_static,
                  matmul_workspace_bytes, scale,
                  sub)
from ._lib import BlazError, EXPORTS, LIB_PATH  # noqa: F401
