"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds no arithmetic of the compression method: it only draws
matrices.  Both the CPU oracle and the GPU library are fed the same arrays.
"""
from .fields import smooth_field, uniform_matrix, WORKLOADS, workload_inputs  # noqa: F401
