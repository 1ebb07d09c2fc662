"""roctx ranges for rocprofv3's marker trace (``rocprofv3 --marker-trace``).

Ranges are pushed and popped on the calling host thread; they cost nothing
unless a tracer is enabled, and the library is loaded only when a range is
first opened.  The serving loop opens one per tick (``Server(trace=True)``).
"""
from __future__ import annotations

import ctypes

_ROCTX_NAMES = ("librocprofiler-sdk-roctx.so.1", "/opt/rocm/lib/librocprofiler-sdk-roctx.so.1")
_lib = None


def _roctx():
    global _lib
    if _lib is None:
        for name in _ROCTX_NAMES:
            try:
                lib = ctypes.CDLL(name)
                break
            except OSError:
                continue
        else:
            raise RuntimeError("tracing needs ROCm's roctx library (librocprofiler-sdk-roctx.so.1)")
        lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
        lib.roctxRangePushA.restype = ctypes.c_int
        lib.roctxRangePop.argtypes = []
        lib.roctxRangePop.restype = ctypes.c_int
        _lib = lib
    return _lib


class Range:
    """``with Range("name"):`` -- one roctx range around the block."""

    def __init__(self, name: str):
        self.name = name.encode()

    def __enter__(self):
        _roctx().roctxRangePushA(self.name)
        return self

    def __exit__(self, *exc):
        _roctx().roctxRangePop()
        return False
