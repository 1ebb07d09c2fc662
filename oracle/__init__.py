"""FP64 CPU oracle of the blaz method (arXiv 2202.13007) -- test infrastructure.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It wraps ``blaz_oracle.c`` (plain C, one block at a time,
direct sums) with numpy arrays through ctypes.  It shares no code with the HIP
library and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "blaz_oracle.c")
_LIB = os.path.join(_HERE, "libblaz_oracle.so")

NKEPT = 28
# Kept DCT positions (rows 0-1 and columns 0-1), row-major scan order.
KEPT = [(i, j) for i in range(8) for j in range(8) if i < 2 or j < 2]


def kept_count(lines: int) -> int:
    """Codes per block with L kept lines (rows and columns 0..L-1)."""
    return 16 * lines - lines * lines


def code_stride(lines: int) -> int:
    """Bytes per block of the codes array: the codes padded to whole 32-bit words."""
    return 4 * ((kept_count(lines) + 3) // 4)


def kept_positions(lines: int):
    return [(i, j) for i in range(8) for j in range(8) if i < lines or j < lines]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                        "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        sig = {
            "oracle_trace_size": ([], ctypes.c_size_t),
            "oracle_set_threads": ([ctypes.c_int], None),
            "oracle_max_threads": ([], ctypes.c_int),
            "oracle_compress_block": ([P, P], None),
            "oracle_compress_block_predicted": ([P, P], None),
            "oracle_predicted_slopes": ([P, D, P, P], None),
            "oracle_dct_of": ([P, P], None),
            "oracle_normalize": ([P, P], None),
            "oracle_idct": ([P, P], None),
            "oracle_inverse_normalize": ([D, D, P, P], None),
            "oracle_decompress_block": ([D, D, ctypes.c_int, P, P], None),
            "oracle_compress": ([P, I64, I64, I64, P, P, P, P, P, P, P], None),
            "oracle_compress_predicted": ([P, I64, I64, I64, P, P, P, P, P, P, P], None),
            "oracle_compress_blocks": ([P, I64, I64, P, I64, P, P, P, P, P, P, ctypes.c_int], None),
            "oracle_decompress": ([P, P, P, P, I64, I64, P, I64], None),
            "oracle_add": ([I64, P, P, P, P, P, P, P, P, P, P, P, P], None),
            "oracle_scale": ([I64, P, P, P, P, D, P, P, P, P], None),
            "oracle_dot": ([P, P, P, P, I64, P, P, P, P, I64, P, P, I64, P], None),
            "oracle_dot_dense": ([P, P, P, P, I64, P, P, I64, I64, P], None),
            "oracle_gemm": ([P, I64, P, I64, P, I64, I64, I64, I64], None),
            "oracle_kept_count": ([ctypes.c_int], ctypes.c_int),
            "oracle_compress_lines": ([P, I64, I64, I64, ctypes.c_int, I64, P, P, P, P, P, P], None),
            "oracle_decompress_lines": ([P, P, P, P, I64, I64, ctypes.c_int, I64, P, I64], None),
            "oracle_add_codes": ([I64, ctypes.c_int, I64, P, P, P, P, P, P, P, P, P, P, P, P], None),
            "oracle_scale_codes": ([I64, ctypes.c_int, I64, P, P, P, P, D, P, P, P, P], None),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the whole-matrix loops (blocks, product rows, queries are
    split between them; results do not depend on the count)."""
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class BlockTrace(ctypes.Structure):
    """Every intermediate of one block's compression (mirrors oracle_block_trace)."""
    _fields_ = [
        ("f", ctypes.c_double),
        ("delta", ctypes.c_double * 64),
        ("K", ctypes.c_int),
        ("s", ctypes.c_double),
        ("dprime", ctypes.c_double * 64),
        ("psi", ctypes.c_uint8 * 64),
        ("D", ctypes.c_double * 64),
        ("m", ctypes.c_double),
        ("phi_x", ctypes.c_double),
        ("phi", ctypes.c_int),
        ("code_x", ctypes.c_double * NKEPT),
        ("codes", ctypes.c_int8 * NKEPT),
    ]

    def arr(self, name, shape=(8, 8)):
        return np.array(getattr(self, name)).reshape(shape)


def compress_block(M, predicted: bool = False) -> BlockTrace:
    """All five stages on one 8x8 block; returns the full trace.  With
    ``predicted`` the transform takes the predicted slopes (reading B)."""
    L = lib()
    assert L.oracle_trace_size() == ctypes.sizeof(BlockTrace)
    M = np.ascontiguousarray(M, dtype=np.float64).reshape(64)
    tr = BlockTrace()
    fn = L.oracle_compress_block_predicted if predicted else L.oracle_compress_block
    fn(_p(M), ctypes.cast(ctypes.byref(tr), ctypes.c_void_p))
    return tr


def predicted_slopes(dprime, s, psi):
    """The grid points Eq. eqpredict selects, (s - s_max) + Psi * (2 s_max / 256)."""
    dprime = np.ascontiguousarray(dprime, dtype=np.float64).reshape(64)
    psi = np.ascontiguousarray(psi, dtype=np.uint8).reshape(64)
    sp = np.zeros(64)
    lib().oracle_predicted_slopes(_p(dprime), float(s), _p(psi), _p(sp))
    return sp.reshape(8, 8)


def dct_of(x):
    """Eq. eqdct of an 8x8 input, D_00 summed in the fixed pairwise order."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(64)
    D = np.zeros(64)
    lib().oracle_dct_of(_p(x), _p(D))
    return D.reshape(8, 8)


class Compressed:
    """Host-side compressed matrix: f, s, phi, codes (struct of arrays).
    lines = kept lines L (2: the paper's 28 codes); codes is [nblk][code_stride(L)]."""

    def __init__(self, rows, cols, f, s, phi, codes, lines=2):
        self.rows, self.cols = int(rows), int(cols)
        self.f, self.s, self.phi, self.codes = f, s, phi, codes
        self.lines = int(lines)

    @property
    def nblk(self):
        return (self.rows // 8) * (self.cols // 8)

    @staticmethod
    def empty(rows, cols, lines=2):
        nb = (rows // 8) * (cols // 8)
        return Compressed(rows, cols, np.zeros(nb), np.zeros(nb), np.zeros(nb, np.uint8),
                          np.zeros((nb, code_stride(lines)), np.int8), lines)

    def copy(self):
        return Compressed(self.rows, self.cols, self.f.copy(), self.s.copy(), self.phi.copy(),
                          self.codes.copy(), self.lines)


def compress(A, with_debug: bool = False, predicted: bool = False):
    """Compress a rows x cols FP64 matrix (multiples of 8).

    With ``with_debug`` also returns (psi[nblk,64], code_x[nblk,28], phi_x[nblk]):
    Psi and the values before truncation.  ``predicted`` selects reading B
    of the transform's input (the DCT of the predicted slopes)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    rows, cols = A.shape
    assert rows % 8 == 0 and cols % 8 == 0
    out = Compressed.empty(rows, cols)
    nb = out.nblk
    psi = code_x = phi_x = None
    if with_debug:
        psi = np.zeros((nb, 64), np.uint8)
        code_x = np.zeros((nb, NKEPT))
        phi_x = np.zeros(nb)
    fn = lib().oracle_compress_predicted if predicted else lib().oracle_compress
    fn(_p(A), rows, cols, cols, _p(out.f), _p(out.s), _p(out.phi), _p(out.codes), _p(psi), _p(code_x), _p(phi_x))
    if with_debug:
        return out, (psi, code_x, phi_x)
    return out


def compress_blocks(A, blocks, predicted: bool = False):
    """Compress only the listed flat block indices of A (sampled comparison).

    Returns (f, s, phi, codes, code_x, phi_x) for those blocks."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    rows, cols = A.shape
    blocks = np.ascontiguousarray(blocks, dtype=np.int64)
    n = len(blocks)
    f, s = np.zeros(n), np.zeros(n)
    phi = np.zeros(n, np.uint8)
    codes = np.zeros((n, NKEPT), np.int8)
    code_x = np.zeros((n, NKEPT))
    phi_x = np.zeros(n)
    lib().oracle_compress_blocks(_p(A), cols, cols, _p(blocks), n, _p(f), _p(s), _p(phi), _p(codes),
                                 _p(code_x), _p(phi_x), int(predicted))
    return f, s, phi, codes, code_x, phi_x


def compress_lines(A, lines: int, with_debug: bool = False):
    """Compression keeping L lines of DCT coefficients (the tunable rate);
    lines = 2 gives the paper's records.  With ``with_debug`` also returns
    (code_x[nblk, 16L - L^2], phi_x[nblk])."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    rows, cols = A.shape
    assert rows % 8 == 0 and cols % 8 == 0 and 1 <= lines <= 8
    out = Compressed.empty(rows, cols, lines)
    nb = out.nblk
    code_x = np.zeros((nb, kept_count(lines))) if with_debug else None
    phi_x = np.zeros(nb) if with_debug else None
    lib().oracle_compress_lines(_p(A), rows, cols, cols, lines, code_stride(lines), _p(out.f), _p(out.s),
                                _p(out.phi), _p(out.codes), _p(code_x), _p(phi_x))
    if with_debug:
        return out, (code_x, phi_x)
    return out


def decompress(c: Compressed):
    A = np.zeros((c.rows, c.cols))
    if c.lines == 2:
        lib().oracle_decompress(_p(c.f), _p(c.s), _p(c.phi), _p(c.codes), c.rows, c.cols, _p(A), c.cols)
    else:
        lib().oracle_decompress_lines(_p(c.f), _p(c.s), _p(c.phi), _p(c.codes), c.rows, c.cols, c.lines,
                                      code_stride(c.lines), _p(A), c.cols)
    return A


def decompress_block(f, s, phi, codes):
    B = np.zeros(64)
    codes = np.ascontiguousarray(codes, dtype=np.int8)
    lib().oracle_decompress_block(float(f), float(s), int(phi), _p(codes), _p(B))
    return B.reshape(8, 8)


def idct(D):
    D = np.ascontiguousarray(D, dtype=np.float64).reshape(64)
    P = np.zeros(64)
    lib().oracle_idct(_p(D), _p(P))
    return P.reshape(8, 8)


def inverse_normalize(f, s, P):
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(64)
    B = np.zeros(64)
    lib().oracle_inverse_normalize(float(f), float(s), _p(P), _p(B))
    return B.reshape(8, 8)


def add(x: Compressed, y: Compressed) -> Compressed:
    assert (x.rows, x.cols, x.lines) == (y.rows, y.cols, y.lines)
    z = Compressed.empty(x.rows, x.cols, x.lines)
    if x.lines == 2:
        lib().oracle_add(x.nblk, _p(x.f), _p(x.s), _p(x.phi), _p(x.codes), _p(y.f), _p(y.s), _p(y.phi),
                         _p(y.codes), _p(z.f), _p(z.s), _p(z.phi), _p(z.codes))
    else:
        lib().oracle_add_codes(x.nblk, kept_count(x.lines), code_stride(x.lines), _p(x.f), _p(x.s), _p(x.phi),
                               _p(x.codes), _p(y.f), _p(y.s), _p(y.phi), _p(y.codes), _p(z.f), _p(z.s),
                               _p(z.phi), _p(z.codes))
    return z


def scale(x: Compressed, c: float) -> Compressed:
    z = Compressed.empty(x.rows, x.cols, x.lines)
    if x.lines == 2:
        lib().oracle_scale(x.nblk, _p(x.f), _p(x.s), _p(x.phi), _p(x.codes), float(c), _p(z.f), _p(z.s),
                           _p(z.phi), _p(z.codes))
    else:
        lib().oracle_scale_codes(x.nblk, kept_count(x.lines), code_stride(x.lines), _p(x.f), _p(x.s),
                                 _p(x.phi), _p(x.codes), float(c), _p(z.f), _p(z.s), _p(z.phi), _p(z.codes))
    return z


def dot(x: Compressed, xrow, y: Compressed, ycol):
    """Line xrow[q] of X times column ycol[q] of Y, on decompressed values."""
    assert x.cols == y.rows
    xrow = np.ascontiguousarray(xrow, dtype=np.int64)
    ycol = np.ascontiguousarray(ycol, dtype=np.int64)
    out = np.zeros(len(xrow))
    lib().oracle_dot(_p(x.f), _p(x.s), _p(x.phi), _p(x.codes), x.cols, _p(y.f), _p(y.s), _p(y.phi),
                     _p(y.codes), y.cols, _p(xrow), _p(ycol), len(xrow), _p(out))
    return out


def dot_dense(x: Compressed, xrow, v, ldv):
    """Line xrow[q] of X times dense vector v[q*ldv : q*ldv + x.cols]."""
    xrow = np.ascontiguousarray(xrow, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(len(xrow))
    lib().oracle_dot_dense(_p(x.f), _p(x.s), _p(x.phi), _p(x.codes), x.cols, _p(xrow), _p(v), int(ldv),
                           len(xrow), _p(out))
    return out


def gemm(A, B):
    """Plain i-k-j product of dense FP64 matrices."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    C = np.zeros((m, n))
    lib().oracle_gemm(_p(A), k, _p(B), n, _p(C), n, m, n, k)
    return C


def matmul(x: Compressed, y=None, bdense=None):
    """Matrix product of compressed X with compressed Y or dense B: every block
    is decompressed once, then the plain product is taken."""
    xa = decompress(x)
    b = decompress(y) if y is not None else bdense
    return gemm(xa, b)
