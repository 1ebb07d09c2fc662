"""Host-side checks of libblaz that need no GPU: the library loads, exports
every entry point include/libblaz.h declares, and rejects invalid arguments
before enqueuing anything (these calls never reach the HIP runtime; one
test, skipped where a GPU is present, checks that a launch the runtime
refuses comes back as BLAZ_ERR_HIP).
Also checks of the parity rules themselves."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libblaz.h")


@pytest.fixture(scope="module")
def L():
    from paper_2202_13007_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2202_13007_amd import _build
        _build.build()
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(blaz_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    from paper_2202_13007_amd import _lib
    names = declared_functions()
    assert len(names) >= 12
    assert sorted(_lib.EXPORTS) == names
    for n in names:
        assert hasattr(L, n), n


def test_no_other_symbols_exported(L):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", L._name], capture_output=True, text=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert {s for s in syms if s.startswith("blaz_")} == set(declared_functions())


def test_block_count_and_bytes(L):
    assert L.blaz_block_count(16, 24) == 6
    assert L.blaz_block_count(0, 8) == 0
    assert L.blaz_block_count(8, 12) == -2
    assert L.blaz_block_count(-8, 8) == -2
    assert L.blaz_compressed_bytes(16, 16) == 4 * 45
    assert L.blaz_compressed_bytes(8192, 8192) == 47185920
    assert L.blaz_compressed_bytes(7, 8) == 0


MAX_BLOCKS = (1 << 32) - 256  # blocks per matrix: every kernel's grid within 2^32 - 1 work-items
MAX_DOTS = MAX_BLOCKS // 32   # dot products per call: 32 work-items each


def test_shape_limits(L):
    """Shapes must be non-negative multiples of 8 with at most 2^32 - 256
    blocks: the one-lane-per-block kernels round the count up to 256-lane
    workgroups, and a dispatch holds at most 2^32 - 1 work-items."""
    rows, cols = 8 * 256, 8 * ((1 << 24) - 1)
    assert L.blaz_block_count(rows, cols) == MAX_BLOCKS              # exactly the limit
    assert L.blaz_block_count(rows + 8, cols) == -2                  # one block row more
    assert L.blaz_block_count(8 << 16, 8 << 16) == -2                # 2^32 blocks
    assert L.blaz_block_count(-8, 8) == -2 and L.blaz_block_count(12, 8) == -2
    assert L.blaz_compressed_bytes(rows, cols) == 45 * MAX_BLOCKS
    assert L.blaz_compressed_bytes(rows + 8, cols) == 0
    assert L.blaz_matmul_workspace_bytes(8, 8, 12, 0, 0) == 0
    x = mat(rows + 8, cols, 1 << 40)
    assert L.blaz_scale(B(x), 2.0, B(x), None) == -2                 # in place: refused, not launched


def test_dot_count_limit(L):
    """At most 2^27 - 8 dot products per call (eight per 256-lane workgroup).
    At the limit the count passes and the misaligned output is the first
    error; one more is refused as an invalid count."""
    x, y = mat(16, 16, 0x100000), mat(16, 16, 0x200000)
    assert MAX_DOTS == (1 << 27) - 8
    assert L.blaz_dot(B(x), 0x300000, B(y), 0x400000, MAX_DOTS, 0x500004, None) == -4
    assert L.blaz_dot(B(x), 0x300000, B(y), 0x400000, MAX_DOTS + 1, 0x500000, None) == -5
    assert L.blaz_dot_dense(B(x), 0x300000, 0x600000, 0, MAX_DOTS, 0x500004, None) == -4
    assert L.blaz_dot_dense(B(x), 0x300000, 0x600000, 0, MAX_DOTS + 1, 0x500000, None) == -5


def test_matmul_launch_limits(L):
    """A product whose launches would not fit one dispatch is refused as a
    shape error before anything is enqueued: the contraction's grid of
    output tiles, and the rebuild of both compressed operands in one grid."""
    # 2^19 x 2^19 output: 2^26 tiles of 64 x 64, 256 lanes each
    m = n = 1 << 19
    a, b = mat(m, 8, 1 << 40), mat(8, n, 1 << 42)
    need = L.blaz_matmul_workspace_bytes(m, n, 8, 1, 0)
    assert need > 0
    assert L.blaz_matmul_tiled(B(a), B(b), None, n, n, 1 << 44, n, 0, 1 << 46, need, 64, None) == -2
    # 128 tiles with 512 lanes (BF16x3): 2^12 x (2^12 - 1) tiles exceed 2^32 - 1 lanes
    m2, n2 = 128 << 12, 128 * ((1 << 12) - 1)
    a2, b2 = mat(m2, 8, 1 << 40), mat(8, n2, 1 << 42)
    need2 = L.blaz_matmul_workspace_bytes(m2, n2, 8, 1, 2)
    assert L.blaz_matmul_tiled(B(a2), B(b2), None, n2, n2, 1 << 44, n2, 2, 1 << 46, need2, 128, None) == -2
    # rebuilds: A with the largest block count plus B's blocks in one grid of 64-block waves
    k = 8 * ((1 << 24) - 1)
    a3, b3 = mat(8 * 256, k, 1 << 40), mat(k, 8 * 64, 1 << 44)
    need3 = L.blaz_matmul_workspace_bytes(8 * 256, 8 * 64, k, 1, 0)
    assert L.blaz_matmul_tiled(B(a3), B(b3), None, 8 * 64, 8 * 64, 1 << 46, 8 * 64, 0, 1 << 47, need3, 64,
                               None) == -2


def test_leading_dimension_limit(L):
    """A dense operand's last element must lie less than 2^60 elements past
    its first, so that element offsets and byte spans fit in int64; a larger
    ld is a shape error, not a wrapped overlap test."""
    x = mat(16, 16, 0x100000)
    big = (1 << 60) // 15 + 8                  # (rows - 1) * ld just over 2^60
    ok = ((1 << 60) - 16) // 15 // 2 * 2       # the largest even ld allowed for 16 rows
    A = 0x200000
    assert L.blaz_compress(A, big, B(x), 0, None, None) == -2
    assert L.blaz_decompress(B(x), A, big, None) == -2
    assert L.blaz_compress(A, 1 << 62, B(x), 0, None, None) == -2   # (rows - 1) * ld would wrap
    assert L.blaz_dot_dense(B(x), 0x300000, 0x500000, 1 << 62, 4, 0x400000, None) == -2
    a, b = mat(16, 24, 0x100000), mat(24, 8, 0x200000)
    need = L.blaz_matmul_workspace_bytes(16, 8, 24, 0, 0)
    assert L.blaz_matmul(B(a), None, 0x500000, 8, 1 << 62, 0x300000, 8, 0, 0x400000, need, None) == -2
    assert L.blaz_matmul(B(a), B(b), None, 8, 8, 0x300000, 1 << 62, 0, 0x400000, need, None) == -2
    c = mat(16, 8, 0x300000)
    needc = L.blaz_matmul_compressed_workspace_bytes(16, 8, 24, 0, 0)
    assert L.blaz_matmul_compressed(B(a), None, 0x500000, 8, 1 << 62, B(c), 0, 0x400000, needc, 0, None) == -2
    # at the bound the shape passes: the misaligned psi is the first error
    assert L.blaz_compress(A, ok, B(x), 0, 0x300008, None) == -4


def test_binding_rejects_host_tensors(L):
    """The binding passes only CUDA tensors on the current device to the
    library; a host tensor is refused before any call (no GPU needed)."""
    import torch
    import paper_2202_13007_amd as blaz
    from paper_2202_13007_amd import api
    with pytest.raises(ValueError):
        api._check_dense(torch.zeros((16, 16), dtype=torch.float64), "A", 0)
    with pytest.raises(ValueError):
        api._check_index(torch.zeros(4, dtype=torch.int64), "xrow", 4, 0)
    x = blaz.BlazMatrix(16, 16, torch.zeros(4, dtype=torch.float64), torch.zeros(4, dtype=torch.float64),
                        torch.zeros(4, dtype=torch.uint8), torch.zeros((4, 28), dtype=torch.int8))
    with pytest.raises(ValueError):
        x.c(0)


def test_status_strings(L):
    for st in range(-9, 1):
        assert len(L.blaz_status_string(st)) > 5


def test_static_product_refuses_what_the_scratch_cannot_hold(L):
    """blaz_matmul_static refuses a product whose workspace exceeds the
    static array before it looks the array up or enqueues anything."""
    scratch = 256 << 20
    assert L.blaz_matmul_workspace_bytes(4096, 4096, 4096, 1, 0) == scratch
    a, b = mat(4096, 4096, 1 << 40), mat(4096, 4104, 1 << 42)
    assert L.blaz_matmul_workspace_bytes(4096, 4104, 4096, 1, 0) > scratch
    assert L.blaz_matmul_static(B(a), B(b), None, 4104, 4104, 1 << 44, 4104, 0, None) == -9
    # FP32 with a dense B: a 8192 x 8192 A alone needs 256 MiB, the blocked B^T more
    a2 = mat(8192, 8192, 1 << 40)
    assert L.blaz_matmul_static(B(a2), None, 1 << 42, 64, 64, 1 << 44, 64, 1, None) == -9


def mat(rows, cols, base):
    from paper_2202_13007_amd._lib import BlazMatrixC
    nb = max(0, (rows // 8) * (cols // 8))
    # fake device addresses, laid out without overlap; never dereferenced
    return BlazMatrixC(rows, cols, base, base + 8 * nb + 64, base + 16 * nb + 128,
                       base + (17 * nb + 256 + 15) // 16 * 16)


B = ctypes.byref


def test_compress_validation(L):
    out = mat(16, 16, 0x100000)
    A = 0x200000
    assert L.blaz_compress(None, 16, B(out), 0, None, None) == -1
    assert L.blaz_compress(A, 8, B(out), 0, None, None) == -2          # lda < cols
    assert L.blaz_compress(A + 4, 16, B(out), 0, None, None) == -4     # misaligned A
    assert L.blaz_compress(A, 16, B(out), 9, None, None) == -5         # bad precision
    assert L.blaz_compress(0x100000, 16, B(out), 0, None, None) == -5  # A overlaps the output
    bad = mat(12, 16, 0x100000)
    assert L.blaz_compress(A, 16, B(bad), 0, None, None) == -2
    nul = mat(16, 16, 0x100000)
    nul.codes = None
    assert L.blaz_compress(A, 16, B(nul), 0, None, None) == -1
    mis = mat(16, 16, 0x100000)
    mis.codes = 0x100002
    assert L.blaz_compress(A, 16, B(mis), 0, None, None) == -4
    assert L.blaz_compress(A, 16, B(out), 0, 0x300008, None) == -4    # psi not 16-aligned
    empty = mat(0, 16, 0)
    assert L.blaz_compress(None, 16, B(empty), 0, None, None) == 0    # empty: no-op


def test_compress_predicted_validation(L):
    out = mat(16, 16, 0x100000)
    A = 0x200000
    f = L.blaz_compress_predicted
    assert f(None, 16, B(out), None, None) == -1
    assert f(A, 8, B(out), None, None) == -2                  # lda < cols
    assert f(A + 4, 16, B(out), None, None) == -4             # misaligned A
    assert f(A, 16, B(out), 0x300008, None) == -4             # psi not 16-aligned
    assert f(0x100000, 16, B(out), None, None) == -5          # A overlaps the output
    three = mat(16, 16, 0x100000)
    three.lines = 3
    assert f(A, 16, B(three), None, None) == -6               # two kept lines only
    assert f(None, 16, B(mat(0, 16, 0)), None, None) == 0     # empty: no-op


def test_decompress_validation(L):
    x = mat(16, 16, 0x100000)
    assert L.blaz_decompress(B(x), None, 16, None) == -1
    assert L.blaz_decompress(B(x), 0x200000, 15, None) == -2
    assert L.blaz_decompress(B(x), 0x200001, 16, None) == -4
    assert L.blaz_decompress(B(x), 0x100000 - 64, 16, None) == -5    # overlaps f


def test_add_scale_validation(L):
    x, y, z = mat(16, 16, 0x100000), mat(16, 16, 0x200000), mat(16, 16, 0x300000)
    w = mat(16, 24, 0x400000)
    assert L.blaz_add(B(x), B(w), B(z), None) == -3
    assert L.blaz_sub(B(x), B(y), B(w), None) == -3
    part = mat(16, 16, 0x100000 + 8)                                  # overlaps x, not equal
    assert L.blaz_add(B(x), B(y), B(part), None) == -5
    assert L.blaz_scale(B(x), 2.0, B(part), None) == -5
    assert L.blaz_scale(B(x), 2.0, B(w), None) == -3
    assert L.blaz_add(None, B(y), B(z), None) == -1
    e = mat(0, 0, 0)
    assert L.blaz_add(B(e), B(e), B(e), None) == 0


def test_dot_validation(L):
    x, y = mat(16, 24, 0x100000), mat(24, 8, 0x200000)
    idx, out = 0x300000, 0x400000
    assert L.blaz_dot(B(x), idx, B(x), idx, 4, out, None) == -3     # 24 != 16
    assert L.blaz_dot(B(x), idx, B(y), idx, -1, out, None) == -5
    assert L.blaz_dot(B(x), None, B(y), idx, 4, out, None) == -1
    assert L.blaz_dot(B(x), idx + 4, B(y), idx, 4, out, None) == -4
    assert L.blaz_dot(B(x), idx, B(y), idx, 0, None, None) == 0       # count 0: no-op
    assert L.blaz_dot_dense(B(x), idx, 0x500008, 0, 4, out, None) == -4   # v not 16-aligned
    assert L.blaz_dot_dense(B(x), idx, 0x500000, 23, 4, out, None) == -2  # ldv < cols
    assert L.blaz_dot_dense(B(x), idx, 0x500000, 25, 4, out, None) == -4  # odd ldv
    assert L.blaz_dot_dense(B(x), idx, 0x500000, -2, 4, out, None) == -5
    # out is written while the other queries read their indexes and vectors
    assert L.blaz_dot(B(x), idx, B(y), idx, 4, idx + 8, None) == -5          # out over xrow
    assert L.blaz_dot(B(x), idx, B(y), out - 16, 4, out, None) == -5         # out over ycol
    assert L.blaz_dot_dense(B(x), idx, out, 0, 4, out + 64, None) == -5      # out over the shared vector
    assert L.blaz_dot_dense(B(x), idx, out, 24, 4, out + 8 * 80, None) == -5  # over the last vector
    assert L.blaz_dot_dense(B(x), out + 24, 0x500000, 0, 4, out, None) == -5  # out over xrow


def test_matmul_validation(L):
    a, b = mat(16, 24, 0x100000), mat(24, 8, 0x200000)
    C, ws = 0x300000, 0x400000
    need = L.blaz_matmul_workspace_bytes(16, 8, 24, 1, 0)
    assert need >= 8 * (16 * 24 + 24 * 8)
    assert L.blaz_matmul(B(a), B(b), 0x500000, 8, 8, C, 8, 0, ws, need, None) == -5   # both B forms
    assert L.blaz_matmul(B(a), None, None, 8, 8, C, 8, 0, ws, need, None) == -1       # no B
    assert L.blaz_matmul(B(a), B(b), None, 16, 8, C, 16, 0, ws, need, None) == -3     # n != b.cols
    assert L.blaz_matmul(B(a), B(b), None, 8, 8, C, 8, 0, ws, need - 8, None) == -7
    assert L.blaz_matmul(B(a), B(b), None, 8, 8, C, 8, 0, None, need, None) == -7
    assert L.blaz_matmul(B(a), B(b), None, 8, 8, C, 8, 0, ws + 8, need, None) == -4
    assert L.blaz_matmul(B(a), B(b), None, 8, 8, C, 4, 0, ws, need, None) == -2       # ldc < n
    assert L.blaz_matmul(B(a), None, 0x500008, 8, 8, C, 8, 0, ws, need, None) == -4   # B not 16-aligned
    assert L.blaz_matmul(B(a), B(b), None, 8, 8, ws, 8, 0, ws, need, None) == -5      # C overlaps ws
    assert L.blaz_matmul(B(a), B(b), None, 8, 8, C, 8, 5, ws, need, None) == -5       # bad precision
    # the workspace, which the rebuilds write while the inputs are read, must
    # not overlap them: A's record, B's record, a dense B
    assert L.blaz_matmul(B(a), B(b), None, 8, 8, C, 8, 0, 0x100000, need, None) == -5
    assert L.blaz_matmul(B(a), B(b), None, 8, 8, C, 8, 0, 0x200000, need, None) == -5
    need_d = L.blaz_matmul_workspace_bytes(16, 8, 24, 0, 1)
    assert L.blaz_matmul(B(a), None, 0x500000, 8, 8, C, 8, 1, 0x500000, need_d, None) == -5


def test_matmul_compressed_validation(L):
    a, b = mat(16, 24, 0x100000), mat(24, 8, 0x200000)
    c, ws = mat(16, 8, 0x300000), 0x400000
    need = L.blaz_matmul_compressed_workspace_bytes(16, 8, 24, 1, 0)
    assert need >= L.blaz_matmul_workspace_bytes(16, 8, 24, 1, 0) + 8 * 16 * 8
    assert L.blaz_matmul_compressed_workspace_bytes(16, 8, 20, 1, 0) == 0              # k not a multiple of 8
    f = L.blaz_matmul_compressed
    assert f(B(a), B(b), 0x500000, 8, 8, B(c), 0, ws, need, 0, None) == -5   # both B forms
    assert f(B(a), None, None, 8, 8, B(c), 0, ws, need, 0, None) == -1       # no B
    assert f(B(a), B(b), None, 8, 8, B(mat(8, 8, 0x300000)), 0, ws, need, 0, None) == -3   # c shape
    assert f(B(a), B(b), None, 8, 8, B(c), 0, ws, need - 8, 0, None) == -7
    assert f(B(a), B(b), None, 8, 8, B(c), 0, ws + 8, need, 0, None) == -4
    assert f(B(a), B(b), None, 8, 8, B(c), 0, ws, need, 32, None) == -5      # tile
    assert f(B(a), B(b), None, 8, 8, B(c), 7, ws, need, 0, None) == -5       # precision
    assert f(B(a), B(b), None, 8, 8, B(mat(16, 8, ws + 256)), 0, ws, need, 0, None) == -5  # c inside ws
    assert f(B(a), B(b), None, 8, 8, B(mat(16, 8, 0x100000)), 0, ws, need, 0, None) == -5  # c over a


def test_diagnose_validation(L):
    x = mat(16, 16, 0x100000)
    assert L.blaz_diagnose(B(x), None, None) == -1
    assert L.blaz_diagnose(B(x), 0x500004, None) == -4
    assert L.blaz_diagnose(B(x), 0x100000, None) == -5                    # counters inside f
    assert L.blaz_diagnose(B(mat(0, 16, 0)), None, None) == 0             # nothing to count


def test_kept_lines_validation(L):
    """The tunable rate: code strides, sizes, and which calls take L != 2."""
    assert [L.blaz_code_stride(k) for k in range(0, 9)] == [28, 16, 28, 40, 48, 56, 60, 64, 64]
    assert L.blaz_code_stride(9) == -5 and L.blaz_code_stride(-1) == -5
    assert L.blaz_compressed_bytes_lines(16, 16, 3) == 4 * (17 + 40)
    assert L.blaz_compressed_bytes_lines(16, 16, 0) == L.blaz_compressed_bytes(16, 16) == 4 * 45

    def m3(rows, cols, base, lines=3):
        x = mat(rows, cols, base)
        x.lines = lines
        return x
    out = 0x700000
    assert L.blaz_decompress(B(m3(8, 8, 0x100000, 9)), out, 8, None) == -5               # L out of range
    assert L.blaz_decompress(B(m3(8, 8, 0x100000, -1)), out, 8, None) == -5
    x3, y2 = m3(8, 8, 0x100000), mat(8, 8, 0x200000)
    assert L.blaz_add(B(x3), B(y2), B(m3(8, 8, 0x300000)), None) == -3                  # rates differ
    assert L.blaz_scale(B(x3), 2.0, B(mat(8, 8, 0x300000)), None) == -3
    assert L.blaz_compress(0x400000, 8, B(m3(8, 8, 0x100000)), 1, None, None) == -6      # FP32 transform
    assert L.blaz_compress(0x400000, 8, B(m3(8, 8, 0x100000)), 0, 0x500000, None) == -6  # prediction output
    idx = 0x600000
    assert L.blaz_dot(B(x3), idx, B(m3(8, 8, 0x200000)), idx, 1, out, None) == -6
    assert L.blaz_dot_dense(B(x3), idx, 0x500000, 0, 1, out, None) == -6


# --------------------------------------------------------------------------
# The parity rules (tests/parity.py) catch what they should
# --------------------------------------------------------------------------

def test_tie_classifier():
    from oracle.parity import compare_compressed
    f, s = np.zeros(2), np.ones(2)
    phi = np.array([20, 20], np.uint8)
    codes = np.zeros((2, 28), np.int8)
    code_x = np.full((2, 28), 0.5)
    code_x[0, 0] = 126.0 - 1e-14          # a boundary tie
    codes_o = codes.copy()
    codes_o[0, 0] = 125
    codes_g = codes.copy()
    codes_g[0, 0] = 126
    ties = compare_compressed((f, s, phi, codes_g), (f, s, phi, codes_o), code_x, np.array([20.5, 20.5]))
    assert ties == 1
    code_x[0, 0] = 125.7                   # not near an integer: a real mismatch
    with pytest.raises(AssertionError):
        compare_compressed((f, s, phi, codes_g), (f, s, phi, codes_o), code_x, np.array([20.5, 20.5]))
    with pytest.raises(AssertionError):    # s must be bit-exact
        compare_compressed((f, s + 1e-16 * 4, phi, codes), (f, s, phi, codes), code_x, np.array([20.5, 20.5]))


def test_header_is_c99_and_links(L, tmp_path):
    """include/libblaz.h compiles as C99, every function it declares links
    against libblaz.so from a C program, and the host-only calls run."""
    import shutil
    import subprocess
    from paper_2202_13007_amd import _lib
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    names = declared_functions()
    src = tmp_path / "use_header.c"
    src.write_text("#include <stdio.h>\n#include \"libblaz.h\"\n"
                   "int main(void) {\n"
                   + "".join(f"    printf(\"%p\\n\", (void *)&{n});\n" for n in names)
                   + "    if (blaz_block_count(16, 24) != 6) return 1;\n"
                   "    if (blaz_compressed_bytes(16, 24) != 6 * 45) return 2;\n"
                   "    printf(\"%s\\n\", blaz_status_string(BLAZ_ERR_SHAPE));\n"
                   "    return 0;\n}\n")
    exe = tmp_path / "use_header"
    libdir = os.path.dirname(_lib.LIB_PATH)
    cmd = [gcc, "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", str(src), "-o", str(exe), "-L", libdir, "-lblaz", f"-Wl,-rpath,{libdir}"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr[-500:])
    assert len(r.stdout.splitlines()) == len(names) + 1


def test_launch_refused_by_the_runtime_is_reported_as_hip_error(L):
    """Where the HIP runtime cannot launch (here: no GPU), a call whose
    arguments pass validation returns BLAZ_ERR_HIP, and the binding turns it
    into a BlazError naming the status.  The fake addresses are never
    dereferenced: the launch itself is what fails.  Skipped where a GPU is
    present, since there the launch would run on the fake addresses."""
    import torch
    from paper_2202_13007_amd._lib import BLAZ_OK, BlazError, check
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present: the launch would run on fake addresses")
    x, z = mat(64, 64, 1 << 30), mat(64, 64, 1 << 32)
    st = L.blaz_scale(B(x), 2.0, B(z), None)
    assert st == -8 and L.blaz_status_string(st).decode() != ""
    assert L.blaz_add(B(x), B(x), B(z), None) == -8
    with pytest.raises(BlazError, match="BLAZ_ERR_HIP"):
        check(st, "blaz_scale")
    check(BLAZ_OK, "nothing")  # BLAZ_OK passes


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU's shard; asked for more it says so and
    exits with status 2 before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode == 2, (r.returncode, r.stdout[-500:], r.stderr[-500:])
    assert "one GPU only" in r.stdout + r.stderr


def test_extents_past_the_top_of_the_address_space_are_refused(L):
    """An array or dense operand whose byte extent would pass 2^64 cannot be
    an allocation: it is refused as an invalid argument (BLAZ_ERR_ARG)
    before anything is enqueued, also where it would otherwise look
    disjoint from the other operands."""
    from paper_2202_13007_amd._lib import BlazMatrixC
    top = 1 << 64
    high = BlazMatrixC(8, 16, top - 64, top - 32, top - 8, top - 4)  # 2 blocks: every array wraps
    low = mat(8, 16, 1 << 30)
    assert L.blaz_scale(B(high), 2.0, B(low), None) == -5
    assert L.blaz_add(B(low), B(low), B(high), None) == -5
    # a dense operand ending past the top (8 x 16 doubles from 2^64 - 512)
    assert L.blaz_decompress(B(low), ctypes.c_void_p(top - 512), 16, None) == -5
    assert L.blaz_compress(ctypes.c_void_p(top - 512), 16, B(low), 0, None, None) == -5
