"""Property tests of the host-side argument checks, with no GPU: random
descriptors for add, sub and scale against the rules include/libblaz.h
states.  A call those rules accept must get past validation to the launch,
which without a GPU fails as BLAZ_ERR_HIP (or returns BLAZ_OK at once when
there are no blocks); a call they reject must return another error before
anything is enqueued.  The addresses are fake and never dereferenced, so
the tests are skipped where a GPU is present."""
import ctypes
import os

import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

BLAZ_OK, BLAZ_ERR_HIP = 0, -8
MAX_BLOCKS = (1 << 32) - 256
TOP = 1 << 64  # addresses are unsigned 64-bit; an extent reaching TOP wraps
# Derandomized (the same draws on every run) unless BLAZ_PROPERTY_EXPLORE is
# set, which draws afresh.
SETTINGS = settings(max_examples=500, deadline=None, database=None, suppress_health_check=[HealthCheck.too_slow],
                    derandomize=not os.environ.get("BLAZ_PROPERTY_EXPLORE"))


@pytest.fixture(scope="module")
def L():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present: accepted calls would launch on fake addresses")
    from paper_2202_13007_amd import _lib
    return _lib.lib()


def code_stride(lines):
    l = 2 if lines == 0 else lines
    return 4 * ((16 * l - l * l + 3) // 4)


class Desc:
    """A descriptor and the rules' view of it."""

    def __init__(self, rows, cols, lines, f, s, phi, codes):
        self.rows, self.cols, self.lines = rows, cols, lines
        self.ptrs = (f, s, phi, codes)

    def nblk(self):
        return (self.rows // 8) * (self.cols // 8)

    def valid(self):
        r, c = self.rows, self.cols
        if not 0 <= self.lines <= 8:
            return False
        if r < 0 or c < 0 or r % 8 or c % 8:
            return False
        if r and c and self.nblk() > MAX_BLOCKS:
            return False
        if self.nblk() == 0:
            return True
        f, s, phi, codes = self.ptrs
        if not (f and s and phi and codes):
            return False
        if not (f % 8 == 0 and s % 8 == 0 and codes % 4 == 0):
            return False
        return not any(wraps(r) for r in self.ranges())

    def ranges(self):
        n = self.nblk()
        f, s, phi, codes = self.ptrs
        sizes = (8 * n, 8 * n, n, code_stride(self.lines) * n)
        return [(p or 0, (p or 0) + z) for p, z in zip((f, s, phi, codes), sizes)]

    def c(self):
        from paper_2202_13007_amd._lib import BlazMatrixC
        f, s, phi, codes = self.ptrs
        return BlazMatrixC(self.rows, self.cols, f, s, phi, codes, self.lines)


def wraps(r):
    return r[1] > r[0] and r[1] >= TOP


def overlap(r, q):
    """Byte ranges [lo, hi) that overlap; a wrapping range overlaps everything."""
    return wraps(r) or wraps(q) or (r[0] < q[1] and q[0] < r[1])


def same_or_disjoint(z, x):
    if z.ptrs == x.ptrs:
        return True
    return not any(overlap(r, q) for r in z.ranges() for q in x.ranges())


SIDES = st.sampled_from([0, 8, 16, 24, 64, 8, 16, 24, 64, 7, -8, 8 << 22])
LINES = st.sampled_from([0, 0, 2, 1, 3, 8, 9, -1])
# (array index f, s, phi, codes; byte shift, or None for a NULL pointer)
FAULTS = st.sampled_from([None] * 8 + [(0, 1), (0, 4), (1, 4), (2, 1), (3, 1), (3, 2), (3, 4),
                                       (0, None), (1, None), (2, None), (3, None)])
REGIONS = (1 << 30, 1 << 36, 1 << 40)


@st.composite
def descriptor(draw, like=None):
    """A descriptor with its four arrays laid out without overlap from a base
    address, one of them possibly misaligned or NULL.  With `like`, the shape
    and lines are often copied and the arrays may be `like`'s own, shifted
    into them, or elsewhere."""
    if like is not None and draw(st.integers(0, 3)) > 0:
        rows, cols, lines = like.rows, like.cols, like.lines
    else:
        rows, cols, lines = draw(SIDES), draw(SIDES), draw(LINES)
    n = max(0, rows // 8) * max(0, cols // 8)
    where = draw(st.sampled_from(["own", "same", "shifted"])) if like is not None else "own"
    if where == "same":
        return Desc(rows, cols, lines, *like.ptrs)
    if where == "shifted":
        base = (like.ptrs[0] or REGIONS[0]) + draw(st.sampled_from([8, 64, 8 * max(n, 1)]))
    else:
        base = draw(st.sampled_from(REGIONS)) + (1 << 24) * draw(st.integers(0, 3))
    size = max(n, 1) * 64
    ptrs = [base + k * size for k in range(4)]
    # at most one fault per descriptor: an array misaligned or missing
    fault = draw(FAULTS)
    if fault is not None:
        k, shift = fault
        ptrs[k] = None if shift is None else ptrs[k] + shift
    return Desc(rows, cols, lines, *ptrs)


@st.composite
def binary_args(draw):
    x = draw(descriptor())
    y = draw(descriptor(like=x))
    z = draw(descriptor(like=x))
    return x, y, z


def expect(valid, nblk):
    return (BLAZ_ERR_HIP if nblk else BLAZ_OK) if valid else None


def check(status, want, what):
    if want is None:
        assert status not in (BLAZ_OK, BLAZ_ERR_HIP), f"{what}: accepted ({status})"
    else:
        assert status == want, f"{what}: status {status}, expected {want}"


@SETTINGS
@given(binary_args())
def test_add_and_sub_accept_exactly_what_the_rules_allow(L, args):
    x, y, z = args
    ok = all(d.valid() for d in (x, y, z))
    if ok:
        l2 = lambda d: 2 if d.lines == 0 else d.lines
        ok = (x.rows, x.cols, l2(x)) == (y.rows, y.cols, l2(y)) == (z.rows, z.cols, l2(z))
    if ok and x.nblk():
        ok = same_or_disjoint(z, x) and same_or_disjoint(z, y)
    want = expect(ok, x.nblk() if ok else 0)
    cx, cy, cz = x.c(), y.c(), z.c()
    check(L.blaz_add(ctypes.byref(cx), ctypes.byref(cy), ctypes.byref(cz), None), want, "add")
    check(L.blaz_sub(ctypes.byref(cx), ctypes.byref(cy), ctypes.byref(cz), None), want, "sub")


@SETTINGS
@given(binary_args(), st.floats(allow_nan=True))
def test_scale_accepts_exactly_what_the_rules_allow(L, args, c):
    x, _, z = args
    ok = x.valid() and z.valid()
    if ok:
        l2 = lambda d: 2 if d.lines == 0 else d.lines
        ok = (x.rows, x.cols, l2(x)) == (z.rows, z.cols, l2(z))
    if ok and x.nblk():
        ok = same_or_disjoint(z, x)
    want = expect(ok, x.nblk() if ok else 0)
    cx, cz = x.c(), z.c()
    check(L.blaz_scale(ctypes.byref(cx), ctypes.c_double(c), ctypes.byref(cz), None), want, "scale")


def test_null_descriptors_are_refused(L):
    x = Desc(8, 8, 0, 1 << 30, (1 << 30) + 64, (1 << 30) + 128, (1 << 30) + 192).c()
    assert L.blaz_add(None, ctypes.byref(x), ctypes.byref(x), None) not in (BLAZ_OK, BLAZ_ERR_HIP)
    assert L.blaz_scale(ctypes.byref(x), ctypes.c_double(1.0), None, None) not in (BLAZ_OK, BLAZ_ERR_HIP)


def dense_span(base, rows, cols, lda):
    return (base, base + (((rows - 1) * lda + cols) * 8 if rows > 0 else 0))


def overlaps_desc(r, d):
    return any(overlap(r, q) for q in d.ranges())


@st.composite
def dense_args(draw):
    """A descriptor, a dense operand placed apart from it, over its arrays,
    ending on its first element, running past 2^64, misaligned or NULL, a
    leading dimension that may be short, and for compression an optional Psi
    buffer placed apart, over either, or misaligned."""
    m = draw(descriptor())
    cols = max(m.cols, 0)
    lda = cols + draw(st.sampled_from([0, 0, 2, 8, -8, -1]))
    place = draw(st.sampled_from(["apart", "apart", "apart", "apart", "over", "tail", "top", "misaligned", "null"]))
    base = (1 << 44) + (1 << 20) * draw(st.integers(0, 3))
    rows = max(m.rows, 0)
    extent = ((rows - 1) * lda + cols) * 8 if rows > 0 else 0
    f = m.ptrs[0] or base
    # "tail": only the operand's last element lies on the descriptor's f array
    # "top": the operand starts below 2^64 and its extent passes it
    A = {"apart": base, "over": (m.ptrs[3] or base) - 8, "tail": (f - extent + 8) % TOP,
         "top": TOP - 8 * (extent // 16 + 1), "misaligned": base + 4, "null": None}[place]
    pplace = draw(st.sampled_from(["none", "none", "none", "apart", "over_a", "over_m", "misaligned"]))
    pbase = (1 << 46) + (1 << 20) * draw(st.integers(0, 3))
    psi = {"none": None, "apart": pbase, "over_a": A, "over_m": m.ptrs[0], "misaligned": pbase + 8}[pplace]
    prec = draw(st.sampled_from([0, 0, 0, 1, 2, 3, -1]))
    return m, A, lda, psi, prec


def compress_model(m, A, lda, psi, prec):
    """Whether blaz_compress's rules accept the call, and its block count."""
    ok = m.valid() and prec in (0, 1, 2)
    lines = 2 if m.lines == 0 else m.lines
    if ok and lines != 2 and (prec != 0 or psi is not None):
        ok = False
    n = m.nblk() if ok else 0
    if ok and n:
        ok = (A is not None and lda >= m.cols and A % 8 == 0 and (psi is None or psi % 16 == 0))
        if ok:
            ra = dense_span(A, m.rows, m.cols, lda)
            ok = not overlaps_desc(ra, m)
            if ok and psi is not None:
                rp = (psi, psi + 64 * n)
                ok = not overlap(rp, ra) and not overlaps_desc(rp, m)
    return ok, n


@SETTINGS
@given(dense_args())
def test_compress_accepts_exactly_what_the_rules_allow(L, args):
    m, A, lda, psi, prec = args
    ok, n = compress_model(m, A, lda, psi, prec)
    cm = m.c()
    check(L.blaz_compress(ctypes.c_void_p(A), lda, ctypes.byref(cm), prec, ctypes.c_void_p(psi), None),
          expect(ok, n if ok else 0), f"compress prec {prec}")
    # the predicted-slope input: the binary64 rules, two kept lines only
    ok, n = compress_model(m, A, lda, psi, 0)
    ok = ok and m.valid() and (2 if m.lines == 0 else m.lines) == 2
    check(L.blaz_compress_predicted(ctypes.c_void_p(A), lda, ctypes.byref(cm), ctypes.c_void_p(psi), None),
          expect(ok, n if ok else 0), "compress_predicted")


@SETTINGS
@given(dense_args())
def test_decompress_accepts_exactly_what_the_rules_allow(L, args):
    m, A, lda, _, _ = args
    ok = m.valid()
    n = m.nblk() if ok else 0
    if ok and n:
        ok = A is not None and lda >= m.cols and A % 8 == 0 and not overlaps_desc(dense_span(A, m.rows, m.cols, lda), m)
    cm = m.c()
    check(L.blaz_decompress(ctypes.byref(cm), ctypes.c_void_p(A), lda, None), expect(ok, n), "decompress")


MATMUL_FAULTS = [None] * 8 + ["tile", "prec", "both", "neither", "bshape", "n", "cnull", "calign", "ldc",
                              "ldb", "ldbodd", "balign", "wsnull", "wsshort", "wsalign", "c_a", "c_bd", "c_ws",
                              "ws_a", "ws_b", "ws_bd"]


@st.composite
def matmul_args(draw):
    """A valid product (compressed A of at least one block, B compressed or
    dense, C and the workspace apart from each other) with at most one
    fault: a bad tile or precision, both or neither form of B, B's shape,
    n, C or the workspace NULL, misaligned, short or over another operand,
    or a short or odd leading dimension."""
    rows, cols = draw(st.sampled_from([8, 16, 24])), draw(st.sampled_from([8, 16, 24]))
    a = Desc(rows, cols, draw(st.sampled_from([0, 2, 1, 3])), *[(1 << 36) + i * (1 << 20) for i in range(4)])
    m, k = rows, cols
    n = draw(st.sampled_from([8, 16, 24]))
    dense = draw(st.booleans())
    b = None if dense else Desc(k, n, draw(st.sampled_from([0, 2, 3])), *[(1 << 38) + i * (1 << 20) for i in range(4)])
    bdense = (1 << 42) if dense else None
    ldb, ldc = n + draw(st.sampled_from([0, 2])), n + draw(st.sampled_from([0, 8]))
    c, ws, prec, tile, short = 1 << 43, 1 << 45, draw(st.sampled_from([0, 1, 2])), draw(st.sampled_from([0, 64, 128])), 0
    fault = draw(st.sampled_from(MATMUL_FAULTS))
    if fault == "tile":
        tile = 32
    elif fault == "prec":
        prec = 7
    elif fault == "both":
        b, bdense = b or Desc(k, n, 0, *[(1 << 38) + i * (1 << 20) for i in range(4)]), bdense or (1 << 42)
    elif fault == "neither":
        b = bdense = None
    elif fault == "bshape" and b is not None:
        b = Desc(k + 8, n, b.lines, *b.ptrs)
    elif fault == "n":
        n += 4
    elif fault == "cnull":
        c = None
    elif fault == "calign":
        c += 4
    elif fault == "ldc":
        ldc = n - 8
    elif fault == "ldb":
        ldb = n - 2
    elif fault == "ldbodd":
        ldb = n + 1
    elif fault == "balign" and bdense is not None:
        bdense += 8
    elif fault == "wsnull":
        ws = None
    elif fault == "wsshort":
        short = 8
    elif fault == "wsalign":
        ws += 128
    elif fault == "c_a":
        c = a.ptrs[1]
    elif fault == "c_bd" and bdense is not None:
        c = bdense + 8 * n
    elif fault == "c_ws":
        c = ws + 64
    elif fault == "ws_a":
        ws = a.ptrs[0]
    elif fault == "ws_b" and b is not None:
        ws = b.ptrs[3]
    elif fault == "ws_bd" and bdense is not None:
        ws = bdense
    return a, b, bdense, n, ldb, c, ldc, prec, ws, short, tile


def matmul_model(L, a, b, bdense, n, ldb, c, ldc, prec, ws, tile, ws_bytes):
    """Whether the header's rules accept the call, and whether it launches."""
    if tile not in (0, 64, 128) or not a.valid() or prec not in (0, 1, 2):
        return False, False
    m, k = a.rows, a.cols
    if b is not None and bdense is not None:
        return False, False
    if b is None and bdense is None and k > 0:
        return False, False
    if b is not None and (not b.valid() or b.rows != k or b.cols != n):
        return False, False
    if n < 0 or n % 8:
        return False, False
    if m == 0 or n == 0:
        return True, False
    if not c or ldc < n or c % 8:
        return False, False
    if b is None and k > 0 and (ldb < n or bdense % 16 or ldb % 2):
        return False, False
    need = L.blaz_matmul_workspace_bytes(m, n, k, int(b is not None), prec)
    if k > 0 and (not ws or ws_bytes < need or ws % 256):
        return False, False
    rc = dense_span(c, m, n, ldc)
    rb = dense_span(bdense, k, n, ldb) if bdense is not None else None
    rw = (ws, ws + need) if k > 0 else None
    ins = [q for q in a.ranges()] + (b.ranges() if b is not None else []) + ([rb] if rb else [])
    if any(overlap(rc, q) for q in ins) or (rw and overlap(rc, rw)):
        return False, False
    if rw and any(overlap(rw, q) for q in ins):
        return False, False
    return True, True


@SETTINGS
@given(matmul_args())
def test_matmul_accepts_exactly_what_the_rules_allow(L, args):
    a, b, bdense, n, ldb, c, ldc, prec, ws, short, tile = args
    need = L.blaz_matmul_workspace_bytes(max(a.rows, 0), n, max(a.cols, 0), int(b is not None), prec if prec in (0, 1, 2) else 0)
    ws_bytes = max(need - short, 0)
    ok, launches = matmul_model(L, a, b, bdense, n, ldb, c, ldc, prec, ws, tile, ws_bytes)
    ca = a.c()
    cb = b.c() if b is not None else None
    st_ = L.blaz_matmul_tiled(ctypes.byref(ca), ctypes.byref(cb) if cb is not None else None, ctypes.c_void_p(bdense),
                              n, ldb, ctypes.c_void_p(c), ldc, prec, ctypes.c_void_p(ws), ws_bytes, tile, None)
    want = (BLAZ_ERR_HIP if launches else BLAZ_OK) if ok else None
    check(st_, want, f"matmul form {'c' if b else ''}{'d' if bdense else ''} prec {prec} tile {tile}")


DOT_FAULTS = [None] * 6 + ["cols", "lines", "count", "xnull", "ynull", "onull", "xalign", "oalign", "o_x", "o_y",
                           "o_xrow", "o_ycol", "valign", "ldv", "ldvodd", "o_v"]


@st.composite
def dot_args(draw):
    """Valid compressed-pair and dense-vector dot calls with at most one
    fault: mismatched shapes or rates, a bad count, an index, output or
    vector array NULL, misaligned or overlapping the output, a short or
    odd ldv."""
    rows, cols, n = (draw(st.sampled_from([8, 16, 24])) for _ in range(3))
    x = Desc(rows, cols, 0, *[(1 << 36) + i * (1 << 20) for i in range(4)])
    y = Desc(cols, n, 0, *[(1 << 38) + i * (1 << 20) for i in range(4)])
    count = draw(st.sampled_from([0, 1, 4, 9]))
    xrow, ycol, out, v = 1 << 40, (1 << 40) + (1 << 20), 1 << 42, 1 << 44
    ldv = draw(st.sampled_from([0, cols, cols + 2]))
    fault = draw(st.sampled_from(DOT_FAULTS))
    if fault == "cols":
        y = Desc(cols + 8, n, 0, *y.ptrs)
    elif fault == "lines":
        x = Desc(rows, cols, 3, *x.ptrs)
    elif fault == "count":
        count = -1
    elif fault == "xnull":
        xrow = None
    elif fault == "ynull":
        ycol = None
    elif fault == "onull":
        out = None
    elif fault == "xalign":
        xrow += 4
    elif fault == "oalign":
        out += 4
    elif fault == "o_x":
        out = x.ptrs[2]
    elif fault == "o_y":
        out = y.ptrs[0] + 8
    elif fault == "o_xrow":
        out = xrow + 8
    elif fault == "o_ycol":
        out = ycol - 8
    elif fault == "valign":
        v += 8
    elif fault == "ldv":
        ldv = cols - 2
    elif fault == "ldvodd":
        ldv = cols + 1
    elif fault == "o_v":
        out = v + 8 * (ldv * max(count - 1, 0) + cols) - 8
    return x, y, count, xrow, ycol, out, v, ldv


def rng8(p, count):
    return (p, p + 8 * count) if p else (0, 0)


@SETTINGS
@given(dot_args())
def test_dot_and_dot_dense_accept_exactly_what_the_rules_allow(L, args):
    x, y, count, xrow, ycol, out, v, ldv = args
    i64 = ctypes.c_void_p
    # compressed pairs
    ok = x.cols == y.rows and x.lines in (0, 2) and y.lines in (0, 2) and 0 <= count
    if ok and count:
        ok = all(p and p % 8 == 0 for p in (xrow, ycol, out))
        if ok:
            ro = rng8(out, count)
            ok = not (overlaps_desc(ro, x) or overlaps_desc(ro, y) or overlap(ro, rng8(xrow, count))
                      or overlap(ro, rng8(ycol, count)))
    cx, cy = x.c(), y.c()
    check(L.blaz_dot(ctypes.byref(cx), i64(xrow), ctypes.byref(cy), i64(ycol), count, i64(out), None),
          expect(ok, count if ok else 0), "dot")
    # dense vectors
    ok = x.lines in (0, 2) and 0 <= count and ldv >= 0 and (ldv == 0 or ldv >= x.cols)
    if ok and count:
        ok = all(p and p % 8 == 0 for p in (xrow, out)) and v and v % 16 == 0 and ldv % 2 == 0
        if ok:
            ro = rng8(out, count)
            rv = (v, v + (8 * x.cols if ldv == 0 else ((count - 1) * ldv + x.cols) * 8))
            ok = not (overlaps_desc(ro, x) or overlap(ro, rng8(xrow, count)) or overlap(ro, rv))
    check(L.blaz_dot_dense(ctypes.byref(cx), i64(xrow), i64(v), ldv, count, i64(out), None),
          expect(ok, count if ok else 0), "dot_dense")


# Batches: items over a small pool of operands, so that items meet each other
# often; the rule (no item reads or writes another item's output, inputs may
# be shared) is checked by brute force over the pairs.
POOL_X = [(1 << 40) + i * (1 << 20) for i in range(4)]      # compressed 8 x 64 records
POOL_D = [(1 << 42) + i * (1 << 20) for i in range(2)]      # dense 8 x 64, ld 64
POOL_I = [(1 << 44) + i * (1 << 20) for i in range(2)]      # index arrays
POOL_O = [(1 << 45) + i * (1 << 20) for i in range(2)]      # dot outputs
Y_DOT = (1 << 46)                                            # a read-only 64 x 8 record


def pool_desc(base, rows=8, cols=64):
    nb = (rows // 8) * (cols // 8)
    return Desc(rows, cols, 0, base, base + 8 * nb + 64, base + 16 * nb + 128, base + 17 * nb + 256)


@st.composite
def batch_items(draw):
    ops = []
    for _ in range(draw(st.integers(1, 5))):
        op = draw(st.sampled_from(["add", "scale", "compress", "decompress", "dot"]))
        if op == "add":
            ops.append(("add", dict(x=draw(st.sampled_from(POOL_X)), y=draw(st.sampled_from(POOL_X)),
                                    z=draw(st.sampled_from(POOL_X)))))
        elif op == "scale":
            ops.append(("scale", dict(x=draw(st.sampled_from(POOL_X)), z=draw(st.sampled_from(POOL_X)))))
        elif op in ("compress", "decompress"):
            ops.append((op, dict(x=draw(st.sampled_from(POOL_X)), dense=draw(st.sampled_from(POOL_D)))))
        else:
            ops.append(("dot", dict(x=draw(st.sampled_from(POOL_X)), xrow=draw(st.sampled_from(POOL_I)),
                                    ycol=draw(st.sampled_from(POOL_I)), out=draw(st.sampled_from(POOL_O)))))
    return ops


def batch_rw(op, a):
    """(writes, reads) of an item as sets of pool addresses."""
    if op == "add":
        return {a["z"]}, {a["x"], a["y"]}
    if op == "scale":
        return {a["z"]}, {a["x"]}
    if op == "compress":
        return {a["x"]}, {a["dense"]}
    if op == "decompress":
        return {a["dense"]}, {a["x"]}
    return {a["out"]}, {a["x"], a["xrow"], a["ycol"], Y_DOT}


@SETTINGS
@given(batch_items())
def test_batch_plan_refuses_exactly_the_items_that_touch_another_items_output(L, ops):
    from paper_2202_13007_amd import _lib
    conflicts = set()
    for j in range(len(ops)):
        wj, rj = batch_rw(*ops[j])
        for i in range(j):
            wi, ri = batch_rw(*ops[i])
            if wi & wj or wi & rj or ri & wj:
                conflicts.add(j)
    arr = (_lib.BatchItemC * len(ops))()
    for it, (op, a) in zip(arr, ops):
        it.op = _lib.OPS[op]
        if op in ("add", "scale", "compress", "decompress", "dot"):
            it.x = pool_desc(a["x"]).c()
        if op == "add":
            it.y, it.z = pool_desc(a["y"]).c(), pool_desc(a["z"]).c()
        elif op == "scale":
            it.z, it.c = pool_desc(a["z"]).c(), 1.5
        elif op in ("compress", "decompress"):
            it.dense, it.ld = a["dense"], 64
        else:
            it.y = pool_desc(Y_DOT, 64, 8).c()
            it.xrow, it.ycol, it.out, it.count = a["xrow"], a["ycol"], a["out"], 4
    nbytes = L.blaz_batch_plan_bytes(len(ops))
    buf = (ctypes.c_uint8 * nbytes)()
    n_plan, total = ctypes.c_int64(), ctypes.c_int64()
    st_ = L.blaz_batch_plan(ctypes.cast(arr, ctypes.c_void_p), len(ops), ctypes.cast(buf, ctypes.c_void_p), nbytes,
                            ctypes.byref(n_plan), ctypes.byref(total))
    if conflicts:
        assert st_ == -5 and n_plan.value in conflicts, (ops, st_, n_plan.value, conflicts)
    else:
        assert st_ == BLAZ_OK and n_plan.value == len(ops), (ops, st_, n_plan.value)


# Grouped products over a small pool: A (8 x 64 records), B compressed
# (64 x 8 records) or dense (64 x 8, ld 8), C (8 x 8, ld 8) from a pool that
# also holds the dense B regions, so that outputs meet other products'
# operands and outputs.
POOL_A = POOL_X[:3]
POOL_B = [(1 << 47) + i * (1 << 20) for i in range(2)]
POOL_BD = [(1 << 48) + i * (1 << 20) for i in range(2)]
POOL_C = [(1 << 49) + i * (1 << 20) for i in range(3)] + POOL_BD


@st.composite
def group_items(draw):
    items = []
    for _ in range(draw(st.integers(1, 5))):
        a = draw(st.sampled_from(POOL_A))
        if draw(st.booleans()):
            b, bd = draw(st.sampled_from(POOL_B)), None
        else:
            b, bd = None, draw(st.sampled_from(POOL_BD))
        c = draw(st.sampled_from([p for p in POOL_C if p != bd]))  # never over its own operands
        items.append((a, b, bd, c))
    return items


@SETTINGS
@given(group_items())
def test_group_plan_refuses_exactly_the_products_that_touch_another_products_output(L, items):
    from paper_2202_13007_amd import _lib
    conflicts = set()
    for j, (aj, bj, dj, cj) in enumerate(items):
        for i in range(j):
            ai, bi, di, ci = items[i]
            if ci == cj or ci in (aj, bj, dj) or cj in (ai, bi, di):
                conflicts.add(j)
    arr = (_lib.MatmulItemC * len(items))()
    for it, (a, b, bd, c) in zip(arr, items):
        it.a = pool_desc(a).c()
        it.b = pool_desc(b, 64, 8).c() if b is not None else _lib.BlazMatrixC(0, 0, None, None, None, None, 0)
        it.bdense = bd
        it.n, it.ldb, it.c, it.ldc, it.tile, it.reserved = 8, 8, c, 8, 64, 0
    nbytes = L.blaz_matmul_group_plan_bytes(len(items))
    buf = (ctypes.c_uint8 * nbytes)()
    info = _lib.MatmulGroupInfoC()
    st_ = L.blaz_matmul_group_plan(ctypes.cast(arr, ctypes.c_void_p), len(items), ctypes.c_void_p(1 << 50), 1 << 30,
                                   ctypes.cast(buf, ctypes.c_void_p), nbytes, ctypes.byref(info))
    if conflicts:
        assert st_ == -5 and info.rebuild_jobs in conflicts, (items, st_, info.rebuild_jobs, conflicts)
    else:
        assert st_ == BLAZ_OK, (items, st_, info.rebuild_jobs)


@SETTINGS
@given(matmul_args(), st.sampled_from(["apart", "apart", "apart", "over_a", "over_b", "over_ws", "shape", "lines3"]))
def test_matmul_compressed_accepts_exactly_what_the_rules_allow(L, args, cplace):
    """The product recompressed: the operands and workspace drawn as for
    blaz_matmul_tiled, the output a descriptor placed apart, over A, over B
    (compressed or dense) or over the workspace, or of the wrong shape."""
    a, b, bdense, n, ldb, _, _, prec, ws, short, tile = args
    m, k = a.rows, a.cols
    cbase = {"over_a": a.ptrs[2], "over_b": (b.ptrs[0] if b is not None else bdense),
             "over_ws": (ws + 512) if ws else None}.get(cplace) or (1 << 51)
    c = Desc(m + (8 if cplace == "shape" else 0), n, 3 if cplace == "lines3" else 0,
             cbase, cbase + 8 * (1 << 16), cbase + 16 * (1 << 16), cbase + 17 * (1 << 16))
    p = prec if prec in (0, 1, 2) else 0
    need = L.blaz_matmul_compressed_workspace_bytes(m, n, k, int(b is not None), p)
    ws_bytes = max(need - short, 0)
    ok = tile in (0, 64, 128) and a.valid() and c.valid() and prec in (0, 1, 2)
    ok = ok and not (b is not None and bdense is not None) and not (b is None and bdense is None and k > 0)
    if ok and b is not None:
        ok = b.valid() and b.rows == k and b.cols == n
    ok = ok and n >= 0 and n % 8 == 0 and c.rows == m and c.cols == n
    launches = ok and m > 0 and n > 0
    if launches:
        if b is None and k > 0:
            ok = ldb >= n and bdense % 16 == 0 and ldb % 2 == 0
        ok = ok and ws is not None and ws_bytes >= need and ws % 256 == 0
        if ok:
            rw = (ws, ws + need)
            ins = a.ranges() + (b.ranges() if b is not None else []) + \
                ([dense_span(bdense, k, n, ldb)] if bdense is not None else [])
            ok = not overlaps_desc(rw, c) and not any(overlap(rw, q) for q in ins) and \
                not any(overlap(r, q) for r in c.ranges() for q in ins)
        launches = ok
    ca, cc = a.c(), c.c()
    cb = b.c() if b is not None else None
    st_ = L.blaz_matmul_compressed(ctypes.byref(ca), ctypes.byref(cb) if cb is not None else None,
                                   ctypes.c_void_p(bdense), n, ldb, ctypes.byref(cc), prec, ctypes.c_void_p(ws),
                                   ws_bytes, tile, None)
    check(st_, (BLAZ_ERR_HIP if launches else BLAZ_OK) if ok else None, f"matmul_compressed {cplace}")


@SETTINGS
@given(descriptor(), st.sampled_from(["apart", "apart", "over", "misaligned", "null"]))
def test_diagnose_accepts_exactly_what_the_rules_allow(L, x, where):
    """blaz_diagnose: a valid record and, when it holds blocks, four 8-byte
    aligned counters apart from it."""
    cnt = {"apart": 1 << 50, "over": x.ptrs[1], "misaligned": (1 << 50) + 4, "null": None}[where]
    ok = x.valid()
    n = x.nblk() if ok else 0
    if ok and n:
        ok = bool(cnt) and cnt % 8 == 0 and not overlaps_desc((cnt, cnt + 32), x)
    cx = x.c()
    check(L.blaz_diagnose(ctypes.byref(cx), ctypes.c_void_p(cnt), None), expect(ok, n if ok else 0), "diagnose")
