"""Property tests of the host-side argument checks, with no GPU: random
descriptors for add, sub and scale against the rules include/libblaz.h
states.  A call those rules accept must get past validation to the launch,
which without a GPU fails as BLAZ_ERR_HIP (or returns BLAZ_OK at once when
there are no blocks); a call they reject must return another error before
anything is enqueued.  The addresses are fake and never dereferenced, so
the tests are skipped where a GPU is present."""
import ctypes

import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

BLAZ_OK, BLAZ_ERR_HIP = 0, -8
MAX_BLOCKS = (1 << 32) - 256
SETTINGS = settings(max_examples=500, deadline=None, database=None, suppress_health_check=[HealthCheck.too_slow])


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
        return f % 8 == 0 and s % 8 == 0 and codes % 4 == 0

    def ranges(self):
        n = self.nblk()
        f, s, phi, codes = self.ptrs
        sizes = (8 * n, 8 * n, n, code_stride(self.lines) * n)
        return [(p or 0, (p or 0) + z) for p, z in zip((f, s, phi, codes), sizes)]

    def c(self):
        from paper_2202_13007_amd._lib import BlazMatrixC
        f, s, phi, codes = self.ptrs
        return BlazMatrixC(self.rows, self.cols, f, s, phi, codes, self.lines)


def same_or_disjoint(z, x):
    if z.ptrs == x.ptrs:
        return True
    return not any(a < d and c < b for a, b in z.ranges() for c, d in x.ranges())


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
