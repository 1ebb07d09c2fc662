"""Comparison rules between the HIP library and the FP64 oracle -- test
infrastructure, used only by the tests and the benchmark's parity report.

* f, s, phi, codes of a compression: bit-exact, except at rounding-boundary
  ties.  A mismatching code (or phi) is a tie when the oracle's value before
  truncation lies within 2^-40 * max(1, |x|) of an integer and the two
  results differ by exactly 1; such ties must stay under 1e-6 of the codes.
  When phi itself flips at a tie, that block's codes are checked against
  trunc(phi_gpu * D) with D recovered from the oracle's pre-truncation values.
* add, sub, scale: bit-exact.
* decompression: |X_gpu - X_oracle| <= 1e-12 * max|X_oracle| per 8x8 block.
* dot and matmul: |r_gpu - r_oracle| <= 1e-12 * sum_k |x_k y_k|.
* products whose contraction runs in FP32 or BF16 hi+lo (three products):
  |r_gpu - r_oracle| <= low_precision_tol(prec, k) * sum_k |x_k y_k|.
"""
from __future__ import annotations

import numpy as np

TIE_REL = 2.0 ** -40
TIE_RATE_MAX = 1e-6
DECOMP_REL = 1e-12
DOT_REL = 1e-12
U32 = 2.0 ** -24


def low_precision_tol(prec, k):
    """Bound on |C - C64| relative to sum_k |a_k b_k| for a K-term product
    with FP32 accumulation: operand rounding (FP32: 2 u32; BF16x3: 3 * 2^-16
    from the split and the dropped lo*lo term) plus the accumulation (K/4 u32
    for the FP32 16x16x4 form, K u32 for BF16x3, whose MFMA sums 32 products
    per step)."""
    return (2 + k / 4 + 4) * U32 if prec == "fp32" else 3 * 2.0 ** -16 + (k + 4) * U32


def near_integer(x):
    return np.abs(x - np.round(x)) <= TIE_REL * np.maximum(1.0, np.abs(x))


def compare_compressed(gpu, orc, code_x, phi_x, what="compress"):
    """gpu, orc: (f, s, phi, codes) numpy tuples.  Returns the number of ties;
    raises AssertionError on any other difference."""
    gf, gs, gphi, gcodes = gpu
    of, os_, ophi, ocodes = orc
    nb = len(of)
    n = code_x.shape[1]  # codes per block: 28, or 16L - L^2 for L kept lines
    assert gcodes.shape == ocodes.shape and gcodes.shape[0] == nb and gcodes.shape[1] >= n
    assert not gcodes[:, n:].any(), f"{what}: pad bytes after the codes are not zero"
    gcodes, ocodes = gcodes[:, :n], ocodes[:, :n]
    bad_f = np.flatnonzero(gf.view(np.uint64) != of.view(np.uint64))
    assert bad_f.size == 0, f"{what}: f differs at blocks {bad_f[:10]}"
    bad_s = np.flatnonzero(gs.view(np.uint64) != os_.view(np.uint64))
    assert bad_s.size == 0, f"{what}: s differs at blocks {bad_s[:10]}: {gs[bad_s[:3]]} vs {os_[bad_s[:3]]}"
    ties = 0
    phi_diff = np.flatnonzero(gphi != ophi)
    for b in phi_diff:
        ok = abs(int(gphi[b]) - int(ophi[b])) == 1 and near_integer(phi_x[b])
        assert ok, f"{what}: phi differs at block {b}: {gphi[b]} vs {ophi[b]} (127/m = {phi_x[b]!r})"
        ties += 1
        D = code_x[b] / float(ophi[b])
        want = np.trunc(float(gphi[b]) * D)
        diff = gcodes[b].astype(int) - want.astype(int)
        okc = (diff == 0) | ((np.abs(diff) == 1) & near_integer(float(gphi[b]) * D))
        assert np.all(okc), f"{what}: codes of block {b} inconsistent with its flipped phi"
    same_phi = gphi == ophi
    diff = gcodes.astype(int) - ocodes.astype(int)
    mism = (diff != 0) & same_phi[:, None]
    if mism.any():
        bb, tt = np.nonzero(mism)
        tie = (np.abs(diff[bb, tt]) == 1) & near_integer(code_x[bb, tt])
        assert np.all(tie), (f"{what}: {int((~tie).sum())} codes differ off a rounding boundary, e.g. block "
                             f"{bb[~tie][:5]} index {tt[~tie][:5]}: gpu {gcodes[bb[~tie][:5], tt[~tie][:5]]} "
                             f"oracle {ocodes[bb[~tie][:5], tt[~tie][:5]]} x {code_x[bb[~tie][:5], tt[~tie][:5]]}")
        ties += int(tie.sum())
    return ties


def assert_same_compressed(a, b, what):
    """Bit-exact equality of two (f, s, phi, codes) tuples."""
    for name, x, y in zip(("f", "s", "phi", "codes"), a, b):
        x = np.ascontiguousarray(x)
        y = np.ascontiguousarray(y)
        if x.dtype == np.float64:
            bad = np.flatnonzero(x.view(np.uint64).ravel() != y.view(np.uint64).ravel())
        else:
            bad = np.flatnonzero(x.ravel() != y.ravel())
        assert bad.size == 0, f"{what}: {name} differs at {bad[:10]}: {x.ravel()[bad[:3]]} vs {y.ravel()[bad[:3]]}"


def assert_blocks_close(gpu, orc, rel=DECOMP_REL, what="decompress"):
    """Block-normwise closeness of two dense matrices (multiples of 8)."""
    r, c = orc.shape
    g4 = gpu.reshape(r // 8, 8, c // 8, 8)
    o4 = orc.reshape(r // 8, 8, c // 8, 8)
    err = np.abs(g4 - o4).max(axis=(1, 3))
    scale = np.abs(o4).max(axis=(1, 3))
    ok = err <= rel * scale
    if not ok.all():
        I, J = np.nonzero(~ok)
        raise AssertionError(f"{what}: {len(I)} blocks off, e.g. ({I[0]},{J[0]}) err {err[I[0], J[0]]:.3e} "
                             f"scale {scale[I[0], J[0]]:.3e}")


def assert_dots_close(gpu, orc, mag, rel=DOT_REL, what="dot"):
    """|gpu - orc| <= rel * mag elementwise, mag = sum |x_k y_k|."""
    gpu, orc, mag = np.asarray(gpu), np.asarray(orc), np.asarray(mag)
    ok = np.abs(gpu - orc) <= rel * mag
    if not ok.all():
        i = np.flatnonzero(~ok)
        raise AssertionError(f"{what}: {len(i)} results off, e.g. #{i[0]}: {gpu[i[0]]!r} vs {orc[i[0]]!r} "
                             f"(scale {mag[i[0]]:.3e})")
