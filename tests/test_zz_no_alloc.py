"""The product without a caller workspace: blaz_matmul_static takes its
workspace from the library's static scratch array and allocates nothing.

Its results are compared with blaz_matmul's (the entry point with a caller
workspace, which the parity tests hold to the oracle) bit for bit, and with
the oracle under the parity rules, on two calls in a row, the second with a
smaller input (the array keeps the first call's contents); at the largest
size the array holds; and replayed from a captured graph.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2202_13007_amd as blaz
from oracle.parity import DOT_REL, assert_dots_close, low_precision_tol
from synth import smooth_field, uniform_matrix

pytestmark = pytest.mark.gpu


def up(c):
    return blaz.BlazMatrix.from_host(c.rows, c.cols, c.f, c.s, c.phi, c.codes)


def same_bits(a, b):
    return torch.equal(a.view(torch.int64), b.view(torch.int64))


@pytest.mark.parametrize("bform", ["compressed", "dense"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_static_matches_workspace_entry_point_twice(prec, bform):
    for m, k, n, seed in ((392, 264, 200, 1), (64, 72, 40, 2)):
        ox = oracle.compress(smooth_field(m, 6, 3.0, 1e-3, 810 + seed, cols=k))
        if bform == "compressed":
            oy = oracle.compress(smooth_field(k, 6, 3.0, 1e-3, 820 + seed, cols=n))
            B, Bd = up(oy), oracle.decompress(oy)
        else:
            Bd = uniform_matrix(k, n, 830 + seed)
            B = torch.from_numpy(Bd).cuda()
        x = up(ox)
        out = torch.full((m, n), np.nan, dtype=torch.float64, device="cuda")
        blaz.matmul_static(x, B, out=out, prec=prec)
        ref = blaz.matmul(x, B, prec=prec)
        torch.cuda.synchronize()
        assert same_bits(out, ref), (prec, bform, m, k, n)
        Xd = oracle.decompress(ox)
        rel = DOT_REL if prec == "fp64" else low_precision_tol(prec, k)
        assert_dots_close(out.cpu().numpy(), oracle.gemm(Xd, Bd), np.abs(Xd) @ np.abs(Bd), rel=rel,
                          what=f"matmul_static {prec} {bform} {m}x{k}x{n}")


def test_static_largest_product_then_smaller():
    """4096 x 4096 x 4096 with both operands compressed in binary64 needs the
    whole array (two 128 MiB rebuilds); then a small product."""
    n = 4096
    assert blaz.matmul_workspace_bytes(n, n, n, True, "fp64") == blaz.api.STATIC_SCRATCH_BYTES
    x = blaz.compress(torch.from_numpy(smooth_field(n, 8, 4.0, 1e-3, 840)).cuda())
    y = blaz.compress(torch.from_numpy(smooth_field(n, 8, 4.0, 1e-3, 841)).cuda())
    out = torch.empty((n, n), dtype=torch.float64, device="cuda")
    blaz.matmul_static(x, y, out=out)
    ref = blaz.matmul(x, y)
    torch.cuda.synchronize()
    assert same_bits(out, ref)
    small = blaz.compress(torch.from_numpy(smooth_field(64, 4, 2.0, 1e-3, 842)).cuda())
    o2 = torch.empty((64, 64), dtype=torch.float64, device="cuda")
    blaz.matmul_static(small, small, out=o2, prec="bf16x3")
    torch.cuda.synchronize()
    assert same_bits(o2, blaz.matmul(small, small, prec="bf16x3"))


def test_static_product_too_large_is_refused():
    """A product whose workspace exceeds the array is refused before
    anything runs (BLAZ_ERR_TOO_LARGE): 4096 x 4096 times a compressed
    4096 x 4104 needs 128 MiB + 128.25 MiB."""
    x = blaz.BlazMatrix.empty(4096, 4096)
    y = blaz.BlazMatrix.empty(4096, 4104)
    out = torch.empty((4096, 4104), dtype=torch.float64, device="cuda")
    with pytest.raises(blaz.BlazError) as e:
        blaz.matmul_static(x, y, out=out)
    assert e.value.status == -9


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_static_product_replays_from_a_graph(prec):
    """Captured after one eager call (which looks the array up), the call
    replays: each replay, after the output is cleared eagerly, gives the
    eager result bit for bit."""
    ox = oracle.compress(smooth_field(136, 4, 2.0, 1e-3, 850, cols=200))
    oy = oracle.compress(smooth_field(200, 4, 2.0, 1e-3, 851, cols=72))
    x, y = up(ox), up(oy)
    out = torch.empty((136, 72), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        blaz.matmul_static(x, y, out=out, prec=prec)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    want = out.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        blaz.matmul_static(x, y, out=out, prec=prec)
    for _ in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert same_bits(out, want)
