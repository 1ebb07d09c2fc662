"""Grouped binary64 products: many products in at most three launches.

CPU tests cover the host-only planner (validation with blaz_matmul's rules,
workspace sizing, launch counts, dropped empty products).  GPU tests check
every product of a group of uneven sizes (compressed and dense B, k = 0,
both tile classes) against the oracle (within 1e-12 sum |x y|) and bit for
bit against blaz_matmul alone, also when the run is captured in a HIP graph
and replayed.
"""
import ctypes

import numpy as np
import pytest

from synth import smooth_field, uniform_matrix


def _lib():
    import os
    from paper_2202_13007_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2202_13007_amd import _build
        _build.build()
    return L


def fake_matrix(rows, cols, base, lines=0):
    L = _lib()
    nb = (rows // 8) * (cols // 8)
    return L.BlazMatrixC(rows, cols, base, base + 8 * nb + 64, base + 16 * nb + 128,
                         base + (17 * nb + 256 + 15) // 16 * 16, lines)


def item(a, b=None, bdense=0, n=0, ldb=0, c=0, ldc=0, tile=64):
    L = _lib()
    it = L.MatmulItemC()
    it.a = a
    it.b = b if b is not None else L.BlazMatrixC(0, 0, None, None, None, None, 0)
    it.bdense = bdense or None
    it.n, it.ldb, it.c, it.ldc, it.tile, it.reserved = n, ldb, c or None, ldc, tile, 0
    return it


def plan(items, ws=0, ws_bytes=0):
    L = _lib()
    n = len(items)
    arr = (L.MatmulItemC * max(n, 1))(*items)
    nbytes = L.lib().blaz_matmul_group_plan_bytes(n)
    buf = (ctypes.c_uint8 * max(nbytes, 8))()
    info = L.MatmulGroupInfoC()
    st = L.lib().blaz_matmul_group_plan(ctypes.cast(arr, ctypes.c_void_p), n, ws or None, ws_bytes,
                                        ctypes.cast(buf, ctypes.c_void_p), max(nbytes, 8), ctypes.byref(info))
    return st, info


def products():
    return [
        item(fake_matrix(136, 200, 0x1000000), fake_matrix(200, 72, 0x2000000), n=72, c=0x3000000, ldc=72),
        item(fake_matrix(264, 520, 0x4000000), bdense=0x5000000, n=64, ldb=64, c=0x6000000, ldc=64, tile=128),
        item(fake_matrix(0, 64, 0), bdense=0x7000000, n=8, ldb=8, c=0x7100000, ldc=8),       # m = 0: dropped
        item(fake_matrix(64, 0, 0x8000000), bdense=0, n=16, c=0x8100000, ldc=16),           # k = 0: zeros
    ]


def test_plan_sizes_workspace_and_counts():
    st, info = plan(products())
    assert st == -7  # BLAZ_ERR_WORKSPACE until a workspace is given
    need = (136 * 200 * 8 + 255) // 256 * 256 + (200 * 72 * 8 + 255) // 256 * 256 + 264 * 520 * 8
    assert info.workspace_bytes == need
    st, info = plan(products(), ws=0x10000000, ws_bytes=need)
    assert st == 0
    assert info.rebuild_jobs == 3                       # A and B of the first, A of the second
    assert info.rebuild_waves == (17 * 25 + 63) // 64 + (25 * 9 + 63) // 64 + (33 * 65 + 63) // 64
    assert (info.items128, info.items64) == (1, 2)      # the k = 0 product keeps its tile class
    assert info.workgroups128 == 3 * 1                  # 264 x 64 on 128 tiles
    assert info.workgroups64 == 8 + 1                   # 3 x 2 tiles, then the k = 0 product at tile 8
    assert info.plan_bytes > 0


@pytest.mark.parametrize("change,status", [
    (dict(reserved=1), -5),
    (dict(tile=96), -5),
    (dict(n=64), -3),                  # B has 72 columns
    (dict(c=0), -1),
    (dict(ldc=64), -2),                # ldc < n
    (dict(c=0x3000004), -4),
    (dict(c=0x1000000), -5),           # C overlaps A
])
def test_plan_rejects_invalid_product_and_reports_its_index(change, status):
    items = products()
    for k, v in change.items():
        setattr(items[0], k, v)
    st, info = plan(items, ws=0x10000000, ws_bytes=1 << 30)
    assert st == status and info.rebuild_jobs == 0


def test_plan_rejects_other_rates_and_both_forms_of_b():
    items = products()
    items[0].a = fake_matrix(136, 200, 0x1000000, lines=3)
    assert plan(items, ws=0x10000000, ws_bytes=1 << 30)[0] == -6
    items = products()
    items[1].b = fake_matrix(520, 64, 0x9000000)       # dense and compressed B
    st, info = plan(items, ws=0x10000000, ws_bytes=1 << 30)
    assert st == -5 and info.rebuild_jobs == 1


def test_plan_rejects_workspace_overlapping_an_output():
    st, info = plan(products())
    st, info = plan(products(), ws=0x3000000 - 256, ws_bytes=info.workspace_bytes)
    assert st == -5


def test_plan_rejects_an_output_over_another_products_operands_or_output():
    """The products run concurrently: one product's C over another's A, B
    (compressed or dense) or C is refused, naming the later product; products
    sharing an operand are fine."""
    ws = dict(ws=0x10000000, ws_bytes=1 << 30)
    base = products()
    for target in (0x1000000 + 8, 0x2000000, 0x5000000 + 64, 0x6000000 + 8):  # A0, B0, dense B1, C1
        items = products()
        items.append(item(fake_matrix(8, 8, 0xA000000), bdense=0xB000000, n=8, ldb=8, c=target, ldc=8))
        st, info = plan(items, **ws)
        assert st == -5 and info.rebuild_jobs == len(items) - 1, (hex(target), st, info.rebuild_jobs)
    # a later product reading the first product's output is refused as well
    items = products()
    items.append(item(fake_matrix(8, 8, 0xA000000), bdense=0x3000000, n=8, ldb=8, c=0xC000000, ldc=8))
    st, info = plan(items, **ws)
    assert st == -5 and info.rebuild_jobs == len(items) - 1
    # shared operands: the same A and dense B in two products with their own outputs
    items = products()
    items.append(item(base[1].a, bdense=0x5000000, n=64, ldb=64, c=0xD000000, ldc=64, tile=128))
    assert plan(items, **ws)[0] == 0


# --------------------------------------------------------------------------
# GPU: every product against the oracle and against blaz_matmul alone
# --------------------------------------------------------------------------

def make_group(torch, blaz):
    import oracle
    shapes = [  # (m, k, n, compressed B, tile)
        (8, 8, 8, True, 0), (136, 200, 72, True, 0), (264, 520, 64, False, 0), (64, 64, 64, True, 128),
        (1032, 528, 136, True, 0), (392, 136, 264, False, 128), (64, 0, 16, False, 0), (512, 256, 512, True, 0),
    ]
    grp = blaz.MatmulGroup()
    cases = []
    for i, (m, k, n, bc, tile) in enumerate(shapes):
        oa = oracle.compress(smooth_field(m, 4, 2.0, 1e-3, 870 + i, cols=k))
        a = blaz.BlazMatrix.from_host(m, k, oa.f, oa.s, oa.phi, oa.codes)
        if bc:
            ob = oracle.compress(smooth_field(k, 4, 2.0, 1e-3, 880 + i, cols=n))
            b = blaz.BlazMatrix.from_host(k, n, ob.f, ob.s, ob.phi, ob.codes)
            Bd = oracle.decompress(ob)
        else:
            Bd = uniform_matrix(k, n, 890 + i)
            b = torch.from_numpy(Bd).cuda() if k > 0 else torch.empty((0, n), dtype=torch.float64, device="cuda")
        out = torch.full((m, n), np.nan, dtype=torch.float64, device="cuda")
        grp.add(a, b, out, tile=tile)
        Ad = oracle.decompress(oa)
        cases.append((a, b, out, oracle.gemm(Ad, Bd), np.abs(Ad) @ np.abs(Bd), (m, k, n, bc)))
    return grp, cases


def check_cases(torch, blaz, cases):
    from oracle.parity import assert_dots_close
    for a, b, out, want, mag, what in cases:
        got = out.cpu().numpy()
        assert_dots_close(got, want, mag, what=f"group product {what}")
        alone = blaz.matmul(a, b)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int64), alone.view(torch.int64)), what


@pytest.mark.gpu
def test_group_matches_oracle_and_standalone():
    import torch
    import paper_2202_13007_amd as blaz
    grp, cases = make_group(torch, blaz)
    P = grp.plan()
    P.run()
    torch.cuda.synchronize()
    check_cases(torch, blaz, cases)
    # a second run of the same plan gives the same bits
    first = [c[2].clone() for c in cases]
    for c in cases:
        c[2].fill_(np.nan)
    P.run()
    torch.cuda.synchronize()
    for c, f in zip(cases, first):
        assert torch.equal(c[2].view(torch.int64), f.view(torch.int64))


@pytest.mark.gpu
def test_group_graph_capture_replays():
    """A run is at most three kernel launches (no memset, copy or
    allocation), so a captured graph replays it; every replay is checked
    after the outputs are cleared eagerly."""
    import torch
    import paper_2202_13007_amd as blaz
    grp, cases = make_group(torch, blaz)
    P = grp.plan()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        P.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.run()
    for _ in range(3):
        for c in cases:
            c[2].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check_cases(torch, blaz, cases)
