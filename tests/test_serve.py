"""Serving loop: continuous batching with HBM-budget admission.

GPU tests check every request's result against the FP64 oracle under the
parity rules (the resident operands are the oracle's records, uploaded), and
that it is the same alone and in the mix (bit for bit: the batched paths run
the same device code); that a tiny
budget forces queueing without exceeding it, that queued requests past a
deadline are cancelled while the loop keeps serving the rest, and that
requests that cannot run (larger than the budget, a side that is not a
multiple of 8, an unknown operation) are rejected before anything runs
while the others are served.  The CPU test checks the
request generator."""
import numpy as np
import pytest

from paper_2202_13007_amd.serve import OPS, make_requests


def test_request_generator():
    reqs = make_requests(20000, rate=1000.0, seed=501)
    n = np.array([r.n for r in reqs])
    assert np.all(n % 8 == 0) and n.min() >= 64 and n.max() <= 8192
    # log-uniform sides: about half the mass below the geometric mean 724
    assert 0.45 < np.mean(n < 724) < 0.55
    ops = np.array([OPS.index(r.op) for r in reqs])
    share = np.bincount(ops, minlength=5) / len(reqs)
    np.testing.assert_allclose(share, [0.30, 0.25, 0.15, 0.15, 0.15], atol=0.015)
    t = np.array([r.arrival for r in reqs])
    assert t[0] == 0 and np.all(np.diff(t) >= 0)
    assert abs(np.mean(np.diff(t)) - 1e-3) < 5e-5
    again = make_requests(20000, rate=1000.0, seed=501)
    assert [(r.op, r.n, r.arrival) for r in again] == [(r.op, r.n, r.arrival) for r in reqs]


def _setup(n_base=512):
    import torch
    from synth import smooth_field
    A = torch.from_numpy(smooth_field(n_base, 8, 4.0, 1e-3, 700)).cuda()
    B = torch.from_numpy(smooth_field(n_base, 8, 4.0, 1e-3, 701)).cuda()
    return A, B


def _alone(pool, r, prec):
    import paper_2202_13007_amd as blaz
    from paper_2202_13007_amd.serve import SCALE_C
    n = r.n
    if r.op == "compress":
        return blaz.compress(pool.dense(n))
    if r.op == "add":
        return blaz.add(pool.x[n], pool.y[n])
    if r.op == "scale":
        return blaz.scale(pool.x[n], SCALE_C)
    if r.op == "dot":
        return blaz.dot(pool.x[n], pool.idx[n], pool.y[n], pool.idx[n])
    return blaz.matmul(pool.x[n], pool.y[n], prec=prec)


def _same(a, b):
    import torch
    if isinstance(a, torch.Tensor):
        return torch.equal(a.view(torch.int64), b.view(torch.int64))
    return all(torch.equal(getattr(a, k).view(torch.uint8), getattr(b, k).view(torch.uint8))
               for k in ("f", "s", "phi", "codes"))


class OracleOperands:
    """The oracle's side of the serving pool: for every side n, the oracle's
    compressions of the n x n corners of the two fields.  The server's
    resident operands are replaced by uploads of these records, so that both
    sides start from the same inputs and no oracle input comes from the GPU."""

    def __init__(self, pool, sides):
        import oracle
        import paper_2202_13007_amd as blaz
        self.A = pool.A.cpu().numpy()
        self.B = pool.B.cpu().numpy()
        self.x, self.y, self.cache = {}, {}, {}
        for n in sorted(set(sides)):
            self.x[n] = oracle.compress(self.A[:n, :n])
            self.y[n] = oracle.compress(self.B[:n, :n])
            for o, side in ((self.x[n], pool.x), (self.y[n], pool.y)):
                side[n] = blaz.BlazMatrix.from_host(n, n, o.f, o.s, o.phi, o.codes)

    def check(self, r, got, prec):
        """The request's result against the oracle, under the parity rules
        (a low-precision product under its FP32-accumulation bound)."""
        import oracle
        from oracle.parity import (DOT_REL, TIE_RATE_MAX, assert_dots_close, assert_same_compressed,
                                   compare_compressed, low_precision_tol)
        from paper_2202_13007_amd.serve import SCALE_C
        n = r.n
        what = f"request {r.rid} {r.op} n={n}"
        key = (r.op, n)
        if r.op == "compress":
            if key not in self.cache:
                self.cache[key] = oracle.compress(self.A[:n, :n], with_debug=True)
            o, (_, code_x, phi_x) = self.cache[key]
            ties = compare_compressed(got.to_host(), (o.f, o.s, o.phi, o.codes), code_x, phi_x, what)
            assert ties <= TIE_RATE_MAX * (o.codes.size + len(o.phi)), (what, ties)
        elif r.op in ("add", "scale"):
            if key not in self.cache:
                self.cache[key] = (oracle.add(self.x[n], self.y[n]) if r.op == "add"
                                   else oracle.scale(self.x[n], SCALE_C))
            o = self.cache[key]
            assert_same_compressed(got.to_host(), (o.f, o.s, o.phi, o.codes), what)
        else:
            if ("dense", n) not in self.cache:
                self.cache[("dense", n)] = (oracle.decompress(self.x[n]), oracle.decompress(self.y[n]))
            Xd, Yd = self.cache[("dense", n)]
            if r.op == "dot":
                idx = np.arange(n)
                want = oracle.dot(self.x[n], idx, self.y[n], idx)
                mag = np.einsum("ij,ji->i", np.abs(Xd), np.abs(Yd))
                assert_dots_close(got.cpu().numpy(), want, mag, what=what)
            else:
                if key not in self.cache:
                    self.cache[key] = (oracle.gemm(Xd, Yd), np.abs(Xd) @ np.abs(Yd))
                want, mag = self.cache[key]
                rel = DOT_REL if prec == "fp64" else low_precision_tol(prec, n)
                assert_dots_close(got.cpu().numpy(), want, mag, rel=rel, what=f"{what} {prec}")


@pytest.mark.gpu
@pytest.mark.parametrize("prec,group,step", [("fp64", False, "fresh"), ("fp64", True, "graph"),
                                             ("fp64", False, "resident"), ("bf16x3", False, "resident")])
def test_results_same_alone_and_in_the_mix(prec, group, step):
    """Every request of a 300-request mix (sides 8..512, arriving faster than
    they are served, so ticks batch many of them and the batch and the
    contractions overlap; with `group` each tick's products run as one
    grouped launch; each tick's batch a fresh plan, a resident plan buffer's
    one-kernel run, or a replay of a graph captured on that buffer) matches
    the oracle under the parity rules, and equals the same request run alone
    bit for bit."""
    import torch
    from paper_2202_13007_amd.serve import OperandPool, Server
    from paper_2202_13007_amd.tune import Autotuner
    A, B = _setup()
    reqs = make_requests(300, rate=20000.0, seed=11, n_min=8, n_max=512)
    pool = OperandPool(A, B, [r.n for r in reqs])
    orc = OracleOperands(pool, [r.n for r in reqs])
    srv = Server(pool, hbm_budget=1 << 30, matmul_prec=prec, tuner=Autotuner(path=None), keep_results=True,
                 group_products=group, step=step)
    srv.prepare(reqs)
    rep = srv.run(reqs, "batched")
    print(f"{prec} group={group} step={step}: {rep['ticks']} ticks for 300 requests")
    assert rep["requests"] == 300 and rep["ticks"] < 300  # requests were batched together
    for r in reqs:
        assert np.isfinite(r.done) and r.done >= r.arrival
        orc.check(r, r.result, prec)
        assert _same(r.result, _alone(pool, r, prec)), (r.rid, r.op, r.n)
    torch.cuda.synchronize()


@pytest.mark.gpu
def test_tiny_budget_forces_queueing():
    from paper_2202_13007_amd.serve import OperandPool, Server, output_bytes
    A, B = _setup(256)
    reqs = make_requests(120, rate=50000.0, seed=12, n_min=8, n_max=256)
    biggest = max(output_bytes(r.op, r.n, "fp64") for r in reqs)
    pool = OperandPool(A, B, [r.n for r in reqs])
    orc = OracleOperands(pool, [r.n for r in reqs])
    srv = Server(pool, hbm_budget=biggest, keep_results=True, step="graph")
    srv.prepare(reqs)
    rep = srv.run(reqs, "batched")
    assert srv.peak_used <= biggest
    # every request is admitted in exactly one tick and a tick admits at most
    # the budget, whatever the timing
    need = -(-sum(output_bytes(r.op, r.n, "fp64") for r in reqs) // biggest)
    assert need > 1
    assert rep["ticks"] >= need
    for r in reqs:
        orc.check(r, r.result, "fp64")
        assert _same(r.result, _alone(pool, r, "fp64")), (r.rid, r.op, r.n)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_queued_requests_past_their_deadline_are_cancelled(mode):
    """200 requests arrive 20 us apart on average, faster than they are
    served within a budget of the largest one, with a 0.2 ms deadline:
    requests still queued past the deadline are dropped, the loop keeps
    serving later arrivals, and every request it did run matches the oracle
    (and its run alone)."""
    from paper_2202_13007_amd.serve import OperandPool, Server, output_bytes
    A, B = _setup(256)
    reqs = make_requests(200, rate=50000.0, seed=14, n_min=8, n_max=256)
    biggest = max(output_bytes(r.op, r.n, "fp64") for r in reqs)
    pool = OperandPool(A, B, [r.n for r in reqs])
    orc = OracleOperands(pool, [r.n for r in reqs])
    srv = Server(pool, hbm_budget=biggest, keep_results=True)
    rep = srv.run(reqs, mode, deadline_ms=0.2)
    served = [r for r in reqs if not r.cancelled]
    print(f"{mode}: {rep['served']} served, {rep['cancelled']} cancelled, {rep['ticks']} ticks")
    assert rep["served"] == len(served) >= 1 and rep["cancelled"] >= 1
    assert rep["served"] + rep["cancelled"] == len(reqs)
    assert srv.peak_used <= biggest
    first_cancel = min(r.arrival for r in reqs if r.cancelled)
    assert any(r.arrival > first_cancel for r in served)  # served after a cancellation
    for r in reqs:
        if r.cancelled:
            assert r.result is None and np.isnan(r.done)
        else:
            assert np.isfinite(r.done) and r.done >= r.arrival
            orc.check(r, r.result, "fp64")
            assert _same(r.result, _alone(pool, r, "fp64")), (r.rid, r.op, r.n)


@pytest.mark.gpu
def test_plain_form_matches_too_and_oversized_request_is_refused():
    from paper_2202_13007_amd.serve import OperandPool, Server, output_bytes
    A, B = _setup(256)
    reqs = make_requests(40, rate=50000.0, seed=13, n_min=8, n_max=256)
    pool = OperandPool(A, B, [r.n for r in reqs])
    orc = OracleOperands(pool, [r.n for r in reqs])
    srv = Server(pool, keep_results=True)
    srv.run(reqs, "plain")
    for r in reqs:
        orc.check(r, r.result, "fp64")
        assert _same(r.result, _alone(pool, r, "fp64")), (r.rid, r.op, r.n)
    small = Server(pool, hbm_budget=min(output_bytes(r.op, r.n, "fp64") for r in reqs) - 1)
    rep = small.run(reqs, "batched")
    assert rep["rejected"] == len(reqs) and rep["served"] == 0 and rep["ticks"] == 0
    assert all(r.result is None and "budget" in r.error for r in reqs)


@pytest.mark.gpu
def test_bad_requests_are_rejected_and_the_rest_served():
    """A side that is not a multiple of 8, an unknown operation and an
    empty side, mixed into a stream: each is rejected with its reason before
    anything runs, and every other request is served and matches the
    oracle."""
    from paper_2202_13007_amd.serve import OperandPool, Request, Server
    A, B = _setup(256)
    good = make_requests(60, rate=20000.0, seed=15, n_min=8, n_max=256)
    bad = [Request(1000, "compress", 12, 0.0005), Request(1001, "bogus", 64, 0.0010), Request(1002, "add", 0, 0.0)]
    pool = OperandPool(A, B, [r.n for r in good])
    orc = OracleOperands(pool, [r.n for r in good])
    srv = Server(pool, keep_results=True)
    rep = srv.run(good + bad, "batched")
    assert rep["rejected"] == 3 and rep["served"] == len(good)
    assert "multiple of 8" in bad[0].error and "unknown operation" in bad[1].error and "multiple of 8" in bad[2].error
    for r in good:
        assert r.error is None and np.isfinite(r.done)
        orc.check(r, r.result, "fp64")
