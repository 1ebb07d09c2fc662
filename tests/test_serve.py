"""Serving loop: continuous batching with HBM-budget admission.

GPU tests check that every request's result is the same alone and in the
mix (bit for bit: the batched paths run the same device code), that a tiny
budget forces queueing without exceeding it, and that a request larger than
the budget is refused before anything runs.  The CPU test checks the
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


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_results_same_alone_and_in_the_mix(prec):
    import torch
    from paper_2202_13007_amd.serve import OperandPool, Server
    from paper_2202_13007_amd.tune import Autotuner
    A, B = _setup()
    reqs = make_requests(300, rate=20000.0, seed=11, n_min=8, n_max=512)
    pool = OperandPool(A, B, [r.n for r in reqs])
    srv = Server(pool, hbm_budget=1 << 30, matmul_prec=prec, tuner=Autotuner(path=None), keep_results=True)
    srv.prepare(reqs)
    rep = srv.run(reqs, "batched")
    assert rep["requests"] == 300 and rep["ticks"] < 300  # requests were batched together
    for r in reqs:
        assert np.isfinite(r.done) and r.done >= r.arrival
        assert _same(r.result, _alone(pool, r, prec)), (r.rid, r.op, r.n)
    torch.cuda.synchronize()


@pytest.mark.gpu
def test_tiny_budget_forces_queueing():
    from paper_2202_13007_amd.serve import OperandPool, Server, output_bytes
    A, B = _setup(256)
    reqs = make_requests(120, rate=50000.0, seed=12, n_min=8, n_max=256)
    biggest = max(output_bytes(r.op, r.n, "fp64") for r in reqs)
    pool = OperandPool(A, B, [r.n for r in reqs])
    srv = Server(pool, hbm_budget=biggest, keep_results=True)
    rep = srv.run(reqs, "batched")
    assert srv.peak_used <= biggest
    # every request is admitted in exactly one tick and a tick admits at most
    # the budget, whatever the timing
    need = -(-sum(output_bytes(r.op, r.n, "fp64") for r in reqs) // biggest)
    assert need > 1
    assert rep["ticks"] >= need
    for r in reqs:
        assert _same(r.result, _alone(pool, r, "fp64")), (r.rid, r.op, r.n)


@pytest.mark.gpu
def test_plain_form_matches_too_and_oversized_request_is_refused():
    from paper_2202_13007_amd.serve import OperandPool, Server, output_bytes
    A, B = _setup(256)
    reqs = make_requests(40, rate=50000.0, seed=13, n_min=8, n_max=256)
    pool = OperandPool(A, B, [r.n for r in reqs])
    srv = Server(pool, keep_results=True)
    srv.run(reqs, "plain")
    for r in reqs:
        assert _same(r.result, _alone(pool, r, "fp64")), (r.rid, r.op, r.n)
    small = Server(pool, hbm_budget=min(output_bytes(r.op, r.n, "fp64") for r in reqs) - 1)
    with pytest.raises(ValueError):
        small.run(reqs, "batched")
