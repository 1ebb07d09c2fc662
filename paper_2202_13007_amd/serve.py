"""Continuous-batching serving loop over the libblaz entry points.

Requests -- compress, add, scale, dot and matmul on square n x n matrices --
arrive over time.  Their operands are compressed matrices resident on the
device (and, for compress, dense matrices resident in HBM).  Two forms:

* ``plain``: every request is launched on its own, with the standalone entry
  points, on one stream, as soon as it has arrived and its memory fits.
* ``batched``: continuous batching.  The server admits arrived requests while
  their outputs (and workspaces) fit an HBM budget, and on every tick turns
  the newly admitted block-level requests (compress, add, scale, dot) into
  one batch -- one persistent launch over a flat chunk queue -- on one
  stream, and launches the admitted matmuls on a few more streams (those
  that fill the GPU alone in order on one of them, the small ones
  round-robin on the others; with ``group_products`` and binary64
  contractions the tick's products of side <= 512 form one group -- one
  rebuild launch and one contraction launch per tile class for all of them),
  so the batch and the contractions overlap on the device.  A tick's batch
  (its request step) takes one of three forms, ``step``: ``fresh`` plans it
  into new buffers and runs it (a counter fill, a reset and the batch
  kernel); ``resident`` copies the plan and its counts into a resident plan
  buffer owned by the tick and launches the one-kernel resident run, which
  reads the counts on the device; ``graph`` does the same copy and replays a
  HIP graph captured for that buffer and launch shape.  Ticks do not wait for each other: up
  to ``max_inflight`` ticks run at once, and requests arriving meanwhile are
  admitted into the next tick as memory frees up.  The matmul contraction
  may run in FP64, FP32 or BF16x3 (``matmul_prec``).

Completion times come from events recorded after each request's work and
read against an event recorded when the run starts, so latency (completion
minus arrival) is on the device's clock, not the polling loop's.  Every
request's result is what the same standalone call computes alone: the
batched code paths run the same device code (tests check this bit for bit).
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api
from .trace import Range

OPS = ("compress", "add", "scale", "dot", "matmul")
SCALE_C = 1.7


@dataclass
class Request:
    rid: int
    op: str
    n: int
    arrival: float                  # seconds after the start of the run
    done: float = math.nan          # seconds after the start (device clock)
    nbytes: int = 0                 # device memory held while in flight
    cancelled: bool = False         # dropped from the queue past its deadline
    error: str | None = None        # why the request was rejected before running
    result: object = None
    _hold: list = field(default_factory=list, repr=False)


def make_requests(count: int, rate: float, seed: int = 501, n_min: int = 64, n_max: int = 8192,
                  mix=(0.30, 0.25, 0.15, 0.15, 0.15)) -> list[Request]:
    """Poisson arrivals (exponential gaps of mean 1/rate seconds), sides
    log-uniform in [n_min, n_max] rounded to multiples of 8, operations drawn
    with probabilities `mix` over (compress, add, scale, dot, matmul)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count) if rate > 0 else np.zeros(count)
    t = np.cumsum(gaps) - gaps[0]
    n = 8 * np.maximum(1, np.round(np.exp(rng.uniform(np.log(n_min), np.log(n_max), count)) / 8)).astype(int)
    n = np.clip(n, n_min, n_max)
    ops = rng.choice(len(OPS), size=count, p=np.asarray(mix) / np.sum(mix))
    return [Request(i, OPS[o], int(s), float(a)) for i, (o, s, a) in enumerate(zip(ops, n, t))]


class OperandPool:
    """Resident operands: for every side n, the n x n top-left corner of two
    dense fields (views with the fields' leading dimension) and their
    compressed forms, plus index vectors 0..n-1 for the dot requests."""

    def __init__(self, A: torch.Tensor, B: torch.Tensor, sides):
        self.A, self.B = A, B
        self.x, self.y, self.idx = {}, {}, {}
        for n in sorted(set(sides)):
            self.x[n] = api.compress(A[:n, :n])
            self.y[n] = api.compress(B[:n, :n])
            self.idx[n] = torch.arange(n, dtype=torch.int64, device=A.device)
        torch.cuda.synchronize()

    def dense(self, n):
        return self.A[:n, :n]


def output_bytes(op: str, n: int, matmul_prec: str) -> int:
    nb = (n // 8) ** 2
    if op in ("compress", "add", "scale"):
        return 45 * nb
    if op == "dot":
        return 8 * n
    return 8 * n * n + api.matmul_workspace_bytes(n, n, n, True, matmul_prec)


def fp64_equiv_bytes(op: str, n: int) -> int:
    """Bytes the same request moves on dense binary64 matrices."""
    return {"compress": 8, "add": 24, "scale": 16, "dot": 16, "matmul": 24}[op] * n * n


class Server:
    def __init__(self, pool: OperandPool, hbm_budget: int = 16 << 30, matmul_prec: str = "fp64",
                 max_inflight: int = 4, tuner=None, keep_results: bool = False, matmul_streams: int = 4,
                 group_products: bool = False, step: str = "resident", trace: bool = False):
        if step not in ("fresh", "resident", "graph"):
            raise ValueError(f"unknown request-step form {step!r}")
        self.pool = pool
        self.step = step
        self.trace = trace  # a roctx range around each tick's launches
        self.group_products = group_products
        self.budget = int(hbm_budget)
        self.matmul_prec = matmul_prec
        self.max_inflight = max_inflight
        self.tuner = tuner
        self.keep = keep_results
        self.s_block = torch.cuda.Stream()
        # Contractions that fill the GPU on their own (at least one 128 x 128
        # output tile per compute unit) run in order on the first matmul
        # stream -- side by side they would only contend; smaller ones go
        # round-robin over the others so that a handful of workgroups each
        # can share the GPU.
        self.s_mm = [torch.cuda.Stream() for _ in range(max(2, matmul_streams))]
        self._next_mm = 0
        self.cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
        # one resident plan buffer per tick that can be in flight; a tick
        # takes a free one and gives it back when its batch has completed
        self._slots = [api.ResidentBatch(self.SLOT_ITEMS) for _ in range(max_inflight)] if step != "fresh" else []
        self._free_slots = list(range(len(self._slots)))

    # -- per-request work ------------------------------------------------------
    def _alloc(self, r: Request):
        n = r.n
        if r.op in ("compress", "add", "scale"):
            r.result = api.BlazMatrix.empty(n, n)
        elif r.op == "dot":
            r.result = torch.empty(n, dtype=torch.float64, device="cuda")
        else:
            r.result = torch.empty((n, n), dtype=torch.float64, device="cuda")
            ws = api.matmul_workspace_bytes(n, n, n, True, self.matmul_prec)
            r._hold.append(torch.empty(max(ws, 1), dtype=torch.uint8, device="cuda"))

    def _standalone(self, r: Request):
        p, n = self.pool, r.n
        if r.op == "compress":
            api.compress(p.dense(n), out=r.result)
        elif r.op == "add":
            api.add(p.x[n], p.y[n], out=r.result)
        elif r.op == "scale":
            api.scale(p.x[n], SCALE_C, out=r.result)
        elif r.op == "dot":
            api.dot(p.x[n], p.idx[n], p.y[n], p.idx[n], out=r.result)
        else:
            tile = self.tuner.matmul_tile(n, n, n, self.matmul_prec, True) if self.tuner else 0
            api.matmul(p.x[n], p.y[n], out=r.result, prec=self.matmul_prec, workspace=r._hold[0], tile=tile)

    def _add_to_batch(self, batch: api.Batch, r: Request):
        p, n = self.pool, r.n
        if r.op == "compress":
            batch.compress(p.dense(n), r.result)
        elif r.op == "add":
            batch.add(p.x[n], p.y[n], r.result)
        elif r.op == "scale":
            batch.scale(p.x[n], SCALE_C, r.result)
        else:
            batch.dot(p.x[n], p.idx[n], p.y[n], p.idx[n], r.result)

    # -- the loop -----------------------------------------------------------------
    def prepare(self, requests: list[Request]):
        """Tune every size class the run will meet before it starts (tuning
        times kernels and would otherwise stall the loop)."""
        if self.tuner:
            for n in sorted({r.n for r in requests if r.op == "matmul"}):
                self.tuner.matmul_tile(n, n, n, self.matmul_prec, True)
            for c in range(0, self.tuner.BATCH_MAX_CLASS + 1):  # every class a tick can meet
                self.tuner.batch_launch(1 << c)
        if self.step == "graph":  # capture the graphs of every launch shape up front
            shapes = {self._resident_shape(1 << c) for c in range(0, 21)}
            with torch.cuda.stream(self.s_block):
                for rb in self._slots:
                    for wg, claim in sorted(shapes):
                        rb.graph(wg, claim)
            torch.cuda.synchronize()

    def _resident_shape(self, total_chunks: int):
        """Launch shape of a resident run: the tuned one, with the grid cut
        to the chunk count's power-of-two class (the run does not trim its
        grid, whose waves beyond the queue only exit, and a captured grid is
        fixed), so at most twice the needed waves are launched."""
        wg, claim = self.tuner.batch_launch(total_chunks) if self.tuner else (8 * self.cus, 0)
        cls = 1 << max(0, int(total_chunks - 1).bit_length())
        return min(wg, cls), claim

    def run(self, requests: list[Request], mode: str = "batched", deadline_ms: float | None = None) -> dict:
        """Serve `requests` (arrival times relative to the start).  With
        `deadline_ms`, a request still queued (arrived, not admitted) that
        long after its arrival is cancelled: it is dropped without running,
        marked `cancelled`, and left out of the latency figures; admitted
        requests always run to completion, and the loop goes on.  A request
        that cannot run -- an unknown operation, a side that is not a
        positive multiple of 8, or an output larger than the whole budget --
        is rejected before anything is launched (its `error` says why) and
        the others are served."""
        assert mode in ("plain", "batched")
        deadline = None if deadline_ms is None else deadline_ms / 1e3
        valid = []
        for r in requests:
            r.cancelled, r.done, r.error = False, math.nan, None
            if r.op not in OPS:
                r.error = f"unknown operation {r.op!r}"
            elif not isinstance(r.n, int) or r.n <= 0 or r.n % 8:
                r.error = f"side {r.n} is not a positive multiple of 8"
            else:
                r.nbytes = output_bytes(r.op, r.n, self.matmul_prec)
                if r.nbytes > self.budget:
                    r.error = f"needs {r.nbytes} bytes, more than the whole budget of {self.budget}"
            if r.error is None:
                valid.append(r)
            else:
                r.result = None
        limit = self.max_inflight if mode == "batched" else 1 << 30
        pending = deque(sorted(valid, key=lambda r: r.arrival))
        ready: deque[Request] = deque()
        units: list = []               # (event, [requests], held objects): one per launch unit
        ticks_inflight: dict = {}      # tick id -> units still running
        used = 0
        self.peak_used = 0
        ndone = 0
        ticks = 0
        # The device clock starts when start_ev executes; the host clock is read
        # only after that, so device-clock completion times are never early
        # with respect to host-clock arrivals (latency is over-estimated by the
        # few microseconds the synchronization takes, never under-estimated).
        start_ev = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start_ev.record(self.s_block)
        for st in self.s_mm:
            st.wait_stream(self.s_block)
        start_ev.synchronize()
        t0 = time.perf_counter()

        def complete_ready():
            nonlocal used, ndone, units
            still, progressed = [], False
            for ev, reqs, held, tick in units:
                if not ev.query():
                    still.append((ev, reqs, held, tick))
                    continue
                for h in held:
                    if isinstance(h, int):  # a resident plan buffer, free again
                        self._free_slots.append(h)
                t_done = start_ev.elapsed_time(ev) / 1e3
                for r in reqs:
                    r.done = t_done
                    used -= r.nbytes
                    r._hold.clear()
                    if not self.keep:
                        r.result = None
                ndone += len(reqs)
                ticks_inflight[tick] -= 1
                if ticks_inflight[tick] == 0:
                    del ticks_inflight[tick]
                progressed = True
            units = still
            return progressed

        while ndone < len(valid):
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                ready.append(pending.popleft())
            progressed = complete_ready()
            # the queue is in arrival order: the first request within its
            # deadline ends the cancellations
            while deadline is not None and ready and now - ready[0].arrival > deadline:
                r = ready.popleft()
                r.cancelled = True
                r.result = None
                ndone += 1
                progressed = True
            if ready and len(ticks_inflight) < limit and used + ready[0].nbytes <= self.budget:
                admitted = []
                while ready and used + ready[0].nbytes <= self.budget and (mode == "batched" or not admitted):
                    r = ready.popleft()
                    used += r.nbytes
                    self._alloc(r)
                    admitted.append(r)
                self.peak_used = max(self.peak_used, used)
                if self.trace:
                    with Range(f"tick {ticks}: {len(admitted)} requests, "
                               f"{sum(r.op == 'matmul' for r in admitted)} matmul"):
                        new_units = self._launch(admitted, mode)
                else:
                    new_units = self._launch(admitted, mode)
                ticks_inflight[ticks] = len(new_units)
                units.extend((ev, reqs, held, ticks) for ev, reqs, held in new_units)
                ticks += 1
                continue
            if not progressed:
                # Nothing to launch.  Poll without sleeping while requests wait
                # for memory or a tick slot, or an arrival is due within
                # SPIN_S (a sleep overshoots by tens of microseconds, which
                # would land on those requests' latency); otherwise sleep
                # until SPIN_S before the next arrival, 200 us at a time.
                wait = pending[0].arrival - now if pending else math.inf
                if not ready and wait > self.SPIN_S:
                    time.sleep(min(wait - self.SPIN_S, 2e-4))
        torch.cuda.synchronize()
        return self._report(requests, mode, ticks)

    def _launch(self, admitted, mode):
        """Enqueue the admitted requests; returns their completion units."""
        units = []
        if mode == "plain":
            with torch.cuda.stream(self.s_block):
                for r in admitted:
                    self._standalone(r)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(self.s_block)
                    units.append((ev, [r], []))
            return units
        blocks = [r for r in admitted if r.op != "matmul"]
        mms = [r for r in admitted if r.op == "matmul"]
        if blocks:
            batch = api.Batch()
            for r in blocks:
                self._add_to_batch(batch, r)
            with torch.cuda.stream(self.s_block):
                if self._slots and len(blocks) <= self.SLOT_ITEMS:
                    # the tick's plan into its resident buffer, then one launch
                    # or one graph replay
                    slot = self._free_slots.pop()
                    rb = self._slots[slot]
                    _, total = rb.load(batch)
                    shape = self._resident_shape(total)
                    if self.step == "graph":
                        rb.graph(*shape).replay()
                    else:
                        rb.run(*shape)
                    held = [slot, batch]
                else:
                    plan = batch.plan()
                    wg, claim = self.tuner.batch_launch(plan.total_chunks) if self.tuner else (0, 0)
                    plan.run(wg, claim)
                    held = [plan]
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(self.s_block)
            units.append((ev, blocks, held))
        tiny = [r for r in mms if r.n <= self.GROUP_MAX_SIDE]
        if self.group_products and self.matmul_prec == "fp64" and len(tiny) > 1:
            # the tick's small binary64 products as one group: one rebuild
            # launch and one contraction launch per tile class for all of them
            grp = api.MatmulGroup()
            for r in tiny:
                grp.add(self.pool.x[r.n], self.pool.y[r.n], r.result)
            st = self.s_mm[1 + self._next_mm % (len(self.s_mm) - 1)]
            self._next_mm += 1
            with torch.cuda.stream(st):
                plan = grp.plan(workspace=self._group_workspace(tiny))
                plan.run()
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(st)
            units.append((ev, tiny, [plan]))
            mms = [r for r in mms if r.n > self.GROUP_MAX_SIDE]
        for r in mms:
            if ((r.n + 127) // 128) ** 2 >= self.cus:
                st = self.s_mm[0]
            else:
                st = self.s_mm[1 + self._next_mm % (len(self.s_mm) - 1)]
                self._next_mm += 1
            with torch.cuda.stream(st):
                self._standalone(r)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(st)
            units.append((ev, [r], []))
        return units

    GROUP_MAX_SIDE = 512  # products grouped per tick: those whose launch costs more than their work
    SLOT_ITEMS = 2048     # block-level requests per resident tick (larger ticks run a fresh plan)
    SPIN_S = 1e-3         # poll without sleeping when the next arrival is this close

    @staticmethod
    def _group_workspace(reqs):
        """The group's rebuilt operands live in the workspaces the requests
        were admitted with; one tensor of their summed size (each request's
        workspace is at least its rebuilds' size) is taken for the group."""
        need = sum(api.matmul_workspace_bytes(r.n, r.n, r.n, True, "fp64") for r in reqs)
        for r in reqs:
            r._hold.clear()
        return torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")

    def _report(self, requests, mode, ticks) -> dict:
        served = [r for r in requests if not r.cancelled and r.error is None]
        lat = np.array([(r.done - r.arrival) * 1e3 for r in served]) if served else np.zeros(1)
        first = min((r.arrival for r in requests), default=0.0)
        last = max((r.done for r in served), default=first)
        span = max(last - first, 1e-9)
        eq = sum(fp64_equiv_bytes(r.op, r.n) for r in served)
        flop = sum(2 * r.n ** 3 for r in served if r.op == "matmul")
        return {"mode": mode, "requests": len(requests), "served": len(served),
                "cancelled": sum(r.cancelled for r in requests),
                "rejected": sum(r.error is not None for r in requests), "ticks": ticks,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "makespan_s": span, "req_per_s": len(served) / span,
                "fp64_equiv_GBps": eq / span / 1e9, "matmul_TFLOPs": flop / span / 1e12,
                "matmul_prec": self.matmul_prec}
