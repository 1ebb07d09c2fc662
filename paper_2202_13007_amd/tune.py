"""Autotuner for the launch shapes the library exposes.

Three knobs are tuned by timing the candidates on the device and caching the
winner per (GPU architecture, operation, size class) in a JSON file:

* the output tile of the matmul contraction (``blaz_matmul_tiled``: 64 or
  128), per precision, B form and size class (powers of two of m*n and k);
* the number of persistent workgroups of a batch run (``blaz_batch_run``)
  and, jointly with it,
* the chunks a wave claims per pop of the work counter (1, 2 or 4, i.e.
  64, 128 or 256 blocks per claim), both per size class of the work queue
  (powers of two of the chunk count).

Every candidate computes the same result (the tile does not change the
summation order; the grid and the claim size only change which workgroup
takes which chunk), so tuning never changes numbers, only time.
"""
from __future__ import annotations

import json
import math
import os
import threading

import torch

from . import api

_DEFAULT_PATH = os.path.join(os.path.expanduser("~"), ".cache", "blaz", "tune.json")


def _pow2_class(x: int) -> int:
    return 0 if x <= 1 else int(math.ceil(math.log2(x)))


class Autotuner:
    """Cache of tuned choices; ``path=None`` keeps it in memory only."""

    MATMUL_TILES = (64, 128)
    WG_PER_CU = (2, 4, 8, 16)
    CHUNKS_PER_CLAIM = (1, 2, 4)

    def __init__(self, path: str | None = _DEFAULT_PATH, reps: int = 3):
        self.path = path
        self.reps = reps
        self._lock = threading.Lock()
        self.cache: dict[str, int] = {}
        if path and os.path.exists(path):
            try:
                with open(path) as fh:
                    self.cache = {k: int(v) for k, v in json.load(fh).items()}
            except (OSError, ValueError):
                self.cache = {}
        props = torch.cuda.get_device_properties(torch.cuda.current_device())
        self.arch = getattr(props, "gcnArchName", props.name).split(":")[0]
        self.cus = props.multi_processor_count

    def _save(self):
        if not self.path:
            return
        os.makedirs(os.path.dirname(self.path), exist_ok=True)
        tmp = self.path + f".tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(self.cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def _time(self, fn) -> float:
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(self.reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            best = min(best, a.elapsed_time(b))
        return best

    # -- matmul tile ----------------------------------------------------------
    def matmul_key(self, m: int, n: int, k: int, prec: str, b_compressed: bool) -> str:
        return f"{self.arch}|matmul|{prec}|{'cb' if b_compressed else 'db'}|mn{_pow2_class(m * n)}|k{_pow2_class(k)}"

    def matmul_tile(self, m: int, n: int, k: int, prec: str = "fp64", b_compressed: bool = False) -> int:
        key = self.matmul_key(m, n, k, prec, b_compressed)
        with self._lock:
            if key in self.cache:
                return self.cache[key]
        # representative square-ish operands of this class
        dev = torch.device("cuda")
        a = api.compress(torch.randn((m, k), dtype=torch.float64, device=dev))
        b = (api.compress(torch.randn((k, n), dtype=torch.float64, device=dev)) if b_compressed
             else torch.randn((k, n), dtype=torch.float64, device=dev))
        out = torch.empty((m, n), dtype=torch.float64, device=dev)
        ws = torch.empty(max(1, api.matmul_workspace_bytes(m, n, k, b_compressed, prec)), dtype=torch.uint8,
                         device=dev)
        times = {t: self._time(lambda t=t: api.matmul(a, b, out=out, prec=prec, workspace=ws, tile=t))
                 for t in self.MATMUL_TILES}
        best = min(times, key=times.get)
        with self._lock:
            self.cache[key] = best
            self._save()
        return best

    # -- persistent grid ------------------------------------------------------
    # Queues of more chunks than this share one size class: the synthetic
    # batch a class is tuned on is capped at this size anyway.
    BATCH_MAX_CLASS = 14

    def batch_key(self, total_chunks: int) -> str:
        return f"{self.arch}|batch|chunks{min(_pow2_class(total_chunks), self.BATCH_MAX_CLASS)}"

    def batch_launch(self, total_chunks: int) -> tuple[int, int]:
        """(workgroups, chunks per claim) for a batch run whose queue holds
        total_chunks chunks, tuned jointly on a synthetic batch of that size
        class (compressions of a random matrix, one 64-block chunk per block
        row of 512 columns)."""
        key = self.batch_key(total_chunks)
        with self._lock:
            if key + "|wg" in self.cache and key + "|claim" in self.cache:
                return self.cache[key + "|wg"], self.cache[key + "|claim"]
        chunks = 1 << min(_pow2_class(max(total_chunks, 1)), self.BATCH_MAX_CLASS)
        dev = torch.device("cuda")
        dense = torch.randn((8 * chunks, 512), dtype=torch.float64, device=dev)
        out = api.BlazMatrix.empty(8 * chunks, 512, dev)
        plan = api.Batch().compress(dense, out).plan(dev)
        times = {(w * self.cus, c): self._time(lambda w=w, c=c: plan.run(w * self.cus, c))
                 for w in self.WG_PER_CU for c in self.CHUNKS_PER_CLAIM}
        best = min(times, key=times.get)
        with self._lock:
            self.cache[key + "|wg"], self.cache[key + "|claim"] = best
            self._save()
        return best

    def batch_workgroups(self, total_chunks: int) -> int:
        """The tuned workgroup count alone (see batch_launch)."""
        return self.batch_launch(total_chunks)[0]
