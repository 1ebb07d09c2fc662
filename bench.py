#!/usr/bin/env python3
"""Benchmark of the blaz hot path on one MI355X.

Workload: two 8192x8192 binary64 smooth fields (16 seeded sinusoids of at
most 8 cycles per side, amplitude U[0.5, 2], + N(0, 1e-3) noise), resident in
HBM.  One step = compress both, add the compressed matrices (Algorithm 1),
scale the sum by 1.7 (Algorithm 2, out of place), decompress the result.

value = FP64-equivalent bytes of the step / step time: the bytes the same
operations move on dense binary64 matrices (compress and decompress 8 n^2
each, add 3 * 8 n^2, scale 2 * 8 n^2; 64 n^2 per step).

The JSON line also carries, per operation, the time and the actual and
FP64-equivalent GB/s inside the step; the same operations on dense FP64 on
this GPU ("plain"); the roofline of the dominant kernel (compress) from HIP
events on its stream; each operation launched alone with a cold and a warm
Infinity Cache; the 64x64 latencies, eager and graph-replayed; the 4096^2
linear algebra (compressed field times dense U[-1, 1] in FP64, FP32 and
BF16x3, and 4096 row dot products); the 16384^2 mixed-precision transform
(codes against the FP64 path, errors against the field); the serving mix at
three loads; and the CPU oracle timed on a bounded sample of the step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix
RECORD = 45                    # compressed bytes per block
BLOCK = 512                    # dense bytes per block


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=8192, help="matrix side (default: the 8192 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-matmul", action="store_true", help="skip the matmul leg")
    ap.add_argument("--cpu-rows", type=int, default=768, help="rows of each field the oracle times")
    ap.add_argument("--serve-requests", type=int, default=20000, help="requests of the serving mix (0 skips it)")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0, help="HBM budget of the serving loop")
    ap.add_argument("--serve-trace", action="store_true",
                    help="a roctx range around every serving tick (for rocprofv3 --marker-trace)")
    ap.add_argument("--serve-step", default="resident", choices=("fresh", "resident", "graph"),
                    help="form of the batched serving loop's request step: a fresh plan, a resident plan buffer "
                         "and one launch, or a resident buffer and a graph replay")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 64x64 latency, cold-cache, tunable-rate and 16384x16384 mixed-precision legs")
    ap.add_argument("--only", default="",
                    help="comma-separated legs to run after the step (cold, rates, transform, serving, latency, "
                         "matmul, mixed, cpu; dots runs the dot products of the matmul leg alone); default: every "
                         "leg the other flags leave on")
    args = ap.parse_args()
    args.legs = {"cold", "rates", "transform", "serving", "latency", "matmul", "mixed", "cpu"}
    if args.only:
        args.legs = (args.legs | {"dots"}) & set(args.only.split(","))
    if args.no_extra:
        args.legs -= {"cold", "rates", "transform", "latency", "mixed"}
    if args.no_matmul:
        args.legs.discard("matmul")
    if args.no_cpu_baseline:
        args.legs.discard("cpu")
    if args.serve_requests <= 0:
        args.legs.discard("serving")
    return args


def elapsed_ms(pairs):
    return [a.elapsed_time(b) for a, b in pairs]


def timed_each(torch, fn, reps, warm=3, flush=None):
    """Sorted per-launch times in ms, from an event pair around each launch.
    With `flush` (a 1 GiB tensor), the buffer is read before every launch,
    outside the timed pair, so that operands come from HBM and not from the
    256 MB Infinity Cache.  A read leaves only clean lines behind; a write
    would leave dirty ones whose write-back lands inside the timed launch."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    pairs = []
    for _ in range(reps):
        if flush is not None:
            flush.sum()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        pairs.append((a, b))
    torch.cuda.synchronize()
    return sorted(elapsed_ms(pairs))


def median(xs):
    return xs[len(xs) // 2]


CODEC_SOURCES = ("paper_2202_13007_amd/csrc/codec.hip", "paper_2202_13007_amd/csrc/blaz_codec.hpp",
                 "paper_2202_13007_amd/csrc/blaz_device.hpp")


def sources_sha256(paths):
    """SHA-256 over the named source files, concatenated in order."""
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(kernel: str, sources):
    """HBM bytes per launch measured with rocprofv3 counters, if the kernel's
    sources are unchanged since the measurement."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(kernel)
    if not rec or rec.get("sources") != list(sources):
        return None
    if rec.get("sources_sha256") != sources_sha256(sources):
        return None
    return rec.get("bytes_per_launch")


def host_identity():
    """Threads the oracle may use (the process's CPU affinity, capped by
    OMP_NUM_THREADS when that is set) and the CPU model string."""
    import subprocess
    cores = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(cores, int(env)) if env.isdigit() and int(env) > 0 else cores
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        model = next((ln.split(":", 1)[1].strip() for ln in out.splitlines() if ln.startswith("Model name")), "")
    except (OSError, subprocess.SubprocessError):
        pass
    if not model and os.path.exists("/proc/cpuinfo"):
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    return cores, threads, model


def oracle_step(oracle, a, b):
    """The step on the oracle: compress both, add, scale by 1.7, decompress."""
    x = oracle.compress(a)
    y = oracle.compress(b)
    w = oracle.scale(oracle.add(x, y), 1.7)
    oracle.decompress(w)
    return x, y


def cpu_baseline(A, B, rows, workload_inputs, band=64, queries=128):
    """The oracle (plain C, FP64, one block at a time) timed on this host on
    bounded samples of the workloads, single-threaded and with its block loops
    on every allowed core: the step on the first `rows` rows of both 8192^2
    fields (FP64-equivalent GB/s, as `value`), a band of rows of the 4096^3
    product (decompress the band of A, then the i-k-j product; `band` rows
    single-threaded, 8x as many on all cores) and a set of the 4096 row dot
    products with their own vectors (`queries`, 8x as many on all cores).
    Returns the report and the oracle's records of the step sample (for
    parity)."""
    import oracle

    cores, threads, model = host_identity()
    a = np.ascontiguousarray(A[:rows])
    b = np.ascontiguousarray(B[:rows])
    n2 = a.shape[0] * a.shape[1]
    Am, Bm, Vm = workload_inputs("linalg-4096")
    n = Am.shape[0]
    res = {}
    recs = None
    for name, t, scale in (("single_thread", 1, 1), ("all_cores", threads, 8)):
        nb_rows, nq = band * scale, queries * scale
        xa = oracle.compress(np.ascontiguousarray(Am[:nb_rows]))
        xr = oracle.compress(np.ascontiguousarray(Am[: 8 * ((nq + 7) // 8)]))
        qrows = np.arange(nq)
        V = np.ascontiguousarray(Vm[:nq])
        oracle.set_threads(t)
        t0 = time.perf_counter()
        out = oracle_step(oracle, a, b)
        dt = time.perf_counter() - t0
        recs = recs or out
        t1 = time.perf_counter()
        oracle.gemm(oracle.decompress(xa), Bm)
        dm = time.perf_counter() - t1
        t2 = time.perf_counter()
        oracle.dot_dense(xr, qrows, V, n)
        dd = time.perf_counter() - t2
        res[name] = {"threads": t, "step_GBps_fp64_equiv": round(64.0 * n2 / dt / 1e9, 4), "step_s": round(dt, 2),
                     "matmul_band_rows": nb_rows, "matmul_GFLOPs": round(2.0 * nb_rows * n * n / dm / 1e9, 3),
                     "matmul_s": round(dm, 2), "dots": nq,
                     "dots_GBps": round((45 * (n // 8) + 8 * n + 16) * nq / dd / 1e9, 4), "dots_s": round(dd, 2)}
    oracle.set_threads(threads)
    return {
        "value": res["all_cores"]["step_GBps_fp64_equiv"],
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"step (compress x2, add, scale 1.7, decompress) on the first {rows} rows of both fields "
                  f"({a.shape[0]}x{a.shape[1]}, {n2 // 64} blocks each); 4096^3 product on a band of rows "
                  f"(decompress + i-k-j); a set of the 4096 row dots with own vectors; value = the step on all "
                  f"cores",
        "host_cores": cores,
        "model": model,
        **res,
    }, recs


def parity_report(A, B, gx, gy, ox, oy):
    """The GPU's records of the step against the oracle's on the oracle's
    sample (a prefix of block rows): f and s bit-exact, phi and codes
    bit-exact except classified rounding-boundary ties, whose count and rate
    per code are reported (the rate must stay under 1e-6)."""
    import oracle
    from oracle.parity import TIE_RATE_MAX, compare_compressed

    rep = {"blocks": 0, "codes": 0, "ties": 0, "f_s_exact": True, "ok": True}
    try:
        for M, g, o in ((A, gx, ox), (B, gy, oy)):
            nb = o.nblk
            gf = g.f[:nb].cpu().numpy()
            gs = g.s[:nb].cpu().numpy()
            gphi = g.phi[:nb].cpu().numpy()
            gc = g.codes[:nb].cpu().numpy()
            exact = (np.array_equal(gf.view(np.uint64), o.f.view(np.uint64))
                     and np.array_equal(gs.view(np.uint64), o.s.view(np.uint64)))
            rep["f_s_exact"] = rep["f_s_exact"] and exact
            diff = np.flatnonzero((gphi != o.phi) | np.any(gc != o.codes, axis=1))
            if diff.size:
                _, _, _, _, code_x, phi_x = oracle.compress_blocks(M, diff)
                rep["ties"] += compare_compressed((gf[diff], gs[diff], gphi[diff], gc[diff]),
                                                  (o.f[diff], o.s[diff], o.phi[diff], o.codes[diff]),
                                                  code_x, phi_x, "bench sample")
            rep["blocks"] += nb
            rep["codes"] += 29 * nb
    except AssertionError as e:
        rep["ok"] = False
        rep["error"] = str(e)[:300]
    rep["tie_rate"] = float(f"{rep['ties'] / max(rep['codes'], 1):.3e}")
    rep["ok"] = rep["ok"] and rep["f_s_exact"] and rep["tie_rate"] < TIE_RATE_MAX
    rep["rule"] = ("f, s bit-exact; phi and 28 codes per block bit-exact except rounding-boundary ties "
                   "(oracle value within 2^-40 of an integer, results 1 apart); codes = 29 per block")
    return rep


def matmul_leg(blaz, torch, workload_inputs):
    """Compressed 4096^2 field A times dense U[-1, 1] B in FP64, FP32 and
    BF16x3, against torch's FP64 product of the decompressed A ("plain").
    Errors: each precision against the FP64 path (relative Frobenius), and the
    method's own error, |A_hat B - A B| / |A B| with A the uncompressed field."""
    Am, Bm, Vm = workload_inputs("linalg-4096")
    n = Am.shape[0]
    dA = torch.from_numpy(Am).cuda()
    g = blaz.compress(dA)
    dB = torch.from_numpy(Bm).cuda()
    ws = torch.empty(max(blaz.matmul_workspace_bytes(n, n, n, False, p) for p in ("fp64", "fp32", "bf16x3")),
                     dtype=torch.uint8, device="cuda")
    Ad = blaz.decompress(g)
    outs = {p: torch.empty((n, n), dtype=torch.float64, device="cuda") for p in ("fp64", "fp32", "bf16x3", "plain")}
    legs = {}
    runs = [(p, (lambda p=p: blaz.matmul(g, dB, out=outs[p], prec=p, workspace=ws))) for p in ("fp64", "fp32", "bf16x3")]
    runs.append(("plain", lambda: torch.matmul(Ad, dB, out=outs["plain"])))
    # the vendor library's plain BF16 product (FP32 output) of the rounded
    # operands: the MFMA work rate a single BF16 GEMM reaches on this part
    aB, bB = Ad.to(torch.bfloat16).contiguous(), dB.to(torch.bfloat16).contiguous()
    runs.append(("vendor_bf16", lambda: torch.mm(aB, bB, out_dtype=torch.float32)))
    # and its FP32 GEMM (no reduced-precision inner products)
    tf32 = torch.backends.cuda.matmul.allow_tf32
    torch.backends.cuda.matmul.allow_tf32 = False
    aF, bF = Ad.float(), dB.float()
    runs.append(("vendor_fp32", lambda: torch.mm(aF, bF)))
    peaks = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3, "plain": 78.6, "vendor_bf16": 2500.0,
             "vendor_fp32": 157.3}
    # three interleaved rounds of 5 back-to-back launches per variant, median
    # round: the clock drifts with the power draw of FP64 matrix work, so a
    # fixed order would favour whichever variant runs in the better state
    per = {name: [] for name, _ in runs}
    for name, fn in runs:
        fn()
    torch.cuda.synchronize()
    for _ in range(3):
        for name, fn in runs:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(5):
                fn()
            b.record()
            torch.cuda.synchronize()
            per[name].append(a.elapsed_time(b) / 5)
    for name, _ in runs:
        ms = median(per[name])
        tf = 2 * n ** 3 / ms / 1e9
        legs[name] = {"ms": round(ms, 4), "TFLOPs": round(tf, 2), "mfma_frac": round(tf / peaks[name], 4),
                      "rounds_ms": [round(t, 4) for t in per[name]]}
    # the product recompressed (results kept in the 45-byte form)
    gB = blaz.compress(dB)
    wsc = torch.empty(max(blaz.matmul_compressed_workspace_bytes(n, n, n, True, p) for p in ("fp64", "bf16x3")),
                      dtype=torch.uint8, device="cuda")
    cout = blaz.BlazMatrix.empty(n, n)
    for p in ("fp64", "bf16x3"):
        ms = median(timed_each(torch, lambda p=p: blaz.matmul_compressed(g, gB, out=cout, prec=p, workspace=wsc), 5))
        dms = median(timed_each(torch, lambda p=p: blaz.matmul(g, gB, out=outs[p], prec=p, workspace=wsc), 5))
        legs[p]["compressed_output"] = {"ms": round(ms, 4), "dense_output_ms_same_operands": round(dms, 4),
                                        "what": "compressed A x compressed B, product recompressed"}
    del wsc, cout, gB
    for p in ("fp64", "bf16x3"):
        blaz.matmul(g, dB, out=outs[p], prec=p, workspace=ws)
    ref = outs["fp64"]
    nref = torch.linalg.norm(ref).item()
    for p in ("fp32", "bf16x3", "plain"):
        legs[p]["rel_err_vs_fp64"] = float(f"{torch.linalg.norm(outs[p] - ref).item() / nref:.3e}")
    exact = torch.matmul(dA, dB)
    method = torch.linalg.norm(ref - exact).item() / torch.linalg.norm(exact).item()
    legs["plain"]["what"] = "torch FP64 matmul of the decompressed A"
    legs["bf16x3"]["mfma_frac_note"] = "against 1/3 of the BF16 peak (three products)"
    legs["vendor_bf16"]["what"] = ("one BF16 x BF16 -> FP32 product of the rounded operands by the vendor library "
                                   "(torch.mm): the MFMA work rate of a plain BF16 GEMM, for reference")
    legs["bf16x3"]["mfma_work_vs_vendor_bf16"] = round(3 * legs["bf16x3"]["TFLOPs"] / legs["vendor_bf16"]["TFLOPs"], 4)
    legs["vendor_fp32"]["what"] = "the vendor library's FP32 GEMM (torch.mm, TF32 off) of the same operands in FP32"
    legs["fp32"]["vs_vendor_fp32"] = round(legs["fp32"]["TFLOPs"] / legs["vendor_fp32"]["TFLOPs"], 4)
    legs["fp64"]["vs_vendor_fp64"] = round(legs["fp64"]["TFLOPs"] / legs["plain"]["TFLOPs"], 4)
    torch.backends.cuda.matmul.allow_tf32 = tf32
    del outs, exact, ws, aB, bB, aF, bF
    return {"legs": legs, "method_rel_err": float(f"{method:.3e}"),
            "note": "TFLOPs count 2 n^3 useful flops; times include decompressing A and preparing B",
            "dots": dot_leg(blaz, torch, g, Ad, dB, torch.from_numpy(Vm).cuda())}


def dot_leg(blaz, torch, g, Ad, dB, dV, reps=20):
    """4096 dot products of compressed rows: row i of A with its own dense
    vector V[i] (algorithmic bytes: compressed A once + V + indices + out),
    with one shared vector (GEMV), and with column i of a compressed B
    (2 (n/8) records per dot).  'plain' is torch on the decompressed A."""
    n = Ad.shape[0]
    nblk = g.nblk
    rows = torch.arange(n, dtype=torch.int64, device="cuda")
    gb = blaz.compress(dB)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    tmp = torch.empty(n, dtype=torch.float64, device="cuda")
    v0 = dV[0].contiguous()
    cases = {
        "own_vectors": (lambda: blaz.dot_dense(g, rows, dV, out=out), RECORD * nblk + 8 * n * n + 16 * n,
                        lambda: torch.sum(Ad * dV, dim=1)),
        "shared_vector": (lambda: blaz.dot_dense(g, rows, v0, out=out), RECORD * nblk + 24 * n,
                          lambda: torch.mv(Ad, v0)),
        "compressed_pairs": (lambda: blaz.dot(g, rows, gb, rows, out=out), 2 * (n // 8) * RECORD * n + 24 * n,
                             lambda: torch.sum(Ad * blaz.decompress(gb).t(), dim=1)),
    }
    res = {"count": n, "length": n}
    for k, (fn, nbytes, want) in cases.items():
        ms = median(timed_each(torch, fn, reps))
        fn()
        w = want()
        scale = torch.max(torch.abs(w)).item()
        r = {"ms": round(ms, 5), "GBps": round(nbytes / ms / 1e6, 1),
             "max_abs_diff_vs_plain_rel": float(f"{torch.max(torch.abs(out - w)).item() / scale:.3e}")}
        if k != "compressed_pairs":
            pms = median(timed_each(torch, lambda: tmp.copy_(want()), reps))
            r["plain_ms"] = round(pms, 5)
        res[k] = r
    res["note"] = ("GBps = algorithmic bytes / time; compressed_pairs counts 2 (n/8) records per dot, "
                   "most of them served from cache")
    return res


def latency_leg(blaz, torch, workload_inputs, reps=50):
    """The 64x64 workload: per-operation latency (median of single launches)
    and the whole sequence -- compress both, add, scale by 1.7, decompress,
    dot of row 0 of A with column 0 of B, compressed x compressed matmul --
    launched eagerly and replayed from a captured graph."""
    A, B = workload_inputs("plain-64")
    n = A.shape[0]
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    x, y, z, w = (blaz.BlazMatrix.empty(n, n) for _ in range(4))
    D = torch.empty((n, n), dtype=torch.float64, device="cuda")
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    idx = torch.zeros(1, dtype=torch.int64, device="cuda")
    o = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(max(1, blaz.matmul_workspace_bytes(n, n, n, True, "fp64")), dtype=torch.uint8, device="cuda")
    ops = {"compress": lambda: blaz.compress(dA, out=x),
           "compress_y": lambda: blaz.compress(dB, out=y),
           "add": lambda: blaz.add(x, y, out=z),
           "scale": lambda: blaz.scale(z, 1.7, out=w),
           "decompress": lambda: blaz.decompress(w, out=D),
           "dot": lambda: blaz.dot(x, idx, y, idx, out=o),
           "matmul": lambda: blaz.matmul(x, y, out=C, workspace=ws)}

    def seq():
        for fn in ops.values():
            fn()

    out = {k: round(1e3 * median(timed_each(torch, fn, reps)), 2) for k, fn in ops.items() if k != "compress_y"}
    res = {"unit": "us", "per_op_median": out}
    res["sequence_eager_us"] = round(1e3 * median(timed_each(torch, seq, reps)), 2)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        seq()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        seq()
    res["sequence_graph_us"] = round(1e3 * median(timed_each(torch, g.replay, reps)), 2)
    res["note"] = "device time between events; the graph replays the same seven launches"
    return res


def cold_ops_leg(blaz, torch, dA, dB, reps=20):
    """Each operation of the step on its own, median of single launches, with
    the operands evicted from the Infinity Cache before every launch (cold)
    and without (warm); scale also in place (16 B read + 16 B written per
    block)."""
    n = dA.shape[0]
    x = blaz.compress(dA)
    y = blaz.compress(dB)
    z, w = blaz.BlazMatrix.empty(n, n), blaz.BlazMatrix.empty(n, n)
    blaz.add(x, y, out=z)
    D = torch.empty_like(dA)
    nblk = x.nblk
    flush = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")
    cases = {"compress": (lambda: blaz.compress(dA, out=w), (BLOCK + RECORD) * nblk),
             "decompress": (lambda: blaz.decompress(x, out=D), (BLOCK + RECORD) * nblk),
             "add": (lambda: blaz.add(x, y, out=w), 3 * RECORD * nblk),
             "scale": (lambda: blaz.scale(x, 1.7, out=w), 2 * RECORD * nblk),
             "scale_in_place": (lambda: blaz.scale(z, 1.0000001, out=z), 32 * nblk)}
    res = {}
    for k, (fn, nbytes) in cases.items():
        cold = median(timed_each(torch, fn, reps, flush=flush))
        warm = median(timed_each(torch, fn, reps))
        res[k] = {"cold_ms": round(cold, 5), "cold_GBps": round(nbytes / cold / 1e6, 1),
                  "cold_hbm_frac": round(nbytes / cold / 1e6 / HBM_PEAK_GBS, 4),
                  "warm_ms": round(warm, 5), "warm_GBps": round(nbytes / warm / 1e6, 1)}
    del flush
    return res


def rates_leg(blaz, torch, dA, reps=10):
    """The tunable rate on the first 8192^2 field: L kept lines of DCT
    coefficients (L = 2 is the paper's scheme).  Per L: bits per block, the
    median compress / decompress / add times, their GB/s over the bytes each
    moves, and the relative Frobenius error of the decoded field."""
    n = dA.shape[0]
    norm = torch.linalg.norm(dA).item()
    D = torch.empty_like(dA)
    res = {}
    for L in range(1, 9):
        rec = 17 + blaz.code_stride(L)
        x = blaz.compress(dA, lines=L)
        z = blaz.BlazMatrix.empty(n, n, lines=L)
        nblk = x.nblk
        tc = median(timed_each(torch, lambda: blaz.compress(dA, out=x), reps))
        td = median(timed_each(torch, lambda: blaz.decompress(x, out=D), reps))
        ta = median(timed_each(torch, lambda: blaz.add(x, x, out=z), reps))
        err = torch.linalg.norm(D - dA).item() / norm
        res[str(L)] = {"bits_per_block": 8 * rec, "ratio": round(4096 / (8 * rec), 3),
                       "compress_ms": round(tc, 4), "compress_GBps": round((BLOCK + rec) * nblk / tc / 1e6, 1),
                       "decompress_ms": round(td, 4), "decompress_GBps": round((BLOCK + rec) * nblk / td / 1e6, 1),
                       "add_ms": round(ta, 4), "add_GBps": round(3 * rec * nblk / ta / 1e6, 1),
                       "rel_err": float(f"{err:.4e}")}
        del x, z
    del D
    return res


def transform_input_leg(blaz, torch, dA, reps=10):
    """The two readings of the transform's input on the first 8192^2 field:
    the DCT of Delta' (the library's default) and the DCT of the predicted
    slopes (Psi's grid points).  Median times and GB/s of 557 B per block,
    the relative Frobenius error of each decoded field, the share of codes
    that differ between the readings, and compress with the Psi side output."""
    n = dA.shape[0]
    norm = torch.linalg.norm(dA).item()
    D = torch.empty_like(dA)
    xa, xb = blaz.BlazMatrix.empty(n, n), blaz.BlazMatrix.empty(n, n)
    psi = torch.empty((xa.nblk, 64), dtype=torch.uint8, device="cuda")
    nblk = xa.nblk
    res = {}
    for name, fn, out in (("delta_prime", lambda: blaz.compress(dA, out=xa), xa),
                          ("predicted_slopes", lambda: blaz.compress_predicted(dA, out=xb), xb)):
        t = median(timed_each(torch, fn, reps))
        blaz.decompress(out, out=D)
        err = torch.linalg.norm(D - dA).item() / norm
        res[name] = {"compress_ms": round(t, 4), "compress_GBps": round((BLOCK + 45) * nblk / t / 1e6, 1),
                     "rel_err": float(f"{err:.4e}")}
    tp = median(timed_each(torch, lambda: blaz.compress(dA, out=xa, psi=psi), reps))
    res["delta_prime"]["with_psi_ms"] = round(tp, 4)
    res["codes_differing"] = float(f"{(xa.codes != xb.codes).float().mean().item():.4e}")
    res["phi_differing"] = float(f"{(xa.phi != xb.phi).float().mean().item():.4e}")
    del D, xa, xb, psi
    return res


def mixed_leg(blaz, torch, workload_inputs, reps=10):
    """The 16384x16384 field compressed with the transform in FP64, FP32 and
    BF16x3.  Codes and phi are compared with the FP64 path's; errors of the
    decompressed matrices are relative Frobenius norms against the field
    itself (the method's own error for FP64) and against the FP64 path."""
    (M,) = workload_inputs("mixed-16384")
    n = M.shape[0]
    dM = torch.from_numpy(M).cuda()
    del M
    precs = ("fp64", "fp32", "bf16x3")
    outs = {p: blaz.BlazMatrix.empty(n, n) for p in precs}
    nblk = outs["fp64"].nblk
    res = {"n": n, "blocks": nblk, "codes": 28 * nblk}
    norm = torch.linalg.norm(dM).item()
    ref = outs["fp64"]
    D64 = None
    for p in precs:
        ms = median(timed_each(torch, lambda p=p: blaz.compress(dM, out=outs[p], prec=p), reps))
        r = {"ms": round(ms, 4), "GBps_actual": round((BLOCK + RECORD) * nblk / ms / 1e6, 1),
             "GBps_fp64_equiv": round(8 * n * n / ms / 1e6, 1)}
        D = blaz.decompress(outs[p])
        r["rel_err_vs_field"] = float(f"{torch.linalg.norm(D - dM).item() / norm:.4e}")
        if p == "fp64":
            D64 = D
        else:
            o = outs[p]
            r["f_s_identical"] = bool(torch.equal(o.f.view(torch.int64), ref.f.view(torch.int64))
                                      and torch.equal(o.s.view(torch.int64), ref.s.view(torch.int64)))
            r["code_mismatch_rate"] = float(f"{(o.codes != ref.codes).sum().item() / (28 * nblk):.3e}")
            r["phi_flip_rate"] = float(f"{(o.phi != ref.phi).sum().item() / nblk:.3e}")
            r["rel_err_vs_fp64_path"] = float(f"{torch.linalg.norm(D - D64).item() / norm:.4e}")
            del D
        res[p] = r
    res["note"] = ("mismatches are against the FP64 path, which the parity tests hold to the oracle "
                   "(bit-exact except boundary ties); rel_err_vs_field of fp64 is the method's own error")
    return res


def request_step_cost(torch, pool, ticks=400):
    """Host-inclusive cost of one tick's block-level request step, for a
    tick of one small request (scale of the smallest resident operand): a
    fresh plan (pinned staging, plan copy, counter fill, reset and batch
    kernels); a copy into a resident plan buffer plus one replay of the
    graph captured for it; the same copy plus the resident run launched
    directly (one kernel).  Four rotating outputs and buffers, one stream,
    synchronized at the end; the second of two passes counts."""
    import time
    from paper_2202_13007_amd import api
    n = min(pool.x)
    x = pool.x[n]
    outs = [api.BlazMatrix.empty(n, n) for _ in range(4)]
    slots = [api.ResidentBatch(16) for _ in range(4)]

    def fresh(i):
        api.Batch().scale(x, 1.7, outs[i % 4]).plan().run()

    def replay(i):
        rb = slots[i % 4]
        rb.load(api.Batch().scale(x, 1.7, outs[i % 4]))
        rb.graph(1, 1).replay()  # one chunk: one workgroup, as the fresh plan's run trims it

    def direct(i):
        rb = slots[i % 4]
        rb.load(api.Batch().scale(x, 1.7, outs[i % 4]))
        rb.run(1, 1)

    s = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(s):
        for rb in slots:
            rb.graph(1, 1)
        for name, f in (("fresh_plan_us", fresh), ("graph_replay_us", replay), ("resident_launch_us", direct)) * 2:
            for i in range(20):
                f(i)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(ticks):
                f(i)
            torch.cuda.synchronize()
            res[name] = round((time.perf_counter() - t0) / ticks * 1e6, 2)
    res["side"] = n
    res["note"] = "host-inclusive time per tick over a stream of one-request ticks"
    return res


def serving_leg(torch, dA, dB, count, budget_gib, loads=(0.5, 0.8, 1.2), step="resident", trace=False):
    """The serving mix: `count` requests (compress 30%, add 25%, scale 15%,
    dot 15%, matmul 15%), sides log-uniform in [64, 8192], on the two 8192^2
    fields (each side n uses their n x n corners).  The plain form's capacity
    is measured with every request of a calibration set arriving at once;
    the Poisson stream then arrives at 0.5x, 0.8x and 1.2x that rate and is
    served in the plain form, batched with FP64 matmuls (standalone, and
    with each tick's products of side <= 512 as one group), and batched with
    BF16x3 matmuls; `step` is the batched forms' request-step form (see
    paper_2202_13007_amd.serve)."""
    from paper_2202_13007_amd.serve import OperandPool, Server, make_requests
    from paper_2202_13007_amd.tune import Autotuner

    calib = make_requests(min(count, 2000), rate=0.0, seed=502)
    warm = make_requests(200, rate=0.0, seed=503)
    sides = [r.n for r in calib + warm + make_requests(count, rate=1.0, seed=501)]
    pool = OperandPool(dA, dB, sides)
    tuner = Autotuner(path=None)
    budget = int(budget_gib * (1 << 30))
    out = {"requests": count, "hbm_budget_GiB": budget_gib, "mix": "compress .30 add .25 scale .15 dot .15 matmul .15",
           "sides": "log-uniform in [64, 8192], multiples of 8"}
    out["request_step_form"] = step
    servers = {"plain": Server(pool, budget, "fp64", tuner=tuner, trace=trace),
               "batched_fp64": Server(pool, budget, "fp64", tuner=tuner, step=step, trace=trace),
               "batched_fp64_grouped": Server(pool, budget, "fp64", tuner=tuner, group_products=True, step=step,
                                              trace=trace),
               "batched_bf16x3": Server(pool, budget, "bf16x3", tuner=tuner, step=step, trace=trace)}
    for srv in servers.values():
        srv.prepare(calib)
    # warm-up and capacity (everything arrives at t = 0)
    cap = {}
    for name, srv in servers.items():
        mode = "plain" if name == "plain" else "batched"
        srv.run(make_requests(200, rate=0.0, seed=503), mode)  # warm-up (same sides as `warm`)
        # a capacity run is a handful of ticks, whose composition and timing
        # vary from run to run, and the first full-size run after the warm-up
        # still pays first-use costs: three runs, the best one counts
        cap[name] = max(srv.run(make_requests(len(calib), rate=0.0, seed=502), mode)["req_per_s"] for _ in range(3))
    out["capacity_req_per_s"] = {k: round(v, 1) for k, v in cap.items()}
    out["capacity_speedup_vs_plain"] = {k: round(v / cap["plain"], 3) for k, v in cap.items()}
    # How much of the plain form's device time the binary64 products take:
    # the calibration set's matmul requests alone, in the plain form.  Running
    # every other request concurrently with them can shorten the set by at
    # most the remaining share.
    t_all = len(calib) / cap["plain"]
    t_mm = min(servers["plain"].run([r for r in make_requests(len(calib), rate=0.0, seed=502)
                                     if r.op == "matmul"], "plain")["makespan_s"] for _ in range(2))
    mm = [r for r in calib if r.op == "matmul"]
    out["plain_fp64_matmul_share"] = {
        "matmul_requests": len(mm), "matmul_only_s": round(t_mm, 4), "all_requests_s": round(t_all, 4),
        "share": round(t_mm / t_all, 4), "max_gain_from_overlap": round(t_all / t_mm, 4),
        "note": "the calibration set's binary64 products alone in the plain form, against the whole set"}
    out["request_step"] = request_step_cost(torch, pool)
    out["runs"] = {}
    for load in loads:
        rate = load * cap["plain"]
        runs = {"arrival_rate_req_per_s": round(rate, 1)}
        for name, srv in servers.items():
            reqs = make_requests(count, rate=rate, seed=501)
            srv.prepare(reqs)
            rep = srv.run(reqs, "plain" if name == "plain" else "batched")
            runs[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.items()}
            print(f"# serving {load}x {name}: p50 {rep['p50_ms']:.2f} ms p99 {rep['p99_ms']:.2f} ms "
                  f"{rep['req_per_s']:.0f} req/s", file=sys.stderr, flush=True)
        out["runs"][f"{load}x_plain_capacity"] = runs
    return out


# ---------------------------------------------------------------------------
# Summaries of rocprofv3 output (CSV directories written with -d DIR -o run),
# printed as the text tables kept under profiles/.  CPU only.
# ---------------------------------------------------------------------------

def short_kernel_name(name: str) -> str:
    name = name[5:] if name.startswith("void ") else name
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):  # drop the parameter list (outside template brackets)
        depth += ch == "<"
        depth -= ch == ">"
        if ch == "(" and depth == 0:
            cut = i
            break
    name = name[:cut]
    if name.startswith("at::native::"):
        name = "torch " + name[len("at::native::"):]
    return name[:62]


def read_csv(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def summarize_trace(d):
    """Per (kernel, grid size in work-items, workgroup size): calls and the
    average, median, min and max duration from run_kernel_trace.csv."""
    groups = {}
    for r in read_csv(os.path.join(d, "run_kernel_trace.csv")):
        key = (short_kernel_name(r["Kernel_Name"]), int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]),
               int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"]))
        groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = [f"{'kernel':62s} {'grid':>9s} {'wg':>4s} {'calls':>6s} {'avg_us':>9s} {'median_us':>10s} {'min_us':>9s} "
             f"{'max_us':>9s}"]
    for (k, g, w), ts in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        ts = sorted(ts)
        lines.append(f"{k:62s} {g:9d} {w:4d} {len(ts):6d} {sum(ts) / len(ts):9.2f} {ts[len(ts) // 2]:10.2f} "
                     f"{ts[0]:9.2f} {ts[-1]:9.2f}")
    return "\n".join(lines)


def summarize_pmc(d):
    """Per (kernel, grid size): dispatches and each counter's average value."""
    groups = {}
    for r in read_csv(os.path.join(d, "run_counter_collection.csv")):
        key = (short_kernel_name(r["Kernel_Name"]), int(r["Grid_Size"]))
        groups.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    counters = sorted({c for v in groups.values() for c in v})
    lines = [f"{'kernel':62s} {'grid':>9s} {'n':>4s} " + " ".join(f"{c:>22s}" for c in counters)]
    for (k, g), v in sorted(groups.items()):
        n = max(len(x) for x in v.values())
        lines.append(f"{k:62s} {g:9d} {n:4d} " + " ".join(
            f"{sum(v[c]) / len(v[c]):22.4g}" if c in v else f"{'-':>22s}" for c in counters))
    return "\n".join(lines)


def summarize_pmc_runs(d, name):
    """Dispatches of kernels whose name contains `name`, cut into runs of
    consecutive dispatches (a dispatch of another kernel in between ends a
    run), with each counter's average per run: separates the cases of a
    leg that launch the same kernel with the same grid (the dot leg's own
    and shared vectors)."""
    rows = read_csv(os.path.join(d, "run_counter_collection.csv"))
    per = {}
    for r in rows:
        per.setdefault(int(r["Dispatch_Id"]), (r["Kernel_Name"], int(r["Grid_Size"]), {}))[2][r["Counter_Name"]] = \
            float(r["Counter_Value"])
    runs, cur = [], None
    for i in sorted(per):
        k, g, v = per[i]
        if name not in k:
            cur = None
            continue
        if cur is None or cur[0] != (short_kernel_name(k), g):
            cur = ((short_kernel_name(k), g), [])
            runs.append(cur)
        cur[1].append(v)
    counters = sorted({c for _, vs in runs for v in vs for c in v})
    lines = [f"{'run':>3s} {'kernel':40s} {'grid':>9s} {'n':>4s} " + " ".join(f"{c:>20s}" for c in counters)]
    for j, ((k, g), vs) in enumerate(runs):
        lines.append(f"{j:3d} {k[:40]:40s} {g:9d} {len(vs):4d} " + " ".join(
            f"{sum(v.get(c, 0.0) for v in vs) / len(vs):20.4g}" for c in counters))
    return "\n".join(lines)


def summarize_markers(d):
    """The serving loop's tick ranges (roctx, run_marker_api_trace.csv): host
    time to launch a tick, by the number of requests in it."""
    import re
    rows = read_csv(os.path.join(d, "run_marker_api_trace.csv"))
    buckets = {}
    for r in rows:
        m = re.match(r"tick \d+: (\d+) requests, (\d+) matmul", r["Function"])
        if not m:
            continue
        n = int(m.group(1))
        key = "1" if n == 1 else "2-9" if n < 10 else "10-99" if n < 100 else ">=100"
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        buckets.setdefault(key, []).append((us, n))
    lines = [f"{'requests per tick':>17s} {'ticks':>7s} {'median_us':>10s} {'p90_us':>9s} {'p99_us':>9s} "
             f"{'max_us':>9s} {'us_per_request':>14s}"]
    for key in ("1", "2-9", "10-99", ">=100"):
        if key not in buckets:
            continue
        v = sorted(u for u, _ in buckets[key])
        per = sum(u for u, _ in buckets[key]) / sum(n for _, n in buckets[key])
        lines.append(f"{key:>17s} {len(v):7d} {v[len(v) // 2]:10.1f} {v[int(0.9 * (len(v) - 1))]:9.1f} "
                     f"{v[int(0.99 * (len(v) - 1))]:9.1f} {v[-1]:9.1f} {per:14.1f}")
    return "\n".join(lines)


STEP_KERNELS = {  # kernel -> (sources, algorithmic bytes read, written per block) on the plain-8192 step
    "compress_f64_kernel": (CODEC_SOURCES, BLOCK, RECORD),
    "decompress_kernel": (CODEC_SOURCES, RECORD, BLOCK),
    "add_kernel": (("paper_2202_13007_amd/csrc/ops.hip", "paper_2202_13007_amd/csrc/blaz_ops.hpp"), 2 * RECORD, RECORD),
    "scale_kernel": (("paper_2202_13007_amd/csrc/ops.hip", "paper_2202_13007_amd/csrc/blaz_ops.hpp"), RECORD, RECORD),
}


def summarize_traffic(fetch_dir, write_dir, nblk=1 << 20, copy_bytes=1 << 29):
    """HBM bytes per dispatch of the step's kernels from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for the bench's plain copy of a 512 MiB matrix (copy_bytes each way).
    Writes profiles/traffic.json (bench.py fills `roofline.traffic` from it
    while the kernel's sources are unchanged) and returns the text table."""
    def per_kernel(d, counter):
        acc = {}
        for r in read_csv(os.path.join(d, "run_counter_collection.csv")):
            if r["Counter_Name"] != counter:
                continue
            name = short_kernel_name(r["Kernel_Name"])
            if int(r["Grid_Size"]) == 1048576 and name.startswith("blaz::"):
                base = name.split("::")[1].split("<")[0]
            elif "copyBuffer" in name:
                base = "copy"
            else:
                continue
            acc.setdefault(base, []).append(float(r["Counter_Value"]))
        # the run copies 512 MiB (the dense comparison) and 2 GiB (the copy
        # rate); the smaller copies are the calibration
        if "copy" in acc:
            small = min(acc["copy"])
            acc["copy"] = [v for v in acc["copy"] if v < 2 * small]
        return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}
    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    ff = copy_bytes / (fetch["copy"][0] * 1024)
    wf = copy_bytes / (write["copy"][0] * 1024)
    lines = [f"copy: FETCH_SIZE {fetch['copy'][0]:.0f} KiB, WRITE_SIZE {write['copy'][0]:.0f} KiB per dispatch for "
             f"{copy_bytes:,} B each way -> factors {ff:.4f}, {wf:.4f}"]
    rec = {}
    for k, (srcs, rd, wr) in STEP_KERNELS.items():
        if k not in fetch or k not in write:
            continue
        rb, wb = fetch[k][0] * 1024 * ff, write[k][0] * 1024 * wf
        alg = (rd + wr) * nblk
        rec[k] = {"workload": "plain-8192 (1,048,576 blocks)", "sources": list(srcs),
                  "sources_sha256": sources_sha256(srcs), "bytes_per_launch": int(round(rb + wb)),
                  "read_bytes": int(round(rb)), "write_bytes": int(round(wb)), "fetch_factor": round(ff, 5),
                  "write_factor": round(wf, 5), "dispatches": [fetch[k][1], write[k][1]]}
        lines.append(f"{k.split('_')[0]:11s} FETCH_SIZE {fetch[k][0]:10.1f} KiB x{ff:.4f} = {rb / 1e6:8.2f} MB "
                     f"(algorithmic {rd * nblk / 1e6:8.2f})   WRITE_SIZE {write[k][0]:10.1f} KiB x{wf:.4f} = "
                     f"{wb / 1e6:8.2f} MB (algorithmic {wr * nblk / 1e6:8.2f})   total/algorithmic "
                     f"{(rb + wb) / alg:.4f}")
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return "\n".join(lines)


def summarize_main(argv):
    """python bench.py --summarize {trace DIR | pmc DIR | pmc-runs DIR NAME | markers DIR |
    traffic FETCH_DIR WRITE_DIR}"""
    kind = argv[0] if argv else ""
    if kind == "trace":
        print(summarize_trace(argv[1]))
    elif kind == "pmc":
        print(summarize_pmc(argv[1]))
    elif kind == "pmc-runs":
        print(summarize_pmc_runs(argv[1], argv[2]))
    elif kind == "markers":
        print(summarize_markers(argv[1]))
    elif kind == "traffic":
        print(summarize_traffic(argv[1], argv[2]))
    else:
        raise SystemExit(summarize_main.__doc__)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize":
        summarize_main(sys.argv[2:])
        return
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the per-GPU shard is the measured unit; see the sharding notes).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2202_13007_amd as blaz
    from paper_2202_13007_amd import _lib
    from synth import workload_inputs

    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    n = args.n
    t_gen = time.time()
    A, B = workload_inputs("plain-8192", n=n)
    print(f"# inputs generated in {time.time() - t_gen:.1f} s", file=sys.stderr, flush=True)
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    x = blaz.BlazMatrix.empty(n, n)
    y = blaz.BlazMatrix.empty(n, n)
    z = blaz.BlazMatrix.empty(n, n)
    w = blaz.BlazMatrix.empty(n, n)
    D = torch.empty((n, n), dtype=torch.float64, device="cuda")
    nblk = x.nblk
    n2 = n * n

    ops = ("compress_x", "compress_y", "add", "scale", "decompress")
    ev = {k: [] for k in ops}

    def step(record):
        def timed(name, fn):
            if record:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                fn()
                b.record()
                ev[name].append((a, b))
            else:
                fn()
        timed("compress_x", lambda: blaz.compress(dA, out=x))
        timed("compress_y", lambda: blaz.compress(dB, out=y))
        timed("add", lambda: blaz.add(x, y, out=z))
        timed("scale", lambda: blaz.scale(z, 1.7, out=w))
        timed("decompress", lambda: blaz.decompress(w, out=D))

    def timed_steps(record):
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(args.steps):
            step(record)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / args.steps

    for _ in range(args.warmup):
        step(False)
    # The step time comes from a pass without per-operation events (an event
    # pair around each of the five launches adds about 10 % to the step);
    # the per-operation times and the roofline from a second timed pass with
    # an event pair around every launch, on the launching stream.
    ms_step = timed_steps(False)
    ms_step_instrumented = timed_steps(True)
    # The same five launches replayed from a captured graph (launch overhead
    # excluded); reported beside the eager step, which is `value`.
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(False)
    for _ in range(2):
        graph.replay()
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record()
    for _ in range(args.steps):
        graph.replay()
    g1.record()
    torch.cuda.synchronize()
    ms_step_graph = g0.elapsed_time(g1) / args.steps
    del graph

    per = {k: float(np.mean(elapsed_ms(v))) for k, v in ev.items()}
    bytes_actual = {"compress": (BLOCK + RECORD) * nblk, "add": 3 * RECORD * nblk,
                    "scale": 2 * RECORD * nblk, "decompress": (RECORD + BLOCK) * nblk}
    bytes_equiv = {"compress": 8 * n2, "add": 24 * n2, "scale": 16 * n2, "decompress": 8 * n2}
    op_report = {}
    for k, ms in per.items():
        base = k.split("_")[0]
        op_report[k] = {"ms": round(ms, 5),
                        "GBps_actual": round(bytes_actual[base] / ms / 1e6, 1),
                        "GBps_fp64_equiv": round(bytes_equiv[base] / ms / 1e6, 1),
                        "hbm_frac": round(bytes_actual[base] / ms / 1e6 / HBM_PEAK_GBS, 4)}

    # The same operations on dense binary64 on this GPU, and a plain read of
    # the field (harness only).
    C = torch.empty_like(dA)
    plain = {}
    for name, fn, nbytes in (("add", lambda: torch.add(dA, dB, out=C), 24 * n2),
                             ("scale", lambda: torch.mul(dA, 1.7, out=C), 16 * n2),
                             ("copy", lambda: C.copy_(dA), 16 * n2),
                             ("sum", lambda: torch.sum(dA), 8 * n2)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(20):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 20
        plain[name] = {"ms": round(ms, 5), "GBps": round(nbytes / ms / 1e6, 1)}
        if name in per:
            plain[name]["blaz_speedup"] = round(ms / per[name], 2)
    del C
    # A 2 GiB device-to-device copy: the achievable streaming rate, beside the
    # datasheet peak.
    src = torch.empty(1 << 28, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * (1 << 31) / (c0.elapsed_time(c1) / 5) / 1e6
    del src, dst

    # Roofline of the dominant kernel: compress, 557 algorithmic bytes per block.
    comp_ms = (per["compress_x"] + per["compress_y"]) / 2
    achieved = (BLOCK + RECORD) * nblk / comp_ms / 1e6
    traffic = traffic_for("compress_f64_kernel", CODEC_SOURCES)
    roofline = {"kernel": "compress_f64_kernel", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "copy_2GiB_GBps": round(copy_gbs, 1),
                "frac_vs_copy": round(achieved / copy_gbs, 4),
                # a plain streaming read of the same field (torch.sum), for context
                "sum_read_GBps": plain["sum"]["GBps"],
                "frac_vs_sum_read": round(achieved / plain["sum"]["GBps"], 4)}

    result = {
        "metric": "blaz compress+add GB/s (FP64-equiv) vs plain; matmul TFLOP/s; p99 latency",
        "value": round(64.0 * n2 / ms_step / 1e6, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "ms_per_step_with_per_op_events": round(ms_step_instrumented, 5),
        "ms_per_step_graph": round(ms_step_graph, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain-{n}: two {n}x{n} binary64 smooth fields (16 sinusoids, <= 8 cycles/side, "
                               "N(0,1e-3) noise); step = compress x2 + add + scale(1.7) + decompress",
                   "n": n, "blocks_per_matrix": nblk},
        "roofline": roofline,
        "ops": op_report,
        "plain_dense_fp64": plain,
    }
    result["paper_context"] = {
        "hardware": "Intel Core i7-1165G7, 4 cores (the paper's machine; no GPU numbers are published)",
        "blaz_add_n2000_ms": 0.15, "blaz_add_n2000_GBps_fp64_equiv": 640.0,
        "blaz_scale_n2000_ms": 0.14, "blaz_scale_n2000_GBps_fp64_equiv": 457.0,
        "dense_add_n2000_GBps": 10.3,
        # ratios against the uncompressed operation on the same CPU, read from
        # the performance figure (Experimental Evaluation, Performance, Figure
        # figtime); zfp runs at a rate equivalent to blaz's
        "vs_uncompressed": {"blaz_add_speedup": {"n80": 3, "n2000": 62},
                            "zfp_add_slowdown": {"n80": 121, "n2000": 115},
                            "dot_slowdown_n2000": {"blaz": 31, "zfp": 62},
                            "matmul": "blaz close to the uncompressed product, zfp about 10x slower than blaz"},
        "note": "context only, not a target"}
    del D
    legs = args.legs
    if "cold" in legs:
        print("# cold/warm single-op leg", file=sys.stderr, flush=True)
        result["ops_single_launch"] = cold_ops_leg(blaz, torch, dA, dB)
    if "rates" in legs:
        print("# tunable-rate leg", file=sys.stderr, flush=True)
        result["rates_8192"] = rates_leg(blaz, torch, dA)
    if "transform" in legs:
        print("# transform-input leg", file=sys.stderr, flush=True)
        result["transform_input_8192"] = transform_input_leg(blaz, torch, dA)
    if "serving" in legs:
        result["serving"] = serving_leg(torch, dA, dB, args.serve_requests, args.serve_budget_gib,
                                        step=args.serve_step, trace=args.serve_trace)
    del dA, dB

    if "latency" in legs:
        print("# 64x64 latency leg", file=sys.stderr, flush=True)
        result["latency_64"] = latency_leg(blaz, torch, workload_inputs)
    if "matmul" in legs:
        print("# 4096 linear-algebra leg", file=sys.stderr, flush=True)
        result["matmul_4096"] = matmul_leg(blaz, torch, workload_inputs)
    elif "dots" in legs:  # the dot products of the linear-algebra leg alone (for profiling)
        print("# 4096 dot-product leg", file=sys.stderr, flush=True)
        Am, Bm, Vm = workload_inputs("linalg-4096")
        g = blaz.compress(torch.from_numpy(Am).cuda())
        result["dots_4096"] = dot_leg(blaz, torch, g, blaz.decompress(g), torch.from_numpy(Bm).cuda(),
                                      torch.from_numpy(Vm).cuda())
    if "mixed" in legs:
        print("# 16384 mixed-precision leg", file=sys.stderr, flush=True)
        result["mixed_16384"] = mixed_leg(blaz, torch, workload_inputs)
        torch.cuda.empty_cache()

    if "cpu" in legs:
        print("# CPU oracle leg", file=sys.stderr, flush=True)
        result["cpu_baseline"], (ox, oy) = cpu_baseline(A, B, min(args.cpu_rows, n), workload_inputs)
        result["parity"] = parity_report(A, B, x, y, ox, oy)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
