"""Benchmark of the OASM matching path on one MI355X.

One step = the whole hot path over one batch of synthetic input: ingest of
device-resident streams (symbol mapping), the bit-parallel scan for every
(stream, pattern) pair, ordering of the hit ends, hit-set recovery, the
shadow-hit filter, and the delivery of hit ends and occurrences to the host.
Throughput is reported in GCUPS (pattern x text cells per second, cells = sum
of pattern lengths x text bytes) over the whole step; the scan kernel's share
is measured with HIP events on the library's stream and set against the
integer-VALU roofline.

The headline workload is the many-stream one (4096 streams of 1 KiB - 1 MiB,
602 MiB, 1024 patterns): all streams in one batched step, compared with one
launch sequence per stream on the same kernels (`vs_plain`).  The same line
carries the single 64 MiB stream (`long_stream`), the serving loop's p50/p99
segment latency (`serving`, `p99_chunk_latency_ms`) and the oracle timed on a
sample of the headline workload (`cpu_baseline`), the 1 GiB multiword stream
with 4096 patterns of up to 256 bytes (`multiword`), the 100,000-symbol tiny
case (`tiny`), and LEV CALC for every
start of 8 MiB of the long stream and of 64 KiB of the multiword stream
(`levcalc`).

    python bench.py [--steps K] [--warmup W] [--workload batched|long|multiword|tiny]
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

METRIC = "GCUPS (pattern×text cells/s) batched vs plain, 1 MI355X; p99 chunk latency"
# MI355X int32 VALU peak from its unit counts and clock: the fp32 vector rate
# of 157.3 TFLOP/s is 128 32-bit lanes per CU per clock (256 CUs, 2.4 GHz,
# an FMA counted as two flops), i.e. 78.6 T 32-bit lane-ops/s.  Measured on
# the chip, v_and / v_xor / v_add_u32 / v_bitop3 reach 52-62 T lane-ops/s and
# shifts, v_bcnt, v_or3 and the carry adds 34-38 T (the half-rate class).
VALU_PEAK_OPS = 256 * 128 * 2.4e9
# Algorithmic int32 VALU work per 32-bit column word per text symbol, frozen
# from the built kernel's ISA: the column recurrence alone (and, add, three
# bitop3, two self-adds for the shifts, bitop3, or, bitop3).  Hit screening,
# addressing, the cutoff's decisions and replays are overhead and show up as
# a lower roofline fraction.
OPS_PER_WORD_STEP = 10
# The anchored column step of the LEV CALC kernel (every start's distances):
# the same ten plus one v_or that enters the first DP row's +1 horizontal
# delta, for the first word of a column (the words above it use the ten).
OPS_PER_ANCHORED_WORD_STEP = 11


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched", choices=["batched", "long", "tiny", "multiword", "homopolymer"])
    ap.add_argument("--homopolymer-bytes", type=int, default=1 << 20,
                    help="stream bytes of the homopolymer workload (a hit end at every position)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--chunk", type=int, default=0, help="chunk bytes (0 = library default)")
    ap.add_argument("--batched-streams", type=int, default=4096)
    ap.add_argument("--multiword-bytes", type=int, default=1 << 26)
    ap.add_argument("--plain-steps", type=int, default=2, help="timed steps of the per-stream comparison")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-stream launch comparison")
    ap.add_argument("--no-long", action="store_true", help="skip the single-stream leg")
    ap.add_argument("--no-multiword", action="store_true", help="skip the multiword leg")
    ap.add_argument("--multiword-leg-bytes", type=int, default=1 << 30, help="stream bytes of the multiword leg")
    ap.add_argument("--no-tiny", action="store_true", help="skip the tiny leg")
    ap.add_argument("--no-worst-case", action="store_true", help="skip the filter worst-case (homopolymer) leg")
    ap.add_argument("--no-autotune", action="store_true", help="heuristic scan variants instead of measured ones")
    ap.add_argument("--no-graphs", action="store_true", help="launch every kernel of a step instead of graph replay")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--serving-sessions", type=int, default=10_000)
    ap.add_argument("--serving-gbps", type=float, default=20.0)
    ap.add_argument("--serving-window", type=float, default=0.05, help="arrival window at the offered load, s")
    ap.add_argument("--serving-window2", type=float, default=2.0, help="arrival window at 0.8x capacity, s")
    ap.add_argument("--serving-budget", type=int, default=64 << 20, help="unmatched-byte budget")
    ap.add_argument("--serving-pool", type=int, default=1 << 26)
    ap.add_argument("--no-valu-probe", action="store_true", help="skip the VALU throughput probe")
    ap.add_argument("--no-levcalc", action="store_true", help="skip the LEV CALC (every start) leg")
    ap.add_argument("--levcalc-only", action="store_true", help="run only the LEV CALC leg")
    ap.add_argument("--levcalc-leg", default="both", choices=["both", "long", "multiword"])
    ap.add_argument("--serving-only", action="store_true", help="run only the serving leg")
    ap.add_argument("--levcalc-bytes", type=int, default=1 << 23, help="text bytes of the LEV CALC leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy three times (PMC traffic calibration)")
    return ap.parse_args()


def valu_probe():
    """Measured int32 VALU rates of single instructions and of the scan's
    column step (the probe built beside the library; a child process that
    owns its own GPU context, run before this process touches the GPU)."""
    import subprocess

    from paper_1712_03560_amd import build as B

    if not os.path.exists(B.PROBE):
        return None
    try:
        res = subprocess.run([B.PROBE], capture_output=True, text=True, timeout=120)
    except subprocess.TimeoutExpired:
        return None
    if res.returncode != 0:
        return None
    try:
        return json.loads(res.stdout.strip().splitlines()[-1])
    except (ValueError, IndexError):
        return None


def copy_calibration():
    """A plain copy kernel of known size: 256 MiB read and 256 MiB written per dispatch."""
    import torch

    src = torch.ones(1 << 28, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("oasm_scan.hip", "oasm_device.h"):
        with open(os.path.join(ROOT, "paper_1712_03560_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


HBM_PEAK_BYTES = 8.0e12  # MI355X HBM3E, 8 TB/s


def traffic_from_profiles(workload: str):
    """HBM bytes of the scan launches of one step, from the committed
    rocprofv3 PMC summary of this workload, if it was taken with the current
    kernel source: the raw FETCH_SIZE and WRITE_SIZE of the step's scan
    launches, each divided by the factor the counter reads for a kernel of
    known size and the same access kind (scalar-load reads for the fetch, as
    the scan reads its text with scalar loads; plain stores for the write).
    Returns (bytes per step, summary dict) or (None, None)."""
    path = os.path.join(ROOT, "profiles", f"scan_{workload}_traffic.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None, None
    return d.get("hbm_bytes_per_step"), d


WORKLOADS = {
    "long": "long-stream: one 64 MiB ACGT text, 256 patterns m~U[16,32], K=3, 10,000 planted copies",
    "tiny": "tiny: 100,000 ACGT symbols, 16 patterns m~U[8,16], K=2, 200 planted copies",
}


def make_workload(name: str, args):
    from paper_1712_03560_amd import workloads as W

    if name == "homopolymer":
        # the filter's worst case: one stream of a single letter, so that the
        # homopolymer patterns end a hit at every position and every filter
        # segment spans the whole stream
        n = int(args.homopolymer_bytes)
        pats = [b"aaaaaaaa", b"aaaa", b"gcaacc", b"acgttgca", b"a" * 40]
        w = W.Workload("homopolymer", [np.full(n, ord("a"), dtype=np.uint8)], pats,
                       np.array([2, 1, 2, 2, 8], dtype=np.uint16), [])
        return w, (f"homopolymer: one stream of {n} bytes 'a', 5 patterns (aaaaaaaa K=2, aaaa K=1, gcaacc K=2, "
                   f"acgttgca K=2, a*40 K=8): a hit end at every position for three of them")
    if name == "long":
        return W.long_stream(), WORKLOADS["long"]
    if name == "tiny":
        return W.tiny(), WORKLOADS["tiny"]
    if name == "multiword":
        w = W.multiword(n=args.multiword_bytes)
        return w, (f"multiword: one {args.multiword_bytes >> 20} MiB stream of mixture bytes (uniform / printable "
                   f"runs, mean 40), 4096 patterns m~U[16,256], K=floor(m/10), planted copies over 0.1 % of bytes")
    w = W.batched(n_streams=args.batched_streams)
    return w, (f"batched: {len(w.streams)} streams log-uniform in [1 KiB, 1 MiB] ({w.total_bytes} bytes), "
               f"Zipf(1.1) 20 letters, 1024 patterns m~U[8,64], K=floor(m/10), one batched step")


def cpu_model() -> str:
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, target_s: float):
    """The oracle (C; raw hits, hit set and filter per (stream, pattern) pair,
    16 threads over the pairs) on a bounded sample of the workload: a prefix
    of a single stream, or a seeded subset of the streams with every pattern,
    sized to about `target_s` seconds from a probe."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    threads = min(16, os.cpu_count() or 1)
    msum = sum(len(p) for p in w.patterns)

    def run(streams):
        jobs = [(t, i) for t in streams for i in range(len(w.patterns))]
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda j: oracle.run_pair(w.patterns[j[1]], j[0], int(w.ks[j[1]])), jobs))

    if len(w.streams) == 1:
        text = w.streams[0]
        probe = min(text.size, 1 << 18)
        t0 = time.perf_counter()
        run([text[:probe]])
        dt = max(time.perf_counter() - t0, 1e-3)
        nbytes = int(min(text.size, max(probe, probe * target_s / dt)))
        t0 = time.perf_counter()
        run([text[:nbytes]])
        dt = time.perf_counter() - t0
        what = f"first {nbytes} bytes of the stream x all {len(w.patterns)} patterns"
    else:
        order = np.random.default_rng(12).permutation(len(w.streams))
        probe_set = [w.streams[i] for i in order[:8]]
        t0 = time.perf_counter()
        run(probe_set)
        dt = max(time.perf_counter() - t0, 1e-3)
        rate = sum(t.size for t in probe_set) / dt
        want = rate * target_s
        chosen, tot = [], 0
        for i in order[8:]:
            if tot >= want:
                break
            chosen.append(w.streams[i])
            tot += w.streams[i].size
        t0 = time.perf_counter()
        run(chosen)
        dt = time.perf_counter() - t0
        nbytes = tot
        what = (f"{len(chosen)} of the {len(w.streams)} streams (seeded choice, {nbytes} bytes) x all "
                f"{len(w.patterns)} patterns")
    # the same oracle on one thread, over a smaller prefix of the sample
    if len(w.streams) == 1:
        one = [w.streams[0][:max(1, nbytes // (2 * threads))]]
    else:
        one, tot1 = [], 0
        for t in chosen:
            if tot1 >= nbytes // (2 * threads):
                break
            one.append(t)
            tot1 += t.size
    n1 = sum(t.size for t in one)
    t0 = time.perf_counter()
    for t in one:
        for i in range(len(w.patterns)):
            oracle.run_pair(w.patterns[i], t, int(w.ks[i]))
    dt1 = time.perf_counter() - t0
    return {"value": round(msum * nbytes / dt / 1e9, 3), "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{what} (hit ends, hit set and filter), {dt:.1f} s",
            "one_thread": {"value": round(msum * n1 / dt1 / 1e9, 3), "unit": "GCUPS",
                           "sample": f"{len(one)} of those streams ({n1} bytes) x all patterns, {dt1:.1f} s"}}


def run_steps(oasm, torch, w, steps, warmup, chunk=0, plain=False, autotune=True, graphs=True):
    """Time `steps` whole-path steps over device-resident streams (after `warmup`)."""
    dev_streams = [torch.from_numpy(t).cuda() for t in w.streams]
    torch.cuda.synchronize()
    mt = oasm.Matcher(w.patterns, w.ks, chunk_bytes=chunk, plain=plain, autotune=autotune, graphs=graphs)
    tune = mt.tune_report()
    sid = [0]

    # the device buffers stay the same from step to step: build the batched
    # feed's table once and give each step new stream ids
    segs = np.zeros(len(dev_streams), dtype=oasm.FEED_SEG_DTYPE)
    segs["data"] = [t.data_ptr() for t in dev_streams]
    segs["len"] = [t.numel() for t in dev_streams]
    segs["flags"] = oasm.OASM_FEED_LAST
    ids = np.arange(len(dev_streams), dtype=np.uint64)
    hs = torch.cuda.current_stream().cuda_stream

    def step():
        segs["stream"] = ids + np.uint64(sid[0])
        mt.feed_segs(segs, (), hs)
        sid[0] += len(dev_streams)
        mt.sync()
        return mt.results()

    res = None
    for _ in range(warmup):
        res = step()
    torch.cuda.synchronize()
    s0 = mt.stats()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s1 = mt.stats()
    mt.destroy()
    del dev_streams
    return {"s0": s0, "s1": s1, "elapsed": elapsed, "res": res, "tune": tune, "steps": steps}


def host_fed(oasm, torch, w, steps: int = 5, warmup: int = 1):
    """The long stream fed from host memory (numpy): each step copies the
    bytes into the library's pinned staging and over PCIe before matching, so
    the rate includes the host-to-device transfer."""
    mt = oasm.Matcher(w.patterns, w.ks, autotune=True, graphs=True)
    text = w.streams[0]
    sid = 0
    for _ in range(warmup):
        mt.feed(sid, text, last=True)
        mt.sync()
        mt.results()
        sid += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mt.feed(sid, text, last=True)
        mt.sync()
        mt.results()
        sid += 1
    el = (time.perf_counter() - t0) / steps
    mt.destroy()
    cells = sum(len(p) for p in w.patterns) * text.size
    return {"gcups": round(cells / el / 1e9, 1), "ms_per_step": round(el * 1e3, 3),
            "host_GBps": round(text.size / el / 1e9, 2), "steps": steps}


def summarize(w, r, workload):
    """GCUPS, the scan's roofline and the step breakdown of a run_steps result."""
    steps = r["steps"]
    msum = sum(len(p) for p in w.patterns)
    cells = msum * w.total_bytes
    word_steps = sum((len(p) + 31) // 32 for p in w.patterns) * w.total_bytes
    s0, s1, elapsed, res = r["s0"], r["s1"], r["elapsed"], r["res"]
    scan_ms = (s1["scan_ms"] - s0["scan_ms"]) / steps
    done = (s1["word_steps_done"] - s0["word_steps_done"]) / steps
    cut = any(x.startswith("class ") and "cut=1" in x for x in r["tune"].splitlines())
    # the algorithmic unit is the word-step; with the word cutoff the
    # recurrence needs only the words it leaves active (the kernel counts
    # them), without it every word of every pattern column
    ops = done * OPS_PER_WORD_STEP
    achieved = ops / (scan_ms * 1e-3) / 1e12 if scan_ms > 0 else None
    peak = VALU_PEAK_OPS / 1e12
    traffic, tsum = traffic_from_profiles(workload)
    hbm_frac = None
    if traffic and scan_ms > 0:
        hbm_frac = round(traffic / (scan_ms * 1e-3) / HBM_PEAK_BYTES, 5)
    return {
        "gcups": cells / (elapsed / steps) / 1e9,
        "ms_per_step": elapsed / steps * 1e3,
        "cells": cells,
        "roofline": {"bound": "alu", "achieved": round(achieved, 2) if achieved else None, "peak": round(peak, 2),
                     "unit": "TOP/s", "frac": round(achieved / peak, 4) if achieved else None,
                     "traffic": traffic, "traffic_unit": "HBM bytes per step's scan launches",
                     "hbm_frac": hbm_frac, "hbm_peak_GBps": HBM_PEAK_BYTES / 1e9,
                     "traffic_calibration": ({k: tsum[k] for k in ("fetch_factor_scalar_reads",
                                                                     "fetch_factor_vector_reads",
                                                                     "write_factor", "profile")}
                                             if tsum else None),
                     "kernel": "k_scan", "scan_ms_per_step": round(scan_ms, 3),
                     "scan_launches_per_step": (s1["scan_launches"] - s0["scan_launches"]) / steps,
                     "word_steps": int(done), "word_steps_full_columns": word_steps,
                     "ops_per_word_step": OPS_PER_WORD_STEP, "word_cutoff": cut,
                     # algorithmic bytes: the text of the step, read once
                     "algorithmic_bytes_per_step": w.total_bytes},
        "scan_gcups": round(cells / (scan_ms * 1e-3) / 1e9, 1) if scan_ms > 0 else None,
        "step_breakdown_ms": {
            "scan_kernel": round(scan_ms, 3),
            "device_step": round((s1["step_ms"] - s0["step_ms"]) / steps, 3),
            "sync_wall": round((s1["sync_wall_ms"] - s0["sync_wall_ms"]) / steps, 3),
            "sync_waiting": round((s1["wait_ms"] - s0["wait_ms"]) / steps, 3),
            "host_plan_launch_convert_bookkeep": [round((b - a) / steps, 3) for a, b in
                                                  zip(s0["host_ms"], s1["host_ms"])],
            "python_feed_drain": round(elapsed / steps * 1e3 - (s1["sync_wall_ms"] - s0["sync_wall_ms"]) / steps, 3),
            "graph_replays": s1["graph_replays"] - s0["graph_replays"],
        },
        "hits": {"hit_ends": int(res.raw.size), "occurrences": int(res.occ.size),
                 "filtered_hits_per_s": round(res.occ.size / (elapsed / steps), 1)},
        "autotune": [x for x in r["tune"].splitlines() if x],
    }


def serving_measure(oasm, torch, args):
    """Continuous batching of Poisson segment arrivals (10,000 sessions,
    2048 patterns m~U[16,128], 1..64 KiB segments of mixture bytes): one point
    at the configured offered load (20 GB/s, far above one GPU's capacity for
    this dictionary: it measures the sustained rate and the queueing), one at
    0.8x the sustained rate (latency under a load the GPU can carry)."""
    from paper_1712_03560_amd import workloads as W

    pats, ks = W.serving_dictionary()
    pool = W.serving_pool(args.serving_pool)
    # mutated pattern copies in the pool (one per 3.3 KiB on average), so that
    # sessions hold hit ends and the hit-set recovery and the filter have work
    n_plants = args.serving_pool // 3355
    W.plant(np.random.default_rng(23), pool, pats, n_plants, ks, W.LETTERS_MIX)
    dpool = torch.from_numpy(pool).cuda()
    msum = sum(len(p) for p in pats)
    out = {"workload": f"{args.serving_sessions} sessions, {len(pats)} patterns m~U[16,128] K=floor(m/10), "
                       f"segments U[1,64] KiB of a {args.serving_pool >> 20} MiB pool of mixture bytes with "
                       f"{n_plants} planted mutated pattern copies, Poisson arrivals",
           "mem_budget_bytes": args.serving_budget}

    def point(gbps, duration):
        sess, off, ln, t = W.serving_arrivals(args.serving_sessions, duration, gbps, pool.size)
        segs = np.zeros(t.size, dtype=oasm.SEG_DTYPE)
        segs["stream"], segs["offset"], segs["len"], segs["arrival_s"] = sess, off, ln, t
        with oasm.Matcher(pats, ks, mem_budget=args.serving_budget, no_raw=True, autotune=True) as mt:
            # warm the context (kernels, pools, tuning cache) on a small prefix
            mt.serve(segs[:200].copy(), dpool, want_latency=False)
            mt.results()
        with oasm.Matcher(pats, ks, mem_budget=args.serving_budget, no_raw=True, autotune=True) as mt:
            s0 = mt.stats()
            rep, lat = mt.serve(segs, dpool)
            s1 = mt.stats()
            res = mt.results()
        nbytes = int(ln.sum())
        ns = max(1, rep["steps"])
        per_step = {"device_step_ms": round((s1["step_ms"] - s0["step_ms"]) / ns, 4),
                    "scan_ms": round((s1["scan_ms"] - s0["scan_ms"]) / ns, 4),
                    "sync_wall_ms": round((s1["sync_wall_ms"] - s0["sync_wall_ms"]) / ns, 4),
                    "host_plan_launch_convert_bookkeep_ms": [round((b - a) / ns, 4) for a, b in
                                                             zip(s0["host_ms"], s1["host_ms"])],
                    "loop_busy_ms": round(rep["busy_s"] * 1e3 / ns, 4),
                    "hit_ends": s1["raw_hits"] - s0["raw_hits"]}
        return {"offered_GBps": gbps, "arrival_window_s": duration, "segments": int(t.size), "bytes": nbytes,
                "steps": rep["steps"], "deferred": rep["deferred"], "max_batch_bytes": rep["max_batch_bytes"],
                "wall_s": round(rep["wall_s"], 3), "sustained_GBps": round(nbytes / rep["busy_s"] / 1e9, 4),
                "gcups": round(msum * nbytes / rep["busy_s"] / 1e9, 1),
                "latency_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                "latency_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                "occurrences": int(res.occ.size), "per_step": per_step}

    hi = point(args.serving_gbps, args.serving_window)
    out["at_offered_load"] = hi
    lo_rate = 0.8 * hi["sustained_GBps"]
    out["at_0p8_capacity"] = point(lo_rate, args.serving_window2)
    return out


def levcalc_word_steps(m: int, K: int):
    """Word-steps of one start's anchored column in the LEV CALC kernel: step
    j (column l = j + 1) advances min(W, ceil((l + K) / 32)) words before
    the first output and all W words from l = m - K on (the band cutoff);
    and the same without the cutoff, (m + K) * W."""
    W = (m + 31) // 32
    quiet = m - K - 1
    band = sum(min(W, -(-(j + 1 + K) // 32)) if j < quiet else W for j in range(m + K))
    return band, (m + K) * W


def levcalc_measure(oasm, torch, w, n: int, desc: str, reps: int = 5):
    """LEV CALC for every start (the distances between each pattern and the
    2K+1 substrings starting at every text position) over the first n bytes
    of a workload's stream, timed with HIP events on the stream the kernel
    runs on; beside it the oracle on a short prefix (16 threads over the
    patterns)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    text = np.ascontiguousarray(w.streams[0][:n])
    dev = torch.from_numpy(text).cuda()
    ms = np.array([len(p) for p in w.patterns], dtype=np.int64)
    ks = np.asarray(w.ks, dtype=np.int64)
    with oasm.Matcher(w.patterns, w.ks) as mt:
        out = mt.levcalc(dev)  # warm-up (and the output buffer)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            mt.levcalc(dev, out=out)
        e1.record(st)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / reps * 1e-3
    steps = [levcalc_word_steps(int(m), int(k)) for m, k in zip(ms, ks)]
    word_steps = n * sum(b for b, _ in steps)
    full = n * sum(f for _, f in steps)
    first_words = n * int(np.sum(ms + ks))  # the first word of every column step
    ops = word_steps * 10 + first_words * (OPS_PER_ANCHORED_WORD_STEP - 10)
    dists = n * int(np.sum(2 * ks + 1))
    cells = n * int(np.sum(ms * (ms + ks)))
    peak = VALU_PEAK_OPS / 1e12
    achieved = ops / t / 1e12
    # the oracle on a short prefix
    # (sized from the Eq. 1 cells it evaluates, about 1.3e9: a second or two;
    # for long patterns, a seeded subset of them over 4 starts)
    cost = (2 * ks + 1) * ms * (ms + ks)
    nb = max(4, min(2048, int(1.3e9 // max(1, int(np.sum(cost))))))
    sub = np.arange(len(w.patterns))
    if nb * int(np.sum(cost)) > 2.6e9:
        sub = np.random.default_rng(7).permutation(len(w.patterns))
        sub = np.sort(sub[:max(1, int(np.searchsorted(np.cumsum(cost[sub]) * nb, 1.3e9)))])
    span = nb + int(np.max(ms + ks))  # every substring of the first nb starts fits

    def one_pattern(q):
        p, K, m = w.patterns[q], int(ks[q]), int(ms[q])
        if nb >= 4 * (m + K):  # the whole prefix in one call
            return int(np.count_nonzero(oracle.levcalc(p, text[:span], K) != 255))
        for i in range(nb):  # short samples: one Eq. 1 evaluation per distance
            for l in range(m - K, m + K + 1):
                oracle.lev(p, text[i:i + l])
        return nb * (2 * K + 1)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        done = sum(ex.map(one_pattern, sub.tolist()))  # distances the oracle computed
    dt = time.perf_counter() - t0
    return {"workload": desc,
            "ms_per_call": round(t * 1e3, 3), "distances_per_s": round(dists / t, 1),
            "anchored_gcups": round(cells / t / 1e9, 1),
            "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2), "unit": "TOP/s",
                         "frac": round(achieved / peak, 4), "kernel": "k_levcalc", "word_steps": word_steps,
                         "word_steps_full_columns": full,
                         "ops_per_word_step": f"{OPS_PER_ANCHORED_WORD_STEP} (first word), 10 (others)",
                         "output_bytes": dists, "output_GBps": round(dists / t / 1e9, 1)},
            "oracle_sample": {"distances_per_s": round(done / dt, 1), "cores": min(16, os.cpu_count() or 1),
                              "sample": f"the first {nb} starts (and, for short patterns, the rest of "
                                        f"the first {span} bytes) x {sub.size} of the {len(w.patterns)} "
                                        f"patterns ({done} distances), {dt:.2f} s"}}


def levcalc_legs(oasm, torch, args):
    """LEV CALC on the long stream's 256 one-word patterns (8 MiB) and on the
    multiword dictionary's 4096 patterns of 16..256 bytes (64 KiB)."""
    from paper_1712_03560_amd import workloads as W

    out = {}
    if args.levcalc_leg in ("both", "long"):
        n1 = int(args.levcalc_bytes)
        wl = W.long_stream()
        out = levcalc_measure(oasm, torch, wl, n1, f"LEV CALC for every start: first {n1} bytes of the long "
                                                   f"stream (ACGT) x its 256 patterns m~U[16,32], K=3")
        del wl
    if args.levcalc_leg in ("both", "multiword"):
        n2 = 1 << 16
        wm = W.multiword(n=1 << 20)
        out["multiword"] = levcalc_measure(oasm, torch, wm, n2, f"LEV CALC for every start: first {n2} bytes of "
                                                                f"the multiword stream x its 4096 patterns "
                                                                f"m~U[16,256], K=floor(m/10)")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library runs on one GPU "
              f"and has no multi-GPU mode", file=sys.stderr)
        sys.exit(2)
    probe = None if args.no_valu_probe else valu_probe()
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1712_03560_amd import build as B

    if not os.path.exists(B.LIB):
        B.build()
    from paper_1712_03560_amd import oasm

    if args.levcalc_only:
        print(json.dumps({"levcalc": levcalc_legs(oasm, torch, args)}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_measure(oasm, torch, args)}), flush=True)
        return
    if args.calibrate_copy:
        copy_calibration()
    worst = None
    if args.workload != "homopolymer" and not args.no_worst_case:
        # the filter's worst case, measured first (so that the main workload's
        # scans are the last ones a profile of this command sees): a hit end
        # at every position, each pattern's filter segment spanning the stream
        wh, dh = make_workload("homopolymer", args)
        rh = run_steps(oasm, torch, wh, 3, 1, autotune=not args.no_autotune, graphs=not args.no_graphs)
        mh = summarize(wh, rh, "homopolymer")
        worst = {"workload": dh, "ms_per_step": round(mh["ms_per_step"], 3),
                 "device_step_ms": mh["step_breakdown_ms"]["device_step"], "hits": mh["hits"]}
        del rh, wh
    w, desc = make_workload(args.workload, args)
    r = run_steps(oasm, torch, w, args.steps, args.warmup, chunk=args.chunk, autotune=not args.no_autotune,
                  graphs=not args.no_graphs)
    m = summarize(w, r, args.workload)
    line = {
        "metric": METRIC,
        "value": round(m["gcups"], 1),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc, "streams": len(w.streams), "patterns": len(w.patterns),
                   "text_bytes": w.total_bytes, "cells": m["cells"]},
        "roofline": m["roofline"],
        "valu_probe": probe,
        "scan_gcups": m["scan_gcups"],
        "step_breakdown_ms": m["step_breakdown_ms"],
        "hits": m["hits"],
        "autotune": m["autotune"],
    }
    if len(w.streams) > 1 and not args.no_plain:
        # the same workload with one launch sequence per stream (same kernels)
        p = run_steps(oasm, torch, w, args.plain_steps, 1, plain=True, autotune=not args.no_autotune)
        assert p["res"].occ.size == r["res"].occ.size and p["res"].raw.size == r["res"].raw.size
        tp = p["elapsed"] / args.plain_steps
        line["vs_plain"] = {"plain_gcups": round(m["cells"] / tp / 1e9, 1), "plain_ms_per_step": round(tp * 1e3, 2),
                            "batched_gcups": line["value"], "speedup": round(tp * 1e3 / m["ms_per_step"], 2)}
    del r
    if args.workload != "long" and not args.no_long:
        wl, dl = make_workload("long", args)
        rl = run_steps(oasm, torch, wl, max(args.steps, 10), 2, autotune=not args.no_autotune,
                       graphs=not args.no_graphs)
        ml = summarize(wl, rl, "long")
        line["long_stream"] = {"workload": dl, "gcups": round(ml["gcups"], 1),
                               "ms_per_step": round(ml["ms_per_step"], 3), "roofline": ml["roofline"],
                               "step_breakdown_ms": ml["step_breakdown_ms"], "hits": ml["hits"],
                               "autotune": ml["autotune"], "host_fed": host_fed(oasm, torch, wl)}
        del rl, wl
    if args.workload != "multiword" and not args.no_multiword:
        from paper_1712_03560_amd import workloads as W

        nb = int(args.multiword_leg_bytes)
        wm = W.multiword(n=nb)
        rm = run_steps(oasm, torch, wm, 2, 1, autotune=not args.no_autotune, graphs=not args.no_graphs)
        mm = summarize(wm, rm, "multiword")
        line["multiword"] = {"workload": f"multiword: one {nb >> 20} MiB stream of mixture bytes (uniform / printable "
                                         f"runs, mean 40), 4096 patterns m~U[16,256], K=floor(m/10), "
                                         f"{len(wm.plants)} planted copies",
                             "gcups": round(mm["gcups"], 1), "ms_per_step": round(mm["ms_per_step"], 3),
                             "roofline": mm["roofline"], "step_breakdown_ms": mm["step_breakdown_ms"],
                             "hits": mm["hits"], "autotune": mm["autotune"]}
        del rm, wm
    if args.workload != "tiny" and not args.no_tiny:
        wt, dt_ = make_workload("tiny", args)
        rt = run_steps(oasm, torch, wt, 20, 3, autotune=not args.no_autotune, graphs=not args.no_graphs)
        mt_ = summarize(wt, rt, "tiny")
        line["tiny"] = {"workload": dt_, "gcups": round(mt_["gcups"], 1), "ms_per_step": round(mt_["ms_per_step"], 3),
                        "scan_ms_per_step": mt_["roofline"]["scan_ms_per_step"], "hits": mt_["hits"]}
        del rt, wt
    if worst is not None:
        line["filter_worst_case"] = worst
    if not args.no_levcalc:
        line["levcalc"] = levcalc_legs(oasm, torch, args)
    if not args.no_serving:
        line["serving"] = serving_measure(oasm, torch, args)
        line["p99_chunk_latency_ms"] = line["serving"]["at_0p8_capacity"]["latency_p99_ms"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
