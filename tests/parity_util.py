"""Helpers for comparing the HIP path with the CPU oracle, pair by pair."""
from __future__ import annotations

import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def group(rec: np.ndarray, keys=("stream", "pattern")):
    """Split structured records into {(stream, pattern): rows} keeping order."""
    out = {}
    if rec.size == 0:
        return out
    s = rec["stream"].astype(np.int64)
    p = rec["pattern"].astype(np.int64)
    order = np.lexsort((np.arange(rec.size), p, s))
    r = rec[order]
    s, p = s[order], p[order]
    cut = np.flatnonzero((np.diff(s) != 0) | (np.diff(p) != 0)) + 1
    for a, b in zip(np.r_[0, cut], np.r_[cut, r.size]):
        out[(int(s[a]), int(p[a]))] = r[a:b]
    return out


def oracle_pairs(streams: dict, patterns, ks, pairs=None, threads=None, with_filter=True, rules=1):
    """Oracle results for every (stream id, pattern index) pair (or the given ones)."""
    if pairs is None:
        pairs = [(sid, pi) for sid in streams for pi in range(len(patterns))]
    threads = threads or min(16, os.cpu_count() or 1)

    def one(pair):
        sid, pi = pair
        return pair, oracle.run_pair(patterns[pi], streams[sid], int(ks[pi]), with_filter, rules)

    # a progress line every 20 s, so that a long oracle run is seen to advance
    out, t0, last = {}, time.monotonic(), time.monotonic()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for key, val in ex.map(one, pairs):
            out[key] = val
            if time.monotonic() - last > 20:
                last = time.monotonic()
                print(f"[parity] oracle: {len(out)} of {len(pairs)} pairs after {last - t0:.0f} s", file=sys.stderr,
                      flush=True)
    return out


def compare(res, streams: dict, patterns, ks, pairs=None, check_h=False, with_filter=True, label="", rules=1):
    """Assert bit-exact agreement of hit ends, distances, H and S per pair
    (S under the given filter rules, the library's OASM_RULES_* bits)."""
    want = oracle_pairs(streams, patterns, ks, pairs, with_filter=with_filter, rules=rules)
    raw = group(res.raw)
    occ = group(res.occ)
    hh = group(res.h) if check_h and res.h is not None else {}
    n_raw = n_occ = 0
    for (sid, pi), w in want.items():
        g = raw.get((sid, pi))
        ge = g["end"].astype(np.int64) if g is not None else np.zeros(0, np.int64)
        gd = g["dist"].astype(np.int64) if g is not None else np.zeros(0, np.int64)
        assert np.array_equal(ge, w.ends), f"{label} raw ends differ for stream {sid} pattern {pi}: " \
            f"gpu {ge[:10]}... ({ge.size}) oracle {w.ends[:10]}... ({w.ends.size})"
        if not np.array_equal(gd, w.dists):
            bad = np.nonzero(gd != w.dists)[0]
            raise AssertionError(
                f"{label} raw distances differ for stream {sid} pattern {pi} at {bad.size} of {gd.size} ends; "
                f"first: " + ", ".join(f"end {int(ge[b])} gpu {int(gd[b])} oracle {int(w.dists[b])}" for b in bad[:8]))
        n_raw += ge.size
        if with_filter:
            o = occ.get((sid, pi))
            got = np.stack([o["start"].astype(np.int64), o["len"].astype(np.int64), o["k"].astype(np.int64)],
                           1) if o is not None else np.zeros((0, 3), np.int64)
            assert np.array_equal(got, w.occ.reshape(-1, 3)), \
                f"{label} occurrences differ for stream {sid} pattern {pi}:\n gpu {got[:8].tolist()}\n " \
                f"oracle {w.occ[:8].tolist()}"
            n_occ += got.shape[0]
        if check_h:
            h = hh.get((sid, pi))
            got = np.stack([h["start"].astype(np.int64), h["len"].astype(np.int64), h["k"].astype(np.int64)],
                           1) if h is not None else np.zeros((0, 3), np.int64)
            # H is a set (Eq. 2); within one sync it is drained in (start, length)
            # order, and records found by a later sync may start earlier
            got = got[np.lexsort((got[:, 1], got[:, 0]))] if got.size else got
            exp = np.stack([w.H[0], w.H[1].astype(np.int64), w.H[2].astype(np.int64)], 1)
            assert np.array_equal(got, exp), f"{label} hit set differs for stream {sid} pattern {pi}"
    # nothing reported for pairs outside the compared set beyond those pairs
    if pairs is None:
        assert set(raw) <= set(want), f"{label} unexpected pairs {sorted(set(raw) - set(want))[:5]}"
    print(f"[parity] {label}: {len(want)} pairs, {n_raw} hit ends, {n_occ} occurrences", file=sys.stderr,
          flush=True)
    return n_raw, n_occ
