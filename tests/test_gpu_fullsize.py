"""Parity at the full sizes of the many-stream and the 1 GiB workloads, in
the launch configuration the benchmark times (needs an MI355X).

The oracle cannot cover these sizes whole, so:

* many streams (4096 streams, 602 MiB, 1024 patterns): every stream for a
  sample of patterns and every pattern for a sample of streams, each pair in
  full (hit ends, distances and occurrences);
* one 1 GiB stream (4096 patterns up to 256 symbols): hit ends and distances
  of sampled patterns inside 64 uniformly placed 1 MiB windows, which are
  exact after the first m + K - 1 positions of a window (a scan restarted
  anywhere is exact from there on whenever either value is <= K, the lemma
  that also makes chunked scans exact); every planted copy's neighbourhood
  for its own pattern; and, over the whole stream, the hit set and the
  filtered occurrences that the oracle computes from the GPU's hit-end list
  (Eq. 2 at those ends, then Alg. 1), against the GPU's own.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_1712_03560_amd import oasm  # noqa: E402
from paper_1712_03560_amd import workloads as W  # noqa: E402
from parity_util import compare, group  # noqa: E402

THREADS = 16


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


def one_step(w, keep_h=False):
    """One benchmark step: every stream fed from device memory and closed,
    one sync, results drained (autotuned variants, graphs on)."""
    dev = [torch.from_numpy(t).cuda() for t in w.streams]
    torch.cuda.synchronize()
    with oasm.Matcher(w.patterns, w.ks, keep_h=keep_h, autotune=True, graphs=True) as mt:
        for i, t in enumerate(dev):
            mt.feed(i, t, last=True)
        mt.sync()
        res = mt.results()
    del dev
    return res


def test_batched_full_size_sampled():
    w = W.batched()
    say(f"batched: {len(w.streams)} streams, {w.total_bytes} bytes, {len(w.patterns)} patterns")
    res = one_step(w)
    say(f"batched: gpu done, {res.raw.size} hit ends, {res.occ.size} occurrences")
    rng = np.random.default_rng(3)
    pats = sorted(rng.choice(len(w.patterns), size=3, replace=False).tolist())
    sids = sorted(rng.choice(len(w.streams), size=4, replace=False).tolist())
    pairs = [(s, p) for s in range(len(w.streams)) for p in pats]
    pairs += [(s, p) for s in sids for p in range(len(w.patterns)) if p not in pats]
    streams = {i: t for i, t in enumerate(w.streams)}
    compare(res, streams, w.patterns, w.ks, pairs=pairs, label="batched-sampled")


def test_multiword_full_size_windows_and_whole_stream_filter():
    w = W.multiword()
    t = w.streams[0]
    n = t.size
    say(f"multiword: {n} bytes, {len(w.patterns)} patterns, {len(w.plants)} planted copies")
    res = one_step(w, keep_h=True)
    say(f"multiword: gpu done, {res.raw.size} hit ends, {res.h.size} H records, {res.occ.size} occurrences")
    raw = group(res.raw)
    rng = np.random.default_rng(4)
    lens = np.array([len(p) for p in w.patterns])
    # 16 patterns spread over the word-count classes (lengths 16..256)
    order = np.argsort(lens, kind="stable")
    sample = sorted(order[np.linspace(0, len(order) - 1, 16).astype(int)].tolist())
    wins = np.sort(rng.integers(0, n - (1 << 20), size=64))

    def gpu_ends(p, lo, hi):
        g = raw.get((0, p))
        if g is None:
            return np.zeros(0, np.int64), np.zeros(0, np.int64)
        e = g["end"].astype(np.int64)
        sel = (e >= lo) & (e < hi)
        return e[sel], g["dist"].astype(np.int64)[sel]

    def window_check(job):
        p, a, b = job
        m, K = len(w.patterns[p]), int(w.ks[p])
        ends, dists = oracle.raw_hits(w.patterns[p], t[a:b], K)
        exact_from = a + (m + K - 1 if a > 0 else 0)
        ends = ends.astype(np.int64) + a
        sel = ends >= exact_from
        ge, gd = gpu_ends(p, exact_from, b)
        assert np.array_equal(ge, ends[sel]), f"window [{a},{b}) pattern {p}: hit ends differ"
        assert np.array_equal(gd, dists[sel].astype(np.int64)), f"window [{a},{b}) pattern {p}: distances differ"
        return ge.size

    jobs = [(p, int(a), int(a) + (1 << 20)) for p in sample for a in wins]
    # every planted copy, for its own pattern: a window reaching m + K - 1
    # before the site (so the site and its surroundings are exact)
    for pl in w.plants:
        m, K = len(w.patterns[pl.pattern]), int(w.ks[pl.pattern])
        a = max(0, pl.site - 2 * (m + K))
        b = min(n, pl.site + pl.length + m + K)
        jobs.append((pl.pattern, a, b))
    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        checked = sum(ex.map(window_check, jobs))
    say(f"multiword: {len(jobs)} windows checked, {checked} hit ends")
    # recall: each planted copy ends at a hit of its pattern
    for pl in w.plants[:2000]:
        e = pl.site + pl.length - 1
        ge, _ = gpu_ends(pl.pattern, e, e + 1)
        assert ge.size == 1, (pl, "planted copy not reported")

    # H and S over the whole stream from the GPU's hit ends, for 256 patterns
    hh = group(res.h)
    occ = group(res.occ)
    hs_sample = sorted(set(rng.choice(len(w.patterns), size=256, replace=False).tolist()) | set(sample))

    def filter_by_segments(p, ends):
        """Eq. 2 at the given ends, then Alg. 1, run piece by piece: the ends
        are cut wherever two consecutive ones are at least m + K apart (no
        hit of a piece overlaps the next one's, and a pending best completes
        at its own end, so each piece starts from the empty state -- pinned
        on the CPU), and each piece is filtered on coordinates shifted to
        start at 0 (Alg. 1 uses only differences of positions)."""
        m, K = len(w.patterns[p]), int(w.ks[p])
        cuts = np.flatnonzero(np.diff(ends) >= m + K) + 1
        Hs, S = [], []
        for piece in np.split(ends, cuts):
            if piece.size == 0:
                continue
            hs, hl, hk = oracle.hset_at_ends(w.patterns[p], t, K, piece)
            Hs.append(np.stack([hs, hl.astype(np.int64), hk.astype(np.int64)], 1))
            base = int(hs.min())
            occ_p = oracle.filter_hits(hs - base, hl, hk, K, int((hs + hl).max()) - base).occ.reshape(-1, 3)
            S.append(occ_p + np.array([base, 0, 0]))
        if not Hs:
            return np.zeros((0, 3), np.int64), np.zeros((0, 3), np.int64)
        H = np.concatenate(Hs)
        return H[np.lexsort((H[:, 1], H[:, 0]))], np.concatenate(S)

    def hs_check(p):
        ge, _ = gpu_ends(p, 0, n)
        exp, S = filter_by_segments(p, ge)
        h = hh.get((0, p))
        got = np.stack([h["start"].astype(np.int64), h["len"].astype(np.int64), h["k"].astype(np.int64)], 1) \
            if h is not None else np.zeros((0, 3), np.int64)
        got = got[np.lexsort((got[:, 1], got[:, 0]))] if got.size else got
        assert np.array_equal(got, exp), f"hit set differs for pattern {p}"
        o = occ.get((0, p))
        gs = np.stack([o["start"].astype(np.int64), o["len"].astype(np.int64), o["k"].astype(np.int64)], 1) \
            if o is not None else np.zeros((0, 3), np.int64)
        assert np.array_equal(gs, S), f"occurrences differ for pattern {p}"
        return exp.shape[0], S.shape[0]

    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        tot = [sum(x) for x in zip(*ex.map(hs_check, hs_sample))]
    say(f"multiword: H and S of {len(hs_sample)} patterns over the whole stream: {tot[0]} H records, "
        f"{tot[1]} occurrences")
