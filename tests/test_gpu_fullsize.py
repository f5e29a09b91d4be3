"""Parity at the full sizes of the long, many-stream and 1 GiB workloads,
in the launch configuration the benchmark times (needs an MI355X): three
steps each, fed as the benchmark feeds them (one batched device feed, new
stream ids per step), autotuned variants, graphs on.  The first step runs
eagerly and is checked against the oracle; the second is captured as HIP
graphs and the third replays them, and both must give the first step's
records.

The oracle covers, of the first step:

* the 64 MiB long stream: every one of its 256 patterns over the whole
  stream (hit ends, distances and occurrences), and every planted copy;
* many streams (4096 streams, 602 MiB, 1024 patterns): two patterns of every
  (32-bit word count, K) combination over all 4096 streams, and every
  pattern over four streams, each pair in full;
* the 1 GiB stream (4096 patterns up to 256 symbols): hit ends and distances
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


def bench_steps(w, nsteps=3, keep_h=False):
    """Steps exactly as the benchmark times them: every stream fed from
    device memory in one batched feed (new stream ids each step) and closed,
    one sync, results drained; autotuned variants, graphs on.  The first step
    runs eagerly, the second is captured as HIP graphs (its shape repeats the
    first one's), the later ones replay them.  Returns the per-step results
    with stream ids mapped back to 0 .. len(streams) - 1, and the stats."""
    dev = [torch.from_numpy(t).cuda() for t in w.streams]
    torch.cuda.synchronize()
    segs = np.zeros(len(dev), dtype=oasm.FEED_SEG_DTYPE)
    segs["data"] = [t.data_ptr() for t in dev]
    segs["len"] = [t.numel() for t in dev]
    segs["flags"] = oasm.OASM_FEED_LAST
    ids = np.arange(len(dev), dtype=np.uint64)
    out = []
    with oasm.Matcher(w.patterns, w.ks, keep_h=keep_h, autotune=True, graphs=True) as mt:
        hs = torch.cuda.current_stream().cuda_stream
        for step in range(nsteps):
            base = np.uint64(step * len(dev))
            segs["stream"] = ids + base
            mt.feed_segs(segs, (), hs)
            mt.sync()
            res = mt.results()
            for rec in (res.raw, res.occ, res.h):
                if rec is not None and rec.size:
                    assert (rec["stream"] >= base).all() and (rec["stream"] < base + np.uint64(len(dev))).all()
                    rec["stream"] -= base
            # one sync's records come in (stream id, pattern) order, hit ends
            # by end inside a pair (occurrences in emission order)
            for rec, keys in ((res.raw, ("end", "pattern", "stream")), (res.occ, ("pattern", "stream"))):
                if rec.size > 1:
                    order = np.lexsort(tuple(rec[k] for k in keys))
                    assert np.array_equal(order, np.arange(rec.size)), f"step {step}: order by {keys}"
            out.append(res)
            say(f"step {step}: {res.raw.size} hit ends, {res.occ.size} occurrences, "
                f"graph replays {mt.stats()['graph_replays']}")
        stats = mt.stats()
    del dev
    return out, stats


def assert_steps_equal(steps):
    """Captured and replayed steps give the records of the eager first step."""
    for i, r in enumerate(steps[1:], 1):
        for name in ("raw", "occ", "h"):
            a, b = getattr(steps[0], name), getattr(r, name)
            if a is None:
                continue
            assert np.array_equal(a, b), f"step {i} ({'captured' if i == 1 else 'replayed'}) {name} differs"


def per_class_sample(w, per_combo=2):
    """Patterns covering every (32-bit word count, K) combination of a
    dictionary: the shortest and the longest of each (patterns of one word
    count sit in tiles shortest first, so these land in different tiles)."""
    lens = np.array([len(p) for p in w.patterns])
    wc = (lens + 31) // 32
    ks = np.asarray(w.ks, dtype=np.int64)
    pick = set()
    combos = sorted(set(zip(wc.tolist(), ks.tolist())))
    for c in combos:
        idx = np.flatnonzero((wc == c[0]) & (ks == c[1]))
        idx = idx[np.argsort(lens[idx], kind="stable")]
        pick.update(idx[np.linspace(0, idx.size - 1, min(per_combo, idx.size)).astype(int)].tolist())
    return sorted(pick), combos


@pytest.mark.timeout(900)
def test_batched_full_size_graph_steps():
    """The many-stream workload (4096 streams, 602 MiB, 1024 patterns) in the
    benchmark's launch configuration, three steps: the eager step against the
    oracle for two patterns of every (word count, K) combination over all
    4096 streams and for every pattern over four streams; the captured and
    the replayed steps equal to the eager one."""
    w = W.batched()
    say(f"batched: {len(w.streams)} streams, {w.total_bytes} bytes, {len(w.patterns)} patterns")
    steps, stats = bench_steps(w, 3)
    assert stats["graph_replays"] >= 1, stats["graph_replays"]  # step 2 captures, step 3 replays
    assert_steps_equal(steps)
    pats, combos = per_class_sample(w)
    assert len(combos) == 8, combos  # (1, K) for K = 0..3 and (2, K) for K = 3..6
    rng = np.random.default_rng(3)
    sids = sorted(rng.choice(len(w.streams), size=4, replace=False).tolist())
    pairs = [(s, p) for s in range(len(w.streams)) for p in pats]
    pairs += [(s, p) for s in sids for p in range(len(w.patterns)) if p not in pats]
    streams = {i: t for i, t in enumerate(w.streams)}
    say(f"batched: oracle on {len(pats)} patterns x all streams + {len(sids)} streams x all patterns")
    compare(steps[0], streams, w.patterns, w.ks, pairs=pairs, label="batched-per-class")


@pytest.mark.timeout(900)
def test_long_full_size_all_patterns():
    """The 64 MiB single stream with 256 patterns (K = 3, 10,000 planted
    copies) in the benchmark's launch configuration, three steps: the eager
    step against the oracle for every pattern over the whole stream (hit
    ends, distances and occurrences), the captured and replayed steps equal
    to it, and every planted copy reported by its pattern."""
    w = W.long_stream()
    t = w.streams[0]
    say("long: 64 MiB, 256 patterns, K=3")
    steps, stats = bench_steps(w, 3)
    assert stats["graph_replays"] >= 1, stats["graph_replays"]  # step 2 captures, step 3 replays
    assert_steps_equal(steps)
    res = steps[0]
    n_raw, n_occ = compare(res, {0: t}, w.patterns, w.ks, label="long-all-patterns")
    assert n_raw > 10_000 and n_occ > 5_000
    ends = {}
    for pi, e in zip(res.raw["pattern"].tolist(), res.raw["end"].tolist()):
        ends.setdefault(pi, set()).add(e)
    for pl in w.plants:
        e = pl.site + pl.length - 1
        assert e in ends.get(pl.pattern, ()), (pl, "planted copy not reported")


@pytest.mark.timeout(900)
def test_multiword_full_size_windows_and_whole_stream_filter():
    w = W.multiword()
    t = w.streams[0]
    n = t.size
    say(f"multiword: {n} bytes, {len(w.patterns)} patterns, {len(w.plants)} planted copies")
    steps, stats = bench_steps(w, 3, keep_h=True)
    assert stats["graph_replays"] >= 1, stats["graph_replays"]  # step 2 captures, step 3 replays
    assert_steps_equal(steps)
    res = steps[0]
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
