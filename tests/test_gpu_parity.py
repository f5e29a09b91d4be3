"""Parity of the HIP path with the CPU oracle (needs an MI355X).

Every comparison is exact: hit ends and their distances (Less Naive scan),
the hit set at those ends (Eq. 2) and the filtered occurrences (Alg. 1), per
(stream, pattern) pair, on seeded inputs.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1712_03560_amd import oasm  # noqa: E402
from paper_1712_03560_amd import workloads as W  # noqa: E402
from parity_util import compare  # noqa: E402


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


def run(patterns, ks, streams: dict, *, keep_h=True, plain=False, chunk_bytes=0, pieces=None, device=False,
        rules=oasm.OASM_RULES_PAPER, autotune=False, cutoff=True):
    """Feed every stream (optionally in pieces with syncs between), close, sync, drain."""
    with oasm.Matcher(patterns, ks, rules, keep_h=keep_h, plain=plain, chunk_bytes=chunk_bytes,
                      autotune=autotune, cutoff=cutoff) as mt:
        if pieces is None:
            for sid, t in streams.items():
                mt.feed(sid, torch.from_numpy(t).cuda() if device and t.size else t)
        else:
            rng = np.random.default_rng(pieces)
            cuts = {sid: sorted(rng.integers(0, t.size + 1, size=int(rng.integers(1, 6))).tolist()) for sid, t in
                    streams.items()}
            for r in range(6):
                for sid, t in streams.items():
                    cs = [0] + cuts[sid] + [t.size]
                    if r + 1 < len(cs):
                        mt.feed(sid, t[cs[r]:cs[r + 1]])
                mt.sync()
        for sid in streams:
            mt.close(sid)
        mt.sync()
        return mt.results()


def test_tiny_config_full():
    w = W.tiny()
    say("tiny: 100,000 ACGT symbols, 16 patterns, K=2")
    res = run(w.patterns, w.ks, {0: w.streams[0]})
    n_raw, n_occ = compare(res, {0: w.streams[0]}, w.patterns, w.ks, check_h=True, label="tiny")
    assert n_raw > 200 and n_occ > 0


@pytest.mark.parametrize("seed,mlo,mhi,alphabet,kmax", [
    (1, 1, 8, b"AB", None),
    (2, 4, 40, b"ACGT", None),
    (3, 30, 34, b"ACGT", 6),
    (4, 60, 70, b"ACGT", 10),
    (5, 90, 140, b"ab", 20),
    (6, 180, 256, bytes(range(256)), 25),
    (7, 1, 256, bytes([0, 255, 7, 128]), 12),
])
def test_random_dictionaries(seed, mlo, mhi, alphabet, kmax):
    w = W.small_random(seed, 3000, 24, mlo, mhi, alphabet, kmax=kmax, n_plants=20, n_streams=3)
    streams = {10 + i: s for i, s in enumerate(w.streams)}
    say(f"random seed {seed}: m in [{mlo},{mhi}], |alphabet|={len(alphabet)}")
    res = run(w.patterns, w.ks, streams)
    compare(res, streams, w.patterns, w.ks, check_h=True, label=f"random{seed}")


@pytest.mark.parametrize("seed,alphabet,kmax", [(80, b"AB", 40), (81, b"ACGT", 30), (82, bytes(range(32, 127)), 25)])
def test_word_cutoff_matches_full_columns_and_oracle(seed, alphabet, kmax):
    """Multi-word patterns (33..256 symbols) with thresholds up to 40 on text
    with planted copies: the word cutoff (the default) and full columns give
    the same results, equal to the oracle's."""
    w = W.small_random(seed, 12000, 48, 33, 256, alphabet, kmax=kmax, n_plants=60, n_streams=2)
    streams = {i: s for i, s in enumerate(w.streams)}
    say(f"cutoff seed {seed}")
    a = run(w.patterns, w.ks, streams)
    b = run(w.patterns, w.ks, streams, cutoff=False)
    for x, y in ((a.raw, b.raw), (a.occ, b.occ), (a.h, b.h)):
        assert np.array_equal(np.sort(x, order=list(x.dtype.names)), np.sort(y, order=list(y.dtype.names)))
    compare(a, streams, w.patterns, w.ks, check_h=True, label=f"cutoff{seed}")


@pytest.mark.parametrize("m", [31, 32, 33, 63, 64, 65, 127, 128, 129, 192, 193, 255, 256])
def test_word_boundaries(m):
    rng = np.random.default_rng(m)
    pats = [bytes(rng.integers(65, 69, size=m).astype(np.uint8)) for _ in range(5)]
    ks = [0, 1, m // 10, min(63, m // 4), min(63, m - 1)]
    t = rng.integers(65, 69, size=6000).astype(np.uint8)
    for i, p in enumerate(pats):  # plant exact and mutated copies
        t[500 + 1000 * i: 500 + 1000 * i + m] = np.frombuffer(p, np.uint8)
    say(f"word boundary m={m}")
    res = run(pats, ks, {0: t})
    compare(res, {0: t}, pats, ks, check_h=True, label=f"m{m}")


def test_dense_shadow_hits():
    """Homopolymer patterns on low-entropy text: nearly every end is a hit."""
    pats = [b"aaaaaaaa", b"aaaa", b"gcaacc", b"acgttgca", b"a" * 40]
    ks = [2, 1, 2, 2, 8]
    rng = np.random.default_rng(9)
    t = np.where(rng.random(20000) < 0.85, ord("a"), rng.choice(np.frombuffer(b"cgt", np.uint8), 20000)).astype(
        np.uint8)
    res = run(pats, ks, {0: t})
    compare(res, {0: t}, pats, ks, check_h=True, label="dense")


@pytest.mark.parametrize("n", [33 * 8 + 5, 70_000])
def test_long_filter_segments(n):
    """Segments of more than 32 hit ends: up to 255 starts walked by one
    wavefront each from LDS tiles of 256 records, longer ones split over
    their starts (next pointers, the chain, its links re-walked at once):
    homopolymer text, where three patterns end a hit at every position (one
    segment per pattern over the whole stream), mixed with a text whose runs
    of the letter make segments of every length around the tile and
    hand-over sizes; closed and carried (split feeds)."""
    pats = [b"aaaaaaaa", b"aaaa", b"gcaacc", b"acgttgca", b"a" * 40, b"aaagaaa"]
    ks = [2, 1, 2, 2, 8, 3]
    rng = np.random.default_rng(n)
    t1 = np.full(n, ord("a"), dtype=np.uint8)
    t2 = np.full(n, ord("a"), dtype=np.uint8)
    pos = 0
    while pos < n:  # runs of 'a' of 20..700 symbols between single other letters
        pos += int(rng.integers(20, 700))
        if pos < n:
            t2[pos] = rng.choice(np.frombuffer(b"cgt", np.uint8))
    streams = {0: t1, 1: t2}
    say(f"long filter segments, n={n}")
    res = run(pats, ks, streams)
    compare(res, streams, pats, ks, check_h=True, label=f"long-seg{n}")
    res = run(pats, ks, streams, pieces=n)
    compare(res, streams, pats, ks, check_h=True, label=f"long-seg{n}-split")


def test_long_segments_in_graph_replays():
    """Steps of one shape whose filter segments are long enough for the
    parallel walk (next pointers per start, the chain, its links re-walked
    at once), captured as HIP graphs and replayed: every step equals an eager
    run and the oracle; the first step also grows the per-start slots (the
    step runs again)."""
    pats = [b"aaaaaaaa", b"aaaa", b"gcaacc", b"a" * 40, b"aaagaaa"]
    ks = [2, 1, 2, 8, 3]
    rng = np.random.default_rng(77)
    pieces = []
    for i in range(5):
        t = np.full(20000, ord("a"), dtype=np.uint8)
        pos = 0
        while pos < t.size:  # runs of 'a' of 100..3000 symbols
            pos += int(rng.integers(100, 3000))
            if pos < t.size:
                t[pos] = rng.choice(np.frombuffer(b"cgt", np.uint8))
        pieces.append(t)
    say("long segments in graph replays")
    outs = {}
    for graphs in (False, True):
        steps = []
        with oasm.Matcher(pats, ks, graphs=graphs) as mt:
            for i, t in enumerate(pieces):
                mt.feed(i, torch.from_numpy(t).cuda(), last=True)
                mt.sync()
                steps.append(mt.results())
            replays = mt.stats()["graph_replays"]
        outs[graphs] = (steps, replays)
    assert outs[False][1] == 0 and outs[True][1] >= 2
    for a, b in zip(outs[False][0], outs[True][0]):
        assert np.array_equal(a.raw, b.raw) and np.array_equal(a.occ, b.occ)
    streams = {i: t for i, t in enumerate(pieces)}
    merged = oasm.Results(np.concatenate([s.raw for s in outs[True][0]]),
                          np.concatenate([s.occ for s in outs[True][0]]))
    compare(merged, streams, pats, ks, label="long-graphs")


def test_k_zero_and_edge_streams():
    pats = [b"ACGT", b"A", b"TTTTT", b"GATTACA"]
    ks = [0, 0, 1, 0]
    streams = {
        1: np.frombuffer(b"", np.uint8).copy(),
        2: np.frombuffer(b"A", np.uint8).copy(),
        3: np.frombuffer(b"ACG", np.uint8).copy(),
        4: np.frombuffer(b"ACGTACGTGATTACAGATTACATTTTTTT", np.uint8).copy(),
        5: np.frombuffer(b"\x00\xff" * 50, np.uint8).copy(),
    }
    res = run(pats, ks, streams)
    compare(res, streams, pats, ks, check_h=True, label="edges")


@pytest.mark.parametrize("chunk", [64, 128, 448, 1024])
def test_small_chunks_cross_lookback(chunk):
    """Chunks shorter than many look-backs: every chunk boundary is crossed by hits."""
    w = W.small_random(21, 8000, 40, 20, 120, b"ACGT", kmax=12, n_plants=60, n_streams=2)
    streams = {i: s for i, s in enumerate(w.streams)}
    res = run(w.patterns, w.ks, streams, chunk_bytes=chunk)
    compare(res, streams, w.patterns, w.ks, check_h=True, label=f"chunk{chunk}")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_split_feeds_match_whole(seed):
    """Any split of the feeds, with a sync after each piece, gives the same
    hit ends, hit set and occurrences (filter segments carried across syncs)."""
    w = W.small_random(30 + seed, 5000, 30, 6, 60, b"ACG", kmax=8, n_plants=40, n_streams=4)
    streams = {100 + i: s for i, s in enumerate(w.streams)}
    res = run(w.patterns, w.ks, streams, pieces=seed)
    compare(res, streams, w.patterns, w.ks, check_h=True, label=f"split{seed}")


def test_plain_equals_batched_and_device_feed():
    w = W.small_random(40, 20000, 64, 8, 64, b"ACGTN", kmax=6, n_plants=50, n_streams=6)
    streams = {i: s for i, s in enumerate(w.streams)}
    a = run(w.patterns, w.ks, streams, plain=True)
    b = run(w.patterns, w.ks, streams, device=True)
    for x, y in ((a.raw, b.raw), (a.occ, b.occ), (a.h, b.h)):
        assert np.array_equal(np.sort(x, order=list(x.dtype.names)), np.sort(y, order=list(y.dtype.names)))
    compare(b, streams, w.patterns, w.ks, label="device-feed")


def test_feed_many_equals_single_feeds():
    """One batched device feed (pieces of several streams, a stream in
    several pieces, closes inside the call) gives the same results as one
    call per piece, equal to the oracle's; a piece for a stream closed earlier
    in the call is refused and nothing of the call is fed."""
    w = W.small_random(45, 20000, 40, 8, 100, b"ACGT", kmax=8, n_plants=60, n_streams=5)
    streams = {i: s for i, s in enumerate(w.streams)}
    dev = {i: torch.from_numpy(s).cuda() for i, s in streams.items() if s.size}
    items = []
    for i, t in dev.items():  # each stream in two pieces, the second closes it
        h = t.numel() // 3
        items.append((i, t[:h], False))
    for i, t in dev.items():
        items.append((i, t[t.numel() // 3:], True))
    with oasm.Matcher(w.patterns, w.ks, keep_h=True) as mt:
        mt.feed_many(items)
        for i in streams:
            if i not in dev:
                mt.close(i)
        mt.sync()
        a = mt.results()
    b = run(w.patterns, w.ks, streams, device=True)
    for x, y in ((a.raw, b.raw), (a.occ, b.occ), (a.h, b.h)):
        assert np.array_equal(np.sort(x, order=list(x.dtype.names)), np.sort(y, order=list(y.dtype.names)))
    compare(a, streams, w.patterns, w.ks, check_h=True, label="feed-many")
    t0 = next(iter(dev.values()))
    with oasm.Matcher(w.patterns, w.ks) as mt:
        with pytest.raises(oasm.OasmError) as ei:
            mt.feed_many([(7, t0, True), (8, t0, False), (7, t0, False)])
        assert ei.value.status == oasm.OASM_E_CLOSED
        assert mt.stats()["cells"] == 0  # nothing of the refused call was fed
        mt.feed_many([(7, t0, True)])
        mt.sync()
        assert mt.stats()["bytes_scanned"] == t0.numel()
        # stream 7 is finished (its slot may be reused): feeds and closes to it are refused
        with pytest.raises(oasm.OasmError) as ei:
            mt.feed_many([(7, t0, False)])
        assert ei.value.status == oasm.OASM_E_CLOSED
        with pytest.raises(oasm.OasmError) as ei:
            mt.feed(7, t0)
        assert ei.value.status == oasm.OASM_E_CLOSED
        with pytest.raises(oasm.OasmError):
            mt.close(7)


def test_autotuned_variants_match_oracle():
    """With the autotuner on, every pattern class runs the variant it measured
    fastest (patterns per lane, masks in LDS or L1/L2); results are unchanged."""
    w = W.small_random(50, 6000, 300, 8, 200, bytes(range(256)), kmax=20, n_plants=60, n_streams=2)
    streams = {i: s for i, s in enumerate(w.streams)}
    res = run(w.patterns, w.ks, streams, autotune=True)
    compare(res, streams, w.patterns, w.ks, check_h=True, label="autotuned")


def test_rules_none_reports_hits_only():
    w = W.small_random(41, 4000, 10, 8, 20, b"ACGT", kmax=3, n_plants=20)
    streams = {0: w.streams[0]}
    res = run(w.patterns, w.ks, streams, rules=oasm.OASM_RULES_NONE)
    assert res.occ.size == 0
    compare(res, streams, w.patterns, w.ks, check_h=True, with_filter=False, label="rules-none")


@pytest.mark.parametrize("rules", [
    oasm.OASM_RULES_ACC_LAST, oasm.OASM_RULES_EQ3_GE, oasm.OASM_RULES_START_ORDER, oasm.OASM_RULES_DISJOINT,
    oasm.OASM_RULES_ACC_LAST | oasm.OASM_RULES_DISJOINT,
    oasm.OASM_RULES_ACC_LAST | oasm.OASM_RULES_EQ3_GE | oasm.OASM_RULES_START_ORDER | oasm.OASM_RULES_DISJOINT,
])
def test_rule_variants_match_oracle(rules):
    """Alternative readings of Alg. 1: short patterns with K up to m - 1 on
    low-entropy text, where emissions hold several priority levels and the
    readings disagree; split feeds so open segments are carried."""
    rules |= oasm.OASM_RULES_PAPER
    w = W.small_random(70, 6000, 24, 4, 14, b"AB", kmax=None, n_plants=40, n_streams=3)
    ks = [max(1, min(len(p) - 1, 1 + (i % 5))) for i, p in enumerate(w.patterns)]
    streams = {i: s for i, s in enumerate(w.streams)}
    say(f"rules {rules}")
    res = run(w.patterns, ks, streams, rules=rules, pieces=rules)
    compare(res, streams, w.patterns, ks, check_h=True, label=f"rules{rules}", rules=rules)
    base = run(w.patterns, ks, streams)
    assert not np.array_equal(np.sort(res.occ, order=list(res.occ.dtype.names)),
                              np.sort(base.occ, order=list(base.occ.dtype.names))) or rules == 1


def test_graph_replays_equal_eager():
    """Steps of one repeated shape are captured as HIP graphs on the second
    occurrence and replayed afterwards; every replayed step (with eager feeds,
    drains and synchronisations in between) must equal an eager run."""
    w = W.small_random(60, 30000, 40, 8, 90, b"ACGT", kmax=8, n_plants=0)
    rng = np.random.default_rng(60)
    pieces = []
    for i in range(6):  # six streams of one length: six steps of one shape
        t = rng.integers(65, 69, size=30000).astype(np.uint8)
        for q in range(20):  # planted copies so every step has hits
            p = w.patterns[int(rng.integers(0, len(w.patterns)))]
            o = int(rng.integers(0, t.size - len(p)))
            t[o:o + len(p)] = np.frombuffer(p, np.uint8)
        pieces.append(t)
    outs = {}
    for graphs in (False, True):
        steps = []
        with oasm.Matcher(w.patterns, w.ks, graphs=graphs) as mt:
            for i, t in enumerate(pieces):
                mt.feed(i, torch.from_numpy(t).cuda(), last=True)
                mt.sync()
                steps.append(mt.results())
            replays = mt.stats()["graph_replays"]
        outs[graphs] = (steps, replays)
    assert outs[False][1] == 0 and outs[True][1] >= 4
    for a, b in zip(outs[False][0], outs[True][0]):
        assert np.array_equal(a.raw, b.raw) and np.array_equal(a.occ, b.occ)
    streams = {i: t for i, t in enumerate(pieces)}
    merged = oasm.Results(np.concatenate([s.raw for s in outs[True][0]]),
                          np.concatenate([s.occ for s in outs[True][0]]))
    compare(merged, streams, w.patterns, w.ks, label="graphs")
