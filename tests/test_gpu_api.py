"""Behaviour of the C ABI on the GPU beyond parity (needs an MI355X): drains
with a small capacity, create/destroy cycles, admission refusal under a
memory budget followed by progress, and byte-by-byte feeds.  Every result is
still compared with the oracle."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_1712_03560_amd import oasm  # noqa: E402
from paper_1712_03560_amd import workloads as W  # noqa: E402


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


def check_against_oracle(res, patterns, ks, text, stream=0):
    for p in range(len(patterns)):
        want = oracle.run_pair(patterns[p], text, int(ks[p]))
        sel = res.raw[(res.raw["pattern"] == p) & (res.raw["stream"] == stream)]
        assert np.array_equal(sel["end"].astype(np.int64), want.ends), p
        assert np.array_equal(sel["dist"].astype(np.int64), want.dists), p
        occ = res.occ[(res.occ["pattern"] == p) & (res.occ["stream"] == stream)]
        got = np.stack([occ["start"].astype(np.int64), occ["len"].astype(np.int64), occ["k"].astype(np.int64)], 1)
        assert np.array_equal(got, want.occ.reshape(-1, 3)), p


def test_drain_with_small_capacity():
    w = W.tiny(n=30_000, n_plants=60)
    t = w.streams[0]
    say("drain in pieces of 7 records")
    with oasm.Matcher(w.patterns, w.ks) as mt:
        mt.feed(3, t, last=True)
        mt.sync()
        total = oasm.oasm_queued(mt.ctx, oasm.OASM_RAW)
        assert total > 100
        parts = []
        more = ctypes.c_int(1)
        while more.value:
            buf = np.empty(7, dtype=oasm.HIT_DTYPE)
            n = ctypes.c_size_t(0)
            st = oasm.lib.oasm_hits(mt.ctx, oasm.OASM_RAW, buf.ctypes.data_as(ctypes.c_void_p), 7, ctypes.byref(n),
                                    ctypes.byref(more))
            assert st == oasm.OASM_OK
            assert n.value == 7 or not more.value
            parts.append(buf[:n.value])
        raw = np.concatenate(parts)
        assert raw.size == total and oasm.oasm_queued(mt.ctx, oasm.OASM_RAW) == 0
        occ = oasm.oasm_hits(mt.ctx, oasm.OASM_FILTERED)
    check_against_oracle(oasm.Results(raw, occ), w.patterns, w.ks, t, stream=3)


def test_create_destroy_cycles():
    w = W.small_random(31, 5_000, 6, 4, 40, b"ACGT", 4, n_plants=20)
    t = w.streams[0]
    dev = torch.from_numpy(t).cuda()
    torch.cuda.synchronize()
    first = None
    free = []
    say("20 create / feed / sync / destroy cycles")
    for i in range(20):
        if i in (2, 19):  # after the first cycles: code objects and process-wide caches are loaded
            torch.cuda.synchronize()
            free.append(torch.cuda.mem_get_info()[0])
        with oasm.Matcher(w.patterns, w.ks, graphs=bool(i % 2)) as mt:
            mt.feed(i, dev, last=True)
            mt.sync()
            res = mt.results()
        key = (res.raw["end"].tobytes(), res.raw["dist"].tobytes(), res.occ["start"].tobytes(), res.occ["len"].tobytes())
        if first is None:
            first = key
            check_against_oracle(res, w.patterns, w.ks, t, stream=i)
        assert key == first
    say(f"device memory held across cycles 2..19: {(free[0] - free[1]) / 2**20:.1f} MiB")
    assert free[0] - free[1] < (16 << 20), f"{(free[0] - free[1]) >> 20} MiB not returned over 17 cycles"


def test_budget_refusal_then_progress():
    """Feeds beyond the unmatched-byte budget are refused with OASM_E_AGAIN;
    after a sync the same feed is accepted, and the results are exact."""
    w = W.small_random(32, 40_000, 8, 6, 30, b"ACGT", 3, n_plants=40)
    t = w.streams[0]
    budget = 10_000
    pieces = [t[i:i + 4_000] for i in range(0, t.size, 4_000)]
    refused = 0
    say(f"budget {budget} bytes, {len(pieces)} pieces of 4000")
    with oasm.Matcher(w.patterns, w.ks, mem_budget=budget) as mt:
        for k, piece in enumerate(pieces):
            last = k == len(pieces) - 1
            try:
                mt.feed(0, piece, last=last)
            except oasm.OasmError as e:
                assert e.status == oasm.OASM_E_AGAIN
                refused += 1
                mt.sync()  # matches what is pending; the budget frees up
                mt.feed(0, piece, last=last)
        mt.sync()
        res = mt.results()
    assert refused >= len(pieces) // 3
    check_against_oracle(res, w.patterns, w.ks, t)


def test_byte_by_byte_feeds():
    pats = [b"ACGTA", b"TTT", b"GATTACA", b"CC"]
    ks = [1, 0, 2, 1]
    rng = np.random.default_rng(5)
    t = rng.choice(np.frombuffer(b"ACGT", dtype=np.uint8), 97)
    t[40:47] = np.frombuffer(b"GATTACA", dtype=np.uint8)
    say("97 one-byte feeds, a sync after each")
    with oasm.Matcher(pats, ks) as mt:
        for i in range(t.size):
            mt.feed(0, t[i:i + 1], last=i == t.size - 1)
            mt.sync()
        res = mt.results()
    check_against_oracle(res, pats, ks, t)


def test_feeds_from_many_threads():
    """Calls on one context are serialised inside the library: eight host
    threads feed their own streams in pieces at the same time (ctypes lets
    them run concurrently), then one sync; every stream equals the oracle."""
    import threading

    w = W.small_random(33, 6_000, 10, 6, 40, b"ACGT", 4, n_plants=30, n_streams=8)
    say("8 threads feeding 8 streams concurrently")
    errors = []
    with oasm.Matcher(w.patterns, w.ks) as mt:
        def worker(sid, t):
            try:
                cuts = list(range(0, t.size, 397)) + [t.size]
                for a, b in zip(cuts[:-1], cuts[1:]):
                    mt.feed(sid, t[a:b], last=b == t.size)
                if t.size == 0:
                    mt.feed(sid, t, last=True)
            except Exception as e:  # reported below
                errors.append(e)

        threads = [threading.Thread(target=worker, args=(100 + i, t)) for i, t in enumerate(w.streams)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        assert not errors, errors
        mt.sync()
        res = mt.results()
    for i, t in enumerate(w.streams):
        check_against_oracle(res, w.patterns, w.ks, t, stream=100 + i)


def test_small_pieces_long_patterns():
    """Long patterns (m up to 256: the multi-word and cutoff scan variants)
    fed in pieces shorter than their look-back at first, then longer ones,
    with a sync after each round: every step moves an overlapping tail (up to
    m_max + K_max + 3 symbols, more than a workgroup's 256 threads) to the
    front of its staging buffer, and the growing pieces outgrow the buffers,
    through the batched device feed (copies queued with the tail moves) on
    two streams and the single host feed (a copy of its own) on a third.
    Every stream equals the oracle."""
    w = W.small_random(34, 12_000, 12, 150, 256, b"ACGT", 25, n_plants=40, n_streams=3)
    texts = [np.ascontiguousarray(t) for t in w.streams]
    devs = [torch.from_numpy(t).cuda() for t in texts]
    torch.cuda.synchronize()
    pos = [0, 0, 0]
    size = 37.0
    rounds = 0
    say(f"stream lengths {[t.size for t in texts]}, m up to {max(len(p) for p in w.patterns)}")
    with oasm.Matcher(w.patterns, w.ks) as mt:
        while any(pos[i] < texts[i].size for i in range(3)) or rounds == 0:
            n = int(size)
            items = []
            for i in (0, 1):
                a, b = pos[i], min(pos[i] + n, texts[i].size)
                if a < texts[i].size or (a == 0 and texts[i].size == 0 and rounds == 0):
                    items.append((10 + i, devs[i][a:b], b == texts[i].size))
                pos[i] = b
            if items:
                mt.feed_many(items)
            a, b = pos[2], min(pos[2] + n, texts[2].size)
            if a < texts[2].size or (texts[2].size == 0 and rounds == 0):
                mt.feed(12, texts[2][a:b], last=b == texts[2].size)
            pos[2] = b
            mt.sync()
            size = min(size * 1.35, 1500.0)
            rounds += 1
        res = mt.results()
    say(f"{rounds} rounds, {res.raw.size} hit ends, {res.occ.size} occurrences")
    assert rounds >= 8
    assert res.raw.size > 0 and res.occ.size > 0  # the planted copies are found
    for i, t in enumerate(texts):
        check_against_oracle(res, w.patterns, w.ks, t, stream=10 + i)
