"""Checkpoint and resume of streams on the GPU (oasm_stream_export /
oasm_stream_import): a stream matched in pieces by a chain of contexts, each
resuming the previous one's checkpoint, reports together exactly what one
context reports for the whole stream, which is the oracle's result (hit ends,
distances, H and S per pattern).  Splits fall inside filter segments that are
still open, so carried hit ends travel in the checkpoints; other streams of
the exporting context stay untouched.  Invalid checkpoints are refused."""
import struct
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

HEADER = struct.Struct("<IIQQIIII")  # magic, version, dictionary, position, nsym, ncarry, hks, reserved


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


def concat(results):
    raw = np.concatenate([r.raw for r in results])
    occ = np.concatenate([r.occ for r in results])
    h = np.concatenate([r.h for r in results]) if all(r.h is not None for r in results) else None
    return oasm.Results(raw, occ, h)


def run_chain(patterns, ks, text, cuts, sid=7, keep_h=True, graphs=False):
    """Feed text[cuts[i]:cuts[i+1]] to context i, each resuming the previous
    context's checkpoint; returns the results of all contexts and the
    checkpoints."""
    bounds = [0] + list(cuts) + [len(text)]
    results, blobs, prev = [], [], None
    for i in range(len(bounds) - 1):
        m = oasm.Matcher(patterns, ks, keep_h=keep_h, graphs=graphs)
        try:
            if prev is not None:
                m.import_stream(sid, prev)
            last = i == len(bounds) - 2
            m.feed(sid, text[bounds[i]:bounds[i + 1]], last=last)
            if last:
                m.sync()
            else:
                prev = m.export_stream(sid)
                blobs.append(prev)
            results.append(m.results())
        finally:
            m.destroy()
    return concat(results), blobs


def header(blob):
    return HEADER.unpack_from(blob)


def test_resume_chain_equals_oracle_random():
    w = W.small_random(11, 60_000, 24, 4, 70, b"acgt", kmax=9, n_plants=300)
    text = w.streams[0]
    for cuts in ([1], [17, 18, 19], [9_999, 30_001, 45_000], [59_999]):
        say(f"random dictionary, cuts {cuts}")
        res, blobs = run_chain(w.patterns, w.ks, text, cuts)
        for b in blobs:
            magic, version, _, position, nsym, ncarry, hks, _ = header(b)
            assert (magic, version) == (oasm.OASM_CKPT_MAGIC, oasm.OASM_CKPT_VERSION)
            assert position in cuts and nsym <= position
        compare(res, {7: text}, w.patterns, w.ks, check_h=True, label=f"cuts {cuts}")


def test_resume_inside_open_segments_carries_hit_ends():
    # homopolymer runs: hit ends at every position, so a cut inside a run
    # leaves filter segments open and their hit ends travel in the checkpoint
    rng = np.random.default_rng(3)
    text = np.frombuffer(b"a" * 5000 + b"cgt" * 300 + b"a" * 7000, np.uint8).copy()
    text[rng.integers(0, text.size, 40)] = ord("g")
    pats = [b"aaaaaaaa", b"aaaa", b"gcaacc", b"acgttgca", b"a" * 40]
    ks = np.array([2, 1, 2, 2, 8], np.uint16)
    cuts = [2_500, 2_501, 6_000, 9_000]
    say(f"homopolymer runs, cuts {cuts}")
    res, blobs = run_chain(pats, ks, text, cuts)
    carried = [header(b)[5] for b in blobs]
    assert carried[0] > 0 and carried[3] > 0, carried
    compare(res, {7: text}, pats, ks, check_h=True, label="homopolymer cuts")


def test_export_leaves_other_streams_and_the_exported_stream_running():
    w = W.small_random(12, 40_000, 16, 6, 40, b"acgt", kmax=6, n_plants=200, n_streams=3)
    texts = {10 + i: t for i, t in enumerate(w.streams)}
    half = {sid: t.size // 2 for sid, t in texts.items()}
    m = oasm.Matcher(w.patterns, w.ks)
    fork = oasm.Matcher(w.patterns, w.ks)
    try:
        for sid, t in texts.items():
            m.feed(sid, t[:half[sid]])
        say("export stream 11 from a context of three streams")
        blob = m.export_stream(11)
        first = m.results()
        fork.import_stream(11, blob)
        # the same stream in the same context under another id, too
        m.import_stream(99, blob)
        for sid, t in texts.items():
            m.feed(sid, t[half[sid]:], last=True)
        m.feed(99, texts[11][half[11]:], last=True)
        fork.feed(11, texts[11][half[11]:], last=True)
        m.sync()
        fork.sync()
        rest, frk = m.results(), fork.results()
    finally:
        m.destroy()
        fork.destroy()
    whole = concat([first, rest])
    sel = lambda r, sid: oasm.Results(r.raw[r.raw["stream"] == sid], r.occ[r.occ["stream"] == sid], None)  # noqa: E731
    compare(oasm.Results(whole.raw[whole.raw["stream"] != 99], whole.occ[whole.occ["stream"] != 99], None), texts,
            w.patterns, w.ks, label="three streams")
    # the copies resumed from the checkpoint report what stream 11 reported after it
    after11 = sel(rest, 11)
    for r in (sel(frk, 11), sel(rest, 99)):
        for f in ("raw", "occ"):
            a, b = getattr(r, f).copy(), getattr(after11, f).copy()
            a["stream"] = b["stream"] = 0
            assert np.array_equal(a, b), f


def test_resume_with_graphs_and_long_patterns():
    w = W.small_random(13, 50_000, 40, 30, 256, bytes(range(32, 127)), kmax=25, n_plants=150)
    text = w.streams[0]
    cuts = [12_345, 12_346, 33_333]
    say(f"patterns up to 256 bytes, graphs on, cuts {cuts}")
    res, _ = run_chain(w.patterns, w.ks, text, cuts, graphs=True)
    compare(res, {7: text}, w.patterns, w.ks, check_h=True, label="long patterns")


def test_invalid_checkpoints_are_refused():
    w = W.small_random(14, 5_000, 8, 4, 20, b"acgt", kmax=3)
    text = w.streams[0]
    m = oasm.Matcher(w.patterns, w.ks)
    other = oasm.Matcher(w.patterns[:-1], w.ks[:-1])
    try:
        m.feed(1, text[:3000])
        blob = m.export_stream(1)

        def refused(ctx, sid, b, code=oasm.OASM_E_INVAL):
            with pytest.raises(oasm.OasmError) as e:
                ctx.import_stream(sid, b)
            assert e.value.status == code, (e.value.status, str(e.value))

        refused(other, 1, blob)                      # another dictionary
        refused(m, 1, blob)                          # the id is live in this context
        refused(m, 2, blob[:-1])                     # truncated
        refused(m, 2, blob[:20])
        bad = bytearray(blob)
        bad[0] ^= 1
        refused(m, 2, bytes(bad))                    # magic
        bad = bytearray(blob)
        bad[4] = 9
        refused(m, 2, bytes(bad))                    # version
        bad = bytearray(blob)
        struct.pack_into("<I", bad, 24, 10_000)      # more look-back symbols than the context keeps
        refused(m, 2, bytes(bad))
        with pytest.raises(oasm.OasmError) as e:
            m.export_stream(5)                       # unknown stream
        assert e.value.status == oasm.OASM_E_INVAL
        m.feed(1, text[3000:], last=True)
        with pytest.raises(oasm.OasmError) as e:
            m.export_stream(1)                       # a close is pending
        assert e.value.status == oasm.OASM_E_INVAL
        m.sync()
        with pytest.raises(oasm.OasmError) as e:
            m.export_stream(1)                       # closed
        assert e.value.status == oasm.OASM_E_CLOSED
        m.import_stream(2, blob)                     # a valid one still imports
        m.feed(2, text[3000:], last=True)
        m.sync()
    finally:
        m.destroy()
        other.destroy()


def test_resume_at_full_size_equals_one_context():
    """The 64 MiB stream of 256 patterns (10,000 planted copies, so that
    open segments cross the cut) matched by two contexts, the second
    resuming the first's checkpoint, reports what one context reports for
    the whole stream (which the full-size parity tests compare with the
    oracle)."""
    w = W.long_stream()
    text = w.streams[0]
    # the cut falls one byte before the end of a planted copy near the middle,
    # so that the copy's hit ends straddle it and its segment is carried
    mid = min(w.plants, key=lambda pl: abs(pl.site - text.size // 2))
    cut = mid.site + mid.length - 1
    say(f"64 MiB stream, 256 patterns, cut at {cut}")
    dt = torch.from_numpy(text).cuda()

    def feed(m, sid, lo, hi, last):
        m.feed(sid, dt[lo:hi], last=last)

    whole = oasm.Matcher(w.patterns, w.ks)
    try:
        feed(whole, 3, 0, text.size, True)
        whole.sync()
        one = whole.results()
    finally:
        whole.destroy()
    a = oasm.Matcher(w.patterns, w.ks)
    b = oasm.Matcher(w.patterns, w.ks)
    try:
        feed(a, 3, 0, cut, False)
        blob = a.export_stream(3)
        first = a.results()
        b.import_stream(3, blob)
        feed(b, 3, cut, text.size, True)
        b.sync()
        second = b.results()
    finally:
        a.destroy()
        b.destroy()
    assert header(blob)[5] > 0  # hit ends were carried across the cut
    both = concat([first, second])
    for f in ("raw", "occ"):
        x = np.sort(getattr(both, f), order=["pattern", "stream"], kind="stable")
        y = np.sort(getattr(one, f), order=["pattern", "stream"], kind="stable")
        assert x.size == y.size and np.array_equal(x, y), f
