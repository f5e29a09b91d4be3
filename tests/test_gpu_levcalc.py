"""Parity of the LEV CALC kernel (every start's 2K+1 distances) with the
oracle (needs an MI355X).

Exact comparisons of every output byte on seeded inputs that span several
256-start passes with a ragged tail, every word boundary of the pattern
column and the degenerate texts (empty, shorter than the pattern); at the
long workload's size, sampled starts against the oracle and the entries
<= K against the hit set the scan path recovers on the same text.
"""
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


def units(ks):
    w = 2 * np.asarray(ks, dtype=np.int64) + 1
    return np.concatenate([[0], np.cumsum(w)[:-1]]), w


def gpu_levcalc(patterns, ks, text: np.ndarray):
    """The device output, split per pattern into [n, 2K+1] arrays."""
    with oasm.Matcher(patterns, ks) as mt:
        dev = torch.from_numpy(text).cuda() if text.size else torch.empty(0, dtype=torch.uint8, device="cuda")
        out = mt.levcalc(dev)
        torch.cuda.synchronize()
        flat = out.cpu().numpy()
    n = text.size
    off, w = units(ks)
    assert flat.size == n * int(w.sum())
    return [flat[n * off[p]: n * (off[p] + w[p])].reshape(n, w[p]) for p in range(len(patterns))]


def check_all(patterns, ks, text, label):
    got = gpu_levcalc(patterns, ks, text)
    want = oracle.levcalc_many(patterns, ks, text)
    for p in range(len(patterns)):
        if not np.array_equal(got[p], want[p]):
            bad = np.argwhere(got[p] != want[p])[:5]
            raise AssertionError(f"{label}: pattern {p} (m={len(patterns[p])}, K={ks[p]}) differs at "
                                 f"(start, j) {bad.tolist()}: got {[int(got[p][tuple(b)]) for b in bad]} "
                                 f"want {[int(want[p][tuple(b)]) for b in bad]}")
    return sum(int((g <= k).sum()) for g, k in zip(got, ks))


def test_tiny_config_full():
    w = W.tiny()
    say("levcalc tiny: 100,000 ACGT symbols, 16 patterns, K=2")
    h = check_all(w.patterns, w.ks, w.streams[0], "tiny")
    assert h > 200  # the planted copies alone give more


@pytest.mark.parametrize("seed,n,mlo,mhi,alphabet,kmax", [
    (1, 777, 1, 8, b"AB", None),
    (2, 1283, 8, 40, b"ACGT", 8),
    (3, 515, 30, 70, bytes(range(256)), 10),
    (4, 300, 60, 140, b"ACGT", 20),
    (5, 257, 120, 256, bytes([0, 255, 7]), 40),
    (6, 600, 200, 256, b"ACGT", 63),
    (7, 700, 100, 256, bytes(range(256)), 30),  # every byte row of the even-W mask tables
])
def test_random_dictionaries(seed, n, mlo, mhi, alphabet, kmax):
    w = W.small_random(seed, n, 12, mlo, mhi, alphabet, kmax, n_plants=6)
    say(f"levcalc random seed={seed} n={n} m=[{mlo},{mhi}] sigma={len(alphabet)} kmax={kmax}")
    check_all(w.patterns, w.ks, w.streams[0], f"seed {seed}")


def test_every_word_boundary():
    rng = np.random.default_rng(11)
    ms = [1, 2, 31, 32, 33, 63, 64, 65, 95, 96, 97, 127, 128, 129, 192, 193, 255, 256]
    pats = [bytes(rng.integers(0, 4, m).astype(np.uint8) + 65) for m in ms]
    ks = [int(rng.integers(0, min(m, 64))) for m in ms]
    text = (rng.integers(0, 4, 700).astype(np.uint8) + 65)
    for p in pats[::3]:  # exact copies so that small distances occur
        s = int(rng.integers(0, text.size - len(p)))
        text[s:s + len(p)] = np.frombuffer(p, dtype=np.uint8)
    say("levcalc word boundaries m in " + ",".join(map(str, ms)))
    check_all(pats, ks, text, "word boundaries")


def test_degenerate_texts():
    pats = [b"ACGTACGT", b"A", b"TTTTTTTTTTTTTTTTTTTTTTTTTTTTTTTTTTTTTTTTT"]
    ks = [3, 0, 9]
    for n in (0, 1, 5, 8, 40, 256, 257):
        text = np.frombuffer((b"ACGT" * 100)[:n], dtype=np.uint8).copy()
        say(f"levcalc degenerate n={n}")
        check_all(pats, ks, text, f"n={n}")
    # homopolymer text: dense hits at every start
    text = np.full(1000, ord("T"), dtype=np.uint8)
    assert check_all(pats, ks, text, "homopolymer") > 900


def test_rejects_small_output_and_null():
    with oasm.Matcher([b"ACGT"], 1) as mt:
        dev = torch.zeros(100, dtype=torch.uint8, device="cuda")
        small = torch.empty(299, dtype=torch.uint8, device="cuda")
        with pytest.raises(ValueError):
            mt.levcalc(dev, out=small)
        with pytest.raises(oasm.OasmError) as e:  # the library's own check
            oasm.oasm_levcalc(mt.ctx, dev.data_ptr(), 100, small.data_ptr(), small.numel(), None)
        assert e.value.status == oasm.OASM_E_INVAL
        with pytest.raises(oasm.OasmError):
            oasm.oasm_levcalc(mt.ctx, None, 100, small.data_ptr(), 300, None)
        assert oasm.oasm_levcalc_size(mt.ctx, 100) == 300


def test_long_workload_prefix():
    """8 MiB of the long stream x its 256 patterns (the benchmark's LEV CALC
    shape, same call): sampled (pattern, start) rows and every planted
    copy's start against the oracle, and all entries <= K against the hit set
    the scan path recovers on the same text."""
    n = 1 << 23
    w = W.long_stream()
    text = np.ascontiguousarray(w.streams[0][:n])
    K = 3
    assert all(int(k) == K for k in w.ks)
    width = 2 * K + 1
    say("levcalc long prefix: 8 MiB x 256 patterns, K=3")
    dev = torch.from_numpy(text).cuda()
    with oasm.Matcher(w.patterns, w.ks) as mt:
        out = mt.levcalc(dev)
        torch.cuda.synchronize()
    assert out.numel() == n * width * len(w.patterns)
    rng = np.random.default_rng(3)
    rows = [(int(rng.integers(0, len(w.patterns))), int(rng.integers(0, n))) for _ in range(1500)]
    rows += [(pl.pattern, pl.site) for pl in w.plants if pl.site + 64 < n]
    rows += [(0, n - 1), (255, n - 40), (17, 0)]
    idx = torch.tensor([(p * n + s) * width + j for p, s in rows for j in range(width)], dtype=torch.int64,
                       device="cuda")
    got_rows = out[idx].cpu().numpy().reshape(len(rows), width)
    for (p, s), g in zip(rows, got_rows):
        want = oracle.levcalc(w.patterns[p], text[s:s + len(w.patterns[p]) + K], K)[0]
        assert np.array_equal(g, want), (p, s, g.tolist(), want.tolist())
    # entries <= K (the hit set), decoded on the device
    per_pat = out.view(len(w.patterns), n * width)
    parts = []
    for p in range(len(w.patterns)):
        f = torch.nonzero(per_pat[p] <= K).view(-1)
        parts.append((p, f.cpu().numpy(), per_pat[p][f].cpu().numpy().astype(np.int64)))
    pat = np.concatenate([np.full(f.size, p, dtype=np.int64) for p, f, _ in parts])
    start, j = np.divmod(np.concatenate([f for _, f, _ in parts]), width)
    vals = np.concatenate([v for _, _, v in parts])
    with oasm.Matcher(w.patterns, w.ks, keep_h=True) as mt:
        mt.feed(0, dev, last=True)
        mt.sync()
        h = mt.results().h
    ms = np.array([len(p) for p in w.patterns], dtype=np.int64)
    mine = np.stack([pat, start, j + ms[pat] - K, vals], 1)
    theirs = np.stack([h["pattern"].astype(np.int64), h["start"].astype(np.int64), h["len"].astype(np.int64),
                       h["k"].astype(np.int64)], 1)
    mine = mine[np.lexsort(mine.T[::-1])]
    theirs = theirs[np.lexsort(theirs.T[::-1])]
    say(f"levcalc long prefix: {len(mine)} hit-set entries")
    assert len(mine) > 1000
    assert np.array_equal(mine, theirs)


def test_levcalc_between_feeds_on_a_side_stream():
    """LEV CALC calls queued on another HIP stream between the pieces of a
    streamed feed change neither the matcher's results nor their own."""
    w = W.small_random(21, 30_000, 10, 8, 40, b"ACGT", 6, n_plants=40)
    t = w.streams[0]
    cuts = [0, 7_001, 15_000, 22_222, t.size]
    side = torch.cuda.Stream()
    dev = torch.from_numpy(t).cuda()
    with oasm.Matcher(w.patterns, w.ks, keep_h=True) as mt:
        outs = []
        for a, b in zip(cuts[:-1], cuts[1:]):
            mt.feed(0, t[a:b], last=b == t.size)
            with torch.cuda.stream(side):
                outs.append(mt.levcalc(dev[a:b].contiguous()))
            mt.sync()
        side.synchronize()
        res = mt.results()
    # the streamed matcher against the oracle (hit ends and occurrences)
    for p in range(len(w.patterns)):
        want = oracle.run_pair(w.patterns[p], t, int(w.ks[p]))
        sel = res.raw[res.raw["pattern"] == p]
        assert np.array_equal(sel["end"].astype(np.int64), want.ends)
        occ = res.occ[res.occ["pattern"] == p]
        got = np.stack([occ["start"].astype(np.int64), occ["len"].astype(np.int64), occ["k"].astype(np.int64)], 1)
        assert np.array_equal(got, want.occ.reshape(-1, 3))
    # each LEV CALC call against the oracle on its own piece
    for (a, b), out in zip(zip(cuts[:-1], cuts[1:]), outs):
        flat = out.cpu().numpy()
        off = 0
        n = b - a
        for p in range(len(w.patterns)):
            K = int(w.ks[p])
            got = flat[off:off + n * (2 * K + 1)].reshape(n, 2 * K + 1)
            assert np.array_equal(got, oracle.levcalc(w.patterns[p], t[a:b], K)), (a, p)
            off += n * (2 * K + 1)


def test_destroy_waits_for_levcalc():
    """A context destroyed right after a LEV CALC call (no synchronisation in
    between) leaves the queued kernels their dictionary tables."""
    w = W.long_stream(n=1 << 21, n_plants=100)
    text = w.streams[0]
    dev = torch.from_numpy(text).cuda()
    mt = oasm.Matcher(w.patterns, w.ks)
    out = mt.levcalc(dev)
    mt.destroy()
    torch.cuda.synchronize()
    n, K = text.size, 3
    rng = np.random.default_rng(9)
    for _ in range(300):
        p, s = int(rng.integers(0, len(w.patterns))), int(rng.integers(0, n))
        got = out[(p * n + s) * 7:(p * n + s) * 7 + 7].cpu().numpy()
        want = oracle.levcalc(w.patterns[p], text[s:s + len(w.patterns[p]) + K], K)[0]
        assert np.array_equal(got, want), (p, s)
