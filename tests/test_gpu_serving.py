"""The continuous-batching loop (needs an MI355X): every session's results are
the same alone and in the mix, equal to the oracle on the session's
concatenated bytes, with and without a memory budget that defers admissions."""
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


def make_trace(seed=5, sessions=40, pool_bytes=1 << 20, duration=0.05):
    rng = np.random.default_rng(seed)
    pats = W.make_patterns(rng, 48, 12, 70, W.LETTERS_ACGT)
    ks = np.array([min(len(p) // 6, 6) for p in pats], dtype=np.uint16)
    pool = W.LETTERS_ACGT.draw(rng, pool_bytes)
    W.plant(rng, pool, pats, 400, ks, W.LETTERS_ACGT)
    rows = []
    for s in range(sessions):
        nseg = int(rng.integers(2, 8))
        times = np.sort(rng.uniform(0, duration, size=nseg))
        for j, t in enumerate(times):
            ln = int(rng.integers(1, 4096))
            off = int(rng.integers(0, pool_bytes - ln))
            rows.append((1000 + s, off, ln, oasm.OASM_FEED_LAST if j == nseg - 1 else 0, float(t)))
    rows.sort(key=lambda r: r[4])
    segs = np.array(rows, dtype=oasm.SEG_DTYPE)
    return pats, ks, pool, segs


def session_bytes(pool, segs, sid):
    parts = [pool[int(r["offset"]):int(r["offset"]) + int(r["len"])] for r in segs if int(r["stream"]) == sid]
    return np.concatenate(parts) if parts else np.zeros(0, np.uint8)


def serve(pats, ks, dpool, segs, budget=0):
    with oasm.Matcher(pats, ks, mem_budget=budget) as mt:
        rep, lat = mt.serve(segs, dpool)
        res = mt.results()
    return rep, lat, res


def rows_of(res, sid):
    r = res.raw[res.raw["stream"] == sid]
    o = res.occ[res.occ["stream"] == sid]
    return np.sort(r, order=["pattern", "end"]), np.sort(o, order=["pattern", "start"])


@pytest.mark.parametrize("budget", [0, 6000])
def test_alone_equals_mix_equals_oracle(budget):
    pats, ks, pool, segs = make_trace()
    dpool = torch.from_numpy(pool).cuda()
    rep, lat, mix = serve(pats, ks, dpool, segs, budget)
    print(f"[serving] budget {budget}: {rep}", file=sys.stderr, flush=True)
    assert rep["segments"] == segs.size and rep["bytes"] == int(segs["len"].sum())
    assert (lat >= 0).all()
    if budget:
        assert rep["deferred"] > 0 and rep["steps"] > 1
    sids = sorted(set(int(x) for x in segs["stream"]))
    # alone: three sessions, each served by itself
    for sid in sids[:3]:
        _, _, alone = serve(pats, ks, dpool, segs[segs["stream"] == sid])
        a_raw, a_occ = rows_of(alone, sid)
        m_raw, m_occ = rows_of(mix, sid)
        assert np.array_equal(a_raw, m_raw) and np.array_equal(a_occ, m_occ), f"session {sid} differs alone/mix"
    # oracle on every session's concatenated bytes
    streams = {sid: session_bytes(pool, segs, sid) for sid in sids}
    compare(mix, streams, pats, ks, label=f"serving-budget{budget}")


@pytest.mark.timeout(900)
def test_serving_full_size_sampled_sessions():
    """The serving workload at the benchmark's size and settings (10,000
    sessions, 2048 patterns of 16..128 mixture bytes, K = floor(m/10), U[1,64]
    KiB segments arriving at 20 GB/s over 50 ms, a 64 MiB budget, autotuned
    variants), with 20,000 mutated pattern copies planted in the byte pool:
    1 % of the 10,000 sessions (100, seeded) against the oracle on their
    concatenated bytes (every pattern), and 2 of them alone against the mix."""
    pats, ks = W.serving_dictionary()
    pool = W.serving_pool(1 << 26)
    # mutated copies of the patterns in the pool, so that the sessions hold hits
    W.plant(np.random.default_rng(23), pool, pats, 20_000, ks, W.LETTERS_MIX)
    sess, off, ln, t = W.serving_arrivals(10_000, 0.05, 20.0, pool.size)
    segs = np.zeros(t.size, dtype=oasm.SEG_DTYPE)
    segs["stream"], segs["offset"], segs["len"], segs["arrival_s"] = sess, off, ln, t
    dpool = torch.from_numpy(pool).cuda()
    print(f"[serving] full size: {segs.size} segments, {int(ln.sum())} bytes", file=sys.stderr, flush=True)
    sids = sorted(set(int(x) for x in segs["stream"]))
    # the trace leaves its sessions open: each session is closed after the
    # run, so that its last filter segment (still pending when the run ends)
    # completes as in the oracle, which filters each session as a finished
    # stream
    with oasm.Matcher(pats, ks, mem_budget=64 << 20, autotune=True) as mt:
        rep, lat = mt.serve(segs, dpool)
        for sid in sids:
            mt.close(sid)
        mt.sync()
        mix = mt.results()
    assert rep["segments"] == segs.size and rep["deferred"] > 0
    pick = [int(x) for x in np.random.default_rng(17).choice(sids, 100, replace=False)]
    for sid in pick[:2]:
        with oasm.Matcher(pats, ks, autotune=True) as mt:
            mt.serve(segs[segs["stream"] == sid].copy(), dpool, want_latency=False)
            mt.close(sid)
            mt.sync()
            alone = mt.results()
        a_raw, a_occ = rows_of(alone, sid)
        m_raw, m_occ = rows_of(mix, sid)
        assert np.array_equal(a_raw, m_raw) and np.array_equal(a_occ, m_occ), f"session {sid} differs alone/mix"
    streams = {sid: session_bytes(pool, segs, sid) for sid in pick}
    pairs = [(sid, p) for sid in pick for p in range(len(pats))]
    n_raw, n_occ = compare(mix, streams, pats, ks, pairs=pairs, label="serving-full-size")
    assert n_raw > 400 and n_occ > 80
