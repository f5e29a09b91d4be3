"""The two facts a stream checkpoint rests on, checked with the oracle on the
CPU (the GPU tests of oasm_stream_export / oasm_stream_import check the
library itself).

A checkpoint at a frontier c keeps the last min(c, m + K + 3) symbols and the
hit ends of the filter segments still open at c (those whose last end e has
e + m + K > c: a later end, at c or beyond, can still join them).  Then:

* the scan restarted on those symbols reports exactly the hit ends >= c of
  the whole stream (Section 5.1: the last row at e depends on the m + K - 1
  symbols before e only, through the free start of Eq. 1), with their least
  distances;
* Alg. 1 over the closed segments, then over the carried ends together with
  the new ones, gives the whole stream's S (Section 4: the filter's state is
  empty between segments), and the hit set of a carried end, taken from the
  first part of the text, is the one the whole text gives."""
import numpy as np
import pytest

from oracle import oracle as O


def split_run(p, t, K, c):
    m = len(p)
    gap = m + K
    ends, dists = O.raw_hits(p, t, K)
    # the first context: the stream up to c
    e1, d1 = O.raw_hits(p, t[:c], K)
    assert np.array_equal(e1, ends[ends < c]) and np.array_equal(d1, dists[ends < c])
    # segments of the ends before c, and which are still open at c
    closed, carried = [], []
    seg = []
    for e in e1:
        if seg and e - seg[-1] >= gap:
            closed += seg
            seg = []
        seg.append(int(e))
    if seg:
        (carried if seg[-1] + gap > c else closed).extend(seg)
    S1 = O.filter_hits(*O.hset_at_ends(p, t[:c], K, closed), K, c).occ if closed else np.zeros((0, 3), np.int64)
    # the second context: the look-back symbols, then the rest of the stream
    L = min(c, m + K + 3)
    t2 = t[c - L:]
    e2, d2 = O.raw_hits(p, t2, K)
    keep = e2 + (c - L) >= c
    new_ends, new_d = e2[keep] + (c - L), d2[keep]
    assert np.array_equal(new_ends, ends[ends >= c]) and np.array_equal(new_d, dists[ends >= c])
    # hit sets: carried ends from the first part's text, new ones from the second
    hc = O.hset_at_ends(p, t[:c], K, carried)
    hn = O.hset_at_ends(p, t2, K, new_ends - (c - L))
    hs = np.concatenate([hc[0], hn[0] + (c - L)])
    hl = np.concatenate([hc[1], hn[1]])
    hk = np.concatenate([hc[2], hn[2]])
    whole = O.hset_at_ends(p, t, K, ends)
    got = sorted(zip(hs.tolist(), hl.tolist(), hk.tolist()))
    want = [h for h in zip(*(a.tolist() for a in whole)) if h[0] + h[1] - 1 in set(carried) | set(new_ends.tolist())]
    assert got == sorted(want)
    S2 = O.filter_hits(hs, hl, hk, K, len(t)).occ if hs.size else np.zeros((0, 3), np.int64)
    S = O.filter_hits(*whole, K, len(t)).occ
    both = np.concatenate([np.asarray(S1).reshape(-1, 3), np.asarray(S2).reshape(-1, 3)])
    assert np.array_equal(both, np.asarray(S).reshape(-1, 3)), (c, both[:6], S[:6])
    return len(carried)


def test_split_anywhere_random():
    rng = np.random.default_rng(17)
    carried = 0
    for it in range(60):
        m = int(rng.integers(2, 12))
        K = int(rng.integers(0, m))
        alpha = b"ab" if it % 3 == 0 else b"acgt"
        p = bytes(rng.choice(list(alpha), size=m))
        n = int(rng.integers(1, 300))
        if it % 2 == 0:  # repeats of the pattern with noise: open segments at the cuts
            t = bytearray((p * (n // m + 1))[:n])
            for _ in range(n // 25):
                t[int(rng.integers(0, n))] = alpha[int(rng.integers(0, len(alpha)))]
            t = bytes(t)
        else:
            t = bytes(rng.choice(list(alpha), size=n))
        for c in sorted(set(int(x) for x in rng.integers(1, n + 1, size=4))):
            carried += split_run(p, t, K, c)
    assert carried > 50  # the cuts did fall inside open segments


@pytest.mark.parametrize("p,t,K", [
    (b"aaaaaaaa", b"a" * 400, 2),  # one segment over the whole stream
    (b"acacacac", b"ac" * 200, 2),
    (b"acgttgca", b"acgt" * 100, 3),
])
def test_split_inside_periodic_runs(p, t, K):
    for c in (1, 7, 8, 9, 150, 399, len(t)):
        split_run(p, t, K, c)
