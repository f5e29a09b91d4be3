"""The decomposition behind the parallel walk of long filter segments, on a
model of the kernels' walk (CPU).

The GPU walks a segment's hit set in (start, length) order and applies Alg. 1
(Section 4: R1-R3, validation by Eq. 3) lazily: a stored best completes
before the first later start.  From an empty state at a start s the walk up
to its first emission depends on s alone, and an emission leaves the state
empty; so the walk is the chain s0 -> next(s0) -> ..., where next(s) is the
start at which the walk from an empty state at s first emits, and each link
emits what that walk holds there.  The long-segment kernels compute next()
for every start, follow the chain and re-walk its links in parallel.

This test restates that walk in Python (the model, not the oracle), checks
it against the oracle's Alg. 1 on whole segments, and checks that the chain
of first emissions gives the same occurrences as the whole walk, with every
link moving forward and no more links than hit ends (the kernels write link
k in the slot of the segment's k-th hit end)."""
import numpy as np
import pytest

from oracle import oracle as O

NOHIT = 255


def walk_from(E, HK, lo, j1, s, m, K, first):
    """The walk from an empty state at start s over hit ends E[lo:j1] (their
    hit-set bytes HK, indexed by length - (m - K)); returns (the start of the
    first emission or None, occurrences) when `first`, else (None, all)."""
    lmax, lmin, qoff = m + K, max(1, m - K), m - K
    lv, idx, bs, bl, out = {}, K, 0, 0, []

    def emit(pos):
        nonlocal idx, bl
        acc = 0
        for j in range(idx, K + 1):
            if j in lv:
                sj, lj = lv[j]
                if j == idx or (pos - sj + 1) - acc > lj:  # Eq. 3
                    out.append((sj, lj, j))
                    acc += lj
        lv.clear()
        idx, bl = K, 0

    while True:
        while lo < j1 and E[lo] + 1 < s + lmin:
            lo += 1
        if lo >= j1:
            break
        if E[lo] + 1 > s + lmax:  # no hit end reachable from s
            s = E[lo] + 1 - lmax
            continue
        if bl and bs + bl - 1 < s:
            emit(bs + bl - 1)
            if first:
                return s, out
        j = lo
        while j < j1 and E[j] + 1 <= s + lmax:
            l = E[j] + 1 - s
            k = HK[j][l - qoff]
            j += 1
            if k == NOHIT:
                continue
            if k < idx:  # R1
                idx, bs, bl = k, s, l
                lv[k] = (s, l)
            elif k == idx and (bl == 0 or s + l < bs + bl or (s + l == bs + bl and l < bl)):  # R2 / R3
                bs, bl = s, l
                lv[k] = (s, l)
        s += 1
    if bl:
        emit(bs + bl - 1)
    return None, out


def first_end_at_least(E, lo, hi, v):
    while lo < hi:
        mid = (lo + hi) // 2
        if E[mid] < v:
            lo = mid + 1
        else:
            hi = mid
    return lo


def segment_hits(p, t, K):
    m = len(p)
    ends, _ = O.raw_hits(p, t, K)
    hs, hl, hk = O.hset_at_ends(p, t, K, ends)
    H = {(int(a), int(b)): int(c) for a, b, c in zip(hs, hl, hk)}
    E = [int(e) for e in ends]
    HK = [[H.get((e - (m - K + q) + 1, m - K + q), NOHIT) if m - K + q >= 1 else NOHIT for q in range(2 * K + 1)]
          for e in E]
    segs, i = [], 0
    while i < len(E):
        j = i + 1
        while j < len(E) and E[j] - E[j - 1] < m + K:
            j += 1
        segs.append((i, j))
        i = j
    want = [tuple(int(v) for v in r) for r in O.filter_hits(hs, hl, hk, K, len(t)).occ]
    return E, HK, segs, want


def chain_of(E, HK, i, j1, m, K):
    lmax, lmin = m + K, max(1, m - K)
    s0 = E[i] + 1 - lmax if E[i] + 1 >= lmax else 0
    nstarts = E[j1 - 1] + 2 - lmin - s0
    nxt = []
    for x in range(nstarts):
        s = s0 + x
        lo = first_end_at_least(E, i, j1, s + lmin - 1)
        w = walk_from(E, HK, lo, j1, s, m, K, True)[0] if lo < j1 else None
        assert w is None or s < w < s0 + nstarts
        nxt.append(None if w is None else w - s0)
    links = [0]
    while nxt[links[-1]] is not None:
        links.append(nxt[links[-1]])
    assert len(links) <= j1 - i
    out = []
    for k, rel in enumerate(links):
        s = s0 + rel
        w, o = walk_from(E, HK, first_end_at_least(E, i, j1, s + lmin - 1), j1, s, m, K, True)
        assert w == (s0 + links[k + 1] if k + 1 < len(links) else None)
        out += o
    return out


def check(p, t, K):
    m = len(p)
    E, HK, segs, want = segment_hits(p, t, K)
    whole, chained = [], []
    for i, j1 in segs:
        s0 = E[i] + 1 - (m + K) if E[i] + 1 >= m + K else 0
        whole += walk_from(E, HK, i, j1, s0, m, K, False)[1]
        chained += chain_of(E, HK, i, j1, m, K)
    assert whole == want
    assert chained == whole
    return len(E), len(want)


@pytest.mark.parametrize("p,t,K", [
    (b"aaaaaaaa", b"a" * 3000, 2),  # a hit end at every position, one segment
    (b"aaaa", b"a" * 2000, 1),
    (b"a" * 40, b"a" * 3000, 8),
    (b"acacacac", b"ac" * 1500, 2),  # period 2
    (b"aaaaaaaa", b"a" * 500 + b"c" + b"a" * 500, 2),
])
def test_chain_equals_whole_walk_on_periodic_text(p, t, K):
    ends, occ = check(p, t, K)
    assert ends > 900 and occ > 10


def test_chain_equals_whole_walk_random():
    rng = np.random.default_rng(5)
    for it in range(25):
        m = int(rng.integers(2, 14))
        K = int(rng.integers(0, m))
        alpha = b"ab" if it % 3 == 0 else b"acgt"
        p = bytes(rng.choice(list(alpha), size=m))
        n = int(rng.integers(0, 500))
        if it % 4 == 0:  # repeats of the pattern with noise
            t = bytearray((p * (n // m + 1))[:n])
            for _ in range(n // 30):
                t[int(rng.integers(0, n))] = alpha[int(rng.integers(0, len(alpha)))]
            t = bytes(t)
        else:
            t = bytes(rng.choice(list(alpha), size=n))
        check(p, t, K)
