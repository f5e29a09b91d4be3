"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: textbook values of
the Levenshtein distance, an exhaustive shortest-edit-path search (the
definition of the distance as the minimum number of single-symbol edits,
Section 3), brute force over every substring (the "Fully Naive" baseline,
Section 5.1), the worked example of Section 4.2, the exact-match special case
K = 0 (a library routine), the delay bound of Section 4.3, and invariants of
the priority rules and the validation test.
"""
import itertools
import re
from collections import deque

import numpy as np
import pytest

import oracle
from paper_1712_03560_amd import workloads as W


# ---------------------------------------------------------------- edit search
class EditSearch:
    """Distances by breadth-first search over single-symbol edits.

    An optimal edit script can be ordered deletions, substitutions,
    insertions, so no intermediate string is longer than the longer end
    point; the search is therefore exact for strings up to ``maxlen``."""

    def __init__(self, alphabet: str, maxlen: int):
        self.alphabet = alphabet
        self.maxlen = maxlen
        self.cache = {}

    def _neighbours(self, s):
        for j in range(len(s)):
            yield s[:j] + s[j + 1:]
            for c in self.alphabet:
                if c != s[j]:
                    yield s[:j] + c + s[j + 1:]
        if len(s) < self.maxlen:
            for j in range(len(s) + 1):
                for c in self.alphabet:
                    yield s[:j] + c + s[j:]

    def dist_from(self, a):
        if a not in self.cache:
            d = {a: 0}
            q = deque([a])
            while q:
                s = q.popleft()
                for n in self._neighbours(s):
                    if n not in d:
                        d[n] = d[s] + 1
                        q.append(n)
            self.cache[a] = d
        return self.cache[a]

    def __call__(self, a, b):
        return self.dist_from(a)[b]


def strings(alphabet, lo, hi):
    for n in range(lo, hi + 1):
        for t in itertools.product(alphabet, repeat=n):
            yield "".join(t)


# ---------------------------------------------------------------- Eq. 1
def test_lev_textbook_values():
    assert oracle.lev(b"kitten", b"sitting") == 3
    assert oracle.lev(b"flaw", b"lawn") == 2
    assert oracle.lev(b"intention", b"execution") == 5
    assert oracle.lev(b"", b"abc") == 3
    assert oracle.lev(b"abc", b"") == 3
    assert oracle.lev(b"abcdef", b"abcdef") == 0


def test_lev_equals_shortest_edit_path_exhaustive():
    es = EditSearch("ABC", 4)
    for a in strings("ABC", 0, 4):
        d = es.dist_from(a)
        for b in strings("ABC", 0, 4):
            assert oracle.lev(a.encode(), b.encode()) == d[b], (a, b)


def test_fig1_strings():
    """Section 3, Fig. 1: p = ABCD against t[0,3], t[0,4], t[0,5] of
    t = ABBDABCDACDB; the figure's numbers are not in the text, so they are
    re-derived here by edit search."""
    es = EditSearch("ABCD", 5)
    t = "ABBDABCDACDB"
    for ln in (3, 4, 5):
        assert oracle.lev(b"ABCD", t[:ln].encode()) == es("ABCD", t[:ln])
    assert [es("ABCD", t[:ln]) for ln in (3, 4, 5)] == [2, 1, 2]


# ---------------------------------------------------------------- Less Naive
def test_sellers_last_row_is_min_over_starts_exhaustive():
    es = EditSearch("AB", 10)
    for p in strings("AB", 1, 5):
        dp = es.dist_from(p)
        for t in strings("AB", 0, 10):
            D = oracle.sellers_column(p.encode(), t.encode())
            for e in range(len(t)):
                # substrings t[s..e], including the empty one (s = e + 1)
                want = min(dp[t[s:e + 1]] for s in range(e + 2))
                assert D[e] == want, (p, t, e)


def _brute_h(es, p, t, K):
    m = len(p)
    out = []
    for i in range(len(t)):
        for ln in range(max(1, m - K), m + K + 1):
            if i + ln > len(t):
                break
            k = es(p, t[i:i + ln])
            if k <= K:
                out.append((i, ln, k))
    return out


def test_raw_hits_and_hit_set_exhaustive():
    """Raw ends, H by definition (Eq. 2) and the identity between them:
    the ends of H are exactly the raw-hit ends and D[e] is the smallest k
    among the H records ending at e."""
    es = EditSearch("AB", 9)
    for p in strings("AB", 1, 5):
        for t in strings("AB", 0, 9):
            for K in range(len(p)):
                ends, dists = oracle.raw_hits(p.encode(), t.encode(), K)
                H = _brute_h(es, p, t, K)
                hs, hl, hk = oracle.hset_all(p.encode(), t.encode(), K)
                assert list(zip(hs.tolist(), hl.tolist(), hk.tolist())) == H
                h_ends = sorted({i + ln - 1 for i, ln, _ in H})
                assert ends.tolist() == h_ends
                for e, d in zip(ends.tolist(), dists.tolist()):
                    assert d == min(k for i, ln, k in H if i + ln - 1 == e)
                hs2, hl2, hk2 = oracle.hset_at_ends(p.encode(), t.encode(), K, ends)
                assert list(zip(hs2.tolist(), hl2.tolist(), hk2.tolist())) == H


def test_hit_set_at_raw_ends_random():
    rng = np.random.default_rng(5)
    for trial in range(300):
        m = int(rng.integers(1, 12))
        K = int(rng.integers(0, m))
        sigma = int(rng.integers(2, 5))
        p = bytes(rng.integers(0, sigma, size=m).astype(np.uint8) + 65)
        t = bytes(rng.integers(0, sigma, size=int(rng.integers(0, 80))).astype(np.uint8) + 65)
        ends, _ = oracle.raw_hits(p, t, K)
        a = oracle.hset_all(p, t, K)
        b = oracle.hset_at_ends(p, t, K, ends)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_restart_lemma():
    """A scan restarted (free start) at position c reproduces D[e] for every
    e >= c + m + K - 1 whenever either value is <= K; chunked scans with an
    (m + K - 1)-symbol look-back are therefore exact."""
    rng = np.random.default_rng(11)
    for trial in range(400):
        m = int(rng.integers(1, 14))
        K = int(rng.integers(0, m))
        sigma = int(rng.integers(2, 5))
        p = rng.integers(0, sigma, size=m).astype(np.uint8)
        t = rng.integers(0, sigma, size=int(rng.integers(1, 120))).astype(np.uint8)
        D = oracle.sellers_column(p, t)
        c = int(rng.integers(0, t.size))
        Dc = oracle.sellers_column(p, t[c:])
        for e in range(c + m + K - 1, t.size):
            a, b = D[e], Dc[e - c]
            if a <= K or b <= K:
                assert a == b, (trial, e)


# ---------------------------------------------------------------- Alg. 1
def _read_golden(path):
    kv = {"occ": [], "level": []}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = [x.strip() for x in line.split("=", 1)]
        if k in ("occ", "level"):
            kv[k].append(tuple(int(x) for x in v.split()))
        else:
            kv[k] = v
    return kv


def test_worked_example_section_4_2():
    import os

    g = _read_golden(os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt"))
    p, t, K = g["pattern"].encode(), g["text"].encode(), int(g["K"])
    r = oracle.run_pair(p, t, K)
    assert [tuple(x) for x in r.occ.tolist()] == g["occ"]
    fr = oracle.filter_hits(*r.H, K, len(t))
    ev = fr.events
    # one emission, at the end of the priority-0 occurrence (position 14)
    assert set(ev[:, 0].tolist()) == {14}
    levels = [(int(e[1]), int(e[4]), int(e[3]), int(e[6])) for e in ev]
    assert levels == g["level"]
    # the Eq. 3 arithmetic the paper spells out: 8 - 5 > 4 false, 12 - 5 > 3 true
    assert ev[1, 5] == 5 and ev[2, 5] == 5
    # the texts of the three occurrences named in the paper
    assert t[10:15] == b"ACBDA" and t[7:11] == b"CBDA" and t[3:6] == b"CDA"


def test_k0_is_leftmost_non_overlapping_exact_matching():
    """With K = 0 every hit is an exact occurrence of priority 0; the rules
    then keep the leftmost of overlapping ones, which is what re.finditer
    returns, and the raw ends are the ends of all (overlapping) matches."""
    rng = np.random.default_rng(3)
    for trial in range(600):
        sigma = int(rng.integers(1, 4))
        m = int(rng.integers(1, 6))
        p = bytes(rng.integers(0, sigma, size=m).astype(np.uint8) + 97)
        t = bytes(rng.integers(0, sigma, size=int(rng.integers(0, 60))).astype(np.uint8) + 97)
        r = oracle.run_pair(p, t, 0)
        all_ends = [j + m - 1 for j in range(len(t) - m + 1) if t[j:j + m] == p]
        assert r.ends.tolist() == all_ends
        want = [mm.start() for mm in re.finditer(re.escape(p), t)]
        assert r.occ[:, 0].tolist() == want
        assert len(want) == len(re.findall(re.escape(p), t))


def _random_case(rng, mmax=9, nmax=90, sigma_max=4):
    m = int(rng.integers(1, mmax))
    K = int(rng.integers(0, m))
    sigma = int(rng.integers(1, sigma_max + 1))
    p = bytes(rng.integers(0, sigma, size=m).astype(np.uint8) + 65)
    t = bytes(rng.integers(0, sigma, size=int(rng.integers(0, nmax))).astype(np.uint8) + 65)
    return p, t, K


def _check_filter_invariants(p, t, K):
    """Invariants (i)-(v) of the filter and Table 1's ordering on one case."""
    m = len(p)
    r = oracle.run_pair(p, t, K)
    Hset = {(int(a), int(b)): int(c) for a, b, c in zip(*r.H)}
    fr = oracle.filter_hits(*r.H, K, len(t))
    ev = fr.events
    d_bound = m * (K + 1) + K * (K - 1) // 2
    emissions = {}
    for e in ev.tolist():
        emissions.setdefault(e[0], []).append(e)
    prev = []
    for pos, evs in sorted(emissions.items()):
        best = evs[0]
        assert best[6] == 1  # (ii) the best is always accepted
        assert best[0] == best[2] + best[3] - 1  # emitted when the best ends
        assert [e[1] for e in evs] == sorted(e[1] for e in evs)
        acc = 0
        for e in evs:
            _, lvl, s, ln, rr, a0, ok = e
            assert a0 == acc
            assert Hset[(s, ln)] == lvl  # (i) an H record with its own k
            assert rr == pos - s + 1  # counter = symbols seen since its start
            if e is not best:
                assert ok == int(rr - acc > ln)  # Eq. 3
                if ok:  # (iii) disjoint from the best
                    assert s + ln - 1 < best[2] or s > best[2] + best[3] - 1
            if ok:
                acc += ln
                assert pos - s + 1 <= d_bound  # (v) delay bound d of Section 4.3
        occs = [(e[2], e[3]) for e in evs if e[6]]
        for s, ln in occs:  # (iv) disjoint from earlier emissions
            for s2, l2 in prev:
                assert s > s2 + l2 - 1 or s + ln - 1 < s2
        prev += occs
    # the ordering Table 1 shows: |S| <= #raw ends <= |H|
    assert len(r.occ) <= len(r.ends) <= len(Hset)


def test_filter_invariants_random():
    rng = np.random.default_rng(7)
    for trial in range(1500):
        _check_filter_invariants(*_random_case(rng))


def test_filter_invariants_exhaustive():
    """The same invariants for every p in {A,B}^1..4, t in {A,B}^0..9 and K < m."""
    for p in strings("AB", 1, 4):
        for t in strings("AB", 0, 9):
            for K in range(len(p)):
                _check_filter_invariants(p.encode(), t.encode(), K)


def test_filter_segments_are_independent():
    """Splitting the raw ends wherever two consecutive ends are at least
    m + K apart, and filtering each piece from an empty state, reproduces the
    filter over the whole stream (a pending best always completes at its own
    end, before any later piece starts)."""
    rng = np.random.default_rng(13)
    for trial in range(800):
        p, t, K = _random_case(rng, mmax=8, nmax=150, sigma_max=3)
        m = len(p)
        r = oracle.run_pair(p, t, K)
        ends = r.ends.tolist()
        pieces, cur = [], []
        for e in ends:
            if cur and e - cur[-1] >= m + K:
                pieces.append(cur)
                cur = []
            cur.append(e)
        if cur:
            pieces.append(cur)
        got = []
        for piece in pieces:
            H = oracle.hset_at_ends(p, t, K, np.array(piece))
            got += [tuple(x) for x in oracle.filter_hits(*H, K, len(t)).occ.tolist()]
        assert got == [tuple(x) for x in r.occ.tolist()]


def test_planted_copies_are_found():
    """Every planted copy with e edits ends at a raw hit whose distance is at
    most e (the copy itself is a substring at distance <= e)."""
    w = W.tiny(n=20_000, n_plants=40)
    t = w.streams[0]
    for pl in w.plants:
        p = w.patterns[pl.pattern]
        K = int(w.ks[pl.pattern])
        e = pl.site + pl.length - 1
        lo = max(0, e - 200)
        D = oracle.sellers_column(p, t[lo:e + 1])
        assert D[-1] <= min(pl.edits, K) or pl.edits > K
