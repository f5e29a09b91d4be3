"""The word-cutoff rule of the scan, checked on the CPU against the oracle.

A plain model of the bit-parallel column recurrence (Python integers as
whole columns; search mode; 32-row words) that steps only words 0..y and
re-decides y every 4 symbols by the scan's rule:

* word b+1 must be active if s_b <= K + 4 (s_b = value at the bottom row of
  word b);
* a full word b must stay active if s_b <= K + 31;
* the last word (low placement, r pattern rows) must stay active if
  D <= K + r - 1;
* a word that becomes active again restarts from +1 vertical deltas.

Its hit ends and distances must equal the oracle's (the Less Naive last row,
Section 5.1) on random inputs, with the low row placement the cutoff scan
uses (and with the high placement of the full-column scan as well); and
shrinking either margin must break it on some input (so the test can tell a
correct rule from a wrong one).  This checks the rule, not the GPU code: the
GPU parity tests compare the kernel itself with the oracle.
"""
import numpy as np
import pytest

from oracle import oracle


def model_hits(p: bytes, t: np.ndarray, K: int, low: bool, keep_full=31, need=4, G=4):
    m = len(p)
    W = (m + 31) // 32
    nb = 32 * W
    full = (1 << nb) - 1
    g = 0 if low else nb - m  # high placement: g wildcard rows below the pattern
    wild = (1 << g) - 1
    peq = {}
    for c in set(t.tolist()) | set(p):
        v = wild
        for j, ch in enumerate(p):
            if ch == c:
                v |= 1 << (g + j)
        peq[c] = v
    pv = full if low else full & ~wild
    mv = 0
    y = W - 1
    r_last = m - 32 * (W - 1)
    last = (1 << m) - 1 if low else full  # rows read for the last-row value

    def step(pv, mv, eq, nwords):
        msk = (1 << (32 * nwords)) - 1
        pvl, mvl, eql = pv & msk, mv & msk, eq & msk
        xv = eql | mvl
        xh = ((((eql & pvl) + pvl) & msk) ^ pvl) | eql
        ph = mvl | (~(xh | pvl) & msk)
        mh = pvl & xh
        ph2, mh2 = (ph << 1) & msk, (mh << 1) & msk
        npv = mh2 | (~(xv | ph2) & msk)
        hi = ~msk & full
        return (pv & hi) | npv, (mv & hi) | (ph2 & xv)

    def value(pv, mv, msk):
        return bin(pv & msk).count("1") - bin(mv & msk).count("1")

    hits = {}
    cut_groups = 0  # groups run with the last word inactive
    for pos in range(0, t.size, G):
        cut_groups += y < W - 1
        for j in range(pos, min(pos + G, t.size)):
            pv, mv = step(pv, mv, peq.get(int(t[j]), wild), y + 1)
            if y == W - 1:
                d = value(pv, mv, last)
                if d <= K:
                    hits[j] = d
        ynew = 0
        for b in range(y + 1):
            if b < W - 1:
                sb = value(pv, mv, (1 << (32 * (b + 1))) - 1)
                if sb <= K + need:
                    ynew = b + 1
                elif sb <= K + keep_full:
                    ynew = max(ynew, b)
            else:
                d = value(pv, mv, last)
                stay = K + (min(keep_full, r_last - 1) if low else keep_full)
                if d <= stay:
                    ynew = max(ynew, b)
        ynew = min(ynew, W - 1)
        for w in range(y + 1, ynew + 1):  # reactivated words: +1 deltas
            pv |= ((1 << 32) - 1) << (32 * w)
            mv &= ~(((1 << 32) - 1) << (32 * w))
        y = ynew
    return hits, cut_groups


def random_case(rng):
    m = int(rng.integers(33, 140))
    K = int(rng.integers(0, min(m, 30)))
    sigma = int(rng.choice([2, 4, 20]))
    p = bytes(rng.integers(0, sigma, size=m).astype(np.uint8))
    n = int(rng.integers(0, 1500))
    t = rng.integers(0, sigma, size=n).astype(np.uint8)
    for _ in range(int(rng.integers(0, 5))):  # mutated copies, so hits occur
        if n > m + 10:
            o = int(rng.integers(0, n - m))
            t[o:o + m] = np.frombuffer(p, np.uint8)
            for _e in range(int(rng.integers(0, K + 2))):
                t[o + int(rng.integers(0, m))] = int(rng.integers(0, sigma))
    return p, t, K


@pytest.mark.parametrize("low", [True, False])
def test_cutoff_rule_is_exact(low):
    rng = np.random.default_rng(101 if low else 202)
    n_hits = n_cut = 0
    for _ in range(60):
        p, t, K = random_case(rng)
        ends, dists = oracle.raw_hits(p, t, K)
        got, cut = model_hits(p, t, K, low)
        assert got == dict(zip(ends.tolist(), dists.tolist()))
        n_hits += len(got)
        n_cut += cut
    assert n_hits > 100 and n_cut > 1000  # the cases do exercise hits and the cutoff


@pytest.mark.parametrize("low,keep_full,need", [(True, 31, 0), (True, 10, 4), (False, 31, 0), (False, 10, 4)])
def test_shrunk_margins_fail(low, keep_full, need):
    rng = np.random.default_rng(303)
    for _ in range(200):
        p, t, K = random_case(rng)
        ends, dists = oracle.raw_hits(p, t, K)
        if model_hits(p, t, K, low, keep_full, need)[0] != dict(zip(ends.tolist(), dists.tolist())):
            return
    pytest.fail("a rule with a shrunk margin was exact on every input")
