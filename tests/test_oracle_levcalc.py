"""Pins for the oracle's LEV CALC output (no GPU).

LEV CALC (Section 6.2) yields, for every stream index i, the distances
between the pattern and the 2K+1 substrings t[i, l_p-K] .. t[i, l_p+K].
The oracle's version is checked against the distances the worked example of
Section 4.2 gives, against a shortest-edit-path search (the definition of the
distance), and against the hit set reached through the other route: the
Less Naive scan's hit ends and the per-end distances (Eq. 2 at the ends).
"""
import os

import numpy as np

import oracle
from tests.test_oracle_pins import EditSearch, strings

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "levcalc_example.txt")


def _golden():
    d = {"dist": []}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, val = (x.strip() for x in line.split("=", 1))
        if key == "dist":
            d["dist"].append(tuple(int(v) for v in val.split()))
        else:
            d[key] = val
    return d


def test_worked_example_distances():
    g = _golden()
    K = int(g["K"])
    out = oracle.levcalc(g["pattern"].encode(), g["text"].encode(), K)
    m = len(g["pattern"])
    assert out.shape == (len(g["text"]), 2 * K + 1)
    for start, length, dist in g["dist"]:
        assert out[start, length - (m - K)] == dist


def test_levcalc_equals_edit_search_exhaustive():
    es = EditSearch("AB", 8)
    for p in strings("AB", 1, 4):
        for t in strings("AB", 0, 6):
            for K in range(len(p)):
                out = oracle.levcalc(p.encode(), t.encode(), K)
                assert out.shape == (len(t), 2 * K + 1)
                for i in range(len(t)):
                    for j in range(2 * K + 1):
                        l = len(p) - K + j
                        if i + l > len(t):
                            want = 255
                        else:
                            want = min(es(p, t[i:i + l]), K + 1)
                        assert out[i, j] == want, (p, t, K, i, l)


def test_levcalc_hits_equal_hit_set_at_scan_ends():
    """Entries <= K are exactly H, which the Less Naive scan reaches through
    its hit ends (every end of H is a hit end)."""
    rng = np.random.default_rng(5)
    for case in range(120):
        sigma = int(rng.integers(2, 5))
        m = int(rng.integers(1, 10))
        K = int(rng.integers(0, m))
        p = rng.integers(0, sigma, m).astype(np.uint8)
        n = int(rng.integers(0, 120))
        t = rng.integers(0, sigma, n).astype(np.uint8)
        if n > m and case % 2:
            s = int(rng.integers(0, n - m))
            t[s:s + m] = p  # one exact copy
        out = oracle.levcalc(p, t, K)
        ii, jj = np.nonzero(out <= K)
        got = sorted(zip(ii.tolist(), (jj + m - K).tolist(), out[ii, jj].tolist()))
        ends, _ = oracle.raw_hits(p, t, K)
        hs, hl, hk = oracle.hset_at_ends(p, t, K, ends)
        want = sorted(zip(hs.tolist(), hl.tolist(), hk.tolist()))
        assert got == want, case
        # the capped entries: > K exactly where the substring exists and misses
        assert np.all((out == K + 1) | (out <= K) | (out == 255))


def test_levcalc_rejects_k_not_below_length():
    import pytest

    with pytest.raises(ValueError):
        oracle.levcalc(b"AB", b"ABAB", 2)
