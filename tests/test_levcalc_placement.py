"""The row placement and band cutoff of the LEV CALC kernel, checked on the
CPU against the oracle.

A plain model of the anchored bit-vector recurrence (Python integers as
whole columns of W 32-bit words; the first DP row C[0][l] = l enters as a +1
horizontal delta at pattern row 1) with the kernel's choices:

* one-word columns use high placement: row r at bit 32 - m + r - 1, the
  32 - m bits below row 1 match every byte and start with no vertical delta
  (pv = mv = 0), and the last-row value is the popcounts of the whole word
  minus a bias, with no mask;
* wider columns use low placement (row r at bit r - 1) and read the last
  word through a mask;
* the band cutoff: before the first output column (l < m - K) a step
  advances only the N(l) = ceil((b0 + l + K) / 32) words holding the rows
  that can still be <= K; the words above keep their initial state.

Its output for every start must equal the oracle's LEV CALC (Section 6.2,
Eq. 1) on random inputs, and breaking either choice (match-all rows that
start with +1 deltas, or a band narrower by a few rows) must make it differ
on some input, so the test can tell the kernel's rule from a wrong one.
This checks the rule, not the GPU code: the GPU parity tests compare the
kernel itself with the oracle.
"""
import numpy as np
import pytest

from oracle import oracle


def model_levcalc(p, t, K, wild_pv=0, band_slack=0):
    m = len(p)
    W = (m + 31) // 32
    b0 = 32 - m if W == 1 else 0
    nbits = 32 * W
    full = (1 << nbits) - 1
    low = (1 << b0) - 1
    if W == 1:
        sum_mask = full
    else:
        rlast = m - 32 * (W - 1)
        sum_mask = ((1 << (32 * (W - 1))) - 1) | (((1 << rlast) - 1) << (32 * (W - 1)))
    peq = {}
    for c in set(int(x) for x in t) | set(p):
        v = low
        for r in range(m):
            if p[r] == c:
                v |= 1 << (b0 + r)
        peq[c] = v
    n = len(t)
    width = 2 * K + 1
    out = np.full((n, width), 255, dtype=np.int64)
    for s in range(n):
        pv = (full & ~low) | (low if wild_pv else 0)
        cm = full
        for j in range(m + K):
            if s + j >= n:
                break
            l = j + 1
            eq = peq.get(int(t[s + j]), low)
            if l < m - K:
                N = min(W, -(-(b0 + l + K - band_slack) // 32))
                N = max(N, 1)
            else:
                N = W
            nm = (1 << (32 * N)) - 1
            pvn, cmn, eqn = pv & nm, cm & nm, eq & nm
            mv = ~cmn & nm
            u = ((eqn & pvn) + pvn) & nm
            ph = (mv | ~(u | pvn | eqn)) & nm
            mh = pvn & (eqn | (~u & nm))
            ph2 = ((ph << 1) | (1 << b0)) & nm
            mh2 = (mh << 1) & nm
            npv = (mh2 | ~(eqn | mv | ph2)) & nm
            nmv = ph2 & (eqn | mv)
            pv = (pv & ~nm) | npv
            cm = (cm & ~nm) | (~nmv & nm)
            if l >= m - K:
                d = l - m - b0 + bin(pv & sum_mask).count("1") + bin(cm & sum_mask).count("1")
                out[s, l - (m - K)] = min(d, K + 1)
    return out


def cases(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(rng.choice([1, 2, 5, 16, 31, 32, 33, 40, 63, 64, 65, 90, 96, 97]))
        K = int(rng.integers(0, min(m, 12)))
        sig = int(rng.choice([2, 4, 20]))
        p = [int(x) for x in rng.integers(0, sig, m)]
        n = int(rng.integers(1, 50))
        t = rng.integers(0, sig, n).astype(np.uint8)
        if rng.random() < 0.6 and n > m + 2:
            pos = int(rng.integers(0, n - m))
            t[pos:pos + m] = p
            if m > 3:  # one edit
                t[pos + int(rng.integers(0, m))] = int(rng.integers(0, sig))
        out.append((p, t, K))
    return out


def test_placement_and_band_are_exact():
    for p, t, K in cases(11, 160):
        got = model_levcalc(p, t, K)
        want = np.asarray(oracle.levcalc(bytes(p), t, K)).reshape(len(t), 2 * K + 1)
        assert np.array_equal(got, want), (len(p), K, len(t))


@pytest.mark.parametrize("wild_pv,band_slack", [(1, 0), (0, 6)])
def test_broken_rules_fail(wild_pv, band_slack):
    differs = 0
    for p, t, K in cases(12, 160):
        if wild_pv and len(p) >= 32:
            continue  # no match-all rows
        if band_slack and len(p) <= 32:
            continue  # no band cutoff
        got = model_levcalc(p, t, K, wild_pv=wild_pv, band_slack=band_slack)
        want = np.asarray(oracle.levcalc(bytes(p), t, K)).reshape(len(t), 2 * K + 1)
        differs += not np.array_equal(got, want)
    assert differs > 0
