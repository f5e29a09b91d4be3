"""Pins of the oracle's alternative readings of Alg. 1 (CPU only).

The paper fixes one emission of its worked example (Section 4.2) and the
rules R1-R3 and Eq. 3; where its text admits several readings (acc as the
sum or as the last length, ">" or ">=" in Eq. 3, R2 in start order), each
reading is pinned here by small hit sets whose outcome follows from the
rules by hand (derivations in the comments), and by properties every
reading must keep (Section 4.3's delay bound, disjointness across emissions,
the exact-matching special case K = 0).
"""
import itertools
import os
import re

import numpy as np

from oracle import oracle

PAPER = oracle.RULES_PAPER
ACC_LAST = oracle.RULES_ACC_LAST
EQ3_GE = oracle.RULES_EQ3_GE
START_ORDER = oracle.RULES_START_ORDER
DISJOINT = oracle.RULES_DISJOINT
ALL_VARIANTS = [PAPER | sum(c) for r in range(5) for c in itertools.combinations(
    (ACC_LAST, EQ3_GE, START_ORDER, DISJOINT), r)]


def _filter(records, K, n, rules):
    hs = np.array([r[0] for r in records], np.int64)
    hl = np.array([r[1] for r in records], np.int32)
    hk = np.array([r[2] for r in records], np.int32)
    fr = oracle.filter_hits(hs, hl, hk, K, n, rules)
    return [tuple(x) for x in fr.occ.tolist()], fr.events


# Four levels chained (K = 3): t[12;4] k=3 is stored first; t[14;5] k=2
# arrives (R1) while it is pending (it ends at 15), t[16;6] k=1 while t[14;5]
# is pending (ends at 18), t[20;4] k=0 while t[16;6] is pending (ends at 21).
# The emission is at 23, the end of the best.  Counters: r = 23 - s + 1, so
# r(1) = 8, r(2) = 10, r(3) = 12.  With acc = 4 after the best:
#   level 1: 8 - 4 = 4 > 6 is false;  level 2: 10 - 4 = 6 > 5 is true.
# Level 3 then sees acc = 4 + 5 = 9 (sum): 12 - 9 = 3 > 4 false, or acc = 5
# (last): 12 - 5 = 7 > 4 true -- but t[12;4] = [12, 15] overlaps the
# accepted t[14;5] = [14, 18], which DISJOINT refuses.
CHAIN = [(12, 4, 3), (14, 5, 2), (16, 6, 1), (20, 4, 0)]


def test_acc_sum_versus_last_hand_example():
    occ, ev = _filter(CHAIN, 3, 24, PAPER)
    assert occ == [(20, 4, 0), (14, 5, 2)]
    assert ev[:, 4].tolist() == [4, 8, 10, 12]  # counters r(0..3)
    assert ev[:, 5].tolist() == [0, 4, 4, 9]  # acc before each test (sum)
    occ, ev = _filter(CHAIN, 3, 24, PAPER | ACC_LAST)
    assert occ == [(20, 4, 0), (14, 5, 2), (12, 4, 3)]
    assert ev[:, 5].tolist() == [0, 4, 4, 5]  # acc before each test (last)
    occ, _ = _filter(CHAIN, 3, 24, PAPER | ACC_LAST | DISJOINT)
    assert occ == [(20, 4, 0), (14, 5, 2)]
    occ, _ = _filter(CHAIN, 3, 24, PAPER | DISJOINT)
    assert occ == [(20, 4, 0), (14, 5, 2)]


# K = 2: t[0;5] k=2 stored; t[3;6] k=1 arrives while it is pending (ends at
# 4); t[5;4] k=0 arrives while t[3;6] is pending (ends at 8).  Emission at 8,
# acc = 4: level 1: r = 6, 6 - 4 = 2 vs 6 (rejected either way); level 2:
# r = 9, 9 - 4 = 5 vs l = 5: ">" rejects, ">=" accepts.  t[0;5] = [0, 4] ends
# right before the best [5, 8] starts: adjacent and disjoint.
ADJ = [(0, 5, 2), (3, 6, 1), (5, 4, 0)]


def test_eq3_strict_versus_ge_hand_example():
    occ, ev = _filter(ADJ, 2, 9, PAPER)
    assert occ == [(5, 4, 0)]
    assert ev[:, 4].tolist() == [4, 6, 9]
    occ, _ = _filter(ADJ, 2, 9, PAPER | EQ3_GE)
    assert occ == [(5, 4, 0), (0, 5, 2)]
    occ, _ = _filter(ADJ, 2, 9, PAPER | EQ3_GE | DISJOINT)
    assert occ == [(5, 4, 0), (0, 5, 2)]


def test_r2_start_order_hand_example():
    # K = 1, two priority-1 hits: t[0;5] (ends at 4), then t[1;3] (ends at 3).
    # R2 as read (earliest end wins) replaces t[0;5] and emits t[1;3] at 3;
    # literal start order keeps the first, t[0;5], emitted at 4.
    recs = [(0, 5, 1), (1, 3, 1)]
    assert _filter(recs, 1, 6, PAPER)[0] == [(1, 3, 1)]
    assert _filter(recs, 1, 6, PAPER | START_ORDER)[0] == [(0, 5, 1)]


def test_r2_start_order_on_the_worked_example():
    """Section 4.2's example under literal start order.  Level 2 keeps its
    first hit t[1;5] (k = 2 at start 1); t[5;6] k=1 takes over at start 5 and
    is kept against t[6;5] and t[7;4]; t[10;5] k=0 completes at 14.  With
    acc = 5: level 1, r = 14 - 5 + 1 = 10, 10 - 5 > 6 false; level 2, r = 14,
    14 - 5 > 5 true.  So S = {t[10;5], t[1;5]} instead of the paper's
    {t[10;5], t[3;3]}: this reading does not reproduce the example."""
    g = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")):
        if "=" in line and not line.startswith("#"):
            k, v = [x.strip() for x in line.split("=", 1)]
            g.setdefault(k, v)
    p, t, K = g["pattern"].encode(), g["text"].encode(), int(g["K"])
    r = oracle.run_pair(p, t, K, rules=PAPER | START_ORDER)
    assert [tuple(x) for x in r.occ.tolist()] == [(10, 5, 0), (1, 5, 2)]
    ev = oracle.filter_hits(*r.H, K, len(t), PAPER | START_ORDER).events
    assert [(int(e[1]), int(e[2]), int(e[3]), int(e[4]), int(e[6])) for e in ev] == [
        (0, 10, 5, 5, 1), (1, 5, 6, 10, 0), (2, 1, 5, 14, 1)]


def test_every_reading_is_exact_matching_at_k0():
    """K = 0 leaves one level: every reading keeps the leftmost of
    overlapping exact matches (re.finditer)."""
    rng = np.random.default_rng(31)
    for trial in range(150):
        sigma = int(rng.integers(1, 4))
        m = int(rng.integers(1, 6))
        p = bytes(rng.integers(0, sigma, size=m).astype(np.uint8) + 97)
        t = bytes(rng.integers(0, sigma, size=int(rng.integers(0, 60))).astype(np.uint8) + 97)
        want = [mm.start() for mm in re.finditer(re.escape(p), t)]
        for rules in ALL_VARIANTS:
            assert oracle.run_pair(p, t, 0, rules=rules).occ[:, 0].tolist() == want


def test_every_reading_keeps_the_structural_properties():
    """For every combination of readings, on random small cases: accepted
    records are H records with their own k; each emission happens at the end
    of its best and accepts it; occurrences of different emissions are
    disjoint; Section 4.3's delay bound d = m(K+1) + K(K-1)/2 holds; with the
    summed acc (or DISJOINT) the others are disjoint from the best; with
    DISJOINT all occurrences of an emission are pairwise disjoint."""
    rng = np.random.default_rng(37)
    for trial in range(250):
        m = int(rng.integers(2, 9))
        K = int(rng.integers(1, m))
        sigma = int(rng.integers(1, 4))
        p = bytes(rng.integers(0, sigma, size=m).astype(np.uint8) + 65)
        t = bytes(rng.integers(0, sigma, size=int(rng.integers(0, 90))).astype(np.uint8) + 65)
        base = oracle.run_pair(p, t, K)
        Hset = {(int(a), int(b)): int(c) for a, b, c in zip(*base.H)}
        d_bound = m * (K + 1) + K * (K - 1) // 2
        for rules in ALL_VARIANTS:
            ev = oracle.filter_hits(*base.H, K, len(t), rules).events
            emissions = {}
            for e in ev.tolist():
                emissions.setdefault(e[0], []).append(e)
            last_pos = -1
            for pos, evs in sorted(emissions.items()):
                best = evs[0]
                assert best[6] == 1 and best[0] == best[2] + best[3] - 1
                acc_ok = [(e[2], e[2] + e[3] - 1) for e in evs if e[6]]
                for e in evs:
                    assert Hset[(e[2], e[3])] == e[1]
                    assert e[4] == pos - e[2] + 1
                for s, end in acc_ok:
                    assert s > last_pos  # after the previous emission
                    assert pos - s + 1 <= d_bound
                    if (rules & (ACC_LAST | DISJOINT)) != ACC_LAST and (s, end) != acc_ok[0]:
                        assert end < best[2]
                if rules & DISJOINT:
                    for (a0, a1), (b0, b1) in itertools.combinations(acc_ok, 2):
                        assert a1 < b0 or b1 < a0
                last_pos = pos
