"""OASM oracle -- TEST INFRASTRUCTURE ONLY.

Python face of the plain CPU reference in ``oasm_oracle.c``.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import this
module; the product library never does, and it shares no code with it.

What each function computes (sections of arXiv 1712.03560):

* :func:`lev`            -- Eq. 1, the Levenshtein matrix C (Section 3).
* :func:`raw_hits`       -- "Less Naive" (Section 5.1): C with a zero first
                            row; every end e whose last-row value D[e] <= K.
* :func:`hset_all`       -- Eq. 2 by definition: all (i, l, k) with
                            l in [l_p-K, l_p+K] and k = lev(p, t[i,l]) <= K.
* :func:`hset_at_ends`   -- Eq. 2 restricted to substrings ending at given
                            positions.
* :func:`levcalc`        -- the output of LEV CALC (Section 6.2): for every
                            start i the distances to t[i,l] for the 2K+1
                            lengths l in [l_p-K, l_p+K], capped at K+1.
* :func:`filter_hits`    -- Alg. 1 with R1-R3 (Section 4.1) and Eq. 3
                            (Section 4.2), as read in ``oasm_oracle.c``.
* :func:`run_pair`       -- the whole path for one (pattern, text) pair:
                            raw hits, H (at the raw ends) and S.

Only small helpers (sorting with numpy, a thread pool over independent pairs)
sit on top of the C functions; all matching arithmetic is in the C file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oasm_oracle.c")
_LIB = os.path.join(_HERE, "liboasm_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation pragmas)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i32, i64 = ctypes.c_int32, ctypes.c_int64
            lib.oracle_lev.argtypes = [P, i32, P, i32]
            lib.oracle_lev.restype = i32
            lib.oracle_sellers.argtypes = [P, i32, P, i64, i32, P, P, i64, P]
            lib.oracle_sellers.restype = i64
            lib.oracle_hset_all.argtypes = [P, i32, P, i64, i32, P, P, P, i64]
            lib.oracle_hset_all.restype = i64
            lib.oracle_hset_at_ends.argtypes = [P, i32, P, i64, i32, P, i64, P, P, P, i64]
            lib.oracle_hset_at_ends.restype = i64
            lib.oracle_levcalc.argtypes = [P, i32, P, i64, i32, P]
            lib.oracle_levcalc.restype = i64
            lib.oracle_filter.argtypes = [P, P, P, i64, i32, i64, i32] + [P] * 7 + [i64]
            lib.oracle_filter.restype = i64
            _lib = lib
    return _lib


def _u8(x) -> np.ndarray:
    if isinstance(x, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(x), dtype=np.uint8)
    a = np.ascontiguousarray(x, dtype=np.uint8)
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def lev(a, b) -> int:
    """Eq. 1: the Levenshtein distance between two byte strings."""
    A, B = _u8(a), _u8(b)
    return int(_load().oracle_lev(_ptr(A), A.size, _ptr(B), B.size))


def sellers_column(p, t) -> np.ndarray:
    """D[e] for every end e (the last row of C with a zero first row)."""
    P, T = _u8(p), _u8(t)
    D = np.empty(T.size, dtype=np.int32)
    _load().oracle_sellers(_ptr(P), P.size, _ptr(T), T.size, -1, None, None, 0, _ptr(D))
    return D


def raw_hits(p, t, K: int):
    """Every end e with D[e] <= K, and D[e]; both int64/int32 arrays, e ascending."""
    P, T = _u8(p), _u8(t)
    lib = _load()
    cap = 1024
    while True:
        ends = np.empty(cap, dtype=np.int64)
        dists = np.empty(cap, dtype=np.int32)
        cnt = lib.oracle_sellers(_ptr(P), P.size, _ptr(T), T.size, K, _ptr(ends), _ptr(dists), cap, None)
        if cnt < 0:
            raise MemoryError("oracle_sellers")
        if cnt <= cap:
            return ends[:cnt], dists[:cnt]
        cap = int(cnt)


def _hset_call(fn, *args):
    cap = 4096
    while True:
        hs = np.empty(cap, dtype=np.int64)
        hl = np.empty(cap, dtype=np.int32)
        hk = np.empty(cap, dtype=np.int32)
        cnt = fn(*args, _ptr(hs), _ptr(hl), _ptr(hk), cap)
        if cnt < 0:
            raise MemoryError("oracle hset")
        if cnt <= cap:
            return hs[:cnt], hl[:cnt], hk[:cnt]
        cap = int(cnt)


def _sorted_h(hs, hl, hk):
    order = np.lexsort((hl, hs))
    return hs[order], hl[order], hk[order]


def hset_all(p, t, K: int):
    """Eq. 2 by definition over all starts; (i, l, k) arrays in (i, l) order."""
    P, T = _u8(p), _u8(t)
    return _hset_call(_load().oracle_hset_all, _ptr(P), P.size, _ptr(T), T.size, K)


def hset_at_ends(p, t, K: int, ends):
    """Eq. 2 restricted to the given end positions; (i, l, k) in (i, l) order."""
    P, T = _u8(p), _u8(t)
    E = np.ascontiguousarray(ends, dtype=np.int64)
    hs, hl, hk = _hset_call(_load().oracle_hset_at_ends, _ptr(P), P.size, _ptr(T), T.size, K, _ptr(E), E.size)
    return _sorted_h(hs, hl, hk)


def levcalc(p, t, K: int) -> np.ndarray:
    """LEV CALC for every start: uint8 array [n, 2K+1]; entry j is
    min(lev(p, t[i, l_p-K+j]), K+1), or 255 where the substring runs past the end."""
    P, T = _u8(p), _u8(t)
    out = np.empty((T.size, 2 * K + 1), dtype=np.uint8)
    if _load().oracle_levcalc(_ptr(P), P.size, _ptr(T), T.size, K, _ptr(out)) != 0:
        raise ValueError("levcalc needs 0 <= K < len(p)")
    return out


def levcalc_many(patterns, ks, text, threads: int | None = None):
    """levcalc for every pattern of a dictionary on one text (a thread per pattern)."""
    T = _u8(text)
    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(levcalc, p, T, int(k)) for p, k in zip(patterns, ks)]
        return [f.result() for f in futs]


@dataclass
class FilterResult:
    """Output of Alg. 1.

    ``occ`` is S in emission order: rows (i, l, k).  ``events`` holds every
    non-empty priority level examined at an emission: rows
    (emission position, level, i, l, r, acc, accepted).
    """

    occ: np.ndarray
    events: np.ndarray


# Alternative readings of Alg. 1 (bit values equal to the library's
# OASM_RULES_* bits; see oracle_filter in oasm_oracle.c).
RULES_PAPER = 1
RULES_ACC_LAST = 2
RULES_EQ3_GE = 4
RULES_START_ORDER = 8
RULES_DISJOINT = 16


def filter_hits(hs, hl, hk, K: int, n: int, rules: int = RULES_PAPER) -> FilterResult:
    """Alg. 1 over H (any order; sorted here by (i, l)) for a text of n symbols."""
    hs = np.ascontiguousarray(hs, dtype=np.int64)
    hl = np.ascontiguousarray(hl, dtype=np.int32)
    hk = np.ascontiguousarray(hk, dtype=np.int32)
    hs, hl, hk = _sorted_h(hs, hl, hk)
    lib = _load()
    cap = max(16, hs.size * (K + 1) + 16)
    while True:
        cols = [np.empty(cap, dtype=dt) for dt in (np.int64, np.int32, np.int64, np.int32, np.int64, np.int64, np.int32)]
        cnt = lib.oracle_filter(_ptr(hs), _ptr(hl), _ptr(hk), hs.size, K, n, int(rules), *[_ptr(c) for c in cols],
                                cap)
        if cnt < 0:
            raise MemoryError("oracle_filter")
        if cnt <= cap:
            break
        cap = int(cnt)
    ev = np.stack([c[:cnt].astype(np.int64) for c in cols], axis=1) if cnt else np.zeros((0, 7), np.int64)
    acc = ev[:, 6] == 1
    # level index 1 is the priority k of the accepted occurrence
    occ = np.stack([ev[acc, 2], ev[acc, 3], ev[acc, 1]], axis=1) if acc.any() else np.zeros((0, 3), np.int64)
    return FilterResult(occ=occ, events=ev)


@dataclass
class PairResult:
    ends: np.ndarray  # raw-hit ends, ascending
    dists: np.ndarray  # D[e] at those ends
    H: tuple  # (i, l, k) arrays in (i, l) order, restricted to the raw ends
    occ: np.ndarray  # S rows (i, l, k) in emission order


def run_pair(p, t, K: int, with_filter: bool = True, rules: int = RULES_PAPER) -> PairResult:
    """Raw hits, H at the raw ends and S for one pattern on one text."""
    ends, dists = raw_hits(p, t, K)
    H = hset_at_ends(p, t, K, ends)
    occ = filter_hits(*H, K, len(t), rules).occ if with_filter else None
    return PairResult(ends, dists, H, occ)


def run_pairs(patterns, ks, text, threads: int | None = None, with_filter: bool = True, rules: int = RULES_PAPER):
    """run_pair over many patterns of one text, one thread per pattern task."""
    T = _u8(text)
    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(run_pair, p, T, int(k), with_filter, rules) for p, k in zip(patterns, ks)]
        return [f.result() for f in futs]
