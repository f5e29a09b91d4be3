"""Seeded synthetic inputs for the OASM matching path.

This module only draws random bytes: texts, pattern dictionaries, thresholds
and planted mutated pattern copies.  It holds none of the matching
arithmetic, so both the library's tests and the CPU oracle's tests can use
it without sharing any method code.

The workloads follow the shapes of the paper's experiments (random text over
a small alphabet, Section 7) scaled up to dictionary/stream sizes:

* ``tiny``      -- 100,000 symbols over {A,C,G,T}, 16 patterns of 8..16
                   symbols, K = 2, 200 planted copies with 0..2 edits.
* ``long``      -- one 64 MiB stream over {A,C,G,T}, 256 patterns of 16..32
                   symbols, K = 3, 10,000 planted copies with 0..3 edits.
* ``batched``   -- 4096 streams with lengths log-uniform in [1 KiB, 1 MiB],
                   20 letters with Zipf(1.1) frequencies, 1024 patterns of
                   8..64 symbols drawn from the same letters, K = floor(m/10).
* ``multiword`` -- one 1 GiB byte stream, a 50/50 mixture of uniform random
                   bytes and printable-ASCII runs of geometric length (mean
                   40); 4096 patterns of 16..256 bytes from the same process,
                   K = floor(m/10); planted copies covering about 0.1 % of
                   the bytes.
* ``serving``   -- 2048 patterns of 16..128 bytes (mixture process),
                   K = floor(m/10), and 10,000 sessions that send 1..64 KiB
                   segments of a mixture-byte pool with Poisson arrivals.

Every generator is a pure function of its arguments and seed (numpy PCG64).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 17120356

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)
ZIPF20 = np.arange(ord("A"), ord("A") + 20, dtype=np.uint8)


def rng_for(cfg_id: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([SEED_BASE + cfg_id, sub]))


def zipf_probs(n: int = 20, s: float = 1.1) -> np.ndarray:
    w = 1.0 / np.arange(1, n + 1, dtype=np.float64) ** s
    return w / w.sum()


# ----------------------------------------------------------------- letters
class Letters:
    """A letter distribution: uniform over a set, Zipf over a set, or the
    byte mixture process (random-byte and printable runs)."""

    def __init__(self, kind: str, alphabet: np.ndarray | None = None, probs: np.ndarray | None = None,
                 mean_run: float = 40.0):
        self.kind = kind
        self.alphabet = alphabet
        self.probs = probs
        self.mean_run = mean_run

    def draw(self, rng: np.random.Generator, n: int) -> np.ndarray:
        if n <= 0:
            return np.zeros(0, dtype=np.uint8)
        if self.kind == "uniform":
            return self.alphabet[rng.integers(0, self.alphabet.size, size=n)]
        if self.kind == "weighted":
            # a 2^16-entry table with round(p * 2^16) slots per letter (relative
            # probability error below 0.1 % for the Zipf(1.1) letters), indexed
            # by uniform 16-bit draws: much faster than rng.choice for 10^8 draws
            return self._table()[rng.integers(0, 1 << 16, size=n, dtype=np.uint32)]
        if self.kind == "mixture":
            return mixture_bytes(rng, n, self.mean_run)
        raise ValueError(self.kind)

    def _table(self) -> np.ndarray:
        if getattr(self, "_tab", None) is None:
            counts = np.round(self.probs * (1 << 16)).astype(np.int64)
            counts[np.argmax(counts)] += (1 << 16) - counts.sum()
            self._tab = np.repeat(self.alphabet, counts)
        return self._tab

    def other_than(self, rng: np.random.Generator, old: int) -> int:
        """A letter different from ``old`` (for substitutions)."""
        while True:
            c = int(self.draw(rng, 1)[0])
            if c != old:
                return c


def mixture_bytes(rng: np.random.Generator, n: int, mean_run: float = 40.0, block: int = 1 << 26) -> np.ndarray:
    """Runs of geometric length (mean ``mean_run``) that are, by a fair coin,
    uniform random bytes 0x00-0xFF or printable ASCII 0x20-0x7E."""
    out = np.empty(n, dtype=np.uint8)
    p = 1.0 / mean_run
    pos = 0
    while pos < n:
        want = min(block, n - pos)
        nruns = int(want / mean_run * 1.2) + 16
        lens = rng.geometric(p, size=nruns)
        kinds = rng.integers(0, 2, size=nruns, dtype=np.uint8)
        cum = np.cumsum(lens)
        k = int(np.searchsorted(cum, want)) + 1
        lens, kinds = lens[:k], kinds[:k]
        # kind of every byte (np.repeat(kinds, lens)[:want], built as a
        # running XOR of the kind changes at the run starts: much faster)
        flips = np.zeros(want, dtype=np.uint8)
        starts = cum[:k - 1]
        flips[starts[starts < want]] = (kinds[1:] ^ kinds[:-1])[starts < want]
        kind_per_byte = np.bitwise_xor.accumulate(flips) ^ kinds[0]
        rnd = rng.integers(0, 256, size=want, dtype=np.uint16).astype(np.uint8)
        prn = rng.integers(0x20, 0x7F, size=want, dtype=np.uint16).astype(np.uint8)
        out[pos:pos + want] = np.where(kind_per_byte == 1, prn, rnd)
        pos += want
    return out


LETTERS_ACGT = Letters("uniform", ACGT)
LETTERS_ZIPF = Letters("weighted", ZIPF20, zipf_probs())
LETTERS_MIX = Letters("mixture")


# ----------------------------------------------------------------- dataclass
@dataclass
class Plant:
    stream: int
    site: int  # first overwritten byte
    pattern: int
    length: int  # length of the mutated copy
    edits: int  # number of edits applied


@dataclass
class Workload:
    name: str
    streams: list  # list of np.ndarray(uint8)
    patterns: list  # list of bytes
    ks: np.ndarray  # uint16 per pattern
    plants: list = field(default_factory=list)

    @property
    def cells(self) -> int:
        """Nominal pattern x text cells: sum over streams and patterns of m * n."""
        msum = sum(len(p) for p in self.patterns)
        return int(msum) * int(sum(int(s.size) for s in self.streams))

    @property
    def total_bytes(self) -> int:
        return int(sum(int(s.size) for s in self.streams))


# ----------------------------------------------------------------- helpers
def make_patterns(rng: np.random.Generator, count: int, mlo: int, mhi: int, letters: Letters):
    lens = rng.integers(mlo, mhi + 1, size=count)
    return [bytes(letters.draw(rng, int(m))) for m in lens]


def k_tenth(patterns) -> np.ndarray:
    """K = floor(m / 10) per pattern."""
    return np.array([len(p) // 10 for p in patterns], dtype=np.uint16)


def mutate(rng: np.random.Generator, pat: bytes, n_edits: int, letters: Letters) -> bytes:
    """Apply ``n_edits`` random single-symbol edits (substitution, insertion
    or deletion, chosen uniformly) at uniform positions."""
    s = bytearray(pat)
    for _ in range(n_edits):
        op = int(rng.integers(0, 3))
        if op == 2 and len(s) <= 1:
            op = 0
        if op == 0:  # substitution: always changes the letter
            j = int(rng.integers(0, len(s)))
            s[j] = letters.other_than(rng, s[j])
        elif op == 1:  # insertion
            j = int(rng.integers(0, len(s) + 1))
            s.insert(j, int(letters.draw(rng, 1)[0]))
        else:  # deletion
            j = int(rng.integers(0, len(s)))
            del s[j]
    return bytes(s)


def plant(rng: np.random.Generator, text: np.ndarray, patterns, count: int, max_edits,
          letters: Letters, stream: int = 0):
    """Overwrite ``count`` non-overlapping sites of ``text`` with mutated
    pattern copies.  The text is cut into ``count`` equal slots and each copy
    is placed at a uniform offset inside its slot (so sites never overlap).
    ``max_edits`` is an int or a per-pattern array."""
    plants = []
    n = text.size
    if count <= 0 or n == 0:
        return plants
    slot = n // count
    for q in range(count):
        pi = int(rng.integers(0, len(patterns)))
        emax = int(max_edits if np.isscalar(max_edits) else max_edits[pi])
        e = int(rng.integers(0, emax + 1))
        cp = mutate(rng, patterns[pi], e, letters)
        if len(cp) > slot:
            continue
        site = q * slot + int(rng.integers(0, slot - len(cp) + 1))
        text[site:site + len(cp)] = np.frombuffer(cp, dtype=np.uint8)
        plants.append(Plant(stream, site, pi, len(cp), e))
    return plants


# ----------------------------------------------------------------- configs
def tiny(n: int = 100_000, n_patterns: int = 16, n_plants: int = 200, seed_sub: int = 0) -> Workload:
    rng = rng_for(1, seed_sub)
    pats = make_patterns(rng, n_patterns, 8, 16, LETTERS_ACGT)
    text = LETTERS_ACGT.draw(rng, n)
    ks = np.full(n_patterns, 2, dtype=np.uint16)
    pl = plant(rng, text, pats, n_plants, 2, LETTERS_ACGT)
    return Workload("tiny", [text], pats, ks, pl)


def long_stream(n: int = 1 << 26, n_patterns: int = 256, n_plants: int = 10_000, seed_sub: int = 0) -> Workload:
    rng = rng_for(2, seed_sub)
    pats = make_patterns(rng, n_patterns, 16, 32, LETTERS_ACGT)
    text = LETTERS_ACGT.draw(rng, n)
    ks = np.full(n_patterns, 3, dtype=np.uint16)
    pl = plant(rng, text, pats, n_plants, 3, LETTERS_ACGT)
    return Workload("long", [text], pats, ks, pl)


def stream_lengths(rng: np.random.Generator, count: int, lo_log2: float = 10, hi_log2: float = 20) -> np.ndarray:
    return np.floor(2.0 ** rng.uniform(lo_log2, hi_log2, size=count)).astype(np.int64)


def batched(n_streams: int = 4096, n_patterns: int = 1024, lo_log2: float = 10, hi_log2: float = 20,
            seed_sub: int = 0) -> Workload:
    rng = rng_for(3, seed_sub)
    pats = make_patterns(rng, n_patterns, 8, 64, LETTERS_ZIPF)
    lens = stream_lengths(rng, n_streams, lo_log2, hi_log2)
    streams = [LETTERS_ZIPF.draw(rng, int(n)) for n in lens]
    return Workload("batched", streams, pats, k_tenth(pats), [])


def multiword(n: int = 1 << 30, n_patterns: int = 4096, plant_fraction: float = 0.001, seed_sub: int = 0) -> Workload:
    rng = rng_for(4, seed_sub)
    pats = make_patterns(rng, n_patterns, 16, 256, LETTERS_MIX)
    ks = k_tenth(pats)
    text = LETTERS_MIX.draw(rng, n)
    mean_m = float(np.mean([len(p) for p in pats]))
    count = int(round(plant_fraction * n / mean_m))
    pl = plant(rng, text, pats, count, ks, LETTERS_MIX)
    return Workload("multiword", [text], pats, ks, pl)


def serving_dictionary(n_patterns: int = 2048, seed_sub: int = 0):
    """2048 patterns of 16..128 bytes from the mixture process, K = floor(m/10)."""
    rng = rng_for(5, seed_sub)
    pats = make_patterns(rng, n_patterns, 16, 128, LETTERS_MIX)
    return pats, k_tenth(pats)


def serving_pool(pool_bytes: int = 1 << 28, seed_sub: int = 0) -> np.ndarray:
    """The byte pool segments are cut from (mixture process)."""
    return LETTERS_MIX.draw(rng_for(5, 100 + seed_sub), pool_bytes)


def serving_arrivals(n_sessions: int = 10_000, duration_s: float = 1.0, offered_gbps: float = 20.0,
                     pool_bytes: int = 1 << 28, seg_lo: int = 1024, seg_hi: int = 65536, seed_sub: int = 0):
    """Poisson segment arrivals: every session sends segments of U{seg_lo..seg_hi}
    bytes as a Poisson process whose rate makes the aggregate offered load
    ``offered_gbps`` GB/s (1e9 B/s).  Returns arrays (session, offset, length,
    arrival_s) sorted by arrival time; offsets are uniform in the pool."""
    rng = rng_for(5, 200 + seed_sub)
    mean_seg = (seg_lo + seg_hi) / 2.0
    rate = offered_gbps * 1e9 / mean_seg / max(1, n_sessions)  # per session, segments / s
    counts = rng.poisson(rate * duration_s, size=n_sessions)
    total = int(counts.sum())
    session = np.repeat(np.arange(n_sessions, dtype=np.uint64), counts)
    t = rng.uniform(0.0, duration_s, size=total)  # a Poisson process, given its count
    length = rng.integers(seg_lo, seg_hi + 1, size=total).astype(np.uint32)
    offset = (rng.random(total) * (pool_bytes - length)).astype(np.uint64)
    order = np.argsort(t, kind="stable")
    return session[order], offset[order], length[order], t[order]


def small_random(seed: int, n: int, n_patterns: int, mlo: int, mhi: int, alphabet: bytes, kmax: int | None = None,
                 n_plants: int = 0, n_streams: int = 1) -> Workload:
    """A small random case for parity tests: any alphabet, K in [0, min(kmax, m-1)]."""
    rng = np.random.Generator(np.random.PCG64([SEED_BASE, 1000 + seed]))
    letters = Letters("uniform", np.frombuffer(alphabet, dtype=np.uint8))
    pats = make_patterns(rng, n_patterns, mlo, mhi, letters)
    ks = []
    for p in pats:
        hi = len(p) - 1 if kmax is None else min(kmax, len(p) - 1)
        ks.append(int(rng.integers(0, hi + 1)))
    streams = []
    plants = []
    for s in range(n_streams):
        ns = n if n_streams == 1 else int(rng.integers(0, n + 1))
        t = letters.draw(rng, ns)
        plants += plant(rng, t, pats, min(n_plants, max(0, ns // 64)), np.array(ks), letters, stream=s)
        streams.append(t)
    return Workload("small", streams, pats, np.array(ks, dtype=np.uint16), plants)
