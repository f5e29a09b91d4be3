"""Seeded input generators: determinism and shapes (no GPU)."""
import numpy as np

from paper_1712_03560_amd import workloads as W


def test_tiny_shapes_and_determinism():
    a, b = W.tiny(), W.tiny()
    assert a.streams[0].size == 100_000
    assert len(a.patterns) == 16 and all(8 <= len(p) <= 16 for p in a.patterns)
    assert (a.ks == 2).all()
    assert set(np.unique(a.streams[0]).tolist()) <= set(b"ACGT")
    assert np.array_equal(a.streams[0], b.streams[0]) and a.patterns == b.patterns
    assert len(a.plants) == 200


def test_long_shapes_small():
    w = W.long_stream(n=1 << 20, n_plants=100)
    assert w.streams[0].size == 1 << 20
    assert len(w.patterns) == 256 and all(16 <= len(p) <= 32 for p in w.patterns)
    assert (w.ks == 3).all()


def test_batched_shapes_small():
    w = W.batched(n_streams=64, n_patterns=32)
    assert len(w.streams) == 64
    lens = np.array([s.size for s in w.streams])
    assert lens.min() >= 1024 and lens.max() <= 1 << 20
    assert all(8 <= len(p) <= 64 for p in w.patterns)
    assert list(w.ks) == [len(p) // 10 for p in w.patterns]
    allb = np.concatenate(w.streams)
    assert set(np.unique(allb).tolist()) <= set(range(ord("A"), ord("A") + 20))
    # Zipf: the first letter is the most frequent
    cnt = np.bincount(allb, minlength=256)
    assert cnt[ord("A")] == cnt.max()


def test_mixture_process():
    rng = W.rng_for(4, 99)
    x = W.mixture_bytes(rng, 1 << 20)
    printable = ((x >= 0x20) & (x <= 0x7E)).mean()
    # half the runs are printable, and ~37 % of uniform bytes are printable too
    assert 0.6 < printable < 0.75


def test_mutate_edit_count_bound():
    rng = np.random.default_rng(0)
    for _ in range(200):
        p = bytes(rng.integers(65, 69, size=int(rng.integers(2, 20))).astype(np.uint8))
        e = int(rng.integers(0, 4))
        q = W.mutate(rng, p, e, W.LETTERS_ACGT)
        assert abs(len(q) - len(p)) <= e
