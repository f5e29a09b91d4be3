"""Host-side behaviour of the benchmark script (no GPU needed): the one-GPU
contract and the word-step count of the LEV CALC band cutoff."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    # exits before anything touches a GPU
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--no-valu-probe"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_levcalc_word_steps():
    # one-word columns and columns whose first output is the first step are never cut
    for m in (1, 5, 32):
        for K in range(m):
            band, full = bench.levcalc_word_steps(m, K)
            assert band == full == (m + K) * 1
    for m, K in ((33, 32), (256, 255)):
        band, full = bench.levcalc_word_steps(m, K)
        assert band == full
    # otherwise the band advances no more words than the full column, and at least one per step
    for m in (33, 64, 65, 100, 200, 256):
        for K in (0, 3, m // 10, m // 2):
            band, full = bench.levcalc_word_steps(m, K)
            W = (m + 31) // 32
            assert m + K <= band <= full == (m + K) * W
            if (K + 1 + 31) // 32 < W and m - K - 1 > 0:
                assert band < full  # the first step needs fewer than W words
            # the 2K + 1 output steps always advance all W words
            assert band >= (2 * K + 1) * W
