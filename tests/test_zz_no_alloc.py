"""The allocation-free LEV CALC entry point (needs an MI355X), called through
the C ABI: its output equals oasm_levcalc's byte for byte on consecutive
calls, the second with a smaller text, then from a second context with a
smaller dictionary (which rewrites the shared table array) and from the
first context again; a spot check against the oracle; and the refusal of a
dictionary above the table array's size."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_1712_03560_amd import oasm  # noqa: E402
from paper_1712_03560_amd import workloads as W  # noqa: E402


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


def both(mt, text):
    """oasm_levcalc and oasm_levcalc_noalloc on the same text, each into its
    own output (filled with different bytes first)."""
    n = text.numel()
    need = oasm.oasm_levcalc_size(mt.ctx, n)
    ref = torch.full((max(need, 1),), 77, dtype=torch.uint8, device="cuda")
    got = torch.full((max(need, 1),), 99, dtype=torch.uint8, device="cuda")
    hs = torch.cuda.current_stream().cuda_stream
    ctx = ctypes.c_void_p(mt.ctx)
    st = oasm.lib.oasm_levcalc(ctx, text.data_ptr(), n, ref.data_ptr(), ref.numel(), hs)
    assert st == oasm.OASM_OK, oasm.oasm_last_error(mt.ctx)
    st = oasm.lib.oasm_levcalc_noalloc(ctx, text.data_ptr(), n, got.data_ptr(), got.numel(), hs)
    assert st == oasm.OASM_OK, oasm.oasm_last_error(mt.ctx)
    torch.cuda.synchronize()
    return ref[:need], got[:need]


def test_noalloc_equals_levcalc_on_consecutive_calls():
    a = W.small_random(91, 1000, 40, 1, 256, bytes(range(256)), kmax=20, n_plants=0)
    b = W.small_random(92, 1000, 9, 4, 70, b"ACGT", kmax=6, n_plants=0)
    rng = np.random.default_rng(93)
    t1 = torch.from_numpy(rng.integers(0, 256, size=70_001).astype(np.uint8)).cuda()
    t2 = torch.from_numpy(rng.integers(0, 256, size=3_001).astype(np.uint8)).cuda()
    t3 = torch.from_numpy(np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, size=5_000)].copy()).cuda()
    with oasm.Matcher(a.patterns, a.ks) as ma, oasm.Matcher(b.patterns, b.ks) as mb:
        for label, mt, text in (("A, 70,001 bytes", ma, t1), ("A, 3,001 bytes", ma, t2),
                                ("B, 5,000 bytes", mb, t3), ("A, 3,001 bytes again", ma, t2)):
            ref, got = both(mt, text)
            say(f"noalloc {label}: {ref.numel()} distances")
            assert ref.numel() > 0 and torch.equal(ref, got), f"{label}: outputs differ"
        # spot check of the last call against the oracle, pattern by pattern
        flat = got.cpu().numpy()
        txt = t2.cpu().numpy()
        off = 0
        for p, K in zip(a.patterns, a.ks):
            K = int(K)
            blk = flat[off:off + txt.size * (2 * K + 1)].reshape(txt.size, 2 * K + 1)
            assert np.array_equal(blk[:200], oracle.levcalc(p, txt[:200 + len(p) + K], K)[:200])
            off += txt.size * (2 * K + 1)


def test_noalloc_refuses_dictionaries_above_the_table_size():
    pats = [bytes([65 + (i % 4)]) for i in range(oasm.OASM_NOALLOC_MAX_PATTERNS + 1)]
    text = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with oasm.Matcher(pats, 0) as mt:
        need = oasm.oasm_levcalc_size(mt.ctx, 16)
        out = torch.empty(need, dtype=torch.uint8, device="cuda")
        st = oasm.lib.oasm_levcalc_noalloc(ctypes.c_void_p(mt.ctx), text.data_ptr(), 16, out.data_ptr(), need,
                                           torch.cuda.current_stream().cuda_stream)
        assert st == oasm.OASM_E_INVAL
        assert "OASM_NOALLOC_MAX_PATTERNS" in oasm.oasm_last_error(mt.ctx)
