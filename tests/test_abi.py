"""C ABI: the built library exports every function include/oasm_gpu.h declares,
and argument checks that need no device (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oasm_gpu.h")
LIB = os.path.join(ROOT, "paper_1712_03560_amd", "liboasm_gpu.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1712_03560_amd import build

        build.build()
    return ctypes.CDLL(LIB)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(oasm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("oasm_create", "oasm_feed", "oasm_feed_device", "oasm_sync", "oasm_hits", "oasm_close_stream",
                 "oasm_destroy", "oasm_last_error"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_lists_every_symbol():
    from paper_1712_03560_amd import oasm

    assert sorted(oasm.EXPORTED) == declared_functions()


def test_record_layouts():
    from paper_1712_03560_amd import oasm

    assert ctypes.sizeof(oasm.oasm_hit) == 24
    assert ctypes.sizeof(oasm.oasm_occ) == 32
    assert ctypes.sizeof(oasm.oasm_config) == 32
    assert ctypes.sizeof(oasm.oasm_stats) == 136
    assert ctypes.sizeof(oasm.oasm_serve_report) == 56
    assert oasm.SEG_DTYPE.itemsize == 32


def test_status_strings(lib):
    lib.oasm_status_str.restype = ctypes.c_char_p
    assert lib.oasm_status_str(0) == b"OASM_OK"
    assert lib.oasm_status_str(-1) == b"OASM_E_INVAL"
    assert lib.oasm_status_str(-5) == b"OASM_E_DEVICE"


@pytest.mark.parametrize("pats,k", [
    ([], 0),               # empty dictionary
    ([b""], 0),            # empty pattern
    ([b"ACGT"], 4),        # K must be < len (Section 6.3)
    ([b"A" * 257], 1),     # longer than OASM_MAX_PATTERN_LEN
    ([b"A" * 100], 64),    # K above the filter's 63 levels
])
def test_create_rejects_bad_dictionaries(pats, k):
    from paper_1712_03560_amd import oasm

    with pytest.raises(oasm.OasmError) as ei:
        oasm.oasm_create(pats, k)
    assert ei.value.status == oasm.OASM_E_INVAL


def test_null_arguments(lib):
    lib.oasm_sync.argtypes = [ctypes.c_void_p]
    assert lib.oasm_sync(None) == -1
    lib.oasm_feed.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32]
    assert lib.oasm_feed(None, 0, None, 0, 0) == -1
    lib.oasm_destroy.argtypes = [ctypes.c_void_p]
    lib.oasm_destroy(None)  # no-op
