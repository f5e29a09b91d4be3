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
    assert ctypes.sizeof(oasm.oasm_stats) == 144
    assert ctypes.sizeof(oasm.oasm_serve_report) == 56
    assert oasm.SEG_DTYPE.itemsize == 32


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that a C compiler gives the header's struct."""
    import shutil
    import subprocess

    from paper_1712_03560_amd import oasm

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"oasm_config": oasm.oasm_config, "oasm_stats": oasm.oasm_stats,
               "oasm_serve_report": oasm.oasm_serve_report}
    dtypes = {"oasm_segment": oasm.SEG_DTYPE, "oasm_hit": oasm.HIT_DTYPE, "oasm_occ": oasm.OCC_DTYPE,
              "oasm_feed_seg": oasm.FEED_SEG_DTYPE}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "oasm_gpu.h"', "int main(void) {"]
    for name, fields in [(n, [f for f, _ in c._fields_]) for n, c in structs.items()] + \
            [(n, list(d.names)) for n, d in dtypes.items()]:
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field in fields:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(x.split()[:2]): int(x.split()[2]) for x in out if x}
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
    for name, dt in dtypes.items():
        assert got[(name, "size")] == dt.itemsize, name
        for field in dt.names:
            assert got[(name, field)] == dt.fields[field][1], (name, field)


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
    lib.oasm_levcalc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                 ctypes.c_size_t, ctypes.c_void_p]
    assert lib.oasm_levcalc(None, None, 0, None, 0, None) == -1
    lib.oasm_levcalc_size.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    out = ctypes.c_size_t(7)
    assert lib.oasm_levcalc_size(None, 10, ctypes.byref(out)) == -1


@pytest.mark.parametrize("chunk", [(1 << 24) + 64, 0xFFFFFFC0])
def test_create_rejects_oversized_chunks(chunk):
    """A scan record keeps a hit end's offset inside its chunk in 24 bits, so
    chunks above OASM_MAX_CHUNK_BYTES are refused before any device work."""
    from paper_1712_03560_amd import oasm

    cfg = oasm.oasm_config_init()
    cfg.chunk_bytes = chunk
    with pytest.raises(oasm.OasmError) as ei:
        oasm.oasm_create([b"ACGT"], 1, cfg=cfg)
    assert ei.value.status == oasm.OASM_E_INVAL
    assert "chunk_bytes" in oasm.oasm_last_error(None)


def test_serve_writes_the_report_on_errors(lib):
    """oasm_serve fills its report on every return, errors included."""
    from paper_1712_03560_amd import oasm

    rep = oasm.oasm_serve_report()
    rep.segments = rep.bytes = rep.steps = 77
    lib.oasm_serve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_uint64,
                               ctypes.c_void_p, ctypes.POINTER(oasm.oasm_serve_report)]
    assert lib.oasm_serve(None, None, 0, None, 0, None, ctypes.byref(rep)) == oasm.OASM_E_INVAL
    assert (rep.segments, rep.bytes, rep.steps) == (0, 0, 0)


def test_checkpoint_calls_reject_null_context(lib):
    """The checkpoint entry points refuse a NULL context without touching a
    device (OASM_E_INVAL = -1)."""
    size = ctypes.c_size_t(7)
    lib.oasm_stream_export.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.POINTER(ctypes.c_size_t)]
    lib.oasm_stream_import.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t]
    assert lib.oasm_stream_export(None, 1, None, 0, ctypes.byref(size)) == -1
    assert lib.oasm_stream_import(None, 1, None, 0) == -1


def test_checkpoint_constants_match_the_header():
    from paper_1712_03560_amd import oasm

    text = open(HEADER).read()
    magic = int(re.search(r"#define OASM_CKPT_MAGIC (0x[0-9A-Fa-f]+)u", text).group(1), 16)
    version = int(re.search(r"#define OASM_CKPT_VERSION (\d+)u", text).group(1))
    assert (magic, version) == (oasm.OASM_CKPT_MAGIC, oasm.OASM_CKPT_VERSION)
    assert magic.to_bytes(4, "little") == b"OASM"
