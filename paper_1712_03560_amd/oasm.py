"""ctypes binding of liboasm_gpu (the C ABI in include/oasm_gpu.h).

Argument marshalling only: every matching step runs in the library's HIP
kernels.  The functions below carry the C names; :class:`Matcher` wraps a
context for Python callers, and accepts numpy arrays, bytes, or torch tensors
(host or device) as stream data.  PyTorch is used only to hand device memory
and the current HIP stream to the library.

The library must have been built (``paper_1712_03560_amd.build.build()``);
importing this module without it raises ImportError, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboasm_gpu.so")

OASM_OK = 0
OASM_E_INVAL = -1
OASM_E_NOMEM = -2
OASM_E_AGAIN = -3
OASM_E_CLOSED = -4
OASM_E_DEVICE = -5

OASM_RULES_NONE = 0
OASM_RULES_PAPER = 1
OASM_RULES_ACC_LAST = 2
OASM_RULES_EQ3_GE = 4
OASM_RULES_START_ORDER = 8
OASM_RULES_DISJOINT = 16
OASM_FEED_LAST = 1
OASM_CFG_PLAIN = 1
OASM_CFG_KEEP_H = 2
OASM_CFG_NO_RAW = 4
OASM_CFG_AUTOTUNE = 8
OASM_CFG_GRAPHS = 16
OASM_CFG_NO_CUTOFF = 32
OASM_RAW = 0
OASM_FILTERED = 1
OASM_H = 2
OASM_MAX_PATTERN_LEN = 256
OASM_MAX_CHUNK_BYTES = 1 << 24
OASM_NOALLOC_MAX_PATTERNS = 65536

# every symbol the header declares (checked by the ABI test)
OASM_CKPT_MAGIC = 0x4D53414F  # a stream checkpoint's first word ("OASM")
OASM_CKPT_VERSION = 1

EXPORTED = [
    "oasm_config_init",
    "oasm_create",
    "oasm_feed",
    "oasm_feed_device",
    "oasm_feed_device_many",
    "oasm_close_stream",
    "oasm_sync",
    "oasm_hits",
    "oasm_queued",
    "oasm_serve",
    "oasm_get_stats",
    "oasm_destroy",
    "oasm_last_error",
    "oasm_status_str",
    "oasm_tune_report",
    "oasm_levcalc",
    "oasm_levcalc_size",
    "oasm_levcalc_noalloc",
    "oasm_stream_export",
    "oasm_stream_import",
]


class oasm_pattern(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_void_p), ("len", ctypes.c_uint32)]


class oasm_hit(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_uint64), ("end", ctypes.c_uint64), ("pattern", ctypes.c_uint32),
                ("dist", ctypes.c_uint32)]


class oasm_occ(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_uint64), ("start", ctypes.c_uint64), ("pattern", ctypes.c_uint32),
                ("len", ctypes.c_uint32), ("k", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class oasm_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device", ctypes.c_int32), ("hip_stream", ctypes.c_void_p),
                ("chunk_bytes", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("device_mem_budget", ctypes.c_uint64)]


class oasm_stats(ctypes.Structure):
    _fields_ = [("bytes_scanned", ctypes.c_uint64), ("word_steps", ctypes.c_uint64), ("cells", ctypes.c_uint64),
                ("raw_hits", ctypes.c_uint64), ("h_records", ctypes.c_uint64), ("occurrences", ctypes.c_uint64),
                ("syncs", ctypes.c_uint64), ("scan_ms", ctypes.c_double), ("step_ms", ctypes.c_double),
                ("scan_launches", ctypes.c_uint64), ("sync_wall_ms", ctypes.c_double), ("wait_ms", ctypes.c_double),
                ("host_ms", ctypes.c_double * 4), ("graph_replays", ctypes.c_uint64),
                ("word_steps_done", ctypes.c_uint64)]


class oasm_serve_report(ctypes.Structure):
    _fields_ = [("segments", ctypes.c_uint64), ("bytes", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("deferred", ctypes.c_uint64), ("max_batch_bytes", ctypes.c_uint64), ("wall_s", ctypes.c_double),
                ("busy_s", ctypes.c_double)]


SEG_DTYPE = np.dtype([("stream", "<u8"), ("offset", "<u8"), ("len", "<u4"), ("flags", "<u4"), ("arrival_s", "<f8")])
FEED_SEG_DTYPE = np.dtype([("stream", "<u8"), ("data", "<u8"), ("len", "<u8"), ("flags", "<u4"),
                           ("reserved", "<u4")])
HIT_DTYPE = np.dtype([("stream", "<u8"), ("end", "<u8"), ("pattern", "<u4"), ("dist", "<u4")])
OCC_DTYPE = np.dtype([("stream", "<u8"), ("start", "<u8"), ("pattern", "<u4"), ("len", "<u4"), ("k", "<u4"),
                      ("reserved", "<u4")])
assert HIT_DTYPE.itemsize == ctypes.sizeof(oasm_hit) == 24
assert OCC_DTYPE.itemsize == ctypes.sizeof(oasm_occ) == 32


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1712_03560_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    sz = ctypes.c_size_t
    lib.oasm_config_init.argtypes = [ctypes.POINTER(oasm_config)]
    lib.oasm_config_init.restype = i32
    lib.oasm_create.argtypes = [ctypes.POINTER(oasm_pattern), u32, P, ctypes.c_uint16, u32,
                                ctypes.POINTER(oasm_config), ctypes.POINTER(P)]
    lib.oasm_create.restype = i32
    lib.oasm_feed.argtypes = [P, u64, P, sz, u32]
    lib.oasm_feed.restype = i32
    lib.oasm_feed_device.argtypes = [P, u64, P, sz, P, u32]
    lib.oasm_feed_device_many.restype = i32
    lib.oasm_feed_device_many.argtypes = [P, P, sz, P]
    lib.oasm_feed_device.restype = i32
    lib.oasm_close_stream.argtypes = [P, u64]
    lib.oasm_close_stream.restype = i32
    lib.oasm_sync.argtypes = [P]
    lib.oasm_sync.restype = i32
    lib.oasm_hits.argtypes = [P, u32, P, sz, ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_int)]
    lib.oasm_hits.restype = i32
    lib.oasm_serve.argtypes = [P, P, sz, P, u64, P, ctypes.POINTER(oasm_serve_report)]
    lib.oasm_serve.restype = i32
    lib.oasm_queued.argtypes = [P, u32, ctypes.POINTER(sz)]
    lib.oasm_queued.restype = i32
    lib.oasm_get_stats.argtypes = [P, ctypes.POINTER(oasm_stats)]
    lib.oasm_get_stats.restype = i32
    lib.oasm_destroy.argtypes = [P]
    lib.oasm_destroy.restype = None
    lib.oasm_last_error.argtypes = [P]
    lib.oasm_last_error.restype = ctypes.c_char_p
    lib.oasm_tune_report.argtypes = [P]
    lib.oasm_tune_report.restype = ctypes.c_char_p
    lib.oasm_levcalc.argtypes = [P, P, sz, P, sz, P]
    lib.oasm_levcalc.restype = i32
    lib.oasm_levcalc_noalloc.argtypes = [P, P, sz, P, sz, P]
    lib.oasm_levcalc_noalloc.restype = i32
    lib.oasm_levcalc_size.argtypes = [P, sz, ctypes.POINTER(sz)]
    lib.oasm_levcalc_size.restype = i32
    lib.oasm_status_str.argtypes = [i32]
    lib.oasm_status_str.restype = ctypes.c_char_p
    lib.oasm_stream_export.argtypes = [P, u64, P, sz, ctypes.POINTER(sz)]
    lib.oasm_stream_export.restype = i32
    lib.oasm_stream_import.argtypes = [P, u64, P, sz]
    lib.oasm_stream_import.restype = i32
    return lib


lib = _load()


class OasmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{lib.oasm_status_str(status).decode()}: {msg}")
        self.status = status


# ------------------------------------------------------------- C-named calls
def oasm_config_init() -> oasm_config:
    cfg = oasm_config()
    lib.oasm_config_init(ctypes.byref(cfg))
    return cfg


def oasm_create(patterns, k, rules: int = OASM_RULES_PAPER, cfg: oasm_config | None = None) -> int:
    """Create a context; ``k`` is an int (all patterns) or a sequence."""
    pats = [bytes(p) for p in patterns]
    n = len(pats)
    bufs = [ctypes.create_string_buffer(p, len(p)) for p in pats]
    arr = (oasm_pattern * max(n, 1))()
    for i, b in enumerate(bufs):
        arr[i].bytes = ctypes.cast(b, ctypes.c_void_p)
        arr[i].len = len(pats[i])
    if np.isscalar(k):
        kptr, kall = None, int(k)
    else:
        karr = np.ascontiguousarray(k, dtype=np.uint16)
        if karr.size != n:
            raise ValueError("one K per pattern")
        kptr, kall = karr.ctypes.data_as(ctypes.c_void_p), 0
    out = ctypes.c_void_p()
    st = lib.oasm_create(arr, n, kptr, kall, rules, ctypes.byref(cfg) if cfg is not None else None,
                         ctypes.byref(out))
    if st != OASM_OK:
        raise OasmError(st, lib.oasm_last_error(None).decode())
    return out.value


def _check(ctx, st):
    if st != OASM_OK:
        raise OasmError(st, lib.oasm_last_error(ctx).decode())


def oasm_feed(ctx, stream_id: int, data, flags: int = 0):
    a = np.ascontiguousarray(np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else data,
                             dtype=np.uint8)
    _check(ctx, lib.oasm_feed(ctx, stream_id, a.ctypes.data_as(ctypes.c_void_p) if a.size else None, a.size, flags))


def oasm_feed_device(ctx, stream_id: int, ptr: int, n: int, hip_stream: int | None, flags: int = 0):
    _check(ctx, lib.oasm_feed_device(ctx, stream_id, ptr, n, hip_stream, flags))


def oasm_feed_device_many(ctx, segs: np.ndarray, hip_stream: int | None):
    """segs: a FEED_SEG_DTYPE array (stream, data = device address, len, flags, reserved)."""
    segs = np.ascontiguousarray(segs, dtype=FEED_SEG_DTYPE)
    _check(ctx, lib.oasm_feed_device_many(ctx, segs.ctypes.data if segs.size else None, segs.size, hip_stream))


def oasm_close_stream(ctx, stream_id: int):
    _check(ctx, lib.oasm_close_stream(ctx, stream_id))


def oasm_sync(ctx):
    _check(ctx, lib.oasm_sync(ctx))


def oasm_queued(ctx, kind: int) -> int:
    n = ctypes.c_size_t(0)
    _check(ctx, lib.oasm_queued(ctx, kind, ctypes.byref(n)))
    return n.value


def oasm_hits(ctx, kind: int) -> np.ndarray:
    """Drain every queued record of ``kind`` into a structured numpy array."""
    dt = HIT_DTYPE if kind == OASM_RAW else OCC_DTYPE
    total = oasm_queued(ctx, kind)
    buf = np.empty(total, dtype=dt)
    n = ctypes.c_size_t(0)
    more = ctypes.c_int(0)
    _check(ctx, lib.oasm_hits(ctx, kind, buf.ctypes.data_as(ctypes.c_void_p) if total else None, total,
                              ctypes.byref(n), ctypes.byref(more)))
    return buf[: n.value]


def oasm_serve(ctx, segs: np.ndarray, pool_ptr: int, pool_bytes: int, want_latency: bool = True):
    """Run the continuous-batching loop over a SEG_DTYPE array; returns (report dict, latencies or None)."""
    segs = np.ascontiguousarray(segs, dtype=SEG_DTYPE)
    lat = np.zeros(segs.size, dtype=np.float64) if want_latency else None
    rep = oasm_serve_report()
    _check(ctx, lib.oasm_serve(ctx, segs.ctypes.data_as(ctypes.c_void_p) if segs.size else None, segs.size,
                               pool_ptr, pool_bytes,
                               lat.ctypes.data_as(ctypes.c_void_p) if lat is not None and lat.size else None,
                               ctypes.byref(rep)))
    return {name: getattr(rep, name) for name, _ in oasm_serve_report._fields_}, lat


def oasm_stream_export(ctx, stream_id: int) -> bytes:
    """A stream's checkpoint (after matching every byte fed so far)."""
    size = ctypes.c_size_t(0)
    _check(ctx, lib.oasm_stream_export(ctx, stream_id, None, 0, ctypes.byref(size)))
    buf = ctypes.create_string_buffer(max(size.value, 1))
    _check(ctx, lib.oasm_stream_export(ctx, stream_id, buf, size.value, ctypes.byref(size)))
    return buf.raw[: size.value]


def oasm_stream_import(ctx, stream_id: int, blob: bytes):
    """Make `stream_id` a live stream of `ctx` holding a checkpoint's state."""
    blob = bytes(blob)
    _check(ctx, lib.oasm_stream_import(ctx, stream_id, blob, len(blob)))


def oasm_levcalc_size(ctx, n: int) -> int:
    out = ctypes.c_size_t(0)
    _check(ctx, lib.oasm_levcalc_size(ctx, n, ctypes.byref(out)))
    return out.value


def oasm_levcalc(ctx, text_ptr: int, n: int, out_ptr: int, out_bytes: int, hip_stream: int | None):
    _check(ctx, lib.oasm_levcalc(ctx, text_ptr, n, out_ptr, out_bytes, hip_stream))


def oasm_levcalc_noalloc(ctx, text_ptr: int, n: int, out_ptr: int, out_bytes: int, hip_stream: int | None):
    _check(ctx, lib.oasm_levcalc_noalloc(ctx, text_ptr, n, out_ptr, out_bytes, hip_stream))


def oasm_get_stats(ctx) -> dict:
    s = oasm_stats()
    _check(ctx, lib.oasm_get_stats(ctx, ctypes.byref(s)))
    d = {name: getattr(s, name) for name, _ in oasm_stats._fields_}
    d["host_ms"] = list(d["host_ms"])
    return d


def oasm_destroy(ctx):
    if ctx:
        lib.oasm_destroy(ctx)


def oasm_tune_report(ctx) -> str:
    return lib.oasm_tune_report(ctx).decode()


def oasm_last_error(ctx) -> str:
    return lib.oasm_last_error(ctx).decode()


# ------------------------------------------------------------- Python wrapper
@dataclass
class Results:
    raw: np.ndarray  # HIT_DTYPE
    occ: np.ndarray  # OCC_DTYPE
    h: np.ndarray | None = None  # OCC_DTYPE


class Matcher:
    """A dictionary of patterns matched against any number of streams."""

    def __init__(self, patterns, k, rules: int = OASM_RULES_PAPER, *, plain: bool = False, keep_h: bool = False,
                 no_raw: bool = False, chunk_bytes: int = 0, hip_stream: int | None = None, device: int = -1,
                 mem_budget: int = 0, autotune: bool = False, graphs: bool = False, cutoff: bool = True):
        cfg = oasm_config_init()
        cfg.device = device
        cfg.chunk_bytes = chunk_bytes
        cfg.flags = (OASM_CFG_PLAIN if plain else 0) | (OASM_CFG_KEEP_H if keep_h else 0) | (
            OASM_CFG_NO_RAW if no_raw else 0) | (OASM_CFG_AUTOTUNE if autotune else 0) | (
            OASM_CFG_GRAPHS if graphs else 0) | (0 if cutoff else OASM_CFG_NO_CUTOFF)
        cfg.device_mem_budget = mem_budget
        cfg.hip_stream = hip_stream
        self.keep_h = keep_h
        self._device_refs = []  # device tensors fed since the last sync
        self.ctx = oasm_create(patterns, k, rules, cfg)

    def feed(self, stream_id: int, data, last: bool = False):
        """Append bytes to a stream: bytes / numpy (host) or a torch uint8 tensor (host or device)."""
        flags = OASM_FEED_LAST if last else 0
        try:
            import torch  # only for device buffers and streams
        except ImportError:  # pragma: no cover
            torch = None
        if torch is not None and isinstance(data, torch.Tensor):
            if data.dtype != torch.uint8 or not data.is_contiguous():
                raise ValueError("stream tensors must be contiguous uint8")
            if data.is_cuda:
                hs = torch.cuda.current_stream(data.device).cuda_stream
                oasm_feed_device(self.ctx, stream_id, data.data_ptr(), data.numel(), hs, flags)
                self._device_refs.append(data)  # the library reads it until the next sync
                return
            data = data.numpy()
        oasm_feed(self.ctx, stream_id, data, flags)

    def feed_many(self, items):
        """Append many device tensors in one call: items = [(stream_id, tensor, last), ...],
        each a contiguous uint8 CUDA tensor on the current stream's device."""
        import torch  # only for device buffers and streams

        if not items:
            return
        for _, t, _ in items:
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.uint8 or not t.is_contiguous():
                raise ValueError("feed_many takes contiguous uint8 CUDA tensors")
        segs = np.zeros(len(items), dtype=FEED_SEG_DTYPE)
        segs["stream"] = [sid for sid, _, _ in items]
        segs["data"] = [t.data_ptr() for _, t, _ in items]
        segs["len"] = [t.numel() for _, t, _ in items]
        segs["flags"] = [OASM_FEED_LAST if last else 0 for _, _, last in items]
        self.feed_segs(segs, [t for _, t, _ in items], torch.cuda.current_stream(items[0][1].device).cuda_stream)

    def feed_segs(self, segs: np.ndarray, keep=(), hip_stream: int | None = None):
        """The raw batched device feed: `segs` is a FEED_SEG_DTYPE array of
        device addresses; `keep` holds the objects that own that memory (kept
        alive until the next sync); `hip_stream` is the stream the data was
        produced on (None = the library's stream)."""
        oasm_feed_device_many(self.ctx, segs, hip_stream)
        self._device_refs.extend(keep)

    def close(self, stream_id: int):
        oasm_close_stream(self.ctx, stream_id)

    def sync(self):
        oasm_sync(self.ctx)
        self._device_refs.clear()

    def results(self) -> Results:
        raw = oasm_hits(self.ctx, OASM_RAW)
        occ = oasm_hits(self.ctx, OASM_FILTERED)
        h = oasm_hits(self.ctx, OASM_H) if self.keep_h else None
        return Results(raw, occ, h)

    def serve(self, segs: np.ndarray, pool, want_latency: bool = True):
        """Continuous batching over segments of a device-resident pool (a CUDA uint8 tensor)."""
        import torch  # only for the device pool

        if not isinstance(pool, torch.Tensor) or not pool.is_cuda or pool.dtype != torch.uint8:
            raise ValueError("the pool must be a CUDA uint8 tensor")
        torch.cuda.current_stream(pool.device).synchronize()
        return oasm_serve(self.ctx, segs, pool.data_ptr(), pool.numel(), want_latency)

    def levcalc(self, text, out=None):
        """LEV CALC for every start of `text` (a contiguous uint8 CUDA tensor):
        a uint8 CUDA tensor of oasm_levcalc_size bytes (pattern-major, start i
        of pattern p at offset n * unit[p] + i * (2K_p + 1)), queued on the
        current stream.  `out` may supply the output tensor."""
        import torch  # only for device buffers and streams

        if not isinstance(text, torch.Tensor) or not text.is_cuda or text.dtype != torch.uint8 or \
                not text.is_contiguous():
            raise ValueError("levcalc takes a contiguous uint8 CUDA tensor")
        n = text.numel()
        need = oasm_levcalc_size(self.ctx, n)
        if out is None:
            out = torch.empty(max(need, 1), dtype=torch.uint8, device=text.device)
        elif not out.is_cuda or out.dtype != torch.uint8 or not out.is_contiguous() or out.numel() < need:
            raise ValueError("out must be a contiguous uint8 CUDA tensor of at least oasm_levcalc_size bytes")
        hs = torch.cuda.current_stream(text.device).cuda_stream
        oasm_levcalc(self.ctx, text.data_ptr() if n else None, n, out.data_ptr(), out.numel(), hs)
        return out[:need]

    def export_stream(self, stream_id: int) -> bytes:
        """Checkpoint of a live stream (matches every byte fed so far first)."""
        return oasm_stream_export(self.ctx, stream_id)

    def import_stream(self, stream_id: int, blob: bytes):
        """Resume a checkpointed stream under `stream_id` (same dictionary)."""
        oasm_stream_import(self.ctx, stream_id, blob)

    def stats(self) -> dict:
        return oasm_get_stats(self.ctx)

    def tune_report(self) -> str:
        return oasm_tune_report(self.ctx)

    def destroy(self):
        if self.ctx:
            oasm_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
