"""ctypes binding of ``include/zipnn.h`` (libzipnn_hip.so).

The ``zipnn_*`` functions mirror the C ABI one to one and only marshal
arguments; every step of compression and decompression runs in the HIP
kernels of the library.  ``Codec`` adds tensor-level conveniences on top (it
allocates device buffers with PyTorch and passes their pointers and the
current HIP stream).  There is no fallback: if the library is missing or no
GPU is visible, calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzipnn_hip.so")

ZIPNN_OK, ZIPNN_E_INVAL, ZIPNN_E_FORMAT, ZIPNN_E_CORRUPT = 0, -1, -2, -3
ZIPNN_E_NOSPACE, ZIPNN_E_NOMEM, ZIPNN_E_HIP, ZIPNN_E_BUSY, ZIPNN_E_TOOBIG = -4, -5, -6, -7, -8
ZIPNN_NOALLOC_SCRATCH_BYTES = 32 << 20
ZIPNN_BF16, ZIPNN_FP16, ZIPNN_FP32, ZIPNN_FP8_E4M3, ZIPNN_U8 = 1, 2, 3, 4, 5
ZIPNN_AUTO, ZIPNN_HUF, ZIPNN_RAW, ZIPNN_ZG = 0, 1, 2, 3
WIDTH = {ZIPNN_BF16: 2, ZIPNN_FP16: 2, ZIPNN_FP32: 4, ZIPNN_FP8_E4M3: 1, ZIPNN_U8: 1}

# every symbol declared in include/zipnn.h
EXPORTS = [
    "zipnn_strerror", "zipnn_ctx_create", "zipnn_ctx_destroy", "zipnn_ctx_status", "zipnn_default_params",
    "zipnn_check_params", "zipnn_compress_bound", "zipnn_compress", "zipnn_compress_noalloc", "zipnn_decompress",
    "zipnn_decompress_async",
    "zipnn_inspect", "zipnn_compress_batch", "zipnn_encoder_create", "zipnn_encoder_run", "zipnn_encoder_destroy",
    "zipnn_batch_create", "zipnn_batch_decompress", "zipnn_batch_destroy",
    "zipnn_decompress_batch", "zipnn_autotune", "zipnn_clock", "zipnn_server_create", "zipnn_server_destroy",
    "zipnn_server_register", "zipnn_server_submit", "zipnn_server_poll", "zipnn_server_next_done",
    "zipnn_server_release", "zipnn_server_stats", "zipnn_server_set_mode",
]
ZIPNN_SERVE_CONTINUOUS, ZIPNN_SERVE_PER_REQUEST = 0, 1


class ZipnnError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        msg = lib().zipnn_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})" if where else f"{msg} ({code})")


class zipnn_params(ctypes.Structure):
    _fields_ = [("chunk_bytes", ctypes.c_uint32), ("substream_syms", ctypes.c_uint16),
                ("group", ctypes.c_uint8), ("max_code_len", ctypes.c_uint8), ("policy", ctypes.c_uint8 * 4),
                ("probe_skip", ctypes.c_uint8), ("exponent", ctypes.c_uint8), ("reserved", ctypes.c_uint8 * 2)]

    def __repr__(self):
        return (f"zipnn_params(chunk_bytes={self.chunk_bytes}, S={self.substream_syms}, g={self.group}, "
                f"L={self.max_code_len}, policy={list(self.policy)}, K={self.probe_skip}, exp={self.exponent})")


class zipnn_info(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("B", ctypes.c_int), ("n_elems", ctypes.c_uint64),
                ("total_bytes", ctypes.c_uint64), ("n_chunks", ctypes.c_uint32), ("chunk_bytes", ctypes.c_uint32),
                ("S", ctypes.c_uint32), ("g", ctypes.c_uint32), ("L", ctypes.c_uint32), ("is_delta", ctypes.c_int),
                ("bytes_by_mode", ctypes.c_uint64 * 4), ("entries_by_mode", ctypes.c_uint64 * 4)]


class zipnn_tune_entry(ctypes.Structure):
    _fields_ = [("params", zipnn_params), ("ratio", ctypes.c_double), ("decode_gbps", ctypes.c_double),
                ("encode_gbps", ctypes.c_double)]


class zipnn_tune_config(ctypes.Structure):
    _fields_ = [("sample_bytes", ctypes.c_uint64), ("min_chunk", ctypes.c_uint32), ("max_chunk", ctypes.c_uint32),
                ("repeats", ctypes.c_int), ("max_ratio_loss", ctypes.c_double), ("tie", ctypes.c_double),
                ("policy", ctypes.c_uint8 * 4)]


class zipnn_tensor_in(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("n_elems", ctypes.c_uint64), ("base", ctypes.c_void_p)]


class zipnn_server_config(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_int), ("chunks_per_iter", ctypes.c_uint32),
                ("mode", ctypes.c_int)]


class zipnn_timing(ctypes.Structure):
    _fields_ = [("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class zipnn_server_counters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("released", ctypes.c_uint64),
                ("iterations", ctypes.c_uint64), ("chunks", ctypes.c_uint64), ("bytes_out", ctypes.c_uint64),
                ("pool_in_use", ctypes.c_uint64), ("pool_peak", ctypes.c_uint64), ("active_peak", ctypes.c_int)]


_lib = None


def lib():
    """Load libzipnn_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2411_05239_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        P = ctypes.POINTER
        L.zipnn_strerror.argtypes, L.zipnn_strerror.restype = [i32], ctypes.c_char_p
        L.zipnn_ctx_create.argtypes, L.zipnn_ctx_create.restype = [i32, P(vp)], i32
        L.zipnn_ctx_destroy.argtypes, L.zipnn_ctx_destroy.restype = [vp], None
        L.zipnn_ctx_status.argtypes, L.zipnn_ctx_status.restype = [vp, vp, i32], i32
        L.zipnn_default_params.argtypes, L.zipnn_default_params.restype = [i32, P(zipnn_params)], None
        L.zipnn_check_params.argtypes, L.zipnn_check_params.restype = [i32, P(zipnn_params)], i32
        L.zipnn_compress_bound.argtypes, L.zipnn_compress_bound.restype = [i32, u64, P(zipnn_params)], u64
        L.zipnn_compress.argtypes = [vp, vp, i32, u64, vp, P(zipnn_params), vp, u64, P(u64), vp]
        L.zipnn_compress.restype = i32
        L.zipnn_compress_noalloc.argtypes = [vp, vp, i32, u64, vp, P(zipnn_params), vp, u64, P(u64), vp]
        L.zipnn_compress_noalloc.restype = i32
        L.zipnn_decompress.argtypes, L.zipnn_decompress.restype = [vp, vp, u64, vp, vp, u64, vp], i32
        L.zipnn_decompress_async.argtypes = [vp, ctypes.c_char_p, vp, u64, vp, vp, u64, vp]
        L.zipnn_decompress_async.restype = i32
        L.zipnn_inspect.argtypes, L.zipnn_inspect.restype = [vp, u64, P(zipnn_info)], i32
        L.zipnn_compress_batch.argtypes = [vp, i32, P(zipnn_tensor_in), i32, P(zipnn_params), vp, u64, P(u64), vp]
        L.zipnn_compress_batch.restype = i32
        L.zipnn_encoder_create.argtypes = [vp, i32, P(zipnn_tensor_in), i32, P(zipnn_params), vp, u64, P(vp)]
        L.zipnn_encoder_create.restype = i32
        L.zipnn_encoder_run.argtypes, L.zipnn_encoder_run.restype = [vp, vp, P(u64)], i32
        L.zipnn_encoder_destroy.argtypes, L.zipnn_encoder_destroy.restype = [vp], None
        L.zipnn_batch_create.argtypes = [vp, vp, P(u64), i32, P(vp), P(u64), P(vp), P(vp)]
        L.zipnn_batch_create.restype = i32
        L.zipnn_batch_decompress.argtypes, L.zipnn_batch_decompress.restype = [vp, vp], i32
        L.zipnn_batch_destroy.argtypes, L.zipnn_batch_destroy.restype = [vp], None
        L.zipnn_decompress_batch.argtypes = [vp, vp, P(u64), i32, P(vp), P(u64), P(vp), vp]
        L.zipnn_decompress_batch.restype = i32
        L.zipnn_autotune.argtypes = [vp, i32, P(zipnn_tensor_in), i32, P(zipnn_tune_config), P(zipnn_params),
                                     P(zipnn_tune_entry), i32, P(i32)]
        L.zipnn_autotune.restype = i32
        L.zipnn_clock.argtypes, L.zipnn_clock.restype = [], ctypes.c_double
        L.zipnn_server_create.argtypes = [vp, P(zipnn_server_config), P(vp)]
        L.zipnn_server_create.restype = i32
        L.zipnn_server_destroy.argtypes, L.zipnn_server_destroy.restype = [vp], None
        L.zipnn_server_register.argtypes = [vp, vp, u64, vp, P(ctypes.c_uint32)]
        L.zipnn_server_register.restype = i32
        L.zipnn_server_submit.argtypes = [vp, ctypes.c_uint32, ctypes.c_double, P(u64)]
        L.zipnn_server_submit.restype = i32
        L.zipnn_server_poll.argtypes, L.zipnn_server_poll.restype = [vp, u64, P(vp), P(zipnn_timing)], i32
        L.zipnn_server_next_done.argtypes = [vp, ctypes.c_double, P(u64)]
        L.zipnn_server_next_done.restype = i32
        L.zipnn_server_release.argtypes, L.zipnn_server_release.restype = [vp, u64], i32
        L.zipnn_server_stats.argtypes = [vp, P(zipnn_server_counters)]
        L.zipnn_server_stats.restype = i32
        L.zipnn_server_set_mode.argtypes = [vp, i32]
        L.zipnn_server_set_mode.restype = i32
        _lib = L
    return _lib


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise ZipnnError(rc, where)
    return rc


# ---------------------------------------------------------------- C ABI mirror

def zipnn_strerror(code: int) -> str:
    return lib().zipnn_strerror(code).decode()


def zipnn_ctx_create(device: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().zipnn_ctx_create(device, ctypes.byref(h)), "zipnn_ctx_create")
    return h.value


def zipnn_ctx_destroy(ctx: int) -> None:
    lib().zipnn_ctx_destroy(ctx)


def zipnn_ctx_status(ctx: int, stream: int, clear: bool = False) -> int:
    return lib().zipnn_ctx_status(ctx, stream, 1 if clear else 0)


def zipnn_default_params(dtype: int) -> zipnn_params:
    p = zipnn_params()
    lib().zipnn_default_params(dtype, ctypes.byref(p))
    return p


def zipnn_check_params(dtype: int, p: zipnn_params) -> int:
    return lib().zipnn_check_params(dtype, ctypes.byref(p))


def zipnn_compress_bound(dtype: int, n: int, p: zipnn_params) -> int:
    return lib().zipnn_compress_bound(dtype, n, ctypes.byref(p))


def zipnn_compress(ctx, src, dtype, n, base, p, dst, dst_cap, stream) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().zipnn_compress(ctx, src, dtype, n, base, ctypes.byref(p), dst, dst_cap, ctypes.byref(out), stream),
           "zipnn_compress")
    return out.value


def zipnn_compress_noalloc(ctx, src, dtype, n, base, p, dst, dst_cap, stream) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().zipnn_compress_noalloc(ctx, src, dtype, n, base, ctypes.byref(p), dst, dst_cap, ctypes.byref(out),
                                        stream), "zipnn_compress_noalloc")
    return out.value


def zipnn_decompress(ctx, src, src_len, base, dst, dst_cap, stream) -> None:
    _check(lib().zipnn_decompress(ctx, src, src_len, base, dst, dst_cap, stream), "zipnn_decompress")


def zipnn_decompress_async(ctx, header: bytes, src, src_len, base, dst, dst_cap, stream) -> None:
    assert len(header) >= 64
    _check(lib().zipnn_decompress_async(ctx, bytes(header[:64]), src, src_len, base, dst, dst_cap, stream),
           "zipnn_decompress_async")


def zipnn_inspect(host_bytes: bytes) -> zipnn_info:
    info = zipnn_info()
    buf = ctypes.create_string_buffer(bytes(host_bytes), len(host_bytes))
    _check(lib().zipnn_inspect(buf, len(host_bytes), ctypes.byref(info)), "zipnn_inspect")
    return info


def _u64s(vals):
    return (ctypes.c_uint64 * len(vals))(*vals)


def _ptrs(vals):
    return (ctypes.c_void_p * len(vals))(*[v if v else None for v in vals])


def zipnn_compress_batch(ctx, dtype, srcs, ns, bases, p, arena, arena_cap, stream) -> list:
    n = len(srcs)
    ts = (zipnn_tensor_in * n)(*[zipnn_tensor_in(s_, n_, b_) for s_, n_, b_ in zip(srcs, ns, bases)])
    offs = (ctypes.c_uint64 * (n + 1))()
    _check(lib().zipnn_compress_batch(ctx, dtype, ts, n, ctypes.byref(p), arena, arena_cap, offs, stream),
           "zipnn_compress_batch")
    return list(offs)


def zipnn_batch_create(ctx, arena, offsets, dsts, caps, bases=None) -> int:
    n = len(dsts)
    h = ctypes.c_void_p()
    _check(lib().zipnn_batch_create(ctx, arena, _u64s(offsets), n, _ptrs(dsts), _u64s(caps),
                                    _ptrs(bases) if bases is not None else None, ctypes.byref(h)),
           "zipnn_batch_create")
    return h.value


def zipnn_batch_decompress(b, stream) -> None:
    _check(lib().zipnn_batch_decompress(b, stream), "zipnn_batch_decompress")


def zipnn_batch_destroy(b) -> None:
    lib().zipnn_batch_destroy(b)


def zipnn_decompress_batch(ctx, arena, offsets, dsts, caps, bases, stream) -> None:
    _check(lib().zipnn_decompress_batch(ctx, arena, _u64s(offsets), len(dsts), _ptrs(dsts), _u64s(caps),
                                        _ptrs(bases) if bases is not None else None, stream),
           "zipnn_decompress_batch")


def zipnn_autotune(ctx, dtype, srcs, ns, bases, sample_bytes=1 << 30, max_ratio_loss=0.01, policy=None,
                   min_chunk=0, max_chunk=0, repeats=0, tie=0.0):
    """-> (best zipnn_params, list of zipnn_tune_entry)"""
    n = len(srcs)
    ts = (zipnn_tensor_in * n)(*[zipnn_tensor_in(s_, n_, b_) for s_, n_, b_ in zip(srcs, ns, bases)])
    cfg = zipnn_tune_config(sample_bytes, min_chunk, max_chunk, repeats, max_ratio_loss, tie,
                            (ctypes.c_uint8 * 4)(*(list(policy) + [0] * (4 - len(policy)) if policy else [0] * 4)))
    best = zipnn_params()
    ents = (zipnn_tune_entry * 64)()
    cnt = ctypes.c_int(0)
    _check(lib().zipnn_autotune(ctx, dtype, ts, n, ctypes.byref(cfg), ctypes.byref(best), ents, 64, ctypes.byref(cnt)),
           "zipnn_autotune")
    return best, [ents[i] for i in range(cnt.value)]


TUNE_SAMPLE_BYTES = 16 << 30   # a whole 8B checkpoint: steady-state rates need many items per workgroup
TUNE_MIN_CHUNK, TUNE_MAX_CHUNK = 64 << 10, 1 << 20


def tune_checkpoint(codec, xs, bases=None, policy=None):
    """zipnn_autotune over a checkpoint's BF16 tensors with the settings the
    benchmark uses: up to 16 GiB of sample (an 8B checkpoint whole: a smaller
    sample gives each workgroup too few items to show steady-state rates),
    chunks of 64 KiB .. 1 MiB, ratio within 1% of the best.  -> (params, table)"""
    bptr = [b.data_ptr() for b in bases] if bases is not None else [None] * len(xs)
    return zipnn_autotune(codec.ctx, ZIPNN_BF16, [x.data_ptr() for x in xs], [x.numel() for x in xs], bptr,
                          TUNE_SAMPLE_BYTES, 0.01, policy, min_chunk=TUNE_MIN_CHUNK, max_chunk=TUNE_MAX_CHUNK)


def autotune_sample(ns, B: int, sample_bytes: int = 1 << 30, max_chunk: int = 1 << 20) -> list[int]:
    """Elements of each tensor that zipnn_autotune puts in its sample (the
    rule documented with zipnn_autotune), for reporting its composition."""
    ns = [int(n) for n in ns]
    total = sum(n * B for n in ns)
    if total <= sample_bytes:
        return list(ns)
    take = [0] * len(ns)
    sizes = []
    for n in ns:
        if n and n not in sizes:
            sizes.append(n)
    for ln in sizes:
        cls = sum(n for n in ns if n == ln)
        left = -(-cls * B * sample_bytes // total) // B
        for i, n in enumerate(ns):
            if not left:
                break
            if n != ln:
                continue
            k = min(ln, max(left, max_chunk // B))
            take[i] = k
            left -= min(left, k)
    return take


def zipnn_clock() -> float:
    return lib().zipnn_clock()


def zipnn_server_create(ctx, pool_bytes: int, max_inflight: int, chunks_per_iter: int = 0,
                        mode: int = ZIPNN_SERVE_CONTINUOUS) -> int:
    cfg = zipnn_server_config(pool_bytes, max_inflight, chunks_per_iter, mode)
    h = ctypes.c_void_p()
    _check(lib().zipnn_server_create(ctx, ctypes.byref(cfg), ctypes.byref(h)), "zipnn_server_create")
    return h.value


def zipnn_server_destroy(srv) -> None:
    lib().zipnn_server_destroy(srv)


def zipnn_server_register(srv, src, src_len, base=None) -> int:
    h = ctypes.c_uint32(0)
    _check(lib().zipnn_server_register(srv, src, src_len, base, ctypes.byref(h)), "zipnn_server_register")
    return h.value


def zipnn_server_submit(srv, handle: int, t_arrive: float = 0.0) -> int:
    t = ctypes.c_uint64(0)
    _check(lib().zipnn_server_submit(srv, handle, t_arrive, ctypes.byref(t)), "zipnn_server_submit")
    return t.value


def zipnn_server_poll(srv, ticket: int):
    """-> None while pending, else (status, output device pointer, zipnn_timing)."""
    out = ctypes.c_void_p()
    t = zipnn_timing()
    rc = lib().zipnn_server_poll(srv, ticket, ctypes.byref(out), ctypes.byref(t))
    if rc == ZIPNN_E_BUSY:
        return None
    if rc == ZIPNN_E_INVAL:
        raise ZipnnError(rc, "zipnn_server_poll")
    return rc, out.value, t


def zipnn_server_next_done(srv, timeout_s: float):
    """-> ticket of a completed request, or None on time-out."""
    t = ctypes.c_uint64(0)
    rc = lib().zipnn_server_next_done(srv, timeout_s, ctypes.byref(t))
    if rc == ZIPNN_E_BUSY:
        return None
    _check(rc, "zipnn_server_next_done")
    return t.value


def zipnn_server_release(srv, ticket: int) -> None:
    _check(lib().zipnn_server_release(srv, ticket), "zipnn_server_release")


def zipnn_server_set_mode(srv, mode: int) -> None:
    _check(lib().zipnn_server_set_mode(srv, mode), "zipnn_server_set_mode")


def zipnn_server_stats(srv) -> zipnn_server_counters:
    c = zipnn_server_counters()
    _check(lib().zipnn_server_stats(srv, ctypes.byref(c)), "zipnn_server_stats")
    return c


# ---------------------------------------------------------------- tensor helpers

def torch_dtype_code(dt) -> int:
    import torch

    table = {torch.bfloat16: ZIPNN_BF16, torch.float16: ZIPNN_FP16, torch.float32: ZIPNN_FP32,
             torch.float8_e4m3fn: ZIPNN_FP8_E4M3, torch.uint8: ZIPNN_U8, torch.int8: ZIPNN_U8}
    if dt not in table:
        raise ValueError(f"unsupported dtype {dt}")
    return table[dt]


def make_params(dtype: int, chunk_bytes: int | None = None, S: int | None = None, g: int | None = None,
                L: int | None = None, policy=None, probe_skip: int | None = None,
                exponent: bool | None = None) -> zipnn_params:
    p = zipnn_default_params(dtype)
    if chunk_bytes is not None:
        p.chunk_bytes = chunk_bytes
        if S is None:  # keep 256 sub-streams per full chunk
            p.substream_syms = max(1, min(4096, chunk_bytes // WIDTH[dtype] // 256))
    if S is not None:
        p.substream_syms = S
    if g is not None:
        p.group = g
    if L is not None:
        p.max_code_len = L
    if policy is not None:
        for k, v in enumerate(policy):
            p.policy[k] = v
    if probe_skip is not None:
        p.probe_skip = probe_skip
    if exponent is not None:
        p.exponent = int(exponent)
    p.substream_syms = max(p.substream_syms, p.group)
    return p


class Codec:
    """Tensor-level front end of one zipnn context on a HIP device."""

    def __init__(self, device: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the zipnn codec runs only on the GPU")
        self.device = device
        self.ctx = zipnn_ctx_create(device)

    def close(self):
        if self.ctx:
            zipnn_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stream():
        import torch

        return torch.cuda.current_stream().cuda_stream

    def compress(self, x, params: zipnn_params | None = None, base=None, out=None):
        """Compress device tensor x -> uint8 device tensor holding the container."""
        import torch

        dt = torch_dtype_code(x.dtype)
        x = x.contiguous()
        if base is not None:
            base = base.contiguous()
            assert base.dtype == x.dtype and base.numel() == x.numel() and base.device == x.device
        p = params or zipnn_default_params(dt)
        n = x.numel()
        cap = zipnn_compress_bound(dt, n, p)
        if cap == 0:
            raise ZipnnError(ZIPNN_E_INVAL, "params")
        if out is None or out.numel() < cap:
            out = torch.empty(cap, dtype=torch.uint8, device=x.device)
        ln = zipnn_compress(self.ctx, x.data_ptr(), dt, n, base.data_ptr() if base is not None else None, p,
                            out.data_ptr(), out.numel(), self._stream())
        return out[:ln]

    def decompress(self, c, out, base=None, check: bool = True, header: bytes | None = None):
        """Decompress container c (uint8 device tensor) into `out` (any dtype,
        n*B bytes).  `header`: host copy of the container's first 64 bytes, to
        queue the decode without a host round trip.  With check=True,
        synchronises and raises on a device-side error."""
        args = (c.data_ptr(), c.numel(), base.data_ptr() if base is not None else None, out.data_ptr(),
                out.numel() * out.element_size(), self._stream())
        if header is None:
            zipnn_decompress(self.ctx, *args)
        else:
            zipnn_decompress_async(self.ctx, header, *args)
        if check:
            st = zipnn_ctx_status(self.ctx, self._stream(), clear=True)
            if st != ZIPNN_OK:
                raise ZipnnError(st, "zipnn_decompress (device)")
        return out

    def compress_batch(self, xs, params: zipnn_params | None = None, bases=None, arena=None):
        """Compress device tensors xs (one dtype) into one arena.
        Returns (arena uint8 tensor, offsets list of n+1)."""
        import torch

        dt = torch_dtype_code(xs[0].dtype)
        p = params or zipnn_default_params(dt)
        xs = [x.contiguous() for x in xs]
        bases = [None] * len(xs) if bases is None else [b.contiguous() if b is not None else None for b in bases]
        cap = sum(zipnn_compress_bound(dt, x.numel(), p) + 127 for x in xs)   # containers start 128-aligned
        if arena is None or arena.numel() < cap:
            arena = torch.empty(cap, dtype=torch.uint8, device=xs[0].device)
        offs = zipnn_compress_batch(self.ctx, dt, [x.data_ptr() for x in xs], [x.numel() for x in xs],
                                    [b.data_ptr() if b is not None else None for b in bases], p, arena.data_ptr(),
                                    arena.numel(), self._stream())
        return arena, offs

    def prepare_batch(self, arena, offsets, outs, bases=None) -> "Batch":
        return Batch(self, arena, offsets, outs, bases)

    def prepare_encoder(self, xs, params: zipnn_params | None = None, bases=None, arena=None) -> "Encoder":
        return Encoder(self, xs, params, bases, arena)

    def status(self, clear: bool = True) -> int:
        return zipnn_ctx_status(self.ctx, self._stream(), clear)


class Encoder:
    """A prepared batched compression (descriptors on the device and a
    captured hipGraph); run() replays it on the current stream and returns
    the arena offsets (n+1)."""

    def __init__(self, codec: Codec, xs, params=None, bases=None, arena=None):
        import torch

        self.codec = codec
        dt = torch_dtype_code(xs[0].dtype)
        p = params or zipnn_default_params(dt)
        xs = [x.contiguous() for x in xs]
        bases = [None] * len(xs) if bases is None else [b.contiguous() if b is not None else None for b in bases]
        cap = sum(zipnn_compress_bound(dt, x.numel(), p) + 127 for x in xs)
        if arena is None or arena.numel() < cap:
            arena = torch.empty(cap, dtype=torch.uint8, device=xs[0].device)
        self.arena = arena
        self._keep = (xs, bases)
        n = len(xs)
        ts = (zipnn_tensor_in * n)(*[zipnn_tensor_in(x.data_ptr(), x.numel(), b.data_ptr() if b is not None else None)
                                     for x, b in zip(xs, bases)])
        h = ctypes.c_void_p()
        _check(lib().zipnn_encoder_create(codec.ctx, dt, ts, n, ctypes.byref(p), arena.data_ptr(), arena.numel(),
                                          ctypes.byref(h)), "zipnn_encoder_create")
        self.h = h.value
        self.n = n

    def run(self) -> list[int]:
        offs = (ctypes.c_uint64 * (self.n + 1))()
        _check(lib().zipnn_encoder_run(self.h, Codec._stream(), offs), "zipnn_encoder_run")
        return list(offs)

    def close(self):
        if self.h:
            lib().zipnn_encoder_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A prepared batched decompression (descriptor tables on the device and a
    captured hipGraph); run() replays it on the current stream."""

    def __init__(self, codec: Codec, arena, offsets, outs, bases=None):
        self.codec = codec
        self._keep = (arena, list(outs), bases)
        self.h = zipnn_batch_create(codec.ctx, arena.data_ptr(), offsets, [o.data_ptr() for o in outs],
                                    [o.numel() * o.element_size() for o in outs],
                                    None if bases is None else [b.data_ptr() if b is not None else None
                                                                for b in bases])

    def run(self, check: bool = False):
        zipnn_batch_decompress(self.h, Codec._stream())
        if check:
            st = self.codec.status(clear=True)
            if st != ZIPNN_OK:
                raise ZipnnError(st, "batch decompress (device)")

    def close(self):
        if self.h:
            zipnn_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceBytes:
    """A device byte range exposed through __cuda_array_interface__ so that
    torch can view it without a copy."""

    def __init__(self, ptr: int, nbytes: int):
        self.__cuda_array_interface__ = {"shape": (nbytes,), "typestr": "|u1", "data": (ptr, False), "version": 3,
                                         "strides": None}


class Server:
    """Front end of a zipnn decompression server (continuous batching over
    containers resident in device memory)."""

    def __init__(self, codec: Codec, pool_bytes: int, max_inflight: int = 256, chunks_per_iter: int = 0,
                 mode: int = ZIPNN_SERVE_CONTINUOUS):
        self.codec = codec
        self.h = zipnn_server_create(codec.ctx, pool_bytes, max_inflight, chunks_per_iter, mode)
        self._keep = []
        self._nbytes = {}

    def register(self, container, base=None) -> int:
        """container: uint8 device tensor holding one container (kept alive
        by the server object)."""
        self._keep.append((container, base))
        hd = zipnn_server_register(self.h, container.data_ptr(), container.numel(),
                                   base.data_ptr() if base is not None else None)
        import struct

        hdr = container[:64].cpu().numpy().tobytes()
        B, n = hdr[7], struct.unpack_from("<Q", hdr, 8)[0]   # header: u8 B at 7, u64 n_elems at 8
        self._nbytes[hd] = n * B
        return hd

    def submit(self, handle: int, t_arrive: float = 0.0) -> int:
        return zipnn_server_submit(self.h, handle, t_arrive)

    def poll(self, ticket: int):
        return zipnn_server_poll(self.h, ticket)

    def next_done(self, timeout_s: float = 1.0):
        return zipnn_server_next_done(self.h, timeout_s)

    def output(self, ticket: int, handle: int, dtype=None):
        """View of a completed request's output (valid until release)."""
        import torch

        r = self.poll(ticket)
        if r is None:
            raise ZipnnError(ZIPNN_E_BUSY, "Server.output")
        st, ptr, _ = r
        if st != ZIPNN_OK:
            raise ZipnnError(st, "Server.output")
        n = self._nbytes[handle]
        if n == 0:
            v = torch.empty(0, dtype=torch.uint8, device=f"cuda:{self.codec.device}")
        else:
            v = torch.as_tensor(_DeviceBytes(ptr, n), device=f"cuda:{self.codec.device}")
        return v if dtype is None else v.view(dtype)

    def release(self, ticket: int) -> None:
        zipnn_server_release(self.h, ticket)

    def stats(self) -> zipnn_server_counters:
        return zipnn_server_stats(self.h)

    def set_mode(self, mode: int) -> None:
        zipnn_server_set_mode(self.h, mode)

    def close(self):
        if self.h:
            zipnn_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
