"""ZipNN oracle -- TEST INFRASTRUCTURE ONLY.

Two independent CPU implementations of the codec described in ``zipnn_oracle.h``:

* ``zipnn_oracle.c`` (loaded here through ctypes): plain C, bit-by-bit, used for
  the parity tests at real sizes and for the benchmark's ``cpu_baseline`` leg;
* ``spec.py``: pure Python for tiny inputs, written separately, which must
  produce the same container bytes.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may import this package.  The product path (``paper_2411_05239_amd``) never does.

Method sources (ZipNN, arXiv 2411.05239): byte grouping with the exponent byte
first (§III-A, §III-B), Huffman-only coding (§III-A), single-valued streams
reduced to a header and incompressible streams stored (§III-B), 256 KB chunks
with per-byte-group decisions and a map for parallel decode (§V-A), XOR deltas
(§IV-B).  Code construction: package-merge (Larmore & Hirschberg 1990) and
canonical codes (RFC 1951 §3.2.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zipnn_oracle.c")
LIB_PATH = os.path.join(_HERE, "libzipnn_oracle.so")

OK, E_INVAL, E_FORMAT, E_CORRUPT, E_NOSPACE, E_NOMEM = 0, -1, -2, -3, -4, -5
BF16, FP16, FP32, FP8_E4M3, U8 = 1, 2, 3, 4, 5
WIDTH = {BF16: 2, FP16: 2, FP32: 4, FP8_E4M3: 1, U8: 1}
PAY_ALIGN = 128   # payload alignment from the container start (ORC_PAY_ALIGN)


def payload_base(n_chunks: int, B: int) -> int:
    """Offset of a container's payload area: header + map, aligned."""
    return -(-(64 + 16 * n_chunks * B) // PAY_ALIGN) * PAY_ALIGN if n_chunks else 64
AUTO, HUF, RAW, ZG = 0, 1, 2, 3
MODE_RAW, MODE_HUF, MODE_RLE, MODE_ZG = 0, 1, 2, 3


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"oracle error {code} {what}".strip())
        self.code = code


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no intrinsics)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "zipnn_oracle.h"))
    ):
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp]
        )
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u8p, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.orc_compress.argtypes = [u8p, i32, u64, u8p, u32, u32, u32, u32, u8p, u32, i32, u8p, u64,
                                   ctypes.POINTER(u64), i32]
        L.orc_compress.restype = i32
        L.orc_decompress.argtypes = [u8p, u64, u8p, u8p, u64, i32]
        L.orc_decompress.restype = i32
        L.orc_compress_bound.argtypes = [i32, u64, u32, u32]
        L.orc_compress_bound.restype = u64
        L.orc_package_merge.argtypes = [u8p, i32, u8p]
        L.orc_package_merge.restype = i32
        L.orc_canonical_codes.argtypes = [u8p, i32, u8p]
        L.orc_canonical_codes.restype = None
        L.orc_substream_bits.argtypes = [u8p, u64, u32, u32, i32, u8p, u8p, u64, u8p, u64, ctypes.POINTER(u64)]
        L.orc_substream_bits.restype = i32
        L.orc_entry.argtypes = [u8p, u64, u32, i32, ctypes.POINTER(u64), ctypes.POINTER(u64),
                                ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.orc_entry.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags.c_contiguous
    return a.ctypes.data


def as_bytes(x) -> np.ndarray:
    """View any contiguous numpy array (or torch CPU tensor) as uint8."""
    if hasattr(x, "numpy"):  # torch tensor
        import torch

        x = x.contiguous().view(torch.uint8).numpy()
    return np.ascontiguousarray(x).reshape(-1).view(np.uint8)


def compress(x, dtype: int, *, base=None, chunk_bytes: int = 262144, S: int = 512, g: int = 4, L: int = 11,
             policy=(AUTO, AUTO, AUTO, AUTO), skip: int = 0, exp: bool = False, nthreads: int = 1) -> np.ndarray:
    xb = as_bytes(x)
    B = WIDTH[dtype]
    assert xb.size % B == 0
    n = xb.size // B
    bb = None
    if base is not None:
        bb = as_bytes(base)
        assert bb.size == xb.size
    cap = lib().orc_compress_bound(dtype, n, chunk_bytes, S)
    out = np.zeros(max(cap, 64), dtype=np.uint8)
    pol = np.array(list(policy) + [0] * (4 - len(policy)), dtype=np.uint8)
    dlen = ctypes.c_uint64(0)
    rc = lib().orc_compress(_ptr(xb), dtype, n, _ptr(bb), chunk_bytes, S, g, L, _ptr(pol), skip, int(exp), _ptr(out), out.size,
                            ctypes.byref(dlen), nthreads)
    if rc != OK:
        raise OracleError(rc, "compress")
    return out[: dlen.value].copy()


def header(c: np.ndarray) -> dict:
    c = as_bytes(c)
    h = c[:64].tobytes()
    return dict(
        magic=h[:4], version=int.from_bytes(h[4:6], "little"), dtype=h[6], B=h[7],
        n=int.from_bytes(h[8:16], "little"), chunk_bytes=int.from_bytes(h[16:20], "little"),
        S=int.from_bytes(h[20:22], "little"), g=h[22], L=h[23], flags=int.from_bytes(h[24:28], "little"),
        n_chunks=int.from_bytes(h[28:32], "little"), total=int.from_bytes(h[32:40], "little"),
        policy=tuple(h[40:44]), skip=h[44],
    )


def decompress(c, base=None, nthreads: int = 1, out_bytes: int | None = None) -> np.ndarray:
    cb = as_bytes(c)
    if out_bytes is None:
        h = header(cb) if cb.size >= 64 else dict(n=0, B=1)
        out_bytes = h["n"] * h["B"] if cb.size >= 64 and h["B"] in (1, 2, 4) else 0
    out = np.zeros(max(out_bytes, 1), dtype=np.uint8)
    bb = None if base is None else as_bytes(base)
    rc = lib().orc_decompress(_ptr(cb), cb.size, _ptr(bb), _ptr(out), out_bytes, nthreads)
    if rc != OK:
        raise OracleError(rc, "decompress")
    return out[:out_bytes]


def package_merge(freq, L: int) -> np.ndarray:
    f = np.zeros(256, dtype=np.uint64)
    f[: len(freq)] = np.asarray(freq, dtype=np.uint64)
    out = np.zeros(256, dtype=np.uint8)
    rc = lib().orc_package_merge(_ptr(f), L, _ptr(out))
    if rc < 0:
        raise OracleError(rc, "package_merge")
    return out


def canonical_codes(lengths, L: int) -> np.ndarray:
    ln = np.zeros(256, dtype=np.uint8)
    ln[: len(lengths)] = np.asarray(lengths, dtype=np.uint8)
    out = np.zeros(256, dtype=np.uint32)
    lib().orc_canonical_codes(_ptr(ln), L, _ptr(out))
    return out


def substream_bits(sym: np.ndarray, S: int, g: int, L: int, lengths, w: int, flags=None) -> tuple[bytes, int]:
    """Bit string of sub-stream w (the coding without the word layout): the
    packed bytes (LSB-first) and the bit count."""
    s = np.ascontiguousarray(sym, dtype=np.uint8)
    m = s.size
    ln = np.zeros(256, dtype=np.uint8)
    ln[: len(lengths)] = np.asarray(lengths, dtype=np.uint8)
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    W, G = -(-m // S), -(-m // g)
    cap = (-(-G // max(W, 1)) * g * L + 7) // 8 + 8   # the longest sub-stream at L bits a symbol
    out = np.zeros(cap, dtype=np.uint8)
    nb = ctypes.c_uint64(0)
    rc = lib().orc_substream_bits(_ptr(s), m, S, g, L, _ptr(ln), _ptr(fl), w, _ptr(out), out.size, ctypes.byref(nb))
    if rc != OK:
        raise OracleError(rc, "substream_bits")
    return out[: (nb.value + 7) // 8].tobytes(), nb.value


def entry(c: np.ndarray, chunk: int, k: int) -> tuple[int, int, int, int]:
    """(absolute payload offset, payload bytes, mode, rle value) of one map entry."""
    cb = as_bytes(c)
    off, nb = ctypes.c_uint64(0), ctypes.c_uint64(0)
    mode, rle = ctypes.c_int(0), ctypes.c_int(0)
    rc = lib().orc_entry(_ptr(cb), cb.size, chunk, k, ctypes.byref(off), ctypes.byref(nb), ctypes.byref(mode),
                         ctypes.byref(rle))
    if rc != OK:
        raise OracleError(rc, "entry")
    return off.value, nb.value, mode.value, rle.value
