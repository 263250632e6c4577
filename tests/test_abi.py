"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/*.h, and its host-only entry points (parameters, bounds,
container inspection) agree with the oracle's containers."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import oracle
from paper_2411_05239_amd import workloads
from paper_2411_05239_amd import zipnn as Z

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(zipnn_[a-z_0-9]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def hiplib():
    if not os.path.exists(Z.LIB_PATH):
        from paper_2411_05239_amd import build

        build.build()
    return Z.lib()


def test_every_declared_symbol_is_exported(hiplib):
    declared = _declared_functions()
    assert len(declared) >= 10
    assert sorted(Z.EXPORTS) == declared
    for name in declared:
        assert hasattr(hiplib, name), name


def test_default_params(hiplib):
    for dt, S in [(Z.ZIPNN_BF16, 512), (Z.ZIPNN_FP32, 256), (Z.ZIPNN_FP8_E4M3, 1024), (Z.ZIPNN_FP16, 512)]:
        p = Z.zipnn_default_params(dt)
        assert (p.chunk_bytes, p.substream_syms, p.group, p.max_code_len) == (262144, S, 4, 11)
        assert list(p.policy) == [0, 0, 0, 0]
        assert Z.zipnn_check_params(dt, p) == Z.ZIPNN_OK


def test_check_params_rejects(hiplib):
    for kw in [dict(chunk_bytes=1000), dict(chunk_bytes=128), dict(S=3), dict(g=3), dict(g=16), dict(g=1), dict(L=7),
               dict(L=12), dict(S=8192), dict(chunk_bytes=1 << 20, S=64)]:
        p = Z.make_params(Z.ZIPNN_BF16, **kw)
        assert Z.zipnn_check_params(Z.ZIPNN_BF16, p) == Z.ZIPNN_E_INVAL, kw
    assert Z.zipnn_check_params(99, Z.zipnn_default_params(Z.ZIPNN_BF16)) == Z.ZIPNN_E_INVAL


def test_compress_bound_covers_oracle(hiplib, oracle_lib):
    rng = np.random.default_rng(0)
    for dt in (Z.ZIPNN_BF16, Z.ZIPNN_FP32, Z.ZIPNN_FP8_E4M3):
        B = Z.WIDTH[dt]
        for n in (0, 1, 1000, 70_001):
            u = rng.integers(0, 256, size=n * B, dtype=np.uint8)
            for pol in (0, 1):
                p = Z.make_params(dt, chunk_bytes=4096, policy=[pol] * B)
                c = oracle.compress(u, dt, chunk_bytes=4096, S=p.substream_syms, g=p.group, policy=[pol] * B)
                assert c.size <= Z.zipnn_compress_bound(dt, n, p)


def test_inspect_agrees_with_oracle(hiplib, oracle_lib):
    x = workloads.fp32_rows(16, 8192, seed=2)
    p = Z.zipnn_default_params(Z.ZIPNN_FP32)
    c = oracle.compress(x, oracle.FP32, S=p.substream_syms)
    info = Z.zipnn_inspect(c.tobytes())
    h = oracle.header(c)
    assert (info.dtype, info.B, info.n_elems, info.total_bytes, info.n_chunks) == (
        oracle.FP32, 4, x.numel(), c.size, h["n_chunks"])
    assert info.S == p.substream_syms and info.g == 4 and info.L == 11 and info.is_delta == 0
    modes = [oracle.entry(c, ch, k)[2] for ch in range(h["n_chunks"]) for k in range(4)]
    assert [info.entries_by_mode[i] for i in range(3)] == [modes.count(i) for i in range(3)]
    # header + map alone are enough
    Z.zipnn_inspect(c[: 64 + 16 * h["n_chunks"] * 4].tobytes())


def test_inspect_rejects_corrupt_maps(hiplib, oracle_lib):
    x = workloads.bf16_normal(5 * 8192 + 3, seed=1)
    c = oracle.compress(x, oracle.BF16, chunk_bytes=16384, S=32)
    Z.zipnn_inspect(c.tobytes())
    # (a size changed by less than the payload alignment keeps the placement
    # valid: only reading the payload can tell, so the size byte flipped here
    # is the second one)
    for pos in [0, 6, 16, 20, 23, 28, 32, 45, 64, 73, 76, 78, 64 + 16 * 3]:
        d = c.copy()
        d[pos] ^= 0x10 if pos not in (6,) else 0x04
        with pytest.raises(Z.ZipnnError) as ei:
            Z.zipnn_inspect(d.tobytes())
        assert ei.value.code in (Z.ZIPNN_E_FORMAT, Z.ZIPNN_E_CORRUPT)
    with pytest.raises(Z.ZipnnError):
        Z.zipnn_inspect(c[:63].tobytes())


def test_strerror(hiplib):
    assert Z.zipnn_strerror(0) == "ok"
    assert "corrupt" in Z.zipnn_strerror(Z.ZIPNN_E_CORRUPT)


def test_autotune_sample_holds_every_tensor():
    """The documented sample rule: every size class in proportion to its
    bytes, whole tensors in order, the last one cut (at least one largest
    chunk); the whole set when it fits."""
    ns = [1 << 26, 4096, 1 << 22, 1 << 22, 1 << 22, 4096, 1 << 26, 12]
    B, sample = 2, 64 << 20
    got = Z.autotune_sample(ns, B, sample_bytes=sample, max_chunk=1 << 20)
    total = B * sum(ns)
    assert all(0 <= g <= n for g, n in zip(got, ns))
    for ln in set(ns):
        share = -(-sum(n for n in ns if n == ln) * B * sample // total) // B
        took = [g for g, n in zip(got, ns) if n == ln]
        assert took[0] > 0                                   # every class is in the sample
        assert sum(took) == min(sum(n for n in ns if n == ln), max(share, min(ln, (1 << 20) // B)))
        nz = [t for t in took if t]
        assert all(t == ln for t in nz[:-1]) and took[:len(nz)] == nz   # whole tensors in order, the last cut
    assert got[1] == 4096 and got[7] == 12                  # small classes whole
    assert Z.autotune_sample(ns[1:2], B, sample_bytes=1 << 30) == [4096]
