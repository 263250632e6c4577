"""The allocation-free compress entry point (zipnn_compress_noalloc), called
through the C ABI: its containers must equal zipnn_compress's byte for byte
(and so the oracle's), on two calls in a row, the second with a smaller
input, so that the fixed scratch's leftovers from the first call cannot leak
into the second.  Inputs beyond the fixed scratch are refused before any
work is queued."""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_05239_amd import workloads
from paper_2411_05239_amd import zipnn as Z

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def codec():
    c = Z.Codec(0)
    yield c
    c.close()


def _noalloc(codec, x, p, base=None):
    dt = Z.torch_dtype_code(x.dtype)
    cap = Z.zipnn_compress_bound(dt, x.numel(), p)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    n = Z.zipnn_compress_noalloc(codec.ctx, x.data_ptr(), dt, x.numel(), base.data_ptr() if base is not None else None,
                                 p, out.data_ptr(), cap, codec._stream())
    return out[:n].cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32])
def test_noalloc_equals_compress_twice_shrinking(codec, dtype):
    B = torch.empty(0, dtype=dtype).element_size()
    p = Z.zipnn_default_params(Z.torch_dtype_code(dtype))
    E = p.chunk_bytes // B
    big = (workloads.bf16_normal(9 * E + 333, seed=61) if B == 2 else
           workloads.fp32_rows(9 * E // 8192 + 1, 8192, seed=62).reshape(-1)[:9 * E + 333].contiguous()).cuda()
    small = big[: 2 * E + 17].clone()
    for x in (big, small):
        print("noalloc case", dtype, x.numel(), flush=True)
        got = _noalloc(codec, x, p)
        want = codec.compress(x, p).cpu().numpy()
        assert np.array_equal(got, want)
        out = torch.empty_like(x)
        codec.decompress(torch.from_numpy(got).cuda(), out)
        assert torch.equal(out.view(torch.uint8), x.view(torch.uint8))
    ref = oracle.compress(small.cpu(), Z.torch_dtype_code(dtype), nthreads=8, chunk_bytes=p.chunk_bytes,
                          S=p.substream_syms, g=p.group, L=p.max_code_len, policy=list(p.policy))
    assert np.array_equal(_noalloc(codec, small, p), ref)


def test_noalloc_delta_and_zg_twice(codec):
    """A BF16 XOR delta under AUTO (ZG entries) and then a smaller one."""
    p = Z.zipnn_default_params(Z.ZIPNN_BF16)
    base = workloads.bf16_normal(5 * 131072 + 99, seed=63).cuda()
    ft = workloads.finetune_delta(base, seed=64)
    for n in (base.numel(), 131072 + 5):
        b, f = base[:n].clone(), ft[:n].clone()
        print("noalloc delta", n, flush=True)
        got = _noalloc(codec, f, p, base=b)
        want = codec.compress(f, p, base=b).cpu().numpy()
        assert np.array_equal(got, want)


def test_noalloc_refuses_beyond_fixed_scratch(codec):
    """At 256 KiB chunks each chunk-stream needs about 1.3 KiB of scratch:
    a BF16 tensor of 8 GiB would need ~85 MiB.  Refused with E_TOOBIG before
    anything runs (the source pointer is never read)."""
    p = Z.zipnn_default_params(Z.ZIPNN_BF16)
    x = torch.empty(16, dtype=torch.bfloat16, device="cuda")
    n = 4 << 30
    with pytest.raises(Z.ZipnnError) as ei:
        Z.zipnn_compress_noalloc(codec.ctx, x.data_ptr(), Z.ZIPNN_BF16, n, None, p, x.data_ptr(), 1 << 62,
                                 codec._stream())
    assert ei.value.code == Z.ZIPNN_E_TOOBIG


def test_noalloc_empty_tensor(codec):
    p = Z.zipnn_default_params(Z.ZIPNN_BF16)
    x = torch.empty(0, dtype=torch.bfloat16, device="cuda")
    got = _noalloc(codec, x, p)
    assert np.array_equal(got, codec.compress(x, p).cpu().numpy())
