"""GPU parity: the HIP path against the CPU oracle, byte for byte.

Every case checks, on the same seeded input bytes:
  * the GPU container equals the oracle's container (bitstream equality);
  * the GPU decode of that container restores the input bit for bit;
  * the oracle decodes the GPU container to the input.
Tolerance: exactly zero differing bytes everywhere (integer work).
"""
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


def _oracle_kw(p):
    return dict(chunk_bytes=p.chunk_bytes, S=p.substream_syms, g=p.group, L=p.max_code_len, policy=list(p.policy),
                skip=p.probe_skip, exp=bool(p.exponent))


def _u8(t):
    return t.contiguous().view(torch.uint8).reshape(-1)


def roundtrip(codec, x_cpu, p, base_cpu=None, nthreads=8):
    dt = Z.torch_dtype_code(x_cpu.dtype)
    print(f"case dtype={x_cpu.dtype} n={x_cpu.numel()} {p} delta={base_cpu is not None}", flush=True)
    x = x_cpu.cuda()
    base = base_cpu.cuda() if base_cpu is not None else None
    c_gpu = codec.compress(x, p, base=base)
    c_orc = oracle.compress(x_cpu, dt, base=base_cpu, nthreads=nthreads, **_oracle_kw(p))
    got = c_gpu.cpu().numpy()
    assert got.size == c_orc.size, (got.size, c_orc.size)
    if not np.array_equal(got, c_orc):
        bad = np.nonzero(got != c_orc)[0]
        raise AssertionError(f"{bad.size} container bytes differ, first at {bad[:8]}")
    out = torch.empty_like(x)
    codec.decompress(c_gpu, out, base=base)
    assert torch.equal(_u8(out), _u8(x))
    back = oracle.decompress(got, base=base_cpu, nthreads=nthreads)
    assert np.array_equal(back, oracle.as_bytes(x_cpu))
    return c_gpu


def test_bf16_8mb_huf_raw(codec):
    """Single BF16 tensor, 4,194,304 elements ~ N(0, 0.02); s0 HUF, s1 RAW."""
    x = workloads.bf16_normal(4_194_304, seed=0)
    p = Z.make_params(Z.ZIPNN_BF16, policy=[Z.ZIPNN_HUF, Z.ZIPNN_RAW])
    c = roundtrip(codec, x, p)
    assert 0.66 < c.numel() / (2 * x.numel()) < 0.68


def test_fp32_rows_reduced(codec):
    x = workloads.fp32_rows(64, 8192, seed=1)
    roundtrip(codec, x, Z.zipnn_default_params(Z.ZIPNN_FP32))


@pytest.mark.slow
def test_fp32_8192x8192_full(codec):
    """The full FP32 workload: 8192 x 8192, row sigma log-uniform in [1e-3, 1e-1]."""
    x = workloads.fp32_rows(8192, 8192, seed=1)
    c = roundtrip(codec, x, Z.zipnn_default_params(Z.ZIPNN_FP32), nthreads=16)
    assert 0.84 < c.numel() / (4 * x.numel()) < 0.87


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 63, 64, 65, 1000, 3 * 131072 + 37])
def test_ragged_sizes_bf16(codec, n):
    x = workloads.bf16_normal(max(n, 1), seed=n)[:n].contiguous()
    roundtrip(codec, x, Z.zipnn_default_params(Z.ZIPNN_BF16))
    roundtrip(codec, x, Z.make_params(Z.ZIPNN_BF16, chunk_bytes=1024, S=8, g=2, policy=[1, 1]))


@pytest.mark.parametrize("g", [2, 4, 8])
@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32, torch.uint8])
def test_groups_and_dtypes(codec, g, dtype):
    n = 50_000 + 7
    if dtype == torch.uint8:
        x = workloads.make_corpus_tensor(workloads.CorpusItem(0, "fp8", n, 77)).view(torch.uint8)
    elif dtype == torch.float32:
        x = workloads.fp32_rows(1, n, seed=3).reshape(-1)
    else:
        x = workloads.bf16_normal(n, seed=4)
    dt = Z.torch_dtype_code(dtype)
    B = Z.WIDTH[dt]
    roundtrip(codec, x, Z.make_params(dt, chunk_bytes=16384, S=max(g, 16), g=g, policy=[1] * B))
    roundtrip(codec, x, Z.make_params(dt, chunk_bytes=65536, g=g))


def test_many_substreams_per_chunk(codec):
    """W > 256: a chunk is decoded by several workgroup slices."""
    x = workloads.bf16_normal(3 * 524288 + 11, seed=5)
    roundtrip(codec, x, Z.make_params(Z.ZIPNN_BF16, chunk_bytes=1 << 20, S=256))
    roundtrip(codec, x, Z.make_params(Z.ZIPNN_BF16, chunk_bytes=1 << 20, S=128, g=8))


def test_fp8_corpus_tensor(codec):
    x = workloads.make_corpus_tensor(workloads.CorpusItem(0, "fp8", 300_000, 9))
    roundtrip(codec, x, Z.zipnn_default_params(Z.ZIPNN_FP8_E4M3))


def test_fp16_and_special_patterns(codec):
    x = workloads.fp32_rows(4, 4096, seed=6).reshape(-1).clone()
    pats = torch.tensor([0x7F800000, 0xFF800000, 0x7FC00001, 0xFFFFFFFF, 0x80000000, 1, 0x007FFFFF, 0],
                        dtype=torch.int64).to(torch.int32)
    x.view(torch.int32)[:8] = pats
    roundtrip(codec, x, Z.make_params(Z.ZIPNN_FP32, policy=[1, 1, 1, 1]))
    h = (torch.randn(70_000, generator=torch.Generator().manual_seed(1)) * 0.1).to(torch.float16)
    roundtrip(codec, h, Z.zipnn_default_params(Z.ZIPNN_FP16))


def test_raw_rle_and_forced_huffman(codec):
    g = torch.Generator().manual_seed(2)
    u = torch.randint(0, 256, (600_000,), generator=g, dtype=torch.uint8)
    roundtrip(codec, u, Z.zipnn_default_params(Z.ZIPNN_U8))           # AUTO -> RAW
    roundtrip(codec, u, Z.make_params(Z.ZIPNN_U8, policy=[1]))        # forced HUF on random bytes
    z = torch.full((300_001,), 0x3C, dtype=torch.uint8)
    c = roundtrip(codec, z, Z.make_params(Z.ZIPNN_U8, policy=[1]))    # single value -> RLE
    assert c.numel() == oracle.payload_base(2, 1)                     # header + map, no payload
    roundtrip(codec, z, Z.make_params(Z.ZIPNN_U8, policy=[2]))           # forced RAW


def test_code_length_limits(codec):
    """L = 8 with 256 equiprobable symbols, and a skewed source where the
    L = 11 limit binds."""
    g = torch.Generator().manual_seed(3)
    u = torch.randint(0, 256, (200_000,), generator=g, dtype=torch.uint8)
    roundtrip(codec, u, Z.make_params(Z.ZIPNN_U8, L=8, policy=[1]))
    geo = torch.clamp((-torch.log(torch.rand(400_000, generator=g)) * 3).long(), max=255).to(torch.uint8)
    for L in (8, 9, 10, 11):
        roundtrip(codec, geo, Z.make_params(Z.ZIPNN_U8, L=L, policy=[1]))


@pytest.mark.parametrize("dtype,g", [(torch.uint8, 2), (torch.uint8, 4), (torch.uint8, 8), (torch.bfloat16, 8),
                                     (torch.float32, 4)])
def test_longest_codes_at_the_length_limit(codec, dtype, g, base=False):
    """A few sub-streams hold only rare bytes among zeros: with Huffman forced
    their codes all reach the L = 11 limit, so those lanes add the most bits a
    pair can (2L) at every pair and take the most words the layout allows.
    With `base` the same bytes are the XOR delta against a random base (the
    staged path, whose slots are sized for such lanes)."""
    gen = torch.Generator().manual_seed(40 + g)
    bsz = torch.tensor([], dtype=dtype).element_size()
    chunk, S = 65536, 512
    E = chunk // bsz
    W = (E + S - 1) // S
    n = 4 * E - 1000                      # four chunks, the last one partial
    x = torch.zeros(n * bsz, dtype=torch.uint8)
    e = torch.arange(n)
    lane = (e // g) % W
    hot = (lane == 5) | (lane == W // 2 + 3) | (lane == W - 1)
    idx = e[hot]
    for b in range(bsz):
        x[idx * bsz + b] = torch.randint(1, 256, (idx.numel(),), generator=gen, dtype=torch.uint8)
    b = torch.randint(0, 256, (n * bsz,), generator=gen, dtype=torch.uint8) if base else None
    xt = (x ^ b).view(dtype) if base else x.view(dtype)
    p = Z.make_params(Z.torch_dtype_code(dtype), chunk_bytes=chunk, S=S, g=g, policy=[Z.ZIPNN_HUF] * bsz)
    c = roundtrip(codec, xt, p, base_cpu=b.view(dtype) if base else None).cpu().numpy()
    # every entry is Huffman-coded and the rare bytes' codes are at the limit
    for ch in range(4):
        for k in range(bsz):
            off, nbytes, mode, _ = oracle.entry(c, ch, k)
            assert mode == oracle.MODE_HUF
            nib = c[off: off + 128]
            lens = np.stack([nib & 15, nib >> 4], axis=1).reshape(-1)
            assert lens.max() == 11, (ch, k, lens.max())


def test_xor_delta(codec):
    w = workloads.bf16_normal(1_000_003, seed=10)
    ft = workloads.finetune_delta(w, seed=11)
    p = Z.make_params(Z.ZIPNN_BF16, policy=[1, 1])
    c = roundtrip(codec, ft, p, base_cpu=w)
    assert c.numel() < 0.2 * 2 * w.numel()
    # identical tensors: every stream is RLE 0
    c0 = roundtrip(codec, w, p, base_cpu=w)
    assert c0.numel() == oracle.payload_base((w.numel() + 131071) // 131072, 2)


def test_encode_is_deterministic(codec):
    x = workloads.fp32_rows(32, 8192, seed=12).cuda()
    p = Z.zipnn_default_params(Z.ZIPNN_FP32)
    a = codec.compress(x, p).clone()
    b = codec.compress(x, p).clone()
    assert torch.equal(a, b)


def test_decode_never_writes_outside_dst(codec):
    x = workloads.bf16_normal(100_001, seed=13).cuda()
    c = codec.compress(x, Z.zipnn_default_params(Z.ZIPNN_BF16))
    buf = torch.full((x.numel() * 2 + 4096,), 0xAB, dtype=torch.uint8, device="cuda")
    Z.zipnn_decompress(codec.ctx, c.data_ptr(), c.numel(), None, buf.data_ptr(), x.numel() * 2, codec._stream())
    assert codec.status() == Z.ZIPNN_OK
    assert torch.equal(buf[: x.numel() * 2], _u8(x))
    assert bool((buf[x.numel() * 2:] == 0xAB).all())


def _oracle_container(n=3 * 131072 + 99, seed=14):
    x = workloads.bf16_normal(n, seed=seed)
    p = Z.zipnn_default_params(Z.ZIPNN_BF16)
    return x, oracle.compress(x, oracle.BF16, **_oracle_kw(p))


def _decode_status(codec, c_np, n_bytes, base=None, header=None):
    """Status of one decode: the synchronous return if the call itself
    rejects the container, else the device-side sticky status."""
    c = torch.from_numpy(c_np).cuda()
    out = torch.zeros(n_bytes + 256, dtype=torch.uint8, device="cuda")
    args = (c.data_ptr(), c.numel(), None if base is None else base.data_ptr(), out.data_ptr(), n_bytes,
            codec._stream())
    try:
        if header is None:
            Z.zipnn_decompress(codec.ctx, *args)
        else:
            Z.zipnn_decompress_async(codec.ctx, header, *args)
        st = codec.status(clear=True)
    except Z.ZipnnError as e:
        st = e.code
    torch.cuda.synchronize()
    assert bool((out[n_bytes:] == 0).all())
    return st


def test_device_detects_corruption(codec):
    x, c = _oracle_container()
    nb = x.numel() * 2
    assert _decode_status(codec, c, nb) == Z.ZIPNN_OK
    # header fields -> FORMAT
    for pos in (0, 4, 6, 16, 20, 22, 23, 28, 32, 50):
        d = c.copy()
        d[pos] ^= 0x04
        assert _decode_status(codec, d, nb) in (Z.ZIPNN_E_FORMAT, Z.ZIPNN_E_CORRUPT, Z.ZIPNN_E_NOSPACE), pos
    # map entries -> CORRUPT
    for pos in (64, 72, 76, 77, 78, 64 + 16 * 5 + 8):
        d = c.copy()
        d[pos] ^= 0x10
        assert _decode_status(codec, d, nb) == Z.ZIPNN_E_CORRUPT, pos
    # Huffman tables and sub-stream lengths -> CORRUPT
    off, nbytes, mode, _ = oracle.entry(c, 1, 0)
    assert mode == oracle.MODE_HUF
    d = c.copy()
    i = next(i for i in range(128) if d[off + i] & 15)
    d[off + i] = (d[off + i] & 0xF0) | ((d[off + i] & 15) % 11 + 1)
    assert _decode_status(codec, d, nb) == Z.ZIPNN_E_CORRUPT
    d = c.copy()
    d[off + 128 + 2 * 7] ^= 0x01
    assert _decode_status(codec, d, nb) == Z.ZIPNN_E_CORRUPT
    # truncated container, small output
    assert _decode_status(codec, c[: c.size - 16].copy(), nb) == Z.ZIPNN_E_FORMAT
    assert _decode_status(codec, c, nb - 2) == Z.ZIPNN_E_NOSPACE
    # a delta container needs its base, a plain one must not get one
    w = workloads.bf16_normal(1000, seed=1)
    dc = oracle.compress(w, oracle.BF16, base=w, chunk_bytes=1024, S=8)
    assert _decode_status(codec, dc, 2000) in (Z.ZIPNN_E_FORMAT, Z.ZIPNN_E_INVAL)
    assert _decode_status(codec, c, nb, base=x.cuda()) in (Z.ZIPNN_E_FORMAT, Z.ZIPNN_E_INVAL)
    assert codec.status() == Z.ZIPNN_OK


def test_async_decode_with_host_header(codec):
    x, c = _oracle_container()
    nb = x.numel() * 2
    assert _decode_status(codec, c, nb, header=c[:64].tobytes()) == Z.ZIPNN_OK
    # a header that does not describe this container: the device notices
    y = workloads.fp32_rows(2, 4096, seed=3)
    other = oracle.compress(y, oracle.FP32, S=256)
    assert _decode_status(codec, c, nb, header=other[:64].tobytes()) in (Z.ZIPNN_E_FORMAT, Z.ZIPNN_E_NOSPACE)
    g8 = oracle.compress(x, oracle.BF16, S=512, g=8)
    assert _decode_status(codec, c, nb, header=g8[:64].tobytes()) == Z.ZIPNN_E_FORMAT
    out = torch.empty(x.numel(), dtype=torch.bfloat16, device="cuda")
    codec.decompress(torch.from_numpy(c).cuda(), out, header=c[:64].tobytes())
    assert torch.equal(out.view(torch.int16).cpu(), x.view(torch.int16))


def test_api_argument_errors(codec):
    x = workloads.bf16_normal(1000, seed=1).cuda()
    p = Z.zipnn_default_params(Z.ZIPNN_BF16)
    dst = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(Z.ZipnnError) as ei:
        Z.zipnn_compress(codec.ctx, x.data_ptr(), Z.ZIPNN_BF16, x.numel(), None, p, dst.data_ptr(), 64,
                         codec._stream())
    assert ei.value.code == Z.ZIPNN_E_NOSPACE
    with pytest.raises(Z.ZipnnError) as ei:
        Z.zipnn_compress(codec.ctx, x.data_ptr() + 2, Z.ZIPNN_BF16, 10, None, p, dst.data_ptr(), 64,
                         codec._stream())
    assert ei.value.code == Z.ZIPNN_E_INVAL
    bad = Z.make_params(Z.ZIPNN_BF16, g=3)
    with pytest.raises(Z.ZipnnError):
        Z.zipnn_compress(codec.ctx, x.data_ptr(), Z.ZIPNN_BF16, 10, None, bad, dst.data_ptr(), 64, codec._stream())


@pytest.mark.parametrize("K", [1, 7])
def test_probe_skip_fp32(codec, K):
    """Compressibility probing (probe interval K): FP32 rows whose low byte
    groups are incompressible; the chunks after a probe store them raw
    without analysis, exactly as the oracle does."""
    x = workloads.fp32_rows(64, 8192, seed=21).reshape(-1)[: 9 * 65536 + 1001].clone()
    p = Z.make_params(Z.ZIPNN_FP32, probe_skip=K)
    c = roundtrip(codec, x, p)
    assert oracle.header(c.cpu().numpy())["skip"] == K


def test_probe_skip_mixed_chunks_and_batch(codec):
    """Random, then normal, then zero chunks (the normal chunks after a raw
    probe stay raw until the next probe), alone and in a batch where each
    tensor counts its chunks from zero."""
    E = 131072
    mixed = torch.cat([torch.randint(0, 65536, (3 * E,), generator=torch.Generator().manual_seed(5),
                                     dtype=torch.int32).to(torch.int16).view(torch.bfloat16),
                       workloads.bf16_normal(4 * E, seed=6), torch.zeros(2 * E + 7, dtype=torch.bfloat16)])
    p = Z.make_params(Z.ZIPNN_BF16, probe_skip=3)
    roundtrip(codec, mixed, p)
    xs = [mixed[: 5 * E + 3].cuda(), workloads.bf16_normal(3 * E + 11, seed=7).cuda(), mixed[E:].cuda()]
    arena, offs = codec.compress_batch(xs, p)
    a = arena.cpu().numpy()
    for i, x in enumerate(xs):
        ref = oracle.compress(x.cpu(), oracle.BF16, nthreads=8, **_oracle_kw(p))
        assert np.array_equal(a[offs[i]: offs[i] + ref.size], ref), i


@pytest.mark.parametrize("n", [1, 4 * 131072 + 3, 3 * 131072 + 37])
def test_exponent_extraction_bf16(codec, n):
    """Exponent extraction (header flag bit 2) on BF16: AUTO, and forced
    HUF/RAW with a ragged tail (the partial last group decodes element by
    element through the inverse transform)."""
    x = workloads.bf16_normal(n, seed=31)
    c = roundtrip(codec, x, Z.make_params(Z.ZIPNN_BF16, exponent=True))
    assert oracle.header(c.cpu().numpy())["flags"] & 4
    roundtrip(codec, x, Z.make_params(Z.ZIPNN_BF16, policy=[Z.ZIPNN_HUF, Z.ZIPNN_RAW], exponent=True, g=8))


def test_exponent_extraction_fp32_delta_zg_probe(codec):
    """FP32 with exponent extraction, alone, as an XOR delta (where ZG
    streams appear), and with probing."""
    x = workloads.fp32_rows(16, 65536 + 5, seed=32).reshape(-1)
    roundtrip(codec, x, Z.make_params(Z.ZIPNN_FP32, exponent=True))
    roundtrip(codec, x, Z.make_params(Z.ZIPNN_FP32, exponent=True, probe_skip=3))
    w = workloads.bf16_normal(2 * 131072 + 9, seed=33)
    ft = workloads.finetune_delta(w, seed=34)
    c = roundtrip(codec, ft, Z.make_params(Z.ZIPNN_BF16, exponent=True), base_cpu=w)
    assert oracle.header(c.cpu().numpy())["flags"] == 1 | 2 | 4


def test_exponent_extraction_only_bf16_fp32(codec):
    x = torch.zeros(1024, dtype=torch.float16, device="cuda")
    with pytest.raises(Z.ZipnnError) as ei:
        codec.compress(x, Z.make_params(Z.ZIPNN_FP16, exponent=True))
    assert ei.value.code == Z.ZIPNN_E_INVAL


def test_exponent_extraction_special_values_and_norms(codec):
    """Exponent extraction keeps NaN payloads, infinities, signed zeros and
    denormals bit-exact; norm-like BF16 weights (1 + N(0, 0.05)) and the
    maximal probe interval round-trip too."""
    raw = (torch.randn(200_003, generator=torch.Generator().manual_seed(35)) * 0.05).numpy().view(np.uint32).copy()
    special = np.array([0x7F800000, 0xFF800000, 0x7FC00001, 0xFFFFFFFF, 0x80000000, 1, 0x007FFFFF, 0, 0x80000001],
                       dtype=np.uint32)
    raw[1000: 1000 + 64 * len(special)] = np.repeat(special, 64)
    x = torch.from_numpy(raw.view(np.float32))
    roundtrip(codec, x, Z.make_params(Z.ZIPNN_FP32, exponent=True, probe_skip=255))
    norms = (1 + 0.05 * torch.randn(300_001, generator=torch.Generator().manual_seed(36))).to(torch.bfloat16)
    roundtrip(codec, norms, Z.make_params(Z.ZIPNN_BF16, exponent=True))
    roundtrip(codec, norms, Z.make_params(Z.ZIPNN_BF16, exponent=True, policy=[Z.ZIPNN_ZG, Z.ZIPNN_HUF]))


@pytest.mark.parametrize("n", [8 * 65536, 5 * 65536 + 4099])
def test_clean_fp32_single_valued_groups(codec, n):
    """'Clean' FP32 weights (paper §III-B: values that came from BF16, so the
    two low fraction bytes are zero): those byte groups are RLE in every
    chunk, beside a Huffman exponent group and a raw group; the decoder's
    fast loop fills them from a register."""
    x = workloads.bf16_normal(n, seed=37).to(torch.float32)
    c = roundtrip(codec, x, Z.zipnn_default_params(Z.ZIPNN_FP32)).cpu().numpy()
    assert [oracle.entry(c, 0, k)[2] for k in range(4)] == [oracle.MODE_HUF, oracle.MODE_RAW, oracle.MODE_RLE,
                                                             oracle.MODE_RLE]
    d = workloads.finetune_delta(workloads.bf16_normal(n, seed=38), seed=39).to(torch.float32)
    roundtrip(codec, d, Z.zipnn_default_params(Z.ZIPNN_FP32), base_cpu=workloads.bf16_normal(n, seed=38).to(torch.float32))


# ----------------------------------------------------------- 4 MiB chunks (the largest the format allows)

@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32, torch.uint8])
@pytest.mark.parametrize("div", [256, 2048])
def test_4mib_chunks(codec, dtype, div):
    """Chunks of 4 MiB with S = chunk elements / 256 (capped at the largest S,
    4096: W = 512 / 256 / 1024 sub-streams for BF16 / FP32 / U8) and / 2048
    (W = 2048), two full chunks and a ragged third, byte-compared with the
    oracle."""
    B = torch.empty(0, dtype=dtype).element_size()
    E = (4 << 20) // B
    n = 2 * E + 12345
    if dtype == torch.bfloat16:
        x = workloads.bf16_normal(n, seed=41)
    elif dtype == torch.float32:
        x = workloads.fp32_rows(n // 8192 + 1, 8192, seed=42).reshape(-1)[:n].contiguous()
    else:
        g = torch.Generator().manual_seed(43)
        x = (torch.randn(n, generator=g) * 12).round().clamp(-128, 127).to(torch.int16).to(torch.uint8)
    p = Z.make_params(Z.torch_dtype_code(dtype), chunk_bytes=4 << 20, S=min(4096, E // div))
    assert Z.zipnn_check_params(Z.torch_dtype_code(dtype), p) == Z.ZIPNN_OK
    roundtrip(codec, x, p, nthreads=16)


@pytest.mark.parametrize("policy", ["huf", "auto"])
def test_4mib_chunks_delta(codec, policy):
    """A BF16 XOR delta in 4 MiB chunks (S = 2048), both byte groups Huffman,
    or AUTO where ZG takes the mostly-zero groups."""
    E = (4 << 20) // 2
    base = workloads.bf16_normal(2 * E + 777, seed=44)
    ft = workloads.finetune_delta(base, seed=45)
    pol = [Z.ZIPNN_HUF, Z.ZIPNN_HUF] if policy == "huf" else [Z.ZIPNN_AUTO, Z.ZIPNN_AUTO]
    p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=4 << 20, S=2048, policy=pol)
    c = roundtrip(codec, ft, p, base_cpu=base, nthreads=16)
    if policy == "auto":
        info = Z.zipnn_inspect(c[:64 + 16 * 2 * 3].cpu().numpy().tobytes())
        assert info.entries_by_mode[3] > 0   # ZG entries present
