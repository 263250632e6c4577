"""GPU parity of staged packing, the encode path of launches with an XOR base.

There the analysis decides each AUTO byte group's mode from lower bounds of
the candidates' sizes and runs its exact-size pass only for chunks whose
bounds leave the choice open; the packer writes every lane group's words into
a bounded staging slot and records its word count; placement sizes the
payloads from those counts, and a compaction writes the map entries and heads
and moves the words, bitmaps and raw byte groups to their places.  The
containers must equal the oracle's byte for byte, as those of the exact path
do.  The cases below aim at what only this path does: decisions at the
HUF/RAW and HUF/ZG boundaries (where the size pass runs), launches that mix
tensors with and without a base, raw groups copied through the slots with
small and large groups, probing with exponent extraction, replays of a
prepared encoder, and an output too small for the container."""
import numpy as np
import pytest
import torch

import oracle
import test_gpu_parity
from paper_2411_05239_amd import workloads
from paper_2411_05239_amd import zipnn as Z

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def codec():
    c = Z.Codec(0)
    yield c
    c.close()


def _kw(p):
    return dict(chunk_bytes=p.chunk_bytes, S=p.substream_syms, g=p.group, L=p.max_code_len, policy=list(p.policy),
                skip=p.probe_skip, exp=bool(p.exponent))


def _u8(t):
    return t.view(torch.uint8)


def _boundary_bytes(n_chunks, E, q_range, seed):
    """BF16 words whose high byte group runs, chunk by chunk, from slightly
    below to slightly above the size where Huffman stops beating raw (a share
    q of four hot values, the rest spread; where that size lies depends on
    the sub-stream count), and whose low byte group runs across the point
    where ZG starts beating Huffman (a share p0 of zeros)."""
    rng = np.random.default_rng(seed)
    raw = np.zeros((n_chunks * E, 2), np.uint8)
    for c, (q, p0) in enumerate(zip(np.linspace(*q_range, n_chunks), np.linspace(0.5, 0.97, n_chunks))):
        hi = np.where(rng.random(E) < q, rng.choice(np.array([3, 7, 11, 19]), E), rng.integers(0, 256, E))
        lo = np.where(rng.random(E) < p0, 0, rng.integers(1, 256, E))
        raw[c * E:(c + 1) * E, 1] = hi
        raw[c * E:(c + 1) * E, 0] = lo
    return raw.reshape(-1)


@pytest.mark.parametrize("chunk,S,q_range", [(65536, 128, (0.08, 0.16)), (262144, 512, (0.02, 0.10))])
def test_decisions_at_the_size_boundaries(codec, chunk, S, q_range):
    E = chunk // 2
    nch = 24
    raw = _boundary_bytes(nch, E, q_range, seed=chunk + S)
    rng = np.random.default_rng(11)
    base = rng.integers(0, 256, raw.size, dtype=np.uint8)
    x = raw ^ base
    p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=chunk, S=S)
    # the data straddles both decisions: the oracle's own AUTO choices (on the
    # delta, which is `raw`) include RAW and HUF for the high byte group and
    # HUF and ZG for the low one
    auto = oracle.compress(raw, oracle.BF16, chunk_bytes=chunk, S=S)
    modes = [{oracle.entry(auto, c, k)[2] for c in range(nch)} for k in range(2)]
    assert {oracle.MODE_RAW, oracle.MODE_HUF} <= modes[0], modes[0]
    assert {oracle.MODE_HUF, oracle.MODE_ZG} <= modes[1], modes[1]
    # some chunk's Huffman size lies in [m - W, m): its bounds (at most 8
    # bytes per sub-stream apart) overlap the raw size, so that chunk runs the
    # exact-size pass on this path
    W = E // S
    huf = oracle.compress(raw, oracle.BF16, chunk_bytes=chunk, S=S, policy=[oracle.HUF, oracle.HUF])
    assert any(E - W <= oracle.entry(huf, c, 0)[1] < E for c in range(nch))
    xt = torch.from_numpy(x).view(torch.bfloat16).cuda()
    bt = torch.from_numpy(base).view(torch.bfloat16).cuda()
    got = codec.compress(xt, p, base=bt).cpu().numpy()
    want = oracle.compress(x, oracle.BF16, base=base, nthreads=8, **_kw(p))
    assert got.size == want.size
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} bytes differ, first at {bad[:8]}"
    out = torch.empty_like(xt)
    codec.decompress(torch.from_numpy(got).cuda(), out, base=bt)
    assert torch.equal(_u8(out).cpu(), torch.from_numpy(x))


def test_launch_mixing_tensors_with_and_without_base(codec):
    """Every tensor of a launch that has a base somewhere takes the staged
    path, with or without a base of its own: sizes around chunk and lane-group
    boundaries, an empty tensor and tensors of one and a few elements."""
    p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=65536)
    E = 32768
    sizes = [3 * E + 17, 0, 1, 37, E, 2 * E - 5, 300]
    has_base = [True, False, True, True, False, True, False]
    xs, bases = [], []
    for i, (n, hb) in enumerate(zip(sizes, has_base)):
        b = workloads.bf16_normal(n, seed=300 + i)
        bases.append(b.cuda() if hb else None)
        xs.append((workloads.finetune_delta(b, seed=400 + i) if hb else b).cuda())
    arena, offs = codec.compress_batch(xs, p, bases)
    a = arena.cpu().numpy()
    for i, (x, b) in enumerate(zip(xs, bases)):
        want = oracle.compress(x.cpu(), oracle.BF16, base=b.cpu() if b is not None else None, nthreads=8, **_kw(p))
        assert offs[i + 1] - offs[i] >= want.size, i
        assert np.array_equal(a[offs[i]: offs[i] + want.size], want), i
    outs = [torch.empty_like(x) for x in xs]
    b = codec.prepare_batch(arena, offs, outs, bases=bases)
    b.run(check=True)
    torch.cuda.synchronize()
    for o, x in zip(outs, xs):
        assert torch.equal(_u8(o), _u8(x))
    b.close()


@pytest.mark.parametrize("g", [2, 4, 8])
@pytest.mark.parametrize("dtype", ["bf16", "fp32"])
def test_raw_groups_through_the_slots(codec, dtype, g):
    """Raw byte groups pass through the staging slots: copied by the packer's
    pass for groups of at most 16 bytes, by the separate raw copy otherwise,
    then moved by the compaction, next to coded groups."""
    if dtype == "bf16":
        dt, tdt, pol = Z.ZIPNN_BF16, torch.bfloat16, [Z.ZIPNN_HUF, Z.ZIPNN_RAW]
        base = workloads.bf16_normal(5 * 32768 + 999, seed=50 + g)
    else:
        dt, tdt, pol = Z.ZIPNN_FP32, torch.float32, [Z.ZIPNN_HUF, Z.ZIPNN_RAW, Z.ZIPNN_AUTO, Z.ZIPNN_RAW]
        base = torch.randn(3 * 16384 + 501, generator=torch.Generator().manual_seed(60 + g)) * 0.02
    x = workloads.finetune_delta(base, seed=70 + g) if dtype == "bf16" else base + torch.randn(
        base.numel(), generator=torch.Generator().manual_seed(80 + g)) * 1e-4
    p = Z.make_params(dt, chunk_bytes=65536, g=g, policy=pol)
    got = codec.compress(x.cuda(), p, base=base.cuda()).cpu().numpy()
    want = oracle.compress(x, {Z.ZIPNN_BF16: oracle.BF16, Z.ZIPNN_FP32: oracle.FP32}[dt], base=base, nthreads=8,
                           **_kw(p))
    assert np.array_equal(got, want)
    out = torch.empty(x.numel(), dtype=tdt, device="cuda")
    codec.decompress(torch.from_numpy(got).cuda(), out, base=base.cuda())
    assert torch.equal(_u8(out).cpu(), _u8(x))


def test_probing_and_exponent_extraction(codec):
    base = workloads.bf16_normal(6 * 32768 + 77, seed=91)
    x = workloads.finetune_delta(base, seed=92)
    for skip, exp in ((2, False), (0, True), (3, True)):
        p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=65536, probe_skip=skip, exponent=exp)
        got = codec.compress(x.cuda(), p, base=base.cuda()).cpu().numpy()
        want = oracle.compress(x, oracle.BF16, base=base, nthreads=8, **_kw(p))
        assert np.array_equal(got, want), (skip, exp)


def test_prepared_encoder_replays_staged(codec):
    """The prepared encoder replays the staged launches from a hipGraph: the
    same bytes on every replay, with eager work between the replays."""
    p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=65536)
    base = [workloads.bf16_normal(n, seed=500 + i).cuda() for i, n in enumerate((2 * 32768 + 3, 32768, 4099))]
    ft = [workloads.finetune_delta(b, seed=600 + i) for i, b in enumerate(base)]
    a1, o1 = codec.compress_batch(ft, p, base)
    ref = a1[: o1[-1]].cpu().numpy()
    enc = codec.prepare_encoder(ft, p, base)
    for r in range(3):
        assert enc.run() == o1
        got = enc.arena[: o1[-1]].cpu().numpy()
        for i in range(len(ft)):
            want = oracle.compress(ft[i].cpu(), oracle.BF16, base=base[i].cpu(), nthreads=8, **_kw(p))
            assert np.array_equal(got[o1[i]: o1[i] + want.size], want), (r, i)
        assert np.array_equal(got, ref)
        torch.cuda.synchronize()
        _ = (ft[0].float() * 2).sum().item()   # eager work between replays
    enc.close()


def test_output_too_small_leaves_the_rest_untouched(codec):
    base = workloads.bf16_normal(4 * 32768 + 5, seed=93).cuda()
    x = workloads.finetune_delta(base, seed=94)
    p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=65536)
    need = codec.compress(x, p, base=base).numel()
    cap = need - 200
    dst = torch.full((need + 4096,), 0xA5, dtype=torch.uint8, device="cuda")
    with pytest.raises(Z.ZipnnError) as ei:
        Z.zipnn_compress(codec.ctx, x.data_ptr(), Z.ZIPNN_BF16, x.numel(), base.data_ptr(), p, dst.data_ptr(), cap,
                         codec._stream())
    assert ei.value.code == Z.ZIPNN_E_NOSPACE
    torch.cuda.synchronize()
    assert bool((dst[cap:] == 0xA5).all())


@pytest.mark.parametrize("dtype,g", [(torch.uint8, 2), (torch.uint8, 8), (torch.bfloat16, 8), (torch.float32, 4)])
def test_longest_codes_through_the_slots(codec, dtype, g):
    """Lanes whose every code is at the length limit take the most words a
    staging slot is sized for."""
    test_gpu_parity.test_longest_codes_at_the_length_limit(codec, dtype, g, base=True)
