"""Batched encode/decode (one launch per kernel for all tensors of a
checkpoint) against per-tensor calls and the oracle; graph replays of the
prepared batch; mixed kernel classes; XOR deltas.  Zero differing bytes."""
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


def _kw(p):
    return dict(chunk_bytes=p.chunk_bytes, S=p.substream_syms, g=p.group, L=p.max_code_len, policy=list(p.policy),
                skip=p.probe_skip, exp=bool(p.exponent))


def _u8(t):
    return t.contiguous().view(torch.uint8).reshape(-1)


def _small_checkpoint(seed0=50):
    """A scaled-down decoder checkpoint: same kinds of tensors (weights,
    norms, an embedding), sizes cut so the oracle finishes in seconds, plus an
    empty tensor and ragged sizes."""
    specs = workloads.checkpoint_8b_specs(layers=2, hidden=256, kv=64, ffn=896, vocab=3001, seed0=seed0)
    xs = [workloads.make_tensor(s) for s in specs]
    xs.insert(3, torch.empty(0, dtype=torch.bfloat16))
    xs.append(workloads.bf16_normal(131072 * 2 + 5, seed=seed0 + 99))
    return xs


def test_batch_equals_per_tensor_and_oracle(codec):
    xs = _small_checkpoint()
    p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=65536)
    dev = [x.cuda() for x in xs]
    arena, offs = codec.compress_batch(dev, p)
    a = arena.cpu().numpy()
    print("tensors", len(xs), "arena bytes", offs[-1], flush=True)
    for i, x in enumerate(xs):
        assert offs[i] % 128 == 0     # containers start 128-byte aligned in the arena
        total = int.from_bytes(a[offs[i] + 32: offs[i] + 40].tobytes(), "little")   # header: container size
        ci = a[offs[i]: offs[i] + total]
        ref = oracle.compress(x, oracle.BF16, **_kw(p))
        assert np.array_equal(ci, ref), i
        solo = codec.compress(dev[i], p).cpu().numpy()
        assert np.array_equal(solo, ref), i
    outs = [torch.empty_like(x) for x in dev]
    Z.zipnn_decompress_batch(codec.ctx, arena.data_ptr(), offs, [o.data_ptr() for o in outs],
                             [o.numel() * 2 for o in outs], None, codec._stream())
    assert codec.status() == Z.ZIPNN_OK
    for o, x in zip(outs, dev):
        assert torch.equal(_u8(o), _u8(x))


def test_prepared_batch_graph_replays(codec):
    xs = [x.cuda() for x in _small_checkpoint(seed0=70)]
    p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=65536)
    arena, offs = codec.compress_batch(xs, p)
    outs = [torch.zeros_like(x) for x in xs]
    b = codec.prepare_batch(arena, offs, outs)
    for rep in range(4):
        for o in outs:
            o.fill_(rep + 1)   # eager work between replays
        torch.cuda.synchronize()
        b.run(check=True)
        torch.cuda.synchronize()
        for o, x in zip(outs, xs):
            assert torch.equal(_u8(o), _u8(x)), rep
    b.close()


def test_batch_mixed_classes(codec):
    """BF16 (g=4), FP32, FP8 and a BF16 g=8 container in one arena: one
    launch per (B, g, delta) class."""
    xb = workloads.bf16_normal(300_001, seed=1).cuda()
    xf = workloads.fp32_rows(3, 50_000, seed=2).reshape(-1).cuda()
    x8 = workloads.make_corpus_tensor(workloads.CorpusItem(0, "fp8", 400_000, 3)).cuda()
    xg = workloads.bf16_normal(200_000, seed=4).cuda()
    cs = [codec.compress(xb, Z.zipnn_default_params(Z.ZIPNN_BF16)),
          codec.compress(xf, Z.zipnn_default_params(Z.ZIPNN_FP32)),
          codec.compress(x8, Z.zipnn_default_params(Z.ZIPNN_FP8_E4M3)),
          codec.compress(xg, Z.make_params(Z.ZIPNN_BF16, g=8))]
    offs = [0]
    for c in cs:
        offs.append(offs[-1] + (c.numel() + 15) // 16 * 16)
    arena = torch.zeros(offs[-1], dtype=torch.uint8, device="cuda")
    for c, o in zip(cs, offs):
        arena[o: o + c.numel()] = c
    xs = [xb, xf, x8, xg]
    outs = [torch.empty_like(x) for x in xs]
    b = codec.prepare_batch(arena, offs, outs)
    b.run(check=True)
    torch.cuda.synchronize()
    for o, x in zip(outs, xs):
        assert torch.equal(_u8(o), _u8(x))
    b.close()


def test_batch_xor_delta(codec):
    base = [x.cuda() for x in _small_checkpoint(seed0=90)]
    ft = [workloads.finetune_delta(x, seed=2000 + i) if x.numel() else x.clone() for i, x in enumerate(base)]
    p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=65536, policy=[Z.ZIPNN_HUF, Z.ZIPNN_HUF])
    arena, offs = codec.compress_batch(ft, p, bases=base)
    a = arena.cpu().numpy()
    for i in (0, 1, len(base) - 1):
        ref = oracle.compress(ft[i].cpu(), oracle.BF16, base=base[i].cpu(), **_kw(p))
        assert np.array_equal(a[offs[i]: offs[i] + ref.size], ref), i
    outs = [torch.empty_like(x) for x in ft]
    b = codec.prepare_batch(arena, offs, outs, bases=base)
    b.run(check=True)
    torch.cuda.synchronize()
    for o, x in zip(outs, ft):
        assert torch.equal(_u8(o), _u8(x))
    b.close()
    assert offs[-1] < 0.25 * sum(x.numel() * 2 for x in ft)


def test_batch_errors(codec):
    xs = [workloads.bf16_normal(70_000, seed=5).cuda()]
    arena, offs = codec.compress_batch(xs, Z.zipnn_default_params(Z.ZIPNN_BF16))
    out = torch.empty_like(xs[0])
    with pytest.raises(Z.ZipnnError) as ei:       # output too small
        Z.zipnn_batch_create(codec.ctx, arena.data_ptr(), offs, [out.data_ptr()], [out.numel() * 2 - 2])
    assert ei.value.code == Z.ZIPNN_E_NOSPACE
    with pytest.raises(Z.ZipnnError) as ei:       # misaligned offset
        Z.zipnn_batch_create(codec.ctx, arena.data_ptr(), [8, offs[1]], [out.data_ptr()], [out.numel() * 2])
    assert ei.value.code == Z.ZIPNN_E_INVAL
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(Z.ZipnnError) as ei:       # arena too small
        Z.zipnn_compress_batch(codec.ctx, Z.ZIPNN_BF16, [xs[0].data_ptr()], [xs[0].numel()], [None],
                               Z.zipnn_default_params(Z.ZIPNN_BF16), small.data_ptr(), 64, codec._stream())
    assert ei.value.code == Z.ZIPNN_E_NOSPACE


def _sample_indices(n):
    """Tensors whose containers the oracle recomputes at full size: the
    embedding, the first layer's tensors, every 17th tensor and the head."""
    return sorted(set([0, 1, 2, 3, 4, 5, 6, 7, 8, 9] + list(range(0, n, 17)) + [n - 2, n - 1]))


@pytest.mark.slow
@pytest.mark.parametrize("chunk,S", [(262144, 512), (1048576, 2048), ("tuned", None)])
def test_checkpoint_8b_full(codec, chunk, S):
    """The full 8B-shaped BF16 checkpoint (291 tensors, 16.06 GB) batched:
    one encode launch chain, one prepared (graph) decode, at the paper's
    default chunk, at 1 MiB, and at the autotuner's pick with the benchmark's
    settings (the configuration the benchmark times).  Every tensor
    round-trips bit-exactly; sampled containers equal the oracle's bytes."""
    specs = workloads.checkpoint_8b_specs()
    xs = [workloads.make_tensor(sp, device="cuda") for sp in specs]
    if chunk == "tuned":
        p, _ = Z.tune_checkpoint(codec, xs)
        print("autotuned:", p, flush=True)
    else:
        p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=chunk, S=S)
    arena, offs = codec.compress_batch(xs, p)
    outs = [torch.empty_like(x) for x in xs]
    b = codec.prepare_batch(arena, offs, outs)
    b.run(check=True)
    torch.cuda.synchronize()
    for i, (o, x) in enumerate(zip(outs, xs)):
        assert torch.equal(_u8(o), _u8(x)), i
    del outs
    b.close()
    for i in _sample_indices(len(xs)):
        print("oracle check tensor", i, specs[i].name, flush=True)
        ref = oracle.compress(xs[i].cpu(), oracle.BF16, nthreads=16, **_kw(p))
        got = arena[offs[i]: offs[i] + ref.size].cpu().numpy()
        assert np.array_equal(got, ref), i


@pytest.mark.slow
@pytest.mark.parametrize("policy,chunk,S", [("huf", 262144, 512), ("huf", "tuned", None), ("auto", "tuned", None)])
def test_checkpoint_8b_delta_full(codec, policy, chunk, S):
    """The full XOR-delta checkpoint: fine-tuned copy against the base, both
    streams Huffman (or AUTO, where ZG takes almost every stream), in the
    default shape and at the autotuner's pick with the benchmark's settings;
    every tensor reconstructs bit-exactly; sampled containers equal the
    oracle's."""
    specs = workloads.checkpoint_8b_specs()
    base = [workloads.make_tensor(sp, device="cuda") for sp in specs]
    ft = [workloads.finetune_delta(w, seed=2000 + i) for i, w in enumerate(base)]
    pol = [Z.ZIPNN_HUF, Z.ZIPNN_HUF] if policy == "huf" else [Z.ZIPNN_AUTO, Z.ZIPNN_AUTO]
    if chunk == "tuned":
        p, _ = Z.tune_checkpoint(codec, ft, base, pol if policy == "huf" else None)
        print("autotuned:", p, flush=True)
    else:
        p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=chunk, S=S, policy=pol)
    arena, offs = codec.compress_batch(ft, p, base)
    outs = [torch.empty_like(x) for x in ft]
    b = codec.prepare_batch(arena, offs, outs, base)
    b.run(check=True)
    torch.cuda.synchronize()
    for i, (o, x) in enumerate(zip(outs, ft)):
        assert torch.equal(_u8(o), _u8(x)), i
    del outs
    b.close()
    for i in _sample_indices(len(ft))[::3]:
        print("oracle check delta tensor", i, specs[i].name, flush=True)
        ref = oracle.compress(ft[i].cpu(), oracle.BF16, base=base[i].cpu(), nthreads=16, **_kw(p))
        got = arena[offs[i]: offs[i] + ref.size].cpu().numpy()
        assert np.array_equal(got, ref), i


def test_autotune_picks_fastest_within_ratio_loss(codec):
    """The autotuner measures every candidate (chunk 64 KiB..1 MiB by default
    x 256 to 2048 sub-streams per chunk) on a sample holding a share of every
    tensor; among candidates within the ratio loss, decode rates within `tie`
    of the fastest tie and the smallest chunk, then the best ratio, wins.  Its
    pick compresses to the oracle's bytes."""
    xs = [x.cuda() for x in _small_checkpoint(seed0=300)]
    loss, tie = 0.01, 0.02
    best, table = Z.zipnn_autotune(codec.ctx, Z.ZIPNN_BF16, [x.data_ptr() for x in xs], [x.numel() for x in xs],
                                   [None] * len(xs), 64 << 20, loss, None, tie=tie)
    assert len(table) == 5 * 4
    for e in table:
        E = e.params.chunk_bytes // 2
        assert 64 << 10 <= e.params.chunk_bytes <= 1 << 20 and 256 <= E // e.params.substream_syms <= 2048
    r0 = min(e.ratio for e in table)
    ok = [e for e in table if e.ratio <= r0 * (1 + loss)]
    fastest = max(e.decode_gbps for e in ok)
    ties = [e for e in ok if e.decode_gbps >= fastest * (1 - tie)]
    pick = min(ties, key=lambda e: (e.params.chunk_bytes, e.ratio))
    assert (best.chunk_bytes, best.substream_syms) == (pick.params.chunk_bytes, pick.params.substream_syms)
    x = xs[1]
    c = codec.compress(x, best)
    ref = oracle.compress(x.cpu(), oracle.BF16, nthreads=8, **_kw(best))
    assert np.array_equal(c.cpu().numpy(), ref)
    # another chunk range: only those chunk sizes are measured
    _, t2 = Z.zipnn_autotune(codec.ctx, Z.ZIPNN_BF16, [x.data_ptr()], [x.numel()], [None], 8 << 20, loss, None,
                             min_chunk=2 << 20, max_chunk=4 << 20, repeats=3)
    assert {e.params.chunk_bytes for e in t2} == {2 << 20, 4 << 20}
    # a policy value out of range leaves no candidate: rejected, nothing measured
    with pytest.raises(Z.ZipnnError) as ei:
        Z.zipnn_autotune(codec.ctx, Z.ZIPNN_BF16, [x.data_ptr()], [x.numel()], [None], 1 << 20, loss, [9, 9])
    assert ei.value.code == Z.ZIPNN_E_INVAL
    # an empty or inverted chunk range is rejected
    with pytest.raises(Z.ZipnnError) as ei:
        Z.zipnn_autotune(codec.ctx, Z.ZIPNN_BF16, [x.data_ptr()], [x.numel()], [None], 1 << 20, loss, None,
                         min_chunk=1 << 20, max_chunk=64 << 10)
    assert ei.value.code == Z.ZIPNN_E_INVAL


def test_prepared_encoder_graph_replays(codec):
    """The prepared encoder (descriptors uploaded once, launches captured in a
    hipGraph) gives zipnn_compress_batch's bytes on every replay, with eager
    work of the program (another compress, a decompress, synchronisations)
    between the replays; a delta batch too."""
    xs = [x.cuda() for x in _small_checkpoint(seed0=700)]
    p = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=65536)
    arena, offs = codec.compress_batch(xs, p)
    ref = arena[: offs[-1]].cpu().numpy().copy()

    def containers(a):
        # each container by its header's size (the gap after a 64-byte empty
        # container, up to the next 128-byte offset, is not part of any)
        return [a[o: o + int.from_bytes(a[o + 32: o + 40].tobytes(), "little")] for o in offs[:-1]]

    enc = codec.prepare_encoder(xs, p)
    for r in range(3):
        enc.arena.fill_(0xA5)          # the replay must write every byte of the containers
        got_offs = enc.run()
        assert got_offs == offs, r
        got = containers(enc.arena[: offs[-1]].cpu().numpy())
        assert all(np.array_equal(a, b) for a, b in zip(got, containers(ref))), r
        # eager work between replays
        c = codec.compress(xs[1], p)
        out = torch.empty_like(xs[1])
        codec.decompress(c, out)
        torch.cuda.synchronize()
        assert torch.equal(_u8(out), _u8(xs[1]))
    enc.close()
    i = 1
    want = oracle.compress(xs[i].cpu(), oracle.BF16, nthreads=8, **_kw(p))
    assert np.array_equal(ref[offs[i]: offs[i] + want.size], want)
    base = [workloads.bf16_normal(x.numel(), seed=800 + k).cuda() if x.numel() else x for k, x in enumerate(xs)]
    ft = [workloads.finetune_delta(b, seed=900 + k) if b.numel() else b for k, b in enumerate(base)]
    a2, o2 = codec.compress_batch(ft, p, base)
    enc = codec.prepare_encoder(ft, p, base)
    ref2 = a2[: o2[-1]].cpu().numpy()
    for r in range(2):
        assert enc.run() == o2
        got = enc.arena[: o2[-1]].cpu().numpy()
        assert all(np.array_equal(got[o: o + len(c)], c) for o, c in zip(o2[:-1], [ref2[o:][: int.from_bytes(
            ref2[o + 32: o + 40].tobytes(), "little")] for o in o2[:-1]]))
    enc.close()
