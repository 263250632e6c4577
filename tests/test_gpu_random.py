"""GPU parity on seeded random shapes: the HIP container equals the oracle's
byte for byte and both decode to the input.

Each seed draws a word type, a chunk size, S, g, L, a policy per byte group
(AUTO, HUF, RAW or ZG), an XOR base or none, probing and a length around a
chunk and lane-group boundary.  The values mix zeros, a few frequent bytes
and spread bytes, so that one chunk can hold RAW, RLE, HUF and ZG groups
side by side: the packer writes all coded groups of a chunk in one pass, and
the decoder meets every mode set.  Bar: zero differing bytes."""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_05239_amd import zipnn as Z

pytestmark = pytest.mark.gpu

DTYPES = [(Z.ZIPNN_BF16, torch.bfloat16), (Z.ZIPNN_FP16, torch.float16), (Z.ZIPNN_FP32, torch.float32),
          (Z.ZIPNN_FP8_E4M3, torch.float8_e4m3fn), (Z.ZIPNN_U8, torch.uint8)]


@pytest.fixture(scope="module")
def codec():
    c = Z.Codec(0)
    yield c
    c.close()


def _case(seed):
    rng = np.random.default_rng(5000 + seed)
    dt, tdt = DTYPES[seed % len(DTYPES)]
    B = Z.WIDTH[dt]
    chunk = int(rng.choice([1024, 4096, 16384, 65536, 262144]))
    g = int(rng.choice([2, 4, 8]))
    E = chunk // B
    S = int(rng.choice([s for s in (2, 4, 8, 16, 32, 64, 128, 256, 512) if s >= g and E // s <= 4096 and chunk // s <= 8192]))
    L = int(rng.integers(8, 12))
    policy = [int(rng.choice([Z.ZIPNN_AUTO, Z.ZIPNN_HUF, Z.ZIPNN_RAW, Z.ZIPNN_ZG])) for _ in range(B)]
    skip = int(rng.choice([0, 0, 0, 1, 3]))
    if seed % 13 == 0:
        n = int(rng.integers(1, 70))   # fewer elements than one lane group has sub-streams
    else:
        n = max(g + 1, int(rng.integers(1, 4)) * E + int(rng.integers(-3 * S, 3 * S + 1)) + int(rng.integers(0, 9)))
    # bytes: per byte group a mix of zeros, a few hot values and spread values
    raw = np.zeros((n, B), dtype=np.uint8)
    for k in range(B):
        kind = rng.integers(0, 4)
        if kind == 0:      # mostly zero, some spread bytes (delta-like)
            v = np.where(rng.random(n) < 0.8, 0, rng.integers(0, 256, n))
        elif kind == 1:    # a few hot values (exponent-like)
            v = rng.choice(np.array([0x3C, 0x3D, 0x3E, 0xBC, 0xBD]), n, p=[0.4, 0.3, 0.15, 0.1, 0.05])
        elif kind == 2:    # spread (fraction-like)
            v = rng.integers(0, 256, n)
        else:              # a single value (RLE)
            v = np.full(n, int(rng.integers(0, 256)))
        raw[:, B - 1 - k] = v.astype(np.uint8)
    x = torch.from_numpy(raw.reshape(-1).copy()).view(tdt)
    base = None
    if rng.random() < 0.3:
        base = torch.from_numpy(rng.integers(0, 256, n * B, dtype=np.uint8)).view(tdt)
        x = torch.from_numpy((raw.reshape(-1) ^ base.view(torch.uint8).numpy())).view(tdt)
    p = Z.make_params(dt, chunk_bytes=chunk, S=S, g=g, L=L, policy=policy, probe_skip=skip)
    return dt, x, base, p


@pytest.mark.parametrize("seed", range(40))
def test_random_shapes_match_oracle(codec, seed):
    dt, x_cpu, base_cpu, p = _case(seed)
    print(f"seed {seed}: dtype {dt} n {x_cpu.numel()} chunk {p.chunk_bytes} S {p.substream_syms} g {p.group} "
          f"L {p.max_code_len} policy {list(p.policy)} skip {p.probe_skip} delta {base_cpu is not None}", flush=True)
    x = x_cpu.cuda()
    base = base_cpu.cuda() if base_cpu is not None else None
    c_gpu = codec.compress(x, p, base=base)
    c_orc = oracle.compress(x_cpu, dt, base=base_cpu, nthreads=8, chunk_bytes=p.chunk_bytes, S=p.substream_syms,
                            g=p.group, L=p.max_code_len, policy=list(p.policy), skip=p.probe_skip, exp=False)
    got = c_gpu.cpu().numpy()
    assert got.size == c_orc.size, (got.size, c_orc.size)
    if not np.array_equal(got, c_orc):
        bad = np.nonzero(got != c_orc)[0]
        raise AssertionError(f"{bad.size} container bytes differ, first at {bad[:8]}")
    out = torch.empty_like(x)
    codec.decompress(c_gpu, out, base=base)
    assert torch.equal(out.view(torch.uint8), x.view(torch.uint8))
    back = oracle.decompress(got, base=base_cpu, nthreads=8)
    assert np.array_equal(back, oracle.as_bytes(x_cpu))
