"""Pins for the CPU oracle: what the paper and the mathematics fix, checked
against things other than the oracle itself (closed forms, hand-worked
examples, brute force, textbook Huffman, entropy bounds, a second independent
implementation)."""
import heapq
import itertools
import math
import os
import struct

import numpy as np
import pytest
import torch

import oracle
import oracle.spec as spec
from paper_2411_05239_amd import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _bf16_words(hexes):
    return np.array([int(h, 16) for h in hexes], dtype=np.uint16)


# ----------------------------------------------------------- byte grouping

@pytest.mark.parametrize("dtype,torch_dtype,value,expect", [
    (oracle.BF16, torch.bfloat16, 1.0, [0x3F, 0x80]),
    (oracle.FP32, torch.float32, 1.0, [0x3F, 0x80, 0x00, 0x00]),
    (oracle.FP32, torch.float32, -2.0, [0xC0, 0x00, 0x00, 0x00]),
    (oracle.FP16, torch.float16, 1.0, [0x3C, 0x00]),
])
def test_split_known_words(oracle_lib, dtype, torch_dtype, value, expect):
    """Stream k holds byte B-1-k: stream 0 is sign + exponent (paper §III-A)."""
    x = torch.tensor([value, value], dtype=torch_dtype)
    c = oracle.compress(x, dtype, chunk_bytes=256, policy=(oracle.RAW,) * 4)
    for k, byte in enumerate(expect):
        off, nb, mode, _ = oracle.entry(c, 0, k)
        assert mode == oracle.MODE_RAW and nb == 2
        assert list(c[off:off + 2]) == [byte, byte]


def test_split_matches_numpy_view(oracle_lib):
    """RAW payloads equal the closed form x.view(u8).reshape(n,B)[:, ::-1].T."""
    x = workloads.fp32_rows(4, 64, seed=5)
    c = oracle.compress(x, oracle.FP32, chunk_bytes=256, policy=(oracle.RAW,) * 4)
    a = x.numpy().view(np.uint8).reshape(-1, 4)[:, ::-1].T
    E = 256 // 4
    for ch in range(x.numel() // E):
        for k in range(4):
            off, nb, _, _ = oracle.entry(c, ch, k)
            assert np.array_equal(c[off:off + nb], a[k, ch * E:(ch + 1) * E])


# ----------------------------------------------------------- package-merge

def _read_pm_examples():
    rows = []
    for line in open(os.path.join(GOLD, "package_merge_examples.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        L, f, l = (p.strip() for p in line.split("|"))
        rows.append((int(L), [int(v) for v in f.split()], [int(v) for v in l.split()]))
    return rows


@pytest.mark.parametrize("L,freq,expect", _read_pm_examples())
def test_package_merge_worked_examples(oracle_lib, L, freq, expect):
    got = oracle.package_merge(freq, L)[:len(freq)]
    assert list(got) == expect
    s = spec.pm_lengths(dict(enumerate(freq)), L)
    assert [s[i] for i in range(len(freq))] == expect


def _brute_force_cost(freq, L):
    best = None
    n = len(freq)
    for lens in itertools.product(range(1, L + 1), repeat=n):
        if sum(2.0 ** -l for l in lens) <= 1.0 + 1e-12:
            c = sum(f * l for f, l in zip(freq, lens))
            best = c if best is None else min(best, c)
    return best


def test_package_merge_optimal_vs_brute_force(oracle_lib):
    """Cost sum f*l equals the minimum over ALL length vectors in [1..L]^n
    with Kraft sum <= 1 (exhaustive), for random tiny alphabets."""
    rng = np.random.default_rng(7)
    checked = 0
    for _ in range(300):
        n = int(rng.integers(2, 7))
        L = int(rng.integers(max(1, math.ceil(math.log2(n))), 6))
        freq = [int(v) for v in rng.integers(1, 60, size=n)]
        if rng.random() < 0.3:  # skewed, so the limit binds
            freq = [int(2 ** rng.integers(0, 12)) for _ in range(n)]
        got = oracle.package_merge(freq, L)[:n]
        assert max(got) <= L
        assert sum(2.0 ** -int(l) for l in got) == 1.0            # Kraft equality
        assert sum(f * int(l) for f, l in zip(freq, got)) == _brute_force_cost(freq, L)
        checked += 1
    assert checked == 300


def _huffman_cost_and_depth(freq):
    """Textbook Huffman with a heap: returns (cost, max depth)."""
    heap = [(f, i, {i: 0}) for i, f in enumerate(freq)]
    heapq.heapify(heap)
    uid = len(freq)
    while len(heap) > 1:
        fa, _, a = heapq.heappop(heap)
        fb, _, b = heapq.heappop(heap)
        d = {k: v + 1 for k, v in {**a, **b}.items()}
        heapq.heappush(heap, (fa + fb, uid, d))
        uid += 1
    depths = heap[0][2]
    return sum(freq[i] * depths[i] for i in depths), max(depths.values())


def test_package_merge_equals_huffman_when_unrestricted(oracle_lib):
    rng = np.random.default_rng(11)
    for _ in range(200):
        n = int(rng.integers(2, 257))
        freq = [int(v) for v in rng.integers(1, 10000, size=n)]
        cost, depth = _huffman_cost_and_depth(freq)
        got = oracle.package_merge(freq, 11)[:n]
        pm_cost = sum(f * int(l) for f, l in zip(freq, got))
        if depth <= 11:
            assert pm_cost == cost
        else:
            assert pm_cost >= cost


def test_package_merge_limit_binds_on_fibonacci(oracle_lib):
    """Fibonacci weights give an unrestricted Huffman depth of n-1; with 16
    symbols and L = 11 the limit must bind, and the code stays complete."""
    fib = [1, 1]
    while len(fib) < 16:
        fib.append(fib[-1] + fib[-2])
    cost, depth = _huffman_cost_and_depth(fib)
    assert depth == 15
    got = oracle.package_merge(fib, 11)[:16]
    assert int(max(got)) == 11
    assert sum(2.0 ** -int(l) for l in got) == 1.0
    assert sum(f * int(l) for f, l in zip(fib, got)) > cost


# ----------------------------------------------------------- canonical codes

def test_canonical_codes_rfc1951_example(oracle_lib):
    d = {}
    for line in open(os.path.join(GOLD, "rfc1951_canonical.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, *v = line.split()
            d[k] = v
    L = int(d["L"][0])
    lengths = [int(v) for v in d["lengths"]]
    codes = oracle.canonical_codes(lengths, L)
    for s, expect in enumerate(d["codes"]):
        assert format(int(codes[s]), f"0{lengths[s]}b") == expect
    sp = spec.canonical(dict(enumerate(lengths)))
    for s, expect in enumerate(d["codes"]):
        assert format(sp[s][0], f"0{sp[s][1]}b") == expect


def test_canonical_codes_prefix_free_and_ordered(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(50):
        n = int(rng.integers(2, 257))
        freq = rng.integers(1, 5000, size=n)
        lens = oracle.package_merge(freq, 11)[:n]
        codes = oracle.canonical_codes(lens, 11)[:n]
        words = [format(int(c), f"0{int(l)}b") for c, l in zip(codes, lens)]
        for a, b in itertools.combinations(words, 2):
            assert not a.startswith(b) and not b.startswith(a)
        order = sorted(range(n), key=lambda s: (int(lens[s]), s))
        left = [int(codes[s]) << (11 - int(lens[s])) for s in order]
        assert left == sorted(left) and len(set(left)) == n


# ----------------------------------------------------------- hand-derived container

def _read_fixture(name):
    rows = [l.split("#")[0].strip() for l in open(os.path.join(GOLD, name))]
    rows = [r for r in rows if r]
    words, params, blob = None, {}, None
    for r in rows:
        k, *v = r.split()
        if k == "input":
            words = _bf16_words(v)
        elif k == "input_u8_mod3":
            n = int(v[0])
            words = np.array([0xFF if e % 3 == 0 else 0 for e in range(n)], dtype=np.uint8)
        elif k == "input_u8_fill":
            words = np.full(int(v[0]), int(v[1], 16), dtype=np.uint8)
        elif k == "set":
            data = bytes.fromhex("".join(v[1:]))
            words[int(v[0]):int(v[0]) + len(data)] = np.frombuffer(data, np.uint8)
        elif k == "set_groups":
            # set_groups W g wmod wrem steps HEX: every group q of g symbols with
            # (q mod W) mod wmod == wrem and q div W in steps holds HEX
            W, gg, wmod, wrem = (int(x) for x in v[:4])
            steps = {int(x) for x in v[4].split(",")}
            data = np.frombuffer(bytes.fromhex("".join(v[5:])), np.uint8)
            for q in range(-(-len(words) // gg)):
                if (q % W) % wmod == wrem and q // W in steps:
                    words[q * gg:q * gg + gg] = data
        elif k == "set_iota":
            words[int(v[0]):int(v[0]) + int(v[1])] = np.arange(int(v[1])) & 0xFF
        elif k == "set_fill":
            words[int(v[0]):int(v[0]) + int(v[1])] = int(v[2], 16)
        elif k == "iota":
            blob[int(v[0]):int(v[0]) + int(v[1])] = bytes(i & 0xFF for i in range(int(v[1])))
        elif k == "fill":
            blob[int(v[0]):int(v[0]) + int(v[1])] = bytes([int(v[2], 16)]) * int(v[1])
        elif k == "params":
            for kv in v:
                a, b = kv.split("=")
                params[a] = tuple(int(x) for x in b.split(",")) if "," in b else int(b)
        elif k == "size":
            blob = bytearray(int(v[0]))
        elif k == "rep":
            # rep OFF COUNT HEX: HEX written COUNT times from OFF
            off, count = int(v[0]), int(v[1])
            data = bytes.fromhex("".join(v[2:])) * count
            blob[off:off + len(data)] = data
        elif k == "at":
            off = int(v[0])
            data = bytes.fromhex("".join(v[1:]))
            blob[off:off + len(data)] = data
    if not isinstance(params["policy"], tuple):
        params["policy"] = (params["policy"],)
    return words, params, bytes(blob)


@pytest.mark.parametrize("name", ["tiny_bf16_container.txt", "tiny_u8_rounds.txt", "tiny_u8_zg.txt",
                                  "tiny_u8_probe.txt", "tiny_bf16_exp.txt", "tiny_u8_lanegroups.txt",
                                  "tiny_u8_zg_lanegroups.txt"])
def test_tiny_containers_match_hand_derivation(oracle_lib, name):
    words, p, expect = _read_fixture(name)
    kw = dict(chunk_bytes=p["chunk_bytes"], S=p["S"], g=p["g"], L=p["L"], policy=p["policy"], skip=p.get("skip", 0),
              exp=bool(p.get("exp", 0)))
    c = oracle.compress(words, p["dtype"], **kw)
    assert c.tobytes() == expect
    assert spec.compress(words, p["dtype"], **kw) == expect
    assert np.array_equal(oracle.decompress(np.frombuffer(expect, np.uint8)), words.view(np.uint8))
    assert np.array_equal(spec.decompress(expect), words.view(np.uint8))


# ----------------------------------------------------------- round trip + agreement

SPECIAL_FP32 = np.array([0x7F800000, 0xFF800000, 0x7FC00001, 0xFFFFFFFF, 0x80000000, 0x00000001, 0x007FFFFF,
                         0x00000000, 0x3F800000], dtype=np.uint32)


@pytest.mark.parametrize("dtype", [oracle.BF16, oracle.FP16, oracle.FP32, oracle.FP8_E4M3, oracle.U8])
@pytest.mark.parametrize("n_extra", [0, 1, 37])
def test_roundtrip_and_spec_agreement(oracle_lib, dtype, n_extra):
    B = oracle.WIDTH[dtype]
    chunk = 1024
    E = chunk // B
    n = 3 * E + n_extra
    g = torch.Generator().manual_seed(dtype * 100 + n_extra)
    raw = (torch.randn(n * B // 2 + 1, generator=g) * 0.02).to(torch.bfloat16).view(torch.uint8)[: n * B].numpy()
    raw = raw.copy()
    if dtype == oracle.FP32:  # sprinkle NaN / Inf / -0 / denormals (opaque bytes)
        w = raw.view(np.uint32)
        w[: len(SPECIAL_FP32)] = SPECIAL_FP32
    for policy in [(oracle.AUTO,) * 4, (oracle.HUF,) * 4, (oracle.RAW, oracle.HUF, oracle.AUTO, oracle.HUF)]:
        for S, gg in [(64, 4), (16, 2), (128, 8), (2, 2)]:
            c = oracle.compress(raw, dtype, chunk_bytes=chunk, S=S, g=gg, policy=policy[:B])
            assert np.array_equal(oracle.decompress(c), raw)
            assert spec.compress(raw, dtype, chunk_bytes=chunk, S=S, g=gg, policy=policy[:B]) == c.tobytes()
            assert np.array_equal(spec.decompress(c.tobytes()), raw)


def test_empty_tensor(oracle_lib):
    c = oracle.compress(np.zeros(0, np.uint8), oracle.BF16)
    assert c.size == 64 and oracle.header(c)["n_chunks"] == 0
    assert oracle.decompress(c).size == 0


def test_threads_do_not_change_bytes(oracle_lib):
    x = workloads.bf16_normal(200_000, seed=3)
    a = oracle.compress(x, oracle.BF16, chunk_bytes=16384, nthreads=1)
    b = oracle.compress(x, oracle.BF16, chunk_bytes=16384, nthreads=8)
    assert np.array_equal(a, b)
    assert np.array_equal(oracle.decompress(a, nthreads=4), oracle.as_bytes(x))


# ----------------------------------------------------------- modes and sizes

def test_uniform_random_is_raw_and_constant_is_rle(oracle_lib):
    rng = np.random.default_rng(0)
    u = rng.integers(0, 256, size=4 * 65536, dtype=np.uint8)
    c = oracle.compress(u, oracle.FP32, chunk_bytes=65536)
    h = oracle.header(c)
    for ch in range(h["n_chunks"]):
        for k in range(4):
            assert oracle.entry(c, ch, k)[2] == oracle.MODE_RAW
    z = np.full(4 * 65536, 0x3C, np.uint8)
    c = oracle.compress(z, oracle.FP32, chunk_bytes=65536, policy=(oracle.HUF,) * 4)
    assert c.size == oracle.payload_base(4, 4) == 384
    for ch in range(4):
        for k in range(4):
            _, nb, mode, rle = oracle.entry(c, ch, k)
            assert (mode, nb, rle) == (oracle.MODE_RLE, 0, 0x3C)
    assert np.array_equal(oracle.decompress(c), z)


def test_no_expansion_under_auto(oracle_lib):
    """AUTO never stores more than raw: container <= n*B + header + map + alignment."""
    rng = np.random.default_rng(1)
    for dtype in (oracle.BF16, oracle.FP32, oracle.FP8_E4M3):
        B = oracle.WIDTH[dtype]
        u = rng.integers(0, 256, size=B * 50_000, dtype=np.uint8)
        c = oracle.compress(u, dtype, chunk_bytes=4096)
        nc = oracle.header(c)["n_chunks"]
        assert c.size <= u.size + oracle.payload_base(nc, B) + (oracle.PAY_ALIGN - 1) * nc * B


def test_auto_threshold_is_strict(oracle_lib):
    """AUTO keeps HUF iff the Huffman payload is strictly smaller than raw.
    The HUF-forced payload of each stream also sits between its entropy-coded
    bit count and that plus the word padding (<= 2 words per sub-stream)."""
    x = workloads.fp32_rows(64, 8192, seed=1)
    S = 256
    auto = oracle.compress(x, oracle.FP32, chunk_bytes=262144, S=S)
    huf = oracle.compress(x, oracle.FP32, chunk_bytes=262144, S=S, policy=(oracle.HUF,) * 4)
    raw = oracle.as_bytes(x).reshape(-1, 4)
    E = 65536
    W = E // S
    head = (128 + 4 * ((W + 63) // 64) + 15) // 16 * 16
    seen = set()
    for ch in range(oracle.header(auto)["n_chunks"]):
        for k in range(4):
            s = raw[ch * E:(ch + 1) * E, 3 - k]
            f = np.bincount(s, minlength=256)
            T = int((f * oracle.package_merge(f, 11).astype(np.int64)).sum())
            _, nb_h, mode_h, _ = oracle.entry(huf, ch, k)
            _, nb_a, mode_a, _ = oracle.entry(auto, ch, k)
            assert mode_h == oracle.MODE_HUF
            assert head + (T + 7) // 8 <= nb_h <= head + (T + 7) // 8 + 8 * W
            if nb_h < E:
                assert (mode_a, nb_a) == (oracle.MODE_HUF, nb_h)
            else:
                assert (mode_a, nb_a) == (oracle.MODE_RAW, E)
            seen.add(mode_a)
    assert seen == {oracle.MODE_HUF, oracle.MODE_RAW}


def test_entropy_bounds(oracle_lib):
    """Shannon: T >= m*H; and T < m*(H+1) when the unrestricted depth <= L."""
    x = workloads.bf16_normal(131072 * 4, seed=0)
    raw = oracle.as_bytes(x).reshape(-1, 2)
    for ch in range(4):
        s = raw[ch * 131072:(ch + 1) * 131072, 1]
        f = np.bincount(s, minlength=256)
        p = f[f > 0] / f.sum()
        H = float(-(p * np.log2(p)).sum())
        lens = oracle.package_merge(f, 11)
        T = int((f * lens.astype(np.int64)).sum())
        m = int(f.sum())
        assert T >= m * H - 1e-6
        _, depth = _huffman_cost_and_depth([int(v) for v in f[f > 0]])
        if depth <= 11:
            assert T < m * (H + 1)
        # stream 0 of N(0, 0.02) BF16 compresses to about a third (paper §III-A)
        assert 0.25 < T / (8 * m) < 0.40


def test_bf16_size_band(oracle_lib):
    """Paper §III-A closed form: BF16 regular models compress to about 66.6%."""
    x = workloads.bf16_normal(4 * 131072, seed=0)
    c = oracle.compress(x, oracle.BF16)
    r = c.size / (x.numel() * 2)
    assert 0.62 < r < 0.70


# ----------------------------------------------------------- XOR delta

def test_xor_delta_roundtrip(oracle_lib):
    w = workloads.bf16_normal(70_000, seed=4)
    ft = workloads.finetune_delta(w, seed=5)
    c = oracle.compress(ft, oracle.BF16, base=w, chunk_bytes=16384, policy=(oracle.HUF, oracle.HUF))
    assert oracle.header(c)["flags"] & 1
    assert np.array_equal(oracle.decompress(c, base=w), oracle.as_bytes(ft))
    assert spec.compress(oracle.as_bytes(ft), oracle.BF16, base=oracle.as_bytes(w), chunk_bytes=16384,
                         policy=(1, 1)) == c.tobytes()
    # x XOR x = 0: every stream collapses to RLE 0
    c0 = oracle.compress(w, oracle.BF16, base=w, chunk_bytes=16384, policy=(oracle.HUF, oracle.HUF))
    nc = oracle.header(c0)["n_chunks"]
    assert c0.size == oracle.payload_base(nc, 2)
    with pytest.raises(oracle.OracleError):
        oracle.decompress(c)  # a delta container needs its base


# ----------------------------------------------------------- corruption

def _container():
    x = workloads.bf16_normal(3 * 8192 + 5, seed=9)
    return oracle.compress(x, oracle.BF16, chunk_bytes=16384, S=512), x


def test_corrupt_header_and_map_rejected(oracle_lib):
    c, x = _container()
    base = oracle.decompress(c)
    assert np.array_equal(base, oracle.as_bytes(x))
    nc = oracle.header(c)["n_chunks"]
    bad_positions = [0, 4, 6, 7, 16, 20, 22, 23, 24, 28, 32, 50]          # header fields
    for e in range(nc * 2):                                                # map: offset, bytes, mode
        bad_positions += [64 + 16 * e, 64 + 16 * e + 8, 64 + 16 * e + 12, 64 + 16 * e + 14]
    for pos in bad_positions:
        d = c.copy()
        d[pos] ^= 0x01 if pos not in (6, 7) else 0x04
        with pytest.raises(oracle.OracleError) as ei:
            oracle.decompress(d, out_bytes=x.numel() * 2)
        assert ei.value.code in (oracle.E_FORMAT, oracle.E_CORRUPT, oracle.E_NOSPACE, oracle.E_INVAL)


def test_corrupt_huffman_tables_rejected(oracle_lib):
    c, x = _container()
    nc = oracle.header(c)["n_chunks"]
    assert oracle.entry(c, 0, 0)[2] == oracle.MODE_HUF
    for ch in range(nc):
        off, nb, mode, _ = oracle.entry(c, ch, 0)
        if mode != oracle.MODE_HUF:   # the 5-element tail chunk is stored raw
            continue
        # a code length changed: Kraft sum no longer one
        d = c.copy()
        i = next(i for i in range(128) if d[off + i] & 15)
        d[off + i] = (d[off + i] & 0xF0) | ((d[off + i] & 15) % 11 + 1)
        with pytest.raises(oracle.OracleError) as ei:
            oracle.decompress(d)
        assert ei.value.code == oracle.E_CORRUPT
        # a sub-stream length changed: the bit count no longer matches
        d = c.copy()
        d[off + 128] ^= 0x01
        with pytest.raises(oracle.OracleError) as ei:
            oracle.decompress(d)
        assert ei.value.code == oracle.E_CORRUPT


def test_truncated_and_small_output_rejected(oracle_lib):
    c, x = _container()
    for cut in (0, 10, 63, 64, c.size // 2, c.size - 1):
        with pytest.raises(oracle.OracleError):
            oracle.decompress(c[:cut].copy(), out_bytes=x.numel() * 2)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.decompress(c, out_bytes=x.numel() * 2 - 1)
    assert ei.value.code == oracle.E_NOSPACE


def test_invalid_params_rejected(oracle_lib):
    x = np.zeros(100, np.uint16)
    for kw in [dict(chunk_bytes=1000), dict(chunk_bytes=128), dict(S=3), dict(g=3), dict(S=2, g=4),
               dict(L=7), dict(L=12), dict(S=8192), dict(g=16, S=64), dict(g=1),
               dict(chunk_bytes=1 << 20, S=64)]:
        with pytest.raises(oracle.OracleError) as ei:
            oracle.compress(x, oracle.BF16, **kw)
        assert ei.value.code == oracle.E_INVAL


# ----------------------------------------------------------- ZG (zero-aware delta coding)

def _zg_closed_form(s, g, L):
    """Fill value, bitmap bytes and coded bit count of one stream, computed
    with numpy from the definition: z = most frequent value (smallest on
    ties), a group is marked when it holds any value other than z, and the
    symbols of marked groups are coded with the optimal length-limited code
    of their own histogram."""
    f = np.bincount(s, minlength=256)
    z = int(np.flatnonzero(f == f.max())[0])
    G = -(-len(s) // g)
    pad = np.full(G * g, z, np.uint8)
    pad[: len(s)] = s
    marked = (pad.reshape(G, g) != z).any(axis=1)
    bitmap = np.packbits(marked, bitorder="little").tobytes()
    coded = pad.reshape(G, g)[marked].reshape(-1)
    if marked.any() and marked[-1] and len(s) % g:   # the padding is not coded
        coded = coded[: len(coded) - (G * g - len(s))]
    f2 = np.bincount(coded, minlength=256)
    T2 = int((f2 * oracle.package_merge(f2, L).astype(np.int64)).sum()) if (f2 > 0).sum() >= 2 else None
    return z, bitmap, T2, (f2 > 0).sum()


def test_zg_matches_closed_form_and_auto_picks_smallest(oracle_lib):
    """On XOR deltas of a sparse fine-tune (paper §IV-B), forced-ZG streams
    carry z in the map and the bitmap given by the definition, their size lies
    between the coded bit count and that plus the word padding, and AUTO keeps
    the smallest of RAW, HUF and ZG (ZG only when z fills half the stream)."""
    w = workloads.bf16_normal(4 * 8192 + 37, seed=21)
    ft = workloads.finetune_delta(w, seed=22)
    raw = oracle.as_bytes(ft) ^ oracle.as_bytes(w)
    S, g, L, chunk = 256, 4, 11, 16384
    kw = dict(chunk_bytes=chunk, S=S, g=g, L=L)
    zg = oracle.compress(raw, oracle.BF16, policy=(oracle.ZG,) * 2, **kw)
    huf = oracle.compress(raw, oracle.BF16, policy=(oracle.HUF,) * 2, **kw)
    auto = oracle.compress(raw, oracle.BF16, **kw)
    assert np.array_equal(oracle.decompress(zg), raw)
    assert np.array_equal(oracle.decompress(auto), raw)
    pairs = raw.reshape(-1, 2)
    E = chunk // 2
    picked = set()
    for ch in range(oracle.header(zg)["n_chunks"]):
        for k in range(2):
            s = pairs[ch * E:(ch + 1) * E, 1 - k]
            m = len(s)
            z, bitmap, T2, d2 = _zg_closed_form(s, g, L)
            off, nb, mode, val = oracle.entry(zg, ch, k)
            if len(np.unique(s)) == 1:
                assert mode == oracle.MODE_RLE
                continue
            if d2 < 2:
                assert mode == oracle.MODE_HUF
                continue
            assert (mode, val) == (oracle.MODE_ZG, z)
            W = -(-m // S)
            H = (128 + 4 * ((W + 63) // 64) + 15) // 16 * 16
            BM = (len(bitmap) + 15) // 16 * 16
            assert bytes(zg[off + H: off + H + len(bitmap)]) == bitmap
            assert not zg[off + H + len(bitmap): off + H + BM].any()
            assert H + BM + (T2 + 7) // 8 <= nb <= H + BM + (T2 + 7) // 8 + 8 * W
            _, nb_h, mode_h, _ = oracle.entry(huf, ch, k)
            assert mode_h == oracle.MODE_HUF
            _, nb_a, mode_a, val_a = oracle.entry(auto, ch, k)
            f = np.bincount(s, minlength=256)
            best = min([(m, 0, oracle.MODE_RAW), (nb_h, 1, oracle.MODE_HUF)]
                       + ([(nb, 2, oracle.MODE_ZG)] if 2 * f[z] >= m else []))
            assert (nb_a, mode_a) == (best[0], best[2])
            picked.add(mode_a)
    assert oracle.MODE_ZG in picked   # the sparse low byte of the delta
    # header bit 1 says whether the map holds ZG entries
    assert oracle.header(zg)["flags"] == 2 and oracle.header(auto)["flags"] == 2
    assert oracle.header(huf)["flags"] == 0


def test_zg_needs_half_the_stream(oracle_lib):
    """AUTO never picks ZG when the most frequent value fills less than half
    of the stream, even where ZG would be smaller; at exactly half it may."""
    rng = np.random.default_rng(5)
    m = 8192
    for zeros, allowed in [(m // 2 - 1, False), (m // 2, True)]:
        s = rng.integers(1, 3, size=m, dtype=np.uint8)
        s[:zeros] = 0   # whole groups of zeros first: ZG would code only the rest
        kw = dict(chunk_bytes=m, g=8)
        nz = oracle.entry(oracle.compress(s, oracle.U8, policy=(oracle.ZG,), **kw), 0, 0)[1]
        nh = oracle.entry(oracle.compress(s, oracle.U8, policy=(oracle.HUF,), **kw), 0, 0)[1]
        assert nz < nh < m
        mode = oracle.entry(oracle.compress(s, oracle.U8, **kw), 0, 0)[2]
        assert mode == (oracle.MODE_ZG if allowed else oracle.MODE_HUF)


def test_corrupt_zg_rejected(oracle_lib):
    words, p, blob = _read_fixture("tiny_u8_zg.txt")
    good = np.frombuffer(blob, np.uint8).copy()
    assert np.array_equal(oracle.decompress(good), words)
    for pos, val in [(272 + 2, 0x01),    # a bitmap bit past the last group
                     (272, 0x42 | 0x01),  # one more marked group: words run short
                     (272, 0x40),         # one fewer marked group: words left over
                     (64 + 8, 0x20),      # payload shorter than head + bitmap
                     (24, 0x00)]:         # a ZG entry without the header's ZG flag
        d = good.copy()
        d[pos] = val
        with pytest.raises(oracle.OracleError) as ei:
            oracle.decompress(d)
        assert ei.value.code in (oracle.E_CORRUPT, oracle.E_FORMAT)


# ----------------------------------------------------------- compressibility probing

@pytest.mark.parametrize("K", [1, 3, 7])
def test_probing_follows_its_definition(oracle_lib, K):
    """Probe interval K (paper §III-B, "Identifying compressibility"): every
    entry equals the one written without probing, except under AUTO in a
    chunk that follows a probe chunk (c mod (K+1) != 0) whose entry for that
    byte group is RAW: there the group is RAW.  Checked on FP32 rows whose
    low bytes are incompressible and a BF16 tensor mixing raw-like and
    compressible chunks (random, then normal, then zero), with a ragged
    tail."""
    E = 1024
    rows = workloads.fp32_rows(6, 1024 + 3, seed=2).reshape(-1)
    mixed = torch.cat([torch.randint(0, 65536, (5 * E,), generator=torch.Generator().manual_seed(4),
                                     dtype=torch.int32).to(torch.int16).view(torch.bfloat16),
                       workloads.bf16_normal(3 * E, seed=3),
                       torch.zeros(2 * E + 17, dtype=torch.bfloat16)])
    for x, dt in [(rows, oracle.FP32), (mixed, oracle.BF16)]:
        B = oracle.WIDTH[dt]
        kw = dict(chunk_bytes=E * B, S=64, g=4)
        pol = [oracle.AUTO, oracle.AUTO, oracle.HUF, oracle.AUTO][:B]
        ref = oracle.compress(x, dt, policy=pol, **kw)
        got = oracle.compress(x, dt, policy=pol, skip=K, **kw)
        assert oracle.header(got)["skip"] == K and oracle.header(ref)["skip"] == 0
        assert np.array_equal(oracle.decompress(got), oracle.as_bytes(x))
        assert spec.compress(oracle.as_bytes(x), dt, policy=pol, skip=K, **kw) == got.tobytes()
        nc = oracle.header(ref)["n_chunks"]
        skipped = 0
        for c in range(nc):
            for k in range(B):
                r = oracle.entry(ref, c, k)
                gmode = oracle.entry(got, c, k)[2:]
                probe = c - c % (K + 1)
                if pol[k] == oracle.AUTO and probe != c and oracle.entry(got, probe, k)[2] == oracle.MODE_RAW:
                    assert gmode == (oracle.MODE_RAW, 0)
                    skipped += r[2] != oracle.MODE_RAW
                else:
                    assert gmode == r[2:]
                    if r[2] != oracle.MODE_RLE:
                        assert oracle.entry(got, c, k)[1] == r[1]
        if dt == oracle.BF16:
            assert skipped > 0   # compressible chunks after a raw probe stay raw until the next probe


# ----------------------------------------------------------- exponent extraction

def test_exponent_extraction_groups_are_the_fields(oracle_lib):
    """With exponent extraction the raw byte groups are the IEEE fields,
    computed here with numpy from the bit layout: BF16 group 0 = exponent,
    group 1 = sign << 7 | fraction; FP32 group 0 = exponent, group 1 =
    sign << 7 | fraction[22:16], groups 2, 3 = fraction bytes."""
    xb = workloads.bf16_normal(3000, seed=8)
    w = xb.view(torch.int16).numpy().view(np.uint16).astype(np.uint32)
    c = oracle.compress(xb, oracle.BF16, chunk_bytes=1 << 16, policy=(oracle.RAW,) * 2, exp=True)
    groups = [(w >> 7) & 0xFF, ((w >> 15) << 7) | (w & 0x7F)]
    for k in range(2):
        off, nb, mode, _ = oracle.entry(c, 0, k)
        assert mode == oracle.MODE_RAW and np.array_equal(c[off:off + nb], groups[k].astype(np.uint8))
    xf = workloads.fp32_rows(3, 1000, seed=9).reshape(-1)
    w = xf.numpy().view(np.uint32).astype(np.uint64)
    c = oracle.compress(xf, oracle.FP32, chunk_bytes=1 << 16, policy=(oracle.RAW,) * 4, exp=True)
    groups = [(w >> 23) & 0xFF, ((w >> 31) << 7) | ((w >> 16) & 0x7F), (w >> 8) & 0xFF, w & 0xFF]
    for k in range(4):
        off, nb, mode, _ = oracle.entry(c, 0, k)
        assert np.array_equal(c[off:off + nb], groups[k].astype(np.uint8)), k
    assert np.array_equal(oracle.decompress(c), oracle.as_bytes(xf))


def test_exponent_extraction_sizes_follow_the_entropy(oracle_lib):
    """On N(0, 0.02) BF16 weights the exponent group's empirical entropy is
    below that of the sign + 7 exponent bits byte; the Huffman payloads of
    both stay within [entropy bound, entropy + 1 bit + padding], so the
    extracted container is smaller by about the entropy difference."""
    x = workloads.bf16_normal(4 * 131072, seed=10)
    w = x.view(torch.int16).numpy().view(np.uint16)

    def H(b):
        f = np.bincount(b, minlength=256)
        p = f[f > 0] / f.sum()
        return float(-(p * np.log2(p)).sum())

    h_plain, h_exp = H((w >> 8).astype(np.uint8)), H(((w >> 7) & 0xFF).astype(np.uint8))
    assert h_exp < h_plain - 0.05
    pol = (oracle.HUF, oracle.RAW)
    a = oracle.compress(x, oracle.BF16, policy=pol)
    b = oracle.compress(x, oracle.BF16, policy=pol, exp=True)
    m = x.numel()
    saved = sum(oracle.entry(a, c, 0)[1] - oracle.entry(b, c, 0)[1] for c in range(4))
    assert abs(saved - m * (h_plain - h_exp) / 8) < 0.02 * m
    assert np.array_equal(oracle.decompress(b), oracle.as_bytes(x))
    assert spec.compress(oracle.as_bytes(x)[: 2 * 4096], oracle.BF16, chunk_bytes=4096, S=64, exp=True) == \
        oracle.compress(oracle.as_bytes(x)[: 2 * 4096], oracle.BF16, chunk_bytes=4096, S=64, exp=True).tobytes()


def test_exponent_extraction_only_for_bf16_fp32(oracle_lib):
    with pytest.raises(oracle.OracleError):
        oracle.compress(np.zeros(16, np.uint8), oracle.FP8_E4M3, exp=True)
    with pytest.raises(oracle.OracleError):
        oracle.compress(np.zeros(16, np.uint16), oracle.FP16, exp=True)
    c = oracle.compress(np.zeros(16, np.uint8), oracle.U8)
    d = c.copy()
    d[24] |= 4   # the flag on a U8 container
    with pytest.raises(oracle.OracleError) as ei:
        oracle.decompress(d)
    assert ei.value.code == oracle.E_FORMAT
