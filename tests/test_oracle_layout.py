"""Pins for the two layers of the oracle's Huffman payload, each checked
against something other than the oracle's own code:

* the coding (one bit string per sub-stream: canonical codes, most
  significant bit first, packed LSB-first), against a character-string build
  written out here, at full chunk size;
* the word layout (the order in which a lock-step decoder of 64 lanes takes
  the 32-bit words), by reading oracle payloads back with the layout's
  declarative definition: sort the (step, pair, lane) decode events, and let a
  lane holding fewer than 2L bits take its next word before its event.  Every
  lane's words must then spell its sub-stream's bit string followed by zero
  bits, and every stored word must be taken exactly once.

The hand-derived containers (``tests/golden/tiny_u8_lanegroups.txt``,
``tiny_u8_zg_lanegroups.txt``) pin the same layout at fixed bytes."""
import struct

import numpy as np
import pytest

import oracle
from paper_2411_05239_amd import workloads

LANES = 64


def _stream(raw: np.ndarray, B: int, k: int) -> np.ndarray:
    """Byte group k = byte B-1-k of each little-endian word (numpy view)."""
    return np.ascontiguousarray(raw.reshape(-1, B)[:, B - 1 - k])


def _groups_of(m: int, S: int, g: int, w: int, flags) -> list[range]:
    W, G = -(-m // S), -(-m // g)
    return [range(q * g, min(q * g + g, m)) for q in range(w, G, W) if flags is None or flags[q]]


def _expected_bits(sym, lengths, codes, groups) -> str:
    """The sub-stream's codes as a string of '0'/'1', first bit first."""
    return "".join(format(int(codes[sym[e]]), f"0{int(lengths[sym[e]])}b") for r in groups for e in r)


def _bits_of_bytes(b: bytes, n: int) -> str:
    return "".join(format(x, "08b")[::-1] for x in b)[:n]


def _bits_of_words(ws) -> str:
    return "".join(format(w, "032b")[::-1] for w in ws)


def _payload_parts(p: bytes, m: int, S: int, g: int, zg: bool):
    """(lengths, per-lane-group word counts, flags or None, words)."""
    lengths = np.zeros(256, dtype=np.int64)
    for i in range(128):
        lengths[2 * i], lengths[2 * i + 1] = p[i] & 15, p[i] >> 4
    W = -(-m // S)
    NG = -(-W // LANES)
    counts = struct.unpack(f"<{NG}I", p[128:128 + 4 * NG])
    H = -(-(128 + 4 * NG) // 16) * 16
    flags, start = None, H
    if zg:
        G = -(-m // g)
        start = H + -(-(-(-G // 8)) // 16) * 16
        flags = [(p[H + q // 8] >> (q % 8)) & 1 for q in range(G)]
    words = struct.unpack(f"<{(len(p) - start) // 4}I", p[start:])
    return lengths, counts, flags, words


def _deinterleave(words, counts, sym, m, S, g, L, lengths, flags) -> dict[int, list[int]]:
    """The words each sub-stream takes, by the layout's definition."""
    W, G = -(-m // S), -(-m // g)
    pos, taken = 0, {}
    for j in range(len(counts)):
        events = []
        for lane in range(min(LANES, W - LANES * j)):
            for step, q in enumerate(range(LANES * j + lane, G, W)):
                if flags is not None and not flags[q]:
                    continue
                grp = sym[q * g:min(q * g + g, m)]
                for pr in range(0, len(grp), 2):
                    events.append((step, pr // 2, lane, int(sum(lengths[s] for s in grp[pr:pr + 2]))))
        events.sort()
        buffered = [0] * LANES
        got = [[] for _ in range(LANES)]
        for _, _, lane, bits in events:
            if buffered[lane] < 2 * L:
                assert pos < len(words), "a lane asks for a word the payload does not hold"
                got[lane].append(words[pos])
                pos += 1
                buffered[lane] += 32
            buffered[lane] -= bits
        assert pos == sum(counts[:j + 1]), f"lane group {j}: word count differs from the events' takes"
        for lane in range(min(LANES, W - LANES * j)):
            taken[LANES * j + lane] = got[lane]
    assert pos == len(words), "words left over after the last event"
    return taken


def _check_container(c: np.ndarray, raw: np.ndarray, B: int, chunk_bytes: int, S: int, g: int, L: int) -> int:
    """Read back every HUF / ZG entry of an oracle container; returns how many."""
    E = chunk_bytes // B
    n = raw.size // B
    checked = 0
    for ch in range(-(-n // E)):
        part = raw[ch * E * B:min(n, (ch + 1) * E) * B]
        m = part.size // B
        for k in range(B):
            off, nbytes, mode, _ = oracle.entry(c, ch, k)
            if mode not in (oracle.MODE_HUF, oracle.MODE_ZG):
                continue
            sym = _stream(part, B, k)
            p = c[off:off + nbytes].tobytes()
            lengths, counts, flags, words = _payload_parts(p, m, S, g, mode == oracle.MODE_ZG)
            codes = oracle.canonical_codes(lengths, L)
            taken = _deinterleave(words, counts, sym, m, S, g, L, lengths, flags)
            for w, ws in taken.items():
                want = _expected_bits(sym, lengths, codes, _groups_of(m, S, g, w, flags))
                have = _bits_of_words(ws)
                assert len(have) >= len(want) and have[:len(want)] == want, f"chunk {ch} stream {k} sub-stream {w}"
                assert set(have[len(want):]) <= {"0"}, "bits past the last code must be zero"
                assert len(ws) <= -(-(len(want) + 2 * L) // 32), "more words than the refill rule allows"
            checked += 1
    return checked


# ----------------------------------------------------------- the coding

@pytest.mark.parametrize("case", ["bf16_s0_full_chunk", "fp32_s1_full_chunk", "zg_delta_g8"])
def test_substream_bits_full_chunk(oracle_lib, case):
    """orc_substream_bits against a string build of the same codes, on every
    sub-stream of a full 256 KiB chunk's byte group."""
    L = 11
    if case == "bf16_s0_full_chunk":
        raw = oracle.as_bytes(workloads.bf16_normal(131072, seed=7))
        sym, S, g, flags = _stream(raw, 2, 0), 512, 4, None
    elif case == "fp32_s1_full_chunk":
        raw = oracle.as_bytes(workloads.fp32_rows(8, 8192, seed=3))
        sym, S, g, flags = _stream(raw, 4, 1), 256, 4, None
    else:
        base = workloads.bf16_normal(131072, seed=8)
        ft = workloads.finetune_delta(base, seed=9)
        raw = oracle.as_bytes(ft) ^ oracle.as_bytes(base)
        sym, S, g = _stream(raw, 2, 1), 512, 8
        G = -(-sym.size // g)
        flags = np.array([np.any(sym[q * g:q * g + g] != 0) for q in range(G)], dtype=np.uint8)
    m = sym.size
    if flags is None:
        hist = np.bincount(sym, minlength=256)
    else:
        hist = np.bincount(np.concatenate([sym[q * g:q * g + g] for q in np.flatnonzero(flags)]), minlength=256)
    lengths = oracle.package_merge(hist, L)
    codes = oracle.canonical_codes(lengths, L)
    W = -(-m // S)
    assert W >= 128
    total = 0
    for w in range(W):
        packed, nbits = oracle.substream_bits(sym, S, g, L, lengths, w, flags)
        want = _expected_bits(sym, lengths, codes, _groups_of(m, S, g, w, flags))
        assert nbits == len(want), f"sub-stream {w}"
        assert _bits_of_bytes(packed, nbits) == want, f"sub-stream {w}"
        total += nbits
    assert total == int(sum(int(hist[s]) * int(lengths[s]) for s in range(256)))


# ----------------------------------------------------------- the layout

@pytest.mark.parametrize("dtype,n,chunk_bytes,S,g,L,policy", [
    (oracle.BF16, 131072 + 4099, 262144, 512, 4, 11, (oracle.HUF, oracle.HUF)),        # W = 256: 4 lane groups
    (oracle.BF16, 3 * 2048 + 77, 4096, 8, 2, 8, (oracle.HUF, oracle.HUF)),           # W = 256, ragged tail
    (oracle.FP32, 2 * 4096 + 5, 16384, 32, 8, 11, (oracle.HUF,) * 4),                # W = 128
    (oracle.U8, 6000, 8192, 64, 4, 9, (oracle.HUF,)),                               # W = 94: partial lane group 1
    (oracle.U8, 9000, 8192, 16, 8, 10, (oracle.ZG,)),                               # W = 512, ZG
])
def test_payloads_read_back_by_the_layout_definition(oracle_lib, dtype, n, chunk_bytes, S, g, L, policy):
    B = oracle.WIDTH[dtype]
    if dtype == oracle.U8:
        rng = np.random.default_rng(n)
        raw = np.where(rng.random(n) < 0.7, 0, rng.geometric(0.2, n) % 256).astype(np.uint8)
    else:
        raw = oracle.as_bytes(workloads.bf16_normal(n * B // 2, seed=n))
    c = oracle.compress(raw, dtype, chunk_bytes=chunk_bytes, S=S, g=g, L=L, policy=policy)
    assert _check_container(c, raw, B, chunk_bytes, S, g, L) > 0


def test_delta_payloads_read_back_by_the_layout_definition(oracle_lib):
    """A BF16 XOR delta under AUTO: ZG and HUF entries with W = 256."""
    base = workloads.bf16_normal(3 * 131072 + 333, seed=21)
    ft = workloads.finetune_delta(base, seed=22)
    raw = oracle.as_bytes(ft) ^ oracle.as_bytes(base)
    c = oracle.compress(ft, oracle.BF16, base=base)
    modes = {oracle.entry(c, ch, k)[2] for ch in range(4) for k in range(2)}
    assert oracle.MODE_ZG in modes
    assert _check_container(c, raw, 2, 262144, 512, 4, 11) > 0


@pytest.mark.parametrize("seed", range(12))
def test_random_payloads_read_back_by_the_layout_definition(oracle_lib, seed):
    """Random shapes: B, chunk size, S, g, L, policy, lengths around chunk
    and lane-group boundaries."""
    rng = np.random.default_rng(1000 + seed)
    dtype = [oracle.BF16, oracle.FP16, oracle.FP32, oracle.FP8_E4M3, oracle.U8][seed % 5]
    B = oracle.WIDTH[dtype]
    chunk_bytes = int(rng.choice([1024, 2048, 4096, 8192]))
    E = chunk_bytes // B
    g = int(rng.choice([2, 4, 8]))
    S = int(rng.choice([s for s in (2, 4, 8, 16, 32) if s >= g and E // s <= 4096]))
    L = int(rng.integers(8, 12))
    n = int(rng.integers(1, 3) * E + rng.integers(-3, 4) * S + rng.integers(0, 7))
    pol = tuple(int(rng.choice([oracle.HUF, oracle.ZG, oracle.AUTO])) for _ in range(B))
    v = rng.standard_normal(n * B) * 0.02
    raw = np.where(rng.random(n * B) < 0.5, 0, (np.abs(v) * 4000).astype(np.int64) % 256).astype(np.uint8)
    c = oracle.compress(raw, dtype, chunk_bytes=chunk_bytes, S=S, g=g, L=L, policy=pol)
    _check_container(c, raw, B, chunk_bytes, S, g, L)
    assert np.array_equal(oracle.decompress(c), raw)
