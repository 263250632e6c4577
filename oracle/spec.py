"""Pure-Python specification of the ZipNN codec -- TEST INFRASTRUCTURE ONLY.

Written separately from ``zipnn_oracle.c`` (different formulations of every
step) so that the two can check each other byte for byte on tiny inputs.  Far
too slow for anything above ~10^5 symbols.

Steps (ZipNN, arXiv 2411.05239):
  split    -- byte grouping, exponent byte first (§III-A, §III-B): a numpy
              view of the words, byte order reversed, transposed;
  lengths  -- optimal length-limited prefix code, package-merge written as the
              "coin collector" with explicit symbol multisets carried by every
              package (Larmore & Hirschberg 1990);
  codes    -- canonical codes by walking the symbols in (length, symbol) order
              (code_{i+1} = (code_i + 1) << (l_{i+1} - l_i)), equivalent to
              RFC 1951 §3.2.2;
  modes    -- RAW / RLE / HUF per byte-group (§III-B, §V-A);
  layout   -- 64-byte header, 16-byte map entries, 16-byte aligned payloads
              (the container described in ``zipnn_oracle.h``).
"""
from __future__ import annotations

import struct

import numpy as np

WIDTH = {1: 2, 2: 2, 3: 4, 4: 1, 5: 1}
AUTO, HUF, RAW = 0, 1, 2
MODE_RAW, MODE_HUF, MODE_RLE = 0, 1, 2


class SpecError(ValueError):
    pass


def split(words: np.ndarray, B: int) -> list[np.ndarray]:
    """Stream k = byte B-1-k of each little-endian word."""
    a = np.ascontiguousarray(words).view(np.uint8).reshape(-1, B)
    return [a[:, B - 1 - k].copy() for k in range(B)]


def merge(streams: list[np.ndarray], B: int) -> np.ndarray:
    m = len(streams[0])
    a = np.zeros((m, B), dtype=np.uint8)
    for k in range(B):
        a[:, B - 1 - k] = streams[k]
    return a.reshape(-1)


def pm_lengths(freq: dict[int, int], L: int) -> dict[int, int]:
    """Coin collector: coins of denomination 2^-d for every symbol at every
    depth d = 1..L, with numismatic value f(s).  Starting from the smallest
    denomination, sort the coins, pair them into packages of the next
    denomination and add that denomination's own coins; finally take the
    2n'-2 cheapest items at denomination 1/2.  A symbol's code length is the
    number of its coins inside the chosen items.

    Every item carries the multiset of symbols it contains.  Order: weight,
    then single coins before packages, single coins by (f, symbol), packages
    in the order they were formed."""
    syms = sorted((s for s in freq if freq[s] > 0), key=lambda s: (freq[s], s))
    n = len(syms)
    if n < 2:
        return {s: 0 for s in syms}
    if n > (1 << L):
        raise SpecError("alphabet too large for L")
    coins = [(freq[s], 0, i, {s: 1}) for i, s in enumerate(syms)]   # (weight, kind, order, multiset)
    current = sorted(coins, key=lambda t: (t[0], t[1], t[2]))
    for _ in range(L - 1):
        packages = []
        for j in range(len(current) // 2):
            a, b = current[2 * j], current[2 * j + 1]
            ms = dict(a[3])
            for s, c in b[3].items():
                ms[s] = ms.get(s, 0) + c
            packages.append((a[0] + b[0], 1, j, ms))
        current = sorted(coins + packages, key=lambda t: (t[0], t[1], t[2]))
    chosen = current[: 2 * n - 2]
    lengths = {s: 0 for s in syms}
    for item in chosen:
        for s, c in item[3].items():
            lengths[s] += c
    return lengths


def canonical(lengths: dict[int, int]) -> dict[int, tuple[int, int]]:
    """symbol -> (code, length), walking symbols in (length, symbol) order."""
    order = sorted((s for s in lengths if lengths[s] > 0), key=lambda s: (lengths[s], s))
    out = {}
    code, prev = 0, lengths[order[0]]
    for i, s in enumerate(order):
        l = lengths[s]
        code = 0 if i == 0 else (code + 1) << (l - prev)
        out[s] = (code, l)
        prev = l
    return out


def _a16(x: int) -> int:
    return (x + 15) // 16 * 16


PAY_ALIGN = 128   # payloads start at multiples of 128 bytes from the container start


def _apay(x: int) -> int:
    return (x + PAY_ALIGN - 1) // PAY_ALIGN * PAY_ALIGN


def _payload_base(n_chunks: int, B: int) -> int:
    return _apay(64 + 16 * n_chunks * B) if n_chunks else 64


LANES = 64


def _substreams(m: int, S: int, g: int) -> list[list[int]]:
    """Element indices of each sub-stream: group q of g symbols -> q mod W."""
    W = -(-m // S)
    subs = [[] for _ in range(W)]
    for q in range(-(-m // g)):
        subs[q % W].extend(range(q * g, min(q * g + g, m)))
    return subs


def _request_schedule(n_syms: list[int], lens_of, L: int) -> list[list[int]]:
    """For one lane group: per round, the lanes (ascending) that take a word.
    A lane with symbols left in round r takes a word when it buffers < 2L bits,
    then consumes the code lengths of its symbols 2r and 2r+1."""
    buffered = [0] * len(n_syms)
    schedule = []
    for r in range(max((n + 1) // 2 for n in n_syms)):
        takers = []
        for lane, n in enumerate(n_syms):
            if 2 * r >= n:
                continue
            if buffered[lane] < 2 * L:
                takers.append(lane)
                buffered[lane] += 32
            buffered[lane] -= sum(lens_of(lane, t) for t in (2 * r, 2 * r + 1) if t < n)
        schedule.append(takers)
    return schedule


def encode_stream(sym: np.ndarray, S: int, g: int, L: int, policy: int) -> tuple[int, int, bytes]:
    """-> (mode, rle value, payload bytes)"""
    m = len(sym)
    if policy == RAW:
        return MODE_RAW, 0, sym.tobytes()
    counts = np.bincount(sym, minlength=256)
    present = [s for s in range(256) if counts[s]]
    if len(present) == 1:
        return MODE_RLE, present[0], b""
    lengths = pm_lengths({s: int(counts[s]) for s in present}, L)
    codes = canonical(lengths)
    subs = _substreams(m, S, g)
    W = len(subs)
    NG = -(-W // LANES)
    H = _a16(128 + 4 * NG)
    counts_out, words_out = [], []
    for j in range(NG):
        group = subs[LANES * j: LANES * j + LANES]
        # each lane's bit string (as a Python int, bit i = i-th stream bit)
        lane_words = []
        for idx in group:
            acc, nbits = 0, 0
            for e in idx:
                c, l = codes[int(sym[e])]
                for b in range(l):
                    acc |= ((c >> (l - 1 - b)) & 1) << nbits
                    nbits += 1
            lane_words.append([(acc >> (32 * k)) & 0xFFFFFFFF for k in range(nbits // 32 + 3)])
        sched = _request_schedule([len(x) for x in group], lambda lane, t: lengths[int(sym[group[lane][t]])], L)
        nxt = [0] * len(group)
        stream = []
        for takers in sched:
            for lane in takers:
                stream.append(lane_words[lane][nxt[lane]])
                nxt[lane] += 1
        counts_out.append(len(stream))
        words_out.extend(stream)
    table = bytes(lengths.get(2 * i, 0) | (lengths.get(2 * i + 1, 0) << 4) for i in range(128))
    head = table + struct.pack(f"<{NG}I", *counts_out)
    payload = head + bytes(H - len(head)) + struct.pack(f"<{len(words_out)}I", *words_out)
    if policy == AUTO and len(payload) >= m:
        return MODE_RAW, 0, sym.tobytes()
    return MODE_HUF, 0, payload


def compress(words: np.ndarray, dtype: int, *, base: np.ndarray | None = None, chunk_bytes: int = 262144,
             S: int = 512, g: int = 4, L: int = 11, policy=(AUTO, AUTO, AUTO, AUTO)) -> bytes:
    B = WIDTH[dtype]
    raw = np.ascontiguousarray(words).view(np.uint8).reshape(-1)
    if base is not None:
        raw = raw ^ np.ascontiguousarray(base).view(np.uint8).reshape(-1)
    n = raw.size // B
    E = chunk_bytes // B
    n_chunks = -(-n // E)
    entries, payloads = [], []
    for c in range(n_chunks):
        chunk = raw[c * E * B: min(n, (c + 1) * E) * B]
        for k, s in enumerate(split(chunk, B)):
            entries.append(encode_stream(s, S, g, L, policy[k]))
    payload_base = _payload_base(n_chunks, B)
    body = bytearray()
    mp = bytearray()
    for mode, rle, p in entries:
        mp += struct.pack("<QIBBH", len(body), len(p), mode, rle, 0)
        if p:
            body += p
            body += bytes(_apay(len(body)) - len(body))
    total = payload_base + len(body)
    pol = bytes(list(policy[:B]) + [0] * (4 - B))
    hdr = b"ZNN1" + struct.pack("<HBBQIHBBIIQ", 1, dtype, B, n, chunk_bytes, S, g, L,
                                1 if base is not None else 0, n_chunks, total) + pol + bytes(20)
    assert len(hdr) == 64
    return bytes(hdr + mp + bytes(payload_base - 64 - len(mp)) + body)


def decompress(blob: bytes, base: np.ndarray | None = None) -> np.ndarray:
    if blob[:4] != b"ZNN1":
        raise SpecError("magic")
    (ver, dtype, B, n, chunk_bytes, S, g, L, flags, n_chunks, total) = struct.unpack("<HBBQIHBBIIQ", blob[4:40])
    E = chunk_bytes // B
    payload_base = _payload_base(n_chunks, B)
    out = np.zeros(n * B, dtype=np.uint8)
    for c in range(n_chunks):
        m = min(n, (c + 1) * E) - c * E
        streams = []
        for k in range(B):
            off, nb, mode, rle, _ = struct.unpack("<QIBBH", blob[64 + 16 * (c * B + k): 80 + 16 * (c * B + k)])
            p = blob[payload_base + off: payload_base + off + nb]
            if mode == MODE_RAW:
                streams.append(np.frombuffer(p, dtype=np.uint8).copy())
            elif mode == MODE_RLE:
                streams.append(np.full(m, rle, dtype=np.uint8))
            else:
                streams.append(_decode_huf(p, m, S, g, L))
        out[c * E * B: (c * E + m) * B] = merge(streams, B)
    if base is not None:
        out ^= np.ascontiguousarray(base).view(np.uint8).reshape(-1)
    return out


def _decode_huf(p: bytes, m: int, S: int, g: int, L: int) -> np.ndarray:
    lengths = {}
    for i in range(128):
        for s, l in ((2 * i, p[i] & 15), (2 * i + 1, p[i] >> 4)):
            if l:
                lengths[s] = l
    book = {(l, c): s for s, (c, l) in canonical(lengths).items()}
    subs = _substreams(m, S, g)
    W = len(subs)
    NG = -(-W // LANES)
    H = _a16(128 + 4 * NG)
    nwords = struct.unpack(f"<{NG}I", p[128:128 + 4 * NG])
    words = struct.unpack(f"<{(len(p) - H) // 4}I", p[H:])
    out = np.zeros(m, dtype=np.uint8)
    pos = 0
    for j in range(NG):
        group = subs[LANES * j: LANES * j + LANES]
        bits = [0] * len(group)       # received bits, as an int per lane
        have = [0] * len(group)       # received bit count
        used = [0] * len(group)       # consumed bit count
        for r in range(max((len(x) + 1) // 2 for x in group)):
            for lane, idx in enumerate(group):
                if 2 * r >= len(idx):
                    continue
                if have[lane] - used[lane] < 2 * L:
                    bits[lane] |= words[pos] << have[lane]
                    have[lane] += 32
                    pos += 1
                for t in (2 * r, 2 * r + 1):
                    if t >= len(idx):
                        break
                    c, l = 0, 0
                    while (l, c) not in book:
                        if l >= L:
                            raise SpecError("bad code")
                        c = (c << 1) | ((bits[lane] >> used[lane]) & 1)
                        used[lane] += 1
                        l += 1
                    out[idx[t]] = book[(l, c)]
        if pos != sum(nwords[: j + 1]):
            raise SpecError("word count")
    return out
