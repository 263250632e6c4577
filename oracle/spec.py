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
  modes    -- RAW / RLE / HUF / ZG per byte-group (§III-B, §IV-B, §V-A), with
              probe chunks every K+1 chunks (§III-B, "Identifying
              compressibility");
  coding   -- one bit string per sub-stream (``substream_bits``);
  layout   -- the lock-step word order of a lane group as a sort of (step,
              pair, lane) events rather than nested loops (``layout``);
  container -- 64-byte header, 16-byte map entries, 128-byte aligned payloads
              (the container described in ``zipnn_oracle.h``).
"""
from __future__ import annotations

import struct

import numpy as np

WIDTH = {1: 2, 2: 2, 3: 4, 4: 1, 5: 1}
AUTO, HUF, RAW, ZG = 0, 1, 2, 3
MODE_RAW, MODE_HUF, MODE_RLE, MODE_ZG = 0, 1, 2, 3


class SpecError(ValueError):
    pass


def split(words: np.ndarray, B: int) -> list[np.ndarray]:
    """Stream k = byte B-1-k of each little-endian word."""
    a = np.ascontiguousarray(words).view(np.uint8).reshape(-1, B)
    return [a[:, B - 1 - k].copy() for k in range(B)]


def extract_exponent(raw: np.ndarray, B: int, inverse: bool = False) -> np.ndarray:
    """Exponent extraction (§III-A): sign, exponent, fraction -> exponent,
    sign, fraction, on little-endian words viewed as unsigned integers."""
    w = raw.view(np.uint16 if B == 2 else np.uint32).astype(np.uint64)
    nb = 8 * B
    frac_mask = (1 << (nb - 9)) - 1
    if not inverse:
        sign, exp = w >> (nb - 1), (w >> (nb - 9)) & 0xFF
        out = (exp << (nb - 8)) + (sign << (nb - 9)) + (w & frac_mask)
    else:
        exp, sign = w >> (nb - 8), (w >> (nb - 9)) & 1
        out = (sign << (nb - 1)) + (exp << (nb - 9)) + (w & frac_mask)
    return out.astype(np.uint16 if B == 2 else np.uint32).view(np.uint8)


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


def _events(m: int, S: int, g: int, coded) -> list[list[tuple[int, list[int]]]]:
    """Per lane group, the decode events in lock-step order.

    Group q of g symbols belongs to sub-stream w = q mod W (lane w mod 64 of
    lane group w div 64) and is its (q div W)-th group: its step.  A coded
    group contributes one event per pair of symbols; sorting the events by
    (step, pair, lane) gives the order in which the lanes of a lane group
    decode, and so the order of their word requests."""
    W = -(-m // S)
    per_group = [[] for _ in range(-(-W // LANES))]
    for q in range(-(-m // g)):
        if not coded(q):
            continue
        w, step = q % W, q // W
        idx = list(range(q * g, min(q * g + g, m)))
        for pr in range(0, len(idx), 2):
            per_group[w // LANES].append(((step, pr, w % LANES), idx[pr:pr + 2]))
    return [[(key[2], idx) for key, idx in sorted(ev)] for ev in per_group]


def substream_bits(sym: np.ndarray, S: int, g: int, codes: dict[int, tuple[int, int]], coded, w: int) -> tuple[int, int]:
    """The coding of sub-stream w: the codes of the symbols of its coded groups
    w, w+W, ... as (bits, count), bit i of the integer = i-th stream bit."""
    m = len(sym)
    W, G = -(-m // S), -(-m // g)
    acc, n = 0, 0
    for q in range(w, G, W):
        if not coded(q):
            continue
        for e in range(q * g, min(q * g + g, m)):
            c, l = codes[int(sym[e])]
            for b in range(l):
                acc |= ((c >> (l - 1 - b)) & 1) << n
                n += 1
    return acc, n


def layout(events: list[tuple[int, list[int]]], lane_bits: dict[int, int], pair_bits, L: int) -> list[int]:
    """The word layout of one lane group: walking its sorted events, a lane
    holding fewer than 2L bits takes its next 32-bit word first."""
    buffered, nxt, out = {}, {}, []
    for lane, idx in events:
        if buffered.get(lane, 0) < 2 * L:
            out.append((lane_bits.get(lane, 0) >> (32 * nxt.get(lane, 0))) & 0xFFFFFFFF)
            nxt[lane] = nxt.get(lane, 0) + 1
            buffered[lane] = buffered.get(lane, 0) + 32
        buffered[lane] -= pair_bits(idx)
    return out


def _huf_payload(sym: np.ndarray, S: int, g: int, L: int, lengths: dict[int, int], bitmap: bytes | None) -> bytes:
    m = len(sym)
    codes = canonical(lengths)
    if bitmap is None:
        coded = lambda q: True
    else:
        coded = lambda q: (bitmap[q // 8] >> (q % 8)) & 1
    W = -(-m // S)
    counts_out, words_out = [], []
    for j, events in enumerate(_events(m, S, g, coded)):
        lane_bits = {l: substream_bits(sym, S, g, codes, coded, LANES * j + l)[0]
                     for l in range(min(LANES, W - LANES * j))}
        stream = layout(events, lane_bits, lambda idx: sum(lengths[int(sym[e])] for e in idx), L)
        counts_out.append(len(stream))
        words_out.extend(stream)
    NG = -(-W // LANES)
    H = _a16(128 + 4 * NG)
    table = bytes(lengths.get(2 * i, 0) | (lengths.get(2 * i + 1, 0) << 4) for i in range(128))
    head = table + struct.pack(f"<{NG}I", *counts_out)
    return head + bytes(H - len(head)) + (bitmap or b"") + struct.pack(f"<{len(words_out)}I", *words_out)


def encode_stream(sym: np.ndarray, S: int, g: int, L: int, policy: int) -> tuple[int, int, bytes]:
    """-> (mode, rle / fill value, payload bytes)"""
    m = len(sym)
    if policy == RAW:
        return MODE_RAW, 0, sym.tobytes()
    counts = np.bincount(sym, minlength=256)
    present = [s for s in range(256) if counts[s]]
    if len(present) == 1:
        return MODE_RLE, present[0], b""
    options = []   # (bytes, preference, mode, value, payload)
    if policy != ZG:
        lengths = pm_lengths({s: int(counts[s]) for s in present}, L)
        huf = _huf_payload(sym, S, g, L, lengths, None)
        options.append((len(huf), 1, MODE_HUF, 0, huf))
    z = int(np.argmax(counts))   # first maximum: the smallest most frequent value
    if policy == ZG or (policy == AUTO and 2 * int(counts[z]) >= m):
        G = -(-m // g)
        marked = [q for q in range(G) if np.any(sym[q * g: q * g + g] != z)]
        bitmap = bytearray(_a16(-(-G // 8)))
        for q in marked:
            bitmap[q // 8] |= 1 << (q % 8)
        sub = np.concatenate([sym[q * g: q * g + g] for q in marked]) if marked else sym[:0]
        counts2 = np.bincount(sub, minlength=256)
        present2 = [s for s in range(256) if counts2[s]]
        if len(present2) >= 2:
            lengths2 = pm_lengths({s: int(counts2[s]) for s in present2}, L)
            zg = _huf_payload(sym, S, g, L, lengths2, bytes(bitmap))
            options.append((len(zg), 2, MODE_ZG, z, zg))
        elif policy == ZG:   # nothing for ZG to code with two values: HUF
            lengths = pm_lengths({s: int(counts[s]) for s in present}, L)
            huf = _huf_payload(sym, S, g, L, lengths, None)
            options.append((len(huf), 1, MODE_HUF, 0, huf))
    if policy == AUTO:
        options.append((m, 0, MODE_RAW, 0, sym.tobytes()))
        _, _, mode, value, payload = min(options, key=lambda o: (o[0], o[1]))
        return mode, value, payload
    _, _, mode, value, payload = max(options, key=lambda o: o[1])   # a forced policy: ZG over HUF
    return mode, value, payload


def compress(words: np.ndarray, dtype: int, *, base: np.ndarray | None = None, chunk_bytes: int = 262144,
             S: int = 512, g: int = 4, L: int = 11, policy=(AUTO, AUTO, AUTO, AUTO), skip: int = 0,
             exp: bool = False) -> bytes:
    B = WIDTH[dtype]
    raw = np.ascontiguousarray(words).view(np.uint8).reshape(-1)
    if base is not None:
        raw = raw ^ np.ascontiguousarray(base).view(np.uint8).reshape(-1)
    if exp:
        raw = extract_exponent(np.ascontiguousarray(raw), B)
    n = raw.size // B
    E = chunk_bytes // B
    n_chunks = -(-n // E)
    entries, payloads = [], []
    for c in range(n_chunks):
        chunk = raw[c * E * B: min(n, (c + 1) * E) * B]
        probe = c - c % (skip + 1)   # the chunk that probed this one's run (itself if c is a probe)
        for k, s in enumerate(split(chunk, B)):
            pol = policy[k]
            if pol == AUTO and probe != c and entries[probe * B + k][0] == MODE_RAW:
                pol = RAW   # the probe found this byte group incompressible: no analysis
            entries.append(encode_stream(s, S, g, L, pol))
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
    flags = (1 if base is not None else 0) | (2 if any(e[0] == MODE_ZG for e in entries) else 0) | (4 if exp else 0)
    hdr = b"ZNN1" + struct.pack("<HBBQIHBBIIQ", 1, dtype, B, n, chunk_bytes, S, g, L,
                                flags, n_chunks, total) + pol + bytes([skip]) + bytes(19)
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
            elif mode == MODE_HUF:
                streams.append(_decode_huf(p, m, S, g, L, None))
            elif mode == MODE_ZG:
                if not flags & 2:
                    raise SpecError("ZG entry without the header flag")
                streams.append(_decode_huf(p, m, S, g, L, rle))
            else:
                raise SpecError("mode")
        out[c * E * B: (c * E + m) * B] = merge(streams, B)
    if flags & 4:
        out = extract_exponent(out, B, inverse=True)
    if base is not None:
        out ^= np.ascontiguousarray(base).view(np.uint8).reshape(-1)
    return out


def _decode_huf(p: bytes, m: int, S: int, g: int, L: int, fill: int | None) -> np.ndarray:
    """HUF payload (fill None) or ZG payload (groups left out of the bitmap
    are all `fill`)."""
    lengths = {}
    for i in range(128):
        for s, l in ((2 * i, p[i] & 15), (2 * i + 1, p[i] >> 4)):
            if l:
                lengths[s] = l
    book = {(l, c): s for s, (c, l) in canonical(lengths).items()}
    W = -(-m // S)
    NG = -(-W // LANES)
    H = _a16(128 + 4 * NG)
    out = np.zeros(m, dtype=np.uint8)
    if fill is None:
        coded = lambda q: True
        start = H
    else:
        G = -(-m // g)
        start = H + _a16(-(-G // 8))
        bitmap = p[H:start]
        coded = lambda q: (bitmap[q // 8] >> (q % 8)) & 1
        for q in range(G):
            if not coded(q):
                out[q * g: q * g + g] = fill
    nwords = struct.unpack(f"<{NG}I", p[128:128 + 4 * NG])
    words = struct.unpack(f"<{(len(p) - start) // 4}I", p[start:])
    pos = 0
    for j, events in enumerate(_events(m, S, g, coded)):
        bits, have, used = {}, {}, {}   # per lane: received bits, their count, bits consumed
        for lane, idx in events:
            if have.get(lane, 0) - used.get(lane, 0) < 2 * L:
                bits[lane] = bits.get(lane, 0) | (words[pos] << have.get(lane, 0))
                have[lane] = have.get(lane, 0) + 32
                pos += 1
            for e in idx:
                c, l = 0, 0
                while (l, c) not in book:
                    if l >= L:
                        raise SpecError("bad code")
                    c = (c << 1) | ((bits[lane] >> used.get(lane, 0)) & 1)
                    used[lane] = used.get(lane, 0) + 1
                    l += 1
                out[e] = book[(l, c)]
        if pos != sum(nwords[: j + 1]):
            raise SpecError("word count")
    return out
