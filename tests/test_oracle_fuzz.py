"""Property tests of the oracle (CPU): random dtypes, lengths around chunk
boundaries, chunk sizes, sub-stream lengths, groups, code-length limits,
policies, value distributions (skewed, uniform, constant, special float bit
patterns) and XOR bases.  The C oracle and the independent Python spec must
write the same bytes, and both must restore the input exactly."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from oracle import spec

DTYPES = [oracle.BF16, oracle.FP16, oracle.FP32, oracle.FP8_E4M3, oracle.U8]


@st.composite
def cases(draw):
    dtype = draw(st.sampled_from(DTYPES))
    B = oracle.WIDTH[dtype]
    chunk = draw(st.sampled_from([256, 512, 1024, 2048]))
    E = chunk // B
    g = draw(st.sampled_from([2, 4, 8]))
    S = draw(st.sampled_from([s for s in (2, 4, 8, 16, 32, 64, 128, 256) if s >= g and E // s <= 4096]))
    L = draw(st.integers(min_value=8, max_value=11))
    n_chunks = draw(st.integers(min_value=0, max_value=3))
    n = max(0, n_chunks * E + draw(st.integers(min_value=-2, max_value=2)))
    kind = draw(st.sampled_from(["normal", "uniform", "constant", "sparse", "special"]))
    policy = tuple(draw(st.sampled_from([oracle.AUTO, oracle.HUF, oracle.RAW, oracle.ZG])) for _ in range(B))
    with_base = draw(st.booleans())
    seed = draw(st.integers(min_value=0, max_value=2**31 - 1))
    skip = draw(st.sampled_from([0, 0, 1, 2, 5]))
    exp = dtype in (oracle.BF16, oracle.FP32) and draw(st.booleans())
    return dtype, B, chunk, S, g, L, n, kind, policy, with_base, seed, skip, exp


def _bytes(kind, n, B, rng):
    nb = n * B
    if kind == "uniform":
        return rng.integers(0, 256, size=nb, dtype=np.uint8)
    if kind == "constant":
        return np.full(nb, rng.integers(0, 256), dtype=np.uint8)
    if kind == "sparse":   # mostly zero bytes, like an XOR delta
        x = np.zeros(nb, dtype=np.uint8)
        idx = rng.random(nb) < 0.05
        x[idx] = rng.integers(1, 256, size=int(idx.sum()), dtype=np.uint8)
        return x
    if kind == "special":  # words built from float special patterns and random bits
        pats = np.array([0x00, 0x80, 0x7F, 0xFF, 0x3F, 0xC0, 0x01], dtype=np.uint8)
        return pats[rng.integers(0, len(pats), size=nb)]
    # "normal": exponent-like top bytes, noisy low bytes
    w = (rng.standard_normal(max(n, 1)) * 0.02).astype(np.float32).view(np.uint32)
    b = w.view(np.uint8).reshape(-1, 4)[:, 4 - B:].reshape(-1)[:nb] if B <= 4 else None
    return np.ascontiguousarray(b)


@settings(max_examples=120, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(cases())
def test_oracle_and_spec_agree_and_round_trip(oracle_lib, case):
    dtype, B, chunk, S, g, L, n, kind, policy, with_base, seed, skip, exp = case
    rng = np.random.default_rng(seed)
    x = _bytes(kind, n, B, rng)
    base = rng.integers(0, 256, size=n * B, dtype=np.uint8) if with_base else None
    if with_base:
        x = x ^ base   # the XOR of x with base is then the chosen distribution
    kw = dict(chunk_bytes=chunk, S=S, g=g, L=L, policy=list(policy), skip=skip, exp=exp)
    c = oracle.compress(x, dtype, base=base, **kw)
    assert np.array_equal(oracle.decompress(c, base=base), x)
    ref = spec.compress(x, dtype, base=base, **kw)
    assert ref == c.tobytes()
    assert np.array_equal(spec.decompress(ref, base=base), x)
    h = oracle.header(c)
    assert h["n"] == n and h["total"] == c.size and c.size % oracle.PAY_ALIGN in (0, 64)
