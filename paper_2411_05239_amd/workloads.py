"""Seeded synthetic inputs shaped like the weights ZipNN compresses.

This module holds no codec arithmetic: it only draws tensors.  The same bytes
are handed to the GPU path and to the CPU oracle.  The paper measures real
checkpoints (BF16 LLMs, FP32 models; paper §III-C, §V-B); those weights are not
available here, so these generators stand in for them with the distributions
the paper reports for regular models (values concentrated in [-1, 1], a skewed
exponent, near-random sign and fraction bits; paper §III-A).

Generators:
  bf16_normal     -- N(0, sigma) rounded to BF16 (single BF16 tensor workload)
  fp32_rows       -- FP32 matrix, row r ~ N(0, sigma_r), log10 sigma_r ~ U(-3, -1)
  checkpoint_8b   -- the 291 tensors of an 8B decoder checkpoint (BF16)
  finetune_delta  -- a fine-tuned copy: N(0, 1e-4) noise on a Bernoulli(0.1) mask
  pruned          -- a copy with a Bernoulli(1 - density) share of its values set to zero
  trajectory      -- training-like checkpoint sequence: each step updates a Bernoulli(p_t)
                     share of the values by N(0, sigma_t), with p_t and sigma_t decaying
  serving_corpus  -- tensors of log-uniform size, 60% BF16 / 30% FP32 / 10% FP8
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def bf16_normal(n: int, sigma: float = 0.02, seed: int = 0, device="cpu") -> torch.Tensor:
    """n values N(0, sigma) (sigma = standard deviation), rounded to BF16 (RNE)."""
    x = torch.randn(n, generator=_gen(seed, device), device=device, dtype=torch.float32)
    return (x * sigma).to(torch.bfloat16)


def fp32_rows(rows: int = 8192, cols: int = 8192, seed: int = 1, device="cpu") -> torch.Tensor:
    """FP32 [rows, cols]; row r ~ N(0, sigma_r), log10(sigma_r) ~ U(-3, -1)."""
    g = _gen(seed, device)
    u = torch.rand(rows, generator=g, device=device, dtype=torch.float64)
    sigma = torch.pow(10.0, -3.0 + 2.0 * u).to(torch.float32)
    x = torch.randn(rows, cols, generator=g, device=device, dtype=torch.float32)
    return x * sigma[:, None]


@dataclass(frozen=True)
class TensorSpec:
    name: str
    shape: tuple
    kind: str          # "normal" (N(0, sigma)) or "norm" (1 + N(0, sigma))
    sigma: float
    seed: int

    @property
    def numel(self) -> int:
        return int(math.prod(self.shape))


def checkpoint_8b_specs(layers: int = 32, hidden: int = 4096, kv: int = 1024, ffn: int = 14336,
                        vocab: int = 128256, seed0: int = 1000) -> list[TensorSpec]:
    """Tensor list of an 8B decoder checkpoint, in file order: embedding, then
    per layer q/k/v/o, gate/up/down and two RMSNorm vectors, then the final
    norm and the (untied) head.  Weights ~ N(0, 0.02); embedding and head
    ~ N(0, 0.01); norms ~ 1 + N(0, 0.05).  Tensor i uses seed seed0 + i."""
    out: list[tuple] = [("embed", (vocab, hidden), "normal", 0.01)]
    for l in range(layers):
        p = f"layers.{l}."
        out += [
            (p + "q", (hidden, hidden), "normal", 0.02),
            (p + "k", (kv, hidden), "normal", 0.02),
            (p + "v", (kv, hidden), "normal", 0.02),
            (p + "o", (hidden, hidden), "normal", 0.02),
            (p + "gate", (ffn, hidden), "normal", 0.02),
            (p + "up", (ffn, hidden), "normal", 0.02),
            (p + "down", (hidden, ffn), "normal", 0.02),
            (p + "attn_norm", (hidden,), "norm", 0.05),
            (p + "mlp_norm", (hidden,), "norm", 0.05),
        ]
    out += [("final_norm", (hidden,), "norm", 0.05), ("head", (vocab, hidden), "normal", 0.01)]
    return [TensorSpec(n, s, k, sg, seed0 + i) for i, (n, s, k, sg) in enumerate(out)]


def make_tensor(spec: TensorSpec, device="cpu", numel: int | None = None) -> torch.Tensor:
    """Draw one checkpoint tensor (flattened, BF16).  ``numel`` draws only a
    prefix-sized sample with the same distribution (for small tests)."""
    n = spec.numel if numel is None else min(numel, spec.numel)
    x = torch.randn(n, generator=_gen(spec.seed, device), device=device, dtype=torch.float32) * spec.sigma
    if spec.kind == "norm":
        x = x + 1.0
    return x.to(torch.bfloat16)


def finetune_delta(w: torch.Tensor, seed: int, p: float = 0.1, sigma: float = 1e-4) -> torch.Tensor:
    """ft = bf16(fp32(w) + M * Z), M ~ Bernoulli(p), Z ~ N(0, sigma)."""
    g = _gen(seed, w.device)
    m = torch.rand(w.numel(), generator=g, device=w.device) < p
    z = torch.randn(w.numel(), generator=g, device=w.device) * sigma
    return (w.float().reshape(-1) + m * z).to(torch.bfloat16).reshape(w.shape)


def pruned(w: torch.Tensor, density: float, seed: int) -> torch.Tensor:
    """w with each value kept with probability `density`, else set to +0."""
    keep = torch.rand(w.numel(), generator=_gen(seed, w.device), device=w.device) < density
    return torch.where(keep, w.reshape(-1), torch.zeros((), dtype=w.dtype, device=w.device)).reshape(w.shape)


def trajectory(ws: list, steps: int, seed: int, p0: float = 0.3, sigma0: float = 3e-4,
               decay: float = 0.7) -> list:
    """Checkpoints 0..steps-1 of a training-like run from the tensors ws:
    checkpoint t+1 = bf16(fp32(checkpoint t) + M * Z) with M ~ Bernoulli(p0
    decay^t) and Z ~ N(0, sigma0 decay^t), per tensor, seeded by (seed, t,
    tensor index).  Changes shrink and thin out as the run converges."""
    out = [list(ws)]
    for t in range(steps - 1):
        cur = []
        for i, w in enumerate(out[-1]):
            g = _gen(seed * 1000003 + t * 1009 + i, w.device)
            m = torch.rand(w.numel(), generator=g, device=w.device) < p0 * decay ** t
            z = torch.randn(w.numel(), generator=g, device=w.device) * (sigma0 * decay ** t)
            cur.append((w.float().reshape(-1) + m * z).to(w.dtype).reshape(w.shape))
        out.append(cur)
    return out


FP8_MAX = 448.0


@dataclass(frozen=True)
class CorpusItem:
    index: int
    dtype: str         # "bf16" | "fp32" | "fp8"
    nbytes: int
    seed: int


def serving_corpus(count: int = 128, seed: int = 3000, min_bytes: int = 64 << 10, max_bytes: int = 1 << 30,
                   mix=(0.6, 0.3, 0.1)) -> list[CorpusItem]:
    """Tensor sizes log-uniform in [min_bytes, max_bytes] (rounded down to a
    multiple of 16 bytes); dtype drawn 60/30/10 BF16/FP32/FP8."""
    g = _gen(seed, "cpu")
    u = torch.rand(count, generator=g, dtype=torch.float64)
    d = torch.rand(count, generator=g, dtype=torch.float64)
    items = []
    for i in range(count):
        nb = int(math.exp(math.log(min_bytes) + float(u[i]) * (math.log(max_bytes) - math.log(min_bytes))))
        nb = max(16, nb // 16 * 16)
        dt = "bf16" if d[i] < mix[0] else ("fp32" if d[i] < mix[0] + mix[1] else "fp8")
        items.append(CorpusItem(i, dt, nb, seed + 1 + i))
    return items


def make_corpus_tensor(item: CorpusItem, device="cpu") -> torch.Tensor:
    g = _gen(item.seed, device)
    if item.dtype == "bf16":
        return (torch.randn(item.nbytes // 2, generator=g, device=device) * 0.02).to(torch.bfloat16)
    if item.dtype == "fp32":
        return torch.randn(item.nbytes // 4, generator=g, device=device) * 0.05
    x = torch.randn(item.nbytes, generator=g, device=device)
    amax = x.abs().max().clamp_min(1e-30)
    return (x * (FP8_MAX / amax)).to(torch.float8_e4m3fn)


def poisson_arrivals(rate: float, count: int, seed: int) -> list[float]:
    """Arrival times (seconds) of a Poisson process of the given rate."""
    g = _gen(seed, "cpu")
    gaps = -torch.log1p(-torch.rand(count, generator=g, dtype=torch.float64)) / rate
    return torch.cumsum(gaps, 0).tolist()
