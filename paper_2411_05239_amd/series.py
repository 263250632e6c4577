"""Periodic-base storage of a sequence of checkpoints (ZipNN, arXiv
2411.05239, §IV-B "Periodic Base"): a host policy over the batched kernels of
the C ABI; every byte of coding runs in the library.

Checkpoint t is stored standalone when t mod P = 0 (a base) and otherwise as
the XOR delta (§IV-B) against
  * "chain": checkpoint t-1, so restoring t decodes the base and then every
    delta after it in order (at most P-1 deltas);
  * "pairs": the last base, so restoring t is one base decode and one delta
    decode, at the cost of deltas against an older model.
Each checkpoint is a list of tensors of one dtype, compressed together into
one arena (one batched launch per kernel); restoring a checkpoint is one
batched decode per link of its chain.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import zipnn as Z


@dataclass
class _Stored:
    arena: object                 # uint8 device tensor
    offsets: list
    base: int | None              # index of the checkpoint it is a delta against
    nbytes: int = field(default=0)


class CheckpointSeries:
    def __init__(self, codec: "Z.Codec", period: int, mode: str = "pairs", params: "Z.zipnn_params | None" = None):
        if period < 1 or mode not in ("chain", "pairs"):
            raise ValueError("period >= 1 and mode 'chain' or 'pairs'")
        self.codec, self.period, self.mode, self.params = codec, period, mode, params
        self.stored: list[_Stored] = []
        self._ref = None   # the tensors the next delta is taken against (device)

    def base_of(self, t: int) -> int | None:
        if t % self.period == 0:
            return None
        return t - 1 if self.mode == "chain" else t - t % self.period

    def append(self, tensors) -> _Stored:
        """Compress checkpoint t = len(self) (device tensors, one dtype)."""
        t = len(self.stored)
        b = self.base_of(t)
        arena, offs = self.codec.compress_batch(tensors, self.params, bases=None if b is None else self._ref)
        s = _Stored(arena[: offs[-1]].clone(), offs, b, offs[-1])
        self.stored.append(s)
        # the reference for the following deltas: this checkpoint (chain) or
        # the last base (pairs)
        if self.mode == "chain" or b is None:
            self._ref = [x.clone() for x in tensors]
        return s

    def __len__(self) -> int:
        return len(self.stored)

    def chain(self, t: int) -> list[int]:
        """The checkpoints decoded, in order, to restore t."""
        links = [t]
        while self.stored[links[-1]].base is not None:
            links.append(self.stored[links[-1]].base)
        return links[::-1]

    def restore(self, t: int, outs) -> int:
        """Decode checkpoint t into the device tensors `outs` (shapes and
        dtype of the original); returns the number of batched decodes."""
        import torch

        links = self.chain(t)
        cur = None
        for i, u in enumerate(links):
            s = self.stored[u]
            dst = outs if i == len(links) - 1 else [torch.empty_like(o) for o in outs]
            Z.zipnn_decompress_batch(self.codec.ctx, s.arena.data_ptr(), s.offsets, [o.data_ptr() for o in dst],
                                     [o.numel() * o.element_size() for o in dst],
                                     None if s.base is None else [c.data_ptr() for c in cur], self.codec._stream())
            cur = dst
        st = self.codec.status(clear=True)
        if st != Z.ZIPNN_OK:
            raise Z.ZipnnError(st, "series restore (device)")
        return len(links)
