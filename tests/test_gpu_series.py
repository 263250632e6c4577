"""GPU tests of periodic-base checkpoint storage (§IV-B "Periodic Base"):
every checkpoint of a training-like sequence restores bit-exactly under both
policies; deltas are smaller than standalone containers; a delta container
equals the oracle's XOR-delta container against the policy's base."""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_05239_amd import workloads
from paper_2411_05239_amd import zipnn as Z
from paper_2411_05239_amd.series import CheckpointSeries

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def codec():
    c = Z.Codec(0)
    yield c
    c.close()


def _model():
    specs = workloads.checkpoint_8b_specs(layers=2, hidden=256, kv=64, ffn=896, vocab=1001, seed0=700)
    return [workloads.make_tensor(s, device="cuda") for s in specs]


@pytest.mark.parametrize("mode", ["chain", "pairs"])
def test_series_restores_every_checkpoint(codec, mode):
    traj = workloads.trajectory(_model(), steps=7, seed=11)
    ser = CheckpointSeries(codec, period=3, mode=mode)
    for ck in traj:
        ser.append(ck)
    assert [ser.stored[t].base for t in range(7)] == (
        [None, 0, 1, None, 3, 4, None] if mode == "chain" else [None, 0, 0, None, 3, 3, None])
    for t, ck in enumerate(traj):
        outs = [torch.empty_like(x) for x in ck]
        n = ser.restore(t, outs)
        assert n == len(ser.chain(t))
        for o, x in zip(outs, ck):
            assert torch.equal(o.view(torch.uint8), x.view(torch.uint8)), (mode, t)
    full = [s.nbytes for s in ser.stored if s.base is None]
    delta = [s.nbytes for s in ser.stored if s.base is not None]
    assert max(delta) < 0.5 * min(full)
    # a delta container is the oracle's XOR delta against the policy's base
    t = 5
    b = ser.stored[t].base
    i = 2
    ref = oracle.compress(traj[t][i].cpu(), oracle.BF16, base=traj[b][i].cpu(), nthreads=8,
                          chunk_bytes=262144, S=512, g=4, L=11, policy=[0, 0])
    s = ser.stored[t]
    got = s.arena[s.offsets[i]: s.offsets[i] + ref.size].cpu().numpy()
    assert np.array_equal(got, ref)
