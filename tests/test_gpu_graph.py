"""Replayed hipGraph batches: every replay, with eager work and
synchronisation between replays, must equal the oracle."""
import numpy as np
import pytest

import gen
import paper_1303_3692_amd as S
from oracle import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_graph_replays_match_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    print("case: graph replays", flush=True)
    dev = torch.device("cuda:0")
    ref, reads = gen.workload("c3", n=600_000, count=30_000)
    text = ref.ascii()
    d = S.sa_upload(S.sa_build(text), 0)
    want = oracle.match(text, oracle.sa_build(text), reads.data, reads.offs)
    d_reads = torch.from_numpy(reads.data.copy()).to(dev)
    d_offs = torch.from_numpy(reads.offs).to(dev)
    stream = torch.cuda.Stream()
    graph_cfg = S.cfg(d, use_graph=1, nbuckets=3, bucket_edge=[64, 160, 320])
    eager_cfg = S.cfg(d, use_graph=0)
    outs = [torch.empty((reads.count, 4), dtype=torch.int32, device=dev) for _ in range(2)]
    half = reads.count // 2
    for rep in range(4):
        for o in outs:
            with torch.cuda.stream(stream):
                o.fill_(-7)
        # replay (captured on the first pass) on the full batch and on half of it
        S.match_batch_dev(d, d_reads, d_offs, outs[0], stream=stream, config=graph_cfg)
        S.match_batch_dev(d, d_reads, d_offs[: half + 1], outs[1], nreads=half, stream=stream, config=graph_cfg)
        stream.synchronize()
        got = outs[0].cpu().numpy()
        assert (got[:, :3] == want[:, :3]).all() and ((got[:, 3] & 1) == want[:, 3]).all(), f"replay {rep}"
        got = outs[1].cpu().numpy()[:half]
        assert (got[:, :3] == want[:half, :3]).all() and ((got[:, 3] & 1) == want[:half, 3]).all(), f"half {rep}"
        # eager work on the same stream between replays
        e = torch.zeros((reads.count, 4), dtype=torch.int32, device=dev)
        S.match_batch_dev(d, d_reads, d_offs, e, stream=stream, config=eager_cfg)
        stream.synchronize()
        got = e.cpu().numpy()
        assert (got[:, :3] == want[:, :3]).all()
