"""Search cost against the paper's bound (Section IV: O(m log n) per query):
with open bounds (-1, n) a binary search makes at most ceil(log2(n + 1))
probes, and a read takes at most four searches (LB and RB of P, LB and RB
of P[0..l)) plus the two neighbour comparisons for l.  The instrumented
kernels count every global probe; their results equal the timed ones."""
import math

import numpy as np
import pytest

import gen
import paper_1303_3692_amd as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


@pytest.mark.parametrize("cfg,n,count", [("c1", 1_000_000, 100_000), ("c2", 2_000_000, 200_000),
                                         ("c3", 2_000_000, 100_000)])
def test_probe_counts_within_the_bound(cfg, n, count):
    print("case: probe counts", cfg, flush=True)
    ref, reads = gen.workload(cfg, n=n, count=count)
    d = S.sa_upload(S.sa_build(ref.ascii()), 0)
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(reads.data).to(dev)
    d_offs = torch.from_numpy(reads.offs).to(dev)
    lg = math.ceil(math.log2(len(d) + 1))
    per_read = {}
    for name, kw in (("plain", dict(kernel=S.SA_KERNEL_PLAIN)), ("tuned", dict()), ("tuned-no-table", dict(prefix_table=0))):
        outs = []
        for count_on in (0, 1):
            c = S.cfg(d, **kw)
            c.count = count_on
            out = torch.zeros((reads.count, 4), dtype=torch.int32, device=dev)
            S.match_batch_dev(d, d_reads, d_offs, out, config=c)
            torch.cuda.synchronize()
            outs.append(out.cpu().numpy())
        assert (outs[0] == outs[1]).all(), name
        cnt = S.sa_probe_counts(d)
        assert cnt["reads"] == reads.count
        assert cnt["global_probes"] <= reads.count * (4 * lg + 2), name
        per_read[name] = cnt["global_probes"] / reads.count
    # the LDS tile and the prefix table only remove global probes
    assert per_read["tuned"] < per_read["tuned-no-table"] < per_read["plain"]
