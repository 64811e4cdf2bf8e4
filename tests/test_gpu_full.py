"""Full-size workloads (1 Mbp / 100,000 reads; 16 Mbp / 4,000,000 reads of 100
bp; 16 Mbp / 4,000,000 reads of 20-300 bp; 250 Mbp / 64,000,000 reads of 150
bp) through the launch configuration the benchmark times.  Every read is
compared with the oracle.  At 250 Mbp the oracle's own comparison sort is
too slow, so it searches the device-built array after checking that it is
the suffix array (a permutation whose neighbouring suffixes ascend)."""
import os
import sys

import numpy as np
import pytest

import gen
import paper_1303_3692_amd as S
from oracle import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


_refs = {}
CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1303_3692_amd",
                     "tuning_cache.jsonl")


def reference(name):
    if name not in _refs:
        ref = gen.make_reference(name)
        text = ref.ascii()
        if name == "c4":
            d = S.sa_build_device(text, 0)
            sa = S.sa_download(d).suffix_array()
            assert oracle.sa_check(text, sa) == 0
        else:
            sa = oracle.sa_build(text)
            d = S.sa_upload(S.sa_build(text), 0)
        _refs[name] = (ref, text, sa, d)
    return _refs[name]


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3", "c4"])
def test_full_workload(device, cfg):
    print("case: full", cfg, flush=True)
    ref, text, sa, d = reference({"c1": "c1", "c4": "c4"}.get(cfg, "c2"))
    print("  index ready", flush=True)
    reads = gen.make_reads_parallel(ref, gen.READ_SPECS[cfg], workers=8)
    print(f"  {reads.count} reads generated", flush=True)
    want = oracle.match(text, sa, reads.data, reads.offs, nthreads=oracle.max_threads())
    print(f"  oracle answered {reads.count} reads", flush=True)
    d_reads = torch.from_numpy(reads.data).to(device)
    d_offs = torch.from_numpy(reads.offs).to(device)
    # the benchmark's launch configuration: its tuning cache, graph replay on a stream of its own
    stream = torch.cuda.Stream()
    S.sa_tune(d, d_reads, d_offs, stream=stream, cache_path=CACHE)
    tuned = S.cfg(d, use_graph=1)
    print(f"  tuned: {tuned.as_dict()}", flush=True)
    for c in (tuned, S.cfg(d, kernel=S.SA_KERNEL_PLAIN)):
        d_out = torch.full((reads.count, 4), -7, dtype=torch.int32, device=device)
        S.match_batch_dev(d, d_reads, d_offs, d_out, stream=stream, config=c)
        stream.synchronize()
        kernel = c.kernel
        got = d_out.cpu().numpy()
        bad = np.nonzero((got[:, :3] != want[:, :3]).any(1) | ((got[:, 3] & 1) != want[:, 3]))[0]
        assert len(bad) == 0, f"{cfg} kernel {kernel}: {len(bad)} mismatches, e.g. {bad[:5]}"
    print(f"  {cfg}: all {reads.count} reads identical, exact fraction {want[:, 3].mean():.4f}", flush=True)
    sys.stdout.flush()
