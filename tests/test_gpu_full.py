"""Full-size workloads (1 Mbp / 100,000 reads; 16 Mbp / 4,000,000 reads of 100
bp; 16 Mbp / 4,000,000 reads of 20-300 bp) through the launch configuration
the benchmark times, every read compared with the oracle."""
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


def reference(name):
    if name not in _refs:
        ref = gen.make_reference(name)
        text = ref.ascii()
        _refs[name] = (ref, text, oracle.sa_build(text), S.sa_upload(S.sa_build(text), 0))
    return _refs[name]


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3"])
def test_full_workload(device, cfg):
    print("case: full", cfg, flush=True)
    ref, text, sa, d = reference("c1" if cfg == "c1" else "c2")
    reads = gen.make_reads(ref, gen.READ_SPECS[cfg])
    want = oracle.match(text, sa, reads.data, reads.offs)
    d_reads = torch.from_numpy(reads.data).to(device)
    d_offs = torch.from_numpy(reads.offs).to(device)
    for kernel in (S.SA_KERNEL_TUNED, S.SA_KERNEL_PLAIN):
        d_out = torch.full((reads.count, 4), -7, dtype=torch.int32, device=device)
        S.match_batch_dev(d, d_reads, d_offs, d_out, config=S.cfg(d, kernel=kernel))
        torch.cuda.synchronize()
        got = d_out.cpu().numpy()
        bad = np.nonzero((got[:, :3] != want[:, :3]).any(1) | ((got[:, 3] & 1) != want[:, 3]))[0]
        assert len(bad) == 0, f"{cfg} kernel {kernel}: {len(bad)} mismatches, e.g. {bad[:5]}"
    print(f"  {cfg}: {reads.count} reads identical, exact fraction {want[:, 3].mean():.4f}", flush=True)
    sys.stdout.flush()
