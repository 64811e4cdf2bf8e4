"""Every launch configuration the autotuner can pick gives the oracle's bits
(Section IV: LB and RB are unique, so no tile depth, workgroup shape, work
split, search start, sort width, packing pass or bucket layout may change a
result), and a full tuner run keeps a configuration whose results match."""
import sys

import numpy as np
import pytest

import gen
import paper_1303_3692_amd as S
from oracle import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def workload(device):
    # the c3 recipe (20-300 bases) on a 2 Mbp reference, 60,000 reads
    ref = gen.make_reference("c2", n=2_000_000)
    reads = gen.make_reads(ref, gen.READ_SPECS["c3"], 60_000)
    text = ref.ascii()
    want = oracle.match(text, oracle.sa_build(text), reads.data, reads.offs)
    d = S.sa_build_device(text, 0)
    return d, reads, want


def assert_same(got, want, label):
    bad = np.nonzero((got[:, :3] != want[:, :3]).any(1) | ((got[:, 3] & 1) != want[:, 3]))[0]
    assert len(bad) == 0, f"{label}: {len(bad)} mismatches, first rows {bad[:5]}"


def test_every_tuner_candidate(device, workload):
    d, reads, want = workload
    d_reads = torch.from_numpy(reads.data).to(device)
    d_offs = torch.from_numpy(reads.offs).to(device)
    cands = S.sa_tune_candidates(d, d_offs)
    # the later stages around a sorted, bucketed configuration too
    around = S.cfg(d, sort=1, nbuckets=2, bucket_edge=[160, 1024], block=512, blocks_per_cu=2)
    cands += S.sa_tune_candidates(d, d_offs, around=around)
    say(f"case: {len(cands)} tuner candidates")
    assert len(cands) >= 30
    assert len({(c.tile_levels, c.block, c.blocks_per_cu) for c in cands}) >= 9
    assert any(c.sort != 0 for c in cands) and any(c.nbuckets > 1 for c in cands)
    assert any(c.prefix_table == 0 for c in cands) and any(c.inline_pack == 0 for c in cands)
    for i, c in enumerate(cands):
        d_out = torch.full((reads.count, 4), -7, dtype=torch.int32, device=device)
        S.match_batch_dev(d, d_reads, d_offs, d_out, config=c)
        torch.cuda.synchronize()
        assert_same(d_out.cpu().numpy(), want, f"candidate {i}: {c.as_dict()}")
    say(f"  all {len(cands)} candidates identical to the oracle")


def test_tuner_run_keeps_a_matching_configuration(device, workload):
    d, reads, want = workload
    d_reads = torch.from_numpy(reads.data).to(device)
    d_offs = torch.from_numpy(reads.offs).to(device)
    say("case: full tuner run (no cache)")
    best, ms = S.sa_tune(d, d_reads, d_offs)  # compares every candidate's results on the device
    assert ms > 0
    assert S.cfg(d).as_dict() == best.as_dict()
    d_out = torch.full((reads.count, 4), -7, dtype=torch.int32, device=device)
    S.match_batch_dev(d, d_reads, d_offs, d_out)
    torch.cuda.synchronize()
    assert_same(d_out.cpu().numpy(), want, f"tuned {best.as_dict()}")


def test_short_read_candidates(device):
    """A batch of 150-base reads (the 250 Mbp recipe's reads, on a 2 Mbp
    text of that recipe) adds the register-light 5-word kernel to the
    candidates; each gives the oracle's bits, and so do reads longer than
    160 bases mixed in, which that kernel leaves to the long-read kernel."""
    ref = gen.make_reference("c4", n=2_000_000)
    reads = gen.make_reads(ref, gen.READ_SPECS["c4"], 50_000)
    text = ref.ascii()
    sa = oracle.sa_build(text)
    want = oracle.match(text, sa, reads.data, reads.offs)
    d = S.sa_build_device(text, 0)
    d_reads = torch.from_numpy(reads.data).to(device)
    d_offs = torch.from_numpy(reads.offs).to(device)
    cands = [c for c in S.sa_tune_candidates(d, d_offs) if c.max_words == 5]
    say(f"case: {len(cands)} five-word candidates")
    assert len(cands) >= 3
    for i, c in enumerate(cands):
        d_out = torch.full((reads.count, 4), -7, dtype=torch.int32, device=device)
        S.match_batch_dev(d, d_reads, d_offs, d_out, config=c)
        torch.cuda.synchronize()
        assert_same(d_out.cpu().numpy(), want, f"candidate {i}: {c.as_dict()}")
    # 150-base reads with one read of 161-320 bases in every 7: the latter take the long-read kernel
    mixed = gen.make_reads(ref, gen.ReadSpec(4, 7_000, 161, 320, 0.2, 0.01, 0.01))
    data = np.concatenate([reads.data, mixed.data])
    offs = np.concatenate([reads.offs, reads.offs[-1] + mixed.offs[1:]])
    want2 = oracle.match(text, sa, data, offs)
    d_out = torch.full((len(offs) - 1, 4), -7, dtype=torch.int32, device=device)
    S.match_batch_dev(d, torch.from_numpy(data).to(device), torch.from_numpy(offs).to(device), d_out,
                      config=cands[0])
    torch.cuda.synchronize()
    assert_same(d_out.cpu().numpy(), want2, "five words, longer reads mixed in")
