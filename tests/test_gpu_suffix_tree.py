"""Suffix-tree search on the device (the paper's comparison index) against
the oracle's suffix-array results, read by read: the paper example, tiny
texts against brute force, generated workloads with reads of 20-1024 bases,
non-ACGT bytes, reads longer than the limit, and equality with the
suffix-array path on the same batch."""
import numpy as np
import pytest

import gen
import paper_1303_3692_amd as S
from oracle import brute, oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def run_st(text, data, offs):
    ix = S.sa_build(text)
    d = S.sa_upload(ix, 0)
    sd = S.st_upload(S.st_build(ix), d)
    dev = torch.device("cuda:0")
    n = len(offs) - 1
    d_reads = torch.from_numpy(np.ascontiguousarray(data) if len(data) else np.zeros(1, np.uint8)).to(dev)
    d_offs = torch.from_numpy(np.ascontiguousarray(offs, dtype=np.int64)).to(dev)
    d_out = torch.full((max(n, 1), 4), -7, dtype=torch.int32, device=dev)
    S.st_match_batch_dev(sd, d_reads, d_offs, d_out, nreads=n)
    torch.cuda.synchronize()
    return d, d_reads, d_offs, d_out.cpu().numpy()[:n]


def assert_same(got, want, label):
    bad = np.nonzero((got[:, :3] != want[:, :3]).any(1) | ((got[:, 3] & 1) != want[:, 3]))[0]
    assert len(bad) == 0, f"{label}: {len(bad)} mismatches, first rows {bad[:5]}, got {got[bad[:3]]} want {want[bad[:3]]}"


def test_paper_example():
    print("case: st paper example", flush=True)
    text = "acggtacgtac"
    reads = ["a", "c", "ggtac", "tac", "g", "ac", "acg", "gt", "gtac", "gtacg", "ta", "acgta", "", "tt", "cc",
             "aca", "acgtt", "tacgtacgt", "acggtacgtacg", "ACGGTACGTAC", "GN", "n"]
    data, offs = oracle.pack_reads(reads)
    _, _, _, got = run_st(text.upper(), data[:-1], offs)
    for r, row in zip(reads, got):
        assert tuple(int(x) for x in row[:3]) + (int(row[3]) & 1,) == brute.match(text, r), r


@pytest.mark.parametrize("alpha", ["A", "AC", "ACGT"])
def test_tiny_texts_against_brute(alpha):
    print("case: st tiny", alpha, flush=True)
    rng = np.random.default_rng(len(alpha))
    for trial in range(6):
        n = int(rng.integers(1, 80))
        text = "".join(rng.choice(list(alpha), size=n))
        reads = []
        for _ in range(60):
            i = int(rng.integers(0, n))
            r = text[i:i + int(rng.integers(0, 12))]
            if rng.random() < 0.3:
                r += "".join(rng.choice(list("ACGT"), size=int(rng.integers(1, 5))))
            reads.append(r)
        data, offs = oracle.pack_reads(reads)
        _, _, _, got = run_st(text, data[:-1], offs)
        want = np.array([brute.match(text, r) for r in reads])
        assert_same(got, want, f"{alpha}/{trial}")


@pytest.mark.parametrize("cfg,n,count", [("c1", 500_000, 50_000), ("c2", 1_000_000, 100_000),
                                         ("c3", 1_000_000, 100_000), ("paper", 1_000_000, 8_000)])
def test_generated_workloads(cfg, n, count):
    print("case: st workload", cfg, flush=True)
    ref, reads = gen.workload(cfg, n=n, count=count)
    text = ref.ascii()
    want = oracle.match(text, oracle.sa_build(text), reads.data, reads.offs)
    d, d_reads, d_offs, got = run_st(text, reads.data, reads.offs)
    assert_same(got, want, cfg)
    # and the suffix-array path on the same device batch
    d_out = torch.zeros((reads.count, 4), dtype=torch.int32, device=d_reads.device)
    S.match_batch_dev(d, d_reads, d_offs, d_out)
    torch.cuda.synchronize()
    assert (d_out.cpu().numpy() == got).all()


def test_long_odd_and_too_long_reads():
    print("case: st long reads", flush=True)
    ref = gen.make_reference("c2", n=200_000)
    text = ref.ascii().tobytes().decode()
    rng = np.random.default_rng(9)
    reads = []
    for m in [1, 31, 32, 33, 319, 320, 321, 700, 1023, 1024]:
        for _ in range(6):
            p = int(rng.integers(0, ref.n - m))
            r = text[p:p + m]
            u = rng.random()
            if u < 0.3:
                j = int(rng.integers(0, m))
                r = r[:j] + "N" + r[j + 1:]
            elif u < 0.6:
                j = int(rng.integers(0, m))
                r = r[:j] + "ACGT"[(ref.codes[p + j] + 1) % 4] + r[j + 1:]
            reads.append(r.lower() if rng.random() < 0.2 else r)
    reads += [text[-50:] + "ACGTT", text[-1024:], "A" * 1025, ""]
    data, offs = oracle.pack_reads(reads)
    _, _, _, got = run_st(text, data[:-1], offs)
    want = oracle.match(text, oracle.sa_build(text), data, offs)
    long_one = len(reads) - 2
    assert tuple(got[long_one]) == (0, 0, 0, S.SA_HIT_TOOLONG)
    keep = np.array([k != long_one for k in range(len(reads))])
    assert_same(got[keep], want[keep], "long")
