"""match_batch_dev_noalloc (the pipeline on the library's fixed device
scratch) against match_batch_dev on the same batches, bit for bit, called
through the C-ABI: two calls in a row, the second with a smaller batch, on
the inline-packing path and on the paths with a pack pass (sorted, plain
kernel), plus long reads and the size limit of the pack-pass path."""
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
def index(device):
    ref = gen.make_reference("c2", n=300_000)
    text = ref.ascii()
    d = S.sa_upload(S.sa_build(text), 0)
    return ref, text, d, oracle.sa_build(text)


def batch(ref, count, seed_spec):
    reads = gen.make_reads(ref, seed_spec, count)
    return reads.data, reads.offs


def run(fn, d, data, offs, device, config):
    n = len(offs) - 1
    d_reads = torch.from_numpy(np.asarray(data, dtype=np.uint8)).to(device)
    d_offs = torch.from_numpy(np.asarray(offs, dtype=np.int64)).to(device)
    d_out = torch.full((n, 4), -7, dtype=torch.int32, device=device)
    fn(d, d_reads, d_offs, d_out, config=config)
    torch.cuda.synchronize()
    return d_out.cpu().numpy()


PATHS = [
    ("inline", dict()),
    ("sorted", dict(sort=8)),
    ("pack-pass", dict(inline_pack=0)),
    ("plain", dict(kernel=S.SA_KERNEL_PLAIN)),
]


@pytest.mark.parametrize("name,kw", PATHS, ids=[p[0] for p in PATHS])
def test_noalloc_matches_match_batch_dev(device, index, name, kw):
    ref, text, d, sa = index
    cfg = S.cfg(d, **kw)
    # a larger batch of mixed lengths with long reads, then a smaller one
    big = batch(ref, 60_000, gen.READ_SPECS["c3"])
    long_ = gen.make_reads(ref, gen.ReadSpec(7, 300, 321, 1024, 0.3, 0.0, 0.01))
    data = np.concatenate([big[0], long_.data])
    offs = np.concatenate([big[1], big[1][-1] + long_.offs[1:]])
    small = batch(ref, 5_000, gen.READ_SPECS["c2"])
    for label, (dat, off) in (("first", (data, offs)), ("second, smaller", small)):
        say(f"case: noalloc {name} {label}: {len(off) - 1} reads")
        want = run(S.match_batch_dev, d, dat, off, device, cfg)
        got = run(S.match_batch_dev_noalloc, d, dat, off, device, cfg)
        assert (got == want).all(), f"{name} {label}: {(got != want).any(1).sum()} rows differ"
        oracle_rows = oracle.match(text, sa, dat[: off[200]], off[:201])
        assert (got[:200, :3] == oracle_rows[:, :3]).all()
        assert ((got[:200, 3] & 1) == oracle_rows[:, 3]).all()


def test_noalloc_limits(device, index):
    ref, text, d, sa = index
    max_pack = S.sa_noalloc_max_reads(True)
    assert 0 < max_pack < S.sa_noalloc_max_reads(False)
    say(f"case: noalloc limits: pack-pass path takes at most {max_pack} reads")
    n = max_pack + 1
    # empty reads: only the sizes matter for the check, which runs before any work
    d_reads = torch.zeros(1, dtype=torch.uint8, device=device)
    d_offs = torch.zeros(n + 1, dtype=torch.int64, device=device)
    d_out = torch.zeros((n, 4), dtype=torch.int32, device=device)
    with pytest.raises(S.SaError) as e:
        S.match_batch_dev_noalloc(d, d_reads, d_offs, d_out, config=S.cfg(d, kernel=S.SA_KERNEL_PLAIN))
    assert e.value.code == S.SA_ENOSPC
    with pytest.raises(S.SaError) as e:
        S.match_batch_dev_noalloc(d, d_reads, d_offs, d_out, config=S.cfg(d, count=1))
    assert e.value.code == S.SA_EINVAL
    # the inline path takes the same batch of empty reads: each is (0, n, 0), exact
    S.match_batch_dev_noalloc(d, d_reads, d_offs, d_out)
    torch.cuda.synchronize()
    got = d_out.cpu().numpy()
    assert (got[:, 0] == 0).all() and (got[:, 1] == len(text)).all() and (got[:, 2] == 0).all()
    assert ((got[:, 3] & 1) == 1).all()
