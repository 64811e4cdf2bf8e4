"""Locate on the device (text positions of each read's occurrences, as a CSR
list in suffix-array order) against the oracle's locate over the oracle's
own match results: exact reads, longest-prefix mode, caps, repetitive texts
with many occurrences, buffer-too-small and bad-interval errors."""
import numpy as np
import pytest

import gen
import paper_1303_3692_amd as S
from oracle import oracle
from tests.golden import paper

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def check(d, text, sa, data, offs, cases):
    want_res = oracle.match(text, sa, data, offs)
    hits = S.match_batch(d, data, offs)
    assert (hits[:, :3] == want_res[:, :3]).all()
    dev = torch.device("cuda:0")
    d_hits = torch.from_numpy(hits.copy()).to(dev)
    for cap, min_len in cases:
        w_offs, w_pos = oracle.locate(sa, want_res, cap=cap, min_len=min_len)
        g_offs, g_pos = S.locate(d, hits, cap, min_len)
        assert (g_offs == w_offs).all(), (cap, min_len)
        assert (g_pos == w_pos).all(), (cap, min_len)
        # device form, exact-size buffer
        d_offs = torch.zeros(len(hits) + 1, dtype=torch.int64, device=dev)
        d_pos = torch.zeros(max(1, len(w_pos)), dtype=torch.int32, device=dev)
        total = S.locate_dev(d, d_hits, cap, min_len, d_offs, d_pos)
        torch.cuda.synchronize()
        assert total == len(w_pos)
        assert (d_offs.cpu().numpy() == w_offs).all()
        assert (d_pos.cpu().numpy()[:total] == w_pos).all()


def test_paper_example():
    print("case: locate paper example", flush=True)
    P = paper.load()
    text = P["text"]
    sa = oracle.sa_build(text)
    d = S.sa_upload(S.sa_build(text), 0)
    data, offs = oracle.pack_reads(["a", "ggtac", "tt", "", "acggtacgtacg", "c"])
    check(d, text, sa, data, offs, [(100, 0), (1, 0), (2, 1), (100, 2)])
    g_offs, g_pos = S.locate(d, S.match_batch(d, data, offs), 100)
    assert list(g_pos[g_offs[0]:g_offs[1]]) == P["occ"]["a"]


def test_generated_workload():
    print("case: locate generated workload", flush=True)
    ref, reads = gen.workload("c3", n=1_500_000, count=150_000)
    text = ref.ascii()
    sa = oracle.sa_build(text)
    d = S.sa_build_device(text, 0)
    check(d, text, sa, reads.data, reads.offs, [(1, 0), (8, 0), (64, 0), (16, 12), (4, 20)])


@pytest.mark.parametrize("kind", ["allA", "period3"])
def test_repetitive_text_many_occurrences(kind):
    print("case: locate repetitive", kind, flush=True)
    n = 20_000
    codes = np.zeros(n, np.uint8) if kind == "allA" else np.tile(np.array([0, 1, 2], np.uint8), n // 3 + 1)[:n]
    text = gen.to_ascii(codes)
    sa = oracle.sa_build(text)
    d = S.sa_build_device(text, 0)
    rng = np.random.default_rng(3)
    rd = []
    for _ in range(300):
        i = int(rng.integers(0, n - 40))
        rd.append(text[i:i + int(rng.integers(1, 40))].tobytes().decode())
    data, offs = oracle.pack_reads(rd)
    check(d, text, sa, data, offs, [(5000, 0), (20_000, 0), (7, 0)])


def test_buffer_too_small_and_bad_interval():
    print("case: locate errors", flush=True)
    ref, reads = gen.workload("c2", n=300_000, count=5_000)
    d = S.sa_build_device(ref.ascii(), 0)
    hits = S.match_batch(d, reads.data, reads.offs)
    dev = torch.device("cuda:0")
    d_hits = torch.from_numpy(hits.copy()).to(dev)
    d_offs = torch.zeros(len(hits) + 1, dtype=torch.int64, device=dev)
    w_offs, w_pos = S.locate(d, hits, 8)
    assert len(w_pos) > 10
    d_pos = torch.full((10,), -5, dtype=torch.int32, device=dev)
    with pytest.raises(S.SaError) as e:
        S.locate_dev(d, d_hits, 8, 0, d_offs, d_pos)
    assert e.value.code == S.SA_ENOSPC
    torch.cuda.synchronize()
    assert (d_offs.cpu().numpy() == w_offs).all()
    assert (d_pos.cpu().numpy() == -5).all()  # nothing written
    bad = hits.copy()
    k = int(np.nonzero(bad[:, 3] & 1)[0][0])
    bad[k, 1] = len(d) + 5
    with pytest.raises(S.SaError) as e:
        S.locate(d, bad, 8)
    assert e.value.code == S.SA_EINVAL
    # empty batch
    o, p = S.locate(d, np.zeros((0, 4), np.int32), 8)
    assert list(o) == [0] and len(p) == 0
