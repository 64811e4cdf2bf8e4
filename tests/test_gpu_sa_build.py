"""Suffix arrays built on the device (prefix doubling with radix sorts) are
the array of Section III: identical to the oracle's (and to brute force on
tiny texts), to the host DC3 array, and, at 250 Mbp, a permutation whose
adjacent suffixes are strictly increasing (which fixes the array).  An
index built on the device answers reads exactly as one uploaded from the
host does."""
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


def device_sa(text):
    d = S.sa_build_device(text, 0)
    sa = S.sa_download(d).suffix_array()
    return d, sa


def text_of(codes):
    return gen.to_ascii(np.asarray(codes, dtype=np.uint8))


def test_tiny_texts_against_brute_force():
    print("case: tiny texts", flush=True)
    rng = np.random.default_rng(5)
    for n in list(range(1, 70)) + [127, 128, 129, 255, 256, 257]:
        for alpha in (1, 2, 4):
            t = text_of(rng.integers(0, alpha, size=n))
            _, sa = device_sa(t)
            want = brute.suffix_array(t.tobytes().decode())
            assert list(sa) == want, (n, alpha)


def test_paper_example():
    _, sa = device_sa(np.frombuffer(b"acggtacgtac", dtype=np.uint8))
    assert list(sa) == [9, 0, 5, 10, 1, 6, 2, 7, 3, 8, 4]


REPETITIVE = {
    "allA": lambda n, rng: np.zeros(n, np.uint8),
    "period3": lambda n, rng: np.tile(np.array([0, 1, 2], np.uint8), n // 3 + 1)[:n],
    "period7": lambda n, rng: np.tile(rng.integers(0, 4, 7).astype(np.uint8), n // 7 + 1)[:n],
    "two_letter": lambda n, rng: rng.integers(0, 2, n).astype(np.uint8),
    "tandem": lambda n, rng: np.concatenate([rng.integers(0, 4, n // 3).astype(np.uint8),
                                             np.tile(rng.integers(0, 4, 50).astype(np.uint8), (n - n // 3) // 50 + 1)
                                             ])[:n],
}


@pytest.mark.parametrize("kind", sorted(REPETITIVE))
@pytest.mark.parametrize("n", [4095, 4096, 4097, 70_001])
def test_repetitive_texts(kind, n):
    print("case: repetitive", kind, n, flush=True)
    rng = np.random.default_rng(n + sum(map(ord, kind)))
    t = text_of(REPETITIVE[kind](n, rng))
    d, sa = device_sa(t)
    assert (sa == oracle.sa_build(t)).all()
    info = d.build_info()
    assert info["steps"] >= 1 and info["sorted_pairs"] >= n


@pytest.mark.parametrize("cfg,n", [("c1", None), ("c2", None), ("c4", 3_000_000)])
def test_generated_references_against_dc3(cfg, n):
    print("case: generated", cfg, n, flush=True)
    t = gen.make_reference(cfg, n=n).ascii()
    _, sa = device_sa(t)
    host = S.sa_build(t).suffix_array()
    assert (sa == host).all()
    if len(t) <= 3_000_000:
        assert (sa == oracle.sa_build(t)).all()


def test_device_index_answers_like_uploaded_index():
    print("case: device-built index vs uploaded index", flush=True)
    ref, reads = gen.workload("c3", n=2_000_000, count=200_000)
    t = ref.ascii()
    d_dev = S.sa_build_device(t, 0)
    d_up = S.sa_upload(S.sa_build(t), 0)
    a = S.match_batch(d_dev, reads.data, reads.offs)
    b = S.match_batch(d_up, reads.data, reads.offs)
    assert (a == b).all()
    want = oracle.match(t, oracle.sa_build(t), reads.data, reads.offs)
    assert (a[:, :3] == want[:, :3]).all() and ((a[:, 3] & 1) == want[:, 3]).all()


def test_download_save_load_roundtrip(tmp_path):
    print("case: save a device-built index", flush=True)
    t = gen.make_reference("c2", n=300_000).ascii()
    d = S.sa_build_device(t, 0)
    ix = S.sa_download(d)
    path = str(tmp_path / "ix.bin")
    S.sa_save(ix, path)
    back = S.sa_load(path)
    assert (back.suffix_array() == oracle.sa_build(t)).all()


def test_rejects_bad_text():
    with pytest.raises(S.SaError) as e:
        S.sa_build_device(np.frombuffer(b"ACGN", dtype=np.uint8), 0)
    assert e.value.code == S.SA_EALPHABET
    with pytest.raises(S.SaError) as e:
        S.sa_build_device(np.zeros(0, dtype=np.uint8), 0)
    assert e.value.code == S.SA_EINVAL


def test_full_c4_reference_is_sorted():
    """250 Mbp: the device array is a permutation with every adjacent pair
    of suffixes strictly increasing, checked by the oracle on all n - 1
    pairs (too slow for the oracle to build itself)."""
    print("case: c4 250 Mbp", flush=True)
    t = gen.make_reference("c4").ascii()
    d, sa = device_sa(t)
    print("  built:", d.build_info(), flush=True)
    assert oracle.sa_check(t, sa) == 0


def test_random_read_rate_probe():
    """The measurement helper bench.py reports beside the search: a plausible
    rate for a small and a large table, the small one not slower."""
    print("case: random read rate", flush=True)
    small = S.sa_random_read_rate(0, 16)
    large = S.sa_random_read_rate(0, 24)
    assert 1e9 < large < 1e12 and 1e9 < small < 1e12
    assert small > 0.8 * large
