"""HIP path against the CPU oracle, bit for bit: {lo, hi, len} and the exact
flag of every read (the results are unique, so any tile depth, pivot rule,
read order, bucket layout or launch shape must give the same bits)."""
import random
import sys

import numpy as np
import pytest

import gen
import paper_1303_3692_amd as S
from oracle import brute, oracle

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


def run_dev(d, data, offs, device, config=None):
    data = np.asarray(data, dtype=np.uint8)
    offs = np.asarray(offs, dtype=np.int64)
    n = len(offs) - 1
    d_reads = torch.from_numpy(data if len(data) else np.zeros(1, np.uint8)).to(device)
    d_offs = torch.from_numpy(offs).to(device)
    d_out = torch.full((max(n, 1), 4), -7, dtype=torch.int32, device=device)
    S.match_batch_dev(d, d_reads, d_offs, d_out, nreads=n, config=config)
    torch.cuda.synchronize()
    return d_out.cpu().numpy()[:n]


def assert_same(got, want, label=""):
    exact = (got[:, 3] & S.SA_HIT_EXACT).astype(np.int32)
    bad = np.nonzero((got[:, :3] != want[:, :3]).any(axis=1) | (exact != want[:, 3]))[0]
    assert len(bad) == 0, f"{label}: {len(bad)} mismatches, first rows {bad[:5]}: got {got[bad[:3]]} want {want[bad[:3]]}"


CONFIGS = [
    ("plain", dict(kernel=S.SA_KERNEL_PLAIN)),
    ("tuned-default", dict()),
    ("tuned-no-table", dict(prefix_table=0)),
    ("tuned-t1-unsorted", dict(tile_levels=1, sort=0, block=256, blocks_per_cu=1)),
    ("tuned-t5-b512", dict(tile_levels=5, block=512, blocks_per_cu=2)),
    ("tuned-t13-b1024", dict(tile_levels=13, block=1024, blocks_per_cu=1)),
    ("tuned-buckets", dict(nbuckets=3, bucket_edge=[64, 160, 320], blocks_per_cu=4)),
    ("tuned-sort-adaptive", dict(sort=1)),
    ("tuned-sort8", dict(sort=8, group=1)),
    ("tuned-sort24-buckets", dict(sort=24, nbuckets=2, bucket_edge=[96, 1024])),
    ("tuned-pack-pass", dict(sort=0, inline_pack=0)),
    ("tuned-inline-t12-b1024", dict(tile_levels=12, block=1024, blocks_per_cu=1, sort=0, inline_pack=1)),
    ("tuned-inline-no-table", dict(prefix_table=0, sort=0, inline_pack=1, group=1)),
    ("tuned-words5-b512", dict(max_words=5, sort=0, inline_pack=1, block=512, blocks_per_cu=3)),
    ("tuned-words5-b256-no-table", dict(max_words=5, sort=0, inline_pack=1, prefix_table=0, block=256,
                                        blocks_per_cu=6, group=1)),
    # reads set aside after 1 probe (most reads with a search), or never
    ("tuned-defer1-b1024", dict(defer=1, sort=0, inline_pack=1, block=1024, blocks_per_cu=1)),
    ("tuned-defer1-words5", dict(defer=1, max_words=5, sort=0, inline_pack=1, block=256, blocks_per_cu=6, group=1)),
    ("tuned-defer1-no-table", dict(defer=1, prefix_table=0, sort=0, inline_pack=1, group=2)),
    ("tuned-no-defer", dict(defer=0, sort=0, inline_pack=1)),
]


def configs_for(d):
    out = []
    for name, kw in CONFIGS:
        kw = dict(kw)
        if "tile_levels" in kw:
            kw["tile_levels"] = min(kw["tile_levels"], d.default_cfg().tile_levels if len(d) < 8191 else 13)
        out.append((name, S.cfg(d, **kw)))
    return out


def check_text(text, reads, device, label):
    t = text.upper() if isinstance(text, str) else text
    ix = S.sa_build(t)
    d = S.sa_upload(ix, 0)
    data, offs = oracle.pack_reads(reads)
    want = oracle.match(t, oracle.sa_build(t), data, offs)
    for name, c in configs_for(d):
        if len(d) < (1 << 13) - 1 and c.kernel == S.SA_KERNEL_TUNED:
            c.tile_levels = min(c.tile_levels, max(1, int(np.ceil(np.log2(len(d) + 1)))))
        assert_same(run_dev(d, data[:-1] if len(data) else data, offs, device, c), want, f"{label}/{name}")
    return d, want


def test_paper_example(device):
    say("case: paper example")
    reads = ["a", "c", "ggtac", "tac", "g", "ac", "acg", "gt", "gtac", "gtacg", "ta", "acgta", "", "tt", "cc",
             "aca", "acgtt", "tacgtacgt", "acggtacgtacg", "ACGGTACGTAC", "GN", "n"]
    d, want = check_text("acggtacgtac", reads, device, "paper")
    # printed ranges (Section IV): LB..RB inclusive
    got = {r: tuple(int(x) for x in row) for r, row in zip(reads, want)}
    assert (got["a"][0], got["a"][1] - 1) == (0, 2)
    assert (got["c"][0], got["c"][1] - 1) == (3, 5)
    assert (got["ggtac"][0], got["ggtac"][1] - 1) == (6, 6)
    assert (got["tac"][0], got["tac"][1] - 1) == (9, 10)
    for r in reads:
        assert got[r] == brute.match("acggtacgtac", r)


@pytest.mark.parametrize("kind", ["iid", "allA", "alt", "tandem"])
def test_tiny_texts_against_brute(device, kind):
    say("case: tiny", kind)
    rng = random.Random(sum(map(ord, kind)))
    for trial in range(6):
        n = rng.randint(1, 90)
        if kind == "iid":
            text = "".join(rng.choice("ACGT") for _ in range(n))
        elif kind == "allA":
            text = "A" * n
        elif kind == "alt":
            text = ("AC" * n)[:n]
        else:
            unit = "".join(rng.choice("ACGT") for _ in range(rng.randint(1, 4)))
            text = (unit * n)[:n]
        reads = ["", text, text + "A", text.lower(), text[: n // 2] + "N"]
        for _ in range(60):
            i = rng.randrange(n)
            r = text[i:i + rng.randint(1, 70)]
            if rng.random() < 0.3:
                j = rng.randrange(len(r))
                r = r[:j] + rng.choice("ACGTN") + r[j + 1:]
            if rng.random() < 0.2:
                r = r + "".join(rng.choice("ACGT") for _ in range(rng.randint(1, 40)))
            reads.append(r)
        check_text(text, reads, device, f"{kind}/{trial}")


def test_long_and_too_long_reads(device):
    say("case: long reads")
    ref = gen.make_reference("c2", n=300_000)
    text = ref.ascii().tobytes().decode()
    rng = np.random.default_rng(3)
    reads = []
    # 1-320 bases: words in registers; 321-1024: the long-read kernel (LDS)
    for m in [31, 32, 33, 63, 64, 65, 255, 256, 257, 300, 319, 320, 321, 352, 400, 511, 512, 513, 777, 1000,
              1023, 1024]:
        for _ in range(8):
            p = int(rng.integers(0, ref.n - m))
            r = text[p:p + m]
            u = rng.random()
            if u < 0.4:
                j = int(rng.integers(0, m))
                r = r[:j] + "ACGT"[(ref.codes[p + j] + 1) % 4] + r[j + 1:]
            elif u < 0.5:
                j = int(rng.integers(0, m))
                r = r[:j] + "N" + r[j + 1:]
            elif u < 0.6:
                r = "".join(rng.choice(list("ACGT"), size=m))
            reads.append(r)
    reads.append(text[-40:] + "ACGT")  # runs off the end of the text
    reads.append(text[-320:])
    reads.append(text[-700:] + "ACGTACGT")
    reads.append(text[-1024:])
    reads.append(text[1000:2000].lower())
    check_text(text, reads, device, "long")
    # 1025 bases: flagged, not searched (device path); refused (host path)
    ix = S.sa_build(text)
    d = S.sa_upload(ix, 0)
    data, offs = oracle.pack_reads(["ACGT", "A" * 1025, "GG", text[5000:5900]])
    got = run_dev(d, data[:-1], offs, device)
    assert tuple(got[1]) == (0, 0, 0, S.SA_HIT_TOOLONG)
    want = oracle.match(text, oracle.sa_build(text), *oracle.pack_reads(["ACGT", "GG", text[5000:5900]]))
    assert_same(got[[0, 2, 3]], want, "around a too-long read")
    with pytest.raises(S.SaError) as e:
        S.match_batch(d, data[:-1], offs)
    assert e.value.code == S.SA_ETOOBIG


def test_invalid_settings_refused(device):
    """Launch settings outside their ranges are refused before any launch,
    with SA_EINVAL; the largest probe budget is accepted."""
    say("case: invalid settings")
    rng = random.Random(5)
    text = "".join(rng.choice("ACGT") for _ in range(8000))
    d = S.sa_upload(S.sa_build(text), 0)
    data, offs = oracle.pack_reads(["ACGT", "GGA", text[100:180]])
    for kw in (dict(defer=-1), dict(defer=1025), dict(max_words=7), dict(block=128), dict(sort=3),
               dict(tile_levels=14), dict(group=65), dict(inline_pack=2)):
        with pytest.raises(S.SaError) as e:
            run_dev(d, data[:-1], offs, device, S.cfg(d, **kw))
        assert e.value.code == S.SA_EINVAL, kw
    want = oracle.match(text, oracle.sa_build(text), data, offs)
    assert_same(run_dev(d, data[:-1], offs, device, S.cfg(d, defer=1024)), want, "largest budget")


@pytest.mark.parametrize("cfg,n,count", [("c1", 1_000_000, 100_000), ("c2", 2_000_000, 200_000),
                                         ("c3", 2_000_000, 150_000), ("c4", 3_000_000, 150_000)])
def test_generated_workloads(device, cfg, n, count):
    say("case: workload", cfg, n, count)
    ref, reads = gen.workload(cfg, n=n, count=count)
    text = ref.ascii()
    d = S.sa_upload(S.sa_build(text), 0)
    want = oracle.match(text, oracle.sa_build(text), reads.data, reads.offs)
    for name, c in configs_for(d):
        assert_same(run_dev(d, reads.data, reads.offs, device, c), want, f"{cfg}/{name}")
    # host entry point, same results
    got = S.match_batch(d, reads.data, reads.offs)
    assert_same(got, want, f"{cfg}/host")


def test_ragged_batch_sizes(device):
    say("case: ragged sizes")
    ref, reads = gen.workload("c3", n=500_000, count=70_001)
    text = ref.ascii()
    d = S.sa_upload(S.sa_build(text), 0)
    want = oracle.match(text, oracle.sa_build(text), reads.data, reads.offs)
    for k in [1, 2, 63, 64, 65, 4095, 4096, 4097, 70_001]:
        got = run_dev(d, reads.data, reads.offs[: k + 1], device)
        assert_same(got, want[:k], f"k={k}")
    # offsets that start inside the buffer
    off2 = reads.offs[1000:3001] - 0
    got = run_dev(d, reads.data, off2, device)
    assert_same(got, want[1000:3000], "offset start")


def test_streams_and_reuse(device):
    say("case: streams")
    ref, reads = gen.workload("c2", n=400_000, count=50_000)
    text = ref.ascii()
    d = S.sa_upload(S.sa_build(text), 0)
    want = oracle.match(text, oracle.sa_build(text), reads.data, reads.offs)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    d_reads = torch.from_numpy(reads.data).to(device)
    d_offs = torch.from_numpy(reads.offs).to(device)
    outs = []
    for s in (s1, s2, s1, s2):
        o = torch.zeros((reads.count, 4), dtype=torch.int32, device=device)
        torch.cuda.synchronize()
        S.match_batch_dev(d, d_reads, d_offs, o, stream=s)
        outs.append((s, o))
    torch.cuda.synchronize()
    for _, o in outs:
        assert_same(o.cpu().numpy(), want, "stream")


@pytest.mark.parametrize("kind", ["iid", "allA", "period3", "tandem", "two-letter"])
def test_prefix_table_edges(device, kind):
    """Texts just above the size that gets a prefix table, whose end suffixes
    (shorter than the table's k) are prefixes of many reads."""
    say("case: prefix table", kind)
    rng = random.Random(len(kind) * 7919)
    for n in (4096, 5000, 17_000):
        if kind == "iid":
            text = "".join(rng.choice("ACGT") for _ in range(n))
        elif kind == "allA":
            text = "A" * n
        elif kind == "period3":
            text = ("ACG" * n)[:n]
        elif kind == "tandem":
            text = "".join(rng.choice("ACGT") for _ in range(n // 2)) + ("GATT" * n)[: n - n // 2]
        else:
            text = "".join(rng.choice("AC") for _ in range(n))
        reads = ["", "A", "C", "G", "T", "AC", "TT"]
        for j in range(1, 20):
            tail = text[-j:]
            reads += [tail, tail + "A", tail + "C", tail + "T", tail[:-1] + "N" if j > 1 else "N",
                      "A" * j, "T" * j, tail + text[:5]]
        for _ in range(300):
            i = rng.randrange(n)
            r = text[i:i + rng.randint(1, 60)]
            if rng.random() < 0.4 and r:
                j = rng.randrange(len(r))
                r = r[:j] + rng.choice("ACGT") + r[j + 1:]
            reads.append(r)
        reads += ["".join(rng.choice("ACGT") for _ in range(rng.randint(5, 40))) for _ in range(100)]
        check_text(text, reads, device, f"{kind}/{n}")


def test_inline_pack_spans(device):
    """The search kernel's own packing against the pack pass and the oracle:
    waves whose 64 reads fill its packing area exactly (320-base reads: 20 KB
    for the kernel that holds 10 query words) or span more than it (300-base
    reads for the 5-word kernel's 10 KB, long reads among short ones),
    offsets that go backwards (a
    negative length is too long; the reads after it lie before the wave's
    span), and the whole batch moved 5 bytes into its buffer."""
    say("case: inline pack spans")
    ref = gen.make_reference("c2", n=400_000)
    text = ref.ascii().tobytes().decode()
    rng = np.random.default_rng(17)

    def sample(m):
        p = int(rng.integers(0, ref.n - m))
        r = text[p:p + m]
        u = rng.random()
        if u < 0.3:
            j = int(rng.integers(0, m))
            r = r[:j] + "ACGT"[(ref.codes[p + j] + 1) % 4] + r[j + 1:]
        elif u < 0.4:
            j = int(rng.integers(0, m))
            r = r[:j] + "n" + r[j + 1:]
        return r

    reads = [sample(300) for _ in range(200)]                                  # 19 KB per wave
    reads += [sample(320) for _ in range(128)]                                 # 20 KB: a full area
    reads += [sample(1000) if k % 4 == 0 else sample(300) for k in range(128)] # 30 KB per wave
    reads += [sample(900) if k % 10 == 3 else sample(100) for k in range(300)]  # long reads among short ones
    reads += [sample(int(rng.integers(1, 200))) for _ in range(300)]
    d = S.sa_upload(S.sa_build(text), 0)
    sa = oracle.sa_build(text)
    data, offs = oracle.pack_reads(reads)
    want = oracle.match(text, sa, data, offs)
    variants = [S.cfg(d, sort=0, inline_pack=v) for v in (1, 0)] + [S.cfg(d, sort=0, inline_pack=1, max_words=5)]
    variants += [S.cfg(d, sort=0, inline_pack=1, defer=1, max_words=w) for w in (5, 10)]
    for c in variants:
        assert_same(run_dev(d, data[:-1], offs, device, c), want, f"inline={c.inline_pack}/{c.max_words}")
        # the same reads 5 bytes into the buffer
        shifted = np.concatenate([np.frombuffer(b"NNNNN", np.uint8), data[:-1]])
        assert_same(run_dev(d, shifted, offs + 5, device, c), want, f"shifted inline={c.inline_pack}")
    # offsets that go backwards: read 70 runs from offs[70] back to an
    # earlier byte (too long); reads 71.. start before the wave's first read
    o2 = offs.copy()
    o2[71:] -= int(offs[71] - offs[10])
    starts, ends = o2[:-1], o2[1:]
    ok = ends >= starts
    assert not ok[70] and ok[:70].all() and ok[71:].all()
    buf = data[:-1]
    w_ok = oracle.match(text, sa, *oracle.pack_reads([bytes(buf[a:b]).decode() for a, b in zip(starts[ok], ends[ok])]))
    for c in variants:
        got = run_dev(d, buf, o2, device, c)
        assert tuple(got[70]) == (0, 0, 0, S.SA_HIT_TOOLONG), f"inline={c.inline_pack}"
        assert_same(got[ok], w_ok, f"backwards inline={c.inline_pack}")


def test_host_batch_in_chunks(device):
    """A host batch larger than one staging chunk (32 MiB of bytes or 2^19
    reads) streams through the two pinned slots: the oracle's results (and
    the device entry point's), for chunks cut by bytes, by read count, and
    for offsets that start inside the buffer."""
    say("case: host batch in chunks")
    ref, reads = gen.workload("c2", n=1_000_000, count=1_000_000)   # ~100 MB: cut by bytes
    text = ref.ascii()
    d = S.sa_upload(S.sa_build(text), 0)
    want = oracle.match(text, oracle.sa_build(text), reads.data, reads.offs)
    assert_same(run_dev(d, reads.data, reads.offs, device), want, "device entry point")
    assert_same(S.match_batch(d, reads.data, reads.offs), want, "by bytes")
    sub = reads.offs[123_457:800_001]
    assert_same(S.match_batch(d, reads.data, sub), want[123_457:800_000], "inside the buffer")
    ref1, short = gen.workload("c1", n=1_000_000, count=1_200_000)  # 25-base reads: cut by count
    text1 = ref1.ascii()
    d1 = S.sa_upload(S.sa_build(text1), 0)
    want1 = oracle.match(text1, oracle.sa_build(text1), short.data, short.offs)
    assert_same(S.match_batch(d1, short.data, short.offs), want1, "by count")


@pytest.mark.parametrize("kind", ["iid", "tandem"])
def test_prefix_table_lengths(device, kind):
    """The prefix table rebuilt for every length from 4 to 16 bases (and
    dropped; 16 bases: 4^16 + 1 entries, built in several dispatches): the
    oracle's bits each time, with the table's first-pivot entries, empty
    brackets and end suffixes shorter than k exercised.  Lengths past 16 are
    refused."""
    say("case: prefix table lengths", kind)
    rng = random.Random(41 if kind == "iid" else 43)
    n = 60_000
    if kind == "iid":
        text = "".join(rng.choice("ACGT") for _ in range(n))
    else:
        text = "".join(rng.choice("ACGT") for _ in range(n // 2)) + ("GATTACA" * n)[: n - n // 2]
    reads = []
    for j in range(1, 16):
        tail = text[-j:]
        reads += [tail, tail + "A", tail + "T", tail + text[:7]]
    for _ in range(4000):
        i = rng.randrange(n)
        r = text[i:i + rng.randint(1, 120)]
        if rng.random() < 0.4 and r:
            j = rng.randrange(len(r))
            r = r[:j] + rng.choice("ACGT") + r[j + 1:]
        reads.append(r)
    reads += ["".join(rng.choice("ACGT") for _ in range(rng.randint(3, 60))) for _ in range(2000)]
    data, offs = oracle.pack_reads(reads)
    want = oracle.match(text, oracle.sa_build(text), data, offs)
    d = S.sa_upload(S.sa_build(text), 0)
    for k in (4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 0):
        d.set_prefix_table(k)
        assert d.index_bytes()["prefix_table"] == (16 * (4 ** k + 1) if k else 0)
        for name, c in (("default", S.cfg(d)), ("b1024", S.cfg(d, block=1024, blocks_per_cu=1, group=1))):
            assert_same(run_dev(d, data, offs, device, c), want, f"{kind}/k={k}/{name}")
    for k in (1, 3, 17, 32):
        with pytest.raises(S.SaError):
            d.set_prefix_table(k)
