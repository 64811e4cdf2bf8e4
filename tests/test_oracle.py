"""Pins for the CPU oracle: values printed in the paper, brute force written
from the definitions (tests/golden and oracle/brute.py share no code with the
C oracle), and invariants that hold at any size."""
import itertools
import random

import numpy as np
import pytest

import gen
from oracle import brute, oracle
from tests.golden import paper

P = paper.load()
T = P["text"]


@pytest.fixture(scope="module")
def sa_example():
    return [int(x) for x in oracle.sa_build(T)]


# --------------------------------------------------------------- paper values


def test_table1_suffix_array(sa_example):
    assert sa_example == P["sa"]


def test_table3_ranks_are_inverse_sa(sa_example):
    rank = [0] * len(T)
    for k, i in enumerate(sa_example):
        rank[i] = k + 1
    assert rank == P["rank_all"]


def test_table2_sample_ranks(sa_example):
    sample = [i for i in sa_example if i % 3 != 0]
    got = [None] * len(T)
    for r, i in enumerate(sample):
        got[i] = r + 1
    assert got == P["rank_sample"]
    assert sorted(i for i in range(len(T)) if i % 3 == 1) == P["b1"]
    assert sorted(i for i in range(len(T)) if i % 3 == 2) == P["b2"]


def test_dc3_step2_nonsample_order(sa_example):
    assert [i for i in sa_example if i % 3 == 0] == P["b0_order"]


def test_section4_rows(sa_example):
    for k, s in P["row"].items():
        assert T[sa_example[k]:] == s


@pytest.mark.parametrize("q", sorted(P["search"]))
def test_section4_search_examples(sa_example, q):
    data, offs = oracle.pack_reads([q])
    for mode in (0, 1):
        lo, hi, l, exact = oracle.match(T, sa_example, data, offs, mode=mode)[0]
        assert (lo, hi - 1) == P["search"][q]
        assert l == len(q) and exact == 1
    assert oracle.scan_one(T, q)[:2] == (P["search"][q][0], P["search"][q][1] + 1)


def test_section4_occurrences(sa_example):
    data, offs = oracle.pack_reads(["a"])
    lo, hi, _, _ = oracle.match(T, sa_example, data, offs)[0]
    assert sorted(sa_example[lo:hi]) == sorted(P["occ"]["a"])


def test_section4_locate_lists_occurrences_in_printed_order(sa_example):
    """Section IV prints the positions of P = a as 9, 0, 5: the SA entries of
    its interval in row order."""
    data, offs = oracle.pack_reads(["a", "ggtac", "tt"])
    res = oracle.match(T, sa_example, data, offs)
    loffs, pos = oracle.locate(sa_example, res, cap=100)
    assert list(pos[loffs[0]:loffs[1]]) == P["occ"]["a"]
    assert list(pos[loffs[1]:loffs[2]]) == [2]
    assert loffs[3] == loffs[2]  # "tt" does not occur: nothing listed
    loffs, pos = oracle.locate(sa_example, res, cap=2)
    assert list(pos[loffs[0]:loffs[1]]) == P["occ"]["a"][:2]


@pytest.mark.parametrize("seed", range(6))
def test_locate_against_brute(seed):
    """Exact reads list every occurrence in suffix order (cap permitting);
    with min_len, reads that do not occur list the occurrences of their
    longest matched prefix."""
    rng = random.Random(seed)
    text = "".join(rng.choice("AC" if seed % 2 else "ACGT") for _ in range(rng.randint(1, 60)))
    sa = oracle.sa_build(text)
    reads = []
    for _ in range(80):
        i = rng.randrange(len(text))
        r = text[i:i + rng.randint(0, 8)]
        if rng.random() < 0.4 and r:
            j = rng.randrange(len(r))
            r = r[:j] + rng.choice("ACGT") + r[j + 1:]
        reads.append(r)
    data, offs = oracle.pack_reads(reads)
    res = oracle.match(text, sa, data, offs)
    for cap in (1, 3, 1000):
        for min_len in (0, 1, 3):
            loffs, pos = oracle.locate(sa, res, cap=cap, min_len=min_len)
            for k, r in enumerate(reads):
                lo, hi, ln, ex = res[k]
                sel = ln >= min_len if min_len else ex == 1
                want = brute.occurrences(text, r[:ln])[:cap] if sel else []
                assert list(pos[loffs[k]:loffs[k + 1]]) == want, (text, r, cap, min_len)


# --------------------------------------------------------------- brute force


def _check_against_brute(text, reads, sa=None):
    sa = oracle.sa_build(text) if sa is None else sa
    assert [int(x) for x in sa] == brute.suffix_array(text.upper())
    data, offs = oracle.pack_reads(reads)
    fast = oracle.match(text, sa, data, offs, mode=0)
    check = oracle.match(text, sa, data, offs, mode=1)
    assert (fast == check).all()
    for r, row in zip(reads, fast):
        want = brute.match(text, r)
        assert tuple(int(x) for x in row) == want, (text, r, row, want)
        lo, hi, l, _ = want
        occ = {i for i in range(len(text)) if text.upper().startswith(r.upper()[:l], i)}
        assert brute.rows_of(text.upper(), [int(x) for x in sa], lo, hi) == occ


def _random_text(rng, n, kind):
    if kind == "iid":
        return "".join(rng.choice("ACGT") for _ in range(n))
    if kind == "allA":
        return "A" * n
    if kind == "alt":
        return ("AC" * n)[:n]
    if kind == "tandem":
        unit = "".join(rng.choice("ACGT") for _ in range(rng.randint(1, 5)))
        pre = "".join(rng.choice("ACGT") for _ in range(rng.randint(0, 5)))
        return (pre + unit * n)[:n]
    if kind == "binary":
        return "".join(rng.choice("AG") for _ in range(n))
    raise ValueError(kind)


def _reads_for(rng, text, k):
    out = ["", text, text + "A", text[:-1] + "N" if text else "N"]
    for _ in range(k):
        kind = rng.randrange(6)
        if kind == 0:  # substring
            i = rng.randrange(len(text))
            out.append(text[i:i + rng.randint(1, 12)])
        elif kind == 1:  # substring with a substitution
            i = rng.randrange(len(text))
            s = list(text[i:i + rng.randint(1, 12)])
            j = rng.randrange(len(s))
            s[j] = rng.choice("ACGT".replace(s[j], ""))
            out.append("".join(s))
        elif kind == 2:  # random
            out.append("".join(rng.choice("ACGT") for _ in range(rng.randint(1, 10))))
        elif kind == 3:  # lower case or with N
            i = rng.randrange(len(text))
            s = text[i:i + rng.randint(1, 10)].lower()
            if rng.random() < 0.5 and s:
                j = rng.randrange(len(s))
                s = s[:j] + rng.choice("Nn-") + s[j + 1:]
            out.append(s)
        elif kind == 4:  # runs past the end of the text
            i = rng.randrange(max(0, len(text) - 3), len(text))
            out.append(text[i:] + "".join(rng.choice("ACGT") for _ in range(rng.randint(1, 4))))
        else:  # longer than the text
            out.append(text * 2)
    return out


@pytest.mark.parametrize("kind", ["iid", "allA", "alt", "tandem", "binary"])
def test_random_tiny_against_brute(kind):
    rng = random.Random(sum(map(ord, kind)))
    for trial in range(25):
        n = rng.randint(1, 60)
        text = _random_text(rng, n, kind)
        _check_against_brute(text, _reads_for(rng, text, 25))


def test_exhaustive_small_texts():
    reads = [""] + ["".join(p) for k in (1, 2, 3) for p in itertools.product("ACGT", repeat=k)]
    data, offs = oracle.pack_reads(reads)
    for n in range(1, 6):
        for tup in itertools.product("ACGT", repeat=n):
            text = "".join(tup)
            sa = oracle.sa_build(text)
            assert [int(x) for x in sa] == brute.suffix_array(text)
            got = oracle.match(text, sa, data, offs)
            for r, row in zip(reads, got):
                assert tuple(int(x) for x in row) == brute.match(text, r)


def test_scan_agrees_with_brute():
    rng = random.Random(7)
    for _ in range(40):
        text = _random_text(rng, rng.randint(1, 80), rng.choice(["iid", "tandem", "binary"]))
        for r in _reads_for(rng, text, 10):
            assert oracle.scan_one(text, r) == brute.match(text, r)


# --------------------------------------------------------------- invariants at size


def test_sa_check_detects_damage():
    text = gen.to_ascii(gen.iid_reference(5000, gen.rng_for(99, 0)))
    sa = oracle.sa_build(text)
    assert oracle.sa_check(text, sa) == 0
    bad = sa.copy()
    bad[10], bad[11] = bad[11], bad[10]
    assert oracle.sa_check(text, bad) == 2
    dup = sa.copy()
    dup[3] = dup[4]
    assert oracle.sa_check(text, dup) == 1


def test_invariants_on_generated_workload():
    ref, reads = gen.workload("c2", n=200_000, count=3000)
    text = ref.ascii()
    sa = oracle.sa_build(text)
    assert oracle.sa_check(text, sa) == 0
    out = oracle.match(text, sa, reads.data, reads.offs, mode=0)
    assert (out == oracle.match(text, sa, reads.data, reads.offs, mode=1)).all()
    lens = reads.lengths()
    for i in range(reads.count):
        lo, hi, l, ex = (int(x) for x in out[i])
        assert 0 <= lo <= hi <= ref.n and 0 <= l <= lens[i]
        assert ex == (l == lens[i])
        assert hi > lo  # the matched prefix always occurs (the empty one at every row)
        if reads.cls[i] != gen.RANDOM and reads.first_sub[i] == lens[i]:
            # an unmodified sampled read occurs, at its source position among others
            assert ex == 1 and reads.pos[i] in set(int(x) for x in sa[lo:hi])
        if reads.cls[i] != gen.RANDOM:
            assert l >= reads.first_sub[i]
    # interval widths equal occurrence counts and l is maximal (spot checks by scan)
    rng = np.random.default_rng(5)
    for i in rng.choice(reads.count, 12, replace=False):
        r = reads.read(int(i))
        assert oracle.scan_one(text, r) == tuple(int(x) for x in out[i])


def test_expected_exact_fraction_c1_recipe():
    ref, reads = gen.workload("c1", count=20_000)
    text = ref.ascii()
    sa = oracle.sa_build(text)
    out = oracle.match(text, sa, reads.data, reads.offs)
    frac = out[:, 3].mean()
    # 37.5 % unmodified copies; a random 25-mer occurs by chance with probability ~1e6/4^25
    assert abs(frac - 0.375) < 0.02
