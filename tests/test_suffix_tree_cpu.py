"""The flattened suffix tree built on the host (no GPU): its nodes are
exactly the lcp-intervals of the suffix array (checked by brute force from
the suffix strings), its child slots partition each node's rows by the next
base, and a walk over the node array written here from the definitions
gives the oracle's match results."""
import random

import numpy as np
import pytest

import gen
import paper_1303_3692_amd as S
from oracle import brute, oracle


def lcp_intervals(text):
    """Brute force: every run [lb, rb) of at least two SA rows whose suffixes
    share exactly d leading bases, maximal (rows outside share fewer), as
    {(lb, rb): d}, plus the root [0, n) at depth 0."""
    sa = brute.suffix_array(text)
    n = len(text)
    suf = [text[p:] for p in sa]

    def lcp(a, b):
        k = 0
        while k < len(a) and k < len(b) and a[k] == b[k]:
            k += 1
        return k

    L = [0] + [lcp(suf[r - 1], suf[r]) for r in range(1, n)]
    out = {(0, n): 0}
    for lb in range(n):
        for rb in range(lb + 2, n + 1):
            d = min(L[lb + 1:rb])
            left = L[lb] if lb > 0 else -1
            right = L[rb] if rb < n else -1
            if left < d and right < d:
                out[(lb, rb)] = d
    return sa, out


@pytest.mark.parametrize("seed", range(12))
def test_nodes_are_the_lcp_intervals(seed):
    rng = random.Random(seed)
    alpha = "ACGT"[: rng.choice([1, 2, 4])]
    text = "".join(rng.choice(alpha) for _ in range(rng.randint(1, 45)))
    sa, want = lcp_intervals(text)
    t = S.st_build(S.sa_build(text))
    nodes = t.nodes()
    root = t.root()
    assert tuple(nodes[root][:3]) == (0, len(text), 0)
    got = {(int(u[0]), int(u[1])): int(u[2]) for u in nodes}
    assert got == want
    # child slots: the rows of each base at offset depth, as a node or a leaf
    for u in nodes:
        lb, rb, d = int(u[0]), int(u[1]), int(u[2])
        for b, ch in enumerate(u[4:]):
            rows = [r for r in range(lb, rb) if sa[r] + d < len(text) and text[sa[r] + d] == "ACGT"[b]]
            if not rows:
                assert ch == -1
            elif len(rows) == 1:
                assert ch == -2 - rows[0]
            else:
                assert ch >= 0 and (int(nodes[ch][0]), int(nodes[ch][1])) == (rows[0], rows[-1] + 1)


def walk(text, sa, nodes, root, read):
    """The tree search from the definitions: descend by the next base while
    the read agrees with the child's first suffix through the child's depth."""
    n = len(text)
    p_ = read.upper()
    mv = 0
    while mv < len(p_) and p_[mv] in "ACGT":
        mv += 1
    lb, rb, d, node = 0, n, 0, root
    while True:
        if d >= mv:
            ell = mv
            break
        ch = int(nodes[node][4 + "ACGT".index(p_[d])])
        if ch == -1:
            ell = d
            break
        if ch >= 0:
            clb, crb, cd = int(nodes[ch][0]), int(nodes[ch][1]), int(nodes[ch][2])
        else:
            clb = -2 - ch
            crb, cd = clb + 1, n - sa[clb]
        suffix = text[sa[clb]:]
        k = 0
        while k < mv and k < len(suffix) and p_[k] == suffix[k]:
            k += 1
        lb, rb = clb, crb
        if ch < 0 or k < cd or mv <= cd:
            ell = min(k, mv)
            break
        node, d = ch, cd
    if ell == 0:
        return (0, n, 0, int(len(p_) == 0))
    return (lb, rb, ell, int(ell == len(p_)))


@pytest.mark.parametrize("kind", ["iid", "two", "allA", "period3", "generated"])
def test_walk_gives_the_oracle_results(kind):
    rng = random.Random(sum(map(ord, kind)))
    if kind == "generated":
        text = gen.make_reference("c2", n=3000).ascii().tobytes().decode()
    elif kind == "allA":
        text = "A" * 300
    elif kind == "period3":
        text = "ACG" * 150
    else:
        text = "".join(rng.choice("ACGT" if kind == "iid" else "AC") for _ in range(500))
    sa = [int(x) for x in oracle.sa_build(text)]
    t = S.st_build(S.sa_build(text))
    nodes, root = t.nodes(), t.root()
    reads = []
    for _ in range(300):
        i = rng.randrange(len(text))
        r = text[i:i + rng.randint(0, 40)]
        u = rng.random()
        if u < 0.3 and r:
            j = rng.randrange(len(r))
            r = r[:j] + rng.choice("ACGT") + r[j + 1:]
        elif u < 0.4:
            r = r + "N" + r
        elif u < 0.5:
            r = "".join(rng.choice("ACGT") for _ in range(rng.randint(1, 30)))
        reads.append(r)
    data, offs = oracle.pack_reads(reads)
    want = oracle.match(text, np.array(sa, dtype=np.int32), data, offs)
    for k, r in enumerate(reads):
        assert walk(text, sa, nodes, root, r) == tuple(int(x) for x in want[k]), (kind, r)


def test_node_count_and_space():
    """At most n - 1 internal nodes (and the root); the device footprint
    counts nodes, suffix array and text."""
    text = gen.make_reference("c2", n=20_000).ascii()
    t = S.st_build(S.sa_build(text))
    assert 1 <= t.node_count() <= len(text)
    assert t.device_bytes() == 32 * t.node_count() + 4 * len(text) + 8 * ((len(text) + 31) // 32)
