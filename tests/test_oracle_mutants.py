"""Plant plausible mistakes in a copy of the C oracle (on the CPU) and check
that the pins catch each one: the paper's printed values, brute force on
small texts, and the agreement of the two longest-prefix modes.

Changes that leave every result the same are not listed: the pivot rule (any
row strictly inside the open bounds gives the same answer) and the scan for
bytes outside ACGT (such a byte equals no reference byte, so the common
prefix stops there anyway)."""
import ctypes
import itertools
import os
import random
import subprocess

import numpy as np
import pytest

from oracle import brute, oracle
from tests.golden import paper

SRC = open(oracle.SRC).read()

MUTANTS = {
    # a proper prefix sorts last instead of first
    "shorter_last": ("return li < lj ? -1 : 1;", "return li < lj ? 1 : -1;"),
    # LB search moves R only on a strict "before"
    "lb_strict": ("if (cmp_row(t, n, sa, p, len, piv) <= 0) R = piv; else L = piv;",
                  "if (cmp_row(t, n, sa, p, len, piv) < 0) R = piv; else L = piv;"),
    # RB search also moves R on a prefix match
    "rb_inclusive": ("if (cmp_row(t, n, sa, p, len, piv) < 0) R = piv; else L = piv;\n    }\n    return R;\n}\n\nstatic int64_t lcp_at",
                     "if (cmp_row(t, n, sa, p, len, piv) <= 0) R = piv; else L = piv;\n    }\n    return R;\n}\n\nstatic int64_t lcp_at"),
    # a suffix that runs out is treated as matching
    "suffix_end_is_prefix": ("return c == len ? 0 : 1;", "return 0;"),
    # byte comparison with the sign flipped
    "cmp_sign": ("return p[i] < t[s + i] ? -1 : 1;", "return p[i] < t[s + i] ? 1 : -1;"),
    # only the right neighbour of the insertion point is used for l
    "one_neighbour": ("if (i0 > 0) { int64_t a = lcp_at(t, n, sa[i0 - 1], buf, mv); if (a > l) l = a; }", ""),
    # LB search starts with row 0 as a known "before" row
    "lb_left_closed": ("int64_t L = -1, R = n;\n    while (R > L + 1) {\n        int64_t piv = L + (R - L) / 2;\n        if (cmp_row(t, n, sa, p, len, piv) <= 0)",
                       "int64_t L = 0, R = n;\n    while (R > L + 1) {\n        int64_t piv = L + (R - L) / 2;\n        if (cmp_row(t, n, sa, p, len, piv) <= 0)"),
    # RB search treats the last row as a known "after" row
    "rb_right_closed": ("int64_t L = -1, R = n;\n    while (R > L + 1) {\n        int64_t piv = L + (R - L) / 2;\n        if (cmp_row(t, n, sa, p, len, piv) < 0)",
                        "int64_t L = -1, R = n - 1;\n    while (R > L + 1) {\n        int64_t piv = L + (R - L) / 2;\n        if (cmp_row(t, n, sa, p, len, piv) < 0)"),
    # lcp lengths compared one byte short
    "lcp_short": ("while (i < len && s + i < n && p[i] == t[s + i]) i++;\n    return i;",
                  "while (i + 1 < len && s + i < n && p[i] == t[s + i]) i++;\n    return i;"),
}


def _build(tmp_path, name, old, new):
    assert SRC.count(old) >= 1, name
    src = SRC.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-w", "-o", str(so), str(c)])
    L = ctypes.CDLL(str(so))
    p, i64 = ctypes.c_void_p, ctypes.c_int64
    L.oracle_sa_build.argtypes = [p, i64, p]
    L.oracle_match.argtypes = [p, i64, p, p, p, i64, p, ctypes.c_int, ctypes.c_int]
    return L


def _run(L, text, reads, mode):
    t = np.frombuffer(text.upper().encode(), dtype=np.uint8).copy()
    sa = np.empty(len(t), dtype=np.int32)
    L.oracle_sa_build(t.ctypes.data, len(t), sa.ctypes.data)
    data, offs = oracle.pack_reads(reads)
    out = np.zeros((len(reads), 4), dtype=np.int32)
    L.oracle_match(t.ctypes.data, len(t), sa.ctypes.data, data.ctypes.data, offs.ctypes.data,
                   len(reads), out.ctypes.data, mode, 1)
    return [int(x) for x in sa], [tuple(int(v) for v in r) for r in out]


def _pins_pass(L) -> bool:
    P = paper.load()
    sa, res = _run(L, P["text"], sorted(P["search"]), 0)
    if sa != P["sa"]:
        return False
    for q, r in zip(sorted(P["search"]), res):
        if (r[0], r[1] - 1) != P["search"][q] or r[2] != len(q):
            return False
    rng = random.Random(11)
    texts = ["".join(t) for n in range(1, 5) for t in itertools.product("ACGT", repeat=n)]
    texts += ["".join(rng.choice("ACGT") for _ in range(rng.randint(5, 40))) for _ in range(60)]
    texts += [("AC" * 20)[:k] for k in (7, 13)] + ["A" * 9]
    reads = ["", "A", "AC", "CA", "GGT", "TTT", "ACGN", "acg", "GATTACA", "ACGTACGTACGTACGTAC"]
    for text in texts:
        extra = [text, text + "A", text[1:] + "C", text[len(text) // 2:] + "G"]
        rs = reads + extra
        sa0, r0 = _run(L, text, rs, 0)
        _, r1 = _run(L, text, rs, 1)
        if sa0 != brute.suffix_array(text) or r0 != r1:
            return False
        if any(r != brute.match(text, q) for q, r in zip(rs, r0)):
            return False
    return True


def test_unmodified_copy_passes(tmp_path):
    assert _pins_pass(_build(tmp_path, "same", "int oracle_max_threads", "int oracle_max_threads"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert not _pins_pass(_build(tmp_path, name, old, new))
