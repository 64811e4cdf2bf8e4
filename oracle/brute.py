"""Brute-force checker for tiny inputs, written straight from the definitions.

Pure Python, shares nothing with the C oracle: the suffix array is Python's
own ordering of the suffix strings (for str, a proper prefix sorts first and
"A" < "C" < "G" < "T"), the longest matched prefix is the best common prefix
over every text position, and the interval is a count of cut suffixes that
sort before the matched prefix plus the number of places it occurs.
"""
from __future__ import annotations


def suffix_array(text: str) -> list[int]:
    return sorted(range(len(text)), key=lambda i: text[i:])


def match(text: str, read: str) -> tuple[int, int, int, int]:
    text = text.upper()
    p = read.upper()
    best = 0
    for i in range(len(text)):
        k = 0
        while k < len(p) and i + k < len(text) and p[k] == text[i + k] and p[k] in "ACGT":
            k += 1
        best = max(best, k)
    q = p[:best]
    occ = [i for i in range(len(text)) if text.startswith(q, i)]
    lo = sum(1 for i in range(len(text)) if text[i:i + best] < q)
    return lo, lo + len(occ), best, int(best == len(p))


def rows_of(text: str, sa: list[int], lo: int, hi: int) -> set[int]:
    return {sa[k] for k in range(lo, hi)}


def occurrences(text: str, read: str) -> list[int]:
    """Every text position where the read occurs, in the order of the
    suffixes that start there."""
    t, p = text.upper(), read.upper()
    occ = [i for i in range(len(t)) if t.startswith(p, i)]
    return sorted(occ, key=lambda i: t[i:])
