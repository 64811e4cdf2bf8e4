"""ctypes front end of the plain C oracle (test infrastructure only).

``sa_build`` sorts every suffix with a comparison sort (the direct
construction of Section III); ``match`` runs the per-read LB / RB binary
searches of Section IV plus the longest-matched-prefix step; ``scan_one``
recomputes one read's result from the definitions by visiting every text
position, without a suffix array; ``locate`` lists the occurrences of each
selected read as the suffix-array entries of its interval (Section IV lists
the occurrences of a read that way).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build() -> str:
    """Compile the oracle library (gcc, OpenMP)."""
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, SRC])
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_sa_build.argtypes = [p, i64, p]
        L.oracle_sa_check.argtypes = [p, i64, p]
        L.oracle_match.argtypes = [p, i64, p, p, p, i64, p, ctypes.c_int, ctypes.c_int]
        L.oracle_scan_one.argtypes = [p, i64, p, i64, p]
        _lib = L
    return _lib


def _u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, str)):
        a = np.frombuffer(a.encode() if isinstance(a, str) else bytes(a), dtype=np.uint8)
    return np.ascontiguousarray(a, dtype=np.uint8)


def normalize_text(text) -> np.ndarray:
    """Upper-case the reference; anything outside ACGT is rejected."""
    t = _u8(text).copy()
    low = (t >= ord("a")) & (t <= ord("z"))
    t[low] -= 32
    ok = (t == ord("A")) | (t == ord("C")) | (t == ord("G")) | (t == ord("T"))
    if not ok.all():
        raise ValueError("reference holds a byte outside ACGT")
    return t


def sa_build(text) -> np.ndarray:
    t = normalize_text(text)
    sa = np.empty(len(t), dtype=np.int32)
    if lib().oracle_sa_build(t.ctypes.data, len(t), sa.ctypes.data) != 0:
        raise ValueError("bad length")
    return sa


def sa_check(text, sa) -> int:
    t = normalize_text(text)
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    if len(sa) != len(t):
        return 1
    return lib().oracle_sa_check(t.ctypes.data, len(t), sa.ctypes.data)


def pack_reads(reads) -> tuple[np.ndarray, np.ndarray]:
    """A list of byte strings as (concatenated bytes, int64 offsets)."""
    bs = [r.encode() if isinstance(r, str) else bytes(r) for r in reads]
    offs = np.zeros(len(bs) + 1, dtype=np.int64)
    np.cumsum([len(b) for b in bs], out=offs[1:])
    data = np.frombuffer(b"".join(bs) + b"\0", dtype=np.uint8)
    return data, offs


def match(text, sa, data, offs, mode: int = 0, nthreads: int = 0) -> np.ndarray:
    """(N, 4) int32 rows {lo, hi, l, exact} for the reads data[offs[i]:offs[i+1]]."""
    t = normalize_text(text)
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    data = _u8(data)
    if len(data) == 0:
        data = np.zeros(1, dtype=np.uint8)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    N = len(offs) - 1
    out = np.zeros((max(N, 0), 4), dtype=np.int32)
    rc = lib().oracle_match(t.ctypes.data, len(t), sa.ctypes.data, data.ctypes.data, offs.ctypes.data,
                            N, out.ctypes.data, mode, nthreads)
    if rc != 0:
        raise ValueError(f"oracle_match failed ({rc})")
    return out


def scan_one(text, read) -> tuple[int, int, int, int]:
    t = normalize_text(text) if not isinstance(text, np.ndarray) or text.dtype != np.uint8 else text
    p = _u8(read)
    buf = np.zeros(len(p) + 1, dtype=np.uint8)
    buf[:len(p)] = p
    out = np.zeros(4, dtype=np.int32)
    if lib().oracle_scan_one(t.ctypes.data, len(t), buf.ctypes.data, len(p), out.ctypes.data) != 0:
        raise ValueError("scan failed")
    return tuple(int(x) for x in out)


def locate(sa, res, cap: int, min_len: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """CSR (offsets int64[N+1], positions int32) of each read's occurrences:
    a read is selected when its result is exact (min_len == 0) or its matched
    length is at least min_len (min_len > 0); a selected read lists
    SA[lo], SA[lo+1], ... for its first min(hi - lo, cap) rows, in SA order.
    ``res`` is ``match``'s (N, 4) output {lo, hi, l, exact}."""
    sa = np.asarray(sa)
    res = np.asarray(res, dtype=np.int64).reshape(-1, 4)
    lo, hi, ln, ex = res[:, 0], res[:, 1], res[:, 2], res[:, 3]
    sel = (ln >= min_len) if min_len > 0 else (ex != 0)
    count = np.where(sel, np.minimum(hi - lo, cap), 0)
    offs = np.zeros(len(res) + 1, dtype=np.int64)
    np.cumsum(count, out=offs[1:])
    rows = np.repeat(lo, count) + (np.arange(offs[-1]) - np.repeat(offs[:-1], count))
    return offs, sa[rows].astype(np.int32)


def max_threads() -> int:
    return lib().oracle_max_threads()
