"""Seeded synthetic workloads for suffix-array read matching.

This module only generates inputs: reference texts, read batches and request
streams.  It holds none of the matching arithmetic, so both the CPU oracle
(test side) and the HIP library (product side) can be fed from it without
sharing any part of the method.

Every random draw comes from numpy's PCG64 seeded with
``SeedSequence([1303, cfg, stream, sub])``.  Streams: 0 reference, 1 Markov
table, 2 repeats, 3 reads, 4 request stream.

The paper measured on NCBI contigs (first 10^7 nt of a human chromosome 1
contig as reference, 1024-nt queries from human and mouse contigs, Section V).
Those records are not available, so these recipes stand in for them:

* ``c1``: 1 Mbp i.i.d. reference, 100,000 reads of 25 bp.
* ``c2``: 16 Mbp order-3 Markov reference (GC 0.41) with 5 % tandem repeats,
  4,000,000 reads of 100 bp (70 % sampled at 0-2 % substitutions, 30 % random).
* ``c3``: the ``c2`` reference, 4,000,000 reads of 20-300 bp, same mix.
* ``c4``: 250 Mbp Markov reference with 10 % interspersed repeats,
  64,000,000 reads of 150 bp (80 % sampled at 1 %, 20 % random).
* ``c5``: an open-loop Poisson request stream over the ``c2`` and ``c4``
  references.

Bases are returned as codes 0..3 for A, C, G, T and converted to ASCII with
:func:`to_ascii`.
"""
from __future__ import annotations

import functools
import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)

# read classes in the truth arrays
RANDOM, COPY, MUTATED = 0, 1, 2


def rng_for(cfg: int, stream: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1303, cfg, stream, sub])))


def to_ascii(codes: np.ndarray) -> np.ndarray:
    return ASCII[codes]


# --------------------------------------------------------------------------- references


def iid_reference(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.integers(0, 4, size=n, dtype=np.uint8)


def _stationary(P: np.ndarray) -> np.ndarray:
    """Stationary distribution of the 64-state chain whose state is the last 3 bases."""
    M = np.zeros((64, 64))
    for s in range(64):
        for b in range(4):
            M[s, ((s << 2) | b) & 63] += P[s, b]
    A = np.vstack([M.T - np.eye(64), np.ones((1, 64))])
    rhs = np.zeros(65)
    rhs[-1] = 1.0
    pi, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    return np.clip(pi, 0.0, None) / np.clip(pi, 0.0, None).sum()


def markov_table(rng: np.random.Generator, gc: float = 0.41):
    """Order-3 transition table with GC content ``gc`` at stationarity.

    Base weights (A,C,G,T) = (0.295, 0.205, 0.205, 0.295), each context's row
    jittered by U(0.8, 1.2) factors, G after C damped by 0.3 (CpG depletion),
    then C and G weights rescaled by one scalar found by bisection so that the
    stationary GC fraction equals ``gc`` (within 5e-4).
    Returns (P[64,4], stationary[64]).
    """
    w = np.array([0.295, 0.205, 0.205, 0.295])[None, :] * rng.uniform(0.8, 1.2, size=(64, 4))
    w[(np.arange(64) & 3) == 1, 2] *= 0.3  # context ends in C: damp the following G

    def build(scale):
        v = w.copy()
        v[:, 1:3] *= scale
        P = v / v.sum(axis=1, keepdims=True)
        pi = _stationary(P)
        g = pi[((np.arange(64) & 3) == 1) | ((np.arange(64) & 3) == 2)].sum()
        return P, pi, g

    lo, hi = 0.05, 20.0
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        P, pi, g = build(mid)
        if abs(g - gc) < 1e-5:
            break
        if g < gc:
            lo = mid
        else:
            hi = mid
    P, pi, g = build(mid)
    assert abs(g - gc) < 5e-4, g
    return P, pi


def markov_sequence(n: int, P: np.ndarray, pi: np.ndarray, rng: np.random.Generator,
                    chain_len: int = 4096) -> np.ndarray:
    """Sample ``n`` bases from the order-3 chain.

    The text is cut into independent segments of ``chain_len`` bases that run
    side by side (vectorised over segments); each segment starts in a state
    drawn from the stationary distribution, so the concatenation has the
    chain's stationary statistics.
    """
    if n <= 0:
        return np.zeros(0, dtype=np.uint8)
    chain_len = max(4, min(chain_len, n))
    C = -(-n // chain_len)
    out = np.empty((C, chain_len), dtype=np.uint8)
    state = rng.choice(64, size=C, p=pi).astype(np.int64)
    out[:, 0] = (state >> 4) & 3
    out[:, 1] = (state >> 2) & 3
    out[:, 2] = state & 3
    cdf = np.cumsum(P, axis=1)[:, :3]
    for t in range(3, chain_len):
        u = rng.random(C)
        c = cdf[state]
        b = (u > c[:, 0]).astype(np.int64) + (u > c[:, 1]) + (u > c[:, 2])
        out[:, t] = b
        state = ((state << 2) | b) & 63
    return out.reshape(-1)[:n].copy()


def _place_nonoverlapping(n: int, lengths: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Uniformly random non-overlapping start positions for segments of ``lengths``
    (in the given order along the text): sorted uniform gaps plus running lengths."""
    free = n - int(lengths.sum())
    assert free >= 0
    gaps = np.sort(rng.integers(0, free + 1, size=len(lengths)))
    before = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    return gaps + before


def add_tandem_repeats(codes: np.ndarray, frac: float, rng: np.random.Generator):
    """Overwrite with tandem arrays (unit U{2..6} iid bases, U{10..50} copies) until
    at least ``frac`` of the bases are covered.  Returns the list of (pos, unit, copies)."""
    n = len(codes)
    target = frac * n
    units, copies = [], []
    total = 0
    while total < target:
        k = 4096
        u = rng.integers(2, 7, size=k)
        c = rng.integers(10, 51, size=k)
        cum = total + np.cumsum(u * c)
        stop = int(np.searchsorted(cum, target)) + 1
        units.extend(u[:stop].tolist())
        copies.extend(c[:stop].tolist())
        total = int(cum[min(stop, k) - 1])
    units = np.array(units)
    copies = np.array(copies)
    lens = units * copies
    pos = _place_nonoverlapping(n, lens, rng)
    arrays = []
    for p, ul, cp in zip(pos.tolist(), units.tolist(), copies.tolist()):
        unit = rng.integers(0, 4, size=ul, dtype=np.uint8)
        codes[p:p + ul * cp] = np.tile(unit, cp)
        arrays.append((p, ul, cp))
    return arrays


def _substitute(codes: np.ndarray, mask: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Replace masked bases by one of the three other bases, uniformly."""
    k = int(mask.sum())
    if k:
        codes[mask] = (codes[mask] + rng.integers(1, 4, size=k, dtype=np.uint8)) & 3
    return codes


def add_interspersed_repeats(codes: np.ndarray, frac: float, P, pi, rng: np.random.Generator,
                             n_elements: int = 20, elem_len: int = 300, divergence: float = 0.10):
    """Copies of ``n_elements`` chain-drawn elements, each copy mutated per base with
    probability ``divergence``, at non-overlapping uniform positions, covering ``frac``."""
    n = len(codes)
    elems = markov_sequence(n_elements * elem_len, P, pi, rng, chain_len=elem_len).reshape(n_elements, elem_len)
    count = int(math.ceil(frac * n / elem_len))
    which = rng.integers(0, n_elements, size=count)
    pos = _place_nonoverlapping(n, np.full(count, elem_len), rng)
    step = 1 << 16
    for s in range(0, count, step):
        w = which[s:s + step]
        block = elems[w].copy()
        _substitute(block, rng.random(block.shape) < divergence, rng)
        idx = pos[s:s + step, None] + np.arange(elem_len)[None, :]
        codes[idx] = block
    return count


@dataclass
class Reference:
    name: str
    codes: np.ndarray  # uint8 0..3
    info: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.codes)

    def ascii(self) -> np.ndarray:
        return to_ascii(self.codes)


def make_reference(cfg: str, n: int | None = None) -> Reference:
    """Reference text of workload ``cfg`` (``n`` overrides the length, same recipe)."""
    if cfg == "c1":
        n = 1_000_000 if n is None else n
        return Reference("c1", iid_reference(n, rng_for(1, 0)), {"model": "iid"})
    if cfg in ("c2", "c3"):
        n = 16_000_000 if n is None else n
        P, pi = markov_table(rng_for(2, 1))
        codes = markov_sequence(n, P, pi, rng_for(2, 0))
        arrays = add_tandem_repeats(codes, 0.05, rng_for(2, 2))
        return Reference("c2", codes, {"model": "markov3+tandem", "tandem_arrays": len(arrays)})
    if cfg == "paper":
        # the paper's reference is 10^7 bases of a human chromosome contig
        # (Section V); the c2 recipe stands in for it, with its own seeds
        n = 10_000_000 if n is None else n
        P, pi = markov_table(rng_for(6, 1))
        codes = markov_sequence(n, P, pi, rng_for(6, 0))
        arrays = add_tandem_repeats(codes, 0.05, rng_for(6, 2))
        return Reference("paper", codes, {"model": "markov3+tandem", "tandem_arrays": len(arrays)})
    if cfg == "c4":
        n = 250_000_000 if n is None else n
        P, pi = markov_table(rng_for(4, 1))
        codes = markov_sequence(n, P, pi, rng_for(4, 0), chain_len=16384)
        copies = add_interspersed_repeats(codes, 0.10, P, pi, rng_for(4, 2))
        return Reference("c4", codes, {"model": "markov3+interspersed", "copies": copies})
    raise ValueError(cfg)


# --------------------------------------------------------------------------- reads


@dataclass(frozen=True)
class ReadSpec:
    cfg_id: int
    count: int
    len_lo: int
    len_hi: int                # inclusive
    frac_random: float
    rate_lo: float = 0.0       # per-base substitution rate of sampled reads ~ U[rate_lo, rate_hi]
    rate_hi: float = 0.0
    exact_subs: tuple | None = None  # (fraction of copies mutated, k_lo, k_hi): c1 recipe


READ_SPECS = {
    "c1": ReadSpec(1, 100_000, 25, 25, 0.5, exact_subs=(0.25, 1, 2)),
    "c2": ReadSpec(2, 4_000_000, 100, 100, 0.3, 0.0, 0.02),
    "c3": ReadSpec(3, 4_000_000, 20, 300, 0.3, 0.0, 0.02),
    "c4": ReadSpec(4, 64_000_000, 150, 150, 0.2, 0.01, 0.01),
    # Section V: 1024-base queries, 512 to 2,097,152 per set, from the human
    # contig and a mouse contig; half sampled from the reference at 0-1 %
    # substitutions, half random (standing in for the unrelated genome)
    "paper": ReadSpec(6, 2_097_152, 1024, 1024, 0.5, 0.0, 0.01),
}


@dataclass
class Reads:
    data: np.ndarray     # uint8 ASCII, concatenated
    offs: np.ndarray     # int64[N+1]
    cls: np.ndarray      # int8 read class (RANDOM, COPY, MUTATED)
    pos: np.ndarray      # int64 source position (-1 for random reads)
    first_sub: np.ndarray  # int32 index of the first substituted base (= length if none)

    @property
    def count(self) -> int:
        return len(self.offs) - 1

    def lengths(self) -> np.ndarray:
        return np.diff(self.offs)

    def read(self, i: int) -> bytes:
        return self.data[self.offs[i]:self.offs[i + 1]].tobytes()


CHUNK = 1 << 16


@functools.lru_cache(maxsize=4)
def _class_labels(spec: ReadSpec, count: int) -> np.ndarray:
    n_rand = int(round(spec.frac_random * count))
    lab = np.full(count, COPY, dtype=np.int8)
    lab[:n_rand] = RANDOM
    if spec.exact_subs is not None:
        n_mut = int(round(spec.exact_subs[0] * (count - n_rand)))
        lab[n_rand:n_rand + n_mut] = MUTATED
    elif spec.rate_hi > 0:
        lab[n_rand:] = MUTATED
    rng_for(spec.cfg_id, 3, 0).shuffle(lab)
    lab.setflags(write=False)  # shared between calls
    return lab


def make_reads(ref: Reference, spec: ReadSpec, count: int | None = None,
               start: int = 0, stop: int | None = None) -> Reads:
    """Reads ``[start, stop)`` of a batch of ``count`` reads drawn by ``spec``.

    Reads are produced in chunks of 2^16 with their own sub-streams, so any
    sub-range comes out identical to the same rows of the whole batch.
    """
    count = spec.count if count is None else count
    stop = count if stop is None else min(stop, count)
    labels = _class_labels(spec, count)
    n = ref.n
    parts = []
    c0 = start // CHUNK
    for c in range(c0, -(-stop // CHUNK)):
        lo_i, hi_i = c * CHUNK, min((c + 1) * CHUNK, count)
        rng = rng_for(spec.cfg_id, 3, c + 1)
        k = hi_i - lo_i
        lab = labels[lo_i:hi_i]
        lens = rng.integers(spec.len_lo, spec.len_hi + 1, size=k)
        if n > 0:
            lens_src = np.minimum(lens, n)
        else:
            lens_src = lens
        pos = (rng.random(k) * (n - lens_src + 1)).astype(np.int64)
        rates = rng.uniform(spec.rate_lo, spec.rate_hi, size=k) if spec.rate_hi > 0 else np.full(k, spec.rate_lo)
        total = int(lens.sum())
        offs = np.zeros(k + 1, dtype=np.int64)
        np.cumsum(lens, out=offs[1:])
        src = lab != RANDOM
        mut = lab == MUTATED
        if spec.len_lo == spec.len_hi and spec.exact_subs is None and spec.len_lo <= n:
            # fixed length: whole rows at once; each base of a sampled read is
            # substituted with probability r, drawn as a binomial count of
            # distinct uniform positions (the same distribution)
            m = spec.len_lo
            codes2 = np.empty((k, m), dtype=np.uint8)
            i_rnd, i_src = np.nonzero(~src)[0], np.nonzero(src)[0]
            codes2[i_rnd] = rng.integers(0, 4, size=(len(i_rnd), m), dtype=np.uint8)
            codes2[i_src] = np.lib.stride_tricks.sliding_window_view(ref.codes, m)[pos[i_src]]
            cnt = np.where(mut, rng.binomial(m, rates), 0)
            rows = np.repeat(np.arange(k), cnt)
            cols = rng.integers(0, m, size=len(rows))
            while len(rows):
                flat = rows.astype(np.int64) * m + cols
                order = np.argsort(flat, kind="stable")
                dup = np.zeros(len(rows), dtype=bool)
                dup[order[1:]] = flat[order[1:]] == flat[order[:-1]]
                if not dup.any():
                    break
                cols[dup] = rng.integers(0, m, size=int(dup.sum()))
            codes2[rows, cols] = (codes2[rows, cols] + rng.integers(1, 4, size=len(rows), dtype=np.uint8)) & 3
            first_sub = np.full(k, m, dtype=np.int32)
            np.minimum.at(first_sub, rows, cols.astype(np.int32))
            pos = np.where(src, pos, -1)
            sl = slice(max(start, lo_i) - lo_i, min(stop, hi_i) - lo_i)
            o0, o1 = offs[sl.start], offs[sl.stop]
            parts.append((to_ascii(codes2.reshape(-1)[o0:o1]), lens[sl], lab[sl], pos[sl], first_sub[sl]))
            continue
        lens32 = lens.astype(np.int32)
        rel = np.arange(total, dtype=np.int32)
        rel -= np.repeat(offs[:-1].astype(np.int32), lens32)
        codes = rng.integers(0, 4, size=total, dtype=np.uint8)
        src_flat = np.repeat(src, lens32)
        src_flat &= rel < np.repeat(lens_src.astype(np.int32), lens32)
        gidx = np.repeat(pos.astype(np.int32), lens32)
        gidx += rel
        codes[src_flat] = ref.codes[gidx[src_flat]]
        del gidx, src_flat
        first_sub = lens.astype(np.int32).copy()
        if spec.exact_subs is not None:
            _, k_lo, k_hi = spec.exact_subs
            nsub = rng.integers(k_lo, k_hi + 1, size=k)
            p1 = (rng.random(k) * lens).astype(np.int64)
            p2 = (p1 + 1 + (rng.random(k) * (lens - 1)).astype(np.int64)) % lens
            mask = np.zeros(total, dtype=bool)
            mask[(offs[:-1] + p1)[mut]] = True
            two = mut & (nsub == 2)
            mask[(offs[:-1] + p2)[two]] = True
            first_sub[mut] = np.where(two, np.minimum(p1, p2), p1)[mut]
        else:
            mask = rng.random(total, dtype=np.float32) < np.repeat(rates.astype(np.float32), lens32)
            mask &= np.repeat(mut, lens32)
            big = np.int32(np.iinfo(np.int32).max)
            hit_rel = np.where(mask, rel, big)
            fs = np.minimum.reduceat(hit_rel, offs[:-1]) if total else np.zeros(0, np.int32)
            fs = np.where(lens > 0, fs, big)
            first_sub = np.minimum(fs, lens).astype(np.int32)
            del hit_rel
        del rel
        _substitute(codes, mask, rng)
        pos = np.where(src, pos, -1)
        sl = slice(max(start, lo_i) - lo_i, min(stop, hi_i) - lo_i)
        o0, o1 = offs[sl.start], offs[sl.stop]
        parts.append((to_ascii(codes[o0:o1]), lens[sl], lab[sl], pos[sl], first_sub[sl]))
    data = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.uint8)
    lens = np.concatenate([p[1] for p in parts]) if parts else np.zeros(0, np.int64)
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    return Reads(data, offs,
                 np.concatenate([p[2] for p in parts]) if parts else np.zeros(0, np.int8),
                 np.concatenate([p[3] for p in parts]) if parts else np.zeros(0, np.int64),
                 np.concatenate([p[4] for p in parts]) if parts else np.zeros(0, np.int32))


def read_offsets(spec: ReadSpec, count: int | None = None) -> np.ndarray:
    """Offsets [count + 1] of a batch drawn by ``spec``, without the reads
    (each chunk's lengths are its sub-stream's first draw)."""
    count = spec.count if count is None else count
    offs = np.zeros(count + 1, dtype=np.int64)
    for c in range(-(-count // CHUNK)):
        lo_i, hi_i = c * CHUNK, min((c + 1) * CHUNK, count)
        lens = rng_for(spec.cfg_id, 3, c + 1).integers(spec.len_lo, spec.len_hi + 1, size=hi_i - lo_i)
        offs[lo_i + 1:hi_i + 1] = lens
    np.cumsum(offs, out=offs)
    return offs


_PAR = {}


def _fill_chunks(span):
    """Worker: write chunks [a, b) into the shared output arrays."""
    a, b = span
    p = _PAR
    lo, hi = a * CHUNK, min(b * CHUNK, p["count"])
    r = make_reads(p["ref"], p["spec"], p["count"], lo, hi)
    o0 = p["offs"][lo]
    p["data"][o0:o0 + len(r.data)] = r.data
    p["cls"][lo:hi] = r.cls
    p["pos"][lo:hi] = r.pos
    p["first_sub"][lo:hi] = r.first_sub
    return hi - lo


def make_reads_parallel(ref: Reference, spec: ReadSpec, count: int | None = None, workers: int = 8,
                        progress=None) -> Reads:
    """``make_reads`` of the whole batch, identical output, with the chunks
    spread over forked worker processes that write into shared anonymous
    memory (workers <= 1: the same spans in this process).  Call it before
    the process starts using a GPU: the workers are forks of the caller.
    ``progress(done, count)``, if given, is called as spans finish."""
    import mmap
    import multiprocessing as mp

    count = spec.count if count is None else count
    nchunks = -(-count // CHUNK)
    if nchunks < 2:
        return make_reads(ref, spec, count)
    offs = read_offsets(spec, count)
    _class_labels(spec, count)  # drawn once, inherited by the workers

    def shared(n, dtype):
        nbytes = max(1, n * np.dtype(dtype).itemsize)
        return np.frombuffer(mmap.mmap(-1, nbytes), dtype=dtype)[:n]

    out = {"data": shared(int(offs[-1]), np.uint8), "cls": shared(count, np.int8), "pos": shared(count, np.int64),
           "first_sub": shared(count, np.int32)}
    _PAR.clear()
    _PAR.update(ref=ref, spec=spec, count=count, offs=offs, **out)
    step = max(1, nchunks // (4 * max(1, workers)))
    spans = [(a, min(a + step, nchunks)) for a in range(0, nchunks, step)]
    done = 0
    try:
        if workers <= 1:
            for sp in spans:
                done += _fill_chunks(sp)
                if progress:
                    progress(done, count)
        else:
            # close + join: the workers finish their last task and leave on
            # their own (no signals)
            pool = mp.get_context("fork").Pool(min(workers, len(spans)))
            try:
                for n in pool.imap_unordered(_fill_chunks, spans):
                    done += n
                    if progress:
                        progress(done, count)
                pool.close()
            except BaseException:
                pool.terminate()
                raise
            finally:
                pool.join()
    finally:
        _PAR.clear()
    assert done == count
    return Reads(out["data"], offs, out["cls"], out["pos"], out["first_sub"])


def workload(cfg: str, n: int | None = None, count: int | None = None):
    """(Reference, Reads) of a named workload; ``n``/``count`` scale it down, same recipe."""
    ref = make_reference(cfg, n)
    spec = READ_SPECS[cfg]
    return ref, make_reads(ref, spec, count)


# --------------------------------------------------------------------------- request stream


@dataclass
class Request:
    t_arrival: float  # seconds from stream start
    ref: int          # 0 = c2 reference, 1 = c4 reference
    reads: Reads


def request_sizes(num: int, rng: np.random.Generator, max_reads: int = 100_000) -> np.ndarray:
    """log-uniform request sizes: floor(exp(U(0, ln(max+1)))) clipped to [1, max]."""
    return np.clip(np.floor(np.exp(rng.uniform(0.0, math.log(max_reads + 1), size=num))), 1, max_reads).astype(np.int64)


def request_pool(refs, num: int, max_reads: int = 100_000, seed_sub: int = 0):
    """``num`` distinct requests, as (ref, Reads): each names reference 0 or 1
    (p = 1/2) and carries a log-uniform number of reads of 30-300 bp drawn with
    that reference's sampling mix (c2: 30 % random, rate U[0, 0.02]; c4: 20 %
    random, 1 %)."""
    rng = rng_for(5, 5, seed_sub)
    which = rng.integers(0, len(refs), size=num)
    sizes = request_sizes(num, rng, max_reads)
    mixes = [ReadSpec(50, 0, 30, 300, 0.3, 0.0, 0.02), ReadSpec(51, 0, 30, 300, 0.2, 0.01, 0.01)]
    out = []
    for i in range(num):
        base = mixes[int(which[i]) % 2]
        spec = ReadSpec(base.cfg_id * 1_000_003 + seed_sub * 7919 + i, int(sizes[i]), 30, 300,
                        base.frac_random, base.rate_lo, base.rate_hi)
        out.append((int(which[i]), make_reads(refs[int(which[i])], spec)))
    return out


def request_stream(refs, num: int, rate_per_s: float, max_reads: int = 100_000, seed_sub: int = 0, pool=None):
    """Open-loop Poisson stream of ``num`` requests at ``rate_per_s``.  Without
    ``pool`` every request is new (``request_pool`` of size ``num``); with one,
    each arrival takes a uniformly chosen request of the pool."""
    rng = rng_for(5, 4, seed_sub)
    gaps = rng.exponential(1.0 / rate_per_s, size=num)
    times = np.cumsum(gaps) - gaps[0]
    if pool is None:
        pool = request_pool(refs, num, max_reads, seed_sub)
        pick = np.arange(num)
    else:
        pick = rng.integers(0, len(pool), size=num)
    return [Request(float(times[i]), pool[int(pick[i])][0], pool[int(pick[i])][1]) for i in range(num)]


def manifest(ref: Reference, reads: Reads) -> dict:
    return {
        "reference": ref.name, "n": ref.n, **ref.info,
        "reference_sha256": hashlib.sha256(ref.codes.tobytes()).hexdigest(),
        "reads": reads.count,
        "reads_sha256": hashlib.sha256(reads.data.tobytes() + reads.offs.tobytes()).hexdigest(),
        "classes": {int(c): int((reads.cls == c).sum()) for c in (RANDOM, COPY, MUTATED)},
    }
