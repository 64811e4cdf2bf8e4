"""ctypes binding of libsamatch.so: the C-ABI of include/samatch.h with the
same names.  Argument marshalling only; every step of the matching runs in
the library.  Device buffers are torch tensors (torch is used for device
memory and streams only).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SAMATCH_LIB names another build of the same library (the sanitizer
# builds of the CPU tests); by default the one built next to this file.
LIB_PATH = os.environ.get("SAMATCH_LIB") or os.path.join(HERE, "libsamatch.so")

SA_OK, SA_PENDING = 0, 1
SA_EINVAL, SA_EALPHABET, SA_ETOOBIG, SA_ENOMEM, SA_EDEVICE = -1, -2, -3, -4, -5
SA_ENOSPC, SA_ECANCELED, SA_EIO, SA_EFORMAT, SA_ENOTFOUND = -6, -7, -8, -9, -10
SA_MAX_READ = 1024
SA_HIT_EXACT, SA_HIT_TOOLONG = 1, 2
SA_KERNEL_TUNED, SA_KERNEL_PLAIN = 0, 1

# every extern "C" symbol the header declares
EXPORTS = [
    "sa_build", "sa_build_from_sa", "sa_index_length", "sa_index_copy_sa", "sa_save", "sa_load", "sa_free",
    "sa_upload", "sa_dfree", "sa_dindex_length", "sa_build_device", "sa_download", "sa_dindex_build_info",
    "sa_dindex_bytes", "sa_set_prefix_table",
    "sa_default_cfg", "match_batch", "match_batch_dev", "match_batch_dev_noalloc", "sa_noalloc_max_reads",
    "sa_stage_times", "sa_probe_counts", "sa_tune", "sa_tune_candidates", "sa_random_read_rate",
    "sa_locate_dev", "sa_locate",
    "st_build", "st_free", "st_node_count", "st_root", "st_copy_nodes", "st_index_bytes", "st_upload", "st_dfree",
    "st_match_batch_dev",
    "sa_server_create", "match_submit", "match_poll", "sa_server_replay", "sa_server_get_stats",
    "sa_server_destroy", "sa_strerror",
    "sa_last_error",
]


class SaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class MatchCfg(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("tile_levels", ctypes.c_int), ("block", ctypes.c_int),
                ("blocks_per_cu", ctypes.c_int), ("nbuckets", ctypes.c_int), ("bucket_edge", ctypes.c_int * 8),
                ("sort", ctypes.c_int), ("use_graph", ctypes.c_int), ("profile", ctypes.c_int),
                ("count", ctypes.c_int), ("group", ctypes.c_int), ("prefix_table", ctypes.c_int),
                ("inline_pack", ctypes.c_int), ("max_words", ctypes.c_int), ("defer", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {"kernel": self.kernel, "tile_levels": self.tile_levels, "block": self.block,
                "blocks_per_cu": self.blocks_per_cu, "nbuckets": self.nbuckets,
                "bucket_edge": list(self.bucket_edge)[:max(1, self.nbuckets)], "sort": self.sort,
                "use_graph": self.use_graph, "group": self.group, "prefix_table": self.prefix_table,
                "inline_pack": self.inline_pack, "max_words": self.max_words, "defer": self.defer}


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_reserve_bytes", ctypes.c_int64), ("max_batch_reads", ctypes.c_int64),
                ("max_inflight_reads", ctypes.c_int64), ("nstreams", ctypes.c_int),
                ("test_fake_free_hbm", ctypes.c_int64), ("test_echo", ctypes.c_int), ("test_fail_batch", ctypes.c_int),
                ("host_pool_bytes", ctypes.c_int64), ("measure", ctypes.c_int), ("batch_linger_us", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_int64), ("reads", ctypes.c_int64), ("upload_bytes", ctypes.c_int64),
                ("search_ms", ctypes.c_double), ("touched_bytes", ctypes.c_int64)]


class ReqStats(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("status", ctypes.c_int), ("nreads", ctypes.c_int64)]


_lib = None


def lib():
    """Load the built library; fails loudly when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python -m paper_1303_3692_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        p, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        pp = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "sa_build": ([p, i64, pp], i32),
            "sa_build_from_sa": ([p, i64, p, pp], i32),
            "sa_index_length": ([p], i64),
            "sa_index_copy_sa": ([p, p], i32),
            "sa_save": ([p, ctypes.c_char_p], i32),
            "sa_load": ([ctypes.c_char_p, pp], i32),
            "sa_free": ([p], None),
            "sa_upload": ([p, i32, pp], i32),
            "sa_dfree": ([p], None),
            "sa_dindex_length": ([p], i64),
            "sa_build_device": ([p, i64, i32, pp], i32),
            "sa_download": ([p, pp], i32),
            "sa_dindex_build_info": ([p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)], i32),
            "sa_default_cfg": ([p, ctypes.POINTER(MatchCfg)], i32),
            "match_batch": ([p, p, p, i64, p, p, ctypes.POINTER(MatchCfg)], i32),
            "match_batch_dev": ([p, p, p, i64, p, p, ctypes.POINTER(MatchCfg)], i32),
            "match_batch_dev_noalloc": ([p, p, p, i64, p, p, ctypes.POINTER(MatchCfg)], i32),
            "sa_noalloc_max_reads": ([i32], i64),
            "sa_stage_times": ([p, p, ctypes.POINTER(ctypes.c_double)], i32),
            "sa_probe_counts": ([p, p, ctypes.POINTER(ctypes.c_int64)], i32),
            "sa_random_read_rate": ([i32, i32, ctypes.POINTER(ctypes.c_double)], i32),
            "sa_tune": ([p, p, p, i64, p, ctypes.c_char_p, ctypes.POINTER(MatchCfg), ctypes.POINTER(ctypes.c_double)], i32),
            "sa_tune_candidates": ([p, p, i64, p, p, p, i32, ctypes.POINTER(ctypes.c_int)], i32),
            "sa_dindex_bytes": ([p, p], i32),
            "sa_set_prefix_table": ([p, i32], i32),
            "sa_locate_dev": ([p, p, i64, i32, i32, p, p, i64, p, ctypes.POINTER(ctypes.c_int64)], i32),
            "sa_locate": ([p, p, i64, i32, i32, p, p, i64, ctypes.POINTER(ctypes.c_int64)], i32),
            "st_build": ([p, pp], i32),
            "st_free": ([p], None),
            "st_node_count": ([p], i64),
            "st_root": ([p], i32),
            "st_copy_nodes": ([p, p], i32),
            "st_index_bytes": ([p], i64),
            "st_upload": ([p, p, pp], i32),
            "st_dfree": ([p], None),
            "st_match_batch_dev": ([p, p, p, i64, p, p], i32),
            "sa_server_create": ([ctypes.POINTER(ctypes.c_void_p), i32, ctypes.POINTER(ServerOpts), pp], i32),
            "match_submit": ([p, i32, p, p, i64, p, ctypes.POINTER(ctypes.c_uint64)], i32),
            "match_poll": ([p, ctypes.c_uint64, i64, ctypes.POINTER(ReqStats)], i32),
            "sa_server_replay": ([p, i64, p, p, p, p, p, p, i32, p, ctypes.POINTER(ReqStats)], i32),
            "sa_server_get_stats": ([p, p], i32),
            "sa_server_destroy": ([p], i32),
            "sa_strerror": ([i32], ctypes.c_char_p),
            "sa_last_error": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int, what: str) -> int:
    if rc < 0:
        L = lib()
        raise SaError(rc, f"{what}: {L.sa_strerror(rc).decode()}: {L.sa_last_error().decode()}")
    return rc


def _bytes(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray)):
        return np.frombuffer(bytes(a), dtype=np.uint8)
    if isinstance(a, str):
        return np.frombuffer(a.encode(), dtype=np.uint8)
    return np.ascontiguousarray(a, dtype=np.uint8)


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ index


class Index:
    """Host index (sa_index): n, packed text, suffix array."""

    def __init__(self, ptr: ctypes.c_void_p):
        self._p = ptr

    @property
    def ptr(self):
        return self._p

    def __len__(self) -> int:
        return int(lib().sa_index_length(self._p))

    def suffix_array(self) -> np.ndarray:
        out = np.empty(len(self), dtype=np.int32)
        _check(lib().sa_index_copy_sa(self._p, out.ctypes.data), "sa_index_copy_sa")
        return out

    def free(self):
        if self._p:
            lib().sa_free(self._p)
            self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sa_build(text) -> Index:
    t = _bytes(text)
    out = ctypes.c_void_p()
    _check(lib().sa_build(t.ctypes.data, len(t), ctypes.byref(out)), "sa_build")
    return Index(out)


def sa_build_from_sa(text, sa) -> Index:
    t = _bytes(text)
    s = np.ascontiguousarray(sa, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(lib().sa_build_from_sa(t.ctypes.data, len(t), s.ctypes.data, ctypes.byref(out)), "sa_build_from_sa")
    return Index(out)


def sa_save(ix: Index, path: str) -> None:
    _check(lib().sa_save(ix.ptr, path.encode()), "sa_save")


def sa_load(path: str) -> Index:
    out = ctypes.c_void_p()
    _check(lib().sa_load(path.encode(), ctypes.byref(out)), "sa_load")
    return Index(out)


class DIndex:
    """Device-resident index (sa_dindex)."""

    def __init__(self, ptr: ctypes.c_void_p, device: int):
        self._p = ptr
        self.device = device

    @property
    def ptr(self):
        return self._p

    def __len__(self) -> int:
        return int(lib().sa_dindex_length(self._p))

    def index_bytes(self) -> dict:
        """Device bytes by part (sa_dindex_bytes)."""
        b = (ctypes.c_int64 * 5)()
        _check(lib().sa_dindex_bytes(self.ptr, b), "sa_dindex_bytes")
        return {"text": b[0], "suffix_array": b[1], "row_records": b[2], "prefix_table": b[3], "tile": b[4]}

    def set_prefix_table(self, k: int) -> None:
        """Rebuild the prefix table for k-base strings (0: drop it)."""
        _check(lib().sa_set_prefix_table(self.ptr, k), "sa_set_prefix_table")

    def build_info(self) -> dict:
        """Suffix sorting rounds and sorted pairs when built by sa_build_device."""
        steps, pairs = ctypes.c_int(), ctypes.c_int64()
        _check(lib().sa_dindex_build_info(self._p, ctypes.byref(steps), ctypes.byref(pairs)), "sa_dindex_build_info")
        return {"steps": steps.value, "sorted_pairs": pairs.value}

    def default_cfg(self) -> MatchCfg:
        c = MatchCfg()
        _check(lib().sa_default_cfg(self._p, ctypes.byref(c)), "sa_default_cfg")
        return c

    def free(self):
        if self._p:
            lib().sa_dfree(self._p)
            self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sa_upload(ix: Index, device: int = 0) -> DIndex:
    out = ctypes.c_void_p()
    _check(lib().sa_upload(ix.ptr, device, ctypes.byref(out)), "sa_upload")
    return DIndex(out, device)


def sa_build_device(text, device: int = 0) -> DIndex:
    """Resident index whose suffix array is built on the device."""
    buf = _bytes(text)
    out = ctypes.c_void_p()
    _check(lib().sa_build_device(buf.ctypes.data if len(buf) else None, len(buf), device, ctypes.byref(out)),
           "sa_build_device")
    return DIndex(out, device)


def sa_download(d: DIndex) -> Index:
    """Host copy of a resident index."""
    out = ctypes.c_void_p()
    _check(lib().sa_download(d.ptr, ctypes.byref(out)), "sa_download")
    return Index(out)


def cfg(d: DIndex | None = None, **kw) -> MatchCfg:
    """A launch configuration: the index defaults (or zeros) with fields overridden."""
    c = d.default_cfg() if d is not None else MatchCfg()
    for k, v in kw.items():
        if k == "bucket_edge":
            for i, e in enumerate(v):
                c.bucket_edge[i] = int(e)
        else:
            setattr(c, k, int(v))
    return c


# ------------------------------------------------------------------ batches


def match_batch(d: DIndex, data, offs, stream=None, config: MatchCfg | None = None) -> np.ndarray:
    """Host batch; returns (N, 4) int32 rows {lo, hi, len, flags} in input order."""
    data = _bytes(data)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    n = len(offs) - 1
    out = np.zeros((max(n, 0), 4), dtype=np.int32)
    if n <= 0:
        return out
    buf = data if len(data) else np.zeros(1, dtype=np.uint8)
    _check(lib().match_batch(d.ptr, buf.ctypes.data, offs.ctypes.data, n, out.ctypes.data,
                             _stream_handle(stream), ctypes.byref(config) if config is not None else None),
           "match_batch")
    return out


def match_batch_dev(d: DIndex, d_reads, d_offs, d_out, nreads: int | None = None, stream=None,
                    config: MatchCfg | None = None) -> None:
    """Device batch on torch tensors: d_reads uint8, d_offs int64 [N+1], d_out int32 [N, 4]."""
    n = (d_offs.numel() - 1) if nreads is None else nreads
    _check(lib().match_batch_dev(d.ptr, ctypes.c_void_p(d_reads.data_ptr()), ctypes.c_void_p(d_offs.data_ptr()), n,
                                 ctypes.c_void_p(d_out.data_ptr()), _stream_handle(stream),
                                 ctypes.byref(config) if config is not None else None), "match_batch_dev")


def match_batch_dev_noalloc(d: DIndex, d_reads, d_offs, d_out, nreads: int | None = None, stream=None,
                            config: MatchCfg | None = None) -> None:
    """match_batch_dev on the library's fixed device scratch (no allocation)."""
    n = (d_offs.numel() - 1) if nreads is None else nreads
    _check(lib().match_batch_dev_noalloc(d.ptr, ctypes.c_void_p(d_reads.data_ptr()),
                                         ctypes.c_void_p(d_offs.data_ptr()), n, ctypes.c_void_p(d_out.data_ptr()),
                                         _stream_handle(stream),
                                         ctypes.byref(config) if config is not None else None),
           "match_batch_dev_noalloc")


def sa_noalloc_max_reads(pack_pass: bool) -> int:
    """Largest batch match_batch_dev_noalloc takes with or without a pack pass."""
    return int(lib().sa_noalloc_max_reads(1 if pack_pass else 0))


def sa_stage_times(d: DIndex, stream=None) -> dict:
    """Stage times (ms) of the last profiled batch on this stream."""
    ms = (ctypes.c_double * 4)()
    _check(lib().sa_stage_times(d.ptr, _stream_handle(stream), ms), "sa_stage_times")
    return {"pack": ms[0], "sort": ms[1], "search": ms[2], "total": ms[3]}


def sa_probe_counts(d: DIndex, stream=None) -> dict:
    """Probe counts of the last counted batch on this stream."""
    c = (ctypes.c_int64 * 10)()
    _check(lib().sa_probe_counts(d.ptr, _stream_handle(stream), c), "sa_probe_counts")
    return {"global_probes": c[0], "text_words": c[1], "tile_probes": c[2], "reads": c[3], "query_words": c[4],
            "key_words": c[5], "table_lookups": c[6], "touched_bytes": c[7], "index_segments": c[8],
            "index_loads": c[9]}


def sa_random_read_rate(device: int = 0, log2_entries: int = 24) -> float:
    """Random 16-byte loads per second the device serves from a table of
    2^log2_entries 16-byte entries (a measurement helper, not part of the
    matching path)."""
    r = ctypes.c_double()
    _check(lib().sa_random_read_rate(device, log2_entries, ctypes.byref(r)), "sa_random_read_rate")
    return r.value


class StIndex:
    """Flattened suffix tree (st_index) built on the host from an Index."""

    def __init__(self, ptr):
        self._p = ptr

    @property
    def ptr(self):
        return self._p

    def node_count(self) -> int:
        return int(lib().st_node_count(self._p))

    def root(self) -> int:
        return int(lib().st_root(self._p))

    def nodes(self) -> np.ndarray:
        """(count, 8) int32: lb, rb, depth, 0, child[a], child[c], child[g], child[t]."""
        out = np.zeros((self.node_count(), 8), dtype=np.int32)
        _check(lib().st_copy_nodes(self._p, out.ctypes.data), "st_copy_nodes")
        return out

    def device_bytes(self) -> int:
        return int(lib().st_index_bytes(self._p))

    def free(self):
        if self._p:
            lib().st_free(self._p)
            self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class StDIndex:
    """Suffix tree resident on the device, searching a resident index's text and SA."""

    def __init__(self, ptr, d):
        self._p = ptr
        self._d = d  # the resident index must outlive the tree

    @property
    def ptr(self):
        return self._p

    def free(self):
        if self._p:
            lib().st_dfree(self._p)
            self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def st_build(ix: Index) -> StIndex:
    out = ctypes.c_void_p()
    _check(lib().st_build(ix.ptr, ctypes.byref(out)), "st_build")
    return StIndex(out)


def st_upload(t: StIndex, d: DIndex) -> StDIndex:
    out = ctypes.c_void_p()
    _check(lib().st_upload(t.ptr, d.ptr, ctypes.byref(out)), "st_upload")
    return StDIndex(out, d)


def st_match_batch_dev(sd: StDIndex, d_reads, d_offs, d_out, nreads: int | None = None, stream=None) -> None:
    """Suffix-tree search of a device batch (torch tensors, as match_batch_dev)."""
    n = (d_offs.numel() - 1) if nreads is None else nreads
    _check(lib().st_match_batch_dev(sd.ptr, ctypes.c_void_p(d_reads.data_ptr()), ctypes.c_void_p(d_offs.data_ptr()),
                                    n, ctypes.c_void_p(d_out.data_ptr()), _stream_handle(stream)),
           "st_match_batch_dev")


def locate(d: DIndex, hits, cap: int, min_len: int = 0):
    """Host locate: (offs int64[N+1], positions int32[offs[-1]]) for hits (N, 4)."""
    hits = np.ascontiguousarray(hits, dtype=np.int32).reshape(-1, 4)
    n = len(hits)
    offs = np.zeros(n + 1, dtype=np.int64)
    total = ctypes.c_int64()
    hp = hits.ctypes.data if n else None
    rc = lib().sa_locate(d.ptr, hp, n, cap, min_len, offs.ctypes.data, None, 0, ctypes.byref(total))
    if rc != SA_ENOSPC:
        _check(rc, "sa_locate")
    pos = np.zeros(max(total.value, 1), dtype=np.int32)
    if total.value:
        _check(lib().sa_locate(d.ptr, hp, n, cap, min_len, offs.ctypes.data, pos.ctypes.data, total.value,
                               ctypes.byref(total)), "sa_locate")
    return offs, pos[:total.value]


def locate_dev(d: DIndex, d_hits, cap: int, min_len: int, d_offs, d_pos, nreads: int | None = None,
               stream=None) -> int:
    """Device locate into torch buffers; returns the total (SaError SA_ENOSPC
    when d_pos is too small: the offsets are written regardless)."""
    n = d_hits.shape[0] if nreads is None else nreads
    total = ctypes.c_int64()
    cap_pos = d_pos.numel() if d_pos is not None else 0
    _check(lib().sa_locate_dev(d.ptr, d_hits.data_ptr(), n, cap, min_len, d_offs.data_ptr(),
                               d_pos.data_ptr() if d_pos is not None else None, cap_pos, _stream_handle(stream),
                               ctypes.byref(total)), "sa_locate_dev")
    return total.value


def sa_tune(d: DIndex, d_reads, d_offs, nreads: int | None = None, stream=None, cache_path: str | None = None):
    """Autotune on a device batch; returns (MatchCfg, ms per batch)."""
    n = (d_offs.numel() - 1) if nreads is None else nreads
    best = MatchCfg()
    ms = ctypes.c_double()
    _check(lib().sa_tune(d.ptr, ctypes.c_void_p(d_reads.data_ptr()), ctypes.c_void_p(d_offs.data_ptr()), n,
                         _stream_handle(stream), cache_path.encode() if cache_path else None, ctypes.byref(best),
                         ctypes.byref(ms)), "sa_tune")
    return best, ms.value


def sa_tune_candidates(d: DIndex, d_offs, nreads: int | None = None, stream=None,
                       around: MatchCfg | None = None) -> list:
    """The configurations sa_tune would time on a batch with these device
    offsets (later stages taken around `around`, default the index's
    defaults)."""
    n = (d_offs.numel() - 1) if nreads is None else nreads
    count = ctypes.c_int()
    args = (d.ptr, ctypes.c_void_p(d_offs.data_ptr()), n, _stream_handle(stream),
            ctypes.byref(around) if around is not None else None)
    _check(lib().sa_tune_candidates(*args, None, 0, ctypes.byref(count)), "sa_tune_candidates")
    out = (MatchCfg * max(1, count.value))()
    _check(lib().sa_tune_candidates(*args, out, count.value, ctypes.byref(count)), "sa_tune_candidates")
    return [out[i] for i in range(count.value)]


# ------------------------------------------------------------------ serving


class Server:
    """Request loop (sa_server) over resident indexes."""

    def __init__(self, refs, **opts):
        o = ServerOpts()
        o.test_fake_free_hbm = -1
        for k, v in opts.items():
            setattr(o, k, int(v))
        self._refs = list(refs)  # keep the indexes alive
        arr = (ctypes.c_void_p * len(self._refs))(*[r.ptr if r is not None else None for r in self._refs])
        out = ctypes.c_void_p()
        _check(lib().sa_server_create(arr, len(self._refs), ctypes.byref(o), ctypes.byref(out)), "sa_server_create")
        self._p = out
        self._pending = {}

    def submit(self, ref: int, data, offs):
        """Queue a request; returns (ticket, out array filled on completion)."""
        data = _bytes(data)
        offs = np.ascontiguousarray(offs, dtype=np.int64)
        n = len(offs) - 1
        out = np.zeros((max(n, 1), 4), dtype=np.int32)
        buf = data if len(data) else np.zeros(1, dtype=np.uint8)
        t = ctypes.c_uint64()
        _check(lib().match_submit(self._p, ref, buf.ctypes.data, offs.ctypes.data, n, out.ctypes.data,
                                  ctypes.byref(t)), "match_submit")
        self._pending[t.value] = out  # must stay alive until the request finishes
        return t.value, out[:n]

    def poll(self, ticket: int, timeout_us: int = 0):
        """(status, stats dict); status SA_PENDING, SA_OK or an error code."""
        st = ReqStats()
        rc = lib().match_poll(self._p, ticket, timeout_us, ctypes.byref(st))
        if rc == SA_ENOTFOUND:
            _check(rc, "match_poll")
        return rc, {"t_submit_ns": st.t_submit_ns, "t_admit_ns": st.t_admit_ns, "t_done_ns": st.t_done_ns,
                    "status": st.status, "nreads": st.nreads}

    def replay(self, refs, datas, offss, arrival_ns, nthreads: int = 8):
        """Open-loop load from native client threads (sa_server_replay):
        request i (reference refs[i], reads datas[i] / offss[i]) is submitted
        arrival_ns[i] ns after the start.  Returns (outs, sched_ns, stats)
        with one (n, 4) int32 result array and one stats dict per request."""
        n = len(refs)
        datas = [_bytes(x) if len(x) else np.zeros(1, dtype=np.uint8) for x in datas]
        offss = [np.ascontiguousarray(o, dtype=np.int64) for o in offss]
        # result arrays written once now, so that their pages are in place
        # before the clock starts (a serving client's buffers are ready)
        outs = [np.full((max(len(o) - 1, 1), 4), -1, dtype=np.int32) for o in offss]
        ref_a = np.ascontiguousarray(refs, dtype=np.int32)
        nr = np.array([len(o) - 1 for o in offss], dtype=np.int64)
        arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        rp = np.array([x.ctypes.data for x in datas], dtype=np.uint64)
        op = np.array([o.ctypes.data for o in offss], dtype=np.uint64)
        outp = np.array([o.ctypes.data for o in outs], dtype=np.uint64)
        sched = np.zeros(n, dtype=np.int64)
        st = (ReqStats * max(n, 1))()
        rc = lib().sa_server_replay(self._p, n, ref_a.ctypes.data, rp.ctypes.data, op.ctypes.data, nr.ctypes.data,
                                    arr.ctypes.data, outp.ctypes.data, nthreads, sched.ctypes.data, st)
        stats = [{"t_submit_ns": st[i].t_submit_ns, "t_admit_ns": st[i].t_admit_ns, "t_done_ns": st[i].t_done_ns,
                  "status": st[i].status, "nreads": st[i].nreads} for i in range(n)]
        _check(rc, "sa_server_replay")
        return [o[:len(f) - 1] for o, f in zip(outs, offss)], sched, stats

    def stats(self) -> dict:
        """Running totals (sa_server_get_stats)."""
        st = ServerStats()
        _check(lib().sa_server_get_stats(self._p, ctypes.byref(st)), "sa_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def destroy(self):
        if self._p:
            _check(lib().sa_server_destroy(self._p), "sa_server_destroy")
            self._p = None
            self._pending.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
