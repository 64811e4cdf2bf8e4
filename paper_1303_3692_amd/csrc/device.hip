// Device-resident index, per-stream scratch, and the batch entry points.
#include <hip/hip_runtime.h>
#include <system_error>
#include <thread>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <vector>
#include <cstring>
#include <mutex>

#include "internal.h"
#include "kernels.h"
#include "device_state.h"

using namespace samatch;

namespace samatch {

int hip_fail(hipError_t e, const char *what) {
    return fail(SA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
}
DeviceGuard::~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
}

void Workspace::drop_graphs() {
    for (GraphEntry &g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
}

Workspace::~Workspace() {
    drop_graphs();
    for (void *p : {(void *)b.qw, (void *)b.qlm, (void *)b.key[0], (void *)b.key[1],
                    (void *)b.val[0], (void *)b.val[1], (void *)b.hist, (void *)b.digit_total,
                    (void *)b.stats})
        if (p) (void)hipFree(p);
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
}

HostSlot::~HostSlot() {
    for (void *p : {(void *)d_reads, (void *)d_offs, (void *)d_out})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)h_reads, (void *)h_offs, (void *)h_out})
        if (p) (void)hipHostFree(p);
    if (done) (void)hipEventDestroy(done);
}

static hipError_t grow(void **p, size_t bytes) {
    if (*p) {
        hipError_t e = hipFree(*p);
        *p = nullptr;
        if (e != hipSuccess) return e;
    }
    return hipMalloc(p, bytes ? bytes : 16);
}

int Workspace::reserve(int64_t nreads) {
    if (nreads <= cap) return SA_OK;
    drop_graphs();  // captured graphs point at the buffers about to be replaced
    const int64_t c = std::max<int64_t>(nreads, 1024);
    const int64_t nblocks = (c + kSortTile - 1) / kSortTile;
    hipError_t e;
    if ((e = grow((void **)&b.qw, sizeof(uint64_t) * kWMax * (size_t)c)) != hipSuccess ||
        (e = grow((void **)&b.qlm, sizeof(int2) * (size_t)c)) != hipSuccess ||
        (e = grow((void **)&b.key[0], sizeof(uint32_t) * (size_t)c)) != hipSuccess ||
        (e = grow((void **)&b.key[1], sizeof(uint32_t) * (size_t)c)) != hipSuccess ||
        (e = grow((void **)&b.val[0], sizeof(uint32_t) * (size_t)c)) != hipSuccess ||
        (e = grow((void **)&b.val[1], sizeof(uint32_t) * (size_t)c)) != hipSuccess ||
        (e = grow((void **)&b.hist, sizeof(uint32_t) * 256 * (size_t)nblocks)) != hipSuccess)
        return hip_fail(e, "scratch allocation");
    if (!b.digit_total && (e = hipMalloc((void **)&b.digit_total, sizeof(uint32_t) * 256)) != hipSuccess)
        return hip_fail(e, "scratch allocation");
    if (!b.stats && (e = hipMalloc((void **)&b.stats, sizeof(unsigned long long) * kStatWords)) != hipSuccess)
        return hip_fail(e, "scratch allocation");
    for (hipEvent_t &ev_i : ev)
        if (!ev_i && (e = hipEventCreate(&ev_i)) != hipSuccess) return hip_fail(e, "event creation");
    cap = c;
    return SA_OK;
}

int HostSlot::reserve(int64_t nreads, int64_t nbytes) {
    hipError_t e;
    if (!done && (e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "event creation");
    if (nbytes > bytes_cap) {
        const int64_t c = std::max<int64_t>(nbytes, 1 << 20);
        if (h_reads) (void)hipHostFree(h_reads);
        h_reads = nullptr;
        bytes_cap = 0;
        if ((e = hipHostMalloc((void **)&h_reads, (size_t)c, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "pinned staging");
        if ((e = grow((void **)&d_reads, (size_t)c)) != hipSuccess) return hip_fail(e, "staging");
        bytes_cap = c;
    }
    if (nreads > reads_cap) {
        const int64_t c = std::max<int64_t>(nreads, 1024);
        if (h_offs) (void)hipHostFree(h_offs);
        if (h_out) (void)hipHostFree(h_out);
        h_offs = nullptr;
        h_out = nullptr;
        reads_cap = 0;
        if ((e = hipHostMalloc((void **)&h_offs, sizeof(int64_t) * (size_t)(c + 1), hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc((void **)&h_out, sizeof(sa_hit) * (size_t)c, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "pinned staging");
        if ((e = grow((void **)&d_offs, sizeof(int64_t) * (size_t)(c + 1))) != hipSuccess ||
            (e = grow((void **)&d_out, sizeof(sa_hit) * (size_t)c)) != hipSuccess)
            return hip_fail(e, "staging");
        reads_cap = c;
    }
    return SA_OK;
}

Workspace *workspace_for(sa_dindex *d, hipStream_t s) {
    std::lock_guard<std::mutex> g(d->mu);
    auto &slot = d->ws[(void *)s];
    if (!slot) slot.reset(new Workspace);
    return slot.get();
}

BucketTable bucket_table(const sa_match_cfg &c) {
    BucketTable bt{};
    bt.count = std::max(1, std::min(8, c.nbuckets));
    for (int i = 0; i < bt.count; i++) bt.edge[i] = c.bucket_edge[i];
    bt.edge[bt.count - 1] = SA_MAX_READ;
    return bt;
}

int check_cfg(const sa_dindex *d, const sa_match_cfg &c) {
    if (c.kernel != SA_KERNEL_TUNED && c.kernel != SA_KERNEL_PLAIN) return fail(SA_EINVAL, "unknown kernel");
    if (c.kernel == SA_KERNEL_PLAIN) return SA_OK;
    if (c.tile_levels < 1 || c.tile_levels > d->tile_levels)
        return fail(SA_EINVAL, "tile_levels must be in 1.." + std::to_string(d->tile_levels));
    if (c.block != 256 && c.block != 512 && c.block != 1024) return fail(SA_EINVAL, "block must be 256, 512 or 1024");
    if (c.blocks_per_cu < 1 || c.blocks_per_cu > 16) return fail(SA_EINVAL, "blocks_per_cu must be in 1..16");
    if (c.nbuckets < 1 || c.nbuckets > 8) return fail(SA_EINVAL, "nbuckets must be in 1..8");
    if (c.group < 1 || c.group > 64) return fail(SA_EINVAL, "group must be in 1..64");
    if (c.sort != 0 && c.sort != 1 && c.sort != 8 && c.sort != 16 && c.sort != 24)
        return fail(SA_EINVAL, "sort must be 0, 1, 8, 16 or 24");
    if (c.inline_pack != 0 && c.inline_pack != 1) return fail(SA_EINVAL, "inline_pack must be 0 or 1");
    if (c.defer < 0 || c.defer > 1024) return fail(SA_EINVAL, "defer must be in 0..1024");
    if (c.max_words != kShortWords && c.max_words != kWMax)
        return fail(SA_EINVAL, "max_words must be " + std::to_string(kShortWords) + " or " + std::to_string(kWMax));
    for (int i = 0; i + 1 < c.nbuckets; i++)
        if (c.bucket_edge[i] < 1 || (i > 0 && c.bucket_edge[i] <= c.bucket_edge[i - 1]))
            return fail(SA_EINVAL, "bucket edges must ascend");
    return SA_OK;
}

sa_match_cfg resolve_cfg(const sa_dindex *d, const sa_match_cfg *cfg) {
    sa_match_cfg c = cfg ? *cfg : d->defaults;
    const sa_match_cfg &def = d->defaults;
    if (c.kernel == SA_KERNEL_TUNED) {
        if (c.tile_levels == 0) c.tile_levels = def.tile_levels;
        if (c.block == 0) c.block = def.block;
        if (c.blocks_per_cu == 0) c.blocks_per_cu = def.blocks_per_cu;
        if (c.group == 0) c.group = def.group;
        if (c.max_words == 0) c.max_words = def.max_words;
        if (c.nbuckets == 0) {
            c.nbuckets = def.nbuckets;
            std::memcpy(c.bucket_edge, def.bucket_edge, sizeof c.bucket_edge);
        }
    }
    return c;
}

bool packs_inline(const sa_match_cfg &c) {
    return c.kernel == SA_KERNEL_TUNED && c.inline_pack && c.sort == 0 &&
           tuned_lds_bytes(c.tile_levels, c.count ? 256 : c.block, true, c.max_words) <= inline_lds_limit();
}

// Enqueue the whole device pipeline for one batch: pack, optional prefix
// sort, search.  All launches go to stream s.  d_ends may be NULL (CSR
// offsets) or give each read's end (reads scattered over d_reads).
int enqueue_batch(sa_dindex *d, Workspace *ws, const uint8_t *d_reads, const int64_t *d_offs, const int64_t *d_ends,
                  int64_t nreads, sa_hit *d_out, hipStream_t s, const sa_match_cfg &c) {
    int rc = ws->reserve(nreads);
    if (rc) return rc;
    rc = enqueue_pipeline(d, ws->b, c.profile ? ws->ev : nullptr, d_reads, d_offs, d_ends, nreads, d_out, s, c);
    if (rc) return rc;
    ws->profiled = c.profile != 0;
    ws->counted = c.count != 0;
    return SA_OK;
}

int enqueue_pipeline(sa_dindex *d, const BatchBuffers &b, const hipEvent_t *ev, const uint8_t *d_reads,
                     const int64_t *d_offs, const int64_t *d_ends, int64_t nreads, sa_hit *d_out, hipStream_t s,
                     const sa_match_cfg &c) {
    const bool prof = ev != nullptr;
    hipError_t e = hipSuccess;
    if (prof && (e = hipEventRecord(ev[0], s)) != hipSuccess) return hip_fail(e, "event record");
    // reads in input order: the tuned kernel can pack them itself when its
    // tile and the waves' packing areas fit in LDS
    const bool inl = packs_inline(c);
    if (inl) {
        e = launch_clear_stats(b, s);
        if (e != hipSuccess) return hip_fail(e, "stats clear launch");
    } else {
        BucketTable bt = bucket_table(c);
        bt.keys = (c.kernel == SA_KERNEL_TUNED && c.sort) ? 1 : 0;
        e = launch_pack(d_reads, d_offs, d_ends, nreads, b, bt, s);
        if (e != hipSuccess) return hip_fail(e, "pack launch");
    }
    if (prof && (e = hipEventRecord(ev[1], s)) != hipSuccess) return hip_fail(e, "event record");
    const uint32_t *order = nullptr, *sorted_key = nullptr;
    int key_shift = 0;
    uint32_t key_mask = 0;
    if (c.kernel == SA_KERNEL_TUNED && c.sort && !inl) {
        // The key is (length bucket << 24 | first 12 bases).  Prefix bits
        // beyond about one group per 64-read chunk put no more lanes on
        // shared pivots, so the sort covers the top 8, 16 or 24 prefix bits
        // (2^bits >= nreads / 64), then the bucket byte when there is one.
        int pbits = 8;
        if (c.sort == 8 || c.sort == 16 || c.sort == 24) pbits = c.sort;
        else while (pbits < 24 && ((int64_t)1 << pbits) < nreads / 64) pbits += 8;
        int which = 0;
        const int lo_bit = 24 - pbits, hi_bit = c.nbuckets > 1 ? 32 : 24;
        e = launch_sort(b, nreads, lo_bit, hi_bit, &which, s);
        if (e != hipSuccess) return hip_fail(e, "sort launch");
        if (nreads > 1) {
            order = b.val[which];
            sorted_key = b.key[which];
            key_shift = lo_bit;
            key_mask = hi_bit - lo_bit >= 32 ? 0xFFFFFFFFu : ((1u << (hi_bit - lo_bit)) - 1u);
        }
    }
    if (prof && (e = hipEventRecord(ev[2], s)) != hipSuccess) return hip_fail(e, "event record");
    if (c.kernel == SA_KERNEL_PLAIN) {
        e = launch_search_plain(d->view, b, nreads, d_out, c.count != 0, s);
        if (e != hipSuccess) return hip_fail(e, "plain search launch");
    } else {
        // persistent workgroups; a batch too small to give each of them
        // `group` chunks of 64 reads takes smaller blocks, and no more
        // workgroups than there are blocks (each one stages the tile)
        const int64_t chunks = (nreads + 63) / 64, gmax = std::max<int64_t>(1, (int64_t)d->cu_count * c.blocks_per_cu);
        const int group = (int)std::max<int64_t>(1, std::min<int64_t>(c.group, chunks / gmax));
        const int grid = (int)std::min<int64_t>(gmax, (chunks + group - 1) / group);
        e = launch_search_tuned(d->view, c.tile_levels, c.prefix_table, c.block, grid, group, c.defer, b, order,
                                inl ? d_reads : nullptr, inl ? d_offs : nullptr, inl ? d_ends : nullptr, nreads,
                                inl ? c.max_words : kWMax, d_out, c.count != 0, s);
        if (e != hipSuccess) return hip_fail(e, "tuned search launch");
    }
    // reads longer than kShortMax: their own kernel, over the tail of the sorted order
    const uint32_t long_field = (long_read_key(c.nbuckets) >> key_shift) & key_mask;
    e = launch_search_long(d->view, d_reads, d_offs, b, order, sorted_key, key_shift, key_mask, long_field,
                           c.prefix_table, inl, 32 * (inl ? c.max_words : kWMax), inl ? d_ends : nullptr,
                           (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)d->cu_count * 8, (nreads + 63) / 64)),
                           nreads, d_out, c.count != 0, s);
    if (e != hipSuccess) return hip_fail(e, "long-read search launch");
    if (prof && (e = hipEventRecord(ev[3], s)) != hipSuccess) return hip_fail(e, "event record");
    return SA_OK;
}

static bool same_cfg(const sa_match_cfg &a, const sa_match_cfg &b) { return std::memcmp(&a, &b, sizeof a) == 0; }

int run_batch(sa_dindex *d, Workspace *ws, const uint8_t *d_reads, const int64_t *d_offs, const int64_t *d_ends,
              int64_t nreads, sa_hit *d_out, hipStream_t s, const sa_match_cfg &c) {
    // the null stream cannot be captured; profiling and counting need eager launches
    if (!c.use_graph || !s || c.profile || c.count)
        return enqueue_batch(d, ws, d_reads, d_offs, d_ends, nreads, d_out, s, c);
    int rc = ws->reserve(nreads);  // no allocation may happen during capture
    if (rc) return rc;
    for (GraphEntry &g : ws->graphs) {
        if (g.reads == d_reads && g.offs == d_offs && g.ends == d_ends && g.out == d_out && g.nreads == nreads &&
            same_cfg(g.cfg, c)) {
            g.last_use = ++ws->graph_clock;
            hipError_t e = hipGraphLaunch(g.exec, s);
            return e == hipSuccess ? SA_OK : hip_fail(e, "graph launch");
        }
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    rc = enqueue_batch(d, ws, d_reads, d_offs, d_ends, nreads, d_out, s, c);
    e = hipStreamEndCapture(s, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "graph instantiation");
    if (ws->graphs.size() >= Workspace::kMaxGraphs) {
        auto oldest = std::min_element(ws->graphs.begin(), ws->graphs.end(),
                                       [](const GraphEntry &x, const GraphEntry &y) { return x.last_use < y.last_use; });
        (void)hipGraphExecDestroy(oldest->exec);
        ws->graphs.erase(oldest);
    }
    ws->graphs.push_back(GraphEntry{d_reads, d_offs, d_ends, d_out, nreads, c, exec, ++ws->graph_clock});
    e = hipGraphLaunch(exec, s);
    return e == hipSuccess ? SA_OK : hip_fail(e, "graph launch");
}

}  // namespace samatch

namespace {

// Prefix-table length of a text of n bases: round(log4 n) + 2, so that a
// table entry's bracket holds about a sixteenth of a row (most lookups then
// need at most the one probe whose suffix travels with the entry, and its
// first 32 bases come with the entry too), at most kMaxPrefixBases, and
// shorter while the table would take more than a quarter of the device
// memory free (free_bytes); none below 4096 bases.  The table takes 4^k
// 16-byte entries, about 256 bytes per base.  On MI355X, for a 250 Mbp
// reference (k = 16, a 68.7 GB table), each base added cut the search by
// about 11-15 % (k = 14: 6.47 ms, 15: 6.05, 16: 5.40); for a 16 Mbp
// reference k = 13 and 14 gained 8 % and 3 %.
int default_prefix_bases(int64_t n, size_t free_bytes) {
    if (n < 4096) return 0;
    int k = std::max(4, std::min(kMaxPrefixBases, (int)std::lround(std::log2((double)n) / 2.0) + 2));
    while (k > 4 && (((size_t)1 << (2 * k)) + 1) * sizeof(PrefixEntry) > free_bytes / 4) k--;
    return k;
}

// (Re)build the prefix table of d with k bases (0: none).  Captured graphs
// hold the old index view, so every workspace drops them.
int set_prefix_table(sa_dindex *d, int k) {
    hipError_t e;
    if (d->d_ptab) {
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "prefix table release");
        (void)hipFree(d->d_ptab);
        d->d_ptab = nullptr;
    }
    d->view.ptab = nullptr;
    d->view.ptab_k = 0;
    d->ptab_bytes = 0;
    {
        std::lock_guard<std::mutex> lk(d->mu);
        for (auto &kv : d->ws) {
            std::lock_guard<std::mutex> wl(kv.second->mu);
            kv.second->drop_graphs();
        }
    }
    if (k > 0) {
        const size_t entries = ((size_t)1 << (2 * k)) + 1;
        if ((e = hipMalloc((void **)&d->d_ptab, entries * sizeof(PrefixEntry))) != hipSuccess)
            return hip_fail(e, "prefix table allocation");
        DevIndex v = d->view;
        v.ptab = d->d_ptab;
        v.ptab_k = k;
        if ((e = launch_build_prefix_table(v, k, d->d_ptab, nullptr)) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess)
            return hip_fail(e, "prefix table build");
        d->view = v;
        d->ptab_bytes = (int64_t)(entries * sizeof(PrefixEntry));
    }
    d->defaults.prefix_table = k > 0 ? 1 : 0;
    d->defaults.sort = k > 0 ? 0 : 1;
    return SA_OK;
}

// Device index from the packed text and either a host suffix array
// (host_sa) or one built here on the device.
int make_dindex(int device, int64_t n, const std::vector<uint64_t> &packed, const int32_t *host_sa,
                sa_dindex **out) {
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(SA_EINVAL, "no such device");
    DeviceGuard g(device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    std::unique_ptr<sa_dindex> d(new sa_dindex);
    d->device = device;
    d->n = n;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if ((e = prepare_kernels()) != hipSuccess) return hip_fail(e, "kernel attributes");
    d->cu_count = prop.multiProcessorCount;
    std::snprintf(d->arch, sizeof d->arch, "%s", prop.gcnArchName);
    const size_t text_bytes = sizeof(uint64_t) * packed.size();
    const size_t sa_bytes = sizeof(int32_t) * (size_t)n;
    int levels = 0;
    while (levels < kMaxTileLevels && ((int64_t)1 << levels) - 1 < n) levels++;
    d->tile_levels = std::max(1, levels);
    const size_t nodes = ((size_t)1 << d->tile_levels) - 1;
    if ((e = hipMalloc((void **)&d->d_text, text_bytes)) != hipSuccess ||
        (e = hipMalloc((void **)&d->d_sa, sa_bytes)) != hipSuccess ||
        (e = hipMalloc((void **)&d->d_tile_key, nodes * sizeof(uint64_t))) != hipSuccess ||
        (e = hipMalloc((void **)&d->d_tile_sa, nodes * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc((void **)&d->d_rows, sizeof(RowRec) * (size_t)n)) != hipSuccess)
        return hip_fail(e, "index allocation");
    if ((e = hipMemcpy(d->d_text, packed.data(), text_bytes, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "index upload");
    if (host_sa) {
        if ((e = hipMemcpy(d->d_sa, host_sa, sa_bytes, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "index upload");
    } else {
        int rc = build_sa_device(d->d_text, n, d->d_sa, nullptr, nullptr, &d->built);
        if (rc) return rc;
    }
    if ((e = launch_build_rows(d->d_text, d->d_sa, (int32_t)n, d->d_rows, nullptr)) != hipSuccess ||
        (e = launch_build_tile(d->d_text, d->d_sa, (int32_t)n, d->tile_levels, d->d_tile_key, d->d_tile_sa,
                               nullptr)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess)
        return hip_fail(e, "tile build");
    DevIndex v{};
    v.text = d->d_text;
    v.sa = d->d_sa;
    v.tile_key = d->d_tile_key;
    v.tile_sa = d->d_tile_sa;
    v.rows = d->d_rows;
    v.n = (int32_t)n;
    d->view = v;
    size_t free_bytes = 0, total_bytes = 0;
    if ((e = hipMemGetInfo(&free_bytes, &total_bytes)) != hipSuccess) return hip_fail(e, "device memory query");
    if (int rc = set_prefix_table(d.get(), default_prefix_bases(n, free_bytes))) return rc;
    sa_match_cfg &c = d->defaults;
    std::memset(&c, 0, sizeof c);
    c.kernel = SA_KERNEL_TUNED;
    // one workgroup of 16 waves per compute unit; with a prefix table the
    // tile serves only reads with fewer than k leading bases
    c.tile_levels = std::min(d->view.ptab_k > 0 ? 8 : 10, d->tile_levels);
    c.block = 1024;
    c.blocks_per_cu = 1;
    c.nbuckets = 1;
    c.bucket_edge[0] = SA_MAX_READ;
    // with the prefix table, reads in input order search as fast as sorted
    // ones and the sort is saved (MI355X, every workload measured)
    c.sort = d->view.ptab_k > 0 ? 0 : 1;
    c.use_graph = 0;
    c.group = 4;
    c.prefix_table = d->view.ptab_k > 0 ? 1 : 0;
    c.inline_pack = 1;
    c.max_words = kWMax;
    c.defer = kDefaultDefer;
    *out = d.release();
    return SA_OK;
}

}  // namespace

extern "C" int sa_upload(const sa_index *ix, int device, sa_dindex **out) {
    clear_error();
    if (!ix || !out) return fail(SA_EINVAL, "NULL argument");
    return make_dindex(device, ix->n, ix->packed, ix->sa.data(), out);
}

extern "C" int sa_build_device(const char *text, int64_t n, int device, sa_dindex **out) {
    clear_error();
    if (!out) return fail(SA_EINVAL, "NULL argument");
    *out = nullptr;
    int rc = check_text(text, n);
    if (rc) return rc;
    std::vector<uint64_t> packed;
    try {
        pack_text(text, n, packed);
    } catch (const std::bad_alloc &) {
        return fail(SA_ENOMEM, "packing");
    }
    return make_dindex(device, n, packed, nullptr, out);
}

extern "C" int sa_download(const sa_dindex *d, sa_index **out) {
    clear_error();
    if (!d || !out) return fail(SA_EINVAL, "NULL argument");
    *out = nullptr;
    std::unique_ptr<sa_index> ix(new (std::nothrow) sa_index);
    if (!ix) return fail(SA_ENOMEM, "index allocation");
    try {
        ix->n = d->n;
        ix->packed.assign((size_t)((d->n + 31) / 32 + kPadWords), 0);
        ix->sa.assign((size_t)d->n, 0);
    } catch (const std::bad_alloc &) {
        return fail(SA_ENOMEM, "index allocation");
    }
    DeviceGuard g(d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    hipError_t e;
    if ((e = hipMemcpy(ix->packed.data(), d->d_text, sizeof(uint64_t) * ix->packed.size(), hipMemcpyDeviceToHost)) !=
            hipSuccess ||
        (e = hipMemcpy(ix->sa.data(), d->d_sa, sizeof(int32_t) * ix->sa.size(), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "index download");
    *out = ix.release();
    return SA_OK;
}

extern "C" int sa_dindex_bytes(const sa_dindex *d, int64_t bytes[5]) {
    clear_error();
    if (!d || !bytes) return fail(SA_EINVAL, "NULL argument");
    const int64_t n = d->n;
    bytes[0] = (int64_t)sizeof(uint64_t) * (((n + 31) >> 5) + kPadWords);
    bytes[1] = (int64_t)sizeof(int32_t) * n;
    bytes[2] = (int64_t)sizeof(RowRec) * n;
    bytes[3] = d->ptab_bytes;
    bytes[4] = (int64_t)((((size_t)1 << d->tile_levels) - 1) * (sizeof(uint64_t) + sizeof(int32_t)));
    return SA_OK;
}

extern "C" int sa_set_prefix_table(sa_dindex *d, int k) {
    clear_error();
    if (!d) return fail(SA_EINVAL, "NULL argument");
    if (k < 0 || (k > 0 && k < 4) || k > kMaxPrefixBases) return fail(SA_EINVAL, "prefix bases must be 0 or 4.." + std::to_string(kMaxPrefixBases));
    if (k > 0 && d->n < 4096) return fail(SA_EINVAL, "a prefix table needs a text of at least 4096 bases");
    DeviceGuard g(d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    return set_prefix_table(d, k);
}

extern "C" int sa_dindex_build_info(const sa_dindex *d, int *steps, int64_t *sorted_pairs) {
    clear_error();
    if (!d) return fail(SA_EINVAL, "NULL argument");
    if (steps) *steps = d->built.steps;
    if (sorted_pairs) *sorted_pairs = d->built.sorted_elems;
    return SA_OK;
}

sa_dindex::~sa_dindex() {
    DeviceGuard g(device);
    ws.clear();
    for (void *p : {(void *)d_text, (void *)d_sa, (void *)d_tile_key, (void *)d_tile_sa, (void *)d_rows,
                    (void *)d_ptab})
        if (p) (void)hipFree(p);
}

extern "C" void sa_dfree(sa_dindex *d) { delete d; }

extern "C" int64_t sa_dindex_length(const sa_dindex *d) { return d ? d->n : -1; }

extern "C" int sa_default_cfg(const sa_dindex *d, sa_match_cfg *cfg) {
    clear_error();
    if (!d || !cfg) return fail(SA_EINVAL, "NULL argument");
    *cfg = d->defaults;
    return SA_OK;
}

extern "C" int match_batch_dev(const sa_dindex *dc, const uint8_t *d_reads, const int64_t *d_offs, int64_t nreads,
                               sa_hit *d_out, void *hip_stream, const sa_match_cfg *cfg) {
    clear_error();
    if (!dc || !d_offs || (nreads > 0 && (!d_reads || !d_out))) return fail(SA_EINVAL, "NULL argument");
    if (nreads < 0 || nreads > INT32_MAX) return fail(SA_EINVAL, "nreads out of range");
    if (nreads == 0) return SA_OK;
    sa_dindex *d = const_cast<sa_dindex *>(dc);
    const sa_match_cfg c = resolve_cfg(d, cfg);
    int rc = check_cfg(d, c);
    if (rc) return rc;
    DeviceGuard g(d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Workspace *ws = workspace_for(d, s);
    std::lock_guard<std::mutex> lk(ws->mu);
    return run_batch(d, ws, d_reads, d_offs, nullptr, nreads, d_out, s, c);
}

// Host batches stream through pinned staging in chunks of whole reads.
constexpr int64_t kHostChunkBytes = (int64_t)32 << 20;
constexpr int64_t kHostChunkReads = (int64_t)1 << 19;

// memcpy split over a few threads (one copy thread moves ~10 GB/s; the
// staging copies would otherwise bound a host batch below the bus rate).
static void host_copy(void *dst, const void *src, size_t bytes) {
    const size_t kPart = (size_t)4 << 20;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>({(size_t)8, (size_t)hw, bytes / kPart});
    if (nt <= 1) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const size_t part = (bytes / nt + 63) & ~(size_t)63;
    std::vector<std::thread> th;
    try {
        for (size_t t = 1; t < nt; t++) {
            const size_t a = t * part, b = std::min(bytes, a + part);
            if (a >= b) break;
            th.emplace_back([=] { std::memcpy((char *)dst + a, (const char *)src + a, b - a); });
        }
    } catch (const std::system_error &) {
        // no more threads: this thread copies what was not handed out
    }
    std::memcpy(dst, src, std::min(bytes, part));
    const size_t done = (th.size() + 1) * part;  // parts 1 .. th.size() went to the threads
    if (done < bytes) std::memcpy((char *)dst + done, (const char *)src + done, bytes - done);
    for (std::thread &x : th) x.join();
}

extern "C" int match_batch(const sa_dindex *dc, const char *reads, const int64_t *offs, int64_t nreads,
                           sa_hit *out, void *hip_stream, const sa_match_cfg *cfg) {
    clear_error();
    if (!dc || !offs || (nreads > 0 && (!reads || !out))) return fail(SA_EINVAL, "NULL argument");
    if (nreads < 0 || nreads > INT32_MAX) return fail(SA_EINVAL, "nreads out of range");
    if (nreads == 0) return SA_OK;
    if (offs[0] < 0) return fail(SA_EINVAL, "negative offset");
    for (int64_t i = 0; i < nreads; i++) {
        const int64_t m = offs[i + 1] - offs[i];
        if (m < 0) return fail(SA_EINVAL, "offsets decrease at read " + std::to_string(i));
        if (m > SA_MAX_READ) return fail(SA_ETOOBIG, "read " + std::to_string(i) + " is longer than SA_MAX_READ");
    }
    sa_dindex *d = const_cast<sa_dindex *>(dc);
    const sa_match_cfg c = resolve_cfg(d, cfg);
    int rc = check_cfg(d, c);
    if (rc) return rc;
    DeviceGuard g(d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Workspace *ws = workspace_for(d, s);
    std::lock_guard<std::mutex> lk(ws->mu);
    // chunks of whole reads, at most kHostChunkBytes of ASCII (or one read)
    // and kHostChunkReads reads each; chunk k uses slot k % 2, so the host
    // copies chunk k in (and chunk k - 2 out) while the device works on k - 1
    std::vector<int64_t> cuts{0};
    int64_t most = 0;
    while (cuts.back() < nreads) {
        const int64_t r0 = cuts.back();
        const int64_t by_bytes =
            (int64_t)(std::upper_bound(offs + r0 + 1, offs + nreads + 1, offs[r0] + kHostChunkBytes) - offs) - 1;
        const int64_t r1 = std::max(r0 + 1, std::min(r0 + kHostChunkReads, by_bytes));
        most = std::max(most, r1 - r0);
        cuts.push_back(r1);
    }
    if ((rc = ws->reserve(most))) return rc;  // no scratch growth between chunks
    const size_t nchunks = cuts.size() - 1;
    auto finish = [&](size_t k) -> int {
        HostSlot &hs = ws->host[k & 1];
        hipError_t e = hipEventSynchronize(hs.done);
        if (e != hipSuccess) return hip_fail(e, "batch download");
        host_copy(out + cuts[k], hs.h_out, sizeof(sa_hit) * (size_t)(cuts[k + 1] - cuts[k]));
        return SA_OK;
    };
    // on an error, nothing may still be in flight on the staging buffers
    auto bail = [&](int code) {
        (void)hipStreamSynchronize(s);
        return code;
    };
    for (size_t k = 0; k < nchunks; k++) {
        HostSlot &hs = ws->host[k & 1];
        if (k >= 2 && (rc = finish(k - 2))) return bail(rc);  // also frees the slot
        const int64_t r0 = cuts[k], n = cuts[k + 1] - r0, b0 = offs[r0], nb = offs[cuts[k + 1]] - b0;
        if ((rc = hs.reserve(n, nb))) return bail(rc);
        host_copy(hs.h_reads, reads + b0, (size_t)nb);
        for (int64_t i = 0; i <= n; i++) hs.h_offs[i] = offs[r0 + i] - b0;
        hipError_t e;
        if ((e = hipMemcpyAsync(hs.d_reads, hs.h_reads, (size_t)nb, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(hs.d_offs, hs.h_offs, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, s)) !=
                hipSuccess)
            return bail(hip_fail(e, "batch upload"));
        if ((rc = enqueue_batch(d, ws, hs.d_reads, hs.d_offs, nullptr, n, hs.d_out, s, c))) return bail(rc);
        if ((e = hipMemcpyAsync(hs.h_out, hs.d_out, sizeof(sa_hit) * (size_t)n, hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipEventRecord(hs.done, s)) != hipSuccess)
            return bail(hip_fail(e, "batch download"));
    }
    for (size_t k = nchunks >= 2 ? nchunks - 2 : 0; k < nchunks; k++)
        if ((rc = finish(k))) return bail(rc);
    return SA_OK;
}

static Workspace *existing_workspace(const sa_dindex *dc, void *stream) {
    sa_dindex *d = const_cast<sa_dindex *>(dc);
    std::lock_guard<std::mutex> g(d->mu);
    auto it = d->ws.find(stream);
    return it == d->ws.end() ? nullptr : it->second.get();
}

extern "C" int sa_stage_times(const sa_dindex *d, void *hip_stream, double ms[4]) {
    clear_error();
    if (!d || !ms) return fail(SA_EINVAL, "NULL argument");
    DeviceGuard g(d->device);
    Workspace *ws = existing_workspace(d, hip_stream);
    if (!ws) return fail(SA_EINVAL, "no batch on this stream");
    std::lock_guard<std::mutex> lk(ws->mu);
    if (!ws->profiled) return fail(SA_EINVAL, "the last batch on this stream was not profiled");
    hipError_t e = hipEventSynchronize(ws->ev[3]);
    if (e != hipSuccess) return hip_fail(e, "event wait");
    float t[3] = {0, 0, 0}, all = 0;
    for (int i = 0; i < 3; i++)
        if ((e = hipEventElapsedTime(&t[i], ws->ev[i], ws->ev[i + 1])) != hipSuccess) return hip_fail(e, "event time");
    if ((e = hipEventElapsedTime(&all, ws->ev[0], ws->ev[3])) != hipSuccess) return hip_fail(e, "event time");
    for (int i = 0; i < 3; i++) ms[i] = t[i];
    ms[3] = all;
    return SA_OK;
}

extern "C" int sa_probe_counts(const sa_dindex *d, void *hip_stream, int64_t c[10]) {
    clear_error();
    if (!d || !c) return fail(SA_EINVAL, "NULL argument");
    DeviceGuard g(d->device);
    Workspace *ws = existing_workspace(d, hip_stream);
    if (!ws) return fail(SA_EINVAL, "no batch on this stream");
    std::lock_guard<std::mutex> lk(ws->mu);
    if (!ws->counted) return fail(SA_EINVAL, "the last batch on this stream was not counted");
    unsigned long long h[10];
    hipError_t e = hipMemcpyAsync(h, ws->b.stats, sizeof h, hipMemcpyDeviceToHost, static_cast<hipStream_t>(hip_stream));
    if (e == hipSuccess) e = hipStreamSynchronize(static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "counter download");
    for (int i = 0; i < 10; i++) c[i] = (int64_t)h[i];
    return SA_OK;
}
