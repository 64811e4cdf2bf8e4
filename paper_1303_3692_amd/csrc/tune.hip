// Autotuner: times candidate launch configurations of the tuned path on a
// caller-supplied device batch and keeps the fastest as the index default.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "device_state.h"

using namespace samatch;

#ifndef SAMATCH_BUILD_ID
#define SAMATCH_BUILD_ID "dev"
#endif

namespace {

// Length histogram of the batch in 32-base classes (device offsets copied
// to the host once).
int length_histogram(const int64_t *d_offs, int64_t nreads, hipStream_t s, std::vector<int64_t> &hist) {
    std::vector<int64_t> offs((size_t)nreads + 1);
    hipError_t e = hipMemcpyAsync(offs.data(), d_offs, sizeof(int64_t) * offs.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "length histogram");
    hist.assign(SA_MAX_READ / 32 + 1, 0);
    for (int64_t i = 0; i < nreads; i++) {
        const int64_t m = std::max<int64_t>(0, std::min<int64_t>(offs[i + 1] - offs[i], SA_MAX_READ));
        hist[(size_t)((m + 31) / 32)]++;
    }
    return SA_OK;
}

std::string cache_key(const sa_dindex *d, const std::vector<int64_t> &hist, int64_t nreads) {
    std::ostringstream k;
    k << SAMATCH_BUILD_ID << "|" << d->arch << "|n=" << d->n << "|cu=" << d->cu_count << "|h=";
    // length classes present with their share in percent, so that batches of
    // the same shape share a tuning
    for (size_t i = 0; i < hist.size(); i++) {
        if (!hist[i]) continue;
        k << i << ":" << (hist[i] * 100 + nreads / 2) / std::max<int64_t>(1, nreads) << ",";
    }
    return k.str();
}

std::string cfg_json(const sa_match_cfg &c) {
    std::ostringstream o;
    o << "\"tile_levels\":" << c.tile_levels << ",\"block\":" << c.block << ",\"blocks_per_cu\":" << c.blocks_per_cu
      << ",\"group\":" << c.group << ",\"prefix_table\":" << c.prefix_table << ",\"sort\":" << c.sort
      << ",\"inline_pack\":" << c.inline_pack << ",\"max_words\":" << c.max_words << ",\"defer\":" << c.defer
      << ",\"nbuckets\":" << c.nbuckets << ",\"bucket_edge\":[";
    for (int i = 0; i < c.nbuckets; i++) o << (i ? "," : "") << c.bucket_edge[i];
    o << "]";
    return o.str();
}

int json_int(const std::string &line, const std::string &name, int dflt) {
    const std::string pat = "\"" + name + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return dflt;
    return std::atoi(line.c_str() + p + pat.size());
}

bool parse_cached(const std::string &path, const std::string &key, sa_match_cfg &c, double &ms) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    const std::string kpat = "\"key\":\"" + key + "\"";
    while (std::getline(f, line)) {
        if (line.find(kpat) == std::string::npos) continue;
        std::memset(&c, 0, sizeof c);
        c.kernel = SA_KERNEL_TUNED;
        c.tile_levels = json_int(line, "tile_levels", 12);
        c.block = json_int(line, "block", 256);
        c.blocks_per_cu = json_int(line, "blocks_per_cu", 8);
        c.group = json_int(line, "group", 4);
        c.prefix_table = json_int(line, "prefix_table", 0);
        c.sort = json_int(line, "sort", 1);
        c.inline_pack = json_int(line, "inline_pack", 1);
        c.max_words = json_int(line, "max_words", kWMax);
        c.defer = json_int(line, "defer", 0);
        c.nbuckets = std::max(1, std::min(8, json_int(line, "nbuckets", 1)));
        const size_t p = line.find("\"bucket_edge\":[");
        if (p != std::string::npos) {
            const char *q = line.c_str() + p + 15;
            for (int i = 0; i < c.nbuckets; i++) {
                c.bucket_edge[i] = std::atoi(q);
                while (*q && *q != ',' && *q != ']') q++;
                if (*q == ',') q++;
            }
        }
        const size_t pm = line.find("\"ms\":");
        ms = pm == std::string::npos ? 0.0 : std::atof(line.c_str() + pm + 5);
        found = true;  // the last matching line wins
    }
    return found;
}

// Bucket layouts to try: one bucket, and edges at multiples of 32 bases
// that split the batch's length classes into 2, 3 or 4 groups of similar
// read counts.
std::vector<std::vector<int>> bucket_layouts(const std::vector<int64_t> &hist) {
    std::vector<std::vector<int>> out;
    out.push_back({SA_MAX_READ});
    int64_t total = 0;
    int classes = 0;
    for (int64_t h : hist) {
        total += h;
        classes += h > 0;
    }
    for (int parts = 2; parts <= 4 && parts <= classes; parts++) {
        std::vector<int> edges;
        int64_t acc = 0;
        int next = 1;
        for (size_t i = 0; i < hist.size() && next < parts; i++) {
            acc += hist[i];
            if (acc * parts >= total * next && hist[i] > 0) {
                edges.push_back((int)i * 32);
                next++;
            }
        }
        edges.push_back(SA_MAX_READ);
        edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
        if ((int)edges.size() >= 2) out.push_back(edges);
    }
    return out;
}

// Counts the reads whose 16-byte results differ between a and b.
__global__ void count_diff_kernel(const int4 *__restrict__ a, const int4 *__restrict__ b, int64_t n,
                                  unsigned long long *__restrict__ diff) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool d = false;
    if (i < n) {
        const int4 x = a[i], y = b[i];
        d = x.x != y.x || x.y != y.y || x.z != y.z || x.w != y.w;
    }
    const unsigned long long m = __ballot(d);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(diff, (unsigned long long)__popcll(m));
}

// A tuned configuration with the built-in search start, sort and packing.
sa_match_cfg base_cfg(const sa_dindex *d) {
    sa_match_cfg c{};
    c.kernel = SA_KERNEL_TUNED;
    c.tile_levels = std::min(12, d->tile_levels);
    c.block = 256;
    c.blocks_per_cu = 8;
    c.nbuckets = 1;
    c.bucket_edge[0] = SA_MAX_READ;
    c.sort = d->view.ptab_k > 0 ? 0 : 1;
    c.inline_pack = 1;
    c.group = 4;
    c.prefix_table = d->view.ptab_k > 0 ? 1 : 0;
    c.max_words = kWMax;
    c.defer = kDefaultDefer;
    return c;
}

// Stage 1: tile depth x workgroup shape.  With the prefix table the tile
// serves only reads with a non-base among their first k bases, so its depth
// changes little but the LDS it takes (and with it how many workgroups fit
// a compute unit): three depths are tried instead of every one.
std::vector<sa_match_cfg> stage1_candidates(const sa_dindex *d) {
    std::vector<int> levels;
    if (d->view.ptab_k > 0) {
        for (int t : {1, 8, 12})
            if (t <= d->tile_levels) levels.push_back(t);
    } else {
        for (int t = std::min(13, d->tile_levels); t >= std::max(1, std::min(9, d->tile_levels)); t--)
            levels.push_back(t);
    }
    std::vector<sa_match_cfg> out;
    for (int lv : levels)
        for (int block : {256, 512, 1024})
            for (int per_cu : {1, 2, 4, 8}) {
                if (block * per_cu > 4096) continue;
                sa_match_cfg c = base_cfg(d);
                c.tile_levels = lv;
                c.block = block;
                c.blocks_per_cu = per_cu;
                out.push_back(c);
            }
    return out;
}

// Stage 1b, around the best shape: block size of the work split, the search
// start (prefix table or LDS tile only), the sort width, and packing in the
// search kernel or in a pass of its own.
std::vector<sa_match_cfg> stage1b_candidates(const sa_dindex *d, const sa_match_cfg &top) {
    std::vector<sa_match_cfg> out;
    for (int g : {1, 2, 8, 16}) {
        sa_match_cfg c = top;
        c.group = g;
        out.push_back(c);
    }
    if (d->view.ptab_k > 0) {
        sa_match_cfg c = top;
        c.prefix_table = !top.prefix_table;
        out.push_back(c);
    }
    for (int bits : {0, 8, 16, 24}) {
        sa_match_cfg c = top;
        c.sort = bits;
        out.push_back(c);
    }
    if (top.sort == 0) {
        sa_match_cfg c = top;
        c.inline_pack = !top.inline_pack;
        out.push_back(c);
    }
    return out;
}

// Stage 1c, when nearly every read of the batch fits kShortWords words
// (the rest go to the long-read kernel): the register-light search kernel
// in the workgroup shapes that fill its six waves per SIMD, around the best
// so far, with a tile of at most 8 levels when the index has a prefix
// table (so that the workgroups' LDS lets that many waves in).
std::vector<sa_match_cfg> stage1c_candidates(const sa_dindex *d, const sa_match_cfg &top,
                                             const std::vector<int64_t> &hist) {
    std::vector<sa_match_cfg> out;
    int64_t total = 0, fit = 0;
    for (size_t i = 0; i < hist.size(); i++) {
        total += hist[i];
        if ((int)i <= kShortWords) fit += hist[i];
    }
    if (top.sort != 0 || !top.inline_pack || fit * 100 < total * 99) return out;
    for (const auto &shape : std::vector<std::pair<int, int>>{{512, 3}, {256, 6}, {256, 5}, {1024, 1}}) {
        sa_match_cfg c = top;
        c.max_words = kShortWords;
        if (d->view.ptab_k > 0) c.tile_levels = std::min(c.tile_levels, 8);
        c.block = shape.first;
        c.blocks_per_cu = shape.second;
        out.push_back(c);
    }
    return out;
}

// Stage 1d, around the best so far, when the search kernel packs its reads:
// the probe budget after which a read is set aside for a chunk of such
// reads (0 = never).
std::vector<sa_match_cfg> stage1d_candidates(const sa_match_cfg &top) {
    std::vector<sa_match_cfg> out;
    if (top.sort != 0 || !top.inline_pack) return out;
    for (int b : {0, 2, 3, 4, 6, 8}) {
        if (b == top.defer) continue;
        sa_match_cfg c = top;
        c.defer = b;
        out.push_back(c);
    }
    return out;
}

// Stage 2, around the best so far: bucket layouts.  Buckets only order the
// reads through the sort keys, so they are tried only when the reads are
// sorted.
std::vector<sa_match_cfg> stage2_candidates(const sa_match_cfg &top, const std::vector<int64_t> &hist) {
    std::vector<sa_match_cfg> out;
    if (top.sort == 0) return out;
    for (const auto &edges : bucket_layouts(hist)) {
        if (edges.size() == 1) continue;
        sa_match_cfg c = top;
        c.nbuckets = (int)edges.size();
        for (size_t i = 0; i < edges.size(); i++) c.bucket_edge[i] = edges[i];
        out.push_back(c);
    }
    return out;
}

}  // namespace

extern "C" int sa_tune_candidates(const sa_dindex *d, const int64_t *d_offs, int64_t nreads, void *hip_stream,
                                  const sa_match_cfg *around, sa_match_cfg *out, int capacity, int *count) {
    clear_error();
    if (!d || !d_offs || nreads < 1 || !count || capacity < 0 || (capacity > 0 && !out))
        return fail(SA_EINVAL, "bad argument");
    DeviceGuard g(d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    std::vector<int64_t> hist;
    int rc = length_histogram(d_offs, nreads, static_cast<hipStream_t>(hip_stream), hist);
    if (rc) return rc;
    const sa_match_cfg top = resolve_cfg(d, around);
    std::vector<sa_match_cfg> all = stage1_candidates(d);
    for (const auto &c : stage1b_candidates(d, top)) all.push_back(c);
    for (const auto &c : stage1c_candidates(d, top, hist)) all.push_back(c);
    for (const auto &c : stage1d_candidates(top)) all.push_back(c);
    sa_match_cfg sorted = top;
    if (sorted.sort == 0) sorted.sort = 1;
    for (const auto &c : stage2_candidates(sorted, hist)) all.push_back(c);
    std::vector<sa_match_cfg> valid;
    for (const auto &c : all)
        if (check_cfg(d, c) == SA_OK) valid.push_back(c);
    clear_error();
    *count = (int)valid.size();
    for (int i = 0; i < capacity && i < (int)valid.size(); i++) out[i] = valid[(size_t)i];
    return SA_OK;
}

extern "C" int sa_tune(sa_dindex *d, const uint8_t *d_reads, const int64_t *d_offs, int64_t nreads,
                       void *hip_stream, const char *cache_path, sa_match_cfg *best, double *best_ms) {
    clear_error();
    if (!d || !d_reads || !d_offs || nreads < 1) return fail(SA_EINVAL, "bad argument");
    DeviceGuard g(d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::vector<int64_t> hist;
    int rc = length_histogram(d_offs, nreads, s, hist);
    if (rc) return rc;
    const std::string key = cache_key(d, hist, nreads);
    sa_match_cfg found{};
    double found_ms = 0;
    if (cache_path && parse_cached(cache_path, key, found, found_ms) && check_cfg(d, found) == SA_OK) {
        d->defaults = found;
        if (best) *best = found;
        if (best_ms) *best_ms = found_ms;
        return SA_OK;
    }
    // every candidate's results are compared on the device with the first
    // one's: results are unique, so a launch setting that changed them would
    // be a defect, and the tuner fails instead of keeping it
    sa_hit *d_out = nullptr, *d_ref = nullptr;
    unsigned long long *d_diff = nullptr;
    hipError_t e = hipMalloc((void **)&d_out, sizeof(sa_hit) * (size_t)nreads);
    if (e == hipSuccess) e = hipMalloc((void **)&d_ref, sizeof(sa_hit) * (size_t)nreads);
    if (e == hipSuccess) e = hipMalloc((void **)&d_diff, sizeof(unsigned long long));
    if (e != hipSuccess) {
        (void)hipFree(d_out);
        (void)hipFree(d_ref);
        return hip_fail(e, "tuner output");
    }
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    Workspace *ws = workspace_for(d, s);
    sa_match_cfg top = d->defaults;
    double top_ms = 1e30;
    bool have_ref = false;
    auto time_cfg = [&](const sa_match_cfg &c, double &ms) -> int {
        if (check_cfg(d, c) != SA_OK) return SA_EINVAL;
        std::lock_guard<std::mutex> lk(ws->mu);
        int r = enqueue_batch(d, ws, d_reads, d_offs, nullptr, nreads, have_ref ? d_out : d_ref, s, c);  // warm-up
        if (r) return r;
        if (have_ref) {
            unsigned long long diff = 0;
            hipError_t ee = hipMemsetAsync(d_diff, 0, sizeof diff, s);
            if (ee == hipSuccess) {
                hipLaunchKernelGGL(count_diff_kernel, dim3((unsigned)((nreads + 255) / 256)), dim3(256), 0, s,
                                   reinterpret_cast<const int4 *>(d_out), reinterpret_cast<const int4 *>(d_ref),
                                   nreads, d_diff);
                ee = hipGetLastError();
            }
            if (ee == hipSuccess) ee = hipMemcpyAsync(&diff, d_diff, sizeof diff, hipMemcpyDeviceToHost, s);
            if (ee == hipSuccess) ee = hipStreamSynchronize(s);
            if (ee != hipSuccess) return hip_fail(ee, "tuner check");
            if (diff)
                return fail(SA_EDEVICE, "tuner: a candidate configuration gave different results for " +
                                            std::to_string(diff) + " reads");
        }
        have_ref = true;
        float best_rep = 1e30f;
        for (int rep = 0; rep < 3; rep++) {
            (void)hipEventRecord(t0, s);
            r = enqueue_batch(d, ws, d_reads, d_offs, nullptr, nreads, d_out, s, c);
            if (r) return r;
            (void)hipEventRecord(t1, s);
            hipError_t ee = hipEventSynchronize(t1);
            if (ee != hipSuccess) return hip_fail(ee, "tuner timing");
            float t = 0;
            (void)hipEventElapsedTime(&t, t0, t1);
            best_rep = std::min(best_rep, t);
        }
        ms = best_rep;
        if (std::getenv("SAMATCH_TUNE_LOG"))
            std::fprintf(stderr,
                         "tune: levels=%d block=%d per_cu=%d group=%d table=%d sort=%d inline=%d words=%d defer=%d buckets=%d -> "
                         "%.4f ms\n",
                         c.tile_levels, c.block, c.blocks_per_cu, c.group, c.prefix_table, c.sort, c.inline_pack,
                         c.max_words, c.defer, c.nbuckets, ms);
        return SA_OK;
    };
    auto try_all = [&](const std::vector<sa_match_cfg> &cands) -> int {
        for (const auto &c : cands) {
            double ms = 0;
            const int r = time_cfg(c, ms);
            if (r == SA_EINVAL) continue;
            if (r) return r;
            if (ms < top_ms) { top_ms = ms; top = c; }
        }
        return SA_OK;
    };
    rc = try_all(stage1_candidates(d));
    if (rc == SA_OK) rc = try_all(stage1b_candidates(d, top));
    if (rc == SA_OK) rc = try_all(stage1c_candidates(d, top, hist));
    if (rc == SA_OK) rc = try_all(stage1d_candidates(top));
    if (rc == SA_OK) rc = try_all(stage2_candidates(top, hist));
    if (rc == SA_OK && top_ms >= 1e30) rc = fail(SA_EINVAL, "tuner: no valid candidate");
    if (rc == SA_OK) {
        clear_error();
        d->defaults = top;
        if (best) *best = top;
        if (best_ms) *best_ms = top_ms;
        if (cache_path) {
            std::ofstream f(cache_path, std::ios::app);
            if (f) f << "{\"key\":\"" << key << "\"," << cfg_json(top) << ",\"ms\":" << top_ms << "}\n";
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipFree(d_out);
    (void)hipFree(d_ref);
    (void)hipFree(d_diff);
    return rc;
}
