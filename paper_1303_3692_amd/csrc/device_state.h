// Device-side state shared by device.hip, tune.hip and server.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <vector>
#include <memory>
#include <mutex>

#include "internal.h"
#include "kernels.h"

namespace samatch {

int hip_fail(hipError_t e, const char *what);

// Makes `dev` current for the scope and restores the caller's device.
struct DeviceGuard {
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
    int prev = -1;
    bool ok = true;
};

// A captured launch sequence and what it was captured for.
struct GraphEntry {
    const void *reads, *offs, *ends, *out;
    int64_t nreads;
    sa_match_cfg cfg;
    hipGraphExec_t exec;
    uint64_t last_use;
};

// Scratch of one (index, stream): device buffers of the pipeline plus pinned
// and device staging for host batches.  Grows on demand, never shrinks.
// One of the two pinned-host / device buffer sets through which match_batch
// streams a batch from host memory, chunk by chunk.
struct HostSlot {
    ~HostSlot();
    int reserve(int64_t nreads, int64_t nbytes);
    int64_t reads_cap = 0, bytes_cap = 0;
    char *h_reads = nullptr;
    int64_t *h_offs = nullptr;
    sa_hit *h_out = nullptr;
    uint8_t *d_reads = nullptr;
    int64_t *d_offs = nullptr;
    sa_hit *d_out = nullptr;
    hipEvent_t done = nullptr;  // recorded after the slot's last chunk came back to h_out
};

struct Workspace {
    ~Workspace();
    int reserve(int64_t nreads);
    void drop_graphs();

    // replayable launch sequences (at most kMaxGraphs, least recently used dropped)
    static constexpr size_t kMaxGraphs = 8;
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0;

    std::mutex mu;
    int64_t cap = 0;
    BatchBuffers b{};
    // stage events of the last profiled batch, and whether counts are held
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool profiled = false, counted = false;
    // host batches: chunks alternate between the two slots
    HostSlot host[2];
};

Workspace *workspace_for(sa_dindex *d, hipStream_t s);
BucketTable bucket_table(const sa_match_cfg &c);
int check_cfg(const sa_dindex *d, const sa_match_cfg &c);
sa_match_cfg resolve_cfg(const sa_dindex *d, const sa_match_cfg *cfg);
int enqueue_batch(sa_dindex *d, Workspace *ws, const uint8_t *d_reads, const int64_t *d_offs, const int64_t *d_ends,
                  int64_t nreads, sa_hit *d_out, hipStream_t s, const sa_match_cfg &c);
// The same pipeline on buffers the caller provides (sized for nreads on the
// path c takes, see packs_inline); ev: four events for the stage times, or
// NULL.
int enqueue_pipeline(sa_dindex *d, const BatchBuffers &b, const hipEvent_t *ev, const uint8_t *d_reads,
                     const int64_t *d_offs, const int64_t *d_ends, int64_t nreads, sa_hit *d_out, hipStream_t s,
                     const sa_match_cfg &c);
// Whether c's tuned search packs reads in input order itself (no pack pass,
// no sort): then the pipeline's only scratch is b.stats.
bool packs_inline(const sa_match_cfg &c);
// enqueue_batch through a captured graph when c.use_graph asks for it (and
// the stream can be captured), else directly.
int run_batch(sa_dindex *d, Workspace *ws, const uint8_t *d_reads, const int64_t *d_offs, const int64_t *d_ends,
              int64_t nreads, sa_hit *d_out, hipStream_t s, const sa_match_cfg &c);

// Suffix array construction on the device (sa_construct.hip).
struct SaBuildInfo {
    int steps = 0;             // sorting rounds: the 21-base keys, then each doubling
    int64_t sorted_elems = 0;  // (key, value) pairs sorted over all rounds
};
int build_sa_device(const uint64_t *d_text, int64_t n, int32_t *d_sa, uint32_t *rank_out, hipStream_t s,
                    SaBuildInfo *info);

}  // namespace samatch

struct sa_dindex {
    ~sa_dindex();
    int device = 0;
    int64_t n = 0;
    int cu_count = 0;
    char arch[64] = {0};
    uint64_t *d_text = nullptr;
    int32_t *d_sa = nullptr;
    uint64_t *d_tile_key = nullptr;
    int32_t *d_tile_sa = nullptr;
    samatch::RowRec *d_rows = nullptr;
    samatch::PrefixEntry *d_ptab = nullptr;
    int64_t ptab_bytes = 0;
    int tile_levels = 0;  // levels stored (the kernel may use fewer)
    samatch::SaBuildInfo built{};  // when the suffix array was built on the device
    samatch::DevIndex view{};
    sa_match_cfg defaults{};
    std::mutex mu;
    std::map<void *, std::unique_ptr<samatch::Workspace>> ws;
};
