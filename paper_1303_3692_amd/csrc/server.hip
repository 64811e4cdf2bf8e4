// Request loop over resident indexes: continuous batching of reads from
// many requests, admission by free device memory, several streams in
// flight, per-request scatter of results and timestamps.
//
// Life of a request: submit copies its reads and offsets into pinned host
// memory (a pool allocated once and mapped into the device's address space;
// submit waits for room when the pool is full, and only a request larger
// than the whole pool goes to pageable memory) and queues it.  The loop
// admits queued requests in arrival order while the device arena, the
// device memory free when the server started less the reserve and the
// streams' own buffers, has room for the request's image and the in-flight
// read budget allows.  Each round of admissions is copied into the arena by
// one upload kernel on a stream of its own that reads the mapped pool over
// the bus with coalesced 16-byte loads (a request in pageable memory is
// copied by the runtime instead), so that the search kernels read their
// reads from HBM, and a round's upload overlaps the searches of the batches
// admitted before it.  Each free stream slot then takes up to
// max_batch_reads unscheduled reads of one reference, from the admitted
// requests of that reference in admission order (with batch_linger_us, only
// once it holds max_batch_reads reads or its oldest read has waited that
// long), and runs one pipeline over them (a small kernel expands the batch's pieces into each read's start
// and end from the offsets stored with the reads).  A scatter thread copies
// a finished batch's results into the owners' output arrays while the loop
// keeps scheduling; a request whose reads are all done is finished and its
// pool and arena space returned.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <system_error>
#include <thread>
#include <vector>

#include "device_state.h"
#include "kernels.h"

using namespace samatch;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over [0, capacity) with coalescing, 256-byte grain.
class Arena {
  public:
    void init(int64_t cap) {
        cap_ = cap;
        free_.clear();
        if (cap > 0) free_[0] = cap;
    }
    int64_t capacity() const { return cap_; }
    // returns the offset or -1
    int64_t alloc(int64_t bytes) {
        bytes = (std::max<int64_t>(bytes, 1) + 255) & ~int64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, left = it->second - bytes;
            free_.erase(it);
            if (left) free_[off + bytes] = left;
            used_ += bytes;
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = (std::max<int64_t>(bytes, 1) + 255) & ~int64_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t used() const { return used_; }

  private:
    int64_t cap_ = 0, used_ = 0;
    std::map<int64_t, int64_t> free_;
};

// A request's host copy and arena image: its bytes, zero padding to a
// multiple of 8, then its nreads + 1 offsets (rebased to 0).
int64_t offs_at(int64_t nbytes) { return (nbytes + 7) & ~int64_t(7); }
int64_t image_bytes(int64_t nbytes, int64_t nreads) { return offs_at(nbytes) + 8 * (nreads + 1); }

// One piece of a batch as the expansion kernel reads it: rows [pos, pos +
// count) are reads first .. first + count - 1 of a request whose bytes start
// at byte `reads_at` and whose offsets of those reads start at byte
// `offs_at` (8-byte aligned), both relative to the arena base (a request
// read from the mapped host pool lies outside the arena: the difference of
// the two addresses).
struct PieceDev {
    int64_t pos, count, reads_at, offs_at;
};
constexpr int kMaxPieces = 4096;  // pieces per batch

// Row r of the batch: its piece (the last one starting at or before r, by
// binary search over the ascending positions), then its start and end.
__global__ void expand_pieces_kernel(const PieceDev *__restrict__ pieces, int npieces,
                                     const uint8_t *__restrict__ arena, int64_t rows, int64_t *__restrict__ st,
                                     int64_t *__restrict__ en) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    int lo = 0, hi = npieces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pieces[mid].pos <= r) lo = mid;
        else hi = mid - 1;
    }
    const PieceDev p = pieces[lo];
    const int64_t *of = reinterpret_cast<const int64_t *>((uintptr_t)arena + (uintptr_t)p.offs_at);
    const int64_t k = r - p.pos;
    st[r] = p.reads_at + of[k];
    en[r] = p.reads_at + of[k + 1];
}

// One request image to upload: bytes [src, src + bytes) of the mapped pool
// to [dst, dst + bytes) of the arena (offsets 256-byte aligned, bytes a
// multiple of 16), and the first 16-byte unit of it in the round's order.
struct CopyItem {
    int64_t src, dst, bytes, unit0;
};
constexpr int kUploadItems = 96;  // items per upload launch (passed by value)
struct UploadList {
    int count;
    int64_t units;  // 16-byte units over all items
    CopyItem item[kUploadItems];
};

// Copies a round's request images from the mapped host pool to the arena:
// thread t moves 16-byte units t, t + threads, ... (neighbouring threads
// neighbouring units, so loads and stores coalesce), each unit's item found
// by binary search over the items' first units.
__global__ __launch_bounds__(256) void upload_kernel(const UploadList list, const uint8_t *__restrict__ pool,
                                                     uint8_t *__restrict__ arena) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < list.units; u += stride) {
        int lo = 0, hi = list.count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (list.item[mid].unit0 <= u) lo = mid;
            else hi = mid - 1;
        }
        const CopyItem &it = list.item[lo];
        const int64_t b = (u - it.unit0) << 4;
        *reinterpret_cast<uint4 *>(arena + it.dst + b) = *reinterpret_cast<const uint4 *>(pool + it.src + b);
    }
}

struct Request {
    uint64_t ticket = 0;
    int ref = 0;
    int64_t nreads = 0;
    std::vector<char> reads;      // host copy when the pinned pool had no room
    const char *h_reads = nullptr;  // the host copy (pool or reads)
    int64_t pool_off = -1, pool_bytes = 0;
    std::vector<int64_t> offs;    // nreads + 1, rebased to 0
    sa_hit *out = nullptr;        // caller's
    int64_t arena_off = -1, arena_bytes = 0;
    int64_t dev_at = 0;           // where the kernels find the image, relative to the arena base
    int64_t next = 0;             // next unscheduled read
    int64_t done = 0;             // reads with results
    int inflight_batches = 0;
    int status = SA_PENDING;
    int fail_code = SA_OK;
    bool admitted = false, failed = false;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
};

struct Piece {
    Request *req;
    int64_t first, count, pos;  // reads [first, first+count) of req at batch rows [pos, pos+count)
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    bool scattering = false;  // done on the device, results being copied out
    int ref = 0;
    int64_t nreads = 0;
    std::vector<Piece> pieces;
    PieceDev *h_pieces = nullptr;  // pinned, kMaxPieces
    PieceDev *d_pieces = nullptr;
    sa_hit *h_out = nullptr;  // pinned
    int64_t *d_se = nullptr;
    sa_hit *d_out = nullptr;
    int error = SA_OK;
};

}  // namespace

struct sa_server {
    std::vector<sa_dindex *> refs;
    sa_server_opts o{};
    int device = 0;
    Arena arena;
    uint8_t *d_arena = nullptr;
    Arena pool;                // pinned host pool for submitted reads (own lock)
    char *h_pool = nullptr;
    uint8_t *pool_dev = nullptr;  // the pool as the device addresses it (reads are taken from it directly)
    std::mutex pool_mu;
    std::condition_variable pool_cv;  // room was returned to the pool, or the server stops
    bool pool_closed = false;         // under pool_mu
    hipStream_t upload_stream = nullptr;
    hipEvent_t uploaded = nullptr;  // recorded on upload_stream after each round of admissions
    bool any_upload = false;
    std::vector<Request *> to_upload;  // admitted this round, reads not yet copied to the arena
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queued;                  // not admitted yet, arrival order
    std::vector<std::deque<Request *>> active;     // per reference, admitted with reads left to schedule
    std::vector<int64_t> unscheduled;              // per reference, reads of `active` not yet in a batch
    std::map<uint64_t, std::unique_ptr<Request>> all;
    uint64_t next_ticket = 1;
    int64_t inflight_reads = 0;
    int64_t batches_run = 0;
    int next_ref = 0;
    bool stop = false;
    std::thread loop;
    // finished batches whose results the scatter thread copies into the
    // owners' arrays (the loop thread meanwhile keeps scheduling)
    std::deque<Slot *> to_scatter;
    std::condition_variable cv_scatter;
    bool scatter_stop = false;
    std::thread scatter;
    // totals for sa_server_stats (under mu)
    sa_server_stats totals{};

    void run();
    bool admit_locked();
    int upload_locked();
    bool launch(Slot &sl, std::unique_lock<std::mutex> &lk);
    int64_t linger_left_ns(int ref, int64_t now) const;
    bool reap(Slot &sl);
    void measure_batch(Slot &sl);
    void settle_locked(Slot &sl);
    void scatter_run();
    void finish_locked(Request *r, int status);
    void echo_execute(Slot &sl);
};

void sa_server::finish_locked(Request *r, int status) {
    if (r->status != SA_PENDING) return;
    r->status = status;
    r->t_done = now_ns();
    if (r->arena_off >= 0) {
        arena.release(r->arena_off, r->arena_bytes);
        r->arena_off = -1;
    }
    if (r->admitted) inflight_reads -= r->nreads;
    if (r->pool_off >= 0) {
        std::lock_guard<std::mutex> pl(pool_mu);
        pool.release(r->pool_off, r->pool_bytes);
        pool_cv.notify_all();
        r->pool_off = -1;
    }
    r->h_reads = nullptr;
    std::vector<char>().swap(r->reads);
    std::vector<int64_t>().swap(r->offs);
    cv_done.notify_all();
}

// Admit queued requests in arrival order while the device arena has room
// for their images and the in-flight read budget allows.  A request that
// could never fit (larger than the arena, or than the budget) is refused
// with SA_ENOSPC.
bool sa_server::admit_locked() {
    bool any = false;
    while (!queued.empty()) {
        Request *r = queued.front();
        const int64_t bytes = image_bytes(r->offs[(size_t)r->nreads], r->nreads);
        if (bytes > arena.capacity() || r->nreads > o.max_inflight_reads) {
            queued.pop_front();
            finish_locked(r, SA_ENOSPC);
            any = true;
            continue;
        }
        if (inflight_reads > 0 && inflight_reads + r->nreads > o.max_inflight_reads) break;
        const int64_t off = arena.alloc(bytes);
        if (off < 0) break;
        r->arena_off = off;
        r->arena_bytes = bytes;
        r->dev_at = off;
        queued.pop_front();
        r->admitted = true;
        r->t_admit = now_ns();
        inflight_reads += r->nreads;
        if (r->nreads == 0) {
            finish_locked(r, SA_OK);
        } else {
            if (!o.test_echo) to_upload.push_back(r);
            active[(size_t)r->ref].push_back(r);
            unscheduled[(size_t)r->ref] += r->nreads;
        }
        any = true;
    }
    return any;
}

// Copy this round's admitted requests to the arena on the upload stream:
// those in the mapped pool with upload kernels (up to kUploadItems requests
// per launch), any other one with a runtime copy; then mark the upload
// stream, and every batch launched afterwards waits for that mark (one
// event for the round instead of one per request).
int sa_server::upload_locked() {
    if (to_upload.empty()) return SA_OK;
    std::vector<Request *> rs;
    rs.swap(to_upload);
    hipError_t e = hipSuccess;
    UploadList list;
    list.count = 0;
    list.units = 0;
    auto flush = [&]() {
        if (list.count == 0 || e != hipSuccess) return;
        const int64_t blocks = std::min<int64_t>((list.units + 255) / 256, 1024);
        hipLaunchKernelGGL(upload_kernel, dim3((unsigned)blocks), dim3(256), 0, upload_stream, list, pool_dev, d_arena);
        e = hipGetLastError();
        list.count = 0;
        list.units = 0;
    };
    for (Request *r : rs) {
        if (e != hipSuccess) break;
        const int64_t bytes = image_bytes(r->offs[(size_t)r->nreads], r->nreads);
        if (pool_dev != nullptr && r->pool_off >= 0) {
            // whole 16-byte units: both allocations are 256-byte aligned and rounded up to 256 bytes
            const int64_t units = (bytes + 15) >> 4;
            list.item[list.count++] = CopyItem{r->pool_off, r->arena_off, units << 4, list.units};
            list.units += units;
            if (list.count == kUploadItems) flush();
        } else {
            e = hipMemcpyAsync(d_arena + r->arena_off, r->h_reads, (size_t)bytes, hipMemcpyHostToDevice,
                               upload_stream);
        }
    }
    flush();
    if (e == hipSuccess)
        for (Request *r : rs) totals.upload_bytes += image_bytes(r->offs[(size_t)r->nreads], r->nreads);
    if (e == hipSuccess) e = hipEventRecord(uploaded, upload_stream);
    if (e == hipSuccess) {
        any_upload = true;
        return SA_OK;
    }
    const int rc = hip_fail(e, "request upload");
    // none of them is in a batch yet: drop them from scheduling
    for (Request *r : rs) {
        auto &q = active[(size_t)r->ref];
        if (std::find(q.begin(), q.end(), r) != q.end()) unscheduled[(size_t)r->ref] -= r->nreads - r->next;
        q.erase(std::remove(q.begin(), q.end(), r), q.end());
        finish_locked(r, SA_EDEVICE);
    }
    return rc;
}

// With batch_linger_us set: how much longer a batch of reference ref waits
// for more reads (0 when it may start: its oldest unscheduled read has
// waited long enough, or it holds max_batch_reads reads).
int64_t sa_server::linger_left_ns(int ref, int64_t now) const {
    const auto &q = active[(size_t)ref];
    if (o.batch_linger_us <= 0 || q.empty() || unscheduled[(size_t)ref] >= o.max_batch_reads) return 0;
    const int64_t left = q.front()->t_admit + o.batch_linger_us * 1000 - now;
    return left > 0 ? left : 0;
}

// Form a batch for a free slot from one reference's admitted requests.
// The pieces are taken with the lock held; the per-read work (start and end
// arrays) and the launches run with it released, so that submitters and
// pollers are not held up (only this thread touches the slots, and a
// request with batches in flight keeps its buffers).
bool sa_server::launch(Slot &sl, std::unique_lock<std::mutex> &lk) {
    const int nref = (int)refs.size();
    const int64_t now = o.batch_linger_us > 0 ? now_ns() : 0;
    int ref = -1;
    for (int k = 0; k < nref; k++) {
        const int cand = (next_ref + k) % nref;
        if (!active[(size_t)cand].empty() && linger_left_ns(cand, now) == 0) { ref = cand; break; }
    }
    if (ref < 0) return false;
    next_ref = (ref + 1) % nref;
    auto &q = active[(size_t)ref];
    sl.pieces.clear();
    sl.ref = ref;
    sl.error = SA_OK;
    int64_t rows = 0;
    while (!q.empty() && rows < o.max_batch_reads && (int)sl.pieces.size() < kMaxPieces) {
        Request *r = q.front();
        const int64_t take = std::min(r->nreads - r->next, o.max_batch_reads - rows);
        sl.pieces.push_back(Piece{r, r->next, take, rows});
        r->next += take;
        unscheduled[(size_t)ref] -= take;
        r->inflight_batches++;
        rows += take;
        if (r->next == r->nreads) q.pop_front();
    }
    sl.nreads = rows;
    sl.busy = true;
    batches_run++;
    const bool inject = o.test_fail_batch > 0 && batches_run == o.test_fail_batch;
    if (o.test_echo) {
        sl.error = inject ? SA_EDEVICE : SA_OK;
        return true;
    }
    if (inject) {
        sl.error = SA_EDEVICE;
        return true;
    }
    lk.unlock();
    struct Relock {
        std::unique_lock<std::mutex> &l;
        ~Relock() { l.lock(); }
    } relock{lk};
    // the pieces, expanded on the device into each read's start and end
    // (relative to the arena base), after any arena uploads of this round
    const int npieces = (int)sl.pieces.size();
    for (int i = 0; i < npieces; i++) {
        const Piece &p = sl.pieces[(size_t)i];
        const int64_t nbytes = p.req->offs[(size_t)p.req->nreads];
        sl.h_pieces[i] = PieceDev{p.pos, p.count, p.req->dev_at, p.req->dev_at + offs_at(nbytes) + 8 * p.first};
    }
    int64_t *d_st = sl.d_se, *d_en = sl.d_se + o.max_batch_reads;
    hipError_t e = hipSuccess;
    if (any_upload) e = hipStreamWaitEvent(sl.stream, uploaded, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.d_pieces, sl.h_pieces, sizeof(PieceDev) * (size_t)npieces, hipMemcpyHostToDevice,
                           sl.stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(expand_pieces_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, sl.stream,
                           sl.d_pieces, npieces, d_arena, rows, d_st, d_en);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        sl.error = hip_fail(e, "batch upload");
        (void)hipStreamSynchronize(sl.stream);  // the staging buffers are reused by the next batch
        return true;
    }
    sa_dindex *d = refs[(size_t)ref];
    Workspace *ws = workspace_for(d, sl.stream);
    int rc;
    // the reads are in the arena, each request's back to back: the search
    // kernel packs them itself (coalesced, with the next chunk's loads in
    // flight), under the deepest LDS tile that leaves room for its packing
    // areas
    sa_match_cfg c = resolve_cfg(d, nullptr);
    if (c.kernel == SA_KERNEL_TUNED) {
        c.sort = 0;
        c.inline_pack = 1;
        while (c.tile_levels > 1 && tuned_lds_bytes(c.tile_levels, c.block, true, c.max_words) > inline_lds_limit())
            c.tile_levels--;
    }
    c.use_graph = 0;
    c.profile = o.measure >= 1 ? 1 : 0;  // stage events, read when the batch is reaped
    c.count = o.measure == 2 ? 1 : 0;
    {
        std::lock_guard<std::mutex> wl(ws->mu);
        rc = enqueue_batch(d, ws, d_arena, sl.d_se, sl.d_se + o.max_batch_reads, rows, sl.d_out, sl.stream, c);
    }
    if (rc) {
        sl.error = rc;
        (void)hipStreamSynchronize(sl.stream);
        return true;
    }
    e = hipMemcpyAsync(sl.h_out, sl.d_out, sizeof(sa_hit) * (size_t)rows, hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) {
        sl.error = hip_fail(e, "batch download");
        (void)hipStreamSynchronize(sl.stream);
    }
    return true;
}

// Deterministic stand-in results for host-only tests: lo = request-local
// read index, hi = lo + ticket, len = read length, flags = reference plus
// 256 times the byte sum of the read's host copy (mod 2^16).
void sa_server::echo_execute(Slot &sl) {
    for (const Piece &p : sl.pieces)
        for (int64_t k = 0; k < p.count; k++) {
            const int64_t i = p.first + k;
            const int64_t b0 = p.req->offs[(size_t)i], b1 = p.req->offs[(size_t)i + 1];
            uint32_t sum = 0;
            for (int64_t b = b0; b < b1; b++) sum += (uint8_t)p.req->h_reads[b];
            sa_hit h;
            h.lo = (int32_t)i;
            h.hi = (int32_t)(i + (int64_t)p.req->ticket);
            h.len = (int32_t)(b1 - b0);
            h.flags = (uint32_t)sl.ref | ((sum & 0xffffu) << 8);
            sl.h_out[p.pos + k] = h;
        }
}

// Collect a finished batch: hand it to the scatter thread (or, for a
// failed batch, settle it here at once).
bool sa_server::reap(Slot &sl) {
    if (!sl.busy || sl.scattering) return false;
    if (!o.test_echo && sl.error == SA_OK) {
        hipError_t e = hipEventQuery(sl.done);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess) sl.error = hip_fail(e, "batch execution");
        if (e == hipSuccess && o.measure >= 1) measure_batch(sl);
    } else if (o.test_echo && sl.error == SA_OK) {
        echo_execute(sl);
    }
    if (sl.error == SA_OK) {
        totals.batches++;
        totals.reads += sl.nreads;
    }
    if (sl.error == SA_OK) {  // the scatter thread copies the results out, then settles the slot
        sl.scattering = true;
        to_scatter.push_back(&sl);
        cv_scatter.notify_one();
        return true;
    }
    settle_locked(sl);
    return true;
}

// Measurement mode: the finished batch's search-stage time from the stage
// events of its (index, stream) workspace, and with counting on, the bytes
// its search kernels touched.
void sa_server::measure_batch(Slot &sl) {
    Workspace *ws = workspace_for(refs[(size_t)sl.ref], sl.stream);
    std::lock_guard<std::mutex> wl(ws->mu);
    float ms = 0;
    if (ws->profiled && hipEventElapsedTime(&ms, ws->ev[2], ws->ev[3]) == hipSuccess) totals.search_ms += ms;
    if (ws->counted) {
        unsigned long long touched = 0;
        if (hipMemcpy(&touched, ws->b.stats + 7, sizeof touched, hipMemcpyDeviceToHost) == hipSuccess)
            totals.touched_bytes += (int64_t)touched;
    }
    (void)hipGetLastError();
}

// Account a finished batch whose results (if any) are in the owners'
// arrays: finish complete requests, free the slot.
void sa_server::settle_locked(Slot &sl) {
    for (const Piece &p : sl.pieces) {
        Request *r = p.req;
        r->inflight_batches--;
        if (sl.error != SA_OK) {
            if (!r->failed) { r->failed = true; r->fail_code = sl.error; }
        } else if (!r->failed) {
            r->done += p.count;
        }
        if (r->inflight_batches == 0) {
            if (r->failed) {
                // drop the rest of a failed request from scheduling
                auto &q = active[(size_t)r->ref];
                if (std::find(q.begin(), q.end(), r) != q.end()) unscheduled[(size_t)r->ref] -= r->nreads - r->next;
                q.erase(std::remove(q.begin(), q.end(), r), q.end());
                finish_locked(r, r->fail_code);
            } else if (r->done == r->nreads) {
                finish_locked(r, SA_OK);
            }
        }
    }
    sl.busy = false;
    sl.scattering = false;
    sl.pieces.clear();
}

// Copy finished batches' results into the owners' output arrays with the
// lock released (a request with a batch in flight is pending, so its array
// stays valid), then settle them.
void sa_server::scatter_run() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        cv_scatter.wait(lk, [&] { return scatter_stop || !to_scatter.empty(); });
        if (to_scatter.empty()) break;  // stopping, nothing left
        Slot *sl = to_scatter.front();
        to_scatter.pop_front();
        lk.unlock();
        for (const Piece &p : sl->pieces)
            std::memcpy(p.req->out + p.first, sl->h_out + p.pos, sizeof(sa_hit) * (size_t)p.count);
        lk.lock();
        settle_locked(*sl);
        cv_work.notify_one();
    }
}

void sa_server::run() {
    if (!o.test_echo) (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progress = false;
        for (Slot &sl : slots) progress |= reap(sl);
        if (!stop) {
            progress |= admit_locked();
            (void)upload_locked();
            for (Slot &sl : slots)
                if (!sl.busy && !stop) progress |= launch(sl, lk);
        }
        bool busy = false;
        for (Slot &sl : slots) busy |= sl.busy;
        if (stop && !busy) break;
        if (progress) continue;
        if (busy) {
            // batches in flight: poll their events without holding the lock long
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            // idle: wake for new work, or when a lingering batch may start
            int64_t wait_ns = 5000000;
            if (o.batch_linger_us > 0) {
                const int64_t now = now_ns();
                for (int ref = 0; ref < (int)refs.size(); ref++) {
                    const int64_t left = linger_left_ns(ref, now);
                    if (left > 0) wait_ns = std::min(wait_ns, left);
                }
            }
            cv_work.wait_for(lk, std::chrono::nanoseconds(wait_ns));
        }
    }
}

// Release what sa_server_create allocated; safe on a partly built server.
static void free_resources(sa_server *s) {
    if (s->o.test_echo) {
        for (Slot &sl : s->slots) delete[] sl.h_out;
        delete[] s->h_pool;
        s->h_pool = nullptr;
        return;
    }
    DeviceGuard g(s->device);
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.h_pieces) (void)hipHostFree(sl.h_pieces);
        if (sl.d_pieces) (void)hipFree(sl.d_pieces);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        if (sl.d_se) (void)hipFree(sl.d_se);
        if (sl.d_out) (void)hipFree(sl.d_out);
        // the indexes keep a workspace per stream; drop this stream's
        if (sl.stream)
            for (sa_dindex *d : s->refs) {
                std::lock_guard<std::mutex> g2(d->mu);
                d->ws.erase((void *)sl.stream);
            }
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        sl = Slot{};
    }
    if (s->upload_stream) {
        (void)hipStreamSynchronize(s->upload_stream);
        (void)hipStreamDestroy(s->upload_stream);
        s->upload_stream = nullptr;
    }
    if (s->uploaded) (void)hipEventDestroy(s->uploaded);
    s->uploaded = nullptr;
    if (s->d_arena) (void)hipFree(s->d_arena);
    s->d_arena = nullptr;
    if (s->h_pool) (void)hipHostFree(s->h_pool);
    s->h_pool = nullptr;
}

extern "C" int sa_server_create(const sa_dindex *const *refs, int nrefs, const sa_server_opts *opts,
                                sa_server **out) {
    clear_error();
    if (!refs || nrefs < 1 || !out) return fail(SA_EINVAL, "bad argument");
    *out = nullptr;
    std::unique_ptr<sa_server> s(new sa_server);
    sa_server_opts o{};
    o.hbm_reserve_bytes = (int64_t)1 << 30;
    o.max_batch_reads = 1 << 20;
    o.max_inflight_reads = (int64_t)8 << 20;
    o.nstreams = 2;
    o.test_fake_free_hbm = -1;
    o.host_pool_bytes = (int64_t)1 << 30;
    if (opts) {
        if (opts->host_pool_bytes != 0) o.host_pool_bytes = std::max<int64_t>(0, opts->host_pool_bytes);
        if (opts->hbm_reserve_bytes > 0) o.hbm_reserve_bytes = opts->hbm_reserve_bytes;
        if (opts->max_batch_reads > 0) o.max_batch_reads = opts->max_batch_reads;
        if (opts->max_inflight_reads > 0) o.max_inflight_reads = opts->max_inflight_reads;
        if (opts->nstreams > 0) o.nstreams = opts->nstreams;
        o.test_fake_free_hbm = opts->test_fake_free_hbm;
        o.test_echo = opts->test_echo;
        o.test_fail_batch = opts->test_fail_batch;
        o.measure = opts->measure;
        o.batch_linger_us = opts->batch_linger_us;
    }
    if (o.measure < 0 || o.measure > 2) return fail(SA_EINVAL, "measure must be 0, 1 or 2");
    if (o.batch_linger_us < 0 || o.batch_linger_us > 1000000)
        return fail(SA_EINVAL, "batch_linger_us must be in 0..1000000");
    if (o.nstreams > 8) return fail(SA_EINVAL, "nstreams must be at most 8");
    if (o.max_batch_reads > INT32_MAX) return fail(SA_EINVAL, "max_batch_reads too large");
    for (int i = 0; i < nrefs; i++) {
        if (!o.test_echo && !refs[i]) return fail(SA_EINVAL, "NULL index");
        s->refs.push_back(const_cast<sa_dindex *>(refs[i]));
    }
    s->o = o;
    s->active.resize((size_t)nrefs);
    s->unscheduled.assign((size_t)nrefs, 0);
    s->slots.resize((size_t)o.nstreams);
    auto setup = [&]() -> int {
        if (o.test_echo) {
            s->arena.init(o.test_fake_free_hbm >= 0 ? std::max<int64_t>(0, o.test_fake_free_hbm - o.hbm_reserve_bytes)
                                                    : ((int64_t)1 << 30));
            for (Slot &sl : s->slots) sl.h_out = new sa_hit[(size_t)o.max_batch_reads];
            if (o.host_pool_bytes > 0) {
                s->h_pool = new (std::nothrow) char[(size_t)o.host_pool_bytes];
                if (!s->h_pool) return fail(SA_ENOMEM, "host pool");
                s->pool.init(o.host_pool_bytes);
            }
        } else {
            s->device = s->refs[0]->device;
            for (sa_dindex *d : s->refs)
                if (d->device != s->device) return fail(SA_EINVAL, "all indexes must be on one device");
            DeviceGuard g(s->device);
            if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
            size_t free_b = 0, total_b = 0;
            hipError_t e = hipMemGetInfo(&free_b, &total_b);
            if (e != hipSuccess) return hip_fail(e, "hipMemGetInfo");
            const int64_t free_hbm = o.test_fake_free_hbm >= 0 ? o.test_fake_free_hbm : (int64_t)free_b;
            // per slot: starts/ends, results, and the pipeline scratch (~120 B per read)
            const int64_t per_slot = o.max_batch_reads * (16 + 16 + 130);
            const int64_t budget = free_hbm - o.hbm_reserve_bytes - per_slot * o.nstreams;
            if (budget < (1 << 20)) return fail(SA_ENOSPC, "not enough free device memory for the server");
            const int64_t arena_bytes = std::min<int64_t>(budget, (int64_t)16 << 30);
            if ((e = hipMalloc((void **)&s->d_arena, (size_t)arena_bytes)) != hipSuccess)
                return hip_fail(e, "arena allocation");
            s->arena.init(arena_bytes);
            if (o.host_pool_bytes > 0) {
                // coherent and mapped: the kernels read requests from it directly
                if ((e = hipHostMalloc((void **)&s->h_pool, (size_t)o.host_pool_bytes,
                                       hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
                    return hip_fail(e, "pinned host pool");
                s->pool.init(o.host_pool_bytes);
                void *dp = nullptr;
                if (hipHostGetDevicePointer(&dp, s->h_pool, 0) == hipSuccess && dp) s->pool_dev = (uint8_t *)dp;
                (void)hipGetLastError();  // without a mapping, requests go through the arena
            }
            if ((e = hipStreamCreateWithFlags(&s->upload_stream, hipStreamNonBlocking)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&s->uploaded, hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e, "stream creation");
            for (Slot &sl : s->slots) {
                if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
                    (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess ||
                    (e = hipHostMalloc((void **)&sl.h_pieces, sizeof(PieceDev) * kMaxPieces, hipHostMallocDefault)) !=
                        hipSuccess ||
                    (e = hipMalloc((void **)&sl.d_pieces, sizeof(PieceDev) * kMaxPieces)) != hipSuccess ||
                    (e = hipHostMalloc((void **)&sl.h_out, sizeof(sa_hit) * (size_t)o.max_batch_reads,
                                       hipHostMallocDefault)) != hipSuccess ||
                    (e = hipMalloc((void **)&sl.d_se, sizeof(int64_t) * 2 * (size_t)o.max_batch_reads)) != hipSuccess ||
                    (e = hipMalloc((void **)&sl.d_out, sizeof(sa_hit) * (size_t)o.max_batch_reads)) != hipSuccess)
                    return hip_fail(e, "slot allocation");
                // size every index's scratch for this stream now, not on the first batch
                for (sa_dindex *d : s->refs) {
                    int rc = workspace_for(d, sl.stream)->reserve(o.max_batch_reads);
                    if (rc) return rc;
                }
            }
        }
        return SA_OK;
    };
    if (int rc = setup()) {
        free_resources(s.get());
        return rc;
    }
    sa_server *raw = s.get();
    try {
        s->scatter = std::thread([raw] { raw->scatter_run(); });
        s->loop = std::thread([raw] { raw->run(); });
    } catch (const std::system_error &) {
        if (s->scatter.joinable()) {
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->scatter_stop = true;
                s->cv_scatter.notify_all();
            }
            s->scatter.join();
        }
        free_resources(s.get());
        return fail(SA_ENOMEM, "server threads");
    }
    *out = s.release();
    return SA_OK;
}

static void release_pool(sa_server *s, Request *r) {
    if (r->pool_off < 0) return;
    std::lock_guard<std::mutex> pl(s->pool_mu);
    s->pool.release(r->pool_off, r->pool_bytes);
    s->pool_cv.notify_all();
    r->pool_off = -1;
}

extern "C" int match_submit(sa_server *s, int ref, const char *reads, const int64_t *offs, int64_t nreads,
                            sa_hit *out, uint64_t *ticket) {
    clear_error();
    if (!s || !offs || !ticket || nreads < 0 || (nreads > 0 && (!reads || !out)))
        return fail(SA_EINVAL, "bad argument");
    if (ref < 0 || ref >= (int)s->refs.size()) return fail(SA_EINVAL, "no such reference");
    if (offs[0] < 0) return fail(SA_EINVAL, "negative offset");
    for (int64_t i = 0; i < nreads; i++) {
        const int64_t m = offs[i + 1] - offs[i];
        if (m < 0) return fail(SA_EINVAL, "offsets decrease");
        if (m > SA_MAX_READ) return fail(SA_ETOOBIG, "read longer than SA_MAX_READ");
    }
    std::unique_ptr<Request> r(new Request);
    r->ref = ref;
    r->nreads = nreads;
    r->out = out;
    r->t_submit = now_ns();
    try {
        const int64_t base = offs[0], nbytes = offs[nreads] - offs[0];
        const int64_t image = image_bytes(nbytes, nreads);
        if (s->h_pool && nreads > 0 && image <= s->pool.capacity()) {
            // wait for room rather than take the pageable path: a pageable
            // request's upload is a synchronous copy on the request loop
            std::unique_lock<std::mutex> pl(s->pool_mu);
            for (;;) {
                r->pool_off = s->pool.alloc(image);
                if (r->pool_off >= 0 || s->pool_closed) break;
                s->pool_cv.wait(pl);
            }
            if (r->pool_off >= 0) r->pool_bytes = image;
        }
        char *img;
        if (r->pool_off >= 0) {
            img = s->h_pool + r->pool_off;
        } else {
            r->reads.resize((size_t)image);
            img = r->reads.data();
        }
        if (nbytes > 0) std::memcpy(img, reads + base, (size_t)nbytes);
        std::memset(img + nbytes, 0, (size_t)(offs_at(nbytes) - nbytes));
        int64_t *io = reinterpret_cast<int64_t *>(img + offs_at(nbytes));
        r->offs.resize((size_t)nreads + 1);
        for (int64_t i = 0; i <= nreads; i++) io[i] = r->offs[(size_t)i] = offs[i] - base;
        r->h_reads = img;
    } catch (const std::bad_alloc &) {
        release_pool(s, r.get());
        return fail(SA_ENOMEM, "request copy");
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        release_pool(s, r.get());
        return fail(SA_ECANCELED, "server is shutting down");
    }
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->queued.push_back(r.get());
    s->all[r->ticket] = std::move(r);
    s->cv_work.notify_one();
    return SA_OK;
}

extern "C" int match_poll(sa_server *s, uint64_t ticket, int64_t timeout_us, sa_req_stats *st) {
    clear_error();
    if (!s) return fail(SA_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(SA_ENOTFOUND, "unknown ticket");
    Request *r = it->second.get();
    if (r->status == SA_PENDING && timeout_us != 0) {
        auto pred = [r] { return r->status != SA_PENDING; };
        if (timeout_us < 0) s->cv_done.wait(lk, pred);
        else s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred);
    }
    if (st) {
        st->t_submit_ns = r->t_submit;
        st->t_admit_ns = r->t_admit;
        st->t_done_ns = r->t_done;
        st->status = r->status;
        st->nreads = r->nreads;
    }
    return r->status;
}

extern "C" int sa_server_get_stats(sa_server *s, sa_server_stats *out) {
    clear_error();
    if (!s || !out) return fail(SA_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->totals;
    return SA_OK;
}

extern "C" int sa_server_destroy(sa_server *s) {
    clear_error();
    if (!s) return SA_OK;
    {
        std::lock_guard<std::mutex> pl(s->pool_mu);
        s->pool_closed = true;  // submitters waiting for room give up
        s->pool_cv.notify_all();
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // queued and admitted-but-unscheduled work is cancelled now; batches
        // already on the device finish first
        while (!s->queued.empty()) {
            s->finish_locked(s->queued.front(), SA_ECANCELED);
            s->queued.pop_front();
        }
        for (auto &q : s->active) {
            for (Request *r : q) {
                if (r->inflight_batches == 0) {
                    s->finish_locked(r, SA_ECANCELED);
                } else if (!r->failed) {
                    r->failed = true;
                    r->fail_code = SA_ECANCELED;
                }
            }
            q.clear();
        }
        std::fill(s->unscheduled.begin(), s->unscheduled.end(), 0);
        s->cv_work.notify_all();
    }
    if (s->loop.joinable()) s->loop.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->scatter_stop = true;
        s->cv_scatter.notify_all();
    }
    if (s->scatter.joinable()) s->scatter.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &kv : s->all)
            if (kv.second->status == SA_PENDING) s->finish_locked(kv.second.get(), SA_ECANCELED);
    }
    free_resources(s);
    delete s;
    return SA_OK;
}

extern "C" int sa_server_replay(sa_server *s, int64_t nreq, const int32_t *ref, const char *const *reads,
                                const int64_t *const *offs, const int64_t *nreads, const int64_t *arrival_ns,
                                sa_hit *const *out, int nthreads, int64_t *sched_ns, sa_req_stats *stats) {
    clear_error();
    if (!s || nreq < 0 || (nreq > 0 && (!ref || !reads || !offs || !nreads || !arrival_ns || !out || !sched_ns ||
                                        !stats)))
        return fail(SA_EINVAL, "bad argument");
    if (nthreads < 1 || nthreads > 64) return fail(SA_EINVAL, "nthreads must be in 1..64");
    std::vector<uint64_t> tickets((size_t)nreq, 0);
    std::vector<int> submit_rc((size_t)nreq, SA_OK);
    const int64_t t0 = now_ns() + 20000000;
    auto client = [&](int t) {
        for (int64_t i = t; i < nreq; i += nthreads) {
            const int64_t due = t0 + arrival_ns[i];
            for (;;) {  // sleep to about 100 us before the due time, then spin
                const int64_t left = due - now_ns();
                if (left <= 0) break;
                if (left > 150000) std::this_thread::sleep_for(std::chrono::nanoseconds(left - 100000));
            }
            sched_ns[i] = due;
            submit_rc[(size_t)i] = match_submit(s, ref[i], reads[i], offs[i], nreads[i], out[i], &tickets[(size_t)i]);
        }
    };
    std::vector<std::thread> th;
    try {
        for (int t = 0; t < nthreads; t++) th.emplace_back(client, t);
    } catch (const std::system_error &) {
        for (std::thread &x : th) x.join();
        return fail(SA_ENOMEM, "client threads");
    }
    for (std::thread &x : th) x.join();
    int first = SA_OK;
    for (int64_t i = 0; i < nreq; i++) {
        std::memset(&stats[i], 0, sizeof(sa_req_stats));
        if (submit_rc[(size_t)i] != SA_OK) {
            stats[i].status = submit_rc[(size_t)i];
            if (first == SA_OK) first = submit_rc[(size_t)i];
            continue;
        }
        (void)match_poll(s, tickets[(size_t)i], -1, &stats[i]);
    }
    if (first != SA_OK) return fail(first, "a replayed request could not be submitted");
    return SA_OK;
}
