// match_batch_dev_noalloc: the batch pipeline of match_batch_dev on a fixed
// device array instead of per-stream scratch that grows on demand, for
// callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"
#include "kernels.h"
#include "device_state.h"

using namespace samatch;

namespace {

constexpr size_t kScratchBytes = (size_t)SA_NOALLOC_SCRATCH_BYTES;
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

// The pipeline's scratch on every device the library runs on.  In host code
// this name is only a handle for hipGetSymbolAddress: kernels get the
// device address that call returns.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Byte layout of the scratch for a batch of nreads: the counters first, then
// (pack pass only) the packed words, lengths, the two key and value arrays
// and the sort histograms.  Returns the bytes used; with base non-NULL also
// fills b.
size_t layout(int64_t nreads, bool pack_pass, unsigned char *base, BatchBuffers *b) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = up(off + bytes);
        return base ? base + at : nullptr;
    };
    BatchBuffers x{};
    x.stats = reinterpret_cast<unsigned long long *>(take(sizeof(unsigned long long) * kStatWords));
    if (pack_pass) {
        const size_t n = (size_t)nreads;
        const size_t nblocks = (n + kSortTile - 1) / kSortTile;
        x.digit_total = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * 256));
        x.qw = reinterpret_cast<uint64_t *>(take(sizeof(uint64_t) * kWMax * n));
        x.qlm = reinterpret_cast<int2 *>(take(sizeof(int2) * n));
        for (int i = 0; i < 2; i++) {
            x.key[i] = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * n));
            x.val[i] = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * n));
        }
        x.hist = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * 256 * nblocks));
    }
    if (b) *b = x;
    return off;
}

// Device address of this device's scratch, looked up once per device with
// that device current.
int scratch_for(int device, unsigned char **out) {
    if (device < 0 || device >= kMaxDevices) return fail(SA_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "scratch symbol lookup");
        if (!p) return fail(SA_EDEVICE, "scratch symbol lookup returned no address");
        g_scratch[device] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch[device]);
    return SA_OK;
}

}  // namespace

extern "C" int64_t sa_noalloc_max_reads(int pack_pass) {
    // the largest batch whose layout fits (layout grows with nreads)
    int64_t lo = 0, hi = INT32_MAX;
    if (!pack_pass) return layout(hi, false, nullptr, nullptr) <= kScratchBytes ? hi : 0;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (layout(mid, true, nullptr, nullptr) <= kScratchBytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

extern "C" int match_batch_dev_noalloc(const sa_dindex *dc, const uint8_t *d_reads, const int64_t *d_offs,
                                       int64_t nreads, sa_hit *d_out, void *hip_stream, const sa_match_cfg *cfg) {
    clear_error();
    if (!dc || !d_offs || (nreads > 0 && (!d_reads || !d_out))) return fail(SA_EINVAL, "NULL argument");
    if (nreads < 0 || nreads > INT32_MAX) return fail(SA_EINVAL, "nreads out of range");
    if (nreads == 0) return SA_OK;
    sa_dindex *d = const_cast<sa_dindex *>(dc);
    sa_match_cfg c = resolve_cfg(d, cfg);
    if (c.profile || c.count)
        return fail(SA_EINVAL, "profile and count keep per-stream state and are not available without allocation");
    c.use_graph = 0;  // a graph instantiation allocates; the launches go to the stream directly
    int rc = check_cfg(d, c);
    if (rc) return rc;
    DeviceGuard g(d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    unsigned char *base = nullptr;
    if ((rc = scratch_for(d->device, &base))) return rc;
    const bool pack_pass = !packs_inline(c);
    const size_t need = layout(nreads, pack_pass, nullptr, nullptr);
    if (need > kScratchBytes)
        return fail(SA_ENOSPC, "batch of " + std::to_string(nreads) + " reads needs " + std::to_string(need) +
                                   " bytes of scratch on this path (pack pass); the fixed scratch holds " +
                                   std::to_string(kScratchBytes) + " (at most " +
                                   std::to_string(sa_noalloc_max_reads(1)) + " reads)");
    BatchBuffers b{};
    layout(nreads, pack_pass, base, &b);
    return enqueue_pipeline(d, b, nullptr, d_reads, d_offs, nullptr, nreads, d_out,
                            static_cast<hipStream_t>(hip_stream), c);
}
