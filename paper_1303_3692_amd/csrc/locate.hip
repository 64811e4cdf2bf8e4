// Locate: the text positions of each read's occurrences, i.e. the suffix
// array entries of its row interval (Section IV lists the occurrences of a
// read this way, in suffix-array order), as a CSR list.
//
//   count    one thread per read: how many rows of [lo, hi) it emits
//            (at most cap), 0 for reads not selected; bad intervals raise a
//            flag instead of being read
//   scan     exclusive sum of the counts into the int64 offsets (per-tile
//            sums, one workgroup over the tile sums, per-tile scan)
//   gather   one thread per read copies SA[lo .. lo + count) to its slot,
//            only when the whole list fits the caller's buffer
#include <hip/hip_runtime.h>

#include "device_state.h"

namespace samatch {
namespace {

constexpr int kLocBlock = 256;
constexpr int kLocItems = 16;
constexpr int kLocTile = kLocBlock * kLocItems;

__device__ __forceinline__ int64_t read_count(const int4 h, int n, int cap, int min_len, unsigned *bad) {
    const bool sel = min_len > 0 ? (h.z >= min_len) : ((h.w & (int)SA_HIT_EXACT) != 0);
    if (!sel) return 0;
    if (h.x < 0 || h.y > n || h.x > h.y) {
        atomicOr(bad, 1u);
        return 0;
    }
    const int c = h.y - h.x;
    return c < cap ? c : cap;
}

// Block-wide inclusive sum of one int64 per thread; returns the total.
__device__ __forceinline__ int64_t block_incl_sum(int64_t v, int64_t &incl, int64_t *lds /* >= blockDim/64 */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    int64_t before = 0, total = 0;
    for (int w = 0; w < nw; ++w) {
        const int64_t s = lds[w];
        if (w < wave) before += s;
        total += s;
    }
    incl = before + x;
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(kLocBlock) void locate_tile_sums_kernel(const int4 *__restrict__ hits, int64_t nreads,
                                                                     int n, int cap, int min_len,
                                                                     int64_t *__restrict__ tile_sum, unsigned *bad) {
    __shared__ int64_t lds[kLocBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kLocTile;
    int64_t s = 0;
    for (int r = 0; r < kLocItems; ++r) {
        const int64_t i = base + r * kLocBlock + threadIdx.x;
        if (i < nreads) s += read_count(hits[i], n, cap, min_len, bad);
    }
    int64_t incl;
    const int64_t total = block_incl_sum(s, incl, lds);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// One workgroup: tile sums become the sum of the tiles before; *total is
// the grand total.
__global__ __launch_bounds__(1024) void locate_scan_tiles_kernel(int64_t *tile_sum, int ntiles, int64_t *total) {
    __shared__ int64_t lds[1024 / 64];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < ntiles; b0 += 1024) {
        const int b = b0 + threadIdx.x;
        const int64_t v = b < ntiles ? tile_sum[b] : 0;
        int64_t incl;
        const int64_t t = block_incl_sum(v, incl, lds);
        const int64_t c = carry;
        if (b < ntiles) tile_sum[b] = c + incl - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + t;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kLocBlock) void locate_offsets_kernel(const int4 *__restrict__ hits, int64_t nreads,
                                                                   int n, int cap, int min_len,
                                                                   const int64_t *__restrict__ tile_sum,
                                                                   int64_t *__restrict__ offs, unsigned *bad) {
    __shared__ int64_t lds[kLocBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kLocTile;
    int64_t carry = tile_sum[blockIdx.x];
    for (int r = 0; r < kLocItems; ++r) {
        const int64_t i = base + r * kLocBlock + threadIdx.x;
        const int64_t c = i < nreads ? read_count(hits[i], n, cap, min_len, bad) : 0;
        int64_t incl;
        const int64_t t = block_incl_sum(c, incl, lds);
        if (i < nreads) offs[i] = carry + incl - c;
        carry += t;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) offs[nreads] = carry;
}

__global__ __launch_bounds__(256) void locate_gather_kernel(const int4 *__restrict__ hits, int64_t nreads,
                                                            const int64_t *__restrict__ offs,
                                                            const int32_t *__restrict__ sa,
                                                            int32_t *__restrict__ pos) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nreads) return;
    const int64_t o = offs[i], c = offs[i + 1] - o;
    const int lo = hits[i].x;
    for (int64_t j = 0; j < c; ++j) pos[o + j] = sa[lo + j];
}

}  // namespace
}  // namespace samatch

using namespace samatch;

extern "C" int sa_locate_dev(const sa_dindex *d, const sa_hit *d_hits, int64_t nreads, int32_t cap, int32_t min_len,
                             int64_t *d_offs, int32_t *d_pos, int64_t pos_capacity, void *hip_stream,
                             int64_t *total) {
    clear_error();
    if (!d || !d_offs || !total || (nreads > 0 && !d_hits)) return fail(SA_EINVAL, "NULL argument");
    if (nreads < 0 || cap < 0 || min_len < 0 || pos_capacity < 0) return fail(SA_EINVAL, "negative size");
    if (pos_capacity > 0 && !d_pos) return fail(SA_EINVAL, "NULL positions buffer");
    DeviceGuard g(d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t ntiles = nreads > 0 ? (nreads + kLocTile - 1) / kLocTile : 1;
    if (ntiles > INT32_MAX) return fail(SA_EINVAL, "too many reads");
    // scratch: tile sums, the total, the bad-interval flag (device), and a
    // pinned copy of total and flag
    struct Scratch {
        int64_t *dev = nullptr;
        int64_t *host = nullptr;
        ~Scratch() {
            if (dev) (void)hipFree(dev);
            if (host) (void)hipHostFree(host);
        }
    } sc;
    hipError_t e;
    if ((e = hipMalloc((void **)&sc.dev, sizeof(int64_t) * (size_t)(ntiles + 2))) != hipSuccess ||
        (e = hipHostMalloc((void **)&sc.host, sizeof(int64_t) * 2, hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "locate scratch");
    int64_t *tile_sum = sc.dev, *d_total = sc.dev + ntiles;
    unsigned *bad = reinterpret_cast<unsigned *>(sc.dev + ntiles + 1);
    const int4 *hits = reinterpret_cast<const int4 *>(d_hits);
    const int n = (int)d->n;
    if ((e = hipMemsetAsync(bad, 0, sizeof(int64_t), s)) != hipSuccess) return hip_fail(e, "locate");
    if (nreads > 0) {
        hipLaunchKernelGGL(locate_tile_sums_kernel, dim3((unsigned)ntiles), dim3(kLocBlock), 0, s, hits, nreads, n,
                           cap, min_len, tile_sum, bad);
        hipLaunchKernelGGL(locate_scan_tiles_kernel, dim3(1), dim3(1024), 0, s, tile_sum, (int)ntiles, d_total);
        hipLaunchKernelGGL(locate_offsets_kernel, dim3((unsigned)ntiles), dim3(kLocBlock), 0, s, hits, nreads, n, cap,
                           min_len, tile_sum, d_offs, bad);
    } else if ((e = hipMemsetAsync(d_offs, 0, sizeof(int64_t), s)) != hipSuccess ||
               (e = hipMemsetAsync(d_total, 0, sizeof(int64_t), s)) != hipSuccess) {
        return hip_fail(e, "locate");
    }
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(sc.host, d_total, sizeof(int64_t) * 2, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "locate counts");
    *total = sc.host[0];
    if ((unsigned)sc.host[1] != 0u) return fail(SA_EINVAL, "a selected hit has an interval outside [0, n]");
    if (*total > pos_capacity) return fail(SA_ENOSPC, "positions buffer too small (see *total)");
    if (nreads > 0 && *total > 0) {
        hipLaunchKernelGGL(locate_gather_kernel, dim3((unsigned)((nreads + 255) / 256)), dim3(256), 0, s, hits, nreads,
                           d_offs, d->d_sa, d_pos);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "locate gather");
    }
    return SA_OK;
}

extern "C" int sa_locate(const sa_dindex *d, const sa_hit *hits, int64_t nreads, int32_t cap, int32_t min_len,
                         int64_t *offs, int32_t *pos, int64_t pos_capacity, int64_t *total) {
    clear_error();
    if (!d || !offs || !total || (nreads > 0 && !hits)) return fail(SA_EINVAL, "NULL argument");
    if (nreads < 0 || pos_capacity < 0) return fail(SA_EINVAL, "negative size");
    if (pos_capacity > 0 && !pos) return fail(SA_EINVAL, "NULL positions buffer");
    DeviceGuard g(d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    struct Buffers {
        sa_hit *hits = nullptr;
        int64_t *offs = nullptr;
        int32_t *pos = nullptr;
        hipStream_t s = nullptr;
        ~Buffers() {
            if (s) (void)hipStreamSynchronize(s);
            if (hits) (void)hipFree(hits);
            if (offs) (void)hipFree(offs);
            if (pos) (void)hipFree(pos);
            if (s) (void)hipStreamDestroy(s);
        }
    } b;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&b.s, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipMalloc((void **)&b.hits, sizeof(sa_hit) * (size_t)(nreads > 0 ? nreads : 1))) != hipSuccess ||
        (e = hipMalloc((void **)&b.offs, sizeof(int64_t) * (size_t)(nreads + 1))) != hipSuccess)
        return hip_fail(e, "locate buffers");
    if (nreads > 0 &&
        (e = hipMemcpyAsync(b.hits, hits, sizeof(sa_hit) * (size_t)nreads, hipMemcpyHostToDevice, b.s)) != hipSuccess)
        return hip_fail(e, "locate upload");
    // counts and offsets first; positions only when they fit
    int rc = sa_locate_dev(d, b.hits, nreads, cap, min_len, b.offs, nullptr, 0, b.s, total);
    if (rc != SA_OK && rc != SA_ENOSPC) return rc;
    if ((e = hipMemcpy(offs, b.offs, sizeof(int64_t) * (size_t)(nreads + 1), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "locate download");
    if (*total == 0) return SA_OK;
    if (*total > pos_capacity) return fail(SA_ENOSPC, "positions buffer too small (see *total)");
    if ((e = hipMalloc((void **)&b.pos, sizeof(int32_t) * (size_t)*total)) != hipSuccess)
        return hip_fail(e, "locate buffers");
    rc = sa_locate_dev(d, b.hits, nreads, cap, min_len, b.offs, b.pos, *total, b.s, total);
    if (rc) return rc;
    if ((e = hipMemcpyAsync(pos, b.pos, sizeof(int32_t) * (size_t)*total, hipMemcpyDeviceToHost, b.s)) != hipSuccess ||
        (e = hipStreamSynchronize(b.s)) != hipSuccess)
        return hip_fail(e, "locate download");
    return SA_OK;
}
