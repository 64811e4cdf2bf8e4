// Suffix array of the packed reference built on the device (Section III
// defines the array: the text positions of all suffixes in ascending
// lexicographic order, a suffix that is a prefix of another sorting first).
//
// The paper builds it with DC3 on the host.  Here the device sorts by
// prefix doubling, which maps onto the radix sort the batch path already
// has:
//   step 0   every position gets a 63-bit key, its first 21 bases as 3-bit
//            codes (0 past the text end, 1..4 for a, c, g, t), and the
//            (key, position) pairs are radix sorted.  rank[i] = 1 + the
//            first row of i's group of equal keys.
//   step h   (h = 21, 42, 84, ...) only suffixes in groups of two or more
//            are kept.  Each gets the key rank[i] * 2^B + rank[i+h]
//            (0 past the end), the kept pairs are sorted, and each old group
//            splits into groups of equal keys, ranked by their first row.
// A group of one is final.  Groups are contiguous runs of rows, so the kept
// list, taken in row order, stays sorted by group; after the sort each
// member goes back to one of its group's rows, the same rows in the same
// order.  All ranks of step h are read before any is rewritten (separate
// kernels), so every key uses ranks of h-prefixes.
//
// Device memory: keys 2 x 8n, values 2 x 4n, kept rows 2 x 4n, rank 4n,
// sort histograms 256 x 4 x ceil(n / 2048) bytes.
#include <hip/hip_runtime.h>

#include <vector>

#include "device_state.h"
#include "radix_sort.h"

namespace samatch {
namespace {

constexpr int kInitBases = 21;  // 3-bit codes in a 63-bit key
constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;

// Step 0 keys: first 21 bases of the suffix at i as 3-bit codes, MSB first.
__global__ __launch_bounds__(256) void sa_init_keys_kernel(const uint64_t *__restrict__ text, int64_t n,
                                                           uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t w = i >> 5;
    const unsigned sh = (unsigned)(i & 31) * 2u;
    const uint64_t lo = text[w], hi = text[w + 1];  // the text carries zero pad words
    const uint64_t x = sh ? (lo << sh) | (hi >> (64u - sh)) : lo;
    const int64_t left = n - i;
    const int take = left < kInitBases ? (int)left : kInitBases;
    uint64_t k = 0;
#pragma unroll
    for (int j = 0; j < kInitBases; ++j) {
        const uint64_t c = j < take ? ((x >> (62 - 2 * j)) & 3u) + 1u : 0u;
        k = (k << 3) | c;
    }
    key[i] = k;
    val[i] = (uint32_t)i;
}

// Step h keys for the kept suffixes: rank of the suffix, then rank of the
// suffix h further on (0 past the end).
__global__ __launch_bounds__(256) void sa_pair_keys_kernel(const uint32_t *__restrict__ rank,
                                                           const uint32_t *__restrict__ suf, int64_t u_count,
                                                           int64_t n, int64_t h, int bits,
                                                           uint64_t *__restrict__ key) {
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u >= u_count) return;
    const int64_t s = suf[u];
    const uint64_t r2 = s + h < n ? rank[s + h] : 0u;
    key[u] = ((uint64_t)rank[s] << bits) | r2;
}

// Per sorted element u of the current list (sorted keys `key`, row of slot
// u `row`, or u itself when row is NULL):
//   head    u starts a run of equal keys
//   single  a run of one (final)
//   mval    1 + row when head, else 0; its running maximum is the new rank
//   keep    not single; its running count places u in the next list
struct ElemFlags {
    uint32_t mval;
    uint32_t keep;
    uint32_t row;
};

__device__ __forceinline__ ElemFlags elem_flags(const uint64_t *__restrict__ key, const uint32_t *__restrict__ row,
                                                int64_t u, int64_t u_count) {
    ElemFlags f{0u, 0u, 0u};
    if (u >= u_count) return f;
    const uint64_t k = key[u];
    const bool head = u == 0 || key[u - 1] != k;
    const bool last = u + 1 == u_count || key[u + 1] != k;
    f.row = row ? row[u] : (uint32_t)u;
    f.mval = head ? f.row + 1u : 0u;
    f.keep = (head && last) ? 0u : 1u;
    return f;
}

// Block scan of (max, sum) pairs, one per thread: inclusive and exclusive
// running maximum, exclusive running sum, and the block totals.  lds holds
// 2 * (blockDim / 64) words.
struct ScanOut {
    uint32_t incl_max, excl_max, excl_sum, tmax, tsum;
};

__device__ __forceinline__ ScanOut block_scan_max_sum(uint32_t m, uint32_t s, uint32_t *lds) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
    uint32_t xm = m, xs = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t ym = __shfl_up(xm, o, 64), ys = __shfl_up(xs, o, 64);
        if (lane >= o) {
            xm = xm > ym ? xm : ym;
            xs += ys;
        }
    }
    const uint32_t pm = __shfl_up(xm, 1, 64);
    if (lane == 63) {
        lds[wave] = xm;
        lds[nw + wave] = xs;
    }
    __syncthreads();
    ScanOut o{0u, 0u, 0u, 0u, 0u};
    uint32_t bm = 0, bs = 0;
    for (int w = 0; w < nw; ++w) {
        const uint32_t wm = lds[w], ws = lds[nw + w];
        if (w < wave) {
            bm = bm > wm ? bm : wm;
            bs += ws;
        }
        o.tmax = o.tmax > wm ? o.tmax : wm;
        o.tsum += ws;
    }
    const uint32_t wexcl = lane ? pm : 0u;
    o.incl_max = xm > bm ? xm : bm;
    o.excl_max = wexcl > bm ? wexcl : bm;
    o.excl_sum = bs + xs - s;
    __syncthreads();
    return o;
}

// Pass 1: per tile, the maximum of mval and the count of kept elements.
__global__ __launch_bounds__(kScanBlock) void sa_flags_reduce_kernel(const uint64_t *__restrict__ key,
                                                                     const uint32_t *__restrict__ row,
                                                                     int64_t u_count, uint32_t *__restrict__ tile_max,
                                                                     uint32_t *__restrict__ tile_sum) {
    __shared__ uint32_t lds[2 * (kScanBlock / 64)];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t m = 0, s = 0;
    for (int r = 0; r < kScanItems; ++r) {
        const ElemFlags f = elem_flags(key, row, base + r * kScanBlock + threadIdx.x, u_count);
        m = m > f.mval ? m : f.mval;
        s += f.keep;
    }
    const ScanOut o = block_scan_max_sum(m, s, lds);
    if (threadIdx.x == 0) {
        tile_max[blockIdx.x] = o.tmax;
        tile_sum[blockIdx.x] = o.tsum;
    }
}

// Pass 2 (one workgroup): tile totals become the running maximum of the
// tiles before and the count of kept elements before; *kept = the total.
__global__ __launch_bounds__(1024) void sa_flags_scan_tiles_kernel(uint32_t *tile_max, uint32_t *tile_sum, int ntiles,
                                                                   uint32_t *kept) {
    __shared__ uint32_t lds[2 * (1024 / 64)];
    __shared__ uint32_t carry_m, carry_s;
    if (threadIdx.x == 0) {
        carry_m = 0;
        carry_s = 0;
    }
    __syncthreads();
    for (int b0 = 0; b0 < ntiles; b0 += 1024) {
        const int b = b0 + threadIdx.x;
        const uint32_t m = b < ntiles ? tile_max[b] : 0u, s = b < ntiles ? tile_sum[b] : 0u;
        const ScanOut o = block_scan_max_sum(m, s, lds);
        const uint32_t cm = carry_m, cs = carry_s;
        if (b < ntiles) {
            tile_max[b] = o.excl_max > cm ? o.excl_max : cm;
            tile_sum[b] = cs + o.excl_sum;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            carry_m = cm > o.tmax ? cm : o.tmax;
            carry_s = cs + o.tsum;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *kept = carry_s;
}

// Pass 3: new ranks, rows of the suffix array, and the next list.
__global__ __launch_bounds__(kScanBlock) void sa_flags_apply_kernel(
    const uint64_t *__restrict__ key, const uint32_t *__restrict__ suf, const uint32_t *__restrict__ row,
    int64_t u_count, const uint32_t *__restrict__ tile_max, const uint32_t *__restrict__ tile_sum,
    uint32_t *__restrict__ rank, int32_t *__restrict__ sa, uint32_t *__restrict__ next_suf,
    uint32_t *__restrict__ next_row) {
    __shared__ uint32_t lds[2 * (kScanBlock / 64)];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t carry_m = tile_max[blockIdx.x], carry_s = tile_sum[blockIdx.x];
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t u = base + r * kScanBlock + threadIdx.x;
        const ElemFlags f = elem_flags(key, row, u, u_count);
        const ScanOut o = block_scan_max_sum(f.mval, f.keep, lds);
        if (u < u_count) {
            const uint32_t nr = o.incl_max > carry_m ? o.incl_max : carry_m;
            const uint32_t s = suf[u];
            sa[f.row] = (int32_t)s;
            rank[s] = nr;
            if (f.keep) {
                const uint32_t at = carry_s + o.excl_sum;
                next_suf[at] = s;
                next_row[at] = f.row;
            }
        }
        carry_m = carry_m > o.tmax ? carry_m : o.tmax;
        carry_s += o.tsum;
    }
}

}  // namespace

// Builds sa[0..n) of the packed text d_text (with zero pad words after the
// text) on stream s; rank_out (nullable, n entries) receives 1 + the row of
// each text position.  Allocates its scratch and frees it before returning.
int build_sa_device(const uint64_t *d_text, int64_t n, int32_t *d_sa, uint32_t *rank_out, hipStream_t s,
                    SaBuildInfo *info) {
    if (n < 1 || n > INT32_MAX) return fail(SA_EINVAL, "text length out of range for device construction");
    const int64_t tiles_scan = (n + kScanTile - 1) / kScanTile;
    uint64_t *key[2] = {nullptr, nullptr};
    uint32_t *val[2] = {nullptr, nullptr}, *row[2] = {nullptr, nullptr};
    uint32_t *rank = nullptr, *hist = nullptr, *digit_total = nullptr, *tmax = nullptr, *tsum = nullptr;
    uint32_t *kept_d = nullptr, *kept_h = nullptr;
    int bits = 1;
    while (((int64_t)1 << bits) <= n) bits++;  // ranks are at most n < 2^bits
    int rc = SA_OK;
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    };
    for (int k = 0; k < 2; ++k) {
        alloc((void **)&key[k], sizeof(uint64_t) * (size_t)n);
        alloc((void **)&val[k], sizeof(uint32_t) * (size_t)n);
        alloc((void **)&row[k], sizeof(uint32_t) * (size_t)n);
    }
    if (rank_out) rank = rank_out;
    else alloc((void **)&rank, sizeof(uint32_t) * (size_t)n);
    alloc((void **)&hist, sizeof(uint32_t) * sort_hist_words<uint64_t>(n));
    alloc((void **)&digit_total, sizeof(uint32_t) * 256);
    alloc((void **)&tmax, sizeof(uint32_t) * (size_t)tiles_scan);
    alloc((void **)&tsum, sizeof(uint32_t) * (size_t)tiles_scan);
    alloc((void **)&kept_d, sizeof(uint32_t));
    if (e == hipSuccess) e = hipHostMalloc((void **)&kept_h, sizeof(uint32_t), hipHostMallocDefault);
    if (e != hipSuccess) rc = hip_fail(e, "suffix array scratch allocation");

    // sort (keys, values) in the pair (key[c], val[c]); returns the buffer
    // index holding the result
    auto sort = [&](int c, int64_t count, int hi_bit, int *out) {
        int which = 0;
        e = radix_sort_pairs<uint64_t>(key[c], val[c], key[c ^ 1], val[c ^ 1], hist, digit_total, count, 0, hi_bit,
                                       &which, s);
        *out = which ? c ^ 1 : c;
    };
    // ranks, SA rows and the next list from the sorted (key[c], val[c]);
    // rows of slots in row_in (NULL: identity).  Returns the kept count.
    auto apply = [&](int c, const uint32_t *row_in, uint32_t *row_out, int64_t count, int64_t *kept) {
        const int nt = (int)((count + kScanTile - 1) / kScanTile);
        hipLaunchKernelGGL(sa_flags_reduce_kernel, dim3(nt), dim3(kScanBlock), 0, s, key[c], row_in, count, tmax,
                           tsum);
        hipLaunchKernelGGL(sa_flags_scan_tiles_kernel, dim3(1), dim3(1024), 0, s, tmax, tsum, nt, kept_d);
        hipLaunchKernelGGL(sa_flags_apply_kernel, dim3(nt), dim3(kScanBlock), 0, s, key[c], val[c], row_in, count,
                           tmax, tsum, rank, d_sa, val[c ^ 1], row_out);
        if ((e = hipGetLastError()) != hipSuccess) return;
        if ((e = hipMemcpyAsync(kept_h, kept_d, sizeof(uint32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return;
        *kept = *kept_h;
    };

    int64_t count = n, kept = 0;
    int c = 0, rsel = 0, steps = 0;
    if (rc == SA_OK) {
        hipLaunchKernelGGL(sa_init_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_text, n,
                           key[0], val[0]);
        if ((e = hipGetLastError()) == hipSuccess) sort(0, n, 3 * kInitBases, &c);
        if (e == hipSuccess) apply(c, nullptr, row[0], n, &kept);
        steps = 1;
        // the next list is in (val[c ^ 1], row[0])
        int64_t h = kInitBases;
        while (e == hipSuccess && kept > 0) {
            count = kept;
            c ^= 1;
            hipLaunchKernelGGL(sa_pair_keys_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, rank,
                               val[c], count, n, h, bits, key[c]);
            if ((e = hipGetLastError()) != hipSuccess) break;
            int sorted = c;
            sort(c, count, 2 * bits, &sorted);
            if (e != hipSuccess) break;
            c = sorted;
            apply(c, row[rsel], row[rsel ^ 1], count, &kept);
            rsel ^= 1;
            steps++;
            h *= 2;
            if (info) info->sorted_elems += count;
            if (h > 2 * n + kInitBases) {  // every group is a single suffix long before this
                rc = fail(SA_EDEVICE, "suffix sorting did not converge");
                break;
            }
        }
        if (e != hipSuccess && rc == SA_OK) rc = hip_fail(e, "suffix array construction");
        else if (rc == SA_OK && (e = hipStreamSynchronize(s)) != hipSuccess) rc = hip_fail(e, "suffix array construction");
    }
    if (info) {
        info->steps = steps;
        info->sorted_elems += n;
    }
    for (int k = 0; k < 2; ++k)
        for (void *p : {(void *)key[k], (void *)val[k], (void *)row[k]})
            if (p) (void)hipFree(p);
    if (!rank_out && rank) (void)hipFree(rank);
    for (void *p : {(void *)hist, (void *)digit_total, (void *)tmax, (void *)tsum, (void *)kept_d})
        if (p) (void)hipFree(p);
    if (kept_h) (void)hipHostFree(kept_h);
    return rc;
}

}  // namespace samatch
