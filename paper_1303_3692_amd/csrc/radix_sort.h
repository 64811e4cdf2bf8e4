// Stable LSD radix sort of (key, 32-bit value) pairs on the device, 8-bit
// digits, for 32- and 64-bit keys.  Used by the batch path (read prefixes)
// and by suffix-array construction (rank pairs).
//
// One pass over bits [shift, shift + 8): per-tile digit counts, a scan of
// the counts into global positions, then a scatter that reorders each tile
// in LDS so that runs of one digit are written to consecutive addresses.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.h"

namespace samatch {
namespace {  // each translation unit that sorts gets its own copy

static_assert(kSortBlock == 256, "the scatter kernel's digit loops assume one digit per thread");

// Keys per workgroup tile: 16 per thread for 32-bit keys, 8 for 64-bit keys
// (the scatter stages a tile's input and output in LDS).
template <class K>
struct SortTile {
    static constexpr int items = sizeof(K) == 4 ? 16 : 8;
    static constexpr int size = kSortBlock * items;
};
static_assert(SortTile<uint32_t>::size == kSortTile, "batch histograms are sized with kSortTile");

// Per-block digit counts, digit-major: hist[d * nblocks + block].
template <class K>
__global__ __launch_bounds__(kSortBlock) void sort_hist_kernel(const K *__restrict__ keys, int64_t n, int shift,
                                                               uint32_t *hist, int nblocks) {
    constexpr int kItems = SortTile<K>::items;
    __shared__ uint32_t h[kSortBlock / 64][256];
    const int t = threadIdx.x, wave = t >> 6;
    for (int i = t; i < (kSortBlock / 64) * 256; i += kSortBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SortTile<K>::size;
    K k[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {  // all loads in flight before the counting
        const int64_t i = base + r * kSortBlock + t;
        k[r] = i < n ? keys[i] : K(0);
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r)
        if (base + r * kSortBlock + t < n) atomicAdd(&h[wave][(uint32_t)(k[r] >> shift) & 255u], 1u);
    __syncthreads();
    for (int d = t; d < 256; d += kSortBlock) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < kSortBlock / 64; ++w) s += h[w][d];
        hist[(size_t)d * nblocks + blockIdx.x] = s;
    }
}

// Block-wide exclusive scan of one value per thread; returns the total.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t &excl, uint32_t *lds /* >= blockDim/64 */) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < nw; ++w) {
        const uint32_t s = lds[w];
        if (w < wave) before += s;
        total += s;
    }
    excl = before + x - v;
    __syncthreads();
    return total;
}

// Totals per digit (one block per digit).
__global__ __launch_bounds__(256) void sort_digit_total_kernel(const uint32_t *__restrict__ hist, int nblocks,
                                                               uint32_t *digit_total) {
    __shared__ uint32_t lds[4];
    const int d = blockIdx.x;
    uint32_t s = 0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += hist[(size_t)d * nblocks + b];
    uint32_t excl;
    const uint32_t total = block_exclusive_scan(s, excl, lds);
    if (threadIdx.x == 0) digit_total[d] = total;
}

// Exclusive scan of hist in place: entry (d, b) becomes the output position
// of block b's first key with digit d.  One block per digit.
__global__ __launch_bounds__(256) void sort_scan_kernel(uint32_t *hist, int nblocks,
                                                        const uint32_t *__restrict__ digit_total) {
    __shared__ uint32_t lds[4];
    __shared__ uint32_t carry;
    const int d = blockIdx.x;
    if (threadIdx.x == 0) {
        uint32_t base = 0;
        for (int e = 0; e < d; ++e) base += digit_total[e];
        carry = base;
    }
    __syncthreads();
    for (int b0 = 0; b0 < nblocks; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const uint32_t v = b < nblocks ? hist[(size_t)d * nblocks + b] : 0u;
        uint32_t excl;
        const uint32_t total = block_exclusive_scan(v, excl, lds);
        const uint32_t c = carry;
        if (b < nblocks) hist[(size_t)d * nblocks + b] = c + excl;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + total;
        __syncthreads();
    }
}

// Lanes of the wave whose digit equals this lane's, found with eight ballots
// (one per digit bit).
__device__ __forceinline__ uint64_t same_digit_lanes(uint32_t d, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const bool set = (d >> bit) & 1u;
        const uint64_t bal = __ballot(set);
        peers &= set ? bal : ~bal;
    }
    return peers;
}

// Stable scatter of one tile of keys.  The tile's keys and values are first
// copied into LDS with 16-byte loads, all in flight together.  Each wave
// owns a contiguous quarter of the tile, taken 64 keys per round in input
// order; lanes with the same digit are ranked by lane order.  Sweep 1
// counts digits per wave; a block scan turns the counts into each wave's
// first slot per digit inside the tile; sweep 2 places every key in a
// second LDS copy of the tile, ordered by digit; the tile is then written
// out so that consecutive threads store consecutive addresses of one
// digit's run.
template <class K>
__global__ __launch_bounds__(kSortBlock) void sort_scatter_kernel(const K *__restrict__ kin,
                                                                  const uint32_t *__restrict__ vin,
                                                                  K *__restrict__ kout, uint32_t *__restrict__ vout,
                                                                  int64_t n, int shift,
                                                                  const uint32_t *__restrict__ hist, int nblocks) {
    constexpr int kTile = SortTile<K>::size;
    constexpr int kWaves = kSortBlock / 64;
    constexpr int kPerWave = kTile / kWaves;
    __shared__ __align__(16) K in_key[kTile];
    __shared__ __align__(16) uint32_t in_val[kTile];
    __shared__ K s_key[kTile];
    __shared__ uint32_t s_val[kTile];
    __shared__ uint32_t wslot[kWaves][256];  // per wave: count, then next slot per digit
    __shared__ uint32_t loc[256];            // first slot of each digit in the tile
    __shared__ uint32_t gbase[256];          // global position of the tile's first key of each digit
    __shared__ uint32_t scan_tmp[kWaves];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t tile0 = (int64_t)blockIdx.x * kTile;
    const int count = (int)((n - tile0) < kTile ? (n - tile0) : kTile);
    if (count == kTile) {
        // a full tile starts at a multiple of kTile elements: 16-byte aligned
        const uint4 *ks = reinterpret_cast<const uint4 *>(kin + tile0);
        const uint4 *vs = reinterpret_cast<const uint4 *>(vin + tile0);
        uint4 *kd = reinterpret_cast<uint4 *>(in_key);
        uint4 *vd = reinterpret_cast<uint4 *>(in_val);
        constexpr int kKeyVecs = kTile * (int)sizeof(K) / 16, kValVecs = kTile * 4 / 16;
#pragma unroll
        for (int c = 0; c < kKeyVecs / kSortBlock; ++c) kd[c * kSortBlock + t] = ks[c * kSortBlock + t];
#pragma unroll
        for (int c = 0; c < kValVecs / kSortBlock; ++c) vd[c * kSortBlock + t] = vs[c * kSortBlock + t];
    } else {
        for (int p = t; p < count; p += kSortBlock) {
            in_key[p] = kin[tile0 + p];
            in_val[p] = vin[tile0 + p];
        }
    }
    for (int i = t; i < kWaves * 256; i += kSortBlock) (&wslot[0][0])[i] = 0;
    for (int d = t; d < 256; d += kSortBlock) gbase[d] = hist[(size_t)d * nblocks + blockIdx.x];
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int base = wave * kPerWave;
    // sweep 1: digit counts per wave
#pragma unroll 1
    for (int r = 0; r < kPerWave / 64; ++r) {
        const int p = base + r * 64 + lane;
        const bool valid = p < count;
        const K key = valid ? in_key[p] : K(0);
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint64_t peers = same_digit_lanes(d, valid);
        if (valid && __popcll(peers & lt_mask) == 0) wslot[wave][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // block scan over digits of the per-digit tile totals; then each wave's
    // first slot for each digit
    for (int d = t; d < 256; d += kSortBlock) {
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) tot += wslot[w][d];
        uint32_t excl;
        block_exclusive_scan(tot, excl, scan_tmp);
        loc[d] = excl;
        uint32_t run = excl;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = wslot[w][d];
            wslot[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
    // sweep 2: place keys in the second LDS tile, stable within each digit
#pragma unroll 1
    for (int r = 0; r < kPerWave / 64; ++r) {
        const int p = base + r * 64 + lane;
        const bool valid = p < count;
        const K key = valid ? in_key[p] : K(0);
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint64_t peers = same_digit_lanes(d, valid);
        const int rank = __popcll(peers & lt_mask);
        if (valid) {
            const uint32_t pos = wslot[wave][d] + (uint32_t)rank;
            s_key[pos] = key;
            s_val[pos] = in_val[p];
        }
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wslot[wave][d] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // write out: runs of one digit go to consecutive addresses
    for (int p = t; p < count; p += kSortBlock) {
        const K k = s_key[p];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint32_t g = gbase[d] + (uint32_t)p - loc[d];
        kout[g] = k;
        vout[g] = s_val[p];
    }
}

// Histogram words radix_sort_pairs<K> needs for n keys.
template <class K>
inline size_t sort_hist_words(int64_t n) {
    return 256 * (size_t)((n + SortTile<K>::size - 1) / SortTile<K>::size);
}

// Sort n pairs by key bits [lo_bit, hi_bit), starting from (k0, v0) with
// (k1, v1) as the other buffer; *which = 0 when the result is in (k0, v0),
// 1 when it is in (k1, v1).  hist holds sort_hist_words<K>(n) counts,
// digit_total 256.  n < 2^32.
template <class K>
hipError_t radix_sort_pairs(K *k0, uint32_t *v0, K *k1, uint32_t *v1, uint32_t *hist, uint32_t *digit_total,
                            int64_t n, int lo_bit, int hi_bit, int *which, hipStream_t s) {
    K *key[2] = {k0, k1};
    uint32_t *val[2] = {v0, v1};
    int cur = 0;
    const int nblocks = (int)((n + SortTile<K>::size - 1) / SortTile<K>::size);
    if (n > 1) {
        for (int shift = lo_bit; shift < hi_bit; shift += 8) {
            hipLaunchKernelGGL(sort_hist_kernel<K>, dim3(nblocks), dim3(kSortBlock), 0, s, key[cur], n, shift, hist,
                               nblocks);
            hipLaunchKernelGGL(sort_digit_total_kernel, dim3(256), dim3(256), 0, s, hist, nblocks, digit_total);
            hipLaunchKernelGGL(sort_scan_kernel, dim3(256), dim3(256), 0, s, hist, nblocks, digit_total);
            hipLaunchKernelGGL(sort_scatter_kernel<K>, dim3(nblocks), dim3(kSortBlock), 0, s, key[cur], val[cur],
                               key[cur ^ 1], val[cur ^ 1], n, shift, hist, nblocks);
            cur ^= 1;
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    *which = cur;
    return hipSuccess;
}

}  // namespace
}  // namespace samatch
