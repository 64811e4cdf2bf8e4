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

// Per-block digit counts, digit-major: hist[d * nblocks + block].
template <class K>
__global__ __launch_bounds__(kSortBlock) void sort_hist_kernel(const K *__restrict__ keys, int64_t n, int shift,
                                                               uint32_t *hist, int nblocks) {
    __shared__ uint32_t h[kSortBlock / 64][256];
    const int t = threadIdx.x, wave = t >> 6;
    for (int i = t; i < (kSortBlock / 64) * 256; i += kSortBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + r * kSortBlock + t;
        if (i < n) atomicAdd(&h[wave][(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
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

// Stable scatter of one tile of kSortTile keys.  Each wave owns a contiguous
// quarter of the tile, taken 64 keys per round in input order; lanes with
// the same digit are ranked by lane order.  Sweep 1 counts digits per wave;
// a block scan turns the counts into each wave's first slot per digit
// inside the tile; sweep 2 places every key in an LDS copy of the tile,
// ordered by digit; the tile is then written out so that consecutive
// threads store consecutive addresses of one digit's run.
template <class K>
__global__ __launch_bounds__(kSortBlock) void sort_scatter_kernel(const K *__restrict__ kin,
                                                                  const uint32_t *__restrict__ vin,
                                                                  K *__restrict__ kout, uint32_t *__restrict__ vout,
                                                                  int64_t n, int shift,
                                                                  const uint32_t *__restrict__ hist, int nblocks) {
    constexpr int kWaves = kSortBlock / 64;
    constexpr int kPerWave = kSortTile / kWaves;
    __shared__ K s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint32_t wslot[kWaves][256];  // per wave: count, then next slot per digit
    __shared__ uint32_t loc[256];            // first slot of each digit in the tile
    __shared__ uint32_t gbase[256];          // global position of the tile's first key of each digit
    __shared__ uint32_t scan_tmp[kWaves];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int i = t; i < kWaves * 256; i += kSortBlock) (&wslot[0][0])[i] = 0;
    for (int d = t; d < 256; d += kSortBlock) gbase[d] = hist[(size_t)d * nblocks + blockIdx.x];
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)wave * kPerWave;
    // sweep 1: digit counts per wave
#pragma unroll 1
    for (int r = 0; r < kPerWave / 64; ++r) {
        const int64_t i = base + r * 64 + lane;
        const bool valid = i < n;
        const K key = valid ? kin[i] : K(0);
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
    // sweep 2: place keys in the LDS tile, stable within each digit (the
    // tile's keys are read again; they are still in cache)
#pragma unroll 1
    for (int r = 0; r < kPerWave / 64; ++r) {
        const int64_t i = base + r * 64 + lane;
        const bool valid = i < n;
        const K key = valid ? kin[i] : K(0);
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint64_t peers = same_digit_lanes(d, valid);
        const int rank = __popcll(peers & lt_mask);
        if (valid) {
            const uint32_t pos = wslot[wave][d] + (uint32_t)rank;
            s_key[pos] = key;
            s_val[pos] = vin[i];
        }
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wslot[wave][d] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // write out: runs of one digit go to consecutive addresses
    const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
    const int count = (int)((n - tile0) < kSortTile ? (n - tile0) : kSortTile);
    for (int p = t; p < count; p += kSortBlock) {
        const K k = s_key[p];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint32_t g = gbase[d] + (uint32_t)p - loc[d];
        kout[g] = k;
        vout[g] = s_val[p];
    }
}

// Sort n pairs by key bits [lo_bit, hi_bit), starting from (k0, v0) with
// (k1, v1) as the other buffer; *which = 0 when the result is in (k0, v0),
// 1 when it is in (k1, v1).  hist holds 256 * ceil(n / kSortTile) counts,
// digit_total 256.  n < 2^32.
template <class K>
hipError_t radix_sort_pairs(K *k0, uint32_t *v0, K *k1, uint32_t *v1, uint32_t *hist, uint32_t *digit_total,
                            int64_t n, int lo_bit, int hi_bit, int *which, hipStream_t s) {
    K *key[2] = {k0, k1};
    uint32_t *val[2] = {v0, v1};
    int cur = 0;
    const int nblocks = (int)((n + kSortTile - 1) / kSortTile);
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
