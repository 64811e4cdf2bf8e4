// Measurement helper, not part of the matching path: the rate at which the
// device serves random 16-byte loads, the access pattern of the search
// kernels' probes (row records, prefix-table entries, text words).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_state.h"
#include "internal.h"
#include "samatch_measure.h"

using namespace samatch;

namespace {

constexpr int kChains = 2;   // independent chains per lane
constexpr int kDepth = 16;   // dependent loads per chain
constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__global__ void probe_fill_kernel(uint4 *tab, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) tab[i] = make_uint4(i, mix32(i), 3u * i, 7u * i);
}

// Each lane follows kChains chains; the next position of a chain depends on
// the entry just loaded (masked to the table, so every load is in bounds).
__global__ __launch_bounds__(kBlock) void probe_chase_kernel(const uint4 *__restrict__ tab, uint32_t mask,
                                                             uint32_t *__restrict__ out) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t idx[kChains], acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) idx[c] = mix32(t * kChains + c + 12345u) & mask;
    for (int d = 0; d < kDepth; ++d) {
        uint4 v[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) v[c] = tab[idx[c]];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            acc += v[c].x;
            idx[c] = mix32(v[c].y ^ idx[c] ^ (uint32_t)d) & mask;
        }
    }
    out[t] = acc;
}

}  // namespace

extern "C" int sa_random_read_rate(int device, int log2_entries, double *loads_per_s) {
    clear_error();
    if (!loads_per_s) return fail(SA_EINVAL, "NULL argument");
    if (log2_entries < 8 || log2_entries > 28) return fail(SA_EINVAL, "log2_entries must be in 8..28");
    DeviceGuard g(device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    hipDeviceProp_t prop;
    hipError_t e;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    const uint32_t n = 1u << log2_entries;
    const int blocks = std::max(1, prop.multiProcessorCount * 4);  // 16 waves per compute unit
    uint4 *tab = nullptr;
    uint32_t *out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    int rc = SA_OK;
    float best = 1e30f;
    if ((e = hipMalloc((void **)&tab, sizeof(uint4) * (size_t)n)) != hipSuccess ||
        (e = hipMalloc((void **)&out, sizeof(uint32_t) * (size_t)blocks * kBlock)) != hipSuccess ||
        (e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
        rc = hip_fail(e, "random-read probe set-up");
        goto done;
    }
    hipLaunchKernelGGL(probe_fill_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, nullptr, tab, n);
    for (int rep = 0; rep < 6; ++rep) {
        (void)hipEventRecord(a, nullptr);
        hipLaunchKernelGGL(probe_chase_kernel, dim3(blocks), dim3(kBlock), 0, nullptr, tab, n - 1, out);
        (void)hipEventRecord(b, nullptr);
        if ((e = hipEventSynchronize(b)) != hipSuccess) {
            rc = hip_fail(e, "random-read probe");
            goto done;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        if (rep > 0) best = std::min(best, ms);  // the first launch warms up
    }
    *loads_per_s = (double)blocks * kBlock * kChains * kDepth / (best * 1e-3);
done:
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (out) (void)hipFree(out);
    if (tab) (void)hipFree(tab);
    return rc;
}
