// Memory-level probe kernels (measurement only): streaming read bandwidth and the
// latency of dependent loads in a buffer whose size selects the memory level that
// holds it (HBM, the MALL, or the L2 of each XCD).

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace pt {
namespace {

constexpr int kProbeBlock = 256;
constexpr uint32_t kLineWords = 32;   // 128-byte lines

// line i's first word holds the next line of a single cycle through all lines:
// i -> (a*i + c) mod nlines, full period for a = 1 mod 4, c odd, nlines a power of two
__global__ __launch_bounds__(kProbeBlock) void k_probe_fill(uint32_t* buf, uint32_t nlines, uint32_t a, uint32_t c) {
    const uint32_t stride = gridDim.x * kProbeBlock;
    for (uint32_t i = blockIdx.x * kProbeBlock + threadIdx.x; i < nlines; i += stride)
        buf[(size_t)i * kLineWords] = (a * i + c) & (nlines - 1u);
}

// passes x n4 float4 reads spread over the grid, the buffer index wrapping around, with
// four independent loads in flight per thread whatever the buffer size
__global__ __launch_bounds__(kProbeBlock) void k_probe_read(const float4* __restrict__ buf, size_t n4, int passes,
                                                            uint32_t* sink) {
    const size_t stride = (size_t)gridDim.x * kProbeBlock;
    const size_t step = stride % n4;
    const size_t total = (size_t)passes * n4;
    size_t j = (size_t)blockIdx.x * kProbeBlock + threadIdx.x;
    size_t idx = j % n4;
    uint32_t acc = 0;
    for (; j + 3 * stride < total; j += 4 * stride) {
        const size_t i0 = idx;
        size_t i1 = i0 + step;
        if (i1 >= n4) i1 -= n4;
        size_t i2 = i1 + step;
        if (i2 >= n4) i2 -= n4;
        size_t i3 = i2 + step;
        if (i3 >= n4) i3 -= n4;
        const float4 v0 = buf[i0], v1 = buf[i1], v2 = buf[i2], v3 = buf[i3];
        acc ^= __float_as_uint(v0.x) ^ __float_as_uint(v1.y) ^ __float_as_uint(v2.z) ^ __float_as_uint(v3.w);
        idx = i3 + step;
        if (idx >= n4) idx -= n4;
    }
    for (; j < total; j += stride) {
        acc ^= __float_as_uint(buf[idx].x);
        idx += step;
        if (idx >= n4) idx -= n4;
    }
    if (acc == 0x9E3779B9u) sink[0] = acc;   // keeps the loads alive; the value is never used
}

// one lane follows the cycle: every load depends on the previous one
__global__ void k_probe_chase(const uint32_t* buf, uint32_t nlines, int steps, uint32_t* sink) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t i = 0;
    for (int s = 0; s < steps; ++s) i = buf[(size_t)(i & (nlines - 1u)) * kLineWords];
    sink[0] = i;
}

}  // namespace

hipError_t launch_probe_fill(uint32_t* buf, uint32_t nlines, hipStream_t st) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    hipLaunchKernelGGL(k_probe_fill, dim3((unsigned)cus * 8), dim3(kProbeBlock), 0, st, buf, nlines, 1664525u * 4u + 1u,
                       1013904223u);
    return hipGetLastError();
}

hipError_t launch_probe_read(const void* buf, size_t bytes, int passes, uint32_t* sink, hipStream_t st) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    hipLaunchKernelGGL(k_probe_read, dim3((unsigned)cus * 8), dim3(kProbeBlock), 0, st, (const float4*)buf, bytes / 16,
                       passes, sink);
    return hipGetLastError();
}

hipError_t launch_probe_chase(const uint32_t* buf, uint32_t nlines, int steps, uint32_t* sink, hipStream_t st) {
    hipLaunchKernelGGL(k_probe_chase, dim3(1), dim3(64), 0, st, buf, nlines, steps, sink);
    return hipGetLastError();
}

}  // namespace pt
