// dsm_probe.hip -- streaming reference kernels (copy, read, write) for the
// benchmark's bandwidth ceiling; see include/dsm_probe.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsm_probe.h"

namespace {

constexpr int kLanes = 256;

__global__ void __launch_bounds__(kLanes) k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * kLanes;
    for (size_t i = (size_t)blockIdx.x * kLanes + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ void __launch_bounds__(kLanes) k_copy_nt(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                    size_t n) {
    const size_t stride = (size_t)gridDim.x * kLanes;
    for (size_t i = (size_t)blockIdx.x * kLanes + threadIdx.x; i < n; i += stride) {
        const uint4 v = src[i];
        __builtin_nontemporal_store(v.x, &dst[i].x);
        __builtin_nontemporal_store(v.y, &dst[i].y);
        __builtin_nontemporal_store(v.z, &dst[i].z);
        __builtin_nontemporal_store(v.w, &dst[i].w);
    }
}

__global__ void __launch_bounds__(kLanes) k_read(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * kLanes;
    const size_t lane = (size_t)blockIdx.x * kLanes + threadIdx.x;
    uint4 acc = {0u, 0u, 0u, 0u};
    for (size_t i = lane; i < n; i += stride) {
        const uint4 v = src[i];
        acc.x ^= v.x;
        acc.y ^= v.y;
        acc.z ^= v.z;
        acc.w ^= v.w;
    }
    dst[lane] = acc;
}

__global__ void __launch_bounds__(kLanes) k_copy4(const unsigned* __restrict__ src, unsigned* __restrict__ dst,
                                                  size_t n) {
    const size_t stride = (size_t)gridDim.x * kLanes;
    for (size_t i = (size_t)blockIdx.x * kLanes + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(src[i], &dst[i]);
}

__global__ void __launch_bounds__(kLanes) k_write(uint4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * kLanes;
    for (size_t i = (size_t)blockIdx.x * kLanes + threadIdx.x; i < n; i += stride) {
        __builtin_nontemporal_store(1u, &dst[i].x);
        __builtin_nontemporal_store(2u, &dst[i].y);
        __builtin_nontemporal_store(3u, &dst[i].z);
        __builtin_nontemporal_store(4u, &dst[i].w);
    }
}

}  // namespace

extern "C" int dsm_probe_stream(int kind, const void* src, void* dst, size_t bytes, int blocks, void* stream) {
    if (blocks < 1 || bytes % 16 || !dst || kind < DSM_PROBE_COPY || kind > DSM_PROBE_COPY4) return -1;
    if (kind != DSM_PROBE_WRITE && !src) return -1;
    if ((uintptr_t)dst % 16 || (uintptr_t)src % 16) return -1;
    const size_t n = bytes / 16;
    hipStream_t st = (hipStream_t)stream;
    const uint4* s = (const uint4*)src;
    uint4* d = (uint4*)dst;
    switch (kind) {
        case DSM_PROBE_COPY: hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(kLanes), 0, st, s, d, n); break;
        case DSM_PROBE_COPY_NT: hipLaunchKernelGGL(k_copy_nt, dim3(blocks), dim3(kLanes), 0, st, s, d, n); break;
        case DSM_PROBE_READ: hipLaunchKernelGGL(k_read, dim3(blocks), dim3(kLanes), 0, st, s, d, n); break;
        case DSM_PROBE_COPY4:
            hipLaunchKernelGGL(k_copy4, dim3(blocks), dim3(kLanes), 0, st, (const unsigned*)src, (unsigned*)dst,
                               4 * n);
            break;
        default: hipLaunchKernelGGL(k_write, dim3(blocks), dim3(kLanes), 0, st, d, n); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
