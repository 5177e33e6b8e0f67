// Plain device-to-device copy with 16-byte non-temporal loads and stores
// (gfx950): the bandwidth reference that the step kernels' HBM roofline is
// read against.  Each thread moves kCopyUnroll 16-byte words, all loads issued
// before the first store.
#include "copy.hpp"

#include <stdint.h>

namespace lbmwet {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyThreads = 256, kCopyUnroll = 4;

__global__ __launch_bounds__(kCopyThreads) void k_copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                        size_t n16) {
    const size_t base = size_t(blockIdx.x) * (kCopyThreads * kCopyUnroll) + threadIdx.x;
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int k = 0; k < kCopyUnroll; ++k) {
        const size_t i = base + size_t(k) * kCopyThreads;
        if (i < n16) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < kCopyUnroll; ++k) {
        const size_t i = base + size_t(k) * kCopyThreads;
        if (i < n16) __builtin_nontemporal_store(v[k], dst + i);
    }
}

}  // namespace

hipError_t launch_copy16(const void *src, void *dst, size_t bytes, hipStream_t st) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const size_t per_block = size_t(kCopyThreads) * kCopyUnroll;
    const size_t blocks = (n16 + per_block - 1) / per_block;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3(uint32_t(blocks)), dim3(kCopyThreads), 0, st, (const u32x4 *)src, (u32x4 *)dst,
                       n16);
    return hipGetLastError();
}

}  // namespace lbmwet
