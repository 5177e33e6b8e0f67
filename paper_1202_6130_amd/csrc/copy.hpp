// Plain device copy used as the bandwidth reference (copy.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>

namespace lbmwet {

// Copies `bytes` (a multiple of 16) from src to dst (both 16-byte aligned) on
// stream st with 16-byte non-temporal loads and stores.
hipError_t launch_copy16(const void *src, void *dst, size_t bytes, hipStream_t st);

}  // namespace lbmwet
