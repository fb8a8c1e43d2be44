// psc_xcd.h -- XCD-aware placement of workgroups for the cell kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace psc {

// The dispatcher deals workgroups out to the chip's 8 XCDs round-robin
// (workgroup b to XCD b mod 8), each XCD with an L2 of its own.  xcd_map
// maps workgroup b of the grid to a logical index such that every XCD takes
// one contiguous range of them (a bijection on [0, gridDim.x)), so that the
// neighbouring cells a stencil reads sit in its own L2.  Measured on the
// field, current and sort kernels it is slower than the dispatch order
// (Weibel 256^3: 3.24 against 3.14 ms per step outside the particle kernel;
// Harris: 0.178 against 0.164 ms), so it is an ablation switch, off by
// default.
constexpr uint32_t kXcds = 8;
__host__ __device__ inline uint32_t xcd_map(uint32_t b, uint32_t G) {
    const uint32_t q = G / kXcds, rem = G % kXcds, x = b % kXcds, r = b / kXcds;
    return x * q + (x < rem ? x : rem) + r;
}
#ifndef PSC_XCD_CELLS
#define PSC_XCD_CELLS 0   // 1: contiguous ranges per XCD (ablation)
#endif
#ifndef PSC_XCD_SORT
#define PSC_XCD_SORT 0    // the same for the sort's prefix and scatter passes
#endif
__device__ __forceinline__ uint32_t xcd_block() { return PSC_XCD_CELLS ? xcd_map(blockIdx.x, gridDim.x) : blockIdx.x; }
__device__ __forceinline__ uint32_t xcd_block_sort() { return PSC_XCD_SORT ? xcd_map(blockIdx.x, gridDim.x) : blockIdx.x; }

}  // namespace psc
