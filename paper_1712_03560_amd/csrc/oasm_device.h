// Device helpers shared by the kernel sources of oasm_gpu (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "oasm_internal.h"

namespace oasm {

typedef __attribute__((address_space(4))) const uint32_t const_u32;

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint32_t dev_n(const DevN &d) {
    if (d.gate && *d.gate > d.gate_max) return 0u;
    const uint32_t v = d.add + (d.p ? *d.p : 0u);
    return v < d.cap ? v : d.cap;
}

// number of set bits of `mask` below this lane
__device__ __forceinline__ uint32_t mbcnt64(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Per-lane row of a tile image: P*W words padded to a power of two so that
// one aligned LDS (or global) vector read fetches it.
__host__ __device__ constexpr int pad_pow2(int x) { return x <= 1 ? 1 : x <= 2 ? 2 : x <= 4 ? 4 : 8; }

}  // namespace oasm
