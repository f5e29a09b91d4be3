// Internal declarations of the staging-buffer kernels that run between steps.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oasm {

// A move of len symbols from src to dst inside the staging memory: the
// look-back tail of a stream moved to the front of its buffer after a step
// (dst below src, the ranges may overlap), or a stream's symbols copied into
// its new, larger buffer (disjoint ranges).  dst above an overlapping src is
// not allowed.  Up to kStagingMovesPerLaunch moves travel in the kernel
// arguments.
struct StagingMove {
    const uint8_t *src;
    uint8_t *dst;
    uint32_t len;
    uint32_t pad;
};
constexpr uint32_t kStagingMovesPerLaunch = 128;
struct StagingMoveBatch {
    StagingMove m[kStagingMovesPerLaunch];
};
hipError_t launch_staging_moves(const StagingMoveBatch &b, uint32_t n, hipStream_t st);

}  // namespace oasm
