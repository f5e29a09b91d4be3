// Internal declarations of the staging-buffer kernels that run between steps.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oasm {

// After a step a stream keeps its last `keep` symbols, moved `drop` bytes
// down to the front of its staging buffer (the ranges may overlap).  Up to
// kTailMovesPerLaunch moves travel in the kernel arguments.
struct TailMove {
    uint8_t *buf;
    uint32_t drop;
    uint32_t keep;
};
constexpr uint32_t kTailMovesPerLaunch = 128;
struct TailMoveBatch {
    TailMove m[kTailMovesPerLaunch];
};
hipError_t launch_tail_moves(const TailMoveBatch &b, uint32_t n, hipStream_t st);

}  // namespace oasm
