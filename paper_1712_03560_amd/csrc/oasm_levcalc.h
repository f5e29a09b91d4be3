// Internal declarations of the dense per-start kernel (K4, LEV CALC).
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "oasm_internal.h"

namespace oasm {

// One launch covers the patterns pat_ids[0 .. npat) of one word count W
// (W = ceil(m / 32) for each of them).  For pattern q = pat_ids[x] the output
// block starts at byte n * out_unit[q] of `out`; inside it, start i's
// 2K_q + 1 distances are at i * (2K_q + 1).
struct LevcalcArgs {
    const uint8_t *text;      // raw stream bytes (device)
    uint64_t n;               // bytes = starts
    const uint32_t *pat_ids;  // patterns of this launch
    uint32_t npat;
    const PatDesc *pats;
    const uint8_t *pat_bytes;
    const uint64_t *out_unit; // per pattern: sum over earlier patterns of (2K + 1)
    uint8_t *out;
};

hipError_t launch_levcalc(int W, const LevcalcArgs &a, hipStream_t st);

// The allocation-free variant's tables: a fixed device array per GPU, held
// until the process ends, of kLcNoallocMaxPatterns * 12 bytes: the per-pattern
// output units (uint64) first, then the pattern ids grouped by word count
// (uint32).
constexpr uint32_t kLcNoallocMaxPatterns = 65536;
constexpr size_t kLcScratchBytes = (size_t)kLcNoallocMaxPatterns * (sizeof(uint64_t) + sizeof(uint32_t));

// The device address of that array on `device`, which must be the current
// device (looked up once per device, then cached).
hipError_t levcalc_scratch(int device, uint8_t **out);

// Build both tables for patterns 0 .. npat-1 (npat <= kLcNoallocMaxPatterns)
// into `scratch`: unit[q] = sum over p < q of (2K_p + 1); ids = the pattern
// numbers ordered by word count ceil(m / 32), ascending numbers inside a
// word count (the order oasm_levcalc's host-built tables use).
hipError_t launch_levcalc_tables(const PatDesc *pats, uint32_t npat, uint8_t *scratch, hipStream_t st);

}  // namespace oasm
