// Internal declarations shared by the host runtime (oasm_runtime.hip) and the
// kernels (oasm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oasm {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr uint32_t kXcds = 8;      // accelerator dies (each with its own L2)
constexpr int kMaxW32 = 8;         // 32-bit words per pattern column (256 rows)
constexpr int kMaxW64 = 4;         // 64-bit words per column in the recovery kernel
constexpr uint8_t kNoHit = 0xFF;   // hit-set byte for "distance above K"
constexpr int kMaxDevices = 64;    // device ordinals the per-device tables cover

// Filter rule bits (the values of the public OASM_RULES_* flags).
constexpr uint32_t kRulePaper = 1, kRuleAccLast = 2, kRuleEq3Ge = 4, kRuleStartOrder = 8, kRuleDisjoint = 16;
constexpr uint32_t kRuleAll = 31;

// One scan work item's text: a run of class-mapped symbols of one stream.
// The first `lookback` symbols only warm the column up (their ends belong to
// the previous item); ends are reported for the remaining symbols.
struct ChunkDesc {
    const uint8_t *sym;     // first symbol to scan (4-byte aligned)
    uint64_t abs_first;     // absolute stream position of sym[lookback]
    uint32_t scan_len;      // symbols to scan, lookback included
    uint32_t lookback;      // warm-up symbols
    uint32_t stream_local;  // step-local stream number
    uint32_t pad;
};

// A tile: up to 64*P patterns of one word count W, one slot per (lane, p).
struct TileDesc {
    uint32_t peq_off;       // offset (in uint32) of the tile's match-mask image
    uint32_t slot_off;      // offset into the slot -> pattern table
    uint32_t n_active;      // active slots (slot = lane * P + p)
    uint32_t pad;
};

// Per-pattern metadata on the device.
struct PatDesc {
    uint32_t off;           // offset of the pattern bytes
    uint16_t m;             // length
    uint16_t k;             // threshold
    uint32_t rpeq_off;      // offset (in uint64) of the reversed match masks
    uint16_t w64;           // 64-bit words of the reversed masks
    uint16_t pad;
};

// Step-local stream descriptor (index = step-local stream number).
struct StreamDesc {
    const uint8_t *sym;     // class-mapped symbols of the staging buffer
    uint64_t base_abs;      // absolute position of sym[0]
    uint64_t frontier;      // absolute end (exclusive) of the scanned bytes after this step
    uint32_t closed;        // stream closes in this step
    uint32_t slot;          // persistent stream slot
};

// A carried record: a hit end whose filter segment was still open.
struct CarryRec {
    uint64_t end_abs;
    uint32_t pattern;
    uint32_t stream_slot;
    uint32_t dist;
    uint32_t pad;
};

// Occurrence as produced by the filter.
struct OccRec {
    uint64_t start_abs;
    uint32_t pattern;
    uint32_t stream_local;
    uint32_t len;
    uint32_t k;
};

// A record count that lives in device memory: min(add + *p, cap) (p may be
// null), or 0 when *gate > gate_max (gate may be null).  Kernels after the
// scan read their sizes this way, so a whole step is queued without the host
// waiting for intermediate counts; `cap` is the capacity the buffers were
// sized for.  The gate is the scan's largest per-item record count: above the
// per-item capacity some records were dropped, the compacted arrays have
// unwritten holes, and every later kernel must do nothing (the step is run
// again with larger buffers, as it is when a count exceeds its capacity).
struct DevN {
    const uint32_t *p;
    uint32_t add;
    uint32_t cap;
    const uint32_t *gate;
    uint32_t gate_max;
};

// ------------------------------------------------------------------ launchers
// Each returns hipSuccess or the launch error.  All run on `st`.

// K0: match masks.  For every pattern, the scan image (high placement,
// wildcard rows below the pattern) into its tile, and the reversed masks
// (low placement) for the recovery kernel.
hipError_t launch_peq_build(const uint8_t *pat_bytes, const PatDesc *pats, uint32_t npat,
                            const uint32_t *pat_tile, const uint32_t *pat_slot, const TileDesc *tiles,
                            const uint32_t *tile_wp, const uint8_t *class_of, uint32_t nclass,
                            uint32_t *peq_img, uint64_t *rpeq, hipStream_t st);

// Map raw bytes to symbol classes: dst[i] = class_of[src[i]].
hipError_t launch_map_symbols(const uint8_t *src, uint8_t *dst, uint64_t n, const uint8_t *class_of,
                              hipStream_t st);

// One segment of a batched ingest: len bytes from src mapped into dst.
struct SegCopy {
    const uint8_t *src;
    uint8_t *dst;
    uint32_t len;
    uint32_t pad;
};
constexpr uint32_t kMapPiece = 4096;  // symbols of one segment piece (one workgroup)
hipError_t launch_map_segments(const SegCopy *segs, uint32_t n, const uint8_t *class_of, hipStream_t st);

// K1: the bit-parallel scan for one word-count class (W words, P patterns
// per lane).  Grid: ceil(nchunks / waves_per_block) rounded up to a multiple
// of kXcds, times ntiles, in one dimension (XCD-aware block order).
struct ScanArgs {
    const ChunkDesc *chunks;
    uint32_t nchunks;
    const TileDesc *tiles;
    uint32_t tile_first;     // first tile of this class
    uint32_t ntiles;
    const uint32_t *peq_img;
    const uint32_t *slot_pat;  // slot -> pattern id
    const PatDesc *pats;
    uint32_t nclass;
    uint32_t *item_rec;      // [nitems][cap] (slot << 24 | end offset)
    uint32_t *item_cnt;      // [nitems]
    uint32_t item_base;      // first item index of this class
    uint32_t cap;
    uint32_t *max_cnt;       // atomic max of per-item counts
    unsigned long long *wsteps;  // += pattern words advanced over reported symbols (may be null)
};
// `cut`: the word-cutoff variant (one pattern per lane, W >= 2).  `mode`:
// where the tile's match masks are read from: 0 = the image in global memory
// (through L1/L2), 1 = the image copied to LDS.  `waves_per_block`: 1..4
// wavefronts, each scanning one chunk with the block's tile.
hipError_t launch_scan(int W, int P, bool cut, const ScanArgs &a, int waves_per_block, int mode, hipStream_t st);
bool scan_variant_exists(int W, int P, bool cut);

// Ordering of the step's hit ends: carried ends first, then the scan items'
// records (key = stream_local * npat + pattern, val = own index, end), then a
// stable radix sort on the key, then a gather into the per-record arrays.
hipError_t launch_place_carry(const CarryRec *carry, uint32_t ncarry, const uint32_t *slot_to_local, uint32_t npat,
                              uint32_t *key, uint32_t *val, uint64_t *end, hipStream_t st);
// The scan items of every word-count class (items chunk-major inside a
// class, the classes one after another), for one compaction launch.
constexpr int kMaxClasses = 8;
static_assert(kMaxClasses >= kMaxW32, "one class per word count");
struct ClassItems {
    uint32_t n;                        // classes
    uint32_t tile_first[kMaxClasses];  // the class's first tile
    uint32_t ntiles[kMaxClasses];
    uint32_t item_base[kMaxClasses];   // the class's first item
};
hipError_t launch_compact_raw(const ChunkDesc *chunks, uint32_t nchunks, const TileDesc *tiles, const ClassItems &cls,
                              const uint32_t *slot_pat, const uint32_t *item_rec, const uint32_t *item_cnt,
                              const uint32_t *item_off, uint32_t cap, uint32_t base, uint32_t cap_n, uint32_t npat,
                              uint32_t *key, uint32_t *val, uint64_t *end, hipStream_t st);
size_t sort_tmp_words(uint32_t cap);
hipError_t launch_radix_sort(uint32_t *key, uint32_t *val, uint32_t *key2, uint32_t *val2, DevN n,
                             uint32_t key_bits, uint32_t *tmp, hipStream_t st, bool &result_in_second);
hipError_t launch_gather_raw(const uint32_t *skey, const uint32_t *sval, DevN n, uint32_t npat, uint32_t ncarry,
                             const uint64_t *end_in, const CarryRec *carry, const uint8_t *carry_hk, uint32_t hks,
                             uint32_t *r_pat, uint32_t *r_sl, uint64_t *r_end, uint8_t *r_flag, uint8_t *r_dist,
                             uint8_t *r_hk, hipStream_t st);

// K2: hit-set recovery at every new hit end (reverse anchored DP).
hipError_t launch_recover(const uint32_t *r_pat, const uint32_t *r_sl, const uint64_t *r_end, const uint8_t *r_flag,
                          DevN n, const PatDesc *pats, const uint64_t *rpeq, const StreamDesc *streams,
                          uint32_t nclass, uint32_t hks, uint8_t *r_hk, uint8_t *r_dist, uint32_t *err,
                          hipStream_t st);

// A long filter segment walked in parallel (see launch_filter).
struct LongDesc {
    uint64_t s0;      // the segment's first start (absolute position)
    uint32_t i, j1;   // its hit-end records
    uint32_t off;     // first slot in the per-start array
    uint32_t len;     // starts s0 .. s0 + len - 1 (0: not walked in parallel)
    uint32_t nchain;  // emissions of the walk
    uint32_t ncheck;  // checkpoints of its chain
};

// Per-step state of the parallel walk of long segments: `desc` holds
// filter_long_list_words(n.cap) descriptors; `next`, `jump[0]` and `jump[1]`
// cap_next slots each (one per start of every such segment; null when
// cap_next is 0); `*res` (two
// words) must be 0 before the launch and counts the descriptors (high 24
// bits) and the slots asked for (low 40 bits), also beyond cap_next: when
// `can_grow` is set, a segment that did not get its slots is left out (its
// occurrences missing) and the caller runs the step again with more slots;
// otherwise it is walked serially.  `*err` is set if a walk's emissions
// outnumber its segment's hit ends (impossible: each emits its own best).
struct LongWalk {
    LongDesc *desc;
    uint32_t *next;
    uint32_t *jump[2];
    uint32_t cap_next;
    uint32_t can_grow;
    unsigned long long *res;
    uint32_t *err;
};

// K3: the filter, one thread per segment of a (stream, pattern) run of up to
// 32 hit ends, a block per longer segment (its end and carry flags; one
// wavefront walks a segment of fewer than kLongParStarts starts), and for a
// longer segment the walk split into links computed in parallel (twelve more
// launches when cap_next > 0).
// `rules`: kRule* bits (0 = no filtering, only the open-segment flags).
// `long_list` holds filter_long_list_words(n.cap) words; `*long_cnt` must be
// 0 before the launch.  out_stride = K_max + 1 <= 64.
constexpr uint32_t kLongParStarts = 256;
hipError_t launch_filter(const uint32_t *r_pat, const uint32_t *r_sl, const uint64_t *r_end, const uint8_t *r_hk,
                         DevN n, uint32_t hks, const PatDesc *pats, const StreamDesc *streams,
                         uint32_t rules, uint32_t out_stride, OccRec *seg_out, uint32_t *seg_cnt,
                         uint32_t *carry_flag, uint32_t *long_list, uint32_t *long_cnt, const LongWalk &lw,
                         hipStream_t st);
size_t filter_long_list_words(uint32_t cap);

// Gather the filter output into a dense array.
hipError_t launch_compact_occ(const OccRec *seg_out, const uint32_t *seg_cnt, const uint32_t *seg_off, DevN n,
                              uint32_t out_stride, OccRec *out, uint32_t out_cap, hipStream_t st);

// Gather carried records for the next step.
hipError_t launch_compact_carry(const uint32_t *r_pat, const uint32_t *r_sl, const uint64_t *r_end,
                                const uint8_t *r_dist, const uint8_t *r_hk, uint32_t hks, const uint32_t *carry_flag,
                                const uint32_t *carry_off, const StreamDesc *streams, DevN n, CarryRec *out,
                                uint8_t *out_hk, uint32_t out_cap, hipStream_t st);

// The step's results written straight into mapped pinned host memory (the
// GPU stores over the bus; the host reads them after its one wait).  Offsets
// are byte offsets into `host`; a zero-length region is skipped.
struct PackArgs {
    const uint32_t *ctl;      // 16 control words
    DevN n;                   // hit ends of the step
    const uint32_t *r_pat, *r_sl;
    const uint64_t *r_end;
    const uint8_t *r_flag, *r_dist, *r_hk;
    uint32_t hks;
    uint32_t with_raw, with_hk;
    const OccRec *occ;
    uint32_t cap_occ;
    const CarryRec *carry;
    uint32_t cap_carry;
    uint8_t *host;
    uint64_t o_ctl, o_pat, o_sl, o_end, o_flag, o_dist, o_hk, o_occ, o_cr;
};
hipError_t launch_pack_results(const PackArgs &a, hipStream_t st);

// Exclusive prefix sum of n uint32 values; writes the total to *total.
// `tmp` must hold scan_tmp_words(n) uint32.
size_t scan_tmp_words(size_t cap);
hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, DevN n, uint32_t *total, uint32_t *tmp,
                                 hipStream_t st);

// Fill nwords uint32 with symbol classes: byte j is table[x >> 48] for x the
// splitmix64 hash of j (the autotuner's synthetic text; `table` holds 65536
// class ids, each class repeated in proportion to its wanted frequency).
hipError_t launch_fill_classes(uint32_t *p, size_t nwords, const uint8_t *table, uint64_t seed, hipStream_t st);

// Fill n uint32 with a value (graph-safe replacement for a memset).
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t st);

}  // namespace oasm
