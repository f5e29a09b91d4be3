// HIP kernels of oasm_gpu for CDNA4 (gfx950).
//
// The hot path of online approximate string matching (arXiv 1712.03560):
//   K0 match-mask build      (dictionary preparation)
//   (K1, the scan, is in oasm_scan.hip)
//   scatter                  scan records into (stream, pattern, end) order
//   K2 recover               the hit set at every hit end (Eq. 2): one
//                            anchored DP per end over the reversed pattern
//   K3 filter                Alg. 1 (Section 4) per (stream, pattern)
//   compactions, prefix scan, symbol mapping.
//
// Integer bit-vector work only; no matrix cores.
#include <algorithm>
#include <utility>

#include "oasm_device.h"
#include "oasm_staging.h"

namespace oasm {

// ------------------------------------------------------------------ K0
// One thread per (pattern, symbol class).
//
// Scan image (K1), high placement (full-column variants): the pattern's rows
// occupy the top m bits of its W-word column (row j at bit 32W - m + j); the
// 32W - m rows below it are wildcard rows whose mask bit is set for every
// symbol.  Started with vertical delta 0, such rows stay at delta 0 forever
// and shift a zero horizontal delta into the first pattern row, which is
// exactly the free-start boundary (the zero first row of the Less Naive
// matrix).  They also make the column sum of the vertical deltas equal to the
// last-row value.
//
// Low placement (word-cutoff variants, tile_wp bit 16): row j at bit j, so
// that the first word holds 32 pattern rows; the zero horizontal delta into
// row 0 comes from the shift itself, and the rows above the last pattern row
// (mask bits 0) do not influence the pattern rows; the scan reads the last
// row through a mask.
//
// Reversed masks (K2): row j <-> p[m-1-j], low placement, 64-bit words.
__global__ void k_peq_build(const uint8_t *__restrict__ pat_bytes, const PatDesc *__restrict__ pats, uint32_t npat,
                            const uint32_t *__restrict__ pat_tile, const uint32_t *__restrict__ pat_slot,
                            const TileDesc *__restrict__ tiles, const uint32_t *__restrict__ tile_wp,
                            const uint8_t *__restrict__ class_of, uint32_t nclass, uint32_t *__restrict__ peq_img,
                            uint64_t *__restrict__ rpeq) {
    uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t p = (uint32_t)(gid / nclass), c = (uint32_t)(gid % nclass);
    if (p >= npat) return;
    const PatDesc d = pats[p];
    const uint8_t *pb = pat_bytes + d.off;
    const int m = d.m;
    const uint32_t tile = pat_tile[p], slot = pat_slot[p];
    const uint32_t wp = tile_wp[tile];
    const int W = (int)(wp & 0xFF), P = (int)((wp >> 8) & 0xFF);
    const bool low = ((wp >> 16) & 1u) != 0;
    const int lane = (int)(slot % kWave), pp = (int)(slot / kWave);
    const int g = low ? 0 : 32 * W - m;
    const int pws = pad_pow2(P * W);
    // lane-major rows [class][lane][P*W padded] (full-column tiles), or
    // word-major [class][word][lane] (cutoff tiles, P = 1)
    uint32_t *img = peq_img + tiles[tile].peq_off;
    for (int w = 0; w < W; ++w) {
        uint32_t word = 0;
        for (int b = 0; b < 32; ++b) {
            int row = 32 * w + b - g;  // pattern row held by bit b of word w
            bool set = row < 0 ? true : (row < m && class_of[pb[row]] == c);
            word |= (uint32_t)set << b;
        }
        if (low)
            img[((size_t)c * W + w) * kWave + lane] = word;
        else
            img[((size_t)c * kWave + lane) * (size_t)pws + (size_t)pp * W + w] = word;
    }
    uint64_t *rp = rpeq + d.rpeq_off + (size_t)c * d.w64;
    for (int w = 0; w < d.w64; ++w) {
        uint64_t word = 0;
        for (int b = 0; b < 64; ++b) {
            int j = 64 * w + b;
            if (j < m && class_of[pb[m - 1 - j]] == c) word |= 1ull << b;
        }
        rp[w] = word;
    }
}

hipError_t launch_peq_build(const uint8_t *pat_bytes, const PatDesc *pats, uint32_t npat, const uint32_t *pat_tile,
                            const uint32_t *pat_slot, const TileDesc *tiles, const uint32_t *tile_wp,
                            const uint8_t *class_of, uint32_t nclass, uint32_t *peq_img, uint64_t *rpeq,
                            hipStream_t st) {
    uint64_t n = (uint64_t)npat * nclass;
    if (n == 0) return hipSuccess;
    uint32_t blocks = (uint32_t)((n + 255) / 256);
    hipLaunchKernelGGL(k_peq_build, dim3(blocks), dim3(256), 0, st, pat_bytes, pats, npat, pat_tile, pat_slot, tiles,
                       tile_wp, class_of, nclass, peq_img, rpeq);
    return hipGetLastError();
}

// ------------------------------------------------------------------ symbols
__global__ void k_map_symbols(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst, uint64_t n,
                              const uint8_t *__restrict__ class_of) {
    __shared__ uint8_t tab[256];
    if (threadIdx.x < 256) tab[threadIdx.x] = class_of[threadIdx.x];
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0) {
        // both 16-byte aligned: one uint4 load and store per 16 symbols
        const uint64_t nv = n / 16;
        const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
        uint4 *d4 = reinterpret_cast<uint4 *>(dst);
        for (uint64_t i = tid; i < nv; i += stride) {
            uint4 v = s4[i];
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t x = w[q];
                w[q] = (uint32_t)tab[x & 0xFF] | ((uint32_t)tab[(x >> 8) & 0xFF] << 8) |
                       ((uint32_t)tab[(x >> 16) & 0xFF] << 16) | ((uint32_t)tab[x >> 24] << 24);
            }
            d4[i] = make_uint4(w[0], w[1], w[2], w[3]);
        }
        for (uint64_t i = nv * 16 + tid; i < n; i += stride) dst[i] = tab[src[i]];
    } else {
        for (uint64_t i = tid; i < n; i += stride) dst[i] = tab[src[i]];
    }
}

hipError_t launch_map_symbols(const uint8_t *src, uint8_t *dst, uint64_t n, const uint8_t *class_of, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const bool vec = (((uintptr_t)src | (uintptr_t)dst) & 15) == 0;
    const uint64_t want = vec ? (n / 16 + 255) / 256 : (n + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 8192 ? (want ? want : 1) : 8192);
    hipLaunchKernelGGL(k_map_symbols, dim3(blocks), dim3(256), 0, st, src, dst, n, class_of);
    return hipGetLastError();
}

// Many segments at once (one block per segment piece of at most kMapPiece
// symbols; the host cuts longer segments into pieces): batched ingest into
// the streams' staging buffers.  Sixteen symbols per thread: four 4-byte
// words when source and destination are 4-byte aligned, else single bytes
// (a wavefront's byte accesses are 64 consecutive bytes).
__global__ void __launch_bounds__(256) k_map_segments(const SegCopy *__restrict__ segs,
                                                      const uint8_t *__restrict__ class_of) {
    static_assert(kMapPiece == 256 * 16, "sixteen symbols per thread");
    __shared__ uint8_t tab[256];
    tab[threadIdx.x] = class_of[threadIdx.x];
    __syncthreads();
    const SegCopy sc = segs[blockIdx.x];
    const uint32_t t = threadIdx.x;
    if ((((uintptr_t)sc.src | (uintptr_t)sc.dst) & 3) == 0) {
        const uint32_t nw = sc.len / 4;
        const uint32_t *s4 = reinterpret_cast<const uint32_t *>(sc.src);
        uint32_t *d4 = reinterpret_cast<uint32_t *>(sc.dst);
        uint32_t x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = t + 256u * r < nw ? s4[t + 256u * r] : 0u;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (t + 256u * r < nw)
                d4[t + 256u * r] = (uint32_t)tab[x[r] & 0xFF] | ((uint32_t)tab[(x[r] >> 8) & 0xFF] << 8) |
                                   ((uint32_t)tab[(x[r] >> 16) & 0xFF] << 16) | ((uint32_t)tab[x[r] >> 24] << 24);
        for (uint32_t i = nw * 4 + t; i < sc.len; i += 256) sc.dst[i] = tab[sc.src[i]];
        return;
    }
    uint8_t v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = t + 256u * r < sc.len ? sc.src[t + 256u * r] : 0;
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (t + 256u * r < sc.len) sc.dst[t + 256u * r] = tab[v[r]];
}

hipError_t launch_map_segments(const SegCopy *segs, uint32_t n, const uint8_t *class_of, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_map_segments, dim3(n), dim3(256), 0, st, segs, class_of);
    return hipGetLastError();
}

// ------------------------------------------------------------------ staging moves
// One workgroup per move.  The move goes forward in chunks of 4 KiB, each
// read whole into LDS before any of it is written; when the ranges overlap
// the destination lies below the source, so a chunk's writes land below
// every byte a later chunk reads.
__global__ void __launch_bounds__(256) k_staging_moves(StagingMoveBatch b) {
    __shared__ uint8_t tmp[4096];
    const StagingMove mv = b.m[blockIdx.x];
    for (uint32_t c0 = 0; c0 < mv.len; c0 += 4096) {
        const uint32_t len = min(4096u, mv.len - c0);
        for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) tmp[i] = mv.src[c0 + i];
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) mv.dst[c0 + i] = tmp[i];
        __syncthreads();
    }
}

hipError_t launch_staging_moves(const StagingMoveBatch &b, uint32_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (n > kStagingMovesPerLaunch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_staging_moves, dim3(n), dim3(256), 0, st, b);
    return hipGetLastError();
}

// ------------------------------------------------------------------ ordering
// The hit ends of a step are put in (stream, pattern, end) order without a
// dense count table: carried ends first, then every scan item's records in
// item order (items are chunk-major, so one pair's records appear chunk by
// chunk, each chunk's in end order), then a stable radix sort on the
// (stream, pattern) key alone.

// Carried ends (already in order) at the front: key, end, source index.
__global__ void k_place_carry(const CarryRec *__restrict__ carry, uint32_t n, const uint32_t *__restrict__ s2l,
                              uint32_t npat, uint32_t *__restrict__ key, uint32_t *__restrict__ val,
                              uint64_t *__restrict__ end) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const CarryRec c = carry[i];
    key[i] = s2l[c.stream_slot] * npat + c.pattern;
    val[i] = i;
    end[i] = c.end_abs;
}

// One wavefront per scan item: its records go to base + item_off[item].
__global__ void __launch_bounds__(256) k_compact_raw(const ChunkDesc *__restrict__ chunks, uint32_t nchunks,
                                                     const TileDesc *__restrict__ tiles, ClassItems cls,
                                                     const uint32_t *__restrict__ slot_pat,
                                                     const uint32_t *__restrict__ item_rec,
                                                     const uint32_t *__restrict__ item_cnt,
                                                     const uint32_t *__restrict__ item_off, uint32_t nitems,
                                                     uint32_t cap, uint32_t base, uint32_t cap_n, uint32_t npat,
                                                     uint32_t *__restrict__ key, uint32_t *__restrict__ val,
                                                     uint64_t *__restrict__ end) {
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(threadIdx.x >> 6);
    const uint32_t item = uniform(blockIdx.x * 4 + wave);
    if (item >= nitems) return;
    uint32_t c = 0;  // the item's class (wave-uniform)
    for (uint32_t k = 1; k < cls.n; ++k)
        if (item >= cls.item_base[k]) c = k;
    const uint32_t ntiles = cls.ntiles[c], local = item - cls.item_base[c];
    const uint32_t chunk = local / ntiles, tile_local = local % ntiles;
    uint32_t n = item_cnt[item];
    if (n > cap) n = cap;
    if (n == 0 || chunk >= nchunks) return;
    const ChunkDesc cd = chunks[chunk];
    const TileDesc td = tiles[cls.tile_first[c] + tile_local];
    const uint32_t *rec = item_rec + (size_t)item * cap;
    const uint32_t dst0 = base + item_off[item];
    const uint32_t kbase = cd.stream_local * npat;
    for (uint32_t i = lane; i < n; i += kWave) {
        const uint32_t r = rec[i];
        const uint32_t d = dst0 + i;
        if (d >= cap_n) break;  // over capacity: the step is run again with larger buffers
        key[d] = kbase + slot_pat[td.slot_off + (r >> 24)];
        val[d] = d;
        end[d] = cd.abs_first + (r & 0xFFFFFFu);
    }
}

hipError_t launch_place_carry(const CarryRec *carry, uint32_t ncarry, const uint32_t *slot_to_local, uint32_t npat,
                              uint32_t *key, uint32_t *val, uint64_t *end, hipStream_t st) {
    if (ncarry == 0) return hipSuccess;
    hipLaunchKernelGGL(k_place_carry, dim3((ncarry + 255) / 256), dim3(256), 0, st, carry, ncarry, slot_to_local, npat,
                       key, val, end);
    return hipGetLastError();
}

hipError_t launch_compact_raw(const ChunkDesc *chunks, uint32_t nchunks, const TileDesc *tiles, const ClassItems &cls,
                              const uint32_t *slot_pat, const uint32_t *item_rec, const uint32_t *item_cnt,
                              const uint32_t *item_off, uint32_t cap, uint32_t base, uint32_t cap_n, uint32_t npat,
                              uint32_t *key, uint32_t *val, uint64_t *end, hipStream_t st) {
    if (cls.n == 0 || cls.n > (uint32_t)kMaxClasses) return cls.n == 0 ? hipSuccess : hipErrorInvalidValue;
    const uint64_t items = cls.item_base[cls.n - 1] + (uint64_t)nchunks * cls.ntiles[cls.n - 1];
    if (items == 0) return hipSuccess;
    if (items > UINT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_compact_raw, dim3((uint32_t)((items + 3) / 4)), dim3(256), 0, st, chunks, nchunks, tiles, cls,
                       slot_pat, item_rec, item_cnt, item_off, (uint32_t)items, cap, base, cap_n, npat, key, val, end);
    return hipGetLastError();
}

// Stable LSD radix sort of (key, val) pairs, 8 bits per pass.  Pass =
// per-block digit histograms (digit-major, so one exclusive scan yields every
// block's output base per digit) and a stable scatter: each block walks its
// tile in rounds of 1024 elements; inside a wavefront the rank among equal
// digits comes from eight ballots, across the block's sixteen wavefronts
// from per-wave digit counts in LDS, turned into per-wave offsets once per
// round.  (Blocks of 1024 threads take a 2048-element tile in two rounds:
// with steps of a few thousand records a pass is one round trip of a few
// blocks, so fewer, wider rounds shorten it.)
constexpr uint32_t kSortThreads = 1024;
constexpr uint32_t kSortWaves = kSortThreads / kWave;
constexpr uint32_t kSortRounds = 2;
constexpr uint32_t kSortTile = kSortThreads * kSortRounds;

__global__ void __launch_bounds__(kSortThreads) k_sort_hist(const uint32_t *__restrict__ key, DevN dn,
                                                            uint32_t shift, uint32_t nblocks,
                                                            uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    const uint32_t n = dev_n(dn);
    const uint32_t t = threadIdx.x;
    if (t < 256) h[t] = 0;
    __syncthreads();
    const uint32_t b0 = blockIdx.x * kSortTile;
    for (uint32_t r = 0; r < kSortRounds; ++r) {
        const uint32_t i = b0 + r * kSortThreads + t;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    if (t < 256) hist[t * nblocks + blockIdx.x] = h[t];
}

__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(const uint32_t *__restrict__ kin,
                                                               const uint32_t *__restrict__ vin, DevN dn,
                                                               uint32_t shift, uint32_t nblocks,
                                                               const uint32_t *__restrict__ offs,
                                                               uint32_t *__restrict__ kout,
                                                               uint32_t *__restrict__ vout) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t tot[256];
    __shared__ uint32_t wc[kSortWaves][256];  // per-wave digit counts, then per-wave offsets
    const uint32_t n = dev_n(dn);
    const uint32_t t = threadIdx.x, wave = t >> 6;
    if (t < 256) base[t] = offs[t * nblocks + blockIdx.x];
    const uint32_t b0 = blockIdx.x * kSortTile;
    for (uint32_t r = 0; r < kSortRounds; ++r) {
        for (uint32_t x = t; x < kSortWaves * 256; x += kSortThreads) (&wc[0][0])[x] = 0;
        __syncthreads();
        const uint32_t i = b0 + r * kSortThreads + t;
        const bool valid = i < n;
        const uint32_t k = valid ? kin[i] : 0u;
        const uint32_t v = valid ? vin[i] : 0u;
        const uint32_t d = (k >> shift) & 0xFFu;
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool one = (d >> bit) & 1u;
            const uint64_t bal = __ballot(valid && one);
            same &= one ? bal : ~bal;
        }
        const uint32_t rank = mbcnt64(same);
        const uint32_t group = (uint32_t)__popcll(same);
        if (valid && rank == group - 1) wc[wave][d] = group;
        __syncthreads();
        if (t < 256) {  // digit t: the offset of each wavefront's run, and the round's total
            uint32_t run = 0;
            for (uint32_t w = 0; w < kSortWaves; ++w) {
                const uint32_t c = wc[w][t];
                wc[w][t] = run;
                run += c;
            }
            tot[t] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t o = base[d] + wc[wave][d] + rank;
            kout[o] = k;
            vout[o] = v;
        }
        __syncthreads();
        if (t < 256) base[t] += tot[t];
    }
}

size_t sort_tmp_words(uint32_t cap) {
    const uint32_t nb = (cap + kSortTile - 1) / kSortTile;
    return (size_t)256 * nb * 2 + scan_tmp_words((size_t)256 * nb) + 16;
}

// Sort the first dev_n(n) pairs; blocks are sized for n.cap (blocks past the
// count see empty tiles).  Each pass ping-pongs between the two arrays.
hipError_t launch_radix_sort(uint32_t *key, uint32_t *val, uint32_t *key2, uint32_t *val2, DevN n,
                             uint32_t key_bits, uint32_t *tmp, hipStream_t st, bool &result_in_second) {
    result_in_second = false;
    if (n.cap <= 1 || key_bits == 0) return hipSuccess;
    const uint32_t nb = (n.cap + kSortTile - 1) / kSortTile;
    uint32_t *hist = tmp;
    uint32_t *offs = tmp + (size_t)256 * nb;
    uint32_t *stmp = offs + (size_t)256 * nb;
    uint32_t *total = stmp + scan_tmp_words((size_t)256 * nb);
    uint32_t *ki = key, *vi = val, *ko = key2, *vo = val2;
    const DevN hn{nullptr, 256u * nb, 256u * nb, nullptr, 0u};
    for (uint32_t shift = 0; shift < key_bits; shift += 8) {
        hipLaunchKernelGGL(k_sort_hist, dim3(nb), dim3(kSortThreads), 0, st, ki, n, shift, nb, hist);
        hipError_t e = launch_exclusive_scan(hist, offs, hn, total, stmp, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(kSortThreads), 0, st, ki, vi, n, shift, nb, offs, ko, vo);
        std::swap(ki, ko);
        std::swap(vi, vo);
        result_in_second = !result_in_second;
    }
    return hipGetLastError();
}

// Sorted (key, source index) -> the per-record arrays of the step.
__global__ void k_gather_raw(const uint32_t *__restrict__ skey, const uint32_t *__restrict__ sval, DevN dn,
                             uint32_t npat, uint32_t ncarry, const uint64_t *__restrict__ end_in,
                             const CarryRec *__restrict__ carry, const uint8_t *__restrict__ carry_hk, uint32_t hks,
                             uint32_t *__restrict__ r_pat, uint32_t *__restrict__ r_sl, uint64_t *__restrict__ r_end,
                             uint8_t *__restrict__ r_flag, uint8_t *__restrict__ r_dist, uint8_t *__restrict__ r_hk) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dev_n(dn)) return;
    const uint32_t k = skey[i], src = sval[i];
    if (src >= dn.cap) return;  // cannot happen when the gate passed; never index past the arrays
    r_pat[i] = k % npat;
    r_sl[i] = k / npat;
    r_end[i] = end_in[src];
    const bool carried = src < ncarry;
    r_flag[i] = carried ? 1 : 0;
    if (carried) {
        r_dist[i] = (uint8_t)carry[src].dist;
        for (uint32_t q = 0; q < hks; ++q) r_hk[(size_t)i * hks + q] = carry_hk[(size_t)src * hks + q];
    }
}

hipError_t launch_gather_raw(const uint32_t *skey, const uint32_t *sval, DevN n, uint32_t npat, uint32_t ncarry,
                             const uint64_t *end_in, const CarryRec *carry, const uint8_t *carry_hk, uint32_t hks,
                             uint32_t *r_pat, uint32_t *r_sl, uint64_t *r_end, uint8_t *r_flag, uint8_t *r_dist,
                             uint8_t *r_hk, hipStream_t st) {
    if (n.cap == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_raw, dim3((n.cap + 255) / 256), dim3(256), 0, st, skey, sval, n, npat, ncarry, end_in,
                       carry, carry_hk, hks, r_pat, r_sl, r_end, r_flag, r_dist, r_hk);
    return hipGetLastError();
}

// A byte in global memory: a pointer read from a descriptor is otherwise
// generic, and generic loads make the compiler wait for every load in flight
// before it uses any of them.
typedef __attribute__((address_space(1))) const uint8_t global_u8;

// The anchored column of K2 for one hit end, NW 64-bit words per column
// (NW at least the pattern's own word count W): steps backwards from the
// hit end over `steps` text symbols, writing each length's distance <= K
// into hk and returning the least one.  Four symbols per batch; the loads
// run ahead of the column steps (the text bytes two batches ahead, the
// masks, which depend on them, one batch ahead, in two register sets used
// in turn), so that a batch waits only for loads issued a batch earlier.
// Every load is unconditional: a symbol past the last step re-reads the
// last one, and a word at or above W re-reads word W - 1.
template <int NW>
__device__ __forceinline__ int recover_column(const global_u8 *t, const uint64_t *rp, int W, int m, int K, int steps,
                                              int lmin, uint8_t *hk) {
    constexpr int kBatch = 4;
    uint64_t pv[NW], mv[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const int nb = m - 64 * w;
        pv[w] = nb >= 64 ? ~0ull : (nb <= 0 ? 0ull : ((1ull << nb) - 1));
        mv[w] = 0;
    }
    const int top_w = (m - 1) >> 6, top_b = (m - 1) & 63;
    int score = m, best = 255;
    auto load_bytes = [&](int l0, uint32_t (&cb)[kBatch]) {
#pragma unroll
        for (int b = 0; b < kBatch; ++b) cb[b] = t[-(min(l0 + b, steps) - 1)];
    };
    auto load_masks = [&](const uint32_t (&cb)[kBatch], uint64_t (&eq)[kBatch][NW]) {
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
#pragma unroll
            for (int w = 0; w < NW; ++w) eq[b][w] = rp[(size_t)cb[b] * W + min(w, W - 1)];
    };
    auto run_batch = [&](int l0, const uint64_t (&eq)[kBatch][NW]) {
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int l = l0 + b;
            const bool live = l <= steps;
            uint64_t ph[NW], mh[NW], xv[NW];
            uint64_t carry = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint64_t e = eq[b][w];
                const uint64_t x = e & pv[w];
                const uint64_t t1 = x + carry;
                const uint64_t c1 = t1 < carry;
                const uint64_t u = t1 + pv[w];
                const uint64_t c2 = u < t1;
                carry = c1 | c2;
                const uint64_t xh = (u ^ pv[w]) | e;
                xv[w] = e | mv[w];
                ph[w] = mv[w] | ~(xh | pv[w]);
                mh[w] = pv[w] & xh;
            }
            uint64_t pt = ph[0], mt = mh[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                pt = top_w == w ? ph[w] : pt;
                mt = top_w == w ? mh[w] : mt;
            }
            const int ns = score + (int)((pt >> top_b) & 1ull) - (int)((mt >> top_b) & 1ull);
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint64_t ph2 = (ph[w] << 1) | (w == 0 ? 1ull : ph[w - 1] >> 63);
                const uint64_t mh2 = (mh[w] << 1) | (w == 0 ? 0ull : mh[w - 1] >> 63);
                const uint64_t npv = mh2 | ~(xv[w] | ph2), nmv = ph2 & xv[w];
                pv[w] = live ? npv : pv[w];
                mv[w] = live ? nmv : mv[w];
            }
            score = live ? ns : score;
            if (live && l >= lmin && score <= K) {
                hk[l - (m - K)] = (uint8_t)score;
                best = score < best ? score : best;
            }
        }
    };
    uint32_t cb[kBatch];
    uint64_t eqa[kBatch][NW], eqb[kBatch][NW];
    load_bytes(1, cb);
    load_masks(cb, eqa);
    load_bytes(1 + kBatch, cb);
    for (int l0 = 1; l0 <= steps; l0 += 2 * kBatch) {
        load_masks(cb, eqb);  // batch l0 + kBatch
        load_bytes(l0 + 2 * kBatch, cb);
        run_batch(l0, eqa);
        if (l0 + kBatch > steps) break;
        load_masks(cb, eqa);  // batch l0 + 2 kBatch
        load_bytes(l0 + 3 * kBatch, cb);
        run_batch(l0 + kBatch, eqb);
    }
    return best;
}

// ------------------------------------------------------------------ K2
// One thread per new hit end e.  The reversed pattern is aligned against
// t[e], t[e-1], ... with an anchored column recurrence (a +1 horizontal delta
// enters the first row, since the DP's first row is 0, 1, 2, ...).  After l
// symbols the last row holds lev(p, t[e-l+1 .. e]), which is written for every
// l in [max(1, m-K), m+K] whose value is <= K: the hit set of Eq. 2 at e, the
// same per-start distances the paper's LEV CALC unit produces.
__global__ void __launch_bounds__(256) k_recover(const uint32_t *__restrict__ r_pat, const uint32_t *__restrict__ r_sl,
                                                 const uint64_t *__restrict__ r_end,
                                                 const uint8_t *__restrict__ r_flag, DevN dn,
                                                 const PatDesc *__restrict__ pats, const uint64_t *__restrict__ rpeq,
                                                 const StreamDesc *__restrict__ streams, uint32_t nclass, uint32_t hks,
                                                 uint8_t *__restrict__ r_hk, uint8_t *__restrict__ r_dist,
                                                 uint32_t *__restrict__ err) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dev_n(dn) || r_flag[i]) return;
    const PatDesc d = pats[r_pat[i]];
    const StreamDesc sd = streams[r_sl[i]];
    const uint64_t e = r_end[i];
    const int m = d.m, K = d.k, W = d.w64;
    const int lmax = m + K;
    const int lmin = m - K < 1 ? 1 : m - K;
    const int steps = (uint64_t)lmax <= e + 1 ? lmax : (int)(e + 1);
    // t[0] = symbol at e; the column walks backwards
    const global_u8 *t = (const global_u8 *)(sd.sym + (e - sd.base_abs));
    const uint64_t *rp = rpeq + d.rpeq_off;
    uint8_t *hk = r_hk + (size_t)i * hks;
    for (uint32_t q = 0; q < hks; ++q) hk[q] = kNoHit;

    // every lane of the wavefront steps as many words as its longest
    // pattern needs (a lane's words above its own count hold values that
    // never reach its lower words)
    uint32_t wm = (uint32_t)W;
    wm = __ballot(wm >= 4) ? 4u : __ballot(wm >= 3) ? 3u : __ballot(wm >= 2) ? 2u : 1u;
    int best = 255;
    switch (__builtin_amdgcn_readfirstlane(wm)) {
        case 1: best = recover_column<1>(t, rp, W, m, K, steps, lmin, hk); break;
        case 2: best = recover_column<2>(t, rp, W, m, K, steps, lmin, hk); break;
        case 3: best = recover_column<3>(t, rp, W, m, K, steps, lmin, hk); break;
        default: best = recover_column<4>(t, rp, W, m, K, steps, lmin, hk); break;
    }
    r_dist[i] = (uint8_t)best;
    if (best > K) atomicAdd(err, 1u);  // the scan reported a hit the recovery does not see
}

hipError_t launch_recover(const uint32_t *r_pat, const uint32_t *r_sl, const uint64_t *r_end, const uint8_t *r_flag,
                          DevN n, const PatDesc *pats, const uint64_t *rpeq, const StreamDesc *streams,
                          uint32_t nclass, uint32_t hks, uint8_t *r_hk, uint8_t *r_dist, uint32_t *err,
                          hipStream_t st) {
    if (n.cap == 0) return hipSuccess;
    hipLaunchKernelGGL(k_recover, dim3((n.cap + 255) / 256), dim3(256), 0, st, r_pat, r_sl, r_end, r_flag, n, pats, rpeq,
                       streams, nclass, hks, r_hk, r_dist, err);
    return hipGetLastError();
}

// ------------------------------------------------------------------ K3
constexpr int kMaxLevels = 64;       // K <= 63
constexpr uint32_t kShortSeg = 32;   // longer segments are walked by a wavefront (k_filter_long)
constexpr uint32_t kTile = 256;      // hit ends per LDS tile of k_filter_long

// A segment is a maximal run of one (stream, pattern)'s hit ends in which
// consecutive ends are less than m + K apart.  Alg. 1's state is empty
// between segments: any pending occurrence ends at or before the last end of
// its segment, completes there, and every hit of the next segment starts
// after it.  So segments are filtered in parallel, each from the initial
// state.
//
// Inside a segment the hit set is walked in (start, length) order, the
// order of Alg. 1's loops: for a start s the candidate ends are the hit ends
// in [s + lmin - 1, s + m + K - 1], visited in increasing order (= increasing
// length); starts with no candidate are skipped.  The completion test of
// Alg. 1 is applied lazily: the stored best completes at its own end, which
// is acted on before the first later start is examined (nothing changes at
// starts without hits).  Hit ends of one pair are distinct and increasing,
// so a start has at most 2K + 1 candidates.
//
// A segment whose last end is within m + K of the stream's scanned frontier
// may still grow: it is not filtered now but carried to the next step.
//
// `rules` bit 0 turns the filter on; the other bits select the alternative
// readings of R2 and Eq. 3 (bit values as the public OASM_RULES_* flags).
// None of them changes when a stored best completes (at its own end), so the
// segment argument holds for every combination.
//
// Alg. 1's mem rows (start, length per priority level) live in LDS, at
// `lv_s[q * lstride]` / `lv_l[q * lstride]` for level q.

// Hit ends and hit-set bytes read straight from the step's arrays.
struct RecsGlobal {
    const uint64_t *end;
    const uint8_t *hk;
    uint32_t hks;
    __device__ __forceinline__ void need(uint32_t, uint32_t) {}
    __device__ __forceinline__ uint64_t e(uint32_t j) const { return end[j]; }
    __device__ __forceinline__ uint32_t k(uint32_t j, int q) const { return hk[(size_t)j * hks + q]; }
};

// The same through a tile of kTile records in LDS, refilled by the one
// wavefront that runs the walk (every lane runs it with the same values)
// whenever a record outside the tile is needed; the tile then starts at the
// walk's lowest live record.  A wavefront's LDS accesses complete in order,
// so a wave barrier (keeping the compiler from moving them) is all the
// ordering the refill needs.
struct RecsTile {
    const uint64_t *end;
    const uint8_t *hk;
    uint32_t hks, j1;
    uint64_t *tend;  // [kTile]
    uint8_t *thk;    // [kTile * hks]
    uint32_t base, lim;
    __device__ __forceinline__ void need(uint32_t lo, uint32_t j) {
        if (j < lim && lo >= base) return;
        const uint32_t lane = threadIdx.x & 63;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();  // the tile's last readers are done
        base = lo;
        lim = min(j1, lo + kTile);
        const uint32_t cnt = lim - base;
        for (uint32_t x = lane; x < cnt; x += 64) tend[x] = end[base + x];
        for (uint32_t x = lane; x < cnt * hks; x += 64) thk[x] = hk[(size_t)base * hks + x];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __device__ __forceinline__ uint64_t e(uint32_t j) const { return tend[j - base]; }
    __device__ __forceinline__ uint32_t k(uint32_t j, int q) const { return thk[(j - base) * hks + q]; }
};

// Alg. 1 over the hit ends of one segment of pattern p in stream sl (records
// lo .. j1-1, lo at or before the first candidate of start s), from an empty
// state at start s, emitting into out.  The stored best (mem row idx) is
// also kept in registers (bs, bl), since R2 compares only with it; the
// candidates of a start are read in batches of CAND (their ends and hit-set
// bytes do not depend on the state) before R1-R3 are applied to them in
// order.  Batches pay where the records come from global memory (8); from an
// LDS tile (k_filter_long's serial walk) they only add reads.
//
// FIRST: stop at the walk's first emission, at the start where it happens
// (returned in `next`; kEndOfSegment when the walk reaches the segment's end
// instead, after emitting what it holds).  An emission leaves the state
// empty, so the walk from an empty state at the start where an emission
// happens is the rest of the walk: this is what the parallel form of long
// segments builds on.  EMIT: write mem rows and occurrences (without it only
// the emission points are computed, for which the best alone decides).
constexpr int kCandGlobal = 8, kCandTile = 1;
// a start's candidates and the batch past them fit one tile of k_filter_long
static_assert(2 * (kMaxLevels - 1) + 1 + kCandTile <= (int)kTile, "filter tile too small");
constexpr uint64_t kEndOfSegment = ~0ull;

struct WalkEnd {
    uint64_t next;  // start of the first emission (FIRST), or kEndOfSegment
    uint32_t cnt;   // occurrences written
};

template <int CAND, bool EMIT, bool FIRST, class Recs>
__device__ WalkEnd walk_from(Recs &R, uint32_t lo, uint32_t j1, uint64_t s, uint32_t p, uint32_t sl, int m, int K,
                             uint32_t rules, uint64_t *lv_s, uint32_t *lv_l, uint32_t lstride, OccRec *out) {
    const bool acc_last = (rules & kRuleAccLast) != 0, eq3_ge = (rules & kRuleEq3Ge) != 0;
    const bool start_order = (rules & kRuleStartOrder) != 0, disjoint = (rules & kRuleDisjoint) != 0;
    const int lmax = m + K;
    const int lmin = m - K < 1 ? 1 : m - K;
    const int qoff = m - K;
    if constexpr (EMIT)
        for (int q = 0; q <= K; ++q) lv_l[q * lstride] = 0;
    int idx = K;
    uint64_t bs = 0;  // mem row idx: start and length (0 = empty)
    uint32_t bl = 0;
    uint32_t cnt = 0;

    auto emit = [&](uint64_t pos) {
        if constexpr (EMIT) {
            int64_t acc = 0;
            uint64_t accepted = 0;  // levels accepted so far in this emission
            for (int j = idx; j <= K; ++j) {
                const uint32_t lj = lv_l[j * lstride];
                if (lj == 0) continue;
                const uint64_t sj = lv_s[j * lstride];
                const int64_t r = (int64_t)(pos - sj + 1);  // validation counter r(j)
                const int64_t l = (int64_t)lj;
                bool ok = j == idx || (eq3_ge ? r - acc >= l : r - acc > l);  // Eq. 3
                if (ok && disjoint && j != idx) {
                    const uint64_t je = sj + lj - 1;
                    for (uint64_t mk = accepted; mk; mk &= mk - 1) {
                        const int q = __builtin_ctzll(mk);
                        const uint64_t qs = lv_s[q * lstride], qe = qs + lv_l[q * lstride] - 1;
                        if (!(je < qs || qe < sj)) ok = false;
                    }
                }
                if (ok) {
                    OccRec o;
                    o.start_abs = sj;
                    o.pattern = p;
                    o.stream_local = sl;
                    o.len = lj;
                    o.k = (uint32_t)j;
                    out[cnt++] = o;
                    acc = acc_last ? l : acc + l;
                    accepted |= 1ull << j;
                }
            }
            for (int j = idx; j <= K; ++j) lv_l[j * lstride] = 0;
        }
        idx = K;
        bl = 0;
    };

    while (true) {
        for (; lo < j1; ++lo) {
            R.need(lo, lo);
            if (R.e(lo) + 1 >= s + lmin) break;
        }
        if (lo >= j1) break;
        const uint64_t elo = R.e(lo);
        if (elo + 1 > s + lmax) {  // no hit end reachable from s: jump
            s = elo + 1 - lmax;
            continue;
        }
        if (bl && bs + bl - 1 < s) {
            emit(bs + bl - 1);
            if constexpr (FIRST) return WalkEnd{s, cnt};
        }
        // the candidates of s: at most 2K + 1 ends, read CAND at a time
        R.need(lo, min(j1, lo + 2 * K + 1 + CAND) - 1);
        for (uint32_t j = lo; j < j1; j += CAND) {
            uint64_t ee[CAND];
            uint32_t kk[CAND];
#pragma unroll
            for (int b = 0; b < CAND; ++b) ee[b] = j + b < j1 ? R.e(j + b) : ~0ull;
#pragma unroll
            for (int b = 0; b < CAND; ++b)
                kk[b] = ee[b] != ~0ull && ee[b] + 1 <= s + lmax ? R.k(j + b, (int)(ee[b] + 1 - s) - qoff) : 0x100u;
            bool past = false;
#pragma unroll
            for (int b = 0; b < CAND; ++b) {
                if (kk[b] == 0x100u) {  // past the last candidate of s
                    past = true;
                    break;
                }
                const uint32_t k = kk[b];
                if (k == kNoHit) continue;
                const uint32_t l = (uint32_t)(ee[b] + 1 - s);
                if ((int)k < idx) {  // R1
                    idx = (int)k;
                    bs = s;
                    bl = l;
                    if constexpr (EMIT) {
                        lv_s[k * lstride] = s;
                        lv_l[k * lstride] = l;
                    }
                } else if ((int)k == idx) {  // R2 / R3: earlier end, then shorter (or: keep the first)
                    if (bl == 0 || (!start_order && (s + l < bs + bl || (s + l == bs + bl && l < bl)))) {
                        bs = s;
                        bl = l;
                        if constexpr (EMIT) {
                            lv_s[k * lstride] = s;
                            lv_l[k * lstride] = l;
                        }
                    }
                }
            }
            if (past) break;
        }
        ++s;
    }
    if (bl) emit(bs + bl - 1);
    return WalkEnd{kEndOfSegment, cnt};
}

// The whole segment i .. j1-1 from its first start; returns the number of
// occurrences written.
template <int CAND, class Recs>
__device__ uint32_t filter_walk(Recs &R, uint32_t i, uint32_t j1, uint32_t p, uint32_t sl, int m, int K,
                                uint32_t rules, uint64_t *lv_s, uint32_t *lv_l, uint32_t lstride, OccRec *out) {
    const uint64_t lmax = (uint64_t)(m + K);
    R.need(i, i);
    const uint64_t e0 = R.e(i);
    const uint64_t s0 = e0 + 1 >= lmax ? e0 + 1 - lmax : 0;
    return walk_from<CAND, true, false>(R, i, j1, s0, p, sl, m, K, rules, lv_s, lv_l, lstride, out).cnt;
}

// The records a block of k_filter can read: its 64 hit ends and the
// kShortSeg after them (a short segment that starts in the block ends
// within them, and its end test reads one record past its last).
// hit ends owned by one k_filter wavefront: few while the step's records
// fill the chip with room to spare, more when there are millions of them
// (each block stages its own and the kShortSeg after them)
constexpr uint32_t kFilterRecsFew = 8, kFilterRecsMany = 64;
constexpr uint32_t kFilterManyCap = 1u << 19;  // record capacities above this use kFilterRecsMany

// The same records through the block's window in LDS.
struct RecsWin {
    const uint64_t *tend;
    const uint8_t *thk;
    uint32_t hks, base;
    __device__ __forceinline__ void need(uint32_t, uint32_t) {}
    __device__ __forceinline__ uint64_t e(uint32_t j) const { return tend[j - base]; }
    __device__ __forceinline__ uint32_t k(uint32_t j, int q) const { return thk[(j - base) * hks + q]; }
};

// Alg. 1 over a short segment (records i .. j1-1 of the block's window) by
// the whole wavefront, every lane with the same state: at each start, lane t
// holds the start's t-th candidate (2K + 1 <= 64).  Of a start's candidates
// in order, those before the first one of priority <= idx change nothing;
// that one, when of priority idx, is the only one R2 can take (a later one
// of the same priority ends later than it, or than the stored best it did
// not replace); and R1 takes exactly the left-to-right minima below idx,
// found with ballots.  Emissions are Alg. 1's, run by every lane with lane 0
// writing the records.  The mem rows are the wave's own LDS rows (stride 1).
__device__ uint32_t wave_walk(const RecsWin &R, uint32_t i, uint32_t j1, uint32_t p, uint32_t sl, int m, int K,
                              uint32_t rules, uint64_t *lv_s, uint32_t *lv_l, OccRec *out) {
    const uint32_t lane = threadIdx.x & 63;
    const bool acc_last = (rules & kRuleAccLast) != 0, eq3_ge = (rules & kRuleEq3Ge) != 0;
    const bool start_order = (rules & kRuleStartOrder) != 0, disjoint = (rules & kRuleDisjoint) != 0;
    const uint64_t lmax = (uint64_t)(m + K), lmin = (uint64_t)(m - K < 1 ? 1 : m - K);
    const int qoff = m - K;
    if (lane <= (uint32_t)K) lv_l[lane] = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    int idx = K;
    uint64_t bs = 0;
    uint32_t bl = 0, cnt = 0;

    auto emit = [&](uint64_t pos) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        int64_t acc = 0;
        uint64_t accepted = 0;
        for (int j = idx; j <= K; ++j) {
            const uint32_t lj = lv_l[j];
            if (lj == 0) continue;
            const uint64_t sj = lv_s[j];
            const int64_t r = (int64_t)(pos - sj + 1);  // validation counter r(j)
            const int64_t l = (int64_t)lj;
            bool ok = j == idx || (eq3_ge ? r - acc >= l : r - acc > l);  // Eq. 3
            if (ok && disjoint && j != idx) {
                const uint64_t je = sj + lj - 1;
                for (uint64_t mk = accepted; mk; mk &= mk - 1) {
                    const int q = __builtin_ctzll(mk);
                    const uint64_t qs = lv_s[q], qe = qs + lv_l[q] - 1;
                    if (!(je < qs || qe < sj)) ok = false;
                }
            }
            if (ok) {
                if (lane == 0) {
                    OccRec o;
                    o.start_abs = sj;
                    o.pattern = p;
                    o.stream_local = sl;
                    o.len = lj;
                    o.k = (uint32_t)j;
                    out[cnt] = o;
                }
                ++cnt;
                acc = acc_last ? l : acc + l;
                accepted |= 1ull << j;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane >= (uint32_t)idx && lane <= (uint32_t)K) lv_l[lane] = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        idx = K;
        bl = 0;
    };

    const uint64_t e0 = R.e(i);
    uint64_t s = e0 + 1 >= lmax ? e0 + 1 - lmax : 0;
    uint32_t lo = i;
    while (true) {
        // the first record (of at most 32 left) that ends a candidate of s or later
        {
            const uint32_t j = lo + lane;
            const uint64_t b = __ballot(j < j1 && R.e(j) + 1 >= s + lmin);
            if (!b) break;
            lo += (uint32_t)__builtin_ctzll(b);
        }
        const uint64_t elo = R.e(lo);
        if (elo + 1 > s + lmax) {  // no hit end reachable from s: jump
            s = elo + 1 - lmax;
            continue;
        }
        if (bl && bs + bl - 1 < s) emit(bs + bl - 1);
        // lane t: the candidate ending at record lo + t (255: none, or no hit)
        uint32_t k = 255u, l = 0;
        {
            const uint32_t j = lo + lane;
            if (j < j1) {
                const uint64_t e = R.e(j);
                if (e + 1 <= s + lmax) {
                    l = (uint32_t)(e + 1 - s);
                    k = R.k(j, (int)l - qoff);
                }
            }
        }
        const uint64_t le = __ballot(k <= (uint32_t)idx);
        if (le) {
            const int f = __builtin_ctzll(le);
            const uint32_t kf = __builtin_amdgcn_readlane(k, f), lf = __builtin_amdgcn_readlane(l, f);
            if ((int)kf == idx && (bl == 0 || (!start_order && (s + lf < bs + bl || (s + lf == bs + bl && lf < bl))))) {
                bs = s;  // R2 / R3
                bl = lf;
                if (lane == 0) {
                    lv_s[kf] = s;
                    lv_l[kf] = lf;
                }
            }
            // R1: the left-to-right minima below idx
            uint64_t below = __ballot(k < (uint32_t)idx);
            while (below) {
                const int t = __builtin_ctzll(below);
                const uint32_t kt = __builtin_amdgcn_readlane(k, t), lt = __builtin_amdgcn_readlane(l, t);
                idx = (int)kt;
                bs = s;
                bl = lt;
                if (lane == 0) {
                    lv_s[kt] = s;
                    lv_l[kt] = lt;
                }
                below = __ballot(k < kt) & ~((2ull << t) - 1ull);
            }
        }
        ++s;
    }
    if (bl) emit(bs + bl - 1);
    return cnt;
}

size_t filter_lds_bytes(uint32_t nlevels, uint32_t hks, uint32_t recs) {
    const size_t win = recs + kShortSeg;
    return (size_t)nlevels * 64 * (sizeof(uint64_t) + sizeof(uint32_t)) + win * (8 + 4 + 4) +
           ((win * hks + 7) & ~size_t(7)) + (size_t)nlevels * (sizeof(uint64_t) + sizeof(uint32_t));
}

// A block of one wavefront owns RECS hit ends, a thread each (few, so that
// the segments one wavefront walks in turn are few and the blocks many,
// unless the step has millions of records); the thread that owns the first end of a segment finds its end and
// carry flags, and hands a segment of more than kShortSeg ends to
// k_filter_long (appended to `long_list`).  The block first copies its
// window of records (its own and the kShortSeg after them: pattern, stream,
// end, hit-set bytes) into LDS with coalesced loads, so that the scans and
// walks, which read one record after another, read LDS.  The short segments
// that need filtering are then walked one after another by the whole
// wavefront (wave_walk; a segment with 2K + 1 > 64 by its own thread).
// Dynamic LDS: the threads' mem rows ([level][thread]), the window, the
// wave's mem rows.
template <uint32_t RECS>
__global__ void __launch_bounds__(64) k_filter(const uint32_t *__restrict__ r_pat, const uint32_t *__restrict__ r_sl,
                                               const uint64_t *__restrict__ r_end, const uint8_t *__restrict__ r_hk,
                                               DevN dn, uint32_t hks, const PatDesc *__restrict__ pats,
                                               const StreamDesc *__restrict__ streams, uint32_t rules,
                                               uint32_t out_stride, OccRec *__restrict__ seg_out,
                                               uint32_t *__restrict__ seg_cnt, uint32_t *__restrict__ carry_flag,
                                               uint32_t *__restrict__ long_list, uint32_t *__restrict__ long_cnt,
                                               uint32_t nlevels) {
    extern __shared__ uint64_t lds_lv[];
    const bool do_filter = (rules & kRulePaper) != 0;
    const uint32_t n = dev_n(dn);
    constexpr uint32_t kFilterWin = RECS + kShortSeg;
    const uint32_t base = blockIdx.x * RECS;
    if (base >= n) return;  // whole block
    uint64_t *tend = lds_lv + (size_t)nlevels * 64 + ((size_t)nlevels * 64 * sizeof(uint32_t) + 7) / 8;
    uint32_t *tpat = reinterpret_cast<uint32_t *>(tend + kFilterWin);
    uint32_t *tsl = tpat + kFilterWin;
    uint8_t *thk = reinterpret_cast<uint8_t *>(tsl + kFilterWin);
    uint64_t *wlv_s = reinterpret_cast<uint64_t *>(thk + (((size_t)kFilterWin * hks + 7) & ~size_t(7)));
    uint32_t *wlv_l = reinterpret_cast<uint32_t *>(wlv_s + nlevels);
    const uint32_t cnt = min(n - base, kFilterWin);
    for (uint32_t x = threadIdx.x; x < cnt; x += 64) {
        tend[x] = r_end[base + x];
        tpat[x] = r_pat[base + x];
        tsl[x] = r_sl[base + x];
    }
    for (uint32_t x = threadIdx.x; x < cnt * hks; x += 64) thk[x] = r_hk[(size_t)base * hks + x];
    __syncthreads();
    const uint32_t w = threadIdx.x, i = base + w;
    bool walk = false;
    uint32_t j1 = i + 1, p = 0, sl = 0;
    int m = 1, K = 0;
    if (w < RECS && i < n) {
        p = tpat[w];
        sl = tsl[w];
        const uint64_t e0 = tend[w];
        const PatDesc d = pats[p];
        m = d.m;
        K = d.k;
        const uint64_t gap = (uint64_t)(m + K);
        const bool start = i == 0 || (w > 0 ? (tpat[w - 1] != p || tsl[w - 1] != sl || e0 - tend[w - 1] >= gap)
                                            : (r_pat[i - 1] != p || r_sl[i - 1] != sl || e0 - r_end[i - 1] >= gap));
        if (!start) {
            seg_cnt[i] = 0;
        } else {
            // (j1 - base < kFilterWin while the scan runs: j1 <= i + kShortSeg)
            while (j1 < n && j1 - i <= kShortSeg && tpat[j1 - base] == p && tsl[j1 - base] == sl &&
                   tend[j1 - base] - tend[j1 - 1 - base] < gap)
                ++j1;
            if (j1 - i > kShortSeg) {  // a long segment: k_filter_long takes it
                seg_cnt[i] = 0;
                long_list[atomicAdd(long_cnt, 1u)] = i;
            } else {
                const StreamDesc sd = streams[sl];
                const bool open = do_filter && !sd.closed && tend[j1 - 1 - base] + gap > sd.frontier;
                for (uint32_t j = i; j < j1; ++j) carry_flag[j] = open ? 1u : 0u;
                if (open || !do_filter) seg_cnt[i] = 0;
                else walk = true;
            }
        }
    }
    RecsWin R{tend, thk, hks, base};
    // the wavefront walks its short segments (at most RECS) one after
    // another, the lanes taking a start's candidates
    for (uint64_t wm = __ballot(walk && 2 * K + 1 <= 64); wm; wm &= wm - 1) {
        const int L = __builtin_ctzll(wm);
        const uint32_t iL = __builtin_amdgcn_readlane(i, L), jL = __builtin_amdgcn_readlane(j1, L);
        const uint32_t pL = __builtin_amdgcn_readlane(p, L), sL = __builtin_amdgcn_readlane(sl, L);
        const int mL = (int)__builtin_amdgcn_readlane((uint32_t)m, L), KL = (int)__builtin_amdgcn_readlane((uint32_t)K, L);
        const uint32_t c = wave_walk(R, iL, jL, pL, sL, mL, KL, rules, wlv_s, wlv_l, seg_out + (size_t)iL * out_stride);
        if (w == 0) seg_cnt[iL] = c;
    }
    if (walk && 2 * K + 1 > 64) {
        uint64_t *lv_s = lds_lv + threadIdx.x;
        uint32_t *lv_l = reinterpret_cast<uint32_t *>(lds_lv + (size_t)nlevels * 64) + threadIdx.x;
        seg_cnt[i] = filter_walk<kCandGlobal>(R, i, j1, p, sl, m, K, rules, lv_s, lv_l, 64,
                                              seg_out + (size_t)i * out_stride);
    }
}

// One block of kLongBlock threads per long segment (grid-stride over the
// list): the block finds the segment's end (each wavefront probes 512
// records per round) and writes its carry flags; a segment with at least
// kLongParStarts starts reserves its per-start slots for the parallel walk
// below, and a shorter one is walked by wavefront 0 alone (every lane with
// the same values) from an LDS tile.  Dynamic LDS: kTile ends, the mem rows,
// kTile * hks bytes.
constexpr uint32_t kLongBlock = 1024;

__global__ void __launch_bounds__(kLongBlock) k_filter_long(const uint32_t *__restrict__ r_pat,
                                                            const uint32_t *__restrict__ r_sl,
                                                            const uint64_t *__restrict__ r_end,
                                                            const uint8_t *__restrict__ r_hk, DevN dn, uint32_t hks,
                                                            const PatDesc *__restrict__ pats,
                                                            const StreamDesc *__restrict__ streams, uint32_t rules,
                                                            uint32_t out_stride, OccRec *__restrict__ seg_out,
                                                            uint32_t *__restrict__ seg_cnt,
                                                            uint32_t *__restrict__ carry_flag,
                                                            const uint32_t *__restrict__ long_list,
                                                            const uint32_t *__restrict__ long_cnt, uint32_t nlevels,
                                                            LongWalk lw, uint32_t desc_cap) {
    extern __shared__ uint64_t lds_tile[];
    __shared__ uint32_t s_brk;
    __shared__ unsigned long long s_res;
    const bool do_filter = (rules & kRulePaper) != 0;
    const uint32_t n = dev_n(dn);
    const uint32_t nlong = *long_cnt;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    uint64_t *tend = lds_tile;
    uint64_t *lv_s = lds_tile + kTile;
    uint32_t *lv_l = reinterpret_cast<uint32_t *>(lv_s + nlevels);
    uint8_t *thk = reinterpret_cast<uint8_t *>(lv_l + nlevels);
    for (uint32_t x = blockIdx.x; x < nlong; x += gridDim.x) {
        const uint32_t i = long_list[x];
        const uint32_t p = r_pat[i], sl = r_sl[i];
        const PatDesc d = pats[p];
        const int m = d.m, K = d.k;
        const uint64_t gap = (uint64_t)(m + K);
        // the segment's end: the first record past i that breaks the run
        constexpr int kProbe = 8;
        uint32_t j1 = n;
        for (uint32_t b = i + 1; b < n; b += nwave * 64 * kProbe) {
            if (tid == 0) s_brk = 0xFFFFFFFFu;
            __syncthreads();
            const uint32_t wb = b + wave * 64 * kProbe;
            bool brk[kProbe];
#pragma unroll
            for (int q = 0; q < kProbe; ++q) {
                const uint32_t j = wb + q * 64 + lane;
                brk[q] = j >= n || r_pat[j] != p || r_sl[j] != sl || r_end[j] - r_end[j - 1] >= gap;
            }
            uint32_t first = 0xFFFFFFFFu;
#pragma unroll
            for (int q = 0; q < kProbe; ++q) {
                const uint64_t bal = __ballot(brk[q]);
                if (bal && first == 0xFFFFFFFFu) first = wb + q * 64 + (uint32_t)__builtin_ctzll(bal);
            }
            if (lane == 0 && first != 0xFFFFFFFFu) atomicMin(&s_brk, first);
            __syncthreads();
            const uint32_t f = s_brk;
            __syncthreads();  // every thread has read it before the next round resets it
            if (f != 0xFFFFFFFFu) {
                j1 = min(f, n);
                break;
            }
        }
        const StreamDesc sd = streams[sl];
        const bool open = do_filter && !sd.closed && r_end[j1 - 1] + gap > sd.frontier;
        for (uint32_t j = i + tid; j < j1; j += blockDim.x) carry_flag[j] = open ? 1u : 0u;
        if (open || !do_filter) {
            if (tid == 0) seg_cnt[i] = 0;
            continue;
        }
        // a segment with many starts is walked in parallel by the kernels
        // below: reserve a slot per start
        const uint64_t lmax = (uint64_t)(m + K), lmin = (uint64_t)(m - K < 1 ? 1 : m - K);
        const uint64_t e0 = r_end[i];
        const uint64_t s0 = e0 + 1 >= lmax ? e0 + 1 - lmax : 0;
        const uint64_t nstarts = r_end[j1 - 1] + 2 - lmin - s0;  // s0 .. the last end's shortest start
        if (lw.desc != nullptr && nstarts >= kLongParStarts && nstarts < (1ull << 31)) {
            if (tid == 0) s_res = atomicAdd(lw.res, (1ull << 40) | nstarts);
            __syncthreads();
            const uint64_t old = s_res;
            const uint32_t di = (uint32_t)(old >> 40);
            const uint64_t off = old & ((1ull << 40) - 1);
            const bool fits = off + nstarts <= lw.cap_next && di < desc_cap;
            if (tid == 0 && di < desc_cap) {
                LongDesc ld;
                ld.s0 = s0;
                ld.i = i;
                ld.j1 = j1;
                ld.off = (uint32_t)(off < lw.cap_next ? off : lw.cap_next);  // keeps offsets ordered
                ld.len = fits ? (uint32_t)nstarts : 0u;
                ld.nchain = 0;
                ld.ncheck = 0;
                lw.desc[di] = ld;
            }
            if (fits || lw.can_grow) {  // walked below (or in the step's next run)
                if (tid == 0) seg_cnt[i] = 0;
                continue;
            }
        }
        if (wave == 0) {
            RecsTile R{r_end, r_hk, hks, j1, tend, thk, 0u, 0u};
            const uint32_t cnt =
                filter_walk<kCandTile>(R, i, j1, p, sl, m, K, rules, lv_s, lv_l, 1, seg_out + (size_t)i * out_stride);
            if (lane == 0) seg_cnt[i] = cnt;
        }
        __syncthreads();  // the next segment's tile and mem rows
    }
}

// ---- long segments walked in parallel
// From an empty state at a start s, the walk up to its first emission
// depends on s alone; after an emission the state is empty again.  So the
// walk of a segment is the chain s0 -> next(s0) -> next(next(s0)) -> ...,
// where next(s) is the start at which the walk from an empty state at s
// first emits, and each link emits what the walk from its start holds at
// the next one.
//   k_long_next    next(s) for every start of every long segment (a slot
//                  per start; slots hold slot indices, kNoNext for a walk
//                  that reaches the segment's end)
//   k_long_double  kChainLevels times: jump(x) = jump(jump(x)), so that the
//                  last level jumps 2^kChainLevels links
//   k_long_chain   one wavefront per segment follows the last level from
//                  s0 and writes every 2^kChainLevels-th link (checkpoints)
//   k_long_enum    from every checkpoint at once, the links up to the next
//                  one, each written at its rank
//   k_long_emit    every link of every chain at once re-walked, link k's
//                  occurrences written in the slot of the segment's k-th
//                  hit end (each emission writes its own best, whose ends
//                  increase, so there are no more links than hit ends),
//                  so that the compaction that follows keeps the walk's
//                  order.
constexpr uint32_t kNoNext = 0xFFFFFFFFu;
constexpr int kChainLevels = 8;

// The descriptor that owns per-start slot x: the last one whose offset is
// <= x (offsets increase with the descriptor index); `nd` > 0.
__device__ __forceinline__ uint32_t long_desc_of(const LongDesc *desc, uint32_t nd, uint32_t x) {
    uint32_t lo = 0, hi = nd;  // desc[lo].off <= x (desc[0].off == 0)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (desc[mid].off <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The first record in [lo, hi) whose end is >= v (ends increase), or hi.
__device__ __forceinline__ uint32_t first_end_at_least(const uint64_t *end, uint32_t lo, uint32_t hi, uint64_t v) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (end[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void long_counts(const LongWalk &lw, uint32_t desc_cap, uint32_t &nd, uint32_t &nslots) {
    const unsigned long long r = *lw.res;
    nd = min((uint32_t)(r >> 40), desc_cap);
    const uint64_t used = r & ((1ull << 40) - 1);
    nslots = (uint32_t)min<uint64_t>(used, lw.cap_next);
}

__global__ void __launch_bounds__(64) k_long_next(const uint32_t *__restrict__ r_pat, const uint32_t *__restrict__ r_sl,
                                                  const uint64_t *__restrict__ r_end, const uint8_t *__restrict__ r_hk,
                                                  uint32_t hks, const PatDesc *__restrict__ pats, uint32_t rules,
                                                  LongWalk lw, uint32_t desc_cap) {
    uint32_t nd, nslots;
    long_counts(lw, desc_cap, nd, nslots);
    if (nd == 0) return;
    RecsGlobal R{r_end, r_hk, hks};
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nslots; x += gridDim.x * blockDim.x) {
        const LongDesc d = lw.desc[long_desc_of(lw.desc, nd, x)];
        uint32_t nx = kNoNext;
        if (x - d.off < d.len) {  // (slots of a descriptor that did not get them stay kNoNext)
            const uint64_t s = d.s0 + (x - d.off);
            const uint32_t p = r_pat[d.i], sl = r_sl[d.i];
            const PatDesc pd = pats[p];
            const int m = pd.m, K = pd.k;
            const uint64_t lmin = (uint64_t)(m - K < 1 ? 1 : m - K);
            const uint32_t lo = first_end_at_least(r_end, d.i, d.j1, s + lmin - 1);
            if (lo < d.j1) {
                const WalkEnd w = walk_from<kCandGlobal, false, true>(R, lo, d.j1, s, p, sl, m, K, rules, nullptr,
                                                                       nullptr, 0, nullptr);
                if (w.next != kEndOfSegment) nx = d.off + (uint32_t)(w.next - d.s0);
            }
        }
        lw.next[x] = nx;
    }
}

__global__ void __launch_bounds__(256) k_long_double(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
                                                     LongWalk lw, uint32_t desc_cap) {
    uint32_t nd, nslots;
    long_counts(lw, desc_cap, nd, nslots);
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nslots; x += gridDim.x * blockDim.x) {
        const uint32_t v = src[x];
        dst[x] = v == kNoNext ? kNoNext : src[v];
    }
}

// One wavefront per descriptor (its lane 0): the checkpoints, into `ckpt`.
__global__ void __launch_bounds__(64) k_long_chain(const uint32_t *__restrict__ far, uint32_t *__restrict__ ckpt,
                                                   LongWalk lw, uint32_t desc_cap) {
    uint32_t nd, nslots;
    long_counts(lw, desc_cap, nd, nslots);
    if (threadIdx.x != 0) return;
    for (uint32_t di = blockIdx.x; di < nd; di += gridDim.x) {
        const LongDesc d = lw.desc[di];
        uint32_t c = 0;
        if (d.len != 0) {
            uint32_t node = d.off;
            while (true) {
                ckpt[d.off + c] = node;
                ++c;
                const uint32_t nx = far[node];
                if (nx == kNoNext || nx <= node || nx >= d.off + d.len) break;  // (links only move forward)
                node = nx;
            }
        }
        lw.desc[di].ncheck = c;
    }
}

// From checkpoint c of a descriptor, links c * 2^kChainLevels onwards, each
// written (as its slot index) at slot off + rank of `chain`.
__global__ void __launch_bounds__(64) k_long_enum(const uint32_t *__restrict__ next, const uint32_t *__restrict__ ckpt,
                                                  uint32_t *__restrict__ chain, LongWalk lw, uint32_t desc_cap) {
    uint32_t nd, nslots;
    long_counts(lw, desc_cap, nd, nslots);
    if (nd == 0) return;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nslots; x += gridDim.x * blockDim.x) {
        const uint32_t di = long_desc_of(lw.desc, nd, x);
        const LongDesc d = lw.desc[di];
        const uint32_t c = x - d.off;
        if (c >= d.len || c >= d.ncheck) continue;
        uint32_t node = ckpt[x];
        const uint32_t r0 = c << kChainLevels;
        for (uint32_t j = 0; j < (1u << kChainLevels); ++j) {
            if (r0 + j >= d.len) break;  // cannot happen: the links are distinct starts
            chain[d.off + r0 + j] = node;
            const uint32_t nx = next[node];
            if (nx == kNoNext || nx <= node || nx >= d.off + d.len) {
                lw.desc[di].nchain = r0 + j + 1;  // the last checkpoint's run reaches the end
                break;
            }
            node = nx;
        }
    }
}

// Every link of every chain at once; mem rows in LDS as k_filter's.
__global__ void __launch_bounds__(64) k_long_emit(const uint32_t *__restrict__ r_pat, const uint32_t *__restrict__ r_sl,
                                                  const uint64_t *__restrict__ r_end, const uint8_t *__restrict__ r_hk,
                                                  uint32_t hks, const PatDesc *__restrict__ pats, uint32_t rules,
                                                  uint32_t out_stride, OccRec *__restrict__ seg_out,
                                                  uint32_t *__restrict__ seg_cnt, const uint32_t *__restrict__ chain,
                                                  LongWalk lw, uint32_t desc_cap, uint32_t nlevels) {
    extern __shared__ uint64_t lds_lv[];
    uint32_t nd, nslots;
    long_counts(lw, desc_cap, nd, nslots);
    if (nd == 0) return;
    uint64_t *lv_s = lds_lv + threadIdx.x;
    uint32_t *lv_l = reinterpret_cast<uint32_t *>(lds_lv + (size_t)nlevels * 64) + threadIdx.x;
    RecsGlobal R{r_end, r_hk, hks};
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nslots; x += gridDim.x * blockDim.x) {
        const LongDesc d = lw.desc[long_desc_of(lw.desc, nd, x)];
        const uint32_t k = x - d.off;
        if (k >= d.len || k >= d.nchain) continue;
        if (d.i + k >= d.j1) {  // cannot happen: one best per emission
            atomicOr(lw.err, 1u);
            continue;
        }
        const uint64_t s = d.s0 + (chain[x] - d.off);
        const uint32_t p = r_pat[d.i], sl = r_sl[d.i];
        const PatDesc pd = pats[p];
        const int m = pd.m, K = pd.k;
        const uint64_t lmin = (uint64_t)(m - K < 1 ? 1 : m - K);
        const uint32_t lo = first_end_at_least(r_end, d.i, d.j1, s + lmin - 1);
        const WalkEnd w = walk_from<kCandGlobal, true, true>(R, lo, d.j1, s, p, sl, m, K, rules, lv_s, lv_l, 64,
                                                             seg_out + (size_t)(d.i + k) * out_stride);
        seg_cnt[d.i + k] = w.cnt;
    }
}

hipError_t launch_filter(const uint32_t *r_pat, const uint32_t *r_sl, const uint64_t *r_end, const uint8_t *r_hk,
                         DevN n, uint32_t hks, const PatDesc *pats, const StreamDesc *streams, uint32_t rules,
                         uint32_t out_stride, OccRec *seg_out, uint32_t *seg_cnt, uint32_t *carry_flag,
                         uint32_t *long_list, uint32_t *long_cnt, const LongWalk &lw, hipStream_t st) {
    if (n.cap == 0) return hipSuccess;
    const uint32_t nlevels = out_stride;  // K_max + 1 levels
    if (nlevels > (uint32_t)kMaxLevels) return hipErrorInvalidValue;
    const size_t sh = (size_t)nlevels * 64 * (sizeof(uint64_t) + sizeof(uint32_t));
    if (n.cap > kFilterManyCap) {
        hipLaunchKernelGGL(k_filter<kFilterRecsMany>, dim3((n.cap + kFilterRecsMany - 1) / kFilterRecsMany), dim3(64),
                           filter_lds_bytes(nlevels, hks, kFilterRecsMany), st, r_pat, r_sl, r_end, r_hk, n, hks, pats,
                           streams, rules, out_stride, seg_out, seg_cnt, carry_flag, long_list, long_cnt, nlevels);
    } else {
        hipLaunchKernelGGL(k_filter<kFilterRecsFew>, dim3((n.cap + kFilterRecsFew - 1) / kFilterRecsFew), dim3(64),
                           filter_lds_bytes(nlevels, hks, kFilterRecsFew), st, r_pat, r_sl, r_end, r_hk, n, hks, pats,
                           streams, rules, out_stride, seg_out, seg_cnt, carry_flag, long_list, long_cnt, nlevels);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // at most one long segment per kShortSeg + 1 hit ends; a fixed grid that
    // reads the count on the device (nothing to do in most steps)
    const uint32_t maxlong = n.cap / (kShortSeg + 1) + 1;
    const uint32_t grid = maxlong < 512 ? maxlong : 512;
    const size_t shl = kTile * sizeof(uint64_t) + (size_t)nlevels * (sizeof(uint64_t) + sizeof(uint32_t)) +
                       (size_t)kTile * hks;
    const uint32_t desc_cap = (uint32_t)filter_long_list_words(n.cap);
    hipLaunchKernelGGL(k_filter_long, dim3(grid), dim3(kLongBlock), shl, st, r_pat, r_sl, r_end, r_hk, n, hks, pats,
                       streams, rules, out_stride, seg_out, seg_cnt, carry_flag, long_list, long_cnt, nlevels, lw,
                       desc_cap);
    e = hipGetLastError();
    if (e != hipSuccess || lw.desc == nullptr || lw.cap_next == 0) return e;
    // the parallel walk: fixed grids, sized by the slot capacity, that read
    // the counts on the device (nothing to do in most steps)
    const uint32_t gs = (uint32_t)std::min<uint64_t>((lw.cap_next + 63) / 64, 4096);
    const uint32_t gd = (uint32_t)std::min<uint64_t>((lw.cap_next + 255) / 256, 2048);
    hipLaunchKernelGGL(k_long_next, dim3(gs), dim3(64), 0, st, r_pat, r_sl, r_end, r_hk, hks, pats, rules, lw,
                       desc_cap);
    e = hipGetLastError();
    // jump levels alternate between the two other slot arrays; the last one
    // (2^kChainLevels links) ends in jump[1] (kChainLevels is even)
    static_assert(kChainLevels % 2 == 0, "the last level must land in jump[1]");
    const uint32_t *src = lw.next;
    for (int lv = 0; lv < kChainLevels && e == hipSuccess; ++lv) {
        uint32_t *dst = lw.jump[lv & 1];
        hipLaunchKernelGGL(k_long_double, dim3(gd), dim3(256), 0, st, src, dst, lw, desc_cap);
        e = hipGetLastError();
        src = dst;
    }
    if (e != hipSuccess) return e;
    // checkpoints into jump[0] (its level is no longer needed), the links
    // by rank into jump[1] (read by k_long_chain only)
    hipLaunchKernelGGL(k_long_chain, dim3(grid), dim3(64), 0, st, lw.jump[1], lw.jump[0], lw, desc_cap);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_long_enum, dim3(gs), dim3(64), 0, st, lw.next, lw.jump[0], lw.jump[1], lw, desc_cap);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_long_emit, dim3(gs), dim3(64), sh, st, r_pat, r_sl, r_end, r_hk, hks, pats, rules,
                       out_stride, seg_out, seg_cnt, lw.jump[1], lw, desc_cap, nlevels);
    return hipGetLastError();
}

size_t filter_long_list_words(uint32_t cap) { return cap / (kShortSeg + 1) + 1; }

// Occurrences of every segment into one dense array.  A thread copies its
// own segment's records; a segment with more than 64 of them is copied by
// the whole wavefront.
__global__ void k_compact_occ(const OccRec *__restrict__ seg_out, const uint32_t *__restrict__ seg_cnt,
                              const uint32_t *__restrict__ seg_off, DevN dn, uint32_t stride,
                              OccRec *__restrict__ out, uint32_t out_cap) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = dev_n(dn);
    const uint32_t c = i < n ? seg_cnt[i] : 0u;
    const uint32_t lane = lane_id();
    const bool big = c > 64;
    if (!big) {
        for (uint32_t q = 0; q < c && seg_off[i] + q < out_cap; ++q)
            out[seg_off[i] + q] = seg_out[(size_t)i * stride + q];
    }
    for (uint64_t bal = __ballot(big); bal; bal &= bal - 1) {
        const uint32_t src = (uint32_t)__builtin_ctzll(bal);
        const uint32_t si = __shfl(i, src, 64), sc = __shfl(c, src, 64);
        const uint32_t so = seg_off[si];
        for (uint32_t q = lane; q < sc && so + q < out_cap; q += 64) out[so + q] = seg_out[(size_t)si * stride + q];
    }
}

hipError_t launch_compact_occ(const OccRec *seg_out, const uint32_t *seg_cnt, const uint32_t *seg_off, DevN n,
                              uint32_t out_stride, OccRec *out, uint32_t out_cap, hipStream_t st) {
    if (n.cap == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact_occ, dim3((n.cap + 255) / 256), dim3(256), 0, st, seg_out, seg_cnt, seg_off, n,
                       out_stride, out, out_cap);
    return hipGetLastError();
}

__global__ void k_compact_carry(const uint32_t *__restrict__ r_pat, const uint32_t *__restrict__ r_sl,
                                const uint64_t *__restrict__ r_end, const uint8_t *__restrict__ r_dist,
                                const uint8_t *__restrict__ r_hk, uint32_t hks,
                                const uint32_t *__restrict__ carry_flag, const uint32_t *__restrict__ carry_off,
                                const StreamDesc *__restrict__ streams, DevN dn, CarryRec *__restrict__ out,
                                uint8_t *__restrict__ out_hk, uint32_t out_cap) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dev_n(dn) || !carry_flag[i]) return;
    const uint32_t o = carry_off[i];
    if (o >= out_cap) return;
    CarryRec c;
    c.end_abs = r_end[i];
    c.pattern = r_pat[i];
    c.stream_slot = streams[r_sl[i]].slot;
    c.dist = r_dist[i];
    c.pad = 0;
    out[o] = c;
    for (uint32_t q = 0; q < hks; ++q) out_hk[(size_t)o * hks + q] = r_hk[(size_t)i * hks + q];
}

hipError_t launch_compact_carry(const uint32_t *r_pat, const uint32_t *r_sl, const uint64_t *r_end,
                                const uint8_t *r_dist, const uint8_t *r_hk, uint32_t hks, const uint32_t *carry_flag,
                                const uint32_t *carry_off, const StreamDesc *streams, DevN n, CarryRec *out,
                                uint8_t *out_hk, uint32_t out_cap, hipStream_t st) {
    if (n.cap == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact_carry, dim3((n.cap + 255) / 256), dim3(256), 0, st, r_pat, r_sl, r_end, r_dist,
                       r_hk, hks, carry_flag, carry_off, streams, n, out, out_hk, out_cap);
    return hipGetLastError();
}

// ------------------------------------------------------------------ results
// Grid-stride copies of the step's results into mapped host memory: control
// words, the hit-end arrays (and hit-set bytes), occurrences, carried ends.
__global__ void __launch_bounds__(256) k_pack_results(PackArgs a) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t n = dev_n(a.n);
    const uint32_t nocc = min(a.ctl[2], a.cap_occ);
    const uint32_t ncar = min(a.ctl[3], a.cap_carry);
    if (tid < 16) reinterpret_cast<uint32_t *>(a.host + a.o_ctl)[tid] = a.ctl[tid];
    if (a.with_raw) {
        uint32_t *hp = reinterpret_cast<uint32_t *>(a.host + a.o_pat);
        uint32_t *hs = reinterpret_cast<uint32_t *>(a.host + a.o_sl);
        uint64_t *he = reinterpret_cast<uint64_t *>(a.host + a.o_end);
        uint8_t *hf = a.host + a.o_flag, *hd = a.host + a.o_dist;
        for (uint32_t i = tid; i < n; i += stride) {
            hp[i] = a.r_pat[i];
            hs[i] = a.r_sl[i];
            he[i] = a.r_end[i];
            hf[i] = a.r_flag[i];
            hd[i] = a.r_dist[i];
        }
    }
    if (a.with_hk) {
        const uint64_t nb = (uint64_t)n * a.hks;
        for (uint64_t i = tid; i < nb; i += stride) a.host[a.o_hk + i] = a.r_hk[i];
    }
    uint64_t *ho = reinterpret_cast<uint64_t *>(a.host + a.o_occ);
    const uint64_t *so = reinterpret_cast<const uint64_t *>(a.occ);
    for (uint64_t i = tid; i < (uint64_t)nocc * 3; i += stride) ho[i] = so[i];
    uint64_t *hc = reinterpret_cast<uint64_t *>(a.host + a.o_cr);
    const uint64_t *sc = reinterpret_cast<const uint64_t *>(a.carry);
    for (uint64_t i = tid; i < (uint64_t)ncar * 3; i += stride) hc[i] = sc[i];
}

hipError_t launch_pack_results(const PackArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_results, dim3(512), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan
// Exclusive prefix sum in three passes: per-block sums, a single-block scan
// of the block sums, and per-block scans offset by the scanned sums.
constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanPer = 8;
constexpr uint32_t kScanTile = kScanThreads * kScanPer;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(v, off, kWave);
        if (lane >= (uint32_t)off) v += t;
    }
    return v;
}

// block-wide exclusive scan of one value per thread; returns the block total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t &excl) {
    __shared__ uint32_t wsum[kScanThreads / kWave];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    uint32_t woff = 0, total = 0;
    for (uint32_t w = 0; w < kScanThreads / kWave; ++w) {
        const uint32_t s = wsum[w];
        if (w < wave) woff += s;
        total += s;
    }
    __syncthreads();
    excl = woff + incl - v;
    return total;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const uint32_t *__restrict__ in, DevN dn,
                                                              uint32_t *__restrict__ sums) {
    const size_t n = dev_n(dn);
    const size_t base = (size_t)blockIdx.x * kScanTile;
    uint32_t v = 0;
#pragma unroll
    for (uint32_t q = 0; q < kScanPer; ++q) {
        const size_t i = base + (size_t)q * kScanThreads + threadIdx.x;
        if (i < n) v += in[i];
    }
    uint32_t excl;
    const uint32_t total = block_excl_scan(v, excl);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(uint32_t *__restrict__ sums, uint32_t nb,
                                                            uint32_t *__restrict__ total) {
    uint32_t carry = 0;
    for (uint32_t b = 0; b < nb; b += kScanThreads) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t v = i < nb ? sums[i] : 0u;
        uint32_t excl;
        const uint32_t t = block_excl_scan(v, excl);
        if (i < nb) sums[i] = carry + excl;
        carry += t;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                             DevN dn, const uint32_t *__restrict__ sums) {
    const size_t n = dev_n(dn);
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t q = 0; q < kScanPer; ++q) {
        v[q] = base + q < n ? in[base + q] : 0u;
        s += v[q];
    }
    uint32_t excl;
    block_excl_scan(s, excl);
    uint32_t run = sums[blockIdx.x] + excl;
#pragma unroll
    for (uint32_t q = 0; q < kScanPer; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
}

// Small counts (up to kSmallMax): the whole exclusive scan in one block of
// 1024 threads, in rounds of kSmallRound values: coalesced loads into LDS,
// each thread's sum of its kSmallPer consecutive values, the block's scan,
// the values' prefixes written back through LDS (coalesced), and the round's
// total carried into the next.
constexpr uint32_t kSmallThreads = 1024, kSmallPer = 8, kSmallRound = kSmallThreads * kSmallPer;
constexpr uint32_t kSmallMax = 16 * kSmallRound;  // larger arrays take the three-pass scan

// LDS index of value i of a round, padded so that the threads' runs of
// kSmallPer values start in different banks.
__device__ __forceinline__ uint32_t small_pad(uint32_t i) { return i + (i >> 5); }

__global__ void __launch_bounds__(kSmallThreads) k_scan_small(const uint32_t *__restrict__ in,
                                                              uint32_t *__restrict__ out, DevN dn,
                                                              uint32_t *__restrict__ total) {
    __shared__ uint32_t buf[kSmallRound + kSmallRound / 32];
    __shared__ uint32_t wsum[kSmallThreads / kWave];
    const uint32_t n = dev_n(dn);
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t carry = 0;  // the sum of the earlier rounds
    for (uint32_t r0 = 0; r0 < n; r0 += kSmallRound) {
        const uint32_t cnt = min(n - r0, kSmallRound);
        // coalesced loads; each thread then owns kSmallPer consecutive values
        for (uint32_t i = threadIdx.x; i < kSmallRound; i += kSmallThreads)
            buf[small_pad(i)] = i < cnt ? in[r0 + i] : 0u;
        __syncthreads();
        const uint32_t b = threadIdx.x * kSmallPer;
        uint32_t s = 0;
#pragma unroll
        for (uint32_t k = 0; k < kSmallPer; ++k) s += buf[small_pad(b + k)];
        const uint32_t incl = wave_incl_scan(s);
        if (lane == kWave - 1) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (uint32_t w = 0; w < kSmallThreads / kWave; ++w) {
            const uint32_t x = wsum[w];
            if (w < wave) before += x;
            all += x;
        }
        uint32_t run = carry + before + incl - s;
#pragma unroll
        for (uint32_t k = 0; k < kSmallPer; ++k) {
            const uint32_t v = buf[small_pad(b + k)];
            buf[small_pad(b + k)] = run;
            run += v;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += kSmallThreads) out[r0 + i] = buf[small_pad(i)];
        carry += all;
        __syncthreads();  // buf and wsum are reused by the next round
    }
    if (threadIdx.x == 0) *total = carry;
}

size_t scan_tmp_words(size_t cap) { return (cap + kScanTile - 1) / kScanTile + 1; }

// Exclusive scan of the first dev_n(n) values (blocks sized for n.cap).
hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, DevN n, uint32_t *total, uint32_t *tmp,
                                 hipStream_t st) {
    if (n.cap <= kSmallMax) {  // one launch instead of three
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kSmallThreads), 0, st, in, out, n, total);
        return hipGetLastError();
    }
    const uint32_t nb = (uint32_t)((n.cap + kScanTile - 1) / kScanTile);
    if (nb > 0) hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, st, tmp, nb, total);
    if (nb > 0) hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, st, in, out, n, tmp);
    return hipGetLastError();
}

__global__ void k_fill_classes(uint32_t *__restrict__ p, size_t nwords, const uint8_t *__restrict__ table,
                               uint64_t seed) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) {
        uint32_t w = 0;
        for (int b = 0; b < 4; ++b) {  // splitmix64 of the byte index
            uint64_t z = seed + (4 * i + b + 1) * 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            w |= (uint32_t)table[z >> 48] << (8 * b);
        }
        p[i] = w;
    }
}

hipError_t launch_fill_classes(uint32_t *p, size_t nwords, const uint8_t *table, uint64_t seed, hipStream_t st) {
    if (nwords == 0) return hipSuccess;
    const size_t want = (nwords + 255) / 256;
    hipLaunchKernelGGL(k_fill_classes, dim3((uint32_t)(want < 8192 ? want : 8192)), dim3(256), 0, st, p, nwords,
                       table, seed);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const size_t want = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)(want < 8192 ? want : 8192)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

}  // namespace oasm
