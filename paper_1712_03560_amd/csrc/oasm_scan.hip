// K1, the hot kernel of oasm_gpu for CDNA4 (gfx950): the bit-parallel scan
// that finds every hit end, min over starts of lev(p, t[s..e]) <= K (Section
// 5.1 "Less Naive"; column recurrence after Myers 1999), for a dictionary
// tiled over wavefront lanes and many streams cut into chunks.
//
// Integer bit-vector work only; no matrix cores.
#include <mutex>

#include "oasm_device.h"

namespace oasm {

// ------------------------------------------------------------------ K1
// Truth-table operands of v_bitop3_b32: the result bit for inputs (a, b, c)
// is bit (a*4 + b*2 + c) of the immediate.
constexpr uint32_t TA = 0xF0, TB = 0xCC, TC = 0xAA;
#define BITOP3(a, b, c, expr) __builtin_amdgcn_bitop3_b32((a), (b), (c), (uint32_t)((expr) & 0xFF))

// Measured on MI355X (independent chains, full occupancy): v_and, v_xor,
// v_add_u32 and v_bitop3 sustain 52-62 T lane-ops/s; shifts, v_or3,
// v_bcnt, v_lshl_or, v_add3, v_alignbit and the carry adds 34-38 T.  The
// column step is written with the fast ones only where it can be.
//
// x + x (= x << 1) as v_add_u32 (the compiler would turn it into a shift).
__device__ __forceinline__ uint32_t add_self(uint32_t x) {
    uint32_t r;
    asm("v_add_u32 %0, %1, %1" : "=v"(r) : "v"(x));
    return r;
}

// popcount(x) + acc as one v_bcnt_u32_b32 (register-only ALU instruction).
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// One column step of the bit-parallel edit-distance recurrence for a
// W-word column (search mode: a zero horizontal delta enters the first row).
// pv: rows whose vertical delta is +1; cm: the complement of the rows whose
// vertical delta is -1 (kept complemented because every use of it is inside
// three-input logic, which absorbs the complement for free, and its
// popcount then feeds the hit test without a NOT); eq: rows whose pattern
// symbol equals the text symbol.  With mv = ~cm and u = (eq & pv) + pv
// (carry through all W words) the horizontal deltas are
//   ph = mv | ~(u | pv | eq),    mh = pv & (eq | ~u)
// and, with ph2 / mh2 the deltas shifted one row down (across words),
//   pv' = mh2 | ~(eq | mv | ph2),    mv' = ph2 & (eq | mv).
// (Myers 1999 / Hyyro's formulation, rewritten for three-input logic: ten
// VALU instructions per 32-bit word on gfx950, all of the fast kind in the
// first word: and, add, three bitop3, two self-adds for the shifts, bitop3,
// or, bitop3.  Nine are possible with a shift-or and a three-way or, but
// those issue at about two thirds of the rate.)
//
// column_step_n<N> advances only the first N words of a W-word column (the
// word cutoff below); column_step<W> advances all of them.
// (hi:lo) as one 64-bit value, and back
__device__ __forceinline__ uint64_t pack64(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }

// a + b on 64 bits as one v_lshl_add_u64 (about twice the rate per 32-bit
// word of a carry-add pair)
__device__ __forceinline__ uint64_t add64(uint64_t a, uint64_t b) {
    uint64_t r;
    asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// a << 1 on 64 bits as one v_lshl_add_u64
__device__ __forceinline__ uint64_t shl1_64(uint64_t a) {
    uint64_t r;
    asm("v_lshl_add_u64 %0, %1, 1, 0" : "=v"(r) : "v"(a));
    return r;
}

template <int N, int W>
__device__ __forceinline__ void column_step_n(uint32_t (&pv)[W], uint32_t (&cm)[W], const uint32_t *eq) {
    static_assert(N >= 1 && N <= W, "words");
    if constexpr (N == 2) {
        // two words as one 64-bit column: the carry add and the one-row
        // shifts are single 64-bit instructions
        const uint64_t u = add64(pack64(eq[0] & pv[0], eq[1] & pv[1]), pack64(pv[0], pv[1]));
        const uint32_t uw[2] = {(uint32_t)u, (uint32_t)(u >> 32)};
        uint32_t ph[2], mh[2];
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const uint32_t o = BITOP3(uw[w], pv[w], eq[w], TA | TB | TC);
            ph[w] = BITOP3(cm[w], o, 0u, ~(TA & TB));
            mh[w] = BITOP3(pv[w], eq[w], uw[w], TA & (TB | ~TC));
        }
        const uint64_t ph2 = shl1_64(pack64(ph[0], ph[1])), mh2 = shl1_64(pack64(mh[0], mh[1]));
        const uint32_t p2[2] = {(uint32_t)ph2, (uint32_t)(ph2 >> 32)};
        const uint32_t m2[2] = {(uint32_t)mh2, (uint32_t)(mh2 >> 32)};
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const uint32_t t = BITOP3(eq[w], cm[w], p2[w], ~(TA | ~TB | TC));
            const uint32_t ncm = BITOP3(p2[w], eq[w], cm[w], ~(TA & (TB | ~TC)));
            pv[w] = m2[w] | t;
            cm[w] = ncm;
        }
        return;
    }
    uint32_t ph[N], mh[N];
    uint32_t carry = 0;
#pragma unroll
    for (int w = 0; w < N; ++w) {
        const uint32_t x = eq[w] & pv[w];
        uint32_t u;
        if (N == 1) {
            u = x + pv[w];
        } else {
            // one add-with-carry per word (v_add_co / v_addc_co)
            u = __builtin_addc(x, pv[w], carry, &carry);
        }
        const uint32_t o = BITOP3(u, pv[w], eq[w], TA | TB | TC);
        ph[w] = BITOP3(cm[w], o, 0u, ~(TA & TB));           // ~cm | ~o
        mh[w] = BITOP3(pv[w], eq[w], u, TA & (TB | ~TC));   // pv & (eq | ~u)
    }
    uint32_t npv[N], ncm[N];
#pragma unroll
    for (int w = 0; w < N; ++w) {
        const uint32_t ph2 = w == 0 ? add_self(ph[0]) : __builtin_amdgcn_alignbit(ph[w], ph[w - 1], 31);
        const uint32_t t = BITOP3(eq[w], cm[w], ph2, ~(TA | ~TB | TC));  // ~(eq | ~cm | ph2)
        npv[w] = (w == 0 ? add_self(mh[0]) : __builtin_amdgcn_alignbit(mh[w], mh[w - 1], 31)) | t;
        ncm[w] = BITOP3(ph2, eq[w], cm[w], ~(TA & (TB | ~TC)));        // ~(ph2 & (eq | ~cm))
    }
#pragma unroll
    for (int w = 0; w < N; ++w) {
        pv[w] = npv[w];
        cm[w] = ncm[w];
    }
}

template <int W>
__device__ __forceinline__ void column_step(uint32_t (&pv)[W], uint32_t (&cm)[W], const uint32_t *eq) {
    column_step_n<W, W>(pv, cm, eq);
}

// Last-row value D = popcount(pv) - popcount(mv) (the column sum of the
// vertical deltas; wildcard rows contribute 0) = popcount(pv) + popcount(cm)
// - 32W.  With bias = -32W - bound - 1 the result's sign bit is set exactly
// when D <= bound.
template <int W>
__device__ __forceinline__ int32_t le_bound(const uint32_t (&pv)[W], const uint32_t (&cm)[W], uint32_t bias) {
    uint32_t d = bias;
#pragma unroll
    for (int w = 0; w < W; ++w) d = bcnt_acc(cm[w], d);
#pragma unroll
    for (int w = 0; w < W; ++w) d = bcnt_acc(pv[w], d);
    return (int32_t)d;
}

// The same with the last word read through `mask` (low placement: the rows
// above the last pattern row are excluded); `bias` then holds
// -32(W-1) - popcount(mask) - bound - 1.
template <int W>
__device__ __forceinline__ int32_t le_bound_masked(const uint32_t (&pv)[W], const uint32_t (&cm)[W], uint32_t bias,
                                                   uint32_t mask) {
    uint32_t d = bias;
#pragma unroll
    for (int w = 0; w < W - 1; ++w) d = bcnt_acc(cm[w], d);
#pragma unroll
    for (int w = 0; w < W - 1; ++w) d = bcnt_acc(pv[w], d);
    d = bcnt_acc(cm[W - 1] & mask, d);
    d = bcnt_acc(pv[W - 1] & mask, d);
    return (int32_t)d;
}

// Per-lane row of a tile image: P*W words padded to a power of two so that
// one aligned LDS (or global) vector read fetches it.
template <int N>
struct alignas(N * 4 < 16 ? N * 4 : 16) Words {
    uint32_t v[N];
};

constexpr int kScanGroup = 4;  // text symbols per scalar load and per hit check

// Byte offset of symbol s's row in an image of `bytes` bytes per class, kept
// opaque so that it stays a scalar: the per-lane address is then one
// full-rate v_add_u32 (left to itself the compiler folds the scaling into a
// half-rate shift-add on the vector side).
__device__ __forceinline__ uint32_t row_off(uint32_t cur, int s, uint32_t bytes) {
    uint32_t off = ((cur >> (8 * s)) & 0xFFu) * bytes;
    asm("" : "+s"(off));
    return off;
}

// p + byte offset
__device__ __forceinline__ const uint32_t *at_bytes(const uint32_t *p, uint32_t off) {
    return reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(p) + off);
}

// A tile's mask image in global memory, read through a buffer resource: the
// symbol's row offset goes in a scalar register and the lane's offset in a
// vector one, so a read costs no vector address arithmetic (a 64-bit vector
// address add issues at a fraction of the full rate).  Reads beyond the
// image's size return 0.
constexpr int kRsrcWord3 = 0x00020000;  // raw (byte-addressed) buffer, 32-bit data format
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const uint32_t *img, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(img), (short)0, bytes, kRsrcWord3);
}

// n consecutive words at byte offset voff + soff of the image
template <int N>
__device__ __forceinline__ void gload(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, uint32_t *dst) {
    if constexpr (N == 1) {
        dst[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0);
    } else if constexpr (N == 2) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0);
        dst[0] = v.x;
        dst[1] = v.y;
    } else {
        static_assert(N % 4 == 0, "1, 2 or a multiple of 4 words");
#pragma unroll
        for (int q = 0; q < N / 4; ++q) {
            const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16 * q, soff, 0);
            dst[4 * q] = v.x;
            dst[4 * q + 1] = v.y;
            dst[4 * q + 2] = v.z;
            dst[4 * q + 3] = v.w;
        }
    }
}

// ------------------------------------------------------------------ cutoff
// Word cutoff for multi-word columns (Ukkonen's cutoff, kept per 32-row word
// as in Myers' block-based algorithm, but decided once per group of 4
// symbols).  Words 0..y are advanced; the words below y are left stale.
// Invariant: every cell of the rows in words > y has a value > K.  Then
// those cells can never matter for a value <= K (a cell <= K is reached
// from a neighbour whose value is <= its own), and no hit can end while the
// last word is inactive.
//
// Decision at the end of a group, from s_b, the value at the bottom row of
// word b (a prefix sum of the vertical deltas):
//   * word b+1 must be active if s_b <= K + 4: otherwise, since a value
//     changes by at most 1 per symbol, s_b stays above K + 3 for the next 4
//     symbols, and the first row of word b+1 (reached from row s_b's cell on
//     the diagonal, or from above) cannot come down to K;
//   * word b must stay active if s_b <= K + 31: the 31 rows above the bottom
//     row of a word are at least s_b - 31, so otherwise all of them are > K.
// The new y is the largest index either rule asks for, over every lane (the
// whole wavefront steps the same words).  A word that becomes active again
// is reset to +1 vertical deltas: values s_y + 1, s_y + 2, ..., which are
// upper bounds of the true ones (a value grows by at most 1 per row), and
// cells whose true value is > K may be overestimated without changing any
// value <= K.  The screen and exact test then read the last row only while
// every word is active.
//
// The cutoff columns use low placement (row j at bit j; the last word holds
// r = m - 32(W-1) pattern rows, and the rows above them, which influence no
// pattern row, are ignored): the first word then holds 32 pattern rows, and
// its bottom value is large unless the text really matches the pattern's
// first 32 symbols.  For the last word the "stay" rule uses D, the last
// pattern row's value, with the r - 1 pattern rows above it in that word:
// D <= K + r - 1.
//
// `kc` = -(K + 5) per lane: acc = kc + popcount of the vertical deltas of
// words 0..b (counted as popc(pv) + popc(~mv)) makes s_b <= K + 4 exactly
// acc < 32(b+1), and s_b <= K + 31 exactly acc < 32(b+1) + 27; for the last
// word (rows read through `mask`), D <= K + r - 1 is acc < `kl` with
// kl = 32(W-1) + 2r - 5 per lane.
template <int W, int N>
__device__ __forceinline__ uint32_t cut_decide(const uint32_t (&pv)[W], const uint32_t (&cm)[W], uint32_t kc,
                                               uint32_t mask, uint32_t kl) {
    uint32_t acc = kc, ynew = 0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
        if (b == W - 1) {
            acc = bcnt_acc(cm[b] & mask, acc);
            acc = bcnt_acc(pv[b] & mask, acc);
            if (__ballot((int32_t)acc < (int32_t)kl)) ynew = W - 1;
            break;
        }
        acc = bcnt_acc(cm[b], acc);
        acc = bcnt_acc(pv[b], acc);
        if (__ballot((int32_t)acc < 32 * (b + 1))) {
            ynew = b + 1;
        } else if (__ballot((int32_t)acc < 32 * (b + 1) + 27)) {
            ynew = ynew > (uint32_t)b ? ynew : (uint32_t)b;
        }
    }
    return ynew < (uint32_t)(W - 1) ? ynew : (uint32_t)(W - 1);
}

// Where a tile's match masks are read from (the MODE template argument):
constexpr int kImgGlobal = 0;  // the image through L1/L2 (buffer resource)
constexpr int kImgLds = 1;     // the image copied to LDS

// Masks of words 0..N-1 of a cutoff tile's lane for symbol s of the group
// `cur`.  The image is word-major ([class][word][lane]: the 64 lanes' masks
// of one word are 256 contiguous bytes).
template <int W, int N, int MODE>
__device__ __forceinline__ void cut_masks(const uint32_t *img, __amdgpu_buffer_rsrc_t rs, uint32_t lane,
                                          uint32_t cur, int s, uint32_t *e) {
    if constexpr (MODE == kImgLds) {
        const uint32_t *r = at_bytes(img + lane, row_off(cur, s, W * kWave * 4));
#pragma unroll
        for (int w = 0; w < N; ++w) e[w] = r[w * kWave];
    } else {
        const uint32_t off = row_off(cur, s, W * kWave * 4);
#pragma unroll
        for (int w = 0; w < N; ++w) gload<1>(rs, lane * 4, off + w * kWave * 4, &e[w]);
    }
}

// One group of 4 symbols with only words 0..N-1 active (N < W): partial
// mask reads, N-word column steps, then the cutoff decision.
//
// The cutoff tiles' images are word-major, [class][word][lane]: the masks of
// word w for the 64 lanes are 256 contiguous bytes, so reading only the
// active words stays one coalesced access per word (a lane-major row of
// 8 words would make every partial read touch 16 cache lines).
template <int W, int N, int MODE>
__device__ __forceinline__ uint32_t cut_group(uint32_t (&pv)[W], uint32_t (&cm)[W], const uint32_t *img,
                                              __amdgpu_buffer_rsrc_t rs, uint32_t lane, uint32_t cur, uint32_t kc,
                                              uint32_t mask, uint32_t kl) {
    uint32_t e[kScanGroup][N];
#pragma unroll
    for (int s = 0; s < kScanGroup; ++s) cut_masks<W, N, MODE>(img, rs, lane, cur, s, e[s]);
#pragma unroll
    for (int s = 0; s < kScanGroup; ++s) column_step_n<N, W>(pv, cm, e[s]);
    return cut_decide<W, N>(pv, cm, kc, mask, kl);
}

// Consecutive groups with exactly N words active, in a loop of its own (so
// that the column state stays in the same registers from group to group):
// runs from `pos` until the decision asks for another word count or the
// chunk ends, and returns that decision.  `next` holds the text word of the
// group at `pos` and is advanced with it; `wsteps` (which starts from every
// word stepped over every reported symbol) loses the W - N inactive words
// over the run's reported symbols.
template <int W, int N, int MODE>
__device__ __forceinline__ uint32_t cut_run(uint32_t (&pv)[W], uint32_t (&cm)[W], const uint32_t *img,
                                            __amdgpu_buffer_rsrc_t rs, uint32_t lane, const const_u32 *text,
                                            uint32_t &next, uint32_t &pos, uint32_t len, uint32_t lb, uint32_t kc,
                                            uint32_t mask, uint32_t kl, uint64_t &wsteps, uint32_t nact) {
    uint32_t ynew;
    const uint32_t first = pos;
    do {
        const uint32_t cur = next;
        next = text[(pos >> 2) + 1];
        ynew = cut_group<W, N, MODE>(pv, cm, img, rs, lane, cur, kc, mask, kl);
        pos += kScanGroup;
    } while (ynew == N - 1 && pos < len);
    const uint32_t s0 = first > lb ? first : lb, s1 = pos < len ? pos : len;
    if (s1 > s0) wsteps -= (uint64_t)(s1 - s0) * ((W - N) * nact);
    return ynew;
}

// K1.  Block = `waves` wavefronts sharing one tile (its match-mask image in
// LDS, or read through the L1 when it does not fit); each wavefront scans
// one chunk.  Lane l holds P patterns of W words (slots l, l+64, ...).
// The text symbol is wave-uniform (scalar loads).  Hits are screened once per
// group of 4 symbols: the last-row value moves by at most 1 per symbol, so
// if D > K + 2 at the group's second symbol no symbol of the group is a hit.
// Only when some lane passes the screen is the group replayed from its saved
// start state with an exact test per symbol, and the hits are compacted with
// a ballot and an mbcnt prefix into the item's own record buffer.
//
// The grid is one-dimensional and XCD-aware: workgroups are handed to the 8
// XCDs round-robin (block b to XCD b % 8), so the ntiles blocks that scan the
// same chunks with different tiles are given ids b, b + 8, ... on one XCD,
// one after the other; the text they share is read from HBM once and then
// hit in that XCD's L2.
//
// CUT: the word cutoff described above (one pattern per lane, W >= 2).
template <int W, int P, int MODE, bool CUT>
__global__ void __launch_bounds__(256, CUT ? (W <= 4 ? 6 : 1) : (P * W <= 4 ? 8 : 1)) k_scan(ScanArgs a) {
    static_assert(!CUT || (P == 1 && W >= 2), "the cutoff is for one multi-word pattern per lane");
    constexpr bool LDSPEQ = MODE == kImgLds;
    extern __shared__ uint32_t lds_img[];
    constexpr int PW = P * W;
    constexpr int PWS = pad_pow2(PW);
    const uint32_t xcd = blockIdx.x & (kXcds - 1), r = blockIdx.x / kXcds;
    const uint32_t tile_local = r % a.ntiles;
    const uint32_t cblock = (r / a.ntiles) * kXcds + xcd;
    if (cblock * (blockDim.x >> 6) >= a.nchunks) return;  // padding blocks (uniform per block)
    const TileDesc td = a.tiles[a.tile_first + tile_local];
    const uint32_t *gimg = a.peq_img + td.peq_off;
    if (LDSPEQ) {
        const uint32_t words = a.nclass * kWave * (CUT ? W : PWS);  // multiple of 64
        const uint4 *src = reinterpret_cast<const uint4 *>(gimg);
        uint4 *dst = reinterpret_cast<uint4 *>(lds_img);
        for (uint32_t i = threadIdx.x; i < words / 4; i += blockDim.x) dst[i] = src[i];
        __syncthreads();
    }
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(threadIdx.x >> 6);
    const uint32_t chunk = uniform(cblock * (blockDim.x >> 6) + wave);
    if (chunk >= a.nchunks) return;
    const ChunkDesc cd = a.chunks[chunk];
    const uint32_t item = a.item_base + chunk * a.ntiles + tile_local;
    uint32_t *rec = a.item_rec + (size_t)item * a.cap;

    // Inactive slots hold all-ones +1 deltas (D = 32W) and bounds of 0, so
    // they never pass the screen or the exact test.  kk / k2 hold the biases
    // of le_bound for the exact test (D <= K) and the screen (D <= K + 2).
    //
    // CUT (low placement): the last word's pattern rows are read through
    // `lmask` (r = m - 32(W-1) rows); kk / k2 then count popcount(lmask) in
    // place of 32 for that word, and kc / kl are cut_decide's biases.
    uint32_t pv[P][W], mv[P][W], kk[P], k2[P], pat[P], kc = 0, kl = 0, lmask = ~0u;
    bool act[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t slot = p * kWave + lane;
        act[p] = slot < td.n_active;
        pat[p] = act[p] ? a.slot_pat[td.slot_off + slot] : 0u;
        const PatDesc d = a.pats[pat[p]];
        if (CUT) {
            const uint32_t r = act[p] ? (uint32_t)d.m - 32u * (W - 1) : 32u;  // 1..32
            lmask = r == 32 ? ~0u : (1u << r) - 1u;
            const uint32_t base = (uint32_t)(-32 * (W - 1) - 1) - r;
            kk[p] = base - (act[p] ? (uint32_t)d.k : 0u);
            k2[p] = base - (act[p] ? (uint32_t)d.k + 2 : 2u);
            kc = (uint32_t)(-5) - (act[p] ? (uint32_t)d.k : 0u);
            kl = 32u * (W - 1) + 2u * r - 5u;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                pv[p][w] = ~0u;  // the first column: row r holds r (+1 deltas)
                mv[p][w] = ~0u;  // complemented: no -1 deltas
            }
            continue;
        }
        kk[p] = (uint32_t)(-32 * W - 1) - (act[p] ? (uint32_t)d.k : 0u);
        k2[p] = (uint32_t)(-32 * W - 1) - (act[p] ? (uint32_t)d.k + 2 : 0u);
        const int g = 32 * W - (int)d.m;  // wildcard rows below the pattern
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int lo = g - 32 * w;  // first pattern bit inside word w
            const uint32_t bits = lo <= 0 ? ~0u : (lo >= 32 ? 0u : (~0u << lo));
            pv[p][w] = act[p] ? bits : ~0u;
            mv[p][w] = ~0u;  // complemented: no -1 deltas
        }
    }
    // last-row test: D <= bound (bias holds the bound)
    auto le = [&](const uint32_t (&v)[W], const uint32_t (&c)[W], uint32_t bias) -> int32_t {
        if constexpr (CUT) return le_bound_masked<W>(v, c, bias, lmask);
        else return le_bound<W>(v, c, bias);
    };
    uint32_t cnt = 0;
    // active pattern slots of this wavefront, and the pattern words it
    // advances over the symbols whose ends it reports (a scalar tally)
    uint32_t nact = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) nact += (uint32_t)__popcll(__ballot(act[p]));
    uint64_t wsteps = 0;  // set below, once the chunk's extent is known

    const const_u32 *text = (const const_u32 *)(cd.sym);
    const uint32_t len = cd.scan_len, lb = cd.lookback;
    const uint32_t lane_off = lane * PWS;
    if (len > lb) wsteps = (uint64_t)(len - lb) * (W * nact);
    const uint32_t *img = MODE == kImgGlobal ? gimg : lds_img;
    const __amdgpu_buffer_rsrc_t rs = image_rsrc(gimg, a.nclass * kWave * (CUT ? W : PWS) * 4);

    uint32_t y = W - 1;  // last active word (CUT); every word starts active
    uint32_t next = text[0];
    uint32_t pos = 0;
    while (pos < len) {
        if (CUT && y < W - 1) {
            // groups with the last word inactive (each word count in a loop
            // of its own, left when the count changes)
            uint32_t ynew = y;
            switch (y) {  // wave-uniform
#define OASM_CUT_CASE(n)                                                                                         \
    case n:                                                                                                      \
        if constexpr (n + 1 < W)                                                                                 \
            ynew = cut_run<W, n + 1, MODE>(pv[0], mv[0], img, rs, lane, text, next, pos, len, lb, kc, lmask, \
                                           kl, wsteps, nact);                                                  \
        break;
                OASM_CUT_CASE(0)
                OASM_CUT_CASE(1)
                OASM_CUT_CASE(2)
                OASM_CUT_CASE(3)
                OASM_CUT_CASE(4)
                OASM_CUT_CASE(5)
                OASM_CUT_CASE(6)
#undef OASM_CUT_CASE
                default: break;
            }
            if (ynew > y) {  // reactivated words restart from +1 deltas
#pragma unroll
                for (int w = 1; w < W; ++w)
                    if ((uint32_t)w > y && (uint32_t)w <= ynew) {
                        pv[0][w] = ~0u;
                        mv[0][w] = ~0u;
                    }
            }
            y = ynew;
            continue;
        }
        const uint32_t cur = next;
        next = text[(pos >> 2) + 1];
        Words<PWS> e[kScanGroup];
#pragma unroll
        for (int s = 0; s < kScanGroup; ++s) {
            if constexpr (CUT) {  // word-major image
                cut_masks<W, W, MODE>(img, rs, lane, cur, s, e[s].v);
            } else if constexpr (LDSPEQ) {
                e[s] = *reinterpret_cast<const Words<PWS> *>(at_bytes(img + lane_off, row_off(cur, s, kWave * PWS * 4)));
            } else {
                gload<PWS>(rs, lane_off * 4, row_off(cur, s, kWave * PWS * 4), e[s].v);
            }
        }
        uint32_t pv0[P][W], mv0[P][W];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int w = 0; w < W; ++w) {
                pv0[p][w] = pv[p][w];
                mv0[p][w] = mv[p][w];
            }
        int32_t screen[P];
#pragma unroll
        for (int s = 0; s < kScanGroup; ++s) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                column_step<W>(pv[p], mv[p], &e[s].v[p * W]);
                if (s == 1) screen[p] = le(pv[p], mv[p], k2[p]);
            }
        }
        uint64_t sb[P], any = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            sb[p] = __ballot(screen[p] < 0);
            any |= sb[p];
        }
        if (any && pos + (kScanGroup - 1) >= lb) {
            // replay the pattern slots that passed the screen from the group's
            // start state, with an exact test per symbol
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (!sb[p]) continue;
#pragma unroll
                for (int s = 0; s < kScanGroup; ++s) {
                    const bool inrange = (pos + s >= lb) && (pos + s < len);
                    column_step<W>(pv0[p], mv0[p], &e[s].v[p * W]);
                    const uint64_t b = __ballot(le(pv0[p], mv0[p], kk[p]) < 0);
                    if (inrange && b) {
                        if ((b >> lane) & 1ull) {
                            const uint32_t idx = cnt + mbcnt64(b);
                            if (idx < a.cap) rec[idx] = ((p * kWave + lane) << 24) | (pos + s - lb);
                        }
                        cnt += (uint32_t)__popcll(b);
                    }
                }
            }
        }
        if (CUT) y = cut_decide<W, W>(pv[0], mv[0], kc, lmask, kl);
        pos += kScanGroup;
    }
    if (lane == 0) {
        a.item_cnt[item] = cnt;
        atomicMax(a.max_cnt, cnt);
        if (a.wsteps) atomicAdd(a.wsteps, (unsigned long long)wsteps);
    }
}

template <int W, int P, bool CUT>
static hipError_t launch_scan_t(const ScanArgs &a, int waves, int mode, hipStream_t st) {
    if (waves < 1 || waves > 4) return hipErrorInvalidValue;
    const uint32_t gx = (a.nchunks + waves - 1) / waves;
    if (gx == 0 || a.ntiles == 0) return hipSuccess;
    const uint64_t blocks = (uint64_t)((gx + kXcds - 1) / kXcds) * kXcds * a.ntiles;
    if (blocks > 0xFFFFFFFFull) return hipErrorInvalidValue;
    if (mode == kImgGlobal) {
        hipLaunchKernelGGL((k_scan<W, P, kImgGlobal, CUT>), dim3((uint32_t)blocks), dim3(waves * kWave), 0, st, a);
        return hipGetLastError();
    }
    const size_t shmem = (size_t)a.nclass * kWave * (CUT ? W : pad_pow2(P * W)) * 4;
    // raise the kernel's dynamic-LDS limit once per device (never inside a
    // graph capture: the first launch of a shape is always an eager one);
    // contexts on several host threads share the table
    static std::mutex mu;
    static size_t configured[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    {
        std::lock_guard<std::mutex> g(mu);
        if (shmem > configured[dev]) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_scan<W, P, kImgLds, CUT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
            if (e != hipSuccess) return e;
            configured[dev] = shmem;
        }
    }
    hipLaunchKernelGGL((k_scan<W, P, kImgLds, CUT>), dim3((uint32_t)blocks), dim3(waves * kWave), shmem, st, a);
    return hipGetLastError();
}

bool scan_variant_exists(int W, int P, bool cut) {
    if (cut) return P == 1 && W >= 2 && W <= kMaxW32;
    switch (W * 16 + P) {
        case 1 * 16 + 1: case 1 * 16 + 2: case 1 * 16 + 4:
        case 2 * 16 + 1: case 2 * 16 + 2:
        case 3 * 16 + 1: case 4 * 16 + 1: case 5 * 16 + 1:
        case 6 * 16 + 1: case 7 * 16 + 1: case 8 * 16 + 1:
            return true;
        default:
            return false;
    }
}

hipError_t launch_scan(int W, int P, bool cut, const ScanArgs &a, int waves, int mode, hipStream_t st) {
    if (mode != kImgGlobal && mode != kImgLds) return hipErrorInvalidValue;
    if (cut) {
        if (P != 1) return hipErrorInvalidValue;
        switch (W) {
            case 2: return launch_scan_t<2, 1, true>(a, waves, mode, st);
            case 3: return launch_scan_t<3, 1, true>(a, waves, mode, st);
            case 4: return launch_scan_t<4, 1, true>(a, waves, mode, st);
            case 5: return launch_scan_t<5, 1, true>(a, waves, mode, st);
            case 6: return launch_scan_t<6, 1, true>(a, waves, mode, st);
            case 7: return launch_scan_t<7, 1, true>(a, waves, mode, st);
            case 8: return launch_scan_t<8, 1, true>(a, waves, mode, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (W * 16 + P) {
        case 1 * 16 + 1: return launch_scan_t<1, 1, false>(a, waves, mode, st);
        case 1 * 16 + 2: return launch_scan_t<1, 2, false>(a, waves, mode, st);
        case 1 * 16 + 4: return launch_scan_t<1, 4, false>(a, waves, mode, st);
        case 2 * 16 + 1: return launch_scan_t<2, 1, false>(a, waves, mode, st);
        case 2 * 16 + 2: return launch_scan_t<2, 2, false>(a, waves, mode, st);
        case 3 * 16 + 1: return launch_scan_t<3, 1, false>(a, waves, mode, st);
        case 4 * 16 + 1: return launch_scan_t<4, 1, false>(a, waves, mode, st);
        case 5 * 16 + 1: return launch_scan_t<5, 1, false>(a, waves, mode, st);
        case 6 * 16 + 1: return launch_scan_t<6, 1, false>(a, waves, mode, st);
        case 7 * 16 + 1: return launch_scan_t<7, 1, false>(a, waves, mode, st);
        case 8 * 16 + 1: return launch_scan_t<8, 1, false>(a, waves, mode, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace oasm
