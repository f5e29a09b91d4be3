// K4: the per-start distances of LEV CALC (Section 6, the LEV CORE
// description: at every stream index i, the distances between p and the
// 2K+1 substrings t[i, l_p-K] .. t[i, l_p+K]; Section 6.2), for every start
// of a device-resident text and every pattern of the dictionary.
//
// The FPGA fills the matrix of Eq. 1 anti-diagonal by anti-diagonal with one
// processing element per pattern row.  Here a thread owns one start i and
// advances the anchored DP column (first row C[0][l] = l, first column
// C[r][0] = r) over t[i], t[i+1], ... as a bit-vector column recurrence,
// 32 pattern rows per 32-bit VALU word; after l symbols the last row holds
// lev(p, t[i,l]).  The 256 threads of a block take 256 consecutive starts
// of one pattern: the pattern's match masks (indexed by byte value) and the
// text window the block's starts read sit in LDS, and the output of a wave
// (64 starts x (2K+1) bytes) is one contiguous run.
//
// Integer bit-vector work only; no matrix cores.
#include <mutex>
#include <type_traits>

#include "oasm_device.h"
#include "oasm_levcalc.h"

namespace oasm {

// Truth-table operands of v_bitop3_b32: the result bit for inputs (a, b, c)
// is bit (a*4 + b*2 + c) of the immediate.
constexpr uint32_t LA = 0xF0, LB = 0xCC, LC = 0xAA;
#define LC_BITOP3(a, b, c, expr) __builtin_amdgcn_bitop3_b32((a), (b), (c), (uint32_t)((expr) & 0xFF))

// x + x as v_add_u32 (a full-rate op; the compiler would emit a shift)
static __device__ __forceinline__ uint32_t lc_add_self(uint32_t x) {
    uint32_t r;
    asm("v_add_u32 %0, %1, %1" : "=v"(r) : "v"(x));
    return r;
}

// popcount(x) + acc
static __device__ __forceinline__ uint32_t lc_bcnt(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// popcount(x) + acc with acc a scalar (uniform) value
static __device__ __forceinline__ uint32_t lc_bcnt_s(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "s"(acc));
    return r;
}

// Fourth word of a raw (untyped, byte-addressed) buffer resource on gfx9-family
// parts: a valid 32-bit data format, so that stores inside the size are kept.
constexpr int kLcRsrcWord3 = 0x00020000;
constexpr int kLcThreads = 256;                   // starts per block pass
constexpr int kLcWin = kLcThreads + 256 + 64;     // + m_max + K_max - 1 symbols, rounded up
constexpr int kLcUnroll = 4;                      // symbols per unrolled group
constexpr int kLcStage = (kLcWin + kLcThreads - 1) / kLcThreads;  // window symbols per thread

// One column of the anchored recurrence (Myers 1999 in Hyyro's form, with
// the +1 horizontal delta of the first DP row entering the first pattern
// row).  Row r (1-based) of the pattern is bit b0 + r - 1 of the W-word
// column.  One-word columns use high placement, b0 = 32 - m: row m is the
// top bit, and the b0 bits below row 1 are rows that match every byte and
// start with no vertical delta; with eq = 1 and pv = mv = 0 they produce
// ph = mh = 0 and keep pv = mv = 0, so they never feed a pattern row, and
// the +1 of the first DP row is put in at bit b0 (`inj` = 1 << b0).  Wider
// columns use low placement, b0 = 0 (row r at bit r - 1, which keeps the
// band cutoff below as tight as possible): the rows above row m at the top
// of the last word take deltas from below but never feed a pattern row, and
// are masked out of the last-row sum.
// pv: rows with vertical delta +1; cm: complement of the rows with vertical
// delta -1; eq: rows whose pattern byte equals the text byte.  With
// u = (eq & pv) + pv (carry across words):
//   ph = mv | ~(u | pv | eq),  mh = pv & (eq | ~u),
//   ph2 = (ph << 1) | inj,     mh2 = mh << 1   (one row down, across words),
//   pv' = mh2 | ~(eq | mv | ph2),  mv' = ph2 & (eq | mv).
//
// anchored_step<N, W> advances only the first N words of the column (the
// band cutoff below); the carry and shifts out of word N-1 are dropped.
template <int N, int W>
__device__ __forceinline__ void anchored_step(uint32_t (&pv)[W], uint32_t (&cm)[W], const uint32_t *eq,
                                              uint32_t inj) {
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
        const uint32_t o = LC_BITOP3(u, pv[w], eq[w], LA | LB | LC);
        ph[w] = LC_BITOP3(cm[w], o, 0u, ~(LA & LB));          // ~cm | ~o
        mh[w] = LC_BITOP3(pv[w], eq[w], u, LA & (LB | ~LC));  // pv & (eq | ~u)
    }
    uint32_t npv[N], ncm[N];
#pragma unroll
    for (int w = 0; w < N; ++w) {
        const uint32_t ph2 = w == 0 ? (lc_add_self(ph[0]) | inj) : __builtin_amdgcn_alignbit(ph[w], ph[w - 1], 31);
        const uint32_t mh2 = w == 0 ? lc_add_self(mh[0]) : __builtin_amdgcn_alignbit(mh[w], mh[w - 1], 31);
        const uint32_t t = LC_BITOP3(eq[w], cm[w], ph2, ~(LA | ~LB | LC));  // ~(eq | ~cm | ph2)
        npv[w] = mh2 | t;
        ncm[w] = LC_BITOP3(ph2, eq[w], cm[w], ~(LA & (LB | ~LC)));        // ~(ph2 & (eq | ~cm))
    }
#pragma unroll
    for (int w = 0; w < N; ++w) {
        pv[w] = npv[w];
        cm[w] = ncm[w];
    }
}

// Band cutoff of the anchored column (Ukkonen's cutoff on the upper side of
// the band): after l symbols, C[r][l] >= r - l, so rows r > l + K hold values
// above K, and a cell above K never leads to a value <= K.  The step that
// produces column l therefore advances only the words holding rows
// 1 .. l + K (bits up to b0 + l + K - 1), N(l) = ceil((b0 + l + K) / 32) of
// them; the words above keep their initial +1 vertical deltas until they are
// first advanced, i.e. values C[r0][l] + (r - r0) at the rows r of a word
// whose lowest row is r0, upper bounds of the true ones (a value grows by at
// most 1 per row).  Upper bounds of cells above K change no value <= K, and
// every output step (l >= m - K) advances all W words.  quiet_band<W, 1>
// runs steps j .. j1-1 (column l = j + 1), word count by word count; kb =
// K + b0.
template <int W, int N>
__device__ __forceinline__ void quiet_band(uint32_t (&pv)[W], uint32_t (&cm)[W], const uint32_t *&wp, uint32_t &j,
                                           uint32_t j1, uint32_t kb, uint32_t inj, const char *tab) {
    if constexpr (N <= W) {
        // steps whose column l = j + 1 needs at most N words: b0 + l + K <= 32 N
        const uint32_t lim_n = 32u * N > kb ? 32u * N - kb : 0u;  // j + 1 + kb <= 32 N  <=>  j < 32 N - kb
        const uint32_t end = N == W ? j1 : (lim_n < j1 ? lim_n : j1);
        constexpr int U = N <= 2 ? kLcUnroll : N <= 4 ? 2 : 1;  // mask rows read ahead (registers)
        for (; j + U <= end; j += U, wp += U) {
            uint32_t eq[U][N];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t *r = reinterpret_cast<const uint32_t *>(tab + wp[u]);
#pragma unroll
                for (int w = 0; w < N; ++w) eq[u][w] = r[w];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) anchored_step<N, W>(pv, cm, eq[u], inj);
        }
        for (; j < end; ++j, ++wp) {
            uint32_t eq[N];
            const uint32_t *r = reinterpret_cast<const uint32_t *>(tab + wp[0]);
#pragma unroll
            for (int w = 0; w < N; ++w) eq[w] = r[w];
            anchored_step<N, W>(pv, cm, eq, inj);
        }
        quiet_band<W, N + 1>(pv, cm, wp, j, j1, kb, inj, tab);
    }
}

// Mask rows are lcStride(W) = W | 1 words apart.  The lanes of a wave each
// read the row of their own text byte: with an odd stride the rows of
// different bytes spread over all of the LDS banks, while a stride of
// 2^a * b words (b odd) would fold them onto a 1/2^a share of the banks.
constexpr int lcStride(int W) { return W | 1; }

// Block (x, y): pattern pat_ids[y] (strided by gridDim.y), starts in passes
// of 256 (strided by gridDim.x).  The window holds, per text symbol, the
// byte offset of its row in the mask table (byte * lcStride(W) * 4), so a
// mask read needs no address arithmetic.  Every index is bounded: the window
// holds 256 + m + K - 1 <= kLcWin symbols, a mask row is
// byte * lcStride(W) + word with word < W.
template <int W>
__global__ void __launch_bounds__(kLcThreads) k_levcalc(LevcalcArgs a) {
    constexpr int S = lcStride(W);
    __shared__ uint32_t peq[256 * S];
    __shared__ uint32_t win[kLcWin];
    const uint32_t tid = threadIdx.x;
    const uint64_t passes = (a.n + kLcThreads - 1) / kLcThreads;
    for (uint32_t x = blockIdx.y; x < a.npat; x += gridDim.y) {
        const uint32_t q = a.pat_ids[x];
        const PatDesc d = a.pats[q];
        const uint32_t m = d.m, K = d.k;
        const uint32_t width = 2 * K + 1;        // lengths m-K .. m+K
        const uint32_t steps = m + K;            // symbols read per start
        const uint32_t quiet = m - K - 1;        // leading steps without output (l < m - K)
        const uint32_t b0 = W == 1 ? 32u - m : 0u;  // match-all rows below row 1, 0..31
        const uint32_t inj = 1u << b0;              // the first DP row's +1 enters at row 1
        const uint32_t low = inj - 1u;              // the match-all rows
        const uint32_t rlast = m - 32u * (W - 1);   // pattern rows in the last word (W > 1), 1..32
        const uint32_t lmask = W == 1 || rlast >= 32 ? ~0u : (1u << rlast) - 1u;
        uint8_t *const out = a.out + a.n * a.out_unit[q];
        const uint8_t *const pb = a.pat_bytes + d.off;

        __syncthreads();  // the previous pattern's masks and window are no longer read
        // every byte's row: the match-all rows set, then pattern row r + 1
        // (0-based r) at bit b0 + r where the byte equals p[r]
        for (uint32_t i = tid; i < 256u * S; i += kLcThreads) peq[i] = i % S == 0 ? low : 0u;
        __syncthreads();
        for (uint32_t r = tid; r < m; r += kLcThreads) {
            const uint32_t q = b0 + r;
            atomicOr(&peq[pb[r] * S + (q >> 5)], 1u << (q & 31));
        }

        // the window of the next pass is loaded into registers while the
        // current one is matched (software pipelining of the text reads)
        const uint32_t wlen = kLcThreads + steps - 1;
        uint32_t nxt[kLcStage];
        auto fetch = [&](uint64_t pass) {
            const uint64_t base = pass * kLcThreads;
#pragma unroll
            for (int k = 0; k < kLcStage; ++k) {
                const uint32_t i = tid + k * kLcThreads;
                nxt[k] = (i < wlen && pass < passes && base + i < a.n) ? a.text[base + i] : 0u;
            }
        };
        fetch(blockIdx.x);
        for (uint64_t pass = blockIdx.x; pass < passes; pass += gridDim.x) {
            const uint64_t base = pass * kLcThreads;
            __syncthreads();  // masks complete; the previous window is no longer read
#pragma unroll
            for (int k = 0; k < kLcStage; ++k) {
                const uint32_t i = tid + k * kLcThreads;
                if (i < wlen) win[i] = nxt[k] * (S * 4u);
            }
            __syncthreads();
            fetch(pass + gridDim.x);
            const uint64_t s = base + tid;
            if (s >= a.n) continue;

            uint32_t pv[W], cm[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                pv[w] = w == 0 ? ~low : ~0u;  // C[r][0] = r: every vertical delta is +1 (0 below row 1)
                cm[w] = ~0u;  // no -1 deltas (complemented)
            }
            const uint32_t *wp = win + tid;
            const char *const tab = reinterpret_cast<const char *>(peq);
            auto masks = [&](uint32_t off, uint32_t (&eq)[W]) {
                const uint32_t *r = reinterpret_cast<const uint32_t *>(tab + off);
#pragma unroll
                for (int w = 0; w < W; ++w) eq[w] = r[w];
            };
            // l = j + 1 below m - K: no output yet (band cutoff)
            uint32_t j = 0;
            quiet_band<W, 1>(pv, cm, wp, j, quiet, K + b0, inj, tab);
            // l = m - K .. m + K: C[m][l] = l + (sum of the vertical deltas of
            // rows 1..m) = l - m + popcount(pv) + popcount(cm) over those
            // rows = l - m - b0 + popcount(pv) + popcount(cm) over the column
            // below the last word's mask (below row 1, pv = 0 and cm = 1).
            // The pass's output (256 starts x width bytes, pattern-major
            // layout) is one buffer: byte i of start s is at tid * width + i,
            // the lane part in a vector register and i in a scalar one, so a
            // store needs no vector address arithmetic; the buffer's size
            // bounds every store.
            const uint64_t left = a.n - base;
            const uint32_t pass_bytes = (uint32_t)(left < (uint64_t)kLcThreads ? left : kLcThreads) * width;
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc(out + base * width, (short)0, pass_bytes, kLcRsrcWord3);
            const uint32_t voff = tid * width;
            auto outputs = [&](auto tail) {
                constexpr bool TAIL = decltype(tail)::value;
                const uint32_t room = TAIL ? (uint32_t)(a.n - s) : 0u;  // symbols from s to the end
                for (uint32_t i = 0; i < width; ++i) {
                    uint32_t eq[W];
                    masks(wp[i], eq);
                    anchored_step<W, W>(pv, cm, eq, inj);
                    const uint32_t l = m - K + i;
                    uint32_t dsum = lc_bcnt_s(pv[0], l - m - b0);  // wraps; the total is >= 0
                    dsum = lc_bcnt(cm[0], dsum);
#pragma unroll
                    for (int w = 1; w < W; ++w) {
                        dsum = lc_bcnt(pv[w] & (w == W - 1 ? lmask : ~0u), dsum);
                        dsum = lc_bcnt(cm[w] & (w == W - 1 ? lmask : ~0u), dsum);
                    }
                    uint32_t v = dsum < K + 1 ? dsum : K + 1;
                    if (TAIL && l > room) v = 255u;  // t[s, l] runs past the end
                    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, rs, voff, i, 0);
                }
            };
            // a pass whose every substring ends inside the text needs no end test
            if (base + kLcThreads + steps - 1 <= a.n)
                outputs(std::false_type{});
            else
                outputs(std::true_type{});
        }
    }
}

template <int W>
hipError_t launch_levcalc_t(const LevcalcArgs &a, hipStream_t st) {
    if (a.n == 0 || a.npat == 0) return hipSuccess;
    const uint64_t passes = (a.n + kLcThreads - 1) / kLcThreads;
    const uint32_t gy = a.npat < 65535u ? a.npat : 65535u;
    // about 32k blocks in all: enough to fill 256 CUs many times over, few
    // enough that each block builds its mask table once for many passes
    uint64_t gx = (32768u + gy - 1) / gy;
    if (gx > passes) gx = passes;
    if (gx > 0x7FFFFFFFull) gx = 0x7FFFFFFFull;
    hipLaunchKernelGGL((k_levcalc<W>), dim3((uint32_t)gx, gy), dim3(kLcThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_levcalc(int W, const LevcalcArgs &a, hipStream_t st) {
    switch (W) {
        case 1: return launch_levcalc_t<1>(a, st);
        case 2: return launch_levcalc_t<2>(a, st);
        case 3: return launch_levcalc_t<3>(a, st);
        case 4: return launch_levcalc_t<4>(a, st);
        case 5: return launch_levcalc_t<5>(a, st);
        case 6: return launch_levcalc_t<6>(a, st);
        case 7: return launch_levcalc_t<7>(a, st);
        case 8: return launch_levcalc_t<8>(a, st);
        default: return hipErrorInvalidValue;
    }
}


// ------------------------------------------------------------------ tables
// The allocation-free entry point's tables live in this array (one copy per
// GPU, held for the life of the process).  Host code never passes the
// array's name to a kernel: it passes the address levcalc_scratch() looked
// up on the device.
static __device__ __align__(256) uint8_t scratch[kLcScratchBytes];

hipError_t levcalc_scratch(int device, uint8_t **out) {
    static std::mutex mu;
    static uint8_t *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = reinterpret_cast<uint8_t *>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

// exclusive scan of one value per thread over a 256-thread block
__device__ __forceinline__ uint32_t lc_block_scan(uint32_t v, uint32_t *wsum, uint32_t &total) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, 64);
        if (lane >= (uint32_t)off) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (uint32_t w = 0; w < kLcThreads / 64; ++w) {
        const uint32_t x = wsum[w];
        if (w < wave) before += x;
        all += x;
    }
    __syncthreads();
    total = all;
    return before + incl - v;
}

// One block: thread t takes a contiguous run of patterns, counts them per
// word count and sums their 2K + 1; block scans turn the counts into each
// run's positions in the word-count-major id list and the sums into output
// units.
__global__ void __launch_bounds__(kLcThreads) k_levcalc_tables(const PatDesc *__restrict__ pats, uint32_t npat,
                                                               uint64_t *__restrict__ unit,
                                                               uint32_t *__restrict__ ids) {
    __shared__ uint32_t wsum[kLcThreads / 64];
    const uint32_t per = (npat + kLcThreads - 1) / kLcThreads;
    const uint32_t q0 = min(npat, threadIdx.x * per), q1 = min(npat, q0 + per);
    uint32_t cnt[kMaxW32] = {}, usum = 0, total = 0;
    for (uint32_t q = q0; q < q1; ++q) {
        const PatDesc d = pats[q];
#pragma unroll
        for (int w = 0; w < kMaxW32; ++w) cnt[w] += ((uint32_t)d.m + 31u) / 32u == (uint32_t)(w + 1) ? 1u : 0u;
        usum += 2u * d.k + 1u;
    }
    uint64_t u = lc_block_scan(usum, wsum, total);
    uint32_t pos[kMaxW32], base = 0;
#pragma unroll
    for (int w = 0; w < kMaxW32; ++w) {
        pos[w] = base + lc_block_scan(cnt[w], wsum, total);
        base += total;
    }
    for (uint32_t q = q0; q < q1; ++q) {
        const PatDesc d = pats[q];
        unit[q] = u;
        u += 2u * d.k + 1u;
        const uint32_t wq = ((uint32_t)d.m + 31u) / 32u;
#pragma unroll
        for (int w = 0; w < kMaxW32; ++w)
            if (wq == (uint32_t)(w + 1)) ids[pos[w]++] = q;
    }
}

hipError_t launch_levcalc_tables(const PatDesc *pats, uint32_t npat, uint8_t *scr, hipStream_t st) {
    if (npat == 0) return hipSuccess;
    if (npat > kLcNoallocMaxPatterns) return hipErrorInvalidValue;
    uint64_t *unit = reinterpret_cast<uint64_t *>(scr);
    uint32_t *ids = reinterpret_cast<uint32_t *>(scr + (size_t)kLcNoallocMaxPatterns * sizeof(uint64_t));
    hipLaunchKernelGGL(k_levcalc_tables, dim3(1), dim3(kLcThreads), 0, st, pats, npat, unit, ids);
    return hipGetLastError();
}

}  // namespace oasm
