// Host runtime and C ABI of oasm_gpu (see include/oasm_gpu.h).
//
// A context owns the dictionary's device tables, one staging buffer of
// class-mapped symbols per stream, reusable device work buffers, and host
// queues of results.  oasm_sync runs one matching step over every stream
// with new bytes (or one step per stream in plain mode):
//
//   plan      chunks of C symbols per stream, each read with an
//             (m_max + K_max - 1)-symbol look-back so its hit ends are exact
//   K1        scan, one launch per word-count class (grid: chunks x tiles),
//             hit ends into per-item record buffers
//   order     hit ends of filter segments left open by the previous step,
//             then the items' records (chunk-major), then a stable radix sort
//             on the (stream, pattern) key: (stream, pattern, end) order
//   K2        hit set at every new hit end
//   K3        Alg. 1 per segment; open segments are carried to the next step
//   compaction and copy-back of hit ends, occurrences and the new carry.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <tuple>
#include <mutex>
#include <thread>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/oasm_gpu.h"
#include "oasm_internal.h"
#include "oasm_levcalc.h"
#include "oasm_staging.h"
#include "oasm_hostpar.h"

#include <rocprofiler-sdk-roctx/roctx.h>

using namespace oasm;

namespace {

constexpr size_t kPad = 64;  // readable slack after every staging buffer
constexpr uint32_t kLongSlotsMax = 1u << 26;  // per-start slots of the parallel filter walk (3 arrays: 768 MiB)

struct HipFail {
    hipError_t e;
    const char *what;
};

inline void ck(hipError_t e, const char *what) {
    if (e != hipSuccess) throw HipFail{e, what};
}

// A device buffer that grows (never shrinks) on demand.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    template <class T>
    T *as() const { return reinterpret_cast<T *>(p); }
    void ensure(size_t bytes, hipStream_t st) {
        if (bytes <= cap) return;
        size_t want = std::max(bytes, cap + cap / 2);
        want = (want + 255) & ~size_t(255);
        if (p) {
            ck(hipStreamSynchronize(st), "sync before realloc");
            ck(hipFree(p), "hipFree");
            p = nullptr;
            cap = 0;
        }
        ck(hipMalloc(&p, want), "hipMalloc");
        cap = want;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// Pinned host buffer that grows on demand.
struct PinBuf {
    void *p = nullptr;
    size_t cap = 0;
    template <class T>
    T *as() const { return reinterpret_cast<T *>(p); }
    void ensure(size_t bytes, hipStream_t st) {
        if (bytes <= cap) return;
        size_t want = std::max(bytes, cap * 2);
        want = (want + 4095) & ~size_t(4095);
        if (p) {
            ck(hipStreamSynchronize(st), "sync before pinned realloc");
            ck(hipHostFree(p), "hipHostFree");
            p = nullptr;
            cap = 0;
        }
        ck(hipHostMalloc(&p, want, hipHostMallocDefault), "hipHostMalloc");
        cap = want;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct StreamState {
    uint64_t id = 0;
    uint32_t slot = 0;
    uint8_t *sym = nullptr;  // class-mapped symbols (device)
    size_t cap = 0;
    uint64_t base_abs = 0;   // absolute position of sym[0]
    size_t valid = 0;        // symbols held (from sym[0])
    size_t scanned = 0;      // of these, symbols already matched; the m_max + K_max + 3 before
                             // sym[scanned] are the look-back of the next chunk
    bool close_pending = false;
    bool closed = false;
    uint32_t ncarry = 0;     // hit ends of this stream held in the device carry
};

struct ClassInfo {
    int W = 1, P = 1;
    uint32_t tile_first = 0, ntiles = 0;
    int lds = 1;       // match masks: 0 image through L1/L2, 1 image in LDS
    bool cut = false;  // word-cutoff scan variant
    int waves = 4;     // wavefronts per block (each scans one chunk)
};

}  // namespace

struct oasm_ctx {
    std::mutex mu;
    int device = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    uint32_t rules = OASM_RULES_PAPER;
    oasm_config cfg{};
    std::string err;
    bool poisoned = false;

    // dictionary
    uint32_t npat = 0;
    std::vector<uint16_t> m, k;
    uint32_t mmax = 0, kmax = 0, hks = 1, lookback = 0, nclass = 1;
    uint8_t class_of[256];
    uint64_t dict_fp = 0;  // dictionary, thresholds, rules and classes (checkpoints)
    uint64_t msum = 0;   // sum of pattern lengths (cells per byte)
    uint64_t wsum = 0;   // sum of 32-bit words (word-steps per byte)
    std::vector<ClassInfo> classes;
    uint32_t ntiles = 0;
    std::vector<uint8_t> h_patbytes;  // host copies for rebuilding tiles
    std::vector<PatDesc> h_pd;
    uint64_t rpeq_words = 0;
    size_t max_lds = 64 * 1024;       // dynamic LDS a block may use on this device
    double chunk_scale = 1.0;         // scale of the chunk-size rule (autotuned)
    std::string tune_log;             // choices made by the autotuner
    DevBuf d_pats, d_slot_pat, d_tiles, d_peq, d_rpeq, d_class, d_patbytes, d_pat_tile, d_pat_slot, d_tile_wp;
    std::vector<uint32_t> class_w32;  // per pattern: words

    // streams
    std::unordered_map<uint64_t, uint32_t> slot_of;
    std::vector<uint32_t> free_slots;      // slots of finished streams, for reuse
    std::unordered_set<uint64_t> closed_ids;  // ids of finished streams (feeds to them are refused)
    std::vector<StreamState> streams;

    // step buffers
    DevBuf plan, offsets, item_rec, item_cnt, ctl, scan_tmp, sort_key, sort_val, sort_end, sort_tmp;
    DevBuf r_pat, r_sl, r_end, r_flag, r_dist, r_hk, seg_cnt, seg_off, carry_flag, carry_off, long_list;
    DevBuf seg_out, occ_out, raw_in;
    // the parallel walk of long filter segments: descriptors and one slot per
    // start (cap_long slots, grown when a step asks for more)
    DevBuf long_desc, long_next, long_jump[2];
    // Hit ends of filter segments that may still grow, for every stream,
    // resident on the device between steps (double-buffered: read one,
    // write the other).  Order: (step-local stream, pattern, end) of the
    // step that wrote them.
    DevBuf carry_buf[2], carry_hk_buf[2];
    int carry_cur = 0;
    uint32_t ncarry = 0;
    PinBuf pin_plan, pin_ctl, pin_out[2], pin_feed;  // results: two buffers, so that a step's results
                                                     // can be read while the next step runs
    size_t pin_feed_used = 0;
    uint32_t cap = 256;         // records per scan item
    uint32_t cap_n = 1u << 16;  // hit ends per step (carried + new)
    uint32_t cap_occ = 1u << 16;
    uint32_t cap_carry = 1u << 12;
    uint32_t cap_long = 0;  // per-start slots of the parallel filter walk
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
    hipEvent_t ev_seg = nullptr;  // after the last upload from pin_seg
    bool seg_pending = false;
    // captured launch sequence of the last repeated step shape
    hipGraphExec_t graph_a = nullptr, graph_b = nullptr;
    std::vector<uint64_t> graph_key, graph_prev_key;

    // results
    HitQueue q_raw;
    OccQueue q_occ, q_h;
    size_t rd_raw = 0, rd_occ = 0, rd_h = 0;

    oasm_stats stats{};
    uint64_t staged_bytes = 0;   // staging capacity held by open streams
    uint64_t pending_bytes = 0;  // fed, not yet matched
    PinBuf pin_seg;
    DevBuf d_seg;

    // LEV CALC (K4) tables, built on first use: pattern ids grouped by word
    // count, and per pattern the sum of (2K + 1) over the patterns before it.
    DevBuf d_lc_ids, d_lc_unit;
    struct LcGroup {
        int W;
        uint32_t first, count;
    };
    std::vector<LcGroup> lc_groups;
    uint64_t lc_unit_total = 0;
    hipEvent_t ev_lc = nullptr;  // after the last LEV CALC launch (on the caller's stream)
    uint8_t *lc_scratch = nullptr;  // this device's table array of oasm_levcalc_noalloc

    // Staging buffers of closed streams, kept for reuse.  Every byte of them
    // was written by this context (cleared at allocation, then mapped
    // symbols), so they hold valid symbol classes only.
    std::multimap<size_t, uint8_t *> pool;  // released staging buffers by capacity
    std::vector<uint8_t *> slabs;           // staging slabs, each cleared once when allocated
    std::unordered_set<uint8_t *> own_alloc;  // staging buffers with an allocation of their own
    uint8_t *slab_cur = nullptr;            // unused part of the newest slab
    size_t slab_left = 0;
    std::vector<StagingMove> moves;         // queued staging moves (launched by flush_moves)
    std::vector<std::pair<uint8_t *, size_t>> move_release;  // buffers the queued moves read
    // While a launched step has not been waited for (the serving loop admits
    // segments meanwhile), buffers that it may read are held back from the
    // pool: a re-run of the step after a capacity overflow reads them again.
    bool hold_release = false;
    std::vector<std::pair<uint8_t *, size_t>> held;
};

namespace {

oasm_status fail(oasm_ctx *c, oasm_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

oasm_status device_fail(oasm_ctx *c, const HipFail &f) {
    if (c) {
        c->poisoned = true;
        c->err = std::string(f.what) + ": " + hipGetErrorString(f.e);
    }
    return OASM_E_DEVICE;
}

// A host allocation that fails inside a matching step leaves the step half
// applied (stream bookkeeping, queued moves, result queues): the context is
// poisoned as after a device error.
oasm_status step_alloc_fail(oasm_ctx *c) {
    c->poisoned = true;
    c->err = "host allocation failed during a matching step; the context is poisoned";
    return OASM_E_NOMEM;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// hipStreamSynchronize, with the blocked time added to the context's stats
void wait_stream(oasm_ctx *c, const char *what);

uint8_t *acquire_staging(oasm_ctx *c, size_t need, size_t &cap);
void flush_moves(oasm_ctx *c, hipStream_t st);
void release_staging(oasm_ctx *c, uint8_t *p, size_t cap);

void wait_stream(oasm_ctx *c, const char *what) {
    const double t0 = now_ms();
    ck(hipStreamSynchronize(c->st), what);
    c->stats.wait_ms += now_ms() - t0;
}

void drop_graphs(oasm_ctx *c) {
    if (c->graph_a) (void)hipGraphExecDestroy(c->graph_a);
    if (c->graph_b) (void)hipGraphExecDestroy(c->graph_b);
    c->graph_a = c->graph_b = nullptr;
    c->graph_key.clear();
}

uint32_t pow2_at_least(uint64_t v) {
    uint32_t r = 1;
    while (r < v && r < (1u << 31)) r <<= 1;
    return r;
}

// ------------------------------------------------------------------ plan
struct StepPlan {
    std::vector<uint32_t> locals;  // stream indices (ctx->streams) in step order
    std::vector<ChunkDesc> chunks;
    std::vector<StreamDesc> sdesc;
    std::vector<uint32_t> slot_to_local;
    uint64_t bytes = 0;
};

template <class T>
size_t put(std::vector<uint8_t> &blob, const std::vector<T> &v) {
    size_t off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

uint32_t choose_chunk(oasm_ctx *c, uint64_t bytes) {
    if (c->cfg.chunk_bytes) return std::max<uint32_t>(64, c->cfg.chunk_bytes & ~63u);
    // enough work items to fill 256 CUs several times over, at most 64 KiB;
    // both scaled by the autotuned factor (0.5, 1 or 2); and a chunk is at
    // least four look-backs long (so the look-back adds at most a quarter)
    const uint64_t target_items = 16384;
    const double sc = c->chunk_scale;
    uint64_t per = (uint64_t)((double)bytes * std::max<uint32_t>(1, c->ntiles) / target_items * sc);
    per = std::min<uint64_t>(per, (uint64_t)(65536 * sc));
    per = std::max<uint64_t>(per, std::max<uint64_t>(256, 4ull * c->lookback));
    return (uint32_t)((per + 63) & ~63ull);
}

// `which` lists the streams matched in this step.  Every other stream that
// holds carried hit ends joins with no new bytes and as not closing, so its
// open segments pass through the step unchanged.
void build_plan(oasm_ctx *c, const std::vector<uint32_t> &which_in, StepPlan &pl) {
    std::vector<uint32_t> which = which_in;
    std::vector<char> target(c->streams.size(), 0);
    for (uint32_t si : which_in) target[si] = 1;
    for (uint32_t si = 0; si < c->streams.size(); ++si)
        if (!target[si] && c->streams[si].ncarry > 0) which.push_back(si);
    // step-local order = stream id order: the step's records are sorted by
    // (step-local stream, pattern, position), which the drain promises as
    // (stream id, pattern, position); slots of finished streams are reused
    // in any order
    std::sort(which.begin(), which.end(),
              [c](uint32_t a, uint32_t b) { return c->streams[a].id < c->streams[b].id; });
    uint64_t total_new = 0;
    for (uint32_t si : which_in) total_new += c->streams[si].valid - c->streams[si].scanned;
    const uint32_t C = choose_chunk(c, total_new);
    pl.slot_to_local.assign(c->streams.size(), 0xFFFFFFFFu);
    for (uint32_t si : which) {
        StreamState &s = c->streams[si];
        const uint32_t local = (uint32_t)pl.locals.size();
        pl.locals.push_back(si);
        pl.slot_to_local[s.slot] = local;
        const uint64_t pend = target[si] ? s.valid - s.scanned : 0;
        const uint64_t nch = (pend + C - 1) / C;
        for (uint64_t j = 0; j < nch; ++j) {
            const uint64_t e0 = s.scanned + j * C;  // staging index of the first reported end
            const uint64_t e1 = std::min<uint64_t>(s.valid, e0 + C);
            uint64_t st0 = e0 >= c->lookback ? e0 - c->lookback : 0;
            st0 &= ~uint64_t(3);
            ChunkDesc cd;
            cd.sym = s.sym + st0;
            cd.abs_first = s.base_abs + e0;
            cd.scan_len = (uint32_t)(e1 - st0);
            cd.lookback = (uint32_t)(e0 - st0);
            cd.stream_local = local;
            cd.pad = 0;
            pl.chunks.push_back(cd);
        }
        StreamDesc sd;
        sd.sym = s.sym;
        sd.base_abs = s.base_abs;
        sd.frontier = s.base_abs + (target[si] ? s.valid : s.scanned);
        sd.closed = target[si] && s.close_pending ? 1u : 0u;
        sd.slot = s.slot;
        pl.sdesc.push_back(sd);
        pl.bytes += pend;
    }
}

// ------------------------------------------------------------------ step
// One matching step, from its launch to its results.  run_step runs the four
// parts back to back; the serving loop launches the next step before it
// converts this one's results (and admits new arrivals while a step runs).
struct StepRun {
    bool active = false;
    StepPlan pl;
    std::vector<uint32_t> which;     // streams with new bytes (ctx->streams indices)
    std::vector<uint64_t> scan_to;   // per `which` entry: absolute end of its symbols matched by this step
    std::vector<char> closing;       // per `which` entry: the stream ends with this step
    std::vector<uint64_t> ids;       // per step-local stream: the stream id
    // fixed at launch (a re-run after a capacity overflow reuses them)
    size_t o_chunks = 0, o_sdesc = 0, o_s2l = 0;
    uint32_t nchunks = 0, ncarry = 0, key_bits = 0;
    int cin = 0, cout = 1, pin = 0;
    bool keep_raw = true, keep_h = false;
    // from the completed step
    PackArgs layout{};
    uint32_t n_new = 0, nocc = 0, ncarry_out = 0;
};

// host time since the last mark, excluding device waits, into phase ph
// A named range in a trace taken with rocprofv3 --marker-trace (roctx);
// without a tool attached a push or pop is a call that returns at once.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// A host phase of a step: its time (less the time spent waiting for the
// device) goes into the statistics, and it is a named trace range.
struct PhaseClock {
    TraceRange range;
    oasm_ctx *c;
    double tmark, twait0;
    PhaseClock(oasm_ctx *cc, const char *name) : range(name), c(cc), tmark(now_ms()), twait0(cc->stats.wait_ms) {}
    void operator()(int ph) {
        const double t = now_ms();
        c->stats.host_ms[ph] += (t - tmark) - (c->stats.wait_ms - twait0);
        tmark = t;
        twait0 = c->stats.wait_ms;
    }
};

// Queue one attempt of the step's launch sequence (buffers sized by the
// context's current capacities), ending with ev2.
void step_enqueue(oasm_ctx *c, StepRun &r) {
    hipStream_t st = c->st;
    uint8_t *pb = c->plan.as<uint8_t>();
    const ChunkDesc *d_chunks = reinterpret_cast<const ChunkDesc *>(pb + r.o_chunks);
    const StreamDesc *d_sdesc = reinterpret_cast<const StreamDesc *>(pb + r.o_sdesc);
    const uint32_t *d_s2l = reinterpret_cast<const uint32_t *>(pb + r.o_s2l);
    const uint32_t nchunks = r.nchunks, ncarry = r.ncarry, key_bits = r.key_bits;
    const int cin = r.cin, cout = r.cout;
    const CarryRec *d_carry = c->carry_buf[cin].as<CarryRec>();
    const uint8_t *d_carry_hk = c->carry_hk_buf[cin].as<uint8_t>();
    uint32_t *ctl = c->ctl.as<uint32_t>();
    const uint64_t nitems = (uint64_t)nchunks * c->ntiles;
    const uint32_t hks = c->hks;
    const uint32_t out_stride = c->kmax + 1;
    const uint32_t rules = c->rules;
    const bool keep_any_raw = r.keep_raw || r.keep_h;
    PinBuf &pin_out = c->pin_out[r.pin];

    const uint32_t cap_n = c->cap_n, cap_occ = c->cap_occ, cap_carry = c->cap_carry;
    const uint64_t n1 = cap_n;
    c->item_rec.ensure(std::max<uint64_t>(1, nitems) * c->cap * 4, st);
    c->scan_tmp.ensure(std::max<size_t>(scan_tmp_words(std::max<uint64_t>({nitems, n1, 1})) * 4, 1024), st);
    c->sort_key.ensure(n1 * 8, st);  // two halves: ping-pong
    c->sort_val.ensure(n1 * 8, st);
    c->sort_end.ensure(n1 * 8, st);
    c->sort_tmp.ensure(sort_tmp_words((uint32_t)n1) * 4, st);
    c->r_pat.ensure(n1 * 4, st);
    c->r_sl.ensure(n1 * 4, st);
    c->r_end.ensure(n1 * 8, st);
    c->r_flag.ensure(n1, st);
    c->r_dist.ensure(n1, st);
    c->r_hk.ensure(n1 * hks, st);
    c->seg_cnt.ensure(n1 * 4, st);
    c->seg_off.ensure(n1 * 4, st);
    c->carry_flag.ensure(n1 * 4, st);
    c->carry_off.ensure(n1 * 4, st);
    c->long_list.ensure(filter_long_list_words((uint32_t)n1) * 4, st);
    c->long_desc.ensure(filter_long_list_words((uint32_t)n1) * sizeof(LongDesc), st);
    if (c->cap_long) {
        c->long_next.ensure((size_t)c->cap_long * 4, st);
        c->long_jump[0].ensure((size_t)c->cap_long * 4, st);
        c->long_jump[1].ensure((size_t)c->cap_long * 4, st);
    }
    c->seg_out.ensure(n1 * out_stride * sizeof(OccRec), st);
    c->occ_out.ensure((uint64_t)cap_occ * sizeof(OccRec), st);
    c->carry_buf[cout].ensure((uint64_t)cap_carry * sizeof(CarryRec), st);
    c->carry_hk_buf[cout].ensure((uint64_t)cap_carry * hks, st);

    // layout of the mapped pinned results buffer, by capacity
    PackArgs pk{};
    {
        size_t off = 0;
        auto region = [&](size_t bytes) {
            const size_t o = (off + 255) & ~size_t(255);
            off = o + bytes;
            return (uint64_t)o;
        };
        pk.o_ctl = region(64);
        pk.o_pat = region(keep_any_raw ? n1 * 4 : 0);
        pk.o_sl = region(keep_any_raw ? n1 * 4 : 0);
        pk.o_end = region(keep_any_raw ? n1 * 8 : 0);
        pk.o_flag = region(keep_any_raw ? n1 : 0);
        pk.o_dist = region(keep_any_raw ? n1 : 0);
        pk.o_hk = region(r.keep_h ? n1 * hks : 0);
        pk.o_occ = region((size_t)cap_occ * sizeof(OccRec));
        pk.o_cr = region((size_t)cap_carry * sizeof(CarryRec));
        pin_out.ensure(off + 256, st);
    }
    void *dev_host = nullptr;
    ck(hipHostGetDevicePointer(&dev_host, pin_out.p, 0), "mapped results buffer");

    // The step's launch sequence in two parts (the scan, then everything
    // after it), with the scan-timing event between them.
    auto part_a = [&]() {
        ck(launch_fill_u32(ctl, 0, 16, st), "fill ctl");
        uint32_t item_base = 0;
        for (const ClassInfo &ci : c->classes) {
            ScanArgs a;
            a.chunks = d_chunks;
            a.nchunks = nchunks;
            a.tiles = c->d_tiles.as<TileDesc>();
            a.tile_first = ci.tile_first;
            a.ntiles = ci.ntiles;
            a.peq_img = c->d_peq.as<uint32_t>();
            a.slot_pat = c->d_slot_pat.as<uint32_t>();
            a.pats = c->d_pats.as<PatDesc>();
            a.nclass = c->nclass;
            a.item_rec = c->item_rec.as<uint32_t>();
            a.item_cnt = c->item_cnt.as<uint32_t>();
            a.item_base = item_base;
            a.cap = c->cap;
            a.max_cnt = ctl + 0;
            a.wsteps = reinterpret_cast<unsigned long long *>(ctl + 8);
            ck(launch_scan(ci.W, ci.P, ci.cut, a, ci.waves, ci.lds, st), "scan launch");
            item_base += nchunks * ci.ntiles;
            c->stats.scan_launches++;
        }
    };
    LongWalk lw;
    lw.desc = c->long_desc.as<LongDesc>();
    lw.next = c->cap_long ? c->long_next.as<uint32_t>() : nullptr;
    lw.jump[0] = c->cap_long ? c->long_jump[0].as<uint32_t>() : nullptr;
    lw.jump[1] = c->cap_long ? c->long_jump[1].as<uint32_t>() : nullptr;
    lw.cap_next = c->cap_long;
    lw.can_grow = c->cap_long < kLongSlotsMax ? 1u : 0u;
    lw.res = reinterpret_cast<unsigned long long *>(ctl + 10);
    lw.err = ctl + 5;
    auto part_b = [&]() {
        const DevN items{nullptr, (uint32_t)nitems, (uint32_t)nitems, nullptr, 0u};
        ck(launch_exclusive_scan(c->item_cnt.as<uint32_t>(), c->offsets.as<uint32_t>(), items, ctl + 1,
                                 c->scan_tmp.as<uint32_t>(), st),
           "item count scan");
        const DevN dn{ctl + 1, ncarry, cap_n, ctl + 0, c->cap};  // carried + new hit ends
        uint32_t *key0 = c->sort_key.as<uint32_t>(), *key1 = key0 + n1;
        uint32_t *val0 = c->sort_val.as<uint32_t>(), *val1 = val0 + n1;
        ck(launch_place_carry(d_carry, std::min(ncarry, cap_n), d_s2l, c->npat, key0, val0, c->sort_end.as<uint64_t>(),
                              st),
           "place carry");
        ClassItems cls{};
        for (const ClassInfo &ci : c->classes) {
            if (cls.n == (uint32_t)kMaxClasses) throw HipFail{hipErrorInvalidValue, "more word-count classes than 8"};
            cls.tile_first[cls.n] = ci.tile_first;
            cls.ntiles[cls.n] = ci.ntiles;
            cls.item_base[cls.n] = cls.n ? cls.item_base[cls.n - 1] + nchunks * cls.ntiles[cls.n - 1] : 0u;
            ++cls.n;
        }
        ck(launch_compact_raw(d_chunks, nchunks, c->d_tiles.as<TileDesc>(), cls, c->d_slot_pat.as<uint32_t>(),
                              c->item_rec.as<uint32_t>(), c->item_cnt.as<uint32_t>(), c->offsets.as<uint32_t>(),
                              c->cap, ncarry, cap_n, c->npat, key0, val0, c->sort_end.as<uint64_t>(), st),
           "compact hit ends");
        bool second = false;
        ck(launch_radix_sort(key0, val0, key1, val1, dn, key_bits, c->sort_tmp.as<uint32_t>(), st, second),
           "radix sort");
        ck(launch_gather_raw(second ? key1 : key0, second ? val1 : val0, dn, c->npat, ncarry,
                             c->sort_end.as<uint64_t>(), d_carry, d_carry_hk, hks, c->r_pat.as<uint32_t>(),
                             c->r_sl.as<uint32_t>(), c->r_end.as<uint64_t>(), c->r_flag.as<uint8_t>(),
                             c->r_dist.as<uint8_t>(), c->r_hk.as<uint8_t>(), st),
           "gather hit ends");
        ck(launch_recover(c->r_pat.as<uint32_t>(), c->r_sl.as<uint32_t>(), c->r_end.as<uint64_t>(),
                          c->r_flag.as<uint8_t>(), dn, c->d_pats.as<PatDesc>(), c->d_rpeq.as<uint64_t>(), d_sdesc,
                          c->nclass, hks, c->r_hk.as<uint8_t>(), c->r_dist.as<uint8_t>(), ctl + 4, st),
           "recover");
        ck(launch_filter(c->r_pat.as<uint32_t>(), c->r_sl.as<uint32_t>(), c->r_end.as<uint64_t>(),
                         c->r_hk.as<uint8_t>(), dn, hks, c->d_pats.as<PatDesc>(), d_sdesc, rules, out_stride,
                         c->seg_out.as<OccRec>(), c->seg_cnt.as<uint32_t>(), c->carry_flag.as<uint32_t>(),
                         c->long_list.as<uint32_t>(), ctl + 6, lw, st),
           "filter");
        ck(launch_exclusive_scan(c->seg_cnt.as<uint32_t>(), c->seg_off.as<uint32_t>(), dn, ctl + 2,
                                 c->scan_tmp.as<uint32_t>(), st),
           "occ scan");
        ck(launch_exclusive_scan(c->carry_flag.as<uint32_t>(), c->carry_off.as<uint32_t>(), dn, ctl + 3,
                                 c->scan_tmp.as<uint32_t>(), st),
           "carry scan");
        ck(launch_compact_occ(c->seg_out.as<OccRec>(), c->seg_cnt.as<uint32_t>(), c->seg_off.as<uint32_t>(), dn,
                              out_stride, c->occ_out.as<OccRec>(), cap_occ, st),
           "compact occ");
        ck(launch_compact_carry(c->r_pat.as<uint32_t>(), c->r_sl.as<uint32_t>(), c->r_end.as<uint64_t>(),
                                c->r_dist.as<uint8_t>(), c->r_hk.as<uint8_t>(), hks, c->carry_flag.as<uint32_t>(),
                                c->carry_off.as<uint32_t>(), d_sdesc, dn, c->carry_buf[cout].as<CarryRec>(),
                                c->carry_hk_buf[cout].as<uint8_t>(), cap_carry, st),
           "compact carry");
        pk.ctl = ctl;
        pk.n = dn;
        pk.r_pat = c->r_pat.as<uint32_t>();
        pk.r_sl = c->r_sl.as<uint32_t>();
        pk.r_end = c->r_end.as<uint64_t>();
        pk.r_flag = c->r_flag.as<uint8_t>();
        pk.r_dist = c->r_dist.as<uint8_t>();
        pk.r_hk = c->r_hk.as<uint8_t>();
        pk.hks = hks;
        pk.with_raw = keep_any_raw ? 1u : 0u;
        pk.with_hk = r.keep_h ? 1u : 0u;
        pk.occ = c->occ_out.as<OccRec>();
        pk.cap_occ = cap_occ;
        pk.carry = c->carry_buf[cout].as<CarryRec>();
        pk.cap_carry = cap_carry;
        pk.host = reinterpret_cast<uint8_t *>(dev_host);
        ck(launch_pack_results(pk, st), "pack results");
    };
    // Replay captured graphs when this step has the same shape (every kernel
    // argument and buffer) as the last; capture when a shape repeats.
    std::vector<uint64_t> gkey;
    if (c->cfg.flags & OASM_CFG_GRAPHS) {
        gkey = {nchunks, ncarry, c->cap, cap_n, cap_occ, cap_carry, key_bits, (uint64_t)r.pl.locals.size(),
                (uint64_t)(uintptr_t)c->plan.p, r.o_chunks, r.o_sdesc, r.o_s2l, (uint64_t)cin,
                (uint64_t)(uintptr_t)c->item_rec.p, (uint64_t)(uintptr_t)c->scan_tmp.p,
                (uint64_t)(uintptr_t)c->sort_key.p, (uint64_t)(uintptr_t)c->sort_tmp.p,
                (uint64_t)(uintptr_t)c->seg_out.p, (uint64_t)(uintptr_t)c->occ_out.p,
                (uint64_t)(uintptr_t)c->carry_buf[cin].p, (uint64_t)(uintptr_t)c->carry_buf[cout].p,
                (uint64_t)(uintptr_t)c->r_hk.p, (uint64_t)(uintptr_t)pin_out.p, (uint64_t)keep_any_raw,
                (uint64_t)r.keep_h, (uint64_t)c->cap_long, (uint64_t)(uintptr_t)c->long_next.p,
                (uint64_t)(uintptr_t)c->long_jump[0].p, (uint64_t)(uintptr_t)c->long_jump[1].p,
                (uint64_t)(uintptr_t)c->long_desc.p};
    }
    if (!gkey.empty() && gkey == c->graph_key && c->graph_a) {
        ck(hipEventRecord(c->ev0, st), "event");
        ck(hipGraphLaunch(c->graph_a, st), "graph launch");
        ck(hipEventRecord(c->ev1, st), "event");
        ck(hipGraphLaunch(c->graph_b, st), "graph launch");
        c->stats.scan_launches += c->classes.size();
        c->stats.graph_replays++;
    } else if (!gkey.empty() && gkey == c->graph_prev_key) {
        drop_graphs(c);
        hipGraph_t ga = nullptr, gb = nullptr;
        ck(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
        part_a();
        ck(hipStreamEndCapture(st, &ga), "end capture");
        ck(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
        part_b();
        ck(hipStreamEndCapture(st, &gb), "end capture");
        ck(hipGraphInstantiate(&c->graph_a, ga, nullptr, nullptr, 0), "graph instantiate");
        ck(hipGraphInstantiate(&c->graph_b, gb, nullptr, nullptr, 0), "graph instantiate");
        ck(hipGraphDestroy(ga), "graph destroy");
        ck(hipGraphDestroy(gb), "graph destroy");
        c->graph_key = gkey;
        ck(hipEventRecord(c->ev0, st), "event");
        ck(hipGraphLaunch(c->graph_a, st), "graph launch");
        ck(hipEventRecord(c->ev1, st), "event");
        ck(hipGraphLaunch(c->graph_b, st), "graph launch");
    } else {
        ck(hipEventRecord(c->ev0, st), "event");
        part_a();
        ck(hipEventRecord(c->ev1, st), "event");
        part_b();
    }
    ck(hipEventRecord(c->ev2, st), "event");
    c->graph_prev_key = gkey;
    r.layout = pk;
}

// Plan the step over `which` (plus the streams holding carried hit ends),
// upload the plan and queue the launch sequence.  Returns without waiting.
void step_launch(oasm_ctx *c, const std::vector<uint32_t> &which, StepRun &r, int pin) {
    hipStream_t st = c->st;
    PhaseClock phase(c, "oasm step launch");
    r = StepRun{};
    r.which = which;
    r.pin = pin;
    build_plan(c, which, r.pl);
    if ((uint64_t)r.pl.locals.size() * c->npat >= (1ull << 32))
        throw HipFail{hipErrorInvalidValue, "step too large (streams x patterns exceed 2^32)"};
    r.ids.resize(r.pl.locals.size());
    for (size_t l = 0; l < r.pl.locals.size(); ++l) r.ids[l] = c->streams[r.pl.locals[l]].id;
    r.scan_to.resize(which.size());
    r.closing.resize(which.size());
    for (size_t k = 0; k < which.size(); ++k) {
        r.scan_to[k] = c->streams[which[k]].base_abs + c->streams[which[k]].valid;
        r.closing[k] = c->streams[which[k]].close_pending ? 1 : 0;
    }

    // upload the plan in one copy
    std::vector<uint8_t> blob;
    r.o_chunks = put(blob, r.pl.chunks);
    r.o_sdesc = put(blob, r.pl.sdesc);
    r.o_s2l = put(blob, r.pl.slot_to_local);
    blob.resize(blob.size() + 16);
    c->pin_plan.ensure(blob.size(), st);
    wait_stream(c, "sync before plan upload");  // the pinned plan of the last step may still be read
    std::memcpy(c->pin_plan.p, blob.data(), blob.size());
    c->plan.ensure(blob.size(), st);
    ck(hipMemcpyAsync(c->plan.p, c->pin_plan.p, blob.size(), hipMemcpyHostToDevice, st), "plan upload");
    phase(0);
    r.nchunks = (uint32_t)r.pl.chunks.size();
    r.ncarry = c->ncarry;
    r.cin = c->carry_cur;
    r.cout = 1 - c->carry_cur;
    c->carry_buf[r.cin].ensure(std::max<uint32_t>(r.ncarry, 1) * sizeof(CarryRec), st);
    c->carry_hk_buf[r.cin].ensure(std::max<uint32_t>(r.ncarry, 1) * (uint64_t)c->hks, st);
    // control words: [0] max item count, [1] new hit ends, [2] occurrences, [3] carried, [4] recovery
    // errors, [6] long filter segments, [8..9] word-steps (all cleared at the step's start)
    c->ctl.ensure(64, st);
    c->pin_ctl.ensure(64, st);
    const uint64_t nitems = (uint64_t)r.nchunks * c->ntiles;
    while (r.key_bits < 32 && ((uint64_t)1 << r.key_bits) < (uint64_t)r.pl.locals.size() * c->npat) ++r.key_bits;
    c->item_cnt.ensure(std::max<uint64_t>(1, nitems) * 4, st);
    c->offsets.ensure(std::max<uint64_t>(1, nitems) * 4, st);
    r.keep_raw = !(c->cfg.flags & OASM_CFG_NO_RAW);
    r.keep_h = (c->cfg.flags & OASM_CFG_KEEP_H) != 0;
    // The whole step is queued at once: every kernel after the scan reads its
    // size from device memory and the buffers are sized by capacities that
    // grow (and the step runs again) when a count exceeds them.
    step_enqueue(c, r);
    r.active = true;
    c->hold_release = true;
    phase(1);
}

// Wait for the step; when a count exceeded its capacity, grow the capacity
// and run the step again (synchronously) until everything fits.
void step_wait(oasm_ctx *c, StepRun &r) {
    PhaseClock phase(c, "oasm step wait");
    for (;;) {
        const double t0 = now_ms();
        ck(hipEventSynchronize(c->ev2), "step sync");
        c->stats.wait_ms += now_ms() - t0;
        const uint32_t *h = reinterpret_cast<const uint32_t *>(c->pin_out[r.pin].as<uint8_t>() + r.layout.o_ctl);
        r.n_new = h[1];
        r.nocc = h[2];
        r.ncarry_out = h[3];
        const uint64_t n_all = (uint64_t)r.ncarry + r.n_new;
        bool again = false;
        if (h[0] > c->cap) {  // a scan item overflowed its record buffer
            c->cap = pow2_at_least(h[0]);
            again = true;
        }
        if (n_all > c->cap_n) {
            c->cap_n = pow2_at_least(2 * n_all);
            again = true;
        }
        if (!again && r.nocc > c->cap_occ) {
            c->cap_occ = pow2_at_least(2ull * r.nocc);
            again = true;
        }
        if (!again && r.ncarry_out > c->cap_carry) {
            c->cap_carry = pow2_at_least(2ull * r.ncarry_out);
            again = true;
        }
        // long filter segments that did not get their per-start slots
        const uint64_t long_slots = (uint64_t)h[10] | ((uint64_t)(h[11] & 0xFFu) << 32);
        if (!again && long_slots > c->cap_long && c->cap_long < kLongSlotsMax) {
            c->cap_long = (uint32_t)std::min<uint64_t>(kLongSlotsMax, pow2_at_least(long_slots));
            again = true;
        }
        if (again) {
            step_enqueue(c, r);
            continue;
        }
        if (h[4]) throw HipFail{hipErrorUnknown, "internal: recovery found no hit-set record at a scan hit end"};
        if (h[5]) throw HipFail{hipErrorUnknown, "internal: a filter walk emitted more often than its segment has ends"};
        c->stats.word_steps_done += (uint64_t)h[8] | ((uint64_t)h[9] << 32);
        float ms = 0;
        if (hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) c->stats.scan_ms += ms;
        if (hipEventElapsedTime(&ms, c->ev0, c->ev2) == hipSuccess) c->stats.step_ms += ms;
        break;
    }
    phase(1);
}

// After the step: the carried hit ends stay on the device (the host keeps
// per-stream counts); every matched stream records how far it is matched
// (its symbols stay in place until reserve_stream needs the room), and a
// stream that ended is released.
void step_bookkeep(oasm_ctx *c, StepRun &r) {
    PhaseClock phase(c, "oasm step bookkeep");
    hipStream_t st = c->st;
    c->hold_release = false;
    for (auto &h : c->held) release_staging(c, h.first, h.second);
    c->held.clear();
    for (uint32_t si : r.pl.locals) c->streams[si].ncarry = 0;
    const CarryRec *hc = reinterpret_cast<const CarryRec *>(c->pin_out[r.pin].as<uint8_t>() + r.layout.o_cr);
    for (uint32_t i = 0; i < r.ncarry_out; ++i) c->streams[hc[i].stream_slot].ncarry++;
    c->ncarry = r.ncarry_out;
    if (r.ncarry_out) c->carry_cur = r.cout;  // nothing carried: keep the buffers (and the step's shape) as they are
    for (size_t k = 0; k < r.which.size(); ++k) {
        StreamState &s = c->streams[r.which[k]];
        // scan_to is absolute: a compaction queued while the step ran may
        // have shifted the buffer's indices
        const uint64_t upto = r.scan_to[k] - s.base_abs;
        const uint64_t done = upto - s.scanned;
        c->stats.bytes_scanned += done;
        c->pending_bytes -= done;
        s.scanned = upto;
        if (r.closing[k]) {
            // finished (no feed is accepted after a close): a closed stream
            // carries nothing (its filter segments all completed in this
            // step), so its slot is free for reuse
            s.close_pending = false;
            s.closed = true;
            c->staged_bytes -= s.cap;
            release_staging(c, s.sym, s.cap);
            s.sym = nullptr;
            s.cap = 0;
            s.valid = s.scanned = 0;
            c->closed_ids.insert(s.id);
            c->slot_of.erase(s.id);
            c->free_slots.push_back(s.slot);
            continue;
        }
        // the matched symbols stay in place: reserve_stream reclaims them
        // when the buffer needs room
    }
    flush_moves(c, st);
    c->stats.raw_hits += r.n_new;
    c->stats.occurrences += r.nocc;
    c->stats.syncs++;
    c->pin_feed_used = 0;
    phase(3);
}

// The step's results (in its mapped pinned buffer) into the drain queues.
void step_convert(oasm_ctx *c, StepRun &r) {
    PhaseClock phase(c, "oasm step convert");
    const uint32_t n = r.ncarry + r.n_new;
    uint8_t *hp = c->pin_out[r.pin].as<uint8_t>();
    const PackArgs &ly = r.layout;
    const uint32_t *hpat = reinterpret_cast<const uint32_t *>(hp + ly.o_pat);
    const uint32_t *hsl = reinterpret_cast<const uint32_t *>(hp + ly.o_sl);
    const uint64_t *hend = reinterpret_cast<const uint64_t *>(hp + ly.o_end);
    const uint8_t *hflag = hp + ly.o_flag;
    const uint8_t *hdist = hp + ly.o_dist;
    const uint8_t *hhk = hp + ly.o_hk;
    const uint32_t hks = c->hks;
    // (a record with its flag set was carried from an earlier step and
    // reported there)
    if (r.keep_raw) convert_raw(hflag, hsl, hend, hpat, hdist, r.ids.data(), n, c->q_raw);
    if (r.keep_h) {
        for (uint32_t i = 0; i < n; ++i) {
            if (hflag[i]) continue;
            const uint64_t sid = r.ids[hsl[i]];
            const uint32_t p = hpat[i];
            const int m = c->m[p], K = c->k[p];
            for (int l = std::max(1, m - K); l <= m + K; ++l) {
                const uint8_t kk = hhk[(size_t)i * hks + (l - (m - K))];
                if (kk == kNoHit) continue;
                c->q_h.push_back(oasm_occ{sid, hend[i] + 1 - (uint64_t)l, p, (uint32_t)l, kk, 0});
                c->stats.h_records++;
            }
        }
    }
    convert_occ(reinterpret_cast<const OccRec *>(hp + ly.o_occ), r.ids.data(), r.nocc, c->q_occ);
    r.active = false;
    phase(2);
}

void run_step(oasm_ctx *c, const std::vector<uint32_t> &which) {
    StepRun r;
    step_launch(c, which, r, 0);
    step_wait(c, r);
    step_bookkeep(c, r);
    step_convert(c, r);
}

void sort_h_queue_tail(oasm_ctx *c, size_t from) {
    std::stable_sort(c->q_h.begin() + (ptrdiff_t)from, c->q_h.end(), [](const oasm_occ &a, const oasm_occ &b) {
        if (a.stream != b.stream) return a.stream < b.stream;
        if (a.pattern != b.pattern) return a.pattern < b.pattern;
        if (a.start != b.start) return a.start < b.start;
        return a.len < b.len;
    });
}

void sync_all(oasm_ctx *c) {
    std::vector<uint32_t> which;
    for (uint32_t i = 0; i < c->streams.size(); ++i) {
        const StreamState &s = c->streams[i];
        if (s.closed) continue;
        if (s.valid > s.scanned || s.close_pending) which.push_back(i);
    }
    if (which.empty()) return;
    const size_t h0 = c->q_h.size();
    if (c->cfg.flags & OASM_CFG_PLAIN) {
        for (uint32_t si : which) run_step(c, std::vector<uint32_t>{si});
    } else {
        run_step(c, which);
    }
    if (c->cfg.flags & OASM_CFG_KEEP_H) sort_h_queue_tail(c, h0);
}

// A live stream by id, created on first use in a free slot (the caller has
// checked closed_ids: finished streams are not live).
StreamState &get_stream(oasm_ctx *c, uint64_t id, bool create) {
    auto it = c->slot_of.find(id);
    if (it != c->slot_of.end()) return c->streams[it->second];
    if (!create) throw std::out_of_range("stream");
    uint32_t slot;
    if (!c->free_slots.empty()) {
        slot = c->free_slots.back();
        c->free_slots.pop_back();
        c->streams[slot] = StreamState{};
    } else {
        slot = (uint32_t)c->streams.size();
        c->streams.emplace_back();
    }
    StreamState &s = c->streams[slot];
    s.id = id;
    s.slot = slot;
    c->slot_of[id] = slot;
    return s;
}

bool is_finished(const oasm_ctx *c, uint64_t id) { return c->closed_ids.count(id) != 0; }

// Staging buffers up to a quarter slab are carved from slabs of kSlab bytes,
// allocated and cleared once: a new stream then costs neither an allocation
// nor a clear of its own.  Larger ones get an allocation of their own.
constexpr size_t kSlab = size_t(16) << 20;

// A device allocation cleared to class 0 (the scan's last group reads up to
// 8 symbols past a stream's end before masking their ends out: every byte
// must be a valid symbol class).  On failure the pooled buffers that have an
// allocation of their own go back to the device and it tries once more.
uint8_t *alloc_cleared(oasm_ctx *c, size_t bytes) {
    uint8_t *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        ck(hipStreamSynchronize(c->st), "sync before pool release");
        for (auto it = c->pool.begin(); it != c->pool.end();) {
            if (c->own_alloc.erase(it->second)) {
                ck(hipFree(it->second), "hipFree pool");
                it = c->pool.erase(it);
            } else {
                ++it;
            }
        }
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    ck(hipMemsetAsync(p, 0, bytes, c->st), "staging clear");
    return p;
}

// A staging buffer of at least `need` bytes: the smallest pooled one that
// fits, else a piece of a slab, else an allocation of its own.
uint8_t *acquire_staging(oasm_ctx *c, size_t need, size_t &cap) {
    auto it = c->pool.lower_bound(need);
    if (it != c->pool.end()) {
        uint8_t *p = it->second;
        cap = it->first;
        c->pool.erase(it);
        return p;
    }
    const size_t want = (need + 255) & ~size_t(255);
    if (want <= kSlab / 4) {
        if (want > c->slab_left) {
            if (uint8_t *sl = alloc_cleared(c, kSlab)) {
                if (c->slab_left) c->pool.emplace(c->slab_left, c->slab_cur);  // the old slab's rest
                c->slabs.push_back(sl);
                c->slab_cur = sl;
                c->slab_left = kSlab;
            }
        }
        if (want <= c->slab_left) {
            uint8_t *p = c->slab_cur;
            c->slab_cur += want;
            c->slab_left -= want;
            cap = want;
            return p;
        }
    }
    uint8_t *p = alloc_cleared(c, want);
    if (!p) return nullptr;
    c->own_alloc.insert(p);
    cap = want;
    return p;
}

void release_staging(oasm_ctx *c, uint8_t *p, size_t cap) {
    if (p) c->pool.emplace(cap, p);
}

// Launch the queued staging moves, 128 per launch, then give the buffers
// they read back to the pool (their next users are ordered after the moves
// on the stream `st`).
void flush_moves(oasm_ctx *c, hipStream_t st) {
    StagingMoveBatch b;
    for (size_t i = 0; i < c->moves.size(); i += kStagingMovesPerLaunch) {
        const uint32_t n = (uint32_t)std::min<size_t>(kStagingMovesPerLaunch, c->moves.size() - i);
        std::copy(c->moves.begin() + (ptrdiff_t)i, c->moves.begin() + (ptrdiff_t)(i + n), b.m);
        ck(launch_staging_moves(b, n, st), "staging moves");
    }
    c->moves.clear();
    for (auto &r : c->move_release) {
        if (c->hold_release)
            c->held.push_back(r);
        else
            release_staging(c, r.first, r.second);
    }
    c->move_release.clear();
}

// Make room for `n` more symbols in a stream's staging buffer.  With
// `queue`, the copy of the stream's symbols into a new buffer joins the
// queued staging moves (the caller runs flush_moves before anything reads
// the new buffer); otherwise it is a copy of its own.
oasm_status reserve_stream(oasm_ctx *c, StreamState &s, size_t n, bool queue = false) {
    if (s.valid + n + kPad <= s.cap) return OASM_OK;
    // symbols matched before the look-back tail are no longer read: the live
    // part (tail and unmatched symbols) moves to the front of the buffer, or
    // into a larger one
    const size_t keep = std::min<size_t>(s.scanned, c->lookback + 4);
    const size_t drop = s.scanned - keep;
    const size_t live = s.valid - drop;
    // While a launched step may still read this buffer (and, should it
    // overflow a capacity, run again after whatever was queued behind it),
    // its bytes must stay where the step's plan put them: compact into
    // another buffer then, and hold this one until the step is booked.
    const bool in_place = !c->hold_release;
    if (in_place && live + n + kPad <= s.cap) {
        if (live <= UINT32_MAX) {
            c->moves.push_back(StagingMove{s.sym + drop, s.sym, (uint32_t)live, 0});
            if (!queue) flush_moves(c, c->st);
        } else {
            ck(hipMemcpyAsync(s.sym, s.sym + drop, live, hipMemcpyDeviceToDevice, c->st), "staging compaction");
        }
        s.base_abs += drop;
        s.valid -= drop;
        s.scanned -= drop;
        return OASM_OK;
    }
    const size_t want = live + n + kPad <= s.cap ? s.cap : std::max(live + n + kPad, s.cap + s.cap / 2);
    size_t cap = 0;
    uint8_t *p = acquire_staging(c, want, cap);
    if (!p) return fail(c, OASM_E_NOMEM, "hipMalloc for stream staging failed");
    if (s.sym) {
        if (queue && live <= UINT32_MAX) {
            if (live) c->moves.push_back(StagingMove{s.sym + drop, p, (uint32_t)live, 0});
            c->move_release.emplace_back(s.sym, s.cap);  // not reused before the move
        } else {
            if (live) ck(hipMemcpyAsync(p, s.sym + drop, live, hipMemcpyDeviceToDevice, c->st), "staging grow");
            if (c->hold_release)
                c->held.emplace_back(s.sym, s.cap);  // a launched step may still read it
            else
                release_staging(c, s.sym, s.cap);
        }
        s.base_abs += drop;
        s.valid -= drop;
        s.scanned -= drop;
    }
    c->staged_bytes += cap - s.cap;
    s.sym = p;
    s.cap = cap;
    return OASM_OK;
}

// ------------------------------------------------------------------ tiles
struct TileChoice {
    int P = 1;         // patterns per lane
    int lds = 1;       // match masks: 0 image through L1/L2, 1 image in LDS
    bool cut = false;  // word cutoff (P = 1, W >= 2)
    int waves = 4;     // wavefronts per block
};

uint32_t pad_pow2_host(uint32_t x) { return x <= 1 ? 1 : x <= 2 ? 2 : x <= 4 ? 4 : 8; }

// Bytes of one tile's match-mask image: lane-major rows padded to a power of
// two (full columns), or word-major with W words per lane (cutoff tiles).
uint64_t image_bytes(const oasm_ctx *c, int W, int P, bool cut = false) {
    return (uint64_t)c->nclass * 64 * (cut ? (uint32_t)W : pad_pow2_host((uint32_t)(P * W))) * 4;
}

// LDS bytes a block of class (W, P, cut) uses with mask mode `lds`.
uint64_t lds_bytes(const oasm_ctx *c, int W, int P, bool cut, int lds) {
    return lds == 1 ? image_bytes(c, W, P, cut) : 0;
}

// The patterns of one word count, shortest first: neighbouring lanes then
// have similar numbers of wildcard rows, and so similar cutoff depths.
std::vector<uint32_t> class_members(const oasm_ctx *c, int W) {
    std::vector<uint32_t> ids;
    for (uint32_t i = 0; i < c->npat; ++i)
        if ((uint32_t)((c->m[i] + 31) / 32) == (uint32_t)W) ids.push_back(i);
    std::stable_sort(ids.begin(), ids.end(), [c](uint32_t a, uint32_t b) { return c->m[a] < c->m[b]; });
    return ids;
}

// Heuristic without measurement: more patterns per lane for short patterns
// when there are enough of them; the word cutoff for multi-word patterns
// (unless disabled); the image in LDS when it leaves room for two blocks per
// CU.
std::vector<TileChoice> default_choices(const oasm_ctx *c) {
    std::vector<TileChoice> ch(kMaxW32 + 1);
    const bool cut_ok = !(c->cfg.flags & OASM_CFG_NO_CUTOFF);
    for (int W = 1; W <= kMaxW32; ++W) {
        const size_t n = class_members(c, W).size();
        int P = 1;
        if (W == 1) P = n > 128 ? 4 : (n > 64 ? 2 : 1);
        ch[W].cut = cut_ok && W >= 2;
        if (W == 2 && !ch[W].cut) P = n > 64 ? 2 : 1;
        ch[W].P = P;
        ch[W].lds = image_bytes(c, W, P, ch[W].cut) <= 64 * 1024 ? 1 : 0;
        ch[W].waves = 4;
    }
    return ch;
}

// Lay out tiles (64*P patterns of one word count each), upload the tables and
// build the match-mask images on the device.
void build_tiles(oasm_ctx *c, const std::vector<TileChoice> &choice) {
    hipStream_t st = c->st;
    const uint32_t n = c->npat;
    std::vector<TileDesc> tiles;
    std::vector<uint32_t> tile_wp, slot_pat, pat_tile(n), pat_slot(n);
    uint64_t img_words = 0;
    c->classes.clear();
    for (int W = 1; W <= kMaxW32; ++W) {
        const std::vector<uint32_t> ids = class_members(c, W);
        if (ids.empty()) continue;
        const int P = choice[W].P;
        ClassInfo ci;
        ci.W = W;
        ci.P = P;
        ci.tile_first = (uint32_t)tiles.size();
        ci.cut = choice[W].cut && P == 1 && W >= 2;
        ci.lds = choice[W].lds;
        if (lds_bytes(c, W, P, ci.cut, ci.lds) > c->max_lds) ci.lds = 0;
        ci.waves = std::max(1, std::min(choice[W].waves, 4));
        const uint32_t per = 64u * P;
        for (size_t t0 = 0; t0 < ids.size(); t0 += per) {
            TileDesc td;
            td.peq_off = (uint32_t)img_words;
            td.slot_off = (uint32_t)slot_pat.size();
            td.n_active = (uint32_t)std::min<size_t>(per, ids.size() - t0);
            td.pad = 0;
            for (uint32_t s = 0; s < td.n_active; ++s) {
                const uint32_t pid = ids[t0 + s];
                slot_pat.push_back(pid);
                pat_tile[pid] = (uint32_t)tiles.size();
                pat_slot[pid] = s;
            }
            tiles.push_back(td);
            tile_wp.push_back((uint32_t)W | ((uint32_t)P << 8) | (ci.cut ? 1u << 16 : 0u));  // bit 16: low placement
            img_words += image_bytes(c, W, P, ci.cut) / 4;
        }
        ci.ntiles = (uint32_t)tiles.size() - ci.tile_first;
        c->classes.push_back(ci);
    }
    c->ntiles = (uint32_t)tiles.size();
    auto upload = [&](DevBuf &d, const void *src, size_t bytes) {
        d.ensure(std::max<size_t>(bytes, 16), st);
        if (bytes) ck(hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, st), "dictionary upload");
    };
    upload(c->d_patbytes, c->h_patbytes.data(), c->h_patbytes.size());
    upload(c->d_pats, c->h_pd.data(), c->h_pd.size() * sizeof(PatDesc));
    upload(c->d_tiles, tiles.data(), tiles.size() * sizeof(TileDesc));
    upload(c->d_tile_wp, tile_wp.data(), tile_wp.size() * 4);
    upload(c->d_slot_pat, slot_pat.data(), slot_pat.size() * 4);
    upload(c->d_pat_tile, pat_tile.data(), pat_tile.size() * 4);
    upload(c->d_pat_slot, pat_slot.data(), pat_slot.size() * 4);
    upload(c->d_class, c->class_of, 256);
    c->d_peq.ensure(std::max<uint64_t>(img_words * 4, 16), st);
    c->d_rpeq.ensure(std::max<uint64_t>(c->rpeq_words * 8, 16), st);
    ck(launch_fill_u32(c->d_peq.as<uint32_t>(), 0, img_words, st), "fill peq");
    ck(launch_peq_build(c->d_patbytes.as<uint8_t>(), c->d_pats.as<PatDesc>(), n, c->d_pat_tile.as<uint32_t>(),
                        c->d_pat_slot.as<uint32_t>(), c->d_tiles.as<TileDesc>(), c->d_tile_wp.as<uint32_t>(),
                        c->d_class.as<uint8_t>(), c->nclass, c->d_peq.as<uint32_t>(), c->d_rpeq.as<uint64_t>(), st),
       "peq build");
    wait_stream(c, "tile build sync");
}

// Device time of one scan launch of class `ci` over `nchunks` chunks of a
// synthetic stream (min of `reps` launches).
double time_class(oasm_ctx *c, const ClassInfo &ci, const ChunkDesc *d_chunks, uint32_t nchunks, int reps) {
    hipStream_t st = c->st;
    const uint64_t nitems = (uint64_t)nchunks * ci.ntiles;
    const uint32_t cap = 64;
    c->item_rec.ensure(nitems * cap * 4, st);
    c->item_cnt.ensure(nitems * 4, st);
    c->ctl.ensure(64, st);
    ScanArgs a;
    a.chunks = d_chunks;
    a.nchunks = nchunks;
    a.tiles = c->d_tiles.as<TileDesc>();
    a.tile_first = ci.tile_first;
    a.ntiles = ci.ntiles;
    a.peq_img = c->d_peq.as<uint32_t>();
    a.slot_pat = c->d_slot_pat.as<uint32_t>();
    a.pats = c->d_pats.as<PatDesc>();
    a.nclass = c->nclass;
    a.item_rec = c->item_rec.as<uint32_t>();
    a.item_cnt = c->item_cnt.as<uint32_t>();
    a.item_base = 0;
    a.cap = cap;
    a.max_cnt = c->ctl.as<uint32_t>();
    a.wsteps = nullptr;
    double best = 1e30;
    for (int r = 0; r < reps; ++r) {
        ck(hipEventRecord(c->ev0, st), "event");
        ck(launch_scan(ci.W, ci.P, ci.cut, a, ci.waves, ci.lds, st), "tune scan");
        ck(hipEventRecord(c->ev1, st), "event");
        wait_stream(c, "tune sync");
        float ms = 0;
        ck(hipEventElapsedTime(&ms, c->ev0, c->ev1), "event time");
        best = std::min(best, (double)ms);
    }
    return best;
}

// Process-wide memory of tuning results, keyed by the class's shape, and of
// the chunk-size scale, keyed by the dictionary's shape.
std::mutex g_tune_mu;
std::map<std::tuple<uint32_t, int, size_t, int>, TileChoice> g_tune_cache;
std::map<std::vector<uint64_t>, double> g_scale_cache;

// The synthetic trial of class W under the tiles last built: a stream of
// `nbytes` symbols cut into chunks by the rule of a real step of that size
// (at the context's current chunk scale).  Returns the device time of one
// launch (min of `reps`).
double time_trial(oasm_ctx *c, int W, const uint8_t *text, size_t nbytes, DevBuf &d_chunks, int reps) {
    hipStream_t st = c->st;
    const ClassInfo *ci = nullptr;
    for (const ClassInfo &k : c->classes)
        if (k.W == W) ci = &k;
    const uint32_t C = choose_chunk(c, nbytes);  // the rule of a real step of nbytes
    std::vector<ChunkDesc> ch;
    for (uint64_t e0 = 0; e0 < nbytes; e0 += C) {
        const uint64_t e1 = std::min<uint64_t>(nbytes, e0 + C);
        uint64_t s0 = e0 >= c->lookback ? e0 - c->lookback : 0;
        s0 &= ~uint64_t(3);
        ch.push_back(ChunkDesc{text + s0, e0, (uint32_t)(e1 - s0), (uint32_t)(e0 - s0), 0, 0});
    }
    d_chunks.ensure(ch.size() * sizeof(ChunkDesc), st);
    ck(hipMemcpyAsync(d_chunks.p, ch.data(), ch.size() * sizeof(ChunkDesc), hipMemcpyHostToDevice, st),
       "tune chunks");
    return time_class(c, *ci, d_chunks.as<ChunkDesc>(), (uint32_t)ch.size(), reps);
}

// Measure the scan variants of every word-count class on a synthetic stream
// of uniformly drawn symbol classes, and keep the fastest per class: patterns
// per lane (1, 2, 4), the word cutoff or full columns, where the match masks
// are read from (the image in LDS or through L1/L2) and wavefronts per block
// (2 or 4).  A trial is a large step of one class: text for
// 16,384 chunks of 64 KiB over the class's tiles, between 4 and 128 MiB, cut
// by the real chunk rule, so that it fills the chip with about as many work
// items, and spreads a block's image copy over about as much text, as a
// large step.  Three interleaved rounds; after the first, only candidates
// within 25 % of the best are timed again.  Then the chunk-size rule's scale
// (0.5, 1, 2): the sum over the classes of their time per byte with their
// chosen variants.
void autotune(oasm_ctx *c, std::vector<TileChoice> &choice) {
    hipStream_t st = c->st;
    const size_t max_bytes = size_t(128) << 20, min_bytes = size_t(4) << 20;
    DevBuf d_text, d_chunks, d_tab;
    // the trial text draws symbol classes with the frequencies they have in
    // the dictionary's patterns (text and patterns usually share an
    // alphabet's skew; how often a pattern's prefix matches decides how far
    // the word cutoff reaches and how often a group is replayed), through a
    // table of 65536 entries; bytes no pattern uses are left out
    {
        std::vector<double> freq(c->nclass, 0.0);
        for (uint8_t b : c->h_patbytes) freq[c->class_of[b]] += 1.0;
        double total = 0;
        for (double f : freq) total += f;
        std::vector<uint8_t> tab;
        tab.reserve(65536);
        for (uint32_t k = 0; k < c->nclass; ++k) {
            const size_t want = (size_t)(freq[k] / total * 65536.0 + 0.5);
            tab.insert(tab.end(), std::min(want, 65536 - tab.size()), (uint8_t)k);
        }
        uint32_t most = 0;
        for (uint32_t k = 1; k < c->nclass; ++k)
            if (freq[k] > freq[most]) most = k;
        tab.resize(65536, (uint8_t)most);  // rounding leftovers to the most frequent class
        d_tab.ensure(65536, st);
        ck(hipMemcpyAsync(d_tab.p, tab.data(), 65536, hipMemcpyHostToDevice, st), "tune table");
        d_text.ensure(max_bytes + kPad, st);
        ck(launch_fill_classes(d_text.as<uint32_t>(), (max_bytes + kPad) / 4, d_tab.as<uint8_t>(),
                               0x9E3779B97F4A7C15ull, st),
           "tune text");
        wait_stream(c, "tune text");
    }
    const bool cut_ok = !(c->cfg.flags & OASM_CFG_NO_CUTOFF);
    // trial text per class: 16,384 chunks of 64 KiB over its tiles
    auto trial_bytes = [&](int W) {
        const ClassInfo *ci = nullptr;
        for (const ClassInfo &k : c->classes)
            if (k.W == W) ci = &k;
        const size_t nbytes = (size_t)16384 * 65536 / std::max<uint32_t>(1, ci->ntiles);
        return std::min(max_bytes, std::max(min_bytes, nbytes)) & ~size_t(0xFFFF);
    };
    char line[192];
    c->chunk_scale = 1.0;
    std::vector<uint64_t> shape{c->nclass, (uint64_t)c->max_lds, (uint64_t)cut_ok};
    for (int W = 1; W <= kMaxW32; ++W) {
        const size_t nW = class_members(c, W).size();
        if (nW == 0) continue;
        shape.push_back((uint64_t)W << 32 | nW);
        const auto key = std::make_tuple(c->nclass, W, nW, (int)c->max_lds * 2 + (cut_ok ? 1 : 0));
        {
            std::lock_guard<std::mutex> g(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                choice[W] = it->second;
                continue;
            }
        }
        // the heuristic default first: another variant must beat it by 3 %
        std::vector<TileChoice> cands{choice[W]};
        for (int P : {1, 2, 4}) {
            for (bool cut : {false, true}) {
                if (cut && !cut_ok) continue;
                if (!scan_variant_exists(W, P, cut) || (P > 1 && nW <= (size_t)64 * (P / 2))) continue;
                for (int lds : {0, 1}) {
                    if (lds_bytes(c, W, P, cut, lds) > c->max_lds) continue;
                    for (int waves : {2, 4}) {
                        const TileChoice &d = choice[W];
                        if (P == d.P && lds == d.lds && cut == d.cut && waves == d.waves) continue;
                        cands.push_back(TileChoice{P, lds, cut, waves});
                    }
                }
            }
        }
        // three rounds over all candidates (interleaved, so that clock and
        // thermal drift during tuning does not favour any one), min per
        // candidate; the first round's first launch of each is a warm-up
        std::vector<double> best_ms(cands.size(), 1e30);
        std::vector<size_t> nbytes_of(cands.size(), 0);
        for (int round = 0; round < 3; ++round) {
            double lead = 1e30;  // best time per word-step so far
            for (size_t q = 0; q < cands.size(); ++q)
                if (nbytes_of[q]) lead = std::min(lead, best_ms[q] / ((double)nW * W * (double)nbytes_of[q]));
            for (size_t q = 0; q < cands.size(); ++q) {
                if (round && best_ms[q] / ((double)nW * W * (double)nbytes_of[q]) > 1.25 * lead) continue;
                std::vector<TileChoice> trial = choice;
                trial[W] = cands[q];
                build_tiles(c, trial);
                nbytes_of[q] = trial_bytes(W);
                const double ms = time_trial(c, W, d_text.as<uint8_t>(), nbytes_of[q], d_chunks, round ? 1 : 2);
                best_ms[q] = std::min(best_ms[q], ms);
            }
        }
        double best = 1e30;
        TileChoice pick = choice[W];
        for (size_t q = 0; q < cands.size(); ++q) {
            const TileChoice &cd = cands[q];
            // time per pattern word per text byte: trials differ in tiles and text
            const double per = best_ms[q] / ((double)nW * W * (double)nbytes_of[q]);
            std::snprintf(line, sizeof line,
                          "W=%d P=%d lds=%d cut=%d waves=%d: %.3f ms for %.0f MiB (%.3f ps per word-step)\n", W, cd.P,
                          cd.lds, (int)cd.cut, cd.waves, best_ms[q], nbytes_of[q] / 1048576.0, per * 1e9);
            c->tune_log += line;
            if (per < (q == 0 ? 1e30 : best * 0.97)) {
                best = per;
                pick = cd;
            }
        }
        choice[W] = pick;
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = pick;
    }
    // the chunk-size scale, with every class's chosen variant
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_scale_cache.find(shape);
        if (it != g_scale_cache.end()) {
            c->chunk_scale = it->second;
            d_text.release();
            d_chunks.release();
            d_tab.release();
            return;
        }
    }
    build_tiles(c, choice);
    const double scales[3] = {1.0, 0.5, 2.0};
    double per_byte[3] = {1e30, 1e30, 1e30};
    for (int round = 0; round < 3; ++round) {
        for (int q = 0; q < 3; ++q) {
            c->chunk_scale = scales[q];
            double sum = 0;
            for (const ClassInfo &ci : std::vector<ClassInfo>(c->classes)) {
                const size_t nbytes = trial_bytes(ci.W);
                sum += time_trial(c, ci.W, d_text.as<uint8_t>(), nbytes, d_chunks, round ? 1 : 2) / (double)nbytes;
            }
            per_byte[q] = std::min(per_byte[q], sum);
        }
    }
    int pick = 0;
    for (int q = 0; q < 3; ++q) {
        std::snprintf(line, sizeof line, "chunk scale %.1f: %.4f ns per text byte over all classes\n", scales[q],
                      per_byte[q] * 1e6);
        c->tune_log += line;
        if (q > 0 && per_byte[q] < per_byte[pick] * 0.97) pick = q;
    }
    c->chunk_scale = scales[pick];
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_scale_cache[shape] = c->chunk_scale;
    }
    d_text.release();
    d_chunks.release();
    d_tab.release();
}

}  // namespace

// ====================================================================== ABI
extern "C" {

oasm_status oasm_config_init(oasm_config *cfg) {
    if (!cfg) return OASM_E_INVAL;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->struct_size = sizeof(oasm_config);
    cfg->device = -1;
    return OASM_OK;
}

const char *oasm_status_str(oasm_status s) {
    switch (s) {
        case OASM_OK: return "OASM_OK";
        case OASM_E_INVAL: return "OASM_E_INVAL";
        case OASM_E_NOMEM: return "OASM_E_NOMEM";
        case OASM_E_AGAIN: return "OASM_E_AGAIN";
        case OASM_E_CLOSED: return "OASM_E_CLOSED";
        case OASM_E_DEVICE: return "OASM_E_DEVICE";
        default: return "OASM_E_UNKNOWN";
    }
}

static thread_local std::string g_create_error;

// FNV-1a over everything a stream's matching state depends on besides its
// own bytes: rules, pattern count, each pattern's length, threshold and
// bytes, and the symbol classes.
static uint64_t dictionary_fingerprint(const oasm_ctx *c, const std::vector<uint8_t> &bytes) {
    uint64_t h = 0xcbf29ce484222325ull;
    auto mix = [&h](const void *p, size_t n) {
        const uint8_t *b = static_cast<const uint8_t *>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001b3ull;
    };
    mix(&c->rules, sizeof c->rules);
    mix(&c->npat, sizeof c->npat);
    for (uint32_t i = 0; i < c->npat; ++i) {
        mix(&c->m[i], sizeof c->m[i]);
        mix(&c->k[i], sizeof c->k[i]);
    }
    mix(bytes.data(), bytes.size());
    mix(c->class_of, sizeof c->class_of);
    return h;
}

oasm_status oasm_create(const oasm_pattern *dict, uint32_t n, const uint16_t *k, uint16_t k_all, uint32_t rules,
                        const oasm_config *cfg, oasm_ctx **out) {
    if (!out) return OASM_E_INVAL;
    *out = nullptr;
    if (!dict || n == 0) {
        g_create_error = "empty dictionary";
        return OASM_E_INVAL;
    }
    static_assert(OASM_RULES_PAPER == kRulePaper && OASM_RULES_ACC_LAST == kRuleAccLast &&
                      OASM_RULES_EQ3_GE == kRuleEq3Ge && OASM_RULES_START_ORDER == kRuleStartOrder &&
                      OASM_RULES_DISJOINT == kRuleDisjoint,
                  "rule bits");
    static_assert(OASM_NOALLOC_MAX_PATTERNS == kLcNoallocMaxPatterns, "noalloc table size");
    if ((rules & ~kRuleAll) != 0 || (rules != OASM_RULES_NONE && !(rules & OASM_RULES_PAPER))) {
        g_create_error = "unknown rules";
        return OASM_E_INVAL;
    }
    if (cfg && cfg->chunk_bytes > OASM_MAX_CHUNK_BYTES) {
        // a scan record holds an end offset inside its chunk in 24 bits
        g_create_error = "chunk_bytes above OASM_MAX_CHUNK_BYTES";
        return OASM_E_INVAL;
    }
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t len = dict[i].len;
        const uint32_t kk = k ? k[i] : k_all;
        if (!dict[i].bytes || len == 0 || len > OASM_MAX_PATTERN_LEN || kk >= len || kk > 63) {
            g_create_error = "pattern " + std::to_string(i) + ": need 1 <= len <= 256, K < len and K <= 63";
            return OASM_E_INVAL;
        }
    }
    oasm_ctx *c = new (std::nothrow) oasm_ctx();
    if (!c) return OASM_E_NOMEM;
    if (cfg) {
        c->cfg = *cfg;
    } else {
        oasm_config_init(&c->cfg);
    }
    c->rules = rules;
    try {
        if (c->cfg.device >= 0) ck(hipSetDevice(c->cfg.device), "hipSetDevice");
        ck(hipGetDevice(&c->device), "hipGetDevice");
        if (c->cfg.hip_stream) {
            c->st = reinterpret_cast<hipStream_t>(c->cfg.hip_stream);
        } else {
            ck(hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking), "hipStreamCreate");
            c->own_stream = true;
        }
        ck(hipEventCreate(&c->ev0), "event");
        ck(hipEventCreate(&c->ev1), "event");
        ck(hipEventCreate(&c->ev2), "event");
        ck(hipEventCreate(&c->ev3), "event");
        ck(hipEventCreate(&c->ev_seg), "event");
        ck(hipEventCreateWithFlags(&c->ev_lc, hipEventDisableTiming), "event");
        // the allocation-free LEV CALC's table array on this device (looked
        // up once per device, with the device current)
        ck(levcalc_scratch(c->device, &c->lc_scratch), "scratch address");
        hipStream_t st = c->st;

        // dictionary on the host: lengths, thresholds, symbol classes
        c->npat = n;
        c->m.resize(n);
        c->k.resize(n);
        bool used[256] = {false};
        std::vector<uint8_t> bytes;
        std::vector<PatDesc> pd(n);
        uint64_t rpeq_words = 0;
        for (uint32_t i = 0; i < n; ++i) {
            c->m[i] = (uint16_t)dict[i].len;
            c->k[i] = k ? k[i] : k_all;
            c->mmax = std::max<uint32_t>(c->mmax, c->m[i]);
            c->kmax = std::max<uint32_t>(c->kmax, c->k[i]);
            c->msum += c->m[i];
            c->wsum += (c->m[i] + 31) / 32;
            pd[i].off = (uint32_t)bytes.size();
            pd[i].m = c->m[i];
            pd[i].k = c->k[i];
            pd[i].w64 = (uint16_t)((c->m[i] + 63) / 64);
            bytes.insert(bytes.end(), dict[i].bytes, dict[i].bytes + dict[i].len);
            for (uint32_t j = 0; j < dict[i].len; ++j) used[dict[i].bytes[j]] = true;
        }
        // classes: class 0 collects bytes no pattern uses (when there are any)
        uint32_t nused = 0;
        for (int b = 0; b < 256; ++b) nused += used[b];
        uint32_t next = nused < 256 ? 1 : 0;
        for (int b = 0; b < 256; ++b) c->class_of[b] = used[b] ? (uint8_t)(next++) : 0;
        c->nclass = next;
        for (uint32_t i = 0; i < n; ++i) {
            pd[i].rpeq_off = (uint32_t)rpeq_words;
            rpeq_words += (uint64_t)pd[i].w64 * c->nclass;
        }
        c->hks = 2 * c->kmax + 1;
        c->lookback = c->mmax + c->kmax - 1;
        c->dict_fp = dictionary_fingerprint(c, bytes);

        c->h_patbytes = bytes;
        c->h_pd = pd;
        c->rpeq_words = rpeq_words;
        int lds_max = 0;
        if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) == hipSuccess &&
            lds_max > 0)
            c->max_lds = (size_t)lds_max;
        std::vector<TileChoice> choice = default_choices(c);
        if (c->cfg.flags & OASM_CFG_AUTOTUNE) autotune(c, choice);
        build_tiles(c, choice);
        for (const ClassInfo &ci : c->classes) {
            char line[128];
            std::snprintf(line, sizeof line, "class W=%d: P=%d lds=%d cut=%d waves=%d tiles=%u\n", ci.W, ci.P,
                          ci.lds, (int)ci.cut, ci.waves, ci.ntiles);
            c->tune_log += line;
        }
        {
            char line[96];
            std::snprintf(line, sizeof line, "chunk scale: %.1f\n", c->chunk_scale);
            c->tune_log += line;
        }
        ck(hipStreamSynchronize(st), "create sync");
    } catch (const HipFail &f) {
        g_create_error = std::string(f.what) + ": " + hipGetErrorString(f.e);
        oasm_destroy(c);
        return OASM_E_DEVICE;
    } catch (const std::bad_alloc &) {
        oasm_destroy(c);
        return OASM_E_NOMEM;
    }
    *out = c;
    return OASM_OK;
}

// Map a list of (source, staging destination, length) copies with one
// launch: long copies are cut into kMapPiece-symbol pieces (one block each),
// the table goes up through pinned memory (reused once its previous upload
// is done).
static void map_copies(oasm_ctx *c, const std::vector<SegCopy> &in) {
    constexpr uint32_t kPiece = kMapPiece;
    std::vector<SegCopy> copies;
    copies.reserve(in.size());
    for (const SegCopy &sc : in)
        for (uint32_t o = 0; o < sc.len; o += kPiece)
            copies.push_back(SegCopy{sc.src + o, sc.dst + o, std::min(kPiece, sc.len - o), 0});
    if (copies.empty()) return;
    if (c->seg_pending) {
        ck(hipEventSynchronize(c->ev_seg), "segment table reuse");
        c->seg_pending = false;
    }
    const size_t bytes = copies.size() * sizeof(SegCopy);
    c->pin_seg.ensure(bytes, c->st);
    c->d_seg.ensure(bytes, c->st);
    std::memcpy(c->pin_seg.p, copies.data(), bytes);
    ck(hipMemcpyAsync(c->d_seg.p, c->pin_seg.p, bytes, hipMemcpyHostToDevice, c->st), "segment table upload");
    ck(hipEventRecord(c->ev_seg, c->st), "segment event");
    c->seg_pending = true;
    ck(launch_map_segments(c->d_seg.as<SegCopy>(), (uint32_t)copies.size(), c->d_class.as<uint8_t>(), c->st),
       "map segments");
}

static oasm_status feed_common(oasm_ctx *c, uint64_t stream_id, const void *src, size_t n, bool device,
                               void *user_stream, uint32_t flags) {
    if (!c) return OASM_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (c->poisoned) return fail(c, OASM_E_DEVICE, "context is poisoned by an earlier error");
    if (n > 0 && !src) return fail(c, OASM_E_INVAL, "NULL bytes with n > 0");
    if (n > (size_t(1) << 31)) return fail(c, OASM_E_INVAL, "feed larger than 2 GiB");
    try {
        if (device) ck(hipSetDevice(c->device), "hipSetDevice");
        if (is_finished(c, stream_id)) return fail(c, OASM_E_CLOSED, "feed to a closed stream");
        StreamState &s = get_stream(c, stream_id, true);
        if (s.closed || s.close_pending) return fail(c, OASM_E_CLOSED, "feed to a closed stream");
        if (n > 0 && c->cfg.device_mem_budget && c->pending_bytes + n > c->cfg.device_mem_budget)
            return fail(c, OASM_E_AGAIN, "device memory budget for unmatched stream data exhausted");
        if (n > 0) {
            oasm_status r = reserve_stream(c, s, n);
            if (r != OASM_OK) return r;
            if (device) {
                hipStream_t us = reinterpret_cast<hipStream_t>(user_stream);
                if (us != c->st) {
                    ck(hipEventRecord(c->ev3, us), "feed event");
                    ck(hipStreamWaitEvent(c->st, c->ev3, 0), "feed wait");
                }
                ck(launch_map_symbols(reinterpret_cast<const uint8_t *>(src), s.sym + s.valid, n,
                                      c->d_class.as<uint8_t>(), c->st),
                   "map symbols");
            } else {
                // copy into pinned memory (the caller may reuse its buffer), then H2D + map
                if (c->pin_feed_used + n > c->pin_feed.cap) {
                    ck(hipStreamSynchronize(c->st), "feed sync");
                    c->pin_feed_used = 0;
                    c->pin_feed.ensure(n, c->st);
                }
                uint8_t *hp = c->pin_feed.as<uint8_t>() + c->pin_feed_used;
                std::memcpy(hp, src, n);
                c->pin_feed_used += n;
                c->raw_in.ensure(n + kPad, c->st);
                ck(hipMemcpyAsync(c->raw_in.p, hp, n, hipMemcpyHostToDevice, c->st), "feed h2d");
                ck(launch_map_symbols(c->raw_in.as<uint8_t>(), s.sym + s.valid, n, c->d_class.as<uint8_t>(), c->st),
                   "map symbols");
            }
            s.valid += n;
            c->pending_bytes += n;
            c->stats.cells += (uint64_t)n * c->msum;
            c->stats.word_steps += (uint64_t)n * c->wsum;
        }
        if (flags & OASM_FEED_LAST) s.close_pending = true;
    } catch (const HipFail &f) {
        return device_fail(c, f);
    } catch (const std::bad_alloc &) {
        return fail(c, OASM_E_NOMEM, "host allocation failed");
    }
    return OASM_OK;
}

oasm_status oasm_feed(oasm_ctx *c, uint64_t stream_id, const uint8_t *bytes, size_t n, uint32_t flags) {
    return feed_common(c, stream_id, bytes, n, false, nullptr, flags);
}

oasm_status oasm_feed_device(oasm_ctx *c, uint64_t stream_id, const void *dev, size_t n, void *hip_stream,
                             uint32_t flags) {
    return feed_common(c, stream_id, dev, n, true, hip_stream, flags);
}

oasm_status oasm_feed_device_many(oasm_ctx *c, const oasm_feed_seg *segs, size_t n, void *hip_stream) {
    if (!c) return OASM_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (c->poisoned) return fail(c, OASM_E_DEVICE, "context is poisoned by an earlier error");
    if (n > 0 && !segs) return fail(c, OASM_E_INVAL, "NULL segs with n > 0");
    // validate everything before touching any stream (all or nothing)
    uint64_t total = 0;
    std::unordered_map<uint64_t, uint64_t> add;  // stream id -> bytes in this call
    std::unordered_map<uint64_t, char> closing;  // stream id -> closed by a piece of this call
    for (size_t i = 0; i < n; ++i) {
        const oasm_feed_seg &sg = segs[i];
        if (sg.reserved != 0) return fail(c, OASM_E_INVAL, "reserved field must be 0");
        if (sg.len > 0 && !sg.data) return fail(c, OASM_E_INVAL, "NULL data with len > 0");
        if (sg.len > (uint64_t(1) << 31)) return fail(c, OASM_E_INVAL, "piece larger than 2 GiB");
        if (closing.count(sg.stream)) return fail(c, OASM_E_CLOSED, "feed to a stream closed earlier in the call");
        if (is_finished(c, sg.stream)) return fail(c, OASM_E_CLOSED, "feed to a closed stream");
        auto it = c->slot_of.find(sg.stream);
        if (it != c->slot_of.end()) {
            const StreamState &s = c->streams[it->second];
            if (s.closed || s.close_pending) return fail(c, OASM_E_CLOSED, "feed to a closed stream");
        }
        if (sg.flags & OASM_FEED_LAST) closing[sg.stream] = 1;
        add[sg.stream] += sg.len;
        total += sg.len;
    }
    if (total > 0 && c->cfg.device_mem_budget && c->pending_bytes + total > c->cfg.device_mem_budget)
        return fail(c, OASM_E_AGAIN, "device memory budget for unmatched stream data exhausted");
    try {
        ck(hipSetDevice(c->device), "hipSetDevice");
        for (auto &kv : add) {
            StreamState &s = get_stream(c, kv.first, true);
            if (kv.second) {
                oasm_status r = reserve_stream(c, s, kv.second, true);
                if (r != OASM_OK) {
                    flush_moves(c, c->st);  // the streams grown so far keep their symbols
                    return r;
                }
            }
        }
        flush_moves(c, c->st);
        std::vector<SegCopy> copies;
        copies.reserve(n);
        for (size_t i = 0; i < n; ++i) {
            const oasm_feed_seg &sg = segs[i];
            StreamState &s = c->streams[c->slot_of[sg.stream]];
            if (sg.len) {
                copies.push_back(SegCopy{reinterpret_cast<const uint8_t *>(sg.data), s.sym + s.valid,
                                         (uint32_t)sg.len, 0});
                s.valid += sg.len;
                c->pending_bytes += sg.len;
                c->stats.cells += sg.len * c->msum;
                c->stats.word_steps += sg.len * c->wsum;
            }
            if (sg.flags & OASM_FEED_LAST) s.close_pending = true;
        }
        hipStream_t us = reinterpret_cast<hipStream_t>(hip_stream);
        if (!copies.empty() && us && us != c->st) {
            ck(hipEventRecord(c->ev3, us), "feed event");
            ck(hipStreamWaitEvent(c->st, c->ev3, 0), "feed wait");
        }
        map_copies(c, copies);
    } catch (const HipFail &f) {
        return device_fail(c, f);
    } catch (const std::bad_alloc &) {
        return fail(c, OASM_E_NOMEM, "host allocation failed");
    }
    return OASM_OK;
}

oasm_status oasm_close_stream(oasm_ctx *c, uint64_t stream_id) {
    if (!c) return OASM_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (is_finished(c, stream_id)) return fail(c, OASM_E_INVAL, "stream already closed");
    auto it = c->slot_of.find(stream_id);
    if (it == c->slot_of.end()) return fail(c, OASM_E_INVAL, "unknown stream");
    StreamState &s = c->streams[it->second];
    if (s.closed || s.close_pending) return fail(c, OASM_E_INVAL, "stream already closed");
    s.close_pending = true;
    return OASM_OK;
}

// ------------------------------------------------------------------ checkpoint
// Record layout (little-endian): CkptHeader, nsym look-back symbols (symbol
// classes), ncarry CkptCarry, then ncarry * hks hit-set bytes.
namespace {
struct CkptHeader {
    uint32_t magic, version;
    uint64_t dict_fp;
    uint64_t position;  // absolute symbols matched
    uint32_t nsym;      // look-back symbols that follow
    uint32_t ncarry;    // carried hit ends that follow
    uint32_t hks;       // hit-set bytes per carried hit end
    uint32_t reserved;
};
struct CkptCarry {
    uint64_t end_abs;
    uint32_t pattern;
    uint32_t dist;
};
static_assert(sizeof(CkptHeader) == 40 && sizeof(CkptCarry) == 16, "checkpoint layout");

size_t ckpt_size(uint64_t nsym, uint64_t ncarry, uint64_t hks) {
    return sizeof(CkptHeader) + nsym + ncarry * (sizeof(CkptCarry) + hks);
}

// The context's carried hit ends (records and hit-set bytes) on the host;
// the caller has no step in flight.
void carry_to_host(oasm_ctx *c, std::vector<CarryRec> &rec, std::vector<uint8_t> &hk) {
    rec.resize(c->ncarry);
    hk.resize((size_t)c->ncarry * c->hks);
    if (!c->ncarry) return;
    ck(hipMemcpyAsync(rec.data(), c->carry_buf[c->carry_cur].p, rec.size() * sizeof(CarryRec),
                      hipMemcpyDeviceToHost, c->st),
       "carry download");
    ck(hipMemcpyAsync(hk.data(), c->carry_hk_buf[c->carry_cur].p, hk.size(), hipMemcpyDeviceToHost, c->st),
       "carry download");
    ck(hipStreamSynchronize(c->st), "carry download");
}
}  // namespace

oasm_status oasm_stream_export(oasm_ctx *c, uint64_t stream_id, void *buf, size_t cap, size_t *size) {
    if (!c || !size) return OASM_E_INVAL;
    *size = 0;
    std::lock_guard<std::mutex> g(c->mu);
    if (c->poisoned) return fail(c, OASM_E_DEVICE, "context is poisoned by an earlier error");
    if (is_finished(c, stream_id)) return fail(c, OASM_E_CLOSED, "export of a closed stream");
    auto it = c->slot_of.find(stream_id);
    if (it == c->slot_of.end()) return fail(c, OASM_E_INVAL, "export of an unknown stream");
    if (c->streams[it->second].close_pending) return fail(c, OASM_E_INVAL, "export of a stream with a close pending");
    try {
        ck(hipSetDevice(c->device), "hipSetDevice");
        sync_all(c);  // every byte fed is matched (the stream stays live: no close was pending)
        const StreamState &s = c->streams[c->slot_of.at(stream_id)];
        const uint32_t nsym = (uint32_t)std::min<uint64_t>(s.scanned, c->lookback + 4);
        const uint32_t n = s.ncarry;
        const size_t need = ckpt_size(nsym, n, c->hks);
        *size = need;
        if (!buf) return OASM_OK;
        if (cap < need) return fail(c, OASM_E_INVAL, "buffer smaller than the checkpoint");
        std::vector<CarryRec> rec;
        std::vector<uint8_t> hk;
        if (n) carry_to_host(c, rec, hk);
        uint8_t *o = static_cast<uint8_t *>(buf);
        const CkptHeader h{OASM_CKPT_MAGIC, OASM_CKPT_VERSION, c->dict_fp, s.base_abs + s.scanned, nsym, n, c->hks, 0};
        std::memcpy(o, &h, sizeof h);
        if (nsym) {
            ck(hipMemcpyAsync(o + sizeof h, s.sym + (s.scanned - nsym), nsym, hipMemcpyDeviceToHost, c->st),
               "look-back download");
            ck(hipStreamSynchronize(c->st), "look-back download");
        }
        uint8_t *oc = o + sizeof h + nsym, *ohk = oc + (size_t)n * sizeof(CkptCarry);
        uint32_t w = 0;
        for (uint32_t i = 0; i < c->ncarry && w < n; ++i) {
            if (rec[i].stream_slot != s.slot) continue;
            const CkptCarry cr{rec[i].end_abs, rec[i].pattern, rec[i].dist};
            std::memcpy(oc + (size_t)w * sizeof cr, &cr, sizeof cr);
            std::memcpy(ohk + (size_t)w * c->hks, hk.data() + (size_t)i * c->hks, c->hks);
            ++w;
        }
        if (w != n) throw HipFail{hipErrorUnknown, "internal: the stream's carried hit ends are not in the carry"};
    } catch (const HipFail &f) {
        return device_fail(c, f);
    } catch (const std::bad_alloc &) {
        return step_alloc_fail(c);
    }
    return OASM_OK;
}

oasm_status oasm_stream_import(oasm_ctx *c, uint64_t stream_id, const void *buf, size_t size) {
    if (!c) return OASM_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (c->poisoned) return fail(c, OASM_E_DEVICE, "context is poisoned by an earlier error");
    if (!buf) return fail(c, OASM_E_INVAL, "NULL checkpoint");
    if (size < sizeof(CkptHeader)) return fail(c, OASM_E_INVAL, "checkpoint truncated");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof h);
    if (h.magic != OASM_CKPT_MAGIC || h.version != OASM_CKPT_VERSION)
        return fail(c, OASM_E_INVAL, "not a stream checkpoint of this version");
    if (h.dict_fp != c->dict_fp || h.hks != c->hks)
        return fail(c, OASM_E_INVAL, "checkpoint of another dictionary, thresholds or rules");
    if (h.reserved || h.nsym > c->lookback + 4 || h.nsym > h.position)
        return fail(c, OASM_E_INVAL, "inconsistent checkpoint header");
    if (size != ckpt_size(h.nsym, h.ncarry, h.hks)) return fail(c, OASM_E_INVAL, "checkpoint size does not match");
    const uint8_t *sym = static_cast<const uint8_t *>(buf) + sizeof h;
    const uint8_t *cb = sym + h.nsym, *hkb = cb + (size_t)h.ncarry * sizeof(CkptCarry);
    for (uint32_t i = 0; i < h.nsym; ++i)
        if (sym[i] >= c->nclass) return fail(c, OASM_E_INVAL, "checkpoint symbol outside the classes");
    std::vector<CkptCarry> cr(h.ncarry);
    if (h.ncarry) std::memcpy(cr.data(), cb, cr.size() * sizeof(CkptCarry));
    {
        // within a pattern the ends increase (the order the filter walks them)
        std::vector<uint64_t> next_min(h.ncarry ? c->npat : 0, 0);
        for (uint32_t i = 0; i < h.ncarry; ++i) {
            if (cr[i].pattern >= c->npat || cr[i].end_abs >= h.position || cr[i].dist > c->k[cr[i].pattern])
                return fail(c, OASM_E_INVAL, "checkpoint hit end out of range");
            if (cr[i].end_abs < next_min[cr[i].pattern])
                return fail(c, OASM_E_INVAL, "checkpoint hit ends out of order");
            next_min[cr[i].pattern] = cr[i].end_abs + 1;
        }
    }
    if (is_finished(c, stream_id) || c->slot_of.count(stream_id))
        return fail(c, OASM_E_INVAL, "stream id already live or closed in this context");
    StreamState *sp = nullptr;
    try {
        ck(hipSetDevice(c->device), "hipSetDevice");
        ck(hipStreamSynchronize(c->st), "import sync");  // nothing reads the carry or a staging buffer now
        std::vector<CarryRec> rec;
        std::vector<uint8_t> hk;
        if (h.ncarry) carry_to_host(c, rec, hk);
        sp = &get_stream(c, stream_id, true);
        StreamState &s = *sp;
        if (h.nsym) {
            const oasm_status r = reserve_stream(c, s, h.nsym);
            if (r != OASM_OK) throw std::bad_alloc();
            ck(hipMemcpyAsync(s.sym, sym, h.nsym, hipMemcpyHostToDevice, c->st), "look-back upload");
        }
        s.base_abs = h.position - h.nsym;
        s.valid = s.scanned = h.nsym;
        if (h.ncarry) {
            for (uint32_t i = 0; i < h.ncarry; ++i)
                rec.push_back(CarryRec{cr[i].end_abs, cr[i].pattern, s.slot, cr[i].dist, 0});
            hk.insert(hk.end(), hkb, hkb + (size_t)h.ncarry * c->hks);
            const int cur = c->carry_cur;
            c->carry_buf[cur].ensure(rec.size() * sizeof(CarryRec), c->st);
            c->carry_hk_buf[cur].ensure(hk.size(), c->st);
            ck(hipMemcpyAsync(c->carry_buf[cur].p, rec.data(), rec.size() * sizeof(CarryRec), hipMemcpyHostToDevice,
                              c->st),
               "carry upload");
            ck(hipMemcpyAsync(c->carry_hk_buf[cur].p, hk.data(), hk.size(), hipMemcpyHostToDevice, c->st),
               "carry upload");
            c->ncarry = (uint32_t)rec.size();
            s.ncarry = h.ncarry;
        }
        ck(hipStreamSynchronize(c->st), "import sync");
    } catch (const HipFail &f) {
        return device_fail(c, f);
    } catch (const std::bad_alloc &) {
        if (sp && sp->ncarry == 0) {  // nothing of the stream reached the carry: take it back out
            c->staged_bytes -= sp->cap;
            release_staging(c, sp->sym, sp->cap);
            c->slot_of.erase(stream_id);
            c->free_slots.push_back(sp->slot);
            *sp = StreamState{};
        }
        return fail(c, OASM_E_NOMEM, "allocation failed during import");
    }
    return OASM_OK;
}

oasm_status oasm_sync(oasm_ctx *c) {
    if (!c) return OASM_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (c->poisoned) return fail(c, OASM_E_DEVICE, "context is poisoned by an earlier error");
    TraceRange range("oasm_sync");
    const double t0 = now_ms();
    try {
        ck(hipSetDevice(c->device), "hipSetDevice");
        sync_all(c);
    } catch (const HipFail &f) {
        c->stats.sync_wall_ms += now_ms() - t0;
        return device_fail(c, f);
    } catch (const std::bad_alloc &) {
        return step_alloc_fail(c);
    }
    c->stats.sync_wall_ms += now_ms() - t0;
    return OASM_OK;
}

oasm_status oasm_serve(oasm_ctx *c, const oasm_segment *segs, size_t n, const void *dev_pool, uint64_t pool_bytes,
                       double *latency_s, oasm_serve_report *report) {
    if (report) *report = oasm_serve_report{};
    if (!c || (n > 0 && (!segs || !dev_pool))) return OASM_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    TraceRange range("oasm_serve");
    if (c->poisoned) return fail(c, OASM_E_DEVICE, "context is poisoned by an earlier error");
    for (size_t i = 0; i < n; ++i) {
        if (segs[i].offset > pool_bytes || segs[i].len > pool_bytes - segs[i].offset)
            return fail(c, OASM_E_INVAL, "segment outside the pool");
        if (i && segs[i].arrival_s < segs[i - 1].arrival_s)
            return fail(c, OASM_E_INVAL, "segments must be sorted by arrival");
    }
    oasm_serve_report rep{};
    const uint8_t *pool = reinterpret_cast<const uint8_t *>(dev_pool);
    const double t0 = now_ms();
    double slept = 0;
    size_t next = 0;
    std::deque<size_t> ready;
    std::vector<size_t> admitted;                // mapped into their streams, not yet in a launched step
    std::vector<SegCopy> copies;
    std::unordered_map<uint64_t, uint64_t> add;  // stream id -> bytes admitted at once
    std::unordered_set<uint64_t> closing;        // streams a segment admitted at once closes
    std::vector<uint32_t> created;               // slots of streams created by that admission
    // Two steps: while one runs on the device, the host converts the results
    // of the one before it and admits and maps the segments that arrive (their
    // copies are queued behind the running step); when it has finished, the
    // segments that arrived meanwhile are admitted too and the next step is
    // launched over all of them.
    StepRun runs[2];
    std::vector<size_t> batch_of[2];
    int fly = -1;   // the step in flight
    int done = -1;  // a finished step whose results are not converted yet
    std::vector<uint32_t> which;

    // Admit the arrived segments in arrival order while the fed-but-unmatched
    // bytes stay within the budget.  Every admitted segment is checked before
    // any stream changes, so an error leaves the streams as they were.
    auto admit_ready = [&]() -> oasm_status {
        const double t = (now_ms() - t0) * 1e-3;
        while (next < n && segs[next].arrival_s <= t) ready.push_back(next++);
        if (ready.empty()) return OASM_OK;
        add.clear();
        closing.clear();
        uint64_t admit = 0;
        size_t take = 0;
        const uint64_t budget = c->cfg.device_mem_budget;
        for (; take < ready.size(); ++take) {
            const oasm_segment &sg = segs[ready[take]];
            if (budget && c->pending_bytes + admit + sg.len > budget && (admit > 0 || c->pending_bytes > 0)) {
                rep.deferred++;
                break;
            }
            bool closed = is_finished(c, sg.stream) || closing.count(sg.stream) != 0;
            if (!closed) {
                auto it = c->slot_of.find(sg.stream);
                if (it != c->slot_of.end())
                    closed = c->streams[it->second].closed || c->streams[it->second].close_pending;
            }
            if (closed) return fail(c, OASM_E_INVAL, "segment for a closed stream");
            add[sg.stream] += sg.len;
            admit += sg.len;
            if (sg.flags & OASM_FEED_LAST) closing.insert(sg.stream);
        }
        if (take == 0) return OASM_OK;
        // one staging reservation per stream; on failure the streams this
        // admission created are removed again (the others only grew)
        created.clear();
        for (auto &kv : add) {
            if (c->slot_of.find(kv.first) == c->slot_of.end()) created.push_back(get_stream(c, kv.first, true).slot);
            oasm_status r = reserve_stream(c, c->streams[c->slot_of[kv.first]], kv.second, true);
            if (r != OASM_OK) {
                flush_moves(c, c->st);  // the streams grown so far keep their symbols
                for (uint32_t slot : created) {
                    StreamState &s = c->streams[slot];
                    if (s.sym) {
                        c->staged_bytes -= s.cap;
                        release_staging(c, s.sym, s.cap);
                    }
                    c->slot_of.erase(s.id);
                    s = StreamState{};
                    c->free_slots.push_back(slot);
                }
                return r;
            }
        }
        flush_moves(c, c->st);
        copies.clear();
        for (size_t q = 0; q < take; ++q) {
            const size_t i = ready[q];
            const oasm_segment &sg = segs[i];
            StreamState &s = c->streams[c->slot_of[sg.stream]];
            if (sg.len) copies.push_back(SegCopy{pool + sg.offset, s.sym + s.valid, sg.len, 0});
            s.valid += sg.len;
            c->pending_bytes += sg.len;
            c->stats.cells += (uint64_t)sg.len * c->msum;
            c->stats.word_steps += (uint64_t)sg.len * c->wsum;
            if (sg.flags & OASM_FEED_LAST) s.close_pending = true;
            admitted.push_back(i);
        }
        ready.erase(ready.begin(), ready.begin() + (ptrdiff_t)take);
        map_copies(c, copies);  // queued behind the step in flight
        return OASM_OK;
    };
    // segments of a finished step (or admitted empty ones) are served: their
    // results are drainable
    auto served = [&](const std::vector<size_t> &idx) {
        const double fin = (now_ms() - t0) * 1e-3;
        for (size_t i : idx) {
            if (latency_s) latency_s[i] = fin - segs[i].arrival_s;
            rep.segments++;
            rep.bytes += segs[i].len;
        }
    };
    auto finish_flying = [&]() {
        if (fly < 0) return;
        step_wait(c, runs[fly]);
        step_bookkeep(c, runs[fly]);
        done = fly;
        fly = -1;
    };
    // the next step, over every stream with unmatched bytes (the admitted
    // segments', and any fed before the run)
    auto launch_pending = [&]() {
        which.clear();
        for (uint32_t i = 0; i < c->streams.size(); ++i) {
            const StreamState &s = c->streams[i];
            if (!s.closed && (s.valid > s.scanned || s.close_pending)) which.push_back(i);
        }
        if (which.empty()) {  // only empty segments: nothing to match
            served(admitted);
            admitted.clear();
            return;
        }
        const int k = done >= 0 ? 1 - done : 0;
        step_launch(c, which, runs[k], k);
        batch_of[k].swap(admitted);
        admitted.clear();
        uint64_t bytes = 0;
        for (size_t i : batch_of[k]) bytes += segs[i].len;
        rep.steps++;
        rep.max_batch_bytes = std::max<uint64_t>(rep.max_batch_bytes, bytes);
        fly = k;
    };
    auto convert_done = [&]() {
        if (done < 0) return;
        const size_t h0 = c->q_h.size();
        step_convert(c, runs[done]);
        if (c->cfg.flags & OASM_CFG_KEEP_H) sort_h_queue_tail(c, h0);
        served(batch_of[done]);
        batch_of[done].clear();
        done = -1;
    };
    // on every return: the step in flight and the admitted segments are
    // matched, and the report counts the segments served (a prefix of the
    // segments in arrival order)
    auto done_with = [&](oasm_status st) {
        if (st != OASM_E_DEVICE && !c->poisoned) {
            try {
                while (fly >= 0 || done >= 0 || !admitted.empty()) {
                    finish_flying();
                    launch_pending();
                    convert_done();
                }
            } catch (const HipFail &f) {
                st = device_fail(c, f);
            } catch (const std::bad_alloc &) {
                st = step_alloc_fail(c);
            }
        }
        rep.wall_s = (now_ms() - t0) * 1e-3;
        rep.busy_s = rep.wall_s - slept;
        if (report) *report = rep;
        return st;
    };
    try {
        ck(hipSetDevice(c->device), "hipSetDevice");
        while (next < n || !ready.empty() || fly >= 0 || !admitted.empty()) {
            oasm_status r = admit_ready();  // while a step runs: overlapped with it
            if (r != OASM_OK) return done_with(r);
            if (fly < 0 && admitted.empty() && ready.empty()) {
                const double dt = segs[next].arrival_s - (now_ms() - t0) * 1e-3;
                if (dt > 0) {
                    const double ts = now_ms();
                    std::this_thread::sleep_for(std::chrono::duration<double>(std::min(dt, 0.01)));
                    slept += (now_ms() - ts) * 1e-3;
                }
                continue;
            }
            const bool had_step = fly >= 0;
            finish_flying();
            r = admit_ready();  // the arrivals during the wait join the next step
            if (r != OASM_OK) return done_with(r);
            launch_pending();
            convert_done();  // while the new step runs
            // nothing ran, nothing was admitted and nothing can be: arrived
            // segments wait for a budget that no step will free (the budget
            // counts bytes that no stream holds); an internal error, not a spin
            if (!had_step && fly < 0 && admitted.empty() && !ready.empty() && c->pending_bytes > 0)
                return done_with(fail(c, OASM_E_DEVICE, "internal: serving budget held by no stream"));
        }
    } catch (const HipFail &f) {
        return done_with(device_fail(c, f));
    } catch (const std::bad_alloc &) {
        return done_with(step_alloc_fail(c));
    }
    return done_with(OASM_OK);
}

oasm_status oasm_queued(const oasm_ctx *c, uint32_t kind, size_t *n) {
    if (!c || !n) return OASM_E_INVAL;
    oasm_ctx *m = const_cast<oasm_ctx *>(c);
    std::lock_guard<std::mutex> g(m->mu);
    if (kind == OASM_RAW) {
        *n = c->q_raw.size() - c->rd_raw;
    } else if (kind == OASM_FILTERED) {
        *n = c->q_occ.size() - c->rd_occ;
    } else if (kind == OASM_H && (c->cfg.flags & OASM_CFG_KEEP_H)) {
        *n = c->q_h.size() - c->rd_h;
    } else {
        return OASM_E_INVAL;
    }
    return OASM_OK;
}

oasm_status oasm_hits(oasm_ctx *c, uint32_t kind, void *out, size_t cap, size_t *n_out, int *more) {
    if (!c || !n_out || (cap > 0 && !out)) return OASM_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    *n_out = 0;
    if (kind == OASM_RAW) {
        const size_t avail = c->q_raw.size() - c->rd_raw;
        const size_t take = std::min(avail, cap);
        if (take) parallel_copy(out, c->q_raw.data() + c->rd_raw, take * sizeof(oasm_hit));
        c->rd_raw += take;
        *n_out = take;
        if (more) *more = avail > take;
        if (c->rd_raw == c->q_raw.size()) {
            c->q_raw.clear();
            c->rd_raw = 0;
        }
        return OASM_OK;
    }
    if (kind == OASM_FILTERED || kind == OASM_H) {
        OccQueue &q = kind == OASM_FILTERED ? c->q_occ : c->q_h;
        size_t &rd = kind == OASM_FILTERED ? c->rd_occ : c->rd_h;
        if (kind == OASM_H && !(c->cfg.flags & OASM_CFG_KEEP_H))
            return fail(c, OASM_E_INVAL, "OASM_H needs OASM_CFG_KEEP_H");
        const size_t avail = q.size() - rd;
        const size_t take = std::min(avail, cap);
        if (take) parallel_copy(out, q.data() + rd, take * sizeof(oasm_occ));
        rd += take;
        *n_out = take;
        if (more) *more = avail > take;
        if (rd == q.size()) {
            q.clear();
            rd = 0;
        }
        return OASM_OK;
    }
    return fail(c, OASM_E_INVAL, "unknown drain kind");
}

oasm_status oasm_get_stats(const oasm_ctx *c, oasm_stats *out) {
    if (!c || !out) return OASM_E_INVAL;
    *out = c->stats;
    return OASM_OK;
}

oasm_status oasm_levcalc_size(const oasm_ctx *c, size_t n, size_t *bytes) {
    if (!c || !bytes) return OASM_E_INVAL;
    uint64_t unit = 0;
    for (uint32_t p = 0; p < c->npat; ++p) unit += 2u * c->k[p] + 1u;
    if (n && unit > SIZE_MAX / n) return OASM_E_INVAL;
    *bytes = n * unit;
    return OASM_OK;
}

oasm_status oasm_levcalc(oasm_ctx *c, const void *dev_text, size_t n, void *dev_out, size_t out_bytes,
                         void *hip_stream) {
    if (!c) return OASM_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (c->poisoned) return fail(c, OASM_E_DEVICE, "context is poisoned by an earlier error");
    if (n > 0 && (!dev_text || !dev_out)) return fail(c, OASM_E_INVAL, "NULL text or output with n > 0");
    size_t need = 0;
    if (oasm_levcalc_size(c, n, &need) != OASM_OK) return fail(c, OASM_E_INVAL, "output size overflows size_t");
    if (out_bytes < need) return fail(c, OASM_E_INVAL, "output buffer too small for n * sum(2K + 1) bytes");
    if (n == 0) return OASM_OK;
    TraceRange range("oasm_levcalc");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    try {
        ck(hipSetDevice(c->device), "hipSetDevice");
        if (c->lc_groups.empty()) {
            std::vector<uint32_t> ids;
            std::vector<uint64_t> unit(c->npat);
            uint64_t acc = 0;
            for (uint32_t p = 0; p < c->npat; ++p) {
                unit[p] = acc;
                acc += 2u * c->k[p] + 1u;
            }
            for (int W = 1; W <= kMaxW32; ++W) {
                oasm_ctx::LcGroup gr{W, (uint32_t)ids.size(), 0};
                for (uint32_t p = 0; p < c->npat; ++p)
                    if ((int)((c->m[p] + 31u) / 32u) == W) ids.push_back(p);
                gr.count = (uint32_t)ids.size() - gr.first;
                if (gr.count) c->lc_groups.push_back(gr);
            }
            c->d_lc_ids.ensure(ids.size() * 4, c->st);
            c->d_lc_unit.ensure(unit.size() * 8, c->st);
            ck(hipMemcpy(c->d_lc_ids.p, ids.data(), ids.size() * 4, hipMemcpyHostToDevice), "levcalc table upload");
            ck(hipMemcpy(c->d_lc_unit.p, unit.data(), unit.size() * 8, hipMemcpyHostToDevice), "levcalc table upload");
            c->lc_unit_total = acc;
        }
        for (const auto &gr : c->lc_groups) {
            LevcalcArgs a;
            a.text = reinterpret_cast<const uint8_t *>(dev_text);
            a.n = n;
            a.pat_ids = c->d_lc_ids.as<uint32_t>() + gr.first;
            a.npat = gr.count;
            a.pats = c->d_pats.as<PatDesc>();
            a.pat_bytes = c->d_patbytes.as<uint8_t>();
            a.out_unit = c->d_lc_unit.as<uint64_t>();
            a.out = reinterpret_cast<uint8_t *>(dev_out);
            ck(launch_levcalc(gr.W, a, st), "levcalc launch");
        }
        // destroy waits for this point: the kernels read the dictionary tables
        ck(hipEventRecord(c->ev_lc, st), "levcalc event record");
    } catch (const HipFail &f) {
        return device_fail(c, f);
    } catch (const std::bad_alloc &) {
        return fail(c, OASM_E_NOMEM, "host allocation failed");
    }
    return OASM_OK;
}

oasm_status oasm_levcalc_noalloc(oasm_ctx *c, const void *dev_text, size_t n, void *dev_out, size_t out_bytes,
                                 void *hip_stream) {
    if (!c) return OASM_E_INVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (c->poisoned) return fail(c, OASM_E_DEVICE, "context is poisoned by an earlier error");
    if (n > 0 && (!dev_text || !dev_out)) return fail(c, OASM_E_INVAL, "NULL text or output with n > 0");
    if (c->npat > OASM_NOALLOC_MAX_PATTERNS)
        return fail(c, OASM_E_INVAL, "dictionary larger than OASM_NOALLOC_MAX_PATTERNS");
    size_t need = 0;
    if (oasm_levcalc_size(c, n, &need) != OASM_OK) return fail(c, OASM_E_INVAL, "output size overflows size_t");
    if (out_bytes < need) return fail(c, OASM_E_INVAL, "output buffer too small for n * sum(2K + 1) bytes");
    if (n == 0) return OASM_OK;
    TraceRange range("oasm_levcalc");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    try {
        ck(hipSetDevice(c->device), "hipSetDevice");
        // groups of the word-count-major id list, counted on the host from
        // the dictionary's lengths (the device builds the same list)
        uint32_t cnt[kMaxW32 + 1] = {};
        for (uint32_t p = 0; p < c->npat; ++p) cnt[(c->m[p] + 31u) / 32u]++;
        ck(launch_levcalc_tables(c->d_pats.as<PatDesc>(), c->npat, c->lc_scratch, st), "levcalc tables");
        const uint64_t *unit = reinterpret_cast<const uint64_t *>(c->lc_scratch);
        const uint32_t *ids =
            reinterpret_cast<const uint32_t *>(c->lc_scratch + (size_t)kLcNoallocMaxPatterns * sizeof(uint64_t));
        uint32_t first = 0;
        for (int W = 1; W <= kMaxW32; ++W) {
            if (!cnt[W]) continue;
            LevcalcArgs a;
            a.text = reinterpret_cast<const uint8_t *>(dev_text);
            a.n = n;
            a.pat_ids = ids + first;
            a.npat = cnt[W];
            a.pats = c->d_pats.as<PatDesc>();
            a.pat_bytes = c->d_patbytes.as<uint8_t>();
            a.out_unit = unit;
            a.out = reinterpret_cast<uint8_t *>(dev_out);
            ck(launch_levcalc(W, a, st), "levcalc launch");
            first += cnt[W];
        }
        ck(hipEventRecord(c->ev_lc, st), "levcalc event record");
    } catch (const HipFail &f) {
        return device_fail(c, f);
    }
    return OASM_OK;
}

void oasm_destroy(oasm_ctx *c) {
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);
    if (c->ev_lc) {
        (void)hipEventSynchronize(c->ev_lc);
        (void)hipEventDestroy(c->ev_lc);
    }
    // every staging buffer is a slab piece or an allocation of its own
    for (uint8_t *p : c->own_alloc) (void)hipFree(p);
    for (uint8_t *p : c->slabs) (void)hipFree(p);
    DevBuf *bufs[] = {&c->d_pats, &c->d_slot_pat, &c->d_tiles, &c->d_peq, &c->d_rpeq, &c->d_class, &c->d_patbytes,
                      &c->d_pat_tile, &c->d_pat_slot, &c->d_tile_wp, &c->plan, &c->offsets, &c->item_rec,
                      &c->item_cnt, &c->ctl, &c->scan_tmp, &c->sort_key, &c->sort_val, &c->sort_end, &c->sort_tmp,
                      &c->r_pat, &c->r_sl, &c->r_end, &c->r_flag, &c->r_dist, &c->r_hk, &c->seg_cnt, &c->seg_off,
                      &c->carry_flag, &c->carry_off, &c->long_list, &c->long_desc, &c->long_next, &c->long_jump[0], &c->long_jump[1], &c->seg_out,
                      &c->occ_out, &c->carry_buf[0], &c->carry_buf[1],
                      &c->carry_hk_buf[0], &c->carry_hk_buf[1], &c->raw_in, &c->d_lc_ids, &c->d_lc_unit};
    for (DevBuf *b : bufs) b->release();
    c->pin_plan.release();
    c->pin_ctl.release();
    c->pin_out[0].release();
    c->pin_out[1].release();
    c->pin_feed.release();
    c->pin_seg.release();
    c->d_seg.release();
    drop_graphs(c);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->ev2) (void)hipEventDestroy(c->ev2);
    if (c->ev3) (void)hipEventDestroy(c->ev3);
    if (c->ev_seg) (void)hipEventDestroy(c->ev_seg);
    if (c->own_stream && c->st) (void)hipStreamDestroy(c->st);
    delete c;
}

const char *oasm_tune_report(const oasm_ctx *c) { return c ? c->tune_log.c_str() : ""; }

const char *oasm_last_error(const oasm_ctx *c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

}  // extern "C"
