// Host-side conversion of a step's results into the drain queues, split
// over a few host threads when a step reports many records (dense hits:
// millions of hit ends per MiB of text).  Plain C++ (no HIP), so that it
// also builds on the CPU under ThreadSanitizer.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include "oasm_gpu.h"

namespace oasm {

// A vector allocator whose resize leaves new elements of trivial types
// uninitialised (the conversion writes every one of them).
template <class T>
struct DefaultInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = DefaultInitAlloc<U>;
    };
    DefaultInitAlloc() = default;
    template <class U>
    DefaultInitAlloc(const DefaultInitAlloc<U> &) noexcept {}
    template <class U>
    void construct(U *p) noexcept(std::is_nothrow_default_constructible<U>::value) {
        ::new (static_cast<void *>(p)) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new (static_cast<void *>(p)) U(std::forward<A>(a)...);
    }
};

using HitQueue = std::vector<oasm_hit, DefaultInitAlloc<oasm_hit>>;
using OccQueue = std::vector<oasm_occ, DefaultInitAlloc<oasm_occ>>;

// Records per thread below which a conversion stays on the calling thread.
constexpr size_t kConvertGrain = size_t(1) << 17;
constexpr unsigned kConvertThreadsMax = 8;

inline unsigned convert_threads(size_t n) {
    const size_t want = n / kConvertGrain;
    if (want < 2) return 1;
    unsigned hw = std::thread::hardware_concurrency();
    if (hw == 0) hw = 1;
    return (unsigned)std::min<size_t>({want, (size_t)kConvertThreadsMax, (size_t)hw});
}

// f(t, lo, hi) over nt contiguous ranges of [0, n); range 0 runs on the
// caller.  f must not throw.  If a thread cannot be started, the caller
// runs the ranges that were not handed out.
template <class F>
void parallel_ranges(size_t n, unsigned nt, F &&f) {
    if (nt < 1) nt = 1;
    auto lo_of = [n, nt](unsigned t) { return (size_t)((unsigned __int128)n * t / nt); };
    std::vector<std::thread> th;
    unsigned t = 1;
    if (nt > 1) {
        th.reserve(nt - 1);
        try {
            for (; t < nt; ++t) th.emplace_back([&f, lo_of, t] { f(t, lo_of(t), lo_of(t + 1)); });
        } catch (...) {
        }
    }
    for (unsigned u = t; u < nt; ++u) f(u, lo_of(u), lo_of(u + 1));
    f(0u, lo_of(0), lo_of(1));
    for (auto &x : th) x.join();
}

// Room for `more` records at the end of a queue, growing it at least
// geometrically (an exact reserve would copy the whole queue at every step
// when the caller drains rarely).
template <class Q>
void grow_for(Q &q, size_t more) {
    if (q.size() + more > q.capacity()) q.reserve(std::max(q.size() + more, 2 * q.capacity()));
}

// The raw hits of a step: record i (of n, in the step's order) is reported
// unless flag[i] is set (a hit end carried from an earlier step, reported
// there); its stream id is ids[sl[i]].  Appended to q in record order.
inline size_t convert_raw(const uint8_t *flag, const uint32_t *sl, const uint64_t *end, const uint32_t *pat,
                          const uint8_t *dist, const uint64_t *ids, size_t n, HitQueue &q) {
    const unsigned nt = convert_threads(n);
    std::vector<size_t> off(nt + 1, 0);
    parallel_ranges(n, nt, [&](unsigned t, size_t lo, size_t hi) {
        size_t c = 0;
        for (size_t i = lo; i < hi; ++i) c += flag[i] == 0;
        off[t + 1] = c;
    });
    for (unsigned t = 0; t < nt; ++t) off[t + 1] += off[t];
    const size_t base = q.size(), total = off[nt];
    grow_for(q, total);
    q.resize(base + total);
    oasm_hit *out = q.data() + base;
    parallel_ranges(n, nt, [&](unsigned t, size_t lo, size_t hi) {
        oasm_hit *w = out + off[t];
        for (size_t i = lo; i < hi; ++i) {
            if (flag[i]) continue;
            w->stream = ids[sl[i]];
            w->end = end[i];
            w->pattern = pat[i];
            w->dist = dist[i];
            ++w;
        }
    });
    return total;
}

// The occurrences of a step, as the device packed them (stream-local index,
// absolute start, pattern, length, level), appended to q in order.
template <class Rec>
void convert_occ(const Rec *rec, const uint64_t *ids, size_t n, OccQueue &q) {
    const unsigned nt = convert_threads(n);
    const size_t base = q.size();
    grow_for(q, n);
    q.resize(base + n);
    oasm_occ *out = q.data() + base;
    parallel_ranges(n, nt, [&](unsigned, size_t lo, size_t hi) {
        for (size_t i = lo; i < hi; ++i)
            out[i] = oasm_occ{ids[rec[i].stream_local], rec[i].start_abs, rec[i].pattern, rec[i].len, rec[i].k, 0};
    });
}

// memcpy split over threads for large drains (the destination's pages are
// often fresh, and their first-touch faults then run in parallel too).
inline void parallel_copy(void *dst, const void *src, size_t bytes) {
    constexpr size_t kGrainBytes = size_t(4) << 20;
    const unsigned nt = bytes / kGrainBytes < 2
                            ? 1u
                            : (unsigned)std::min<size_t>({bytes / kGrainBytes, (size_t)kConvertThreadsMax,
                                                          (size_t)std::max(1u, std::thread::hardware_concurrency())});
    parallel_ranges(bytes, nt, [&](unsigned, size_t lo, size_t hi) {
        std::memcpy(static_cast<char *>(dst) + lo, static_cast<const char *>(src) + lo, hi - lo);
    });
}

}  // namespace oasm
