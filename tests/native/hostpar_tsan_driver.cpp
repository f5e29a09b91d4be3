// Drives the host-side result conversion (oasm_hostpar.h) on the CPU with
// several threads, for a ThreadSanitizer build: the split conversions must
// equal a serial conversion record for record.  Test infrastructure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "oasm_hostpar.h"

namespace {

struct Rec {  // the device's packed occurrence, as the conversion reads it
    uint32_t stream_local;
    uint32_t pattern;
    uint64_t start_abs;
    uint32_t len;
    uint32_t k;
};

int fails = 0;

void expect(bool ok, const char *what, size_t at) {
    if (!ok && fails++ < 10) std::fprintf(stderr, "mismatch: %s at %zu\n", what, at);
}

void check_ranges() {
    // every index covered once, for more ranges than items and for none
    for (size_t n : {size_t(0), size_t(3), size_t(1000), size_t(1) << 20}) {
        for (unsigned nt : {1u, 2u, 5u, 8u}) {
            std::vector<unsigned char> seen(n, 0);
            oasm::parallel_ranges(n, nt, [&](unsigned, size_t lo, size_t hi) {
                for (size_t i = lo; i < hi; ++i) seen[i]++;
            });
            for (size_t i = 0; i < n; ++i) expect(seen[i] == 1, "range cover", i);
        }
    }
}

void check_raw(size_t n, size_t pre, uint32_t seed) {
    std::mt19937_64 rng(seed);
    const size_t nstreams = 97;
    std::vector<uint8_t> flag(n), dist(n);
    std::vector<uint32_t> sl(n), pat(n);
    std::vector<uint64_t> end(n), ids(nstreams);
    for (auto &x : ids) x = rng();
    for (size_t i = 0; i < n; ++i) {
        flag[i] = (rng() % 10) == 0;
        sl[i] = (uint32_t)(rng() % nstreams);
        end[i] = rng();
        pat[i] = (uint32_t)rng();
        dist[i] = (uint8_t)rng();
    }
    oasm::HitQueue q;
    for (size_t i = 0; i < pre; ++i) q.push_back(oasm_hit{i, i, 0, 0});
    const size_t got = oasm::convert_raw(flag.data(), sl.data(), end.data(), pat.data(), dist.data(), ids.data(), n, q);
    size_t w = pre;
    for (size_t i = 0; i < pre; ++i) expect(q[i].stream == i && q[i].end == i, "raw prefix", i);
    for (size_t i = 0; i < n; ++i) {
        if (flag[i]) continue;
        const oasm_hit &h = q[w++];
        expect(h.stream == ids[sl[i]] && h.end == end[i] && h.pattern == pat[i] && h.dist == dist[i], "raw record", i);
    }
    expect(w == q.size() && got == w - pre, "raw count", w);
}

void check_occ(size_t n, size_t pre, uint32_t seed) {
    std::mt19937_64 rng(seed);
    const size_t nstreams = 31;
    std::vector<uint64_t> ids(nstreams);
    for (auto &x : ids) x = rng();
    std::vector<Rec> rec(n);
    for (auto &r : rec) r = Rec{(uint32_t)(rng() % nstreams), (uint32_t)rng(), rng(), (uint32_t)rng(), (uint32_t)rng()};
    oasm::OccQueue q;
    for (size_t i = 0; i < pre; ++i) q.push_back(oasm_occ{i, i, 0, 0, 0, 0});
    oasm::convert_occ(rec.data(), ids.data(), n, q);
    expect(q.size() == pre + n, "occ count", q.size());
    for (size_t i = 0; i < n && pre + i < q.size(); ++i) {
        const oasm_occ &o = q[pre + i];
        expect(o.stream == ids[rec[i].stream_local] && o.start == rec[i].start_abs && o.pattern == rec[i].pattern &&
                   o.len == rec[i].len && o.k == rec[i].k && o.reserved == 0,
               "occ record", i);
    }
}

void check_copy(size_t bytes) {
    std::vector<unsigned char> src(bytes), dst(bytes, 0);
    for (size_t i = 0; i < bytes; ++i) src[i] = (unsigned char)(i * 131 + (i >> 9));
    oasm::parallel_copy(dst.data(), src.data(), bytes);
    for (size_t i = 0; i < bytes; ++i) expect(dst[i] == src[i], "copy", i);
}

}  // namespace

int main() {
    check_ranges();
    check_raw(0, 5, 1);
    check_raw(1000, 0, 2);                 // one thread
    check_raw(size_t(3) << 18, 7, 3);      // several threads
    check_raw((size_t(3) << 18) + 13, 0, 4);
    check_occ(0, 3, 5);
    check_occ(size_t(5) << 17, 11, 6);     // several threads
    check_copy(size_t(3) << 20);           // one thread
    check_copy((size_t(24) << 20) + 77);   // several threads
    std::printf("%s (%d mismatches)\n", fails ? "FAIL" : "ok", fails);
    return fails ? 1 : 0;
}
