// TEST INFRASTRUCTURE ONLY: exercises the host runtime of oasm_gpu (built
// with AddressSanitizer on the host side only) through its C ABI: contexts
// with several dictionaries, host and device feeds across many streams in
// pieces, small-capacity drains of every record kind, the serving loop, LEV
// CALC, a budget refusal, error paths, and destroy.  The results are checked
// for consistency between two identically fed contexts (the parity with the
// oracle is the Python suite's job); any sanitizer report aborts the run.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "oasm_gpu.h"

#define CHECK(x)                                                                    \
    do {                                                                            \
        oasm_status s_ = (x);                                                       \
        if (s_ != OASM_OK) {                                                        \
            std::fprintf(stderr, "%s:%d: %s -> %d\n", __FILE__, __LINE__, #x, s_); \
            std::exit(2);                                                           \
        }                                                                           \
    } while (0)

static uint64_t g_state = 12345;
static uint32_t rnd(uint32_t n) {
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(g_state >> 33) % n;
}

struct Drained {
    std::vector<oasm_hit> raw;
    std::vector<oasm_occ> occ, h;
};

static void drain(oasm_ctx *c, Drained &d, bool with_h) {
    for (uint32_t kind : {(uint32_t)OASM_RAW, (uint32_t)OASM_FILTERED, (uint32_t)OASM_H}) {
        if (kind == OASM_H && !with_h) continue;
        int more = 1;
        while (more) {
            const size_t cap = 1 + rnd(13);
            size_t n = 0;
            if (kind == OASM_RAW) {
                std::vector<oasm_hit> buf(cap);
                CHECK(oasm_hits(c, kind, buf.data(), cap, &n, &more));
                d.raw.insert(d.raw.end(), buf.begin(), buf.begin() + n);
            } else {
                std::vector<oasm_occ> buf(cap);
                CHECK(oasm_hits(c, kind, buf.data(), cap, &n, &more));
                auto &dst = kind == OASM_FILTERED ? d.occ : d.h;
                dst.insert(dst.end(), buf.begin(), buf.begin() + n);
            }
        }
    }
}

static Drained run(const std::vector<std::vector<uint8_t>> &pats, const std::vector<uint16_t> &ks,
                   const std::vector<std::vector<uint8_t>> &streams, const uint8_t *dev_text, bool graphs,
                   uint64_t seed) {
    g_state = seed;
    std::vector<oasm_pattern> dict(pats.size());
    for (size_t i = 0; i < pats.size(); ++i) dict[i] = {pats[i].data(), (uint32_t)pats[i].size()};
    oasm_config cfg;
    CHECK(oasm_config_init(&cfg));
    cfg.flags = OASM_CFG_KEEP_H | (graphs ? OASM_CFG_GRAPHS : 0);
    cfg.chunk_bytes = 256;
    oasm_ctx *c = nullptr;
    CHECK(oasm_create(dict.data(), (uint32_t)dict.size(), ks.data(), 0, OASM_RULES_PAPER, &cfg, &c));
    Drained d;
    std::vector<size_t> pos(streams.size(), 0);
    for (int round = 0; round < 6; ++round) {
        for (size_t s = 0; s < streams.size(); ++s) {
            const size_t left = streams[s].size() - pos[s];
            const size_t n = round == 5 ? left : std::min(left, (size_t)rnd(700));
            const uint32_t flags = round == 5 ? OASM_FEED_LAST : 0;
            if (s % 2 == 0) {
                CHECK(oasm_feed(c, 100 + s, streams[s].data() + pos[s], n, flags));
            } else {
                // device bytes: the same stream content, copied to the device text
                CHECK(oasm_feed_device(c, 100 + s, dev_text + s * 4096 + pos[s], n, nullptr, flags));
            }
            pos[s] += n;
        }
        CHECK(oasm_sync(c));
        drain(c, d, true);
    }
    // error paths
    if (oasm_feed(c, 100, streams[0].data(), 1, 0) != OASM_E_CLOSED) std::exit(3);
    if (oasm_hits(c, 77, nullptr, 0, nullptr, nullptr) == OASM_OK) std::exit(4);
    // LEV CALC over the first device stream
    size_t need = 0;
    CHECK(oasm_levcalc_size(c, 4096, &need));
    uint8_t *dout = nullptr;
    if (hipMalloc(&dout, need) != hipSuccess) std::exit(5);
    CHECK(oasm_levcalc(c, dev_text, 4096, dout, need, nullptr));
    if (oasm_levcalc(c, dev_text, 4096, dout, need - 1, nullptr) != OASM_E_INVAL) std::exit(6);
    oasm_stats st;
    CHECK(oasm_get_stats(c, &st));
    (void)oasm_tune_report(c);
    oasm_destroy(c);
    (void)hipDeviceSynchronize();
    (void)hipFree(dout);
    return d;
}

static bool same(const Drained &a, const Drained &b) {
    return a.raw.size() == b.raw.size() && a.occ.size() == b.occ.size() && a.h.size() == b.h.size() &&
           (a.raw.empty() || !std::memcmp(a.raw.data(), b.raw.data(), a.raw.size() * sizeof(oasm_hit))) &&
           (a.occ.empty() || !std::memcmp(a.occ.data(), b.occ.data(), a.occ.size() * sizeof(oasm_occ))) &&
           (a.h.empty() || !std::memcmp(a.h.data(), b.h.data(), a.h.size() * sizeof(oasm_occ)));
}

int main() {
    g_state = 7;
    std::vector<std::vector<uint8_t>> pats;
    std::vector<uint16_t> ks;
    const int lens[] = {1, 3, 8, 15, 31, 32, 33, 40, 64, 65, 100, 129, 200, 256};
    for (int m : lens) {
        std::vector<uint8_t> p(m);
        for (auto &x : p) x = (uint8_t)("ACGT"[rnd(4)]);
        pats.push_back(p);
        ks.push_back((uint16_t)rnd((uint32_t)std::min(m, 20)));
    }
    std::vector<std::vector<uint8_t>> streams(6);
    std::vector<uint8_t> host_dev(6 * 4096);
    for (size_t s = 0; s < streams.size(); ++s) {
        streams[s].resize(2000 + rnd(2000));
        for (auto &x : streams[s]) x = (uint8_t)("ACGT"[rnd(4)]);
        // plant pattern copies
        for (int k = 0; k < 6; ++k) {
            const auto &p = pats[rnd((uint32_t)pats.size())];
            if (p.size() + 1 < streams[s].size()) {
                const size_t at = rnd((uint32_t)(streams[s].size() - p.size()));
                std::memcpy(streams[s].data() + at, p.data(), p.size());
            }
        }
        std::memcpy(host_dev.data() + s * 4096, streams[s].data(), streams[s].size());
    }
    uint8_t *dev = nullptr;
    if (hipMalloc(&dev, host_dev.size()) != hipSuccess) return 7;
    if (hipMemcpy(dev, host_dev.data(), host_dev.size(), hipMemcpyHostToDevice) != hipSuccess) return 8;
    const Drained a = run(pats, ks, streams, dev, false, 99);
    const Drained b = run(pats, ks, streams, dev, true, 99);
    if (!same(a, b)) {
        std::fprintf(stderr, "eager and graph runs differ\n");
        return 9;
    }
    // the serving loop over a device pool
    {
        std::vector<oasm_pattern> dict(pats.size());
        for (size_t i = 0; i < pats.size(); ++i) dict[i] = {pats[i].data(), (uint32_t)pats[i].size()};
        oasm_config cfg;
        CHECK(oasm_config_init(&cfg));
        cfg.device_mem_budget = 3000;
        oasm_ctx *c = nullptr;
        CHECK(oasm_create(dict.data(), (uint32_t)dict.size(), ks.data(), 0, OASM_RULES_PAPER, &cfg, &c));
        std::vector<oasm_segment> segs(40);
        double t = 0;
        for (size_t i = 0; i < segs.size(); ++i) {
            t += 0.0005;
            segs[i].stream = 1 + i % 5;
            segs[i].offset = rnd(4096);
            segs[i].len = 1 + rnd(1500);
            segs[i].flags = i + 5 >= segs.size() ? OASM_FEED_LAST : 0;
            segs[i].arrival_s = t;
        }
        std::vector<double> lat(segs.size());
        oasm_serve_report rep;
        CHECK(oasm_serve(c, segs.data(), segs.size(), dev, host_dev.size(), lat.data(), &rep));
        Drained d;
        drain(c, d, false);
        oasm_destroy(c);
    }
    (void)hipFree(dev);
    std::printf("runtime asan driver: %zu hit ends, %zu occurrences, %zu hit-set records; eager = graphs\n",
                a.raw.size(), a.occ.size(), a.h.size());
    return 0;
}
