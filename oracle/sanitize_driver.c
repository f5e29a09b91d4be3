/*
 * TEST INFRASTRUCTURE ONLY: drives every function of oasm_oracle.c on
 * seeded random inputs, so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks the oracle's memory accesses and
 * arithmetic.  Output capacities are varied (including 0 and values below the
 * count) to exercise the "count exceeds cap" paths.  Exits 0 when all calls
 * return consistent counts; a sanitizer report aborts with a nonzero status.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int32_t oracle_lev(const uint8_t *p, int32_t lp, const uint8_t *s, int32_t ls);
int64_t oracle_sellers(const uint8_t *p, int32_t m, const uint8_t *t, int64_t n, int32_t K, int64_t *ends,
                       int32_t *dists, int64_t cap, int32_t *dall);
int64_t oracle_hset_all(const uint8_t *p, int32_t m, const uint8_t *t, int64_t n, int32_t K, int64_t *hs,
                        int32_t *hl, int32_t *hk, int64_t cap);
int64_t oracle_hset_at_ends(const uint8_t *p, int32_t m, const uint8_t *t, int64_t n, int32_t K,
                            const int64_t *ends, int64_t nends, int64_t *hs, int32_t *hl, int32_t *hk, int64_t cap);
int64_t oracle_levcalc(const uint8_t *p, int32_t m, const uint8_t *t, int64_t n, int32_t K, uint8_t *out);
int64_t oracle_filter(const int64_t *hs, const int32_t *hl, const int32_t *hk, int64_t nh, int32_t K, int64_t n,
                      int32_t rules, int64_t *ev_pos, int32_t *ev_level, int64_t *ev_i, int32_t *ev_l,
                      int64_t *ev_r, int64_t *ev_acc, int32_t *ev_acc_flag, int64_t cap);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(uint32_t n) { /* splitmix64 */
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return n ? (uint32_t)(z % n) : 0;
}

/* exact-size heap copies, so that any read past the end is reported */
static void *dup(const void *src, size_t bytes) {
    void *d = malloc(bytes ? bytes : 1);
    if (bytes) memcpy(d, src, bytes);
    return d;
}

int main(int argc, char **argv) {
    int cases = argc > 1 ? atoi(argv[1]) : 400;
    for (int c = 0; c < cases; ++c) {
        const int32_t sigma = 2 + (int32_t)rnd(3);
        const int32_t m = 1 + (int32_t)rnd(12);
        const int32_t K = (int32_t)rnd((uint32_t)m);
        const int64_t n = (int64_t)rnd(160);
        uint8_t pb[16], tb[200];
        for (int32_t i = 0; i < m; ++i) pb[i] = (uint8_t)rnd((uint32_t)sigma);
        for (int64_t i = 0; i < n; ++i) tb[i] = (uint8_t)rnd((uint32_t)sigma);
        if (n > m && (c & 1)) memcpy(tb + rnd((uint32_t)(n - m)), pb, (size_t)m);
        uint8_t *p = dup(pb, (size_t)m), *t = dup(tb, (size_t)n);

        (void)oracle_lev(p, m, t, (int32_t)n);
        const int64_t cap_e = (int64_t)rnd(8);
        int64_t *ends = malloc(sizeof(int64_t) * (size_t)(n + 1));
        int32_t *dists = malloc(sizeof(int32_t) * (size_t)(n + 1));
        int32_t *dall = malloc(sizeof(int32_t) * (size_t)(n + 1));
        const int64_t ne_small = oracle_sellers(p, m, t, n, K, ends, dists, cap_e, dall);
        const int64_t ne = oracle_sellers(p, m, t, n, K, ends, dists, n, NULL);
        if (ne != ne_small || ne < 0) return 2;

        const int64_t hcap = n * (2 * K + 1) + 1;
        int64_t *hs = malloc(sizeof(int64_t) * (size_t)hcap);
        int32_t *hl = malloc(sizeof(int32_t) * (size_t)hcap), *hk = malloc(sizeof(int32_t) * (size_t)hcap);
        const int64_t nh2 = oracle_hset_at_ends(p, m, t, n, K, ends, ne, hs, hl, hk, hcap);
        const int64_t nh_small = oracle_hset_all(p, m, t, n, K, hs, hl, hk, (int64_t)rnd(4));
        const int64_t nh = oracle_hset_all(p, m, t, n, K, hs, hl, hk, hcap); /* (start, length) order */
        if (nh != nh_small || nh != nh2) return 3;

        uint8_t *lc = malloc((size_t)(n * (2 * K + 1)) + 1);
        if (oracle_levcalc(p, m, t, n, K, lc) != 0) return 4;

        const int64_t ecap = nh * (K + 1) + 1;
        int64_t *ep = malloc(sizeof(int64_t) * (size_t)ecap), *ei = malloc(sizeof(int64_t) * (size_t)ecap);
        int64_t *er = malloc(sizeof(int64_t) * (size_t)ecap), *ea = malloc(sizeof(int64_t) * (size_t)ecap);
        int32_t *el = malloc(sizeof(int32_t) * (size_t)ecap), *eL = malloc(sizeof(int32_t) * (size_t)ecap);
        int32_t *ef = malloc(sizeof(int32_t) * (size_t)ecap);
        for (int32_t rules = 0; rules < 32; rules += 1 + (int32_t)rnd(7)) {
            const int64_t a = oracle_filter(hs, hl, hk, nh, K, n, rules, ep, el, ei, eL, er, ea, ef, (int64_t)rnd(3));
            const int64_t b = oracle_filter(hs, hl, hk, nh, K, n, rules, ep, el, ei, eL, er, ea, ef, ecap);
            if (a != b || b < 0) return 5;
        }
        free(ep); free(ei); free(er); free(ea); free(el); free(eL); free(ef);
        free(lc); free(hs); free(hl); free(hk); free(ends); free(dists); free(dall); free(p); free(t);
    }
    printf("sanitized oracle run: %d cases ok\n", cases);
    return 0;
}
