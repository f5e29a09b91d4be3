/*
 * OASM oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised CPU reference for what the
 * matching path computes.  It is used by the test suite, by the smoke check
 * and by the benchmark's CPU-baseline leg, and by nothing else: the product
 * library never links, loads or calls it, and the two share no code.
 *
 * Every function follows a passage of "A novel algorithm for online inexact
 * string matching and its FPGA implementation" (Cinti, Bianchi, Martino,
 * Rizzi, arXiv 1712.03560):
 *
 *   oracle_lev           Section 3, Eq. 1 (the Levenshtein matrix C)
 *   oracle_sellers       Section 5.1, "Less Naive": the dummy first row of C
 *                        set to zeros, the last row read as the hit ends
 *   oracle_hset_all      Section 3, Eq. 2: every substring t[i,l] with
 *                        l in [l_p-K, l_p+K] and lev <= K (the full hit set)
 *   oracle_hset_at_ends  Eq. 2 restricted to a given list of end positions
 *   oracle_levcalc       the output of LEV CALC (Section 6, the LEV CORE
 *                        description; Section 6.2): for every start i the
 *                        distances to t[i,l], l in [l_p-K, l_p+K], by Eq. 1
 *   oracle_filter        Section 4, Alg. 1 with the rules R1-R3 (Section 4.1)
 *                        and the validation test Eq. 3 (Section 4.2)
 *
 * Readings taken where the paper is ambiguous (documented again where they
 * are used):
 *   - a hit is "below the threshold" when its distance is <= K (Eq. 2);
 *   - R2 "first encountered" is the first whose last symbol arrives: of two
 *     equal-priority hits the one ending earlier wins, on equal ends the
 *     shorter one (R3); this is the only reading that reproduces the worked
 *     example of Section 4.2;
 *   - the completion test of Alg. 1 is r(idx) == l(idx);
 *   - the acceptance test is Eq. 3, r(k) - acc > l(k), with acc the sum of
 *     the lengths accepted so far in this emission (the pseudo-code's acc);
 *   - empty priority levels are skipped at emission;
 *   - positions are 0-based; t[i,l] covers t[i] .. t[i+l-1].
 * oracle_filter also takes the alternative readings as flag bits (the same
 * values as the library's OASM_RULES_* bits): acc = the last accepted length,
 * ">=" in Eq. 3, R2 literally in start order (keep the first equal-priority
 * hit), and acceptance only of occurrences disjoint from those accepted
 * before them in the emission.
 *
 * Integer arithmetic only.  No blocking, no bit-parallelism, no cut-offs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int32_t min3(int32_t a, int32_t b, int32_t c)
{
    int32_t m = a < b ? a : b;
    return m < c ? m : c;
}

/*
 * Eq. 1: lev(p, s) is element c[l_p][l] of the (l_p+1) x (l+1) matrix C with
 * c[n][0] = n, c[0][m] = m and c[n][m] = min(c[n-1][m]+1, c[n][m-1]+1,
 * c[n-1][m-1] + (p[n-1] != s[m-1])).  Built column by column, keeping one
 * column (the O(min) space remark of Section 3).
 */
int32_t oracle_lev(const uint8_t *p, int32_t lp, const uint8_t *s, int32_t ls)
{
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lp + 1));
    if (!col)
        return -1;
    for (int32_t n = 0; n <= lp; ++n)
        col[n] = n; /* column m = 0: c[n][0] = n */
    for (int32_t m = 1; m <= ls; ++m) {
        int32_t upper_left = col[0];
        col[0] = m; /* row n = 0: c[0][m] = m */
        for (int32_t n = 1; n <= lp; ++n) {
            int32_t left = col[n];
            int32_t upper = col[n - 1];
            int32_t delta = p[n - 1] != s[m - 1];
            col[n] = min3(upper + 1, left + 1, upper_left + delta);
            upper_left = left;
        }
    }
    int32_t d = col[lp];
    free(col);
    return d;
}

/*
 * "Less Naive" (Section 5.1): the same matrix C over the whole text, with the
 * dummy first row initialised to zeros instead of 0..l, so that every column
 * may start a substring.  The last row then holds, for every end position e,
 * D[e] = min over starts of lev(p, t[s..e]).  Every e with D[e] <= K is a hit
 * end.  Writes up to `cap` (end, D) pairs and returns how many exist.  If
 * `dall` is non-NULL it receives D[e] for every e (n entries).
 */
int64_t oracle_sellers(const uint8_t *p, int32_t m, const uint8_t *t, int64_t n,
                       int32_t K, int64_t *ends, int32_t *dists, int64_t cap,
                       int32_t *dall)
{
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
    if (!col)
        return -1;
    for (int32_t r = 0; r <= m; ++r)
        col[r] = r; /* dummy column: c[r][0] = r */
    int64_t count = 0;
    for (int64_t j = 1; j <= n; ++j) {
        int32_t upper_left = col[0];
        col[0] = 0; /* dummy row of zeros: a substring may start anywhere */
        for (int32_t r = 1; r <= m; ++r) {
            int32_t left = col[r];
            int32_t upper = col[r - 1];
            int32_t delta = p[r - 1] != t[j - 1];
            col[r] = min3(upper + 1, left + 1, upper_left + delta);
            upper_left = left;
        }
        int32_t d = col[m];
        if (dall)
            dall[j - 1] = d;
        if (d <= K) {
            if (count < cap) {
                ends[count] = j - 1;
                dists[count] = d;
            }
            ++count;
        }
    }
    free(col);
    return count;
}

/*
 * Eq. 2, by definition: every (i, l, k) with l in [max(1, l_p-K), l_p+K],
 * i + l <= n and k = lev(p, t[i,l]) <= K.  One independent Eq. 1 evaluation
 * per substring.  Output is in (i, l) order.  Returns the number of records.
 */
int64_t oracle_hset_all(const uint8_t *p, int32_t m, const uint8_t *t, int64_t n,
                        int32_t K, int64_t *hs, int32_t *hl, int32_t *hk,
                        int64_t cap)
{
    int32_t lmin = m - K < 1 ? 1 : m - K;
    int64_t count = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t l = lmin; l <= m + K; ++l) {
            if (i + l > n)
                break;
            int32_t k = oracle_lev(p, m, t + i, l);
            if (k <= K) {
                if (count < cap) {
                    hs[count] = i;
                    hl[count] = l;
                    hk[count] = k;
                }
                ++count;
            }
        }
    }
    return count;
}

/*
 * Eq. 2 restricted to substrings that end at one of the given positions:
 * for each end e and each l in [max(1, l_p-K), l_p+K] with e-l+1 >= 0,
 * k = lev(p, t[e-l+1, l]) by Eq. 1; records with k <= K are written in
 * (e ascending, l ascending) order.  Returns the number of records.
 */
int64_t oracle_hset_at_ends(const uint8_t *p, int32_t m, const uint8_t *t,
                            int64_t n, int32_t K, const int64_t *ends,
                            int64_t nends, int64_t *hs, int32_t *hl,
                            int32_t *hk, int64_t cap)
{
    int32_t lmin = m - K < 1 ? 1 : m - K;
    int64_t count = 0;
    for (int64_t q = 0; q < nends; ++q) {
        int64_t e = ends[q];
        if (e < 0 || e >= n)
            continue;
        for (int32_t l = lmin; l <= m + K; ++l) {
            int64_t i = e - l + 1;
            if (i < 0)
                break;
            int32_t k = oracle_lev(p, m, t + i, l);
            if (k <= K) {
                if (count < cap) {
                    hs[count] = i;
                    hl[count] = l;
                    hk[count] = k;
                }
                ++count;
            }
        }
    }
    return count;
}

/*
 * LEV CALC's output for every stream index (Section 6: at each new index it
 * yields the distances between p and the 2K+1 substrings t[i, l_p-K] ..
 * t[i, l_p+K]; Section 6.2).  out[i*(2K+1) + j] for start i in [0, n) and
 * j in [0, 2K] describes l = l_p - K + j:
 *   min(lev(p, t[i,l]), K+1)  when i + l <= n (one Eq. 1 evaluation),
 *   255                        when the substring runs past the text end.
 * Requires 0 <= K < l_p (so l >= 1).  Returns 0, or -1 on bad arguments.
 */
int64_t oracle_levcalc(const uint8_t *p, int32_t m, const uint8_t *t, int64_t n,
                       int32_t K, uint8_t *out)
{
    if (m < 1 || K < 0 || K >= m)
        return -1;
    int32_t width = 2 * K + 1;
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < width; ++j) {
            int32_t l = m - K + j;
            uint8_t v = 255;
            if (i + l <= n) {
                int32_t k = oracle_lev(p, m, t + i, l);
                v = (uint8_t)(k <= K ? k : K + 1);
            }
            out[i * width + j] = v;
        }
    }
    return 0;
}

/* One row of mem (Section 4.2): position i, length l, validation counter r.
 * A row with l == 0 holds no occurrence. */
typedef struct {
    int64_t i;
    int64_t l;
    int64_t r;
} mem_row;

/*
 * Alg. 1 (Section 4) over a hit set H given in (start, length) order, for a
 * text of n symbols.  The outer loop walks the stream index i from 0 to n-1;
 * the inner loop visits the hits that start at i, shortest first, in place
 * of evaluating lev for every l in [l_p-K, l_p+K] (H already holds exactly
 * the lengths whose distance is <= K).
 *
 *   R1 (Section 4.1): a hit with k < idx takes priority level k and becomes
 *      the occurrence under validation (idx = k).
 *   R2/R3: a hit with k == idx replaces the stored one of that level when
 *      the level is empty, when the new hit ends strictly earlier, or when it
 *      ends at the same position and is shorter.
 *   Otherwise the hit is discarded (R1).
 *   Completion: when the counter of level idx equals its length, the levels
 *      idx..K are examined in order; level idx is accepted, a lower-priority
 *      level j is accepted when Eq. 3 holds, r(j) - acc > l(j), where acc is
 *      the sum of the lengths accepted so far in this emission.  Then mem is
 *      reset and idx = K.
 *   Counters: while level idx is incomplete, the counters of levels idx..K
 *      are incremented once per stream symbol.
 *
 * `rules` selects alternative readings (bit values as in the library):
 *   2  ACC_LAST:    acc is the length of the last accepted occurrence;
 *   4  EQ3_GE:      Eq. 3 reads r(j) - acc >= l(j);
 *   8  START_ORDER: R2 replaces the stored hit only when its level is empty;
 *   16 DISJOINT:    a lower level is accepted only if, in addition, its
 *                   interval [i, i+l-1] shares no position with any
 *                   occurrence accepted before it in this emission.
 * rules = 1 (or 0) is the reading described above.
 *
 * Every examined non-empty level at an emission is reported as one event
 * (emission position, level, i, l, r, acc before the test, accepted flag),
 * so the caller can read both S (the accepted events, in emission order) and
 * the counter values the paper quotes for its worked example.
 * Returns the number of events (writes at most `cap`), or -1.
 */
int64_t oracle_filter(const int64_t *hs, const int32_t *hl, const int32_t *hk,
                      int64_t nh, int32_t K, int64_t n, int32_t rules,
                      int64_t *ev_pos, int32_t *ev_level, int64_t *ev_i,
                      int32_t *ev_l, int64_t *ev_r, int64_t *ev_acc,
                      int32_t *ev_acc_flag, int64_t cap)
{
    const int acc_last = (rules & 2) != 0;
    const int eq3_ge = (rules & 4) != 0;
    const int start_order = (rules & 8) != 0;
    const int disjoint = (rules & 16) != 0;
    mem_row *mem = (mem_row *)calloc((size_t)K + 1, sizeof(mem_row));
    if (!mem)
        return -1;
    int32_t idx = K;
    int ins = 0;
    int64_t acc = 0;
    int64_t h = 0;
    int64_t nev = 0;
    for (int64_t i = 0; i < n; ++i) {
        /* skip malformed records that start before i (H must be sorted) */
        while (h < nh && hs[h] < i)
            ++h;
        while (h < nh && hs[h] == i) {
            int64_t l = hl[h];
            int32_t k = hk[h];
            ++h;
            if (k < 0 || k > K)
                continue;
            if (k < idx) { /* R1 */
                idx = k;
                ins = 1;
                mem[idx].i = i;
                mem[idx].l = l;
                mem[idx].r = 1;
            } else if (k == idx) { /* R2 / R3 as read */
                mem_row *b = &mem[idx];
                int take;
                if (start_order)
                    take = b->l == 0;
                else
                    take = b->l == 0 || i + l < b->i + b->l ||
                           (i + l == b->i + b->l && l < b->l);
                if (take) {
                    ins = 1;
                    b->i = i;
                    b->l = l;
                    b->r = 1;
                }
            }
        }
        if (ins == 1 && mem[idx].r == mem[idx].l) {
            int32_t nacc = 0; /* levels accepted so far in this emission */
            int32_t *acc_lv = (int32_t *)malloc(sizeof(int32_t) * ((size_t)K + 1));
            if (!acc_lv) {
                free(mem);
                return -1;
            }
            for (int32_t j = idx; j <= K; ++j) {
                if (mem[j].l == 0)
                    continue;
                int accept;
                if (j == idx)
                    accept = 1;
                else if (eq3_ge)
                    accept = mem[j].r - acc >= mem[j].l; /* Eq. 3, ">=" */
                else
                    accept = mem[j].r - acc > mem[j].l; /* Eq. 3 */
                if (accept && disjoint) {
                    /* closed intervals [i, i+l-1] must share no position */
                    for (int32_t q = 0; q < nacc; ++q) {
                        const mem_row *a = &mem[acc_lv[q]];
                        int64_t a_end = a->i + a->l - 1, j_end = mem[j].i + mem[j].l - 1;
                        if (!(j_end < a->i || a_end < mem[j].i))
                            accept = 0;
                    }
                }
                if (nev < cap) {
                    ev_pos[nev] = i;
                    ev_level[nev] = j;
                    ev_i[nev] = mem[j].i;
                    ev_l[nev] = (int32_t)mem[j].l;
                    ev_r[nev] = mem[j].r;
                    ev_acc[nev] = acc;
                    ev_acc_flag[nev] = accept;
                }
                ++nev;
                if (accept) {
                    acc = acc_last ? mem[j].l : acc + mem[j].l;
                    acc_lv[nacc++] = j;
                }
            }
            free(acc_lv);
            idx = K;
            ins = 0;
            acc = 0;
            memset(mem, 0, sizeof(mem_row) * ((size_t)K + 1));
        }
        if (mem[idx].r != mem[idx].l) {
            for (int32_t j = idx; j <= K; ++j)
                mem[j].r += 1;
        }
    }
    free(mem);
    return nev;
}
