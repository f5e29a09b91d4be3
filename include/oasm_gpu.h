/*
 * oasm_gpu -- online approximate string matching on AMD Instinct MI355X.
 *
 * C ABI of the library.  It implements the hot path of OASM ("A novel
 * algorithm for online inexact string matching and its FPGA
 * implementation", Cinti, Bianchi, Martino, Rizzi, arXiv 1712.03560) for a
 * dictionary of byte patterns against any number of byte streams:
 *
 *   1. the hit ends: every end position e of a stream where some substring
 *      t[s..e] is within unit-cost Levenshtein distance K of a pattern
 *      (Section 3, Eq. 1-2; the "Less Naive" scan of Section 5.1, whose
 *      first DP row is all zeros so a match may start anywhere);
 *   2. the hit set at those ends: every (start, length, k <= K) with
 *      length in [l_p - K, l_p + K] (Eq. 2, the per-start distances the
 *      paper's LEV CALC unit produces, Section 6.2);
 *   3. the online shadow-hit filter: Alg. 1 (Section 4) with the priority
 *      rules R1-R3 (Section 4.1) and the validation test Eq. 3 (Section 4.2),
 *      run independently per (stream, pattern) pair, as in the paper's
 *      multi-pattern system where every pattern has its own search unit
 *      (Section 6.4).
 *
 * All arithmetic is integer and exact; the GPU results equal the plain
 * dynamic-programming definition bit for bit.
 *
 * Conventions
 *   - positions are 0-based absolute offsets in a stream (uint64);
 *   - an end position is inclusive; an occurrence (start, len) covers
 *     bytes start .. start+len-1 (the paper's t[i,l]);
 *   - every byte value 0x00-0xFF is a symbol; equality is byte equality;
 *   - a pattern has 1 <= len <= OASM_MAX_PATTERN_LEN and its threshold obeys
 *     0 <= K < len (Section 6.3: the threshold is always lower than the
 *     pattern length).
 *
 * Readings of the paper used by the filter (the paper's pseudo-code and its
 * worked example disagree; the reading below reproduces the example):
 *   - R2 "first encountered": of two overlapping hits of equal priority the
 *     one whose last symbol arrives first wins; on equal ends the shorter
 *     one wins (R3);
 *   - an occurrence completes when its counter reaches its length;
 *   - a lower-priority occurrence is accepted when r(k) - acc > l(k), with
 *     acc the sum of the lengths already accepted in the same emission.
 *
 * Threading: calls on one context are serialised internally.  Different
 * contexts are independent.  All device work runs on one HIP stream per
 * context (the caller's, or one the library creates at default priority).
 *
 * Memory: the library owns the context, its device buffers and its result
 * queues; the caller owns every input and output array passed in.
 */
#ifndef OASM_GPU_H
#define OASM_GPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OASM_VERSION_MAJOR 0
#define OASM_VERSION_MINOR 1

/* Longest supported pattern (eight 32-bit words per pattern column). */
#define OASM_MAX_PATTERN_LEN 256

/* Largest oasm_config.chunk_bytes (16 MiB): the scan records a hit end as
 * its offset inside the chunk, in 24 bits. */
#define OASM_MAX_CHUNK_BYTES (1u << 24)

/* Status codes (negative = error). */
typedef int32_t oasm_status;
#define OASM_OK 0
#define OASM_E_INVAL (-1)  /* bad argument: NULL pointer, len 0, K >= len ... */
#define OASM_E_NOMEM (-2)  /* host or device allocation failed (from oasm_sync or oasm_serve after a
                            * host allocation failed inside a matching step, the context is poisoned) */
#define OASM_E_AGAIN (-3)  /* device-memory budget exhausted: drain / sync, retry */
#define OASM_E_CLOSED (-4) /* feed to a stream that was closed */
#define OASM_E_DEVICE (-5) /* HIP error; the context is poisoned, only destroy is valid */

/* Filtering rules.  OASM_RULES_NONE, or OASM_RULES_PAPER optionally OR-ed
 * with variant bits that replace one reading of Alg. 1 each (Section 4):
 *   ACC_LAST     Eq. 3 with acc = the length of the occurrence accepted last
 *                in the emission (the wording around Eq. 3) instead of the sum
 *                of the lengths accepted so far (Alg. 1's acc update);
 *   EQ3_GE       Eq. 3 as r(k) - acc >= l(k): an occurrence that ends right
 *                before the accepted block (adjacent, disjoint) is accepted;
 *   START_ORDER  R2 literally in start order: an equal-priority hit replaces
 *                the stored one only when its level is empty, so the first
 *                hit examined (earliest start, then shortest) is kept;
 *   DISJOINT     a lower-priority occurrence is accepted only if, besides
 *                Eq. 3, it shares no position with any occurrence accepted
 *                before it in the same emission.
 * The bits combine freely. */
#define OASM_RULES_NONE 0u  /* report hit ends (and the hit set) only */
#define OASM_RULES_PAPER 1u /* Alg. 1 with R1-R3 and Eq. 3 as read above */
#define OASM_RULES_ACC_LAST 2u
#define OASM_RULES_EQ3_GE 4u
#define OASM_RULES_START_ORDER 8u
#define OASM_RULES_DISJOINT 16u

/* Feed flags. */
#define OASM_FEED_LAST 1u /* this feed ends the stream (as oasm_close_stream) */

/* Configuration flags. */
#define OASM_CFG_PLAIN 1u  /* one launch sequence per stream instead of one batched launch */
#define OASM_CFG_KEEP_H 2u /* keep the hit set for draining with OASM_H (debugging) */
#define OASM_CFG_NO_RAW 4u /* do not queue hit ends for draining (they are still computed) */
#define OASM_CFG_AUTOTUNE 8u /* time the scan variants of every pattern class at create and keep the fastest */
#define OASM_CFG_GRAPHS 16u  /* capture a step's launches as HIP graphs when its shape repeats, and replay them */
#define OASM_CFG_NO_CUTOFF 32u /* step every word of multi-word patterns (no word cutoff; same results) */

/* Drain kinds. */
#define OASM_RAW 0u      /* oasm_hit records: hit ends and their distance */
#define OASM_FILTERED 1u /* oasm_occ records: the occurrence set S */
#define OASM_H 2u        /* oasm_occ records: the hit set H (needs OASM_CFG_KEEP_H) */

typedef struct oasm_ctx oasm_ctx;

/* One dictionary entry: `len` bytes at `bytes` (copied by oasm_create). */
typedef struct oasm_pattern {
    const uint8_t *bytes;
    uint32_t len;
} oasm_pattern;

/* A hit end: min over starts of lev(pattern, stream[s..end]) = dist <= K. */
typedef struct oasm_hit {
    uint64_t stream;
    uint64_t end;
    uint32_t pattern;
    uint32_t dist;
} oasm_hit;

/* An occurrence (or, for OASM_H, a hit-set record): lev(pattern,
 * stream[start .. start+len-1]) = k. */
typedef struct oasm_occ {
    uint64_t stream;
    uint64_t start;
    uint32_t pattern;
    uint32_t len;
    uint32_t k;
    uint32_t reserved;
} oasm_occ;

typedef struct oasm_config {
    uint32_t struct_size;        /* sizeof(oasm_config); set by oasm_config_init */
    int32_t device;              /* HIP device ordinal; -1 = the current device */
    void *hip_stream;            /* hipStream_t to run on; NULL = library-owned stream */
    uint32_t chunk_bytes;        /* text bytes per scan work item (rounded down to a multiple of 64, at
                                    least 64, at most OASM_MAX_CHUNK_BYTES); 0 = chosen by the library */
    uint32_t flags;              /* OASM_CFG_* */
    uint64_t device_mem_budget;  /* bytes of fed, not yet matched stream data allowed; 0 = unlimited */
} oasm_config;

/* One segment of a serving run: `len` bytes at `offset` of a device-resident
 * pool, appended to stream `stream`, arriving `arrival_s` seconds after the
 * start of the run. */
typedef struct oasm_segment {
    uint64_t stream;
    uint64_t offset;
    uint32_t len;
    uint32_t flags;     /* OASM_FEED_LAST: the stream ends with this segment */
    double arrival_s;
} oasm_segment;

/* One piece of a batched device feed: `len` bytes at device address `data`
 * appended to stream `stream`. */
typedef struct oasm_feed_seg {
    uint64_t stream;
    const void *data;
    uint64_t len;
    uint32_t flags;     /* OASM_FEED_LAST: the stream ends with this piece */
    uint32_t reserved;  /* 0 */
} oasm_feed_seg;

/* Summary of a serving run. */
typedef struct oasm_serve_report {
    uint64_t segments;        /* segments served */
    uint64_t bytes;           /* bytes served */
    uint64_t steps;           /* matching steps (batches) run */
    uint64_t deferred;        /* loop iterations that left ready segments waiting for memory */
    uint64_t max_batch_bytes; /* largest batch */
    double wall_s;            /* start of the run to the last completion */
    double busy_s;            /* wall_s less the time spent sleeping for arrivals */
} oasm_serve_report;

/* Per-context counters (cumulative since create). */
typedef struct oasm_stats {
    uint64_t bytes_scanned;     /* stream bytes matched */
    uint64_t word_steps;        /* 32-bit pattern-column words advanced by one symbol */
    uint64_t cells;             /* pattern length x stream bytes, summed */
    uint64_t raw_hits;          /* hit ends found */
    uint64_t h_records;         /* hit-set records */
    uint64_t occurrences;       /* filtered occurrences emitted */
    uint64_t syncs;             /* matching steps run */
    double scan_ms;             /* device time of the scan kernels (HIP events) */
    double step_ms;             /* device time of whole steps (HIP events) */
    uint64_t scan_launches;     /* scan kernel launches */
    double sync_wall_ms;        /* host wall time spent inside oasm_sync */
    double wait_ms;             /* part of it spent waiting for the device */
    double host_ms[4];          /* host time per step phase, device waits excluded: plan and
                                   upload; launches (and re-launches after a capacity overflow);
                                   conversion of the results into the drain queues; stream
                                   bookkeeping (look-back tails, closes, carried ends) */
    uint64_t graph_replays;     /* steps launched from captured graphs */
    uint64_t word_steps_done;   /* pattern-column words the scan advanced over the symbols it
                                   reported: word_steps less the words the word cutoff skipped */
} oasm_stats;

/* Fill `cfg` with defaults (device -1, library stream, autotuned chunks). */
oasm_status oasm_config_init(oasm_config *cfg);

/*
 * Create a matching context for `n` patterns.  `k` gives one threshold per
 * pattern, or is NULL to use `k_all` for every pattern.  `rules` is
 * OASM_RULES_NONE, or OASM_RULES_PAPER with any OASM_RULES_* variant bits.
 * `cfg` may be NULL (defaults).
 * Errors: OASM_E_INVAL for n == 0, a NULL pattern, len == 0,
 * len > OASM_MAX_PATTERN_LEN, K >= len, unknown rule bits (variant bits
 * without OASM_RULES_PAPER included), or cfg->chunk_bytes above
 * OASM_MAX_CHUNK_BYTES; OASM_E_NOMEM; OASM_E_DEVICE.
 * On success *out receives the context; on error *out is set to NULL.
 */
oasm_status oasm_create(const oasm_pattern *dict, uint32_t n, const uint16_t *k, uint16_t k_all,
                        uint32_t rules, const oasm_config *cfg, oasm_ctx **out);

/*
 * Append `n` host bytes to stream `stream_id` (created on first use).  The
 * bytes are copied before the call returns.  Matching runs at the next
 * oasm_sync.  Feeds to one stream are concatenated in call order.  With
 * OASM_FEED_LAST the stream is closed after these bytes.
 * Errors: OASM_E_INVAL (ctx NULL, bytes NULL with n > 0), OASM_E_CLOSED,
 * OASM_E_AGAIN (the fed-but-unmatched bytes would exceed device_mem_budget;
 * sync and retry),
 * OASM_E_NOMEM, OASM_E_DEVICE.
 */
oasm_status oasm_feed(oasm_ctx *ctx, uint64_t stream_id, const uint8_t *bytes, size_t n, uint32_t flags);

/*
 * As oasm_feed, for `n` bytes already in device memory at `dev`.  The read
 * is ordered after the work already queued on `hip_stream` (a hipStream_t,
 * or NULL for the null stream); the caller keeps `dev` alive and unchanged
 * until the next oasm_sync returns.
 */
oasm_status oasm_feed_device(oasm_ctx *ctx, uint64_t stream_id, const void *dev, size_t n, void *hip_stream,
                             uint32_t flags);

/*
 * Feed many device buffers in one call: the same as calling
 * oasm_feed_device for segs[0], segs[1], ... in order (a stream may appear
 * several times; its pieces are appended in order), with one mapping launch
 * for all of them.  The buffers are read on the library's stream after the
 * work already queued on `hip_stream` (NULL = the library's stream); the
 * caller keeps them alive until the next oasm_sync.  All or nothing: on
 * error no piece is fed.  Errors: OASM_E_INVAL (NULL segs with n > 0, a NULL
 * data pointer with len > 0, len > 2 GiB, nonzero reserved), OASM_E_CLOSED
 * (a stream closed earlier or by an earlier piece of this call), OASM_E_AGAIN
 * (the pieces together exceed the device-memory budget), OASM_E_NOMEM,
 * OASM_E_DEVICE.
 */
oasm_status oasm_feed_device_many(oasm_ctx *ctx, const oasm_feed_seg *segs, size_t n, void *hip_stream);

/* Close a stream: the next oasm_sync finishes its filter (Alg. 1 run to the
 * last byte).  Closing an unknown or already closed stream is OASM_E_INVAL. */
oasm_status oasm_close_stream(oasm_ctx *ctx, uint64_t stream_id);

/*
 * Match everything fed since the last sync, over all streams (one batched
 * launch sequence, or one per stream with OASM_CFG_PLAIN), wait for it and
 * queue the results for draining.  Occurrences whose fate still depends on
 * bytes not yet fed stay pending until a later sync (or the stream's close).
 * Errors: OASM_E_INVAL (ctx NULL), OASM_E_NOMEM (a host allocation failed
 * inside the step: the context is poisoned, only destroy is valid),
 * OASM_E_DEVICE.
 */
oasm_status oasm_sync(oasm_ctx *ctx);

/*
 * Checkpoint and resume of one stream.  A stream's whole matching state
 * between feeds is small: the scan restarts exactly from the m_max + K_max
 * - 1 symbols before the matched frontier (the bit-parallel column of
 * Section 5.1 depends on no earlier symbol once that many have been read),
 * and Alg. 1's state is empty between segments (Section 4), so the only
 * filter state is the hit ends of the segments still open at the frontier.
 *
 * oasm_stream_export first matches every byte fed so far, as oasm_sync does
 * (queueing the results it completes), then writes the stream's state into
 * `buf`: a self-describing little-endian record of OASM_CKPT_MAGIC,
 * OASM_CKPT_VERSION, a fingerprint of the dictionary, thresholds, rules and
 * symbol classes, the absolute number of bytes matched, the look-back
 * symbols (as the context's symbol classes) and the carried hit ends (end,
 * pattern, least distance and hit-set bytes each).  *size always receives
 * the record's size; with buf NULL nothing else is written (a size query).
 * The stream stays live in `ctx`.  Errors: OASM_E_INVAL (ctx or size NULL,
 * an unknown stream, a stream with a close pending, cap below the size),
 * OASM_E_CLOSED (a closed stream), and those of oasm_sync.
 *
 * oasm_stream_import makes `stream_id` a live stream of `ctx` that holds the
 * exported state: the next bytes fed to it continue the exported stream at
 * the exported position, and its results (positions absolute, from the
 * exported stream's first byte) are those the exported stream would have
 * reported for the same bytes; what the export's context had reported stays
 * reported there.  `ctx` must be built from the same dictionary, thresholds
 * and rules.  The caller owns `buf` (read only during the call).  Errors:
 * OASM_E_INVAL (NULL arguments, a record that is truncated, of another
 * version or of another dictionary, inconsistent fields, a stream id live or
 * closed in `ctx`), OASM_E_NOMEM, OASM_E_DEVICE.
 */
#define OASM_CKPT_MAGIC 0x4D53414Fu /* "OASM" */
#define OASM_CKPT_VERSION 1u
oasm_status oasm_stream_export(oasm_ctx *ctx, uint64_t stream_id, void *buf, size_t cap, size_t *size);
oasm_status oasm_stream_import(oasm_ctx *ctx, uint64_t stream_id, const void *buf, size_t size);

/*
 * Copy up to `cap` queued records of `kind` into `out` (an array of
 * oasm_hit for OASM_RAW, of oasm_occ otherwise) and remove them from the
 * queue.  *n_out receives the number copied; *more (may be NULL) is set to 1
 * when records remain.  Within one sync, records are ordered by stream id,
 * then pattern, then position: the end for OASM_RAW; the emission order of
 * Alg. 1 for OASM_FILTERED (emissions in stream order, and inside one
 * emission its best occurrence first, then the accepted lower-priority ones
 * by ascending k, which start before it); start then length for OASM_H.
 * Syncs follow each other in call order.
 */
oasm_status oasm_hits(oasm_ctx *ctx, uint32_t kind, void *out, size_t cap, size_t *n_out, int *more);

/*
 * Continuous-batching request loop over `n` segments sorted by arrival_s.
 * Segments are admitted in arrival order as soon as they have arrived, while
 * the fed-but-unmatched bytes stay within cfg.device_mem_budget (0 = no
 * limit; one segment is always admitted when nothing is pending).  Admitted
 * segments are copied from `dev_pool` (device memory of `pool_bytes` bytes,
 * owned by the caller) into their streams by one batched kernel per
 * admission, and one matching step runs over every stream with new bytes, so
 * segments of many streams share each launch.  The loop is pipelined: while
 * a step runs on the device, the host converts the previous step's results
 * and admits and copies the segments that arrive (queued behind the running
 * step); when the step ends, the segments that arrived meanwhile are admitted
 * too and the next step is launched at once.  Bytes fed before the run (not
 * yet matched) are matched with the first step.  The loop runs in real time:
 * when nothing is ready or running it sleeps until the next arrival.
 * latency_s (optional, n entries) receives, per segment, the time from its
 * arrival to the moment the results of the step that matched it are queued
 * (its hit ends are then drainable and its filter has advanced as far as the
 * bytes allow).
 * Results are queued as by oasm_sync.  `report` (optional) is written on
 * every return, errors included: segments are served in arrival order, so
 * the served ones are segs[0 .. report->segments).  Errors: OASM_E_INVAL
 * (NULL pointers, unsorted arrivals, a segment outside the pool, a segment
 * for a closed stream: that iteration's batch is refused whole, before any
 * stream changes), OASM_E_NOMEM (device staging memory: the batch is refused
 * whole and the context stays usable; a host allocation: the context is
 * poisoned), OASM_E_DEVICE.
 */
oasm_status oasm_serve(oasm_ctx *ctx, const oasm_segment *segs, size_t n, const void *dev_pool, uint64_t pool_bytes,
                       double *latency_s, oasm_serve_report *report);

/*
 * LEV CALC for every start (Section 6, the LEV CORE description: at each new
 * stream index i the distances between p and the 2K+1 substrings
 * t[i, l_p-K] .. t[i, l_p+K]; Section 6.2 computes them by Eq. 1).  For every
 * pattern p of the context's dictionary and every start i of the `n` bytes at
 * `dev_text` (device memory), writes 2K_p + 1 bytes to `dev_out` (device
 * memory), for l = m_p - K_p + j, j = 0 .. 2K_p:
 *     min(lev(p, t[i, l]), K_p + 1)   when i + l <= n,
 *     255                             when t[i, l] runs past the text end.
 * Layout: pattern-major; pattern p's block starts at byte
 * n * sum over q < p of (2K_q + 1), and inside it start i's bytes are at
 * i * (2K_p + 1).  The entries <= K_p are exactly the hit set H of Eq. 2.
 * The text is one independent string (no stream state, no filter); the
 * context's streams are not touched.  The work is queued on `hip_stream`
 * (a hipStream_t, NULL = the null stream) and the call returns without
 * waiting; the caller keeps both buffers alive until that stream has passed
 * this point (oasm_destroy waits for the last such point, since the kernels
 * read the context's dictionary).  The first call uploads two small tables
 * (synchronously).
 * Errors: OASM_E_INVAL (NULL pointers with n > 0, out_bytes below the size
 * that oasm_levcalc_size gives), OASM_E_DEVICE (the context is poisoned).
 */
oasm_status oasm_levcalc(oasm_ctx *ctx, const void *dev_text, size_t n, void *dev_out, size_t out_bytes,
                         void *hip_stream);

/* Largest dictionary oasm_levcalc_noalloc accepts. */
#define OASM_NOALLOC_MAX_PATTERNS 65536u

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * call and the same output as oasm_levcalc, but it allocates nothing and
 * copies nothing from the host.  oasm_levcalc's two small tables (the pattern
 * ids grouped by word count, and per pattern the sum of 2K + 1 over the
 * patterns before it, which places its output block) are built on its first
 * call in device memory it allocates; here they are built by a kernel, at
 * every call, in a fixed device array that the library holds per GPU until
 * the process ends (OASM_NOALLOC_MAX_PATTERNS x 12 bytes = 768 KiB).  Every
 * call on a GPU, from any context, writes that GPU's array: calls that
 * overlap in time on one GPU (on different HIP streams, or from different
 * threads) race and may write wrong distances; calls queued on one stream
 * are ordered.  The caller passes the text and the output, as for
 * oasm_levcalc.  Errors: those of oasm_levcalc, and OASM_E_INVAL for a
 * context of more than OASM_NOALLOC_MAX_PATTERNS patterns.
 */
oasm_status oasm_levcalc_noalloc(oasm_ctx *ctx, const void *dev_text, size_t n, void *dev_out, size_t out_bytes,
                                 void *hip_stream);

/* Bytes oasm_levcalc writes for a text of n bytes: n * sum over patterns of
 * (2K + 1).  OASM_E_INVAL for NULL arguments or a size that overflows. */
oasm_status oasm_levcalc_size(const oasm_ctx *ctx, size_t n, size_t *bytes);

/* Number of records of `kind` queued for draining (OASM_E_INVAL for an
 * unknown kind, or OASM_H without OASM_CFG_KEEP_H). */
oasm_status oasm_queued(const oasm_ctx *ctx, uint32_t kind, size_t *n);

/* Cumulative counters and device timings. */
oasm_status oasm_get_stats(const oasm_ctx *ctx, oasm_stats *out);

/* Free the context and everything it owns (NULL is a no-op).  Waits for
 * the context's device work to finish, LEV CALC launches included. */
void oasm_destroy(oasm_ctx *ctx);

/* The scan variants in use and how they were chosen: one line per variant
 * the autotuner timed ("W=<words> P=<patterns per lane> lds=<0|1>
 * cut=<0|1>: <ms> ...", only with OASM_CFG_AUTOTUNE and for classes not
 * already in the process-wide cache), then one line per word-count class
 * ("class W=<words>: P=.. lds=.. cut=.. tiles=.."). */
const char *oasm_tune_report(const oasm_ctx *ctx);

/* Message for the last error on this context (never NULL). */
const char *oasm_last_error(const oasm_ctx *ctx);

/* Name of a status code. */
const char *oasm_status_str(oasm_status s);

#ifdef __cplusplus
}
#endif

#endif /* OASM_GPU_H */
