/*
 * sieve.h -- C ABI of the MI355X segmented wheel sieve (libsieve.so).
 *
 * The library counts and lists the primes of half-open integer ranges
 * [lo, hi) with the incremental segmented Sieve of Eratosthenes over the
 * 6k+1 / 6k+5 wheel of Ning & Kaeli, "Memory Efficient Multithreaded
 * Incremental Segmented Sieve Algorithm" (arXiv 2310.17746):
 *   - only values congruent to 1 or 5 mod 6 are stored, in two arrays A_one
 *     and A_five (Sec. 2.1, Fig. 2), here bit-packed planes in LDS;
 *   - the range is cut into contiguous segments, each owned by one worker
 *     (Sec. 2.2, 2.3), here one workgroup per segment ("tile");
 *   - each base prime P starts at max(P*P, segment start) (Sec. 1.1, 2.4),
 *     at the indices given by Table 1 (Sec. 3), and strides by P indices;
 *   - the survivors are counted, or listed in increasing order (Fig. 1;
 *     Fig. 4 outputs every index left unmarked in either array).
 * 2 and 3 lie outside the wheel and are reported when in range; 1 is not
 * prime and never reported.
 *
 * Conventions for every call:
 *   - Ranges are half-open [lo, hi) with 0 <= lo <= hi <= SIEVE_MAX_HI.
 *     lo == hi is an empty range; lo > hi is SIEVE_E_INVAL.
 *   - Sieving [lo, hi) needs every prime <= isqrt(hi - 1) resident on the
 *     device (sieve_base_primes); otherwise the call returns SIEVE_E_RANGE.
 *   - Every call returns an int status (SIEVE_OK or a negative code).  No
 *     C++ exception crosses this ABI.  The last status of a context is kept
 *     (sieve_last_error).
 *   - The caller owns every buffer it passes, host or device; the library
 *     never frees or retains them after the call returns.
 *   - `stream` arguments take a hipStream_t (for instance
 *     torch.cuda.current_stream().cuda_stream).  NULL selects the context's
 *     own stream, and the call returns when its work has finished (host
 *     outputs are then valid).  A non-NULL stream makes sieve_list,
 *     sieve_count_batch and sieve_list_batch stream-ordered: the job is
 *     enqueued after earlier work on that stream and the call returns; the
 *     host outputs (counts, status, *n_out) are written when the stream
 *     reaches the end of the job, so they are valid after the stream
 *     synchronizes, and the caller keeps those host arrays alive until then.
 *     A job that needs a host decision mid-way (ranges that take the bucket
 *     sieve, whose estimated layout may have to be re-run exactly, and jobs
 *     cut into pieces by the bucket budget) waits for its stream before
 *     returning, with the outputs then valid.  Jobs of one context on
 *     different streams run one after another (the context's scratch is
 *     shared).
 *   - A context is not thread-safe, except for the sieve_server_* calls.
 */
#ifndef SIEVE_H
#define SIEVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define SIEVE_OK 0
#define SIEVE_E_INVAL (-1)     /* bad argument: lo > hi, hi too large, NULL pointer, bad param */
#define SIEVE_E_RANGE (-2)     /* base primes do not cover isqrt(hi - 1) */
#define SIEVE_E_CAPACITY (-3)  /* list longer than the output capacity; count still reported */
#define SIEVE_E_DTYPE (-4)     /* elem_bytes not 4/8, or 4 with hi - 1 > 2^32 - 1 */
#define SIEVE_E_NOMEM (-5)     /* device or host allocation failed */
#define SIEVE_E_DEVICE (-6)    /* HIP runtime error, no device, wrong architecture */
#define SIEVE_E_BUSY (-7)      /* server queue full */
#define SIEVE_E_CANCELLED (-8) /* request cancelled before it finished */
#define SIEVE_E_IO (-9)        /* a file could not be created or written */
#define SIEVE_E_LIMIT (-10)    /* more than the fixed scratch of an allocation-free call holds */

/* Largest accepted hi (ranges are [lo, hi) with hi <= 2^63). */
#define SIEVE_MAX_HI ((uint64_t)1 << 63)

typedef struct sieve_ctx sieve_ctx;

/*
 * Tuning parameters (the paper's inputs t, N, S of Fig. 4 become workgroup
 * size, range and segment bytes).  Zero in any field selects the default.
 *   segment_bytes    LDS bytes per tile for the two bit planes together;
 *                    a multiple of 4096 in [8192, 159744] (156 KiB, leaving
 *                    room for the kernel's static LDS in 160 KiB); default
 *                    155648 (152 KiB: one tile per compute unit).  A tile
 *                    covers 24 * segment_bytes consecutive integers.
 *   block_threads    threads per workgroup: 256, 512 or 1024 (default 1024).
 *   presieve_groups  number of repeating-pattern groups used to initialise
 *                    the planes (0..6; 6 covers every prime 5..73).  0 means
 *                    default (6); SIEVE_PRESIEVE_NONE disables the presieve.
 *   split_hits       target hits per marking work item (default 64): primes
 *                    with more hits per tile are split over several lanes.
 *   bucket_threshold primes at least this large go through the bucket
 *                    sieve on ranges of two or more tiles.  0 (default):
 *                    four plane lengths (16 * segment_bytes), and only on
 *                    ranges with at least 32768 such primes; any other
 *                    value applies to every multi-tile range;
 *                    SIEVE_BUCKET_NEVER disables the bucket sieve.
 *   wg_per_cu        persistent workgroups launched per compute unit
 *                    (default: as many tiles as fit in 160 KiB, at most 4).
 *   use_graph        1: batched calls replay a captured hipGraph.
 *   bucket_slices    bucket storage layout: 0 (default) sizes each tile's
 *                    slice from the expected hit count plus a wide margin
 *                    and re-runs a job exactly when a slice overflows;
 *                    SIEVE_BUCKET_EXACT always counts first (two passes);
 *                    SIEVE_BUCKET_TINY gives every slice one entry, which
 *                    exercises the overflow re-run (tests).
 *   cofactor_skip    where marks whose cofactor is a multiple of 5 are
 *                    skipped (such values are already cleared by the 5 of the
 *                    presieve): SIEVE_SKIP_SPLIT in the bucket sieve and for
 *                    the primes whose tile work is split over several lanes
 *                    (the small ones, many hits), except the fixed-mask
 *                    ones; 0 (default) the same, plus the fixed-mask items
 *                    when the shape runs four waves per SIMD (one 1024- or
 *                    two 512-thread workgroups per CU); SIEVE_SKIP_ALL in
 *                    every per-tile marking loop but the carried-register
 *                    one; SIEVE_SKIP_NONE nowhere.  Needs presieve_groups
 *                    >= 1.
 *   dense_hits       primes with at least this many hits per plane per tile
 *                    (default 512) are split over a multiple of 32 lanes, so
 *                    that each lane's hits share one bit position and need
 *                    one add each; SIEVE_DENSE_NEVER disables it.
 *   bucket_mem_mb    device memory one job may use for bucket entries, in
 *                    MiB (default 16384).  A job whose estimate is larger runs
 *                    as a sequence of jobs over tile-aligned pieces of its
 *                    ranges; results are the same.
 *   visit_order      order in which the sieve kernel's workgroups take the
 *                    ranges' tiles: SIEVE_VISIT_COSTLY_FIRST (0, default:
 *                    most Table 1 starts per tile first), SIEVE_VISIT_REVERSED
 *                    (that order reversed) or SIEVE_VISIT_SHUFFLED (a fixed
 *                    pseudo-random permutation of the ranges).  Results do not
 *                    depend on it; the other two exist for testing.
 *   strip_tiles      tiles per strip, 1..64 (0, default: about a sixteenth of
 *                    a resident workgroup's share of the job's tiles, at
 *                    most 64).  A workgroup sieves the tiles of a strip in
 *                    order and carries each prime's next hit from one tile
 *                    to the next (Sec. 2.4), so a prime takes one Table 1
 *                    start per strip instead of one per tile.  Results do not
 *                    depend on it.
 */
typedef struct sieve_params {
    uint32_t segment_bytes;
    uint32_t block_threads;
    uint32_t presieve_groups;
    uint32_t split_hits;
    uint32_t bucket_threshold;
    uint32_t wg_per_cu;
    uint32_t use_graph;
    uint32_t bucket_slices;
    uint32_t cofactor_skip;
    uint32_t bucket_mem_mb;
    uint32_t dense_hits;
    uint32_t visit_order;
    uint32_t strip_tiles;
    uint32_t reserved[3];
} sieve_params;

#define SIEVE_PRESIEVE_NONE 0xFFFFFFFFu
#define SIEVE_BUCKET_NEVER 0xFFFFFFFFu
#define SIEVE_BUCKET_EXACT 1u
#define SIEVE_BUCKET_TINY 2u
#define SIEVE_SKIP_ALL 1u
#define SIEVE_SKIP_NONE 2u
#define SIEVE_SKIP_SPLIT 3u
#define SIEVE_DENSE_NEVER 0xFFFFFFFFu
#define SIEVE_VISIT_COSTLY_FIRST 0u
#define SIEVE_VISIT_REVERSED 1u
#define SIEVE_VISIT_SHUFFLED 2u

/* Fills *p with the library defaults for gfx950. */
int sieve_default_params(sieve_params *p);

/*
 * Creates a context on HIP device `device` (must be gfx950).  The context
 * owns the resident base primes (the paper's Sieve Data Store, Sec. 4),
 * presieve pattern tables, scratch, captured graphs and a stream.
 * p == NULL selects the defaults: one 1024-thread workgroup per CU with a
 * 152 KiB tile, the best single shape measured over the workloads (the
 * binding's autotuner, autotune.py, picks a shape per workload class on the
 * GPU at hand and passes it here).  On success *ctx is set.
 */
int sieve_create(sieve_ctx **ctx, int device, const sieve_params *p);

/* Releases every resource of ctx (NULL is accepted). */
int sieve_destroy(sieve_ctx *ctx);

/* Copies the parameters the context actually uses into *p. */
int sieve_get_params(const sieve_ctx *ctx, sieve_params *p);

/*
 * Makes every prime <= limit resident on the device: the Sieve Data Store of
 * Sec. 4 (sieving a range needs the primes up to the square root of its
 * end).  Grow-only and idempotent: a
 * smaller limit than the current one does nothing.  limit < 2^32.  The
 * primes beyond isqrt(limit) are produced by this library's own GPU list
 * path.  *n_out (optional) receives the number of resident primes >= 5.
 */
int sieve_base_primes(sieve_ctx *ctx, uint64_t limit, uint64_t *n_out);

/* Current base-prime limit (0 when none are resident). */
int sieve_base_limit(const sieve_ctx *ctx, uint64_t *limit);

/*
 * Number of primes in [lo, hi) into *count (host): the primes of Fig. 1's
 * problem over a segment range (Sec. 2.2), counted from the unmarked entries
 * of A_one / A_five (Fig. 4) plus 2 and 3.  Synchronous, on the context
 * stream.
 */
int sieve_count(sieve_ctx *ctx, uint64_t lo, uint64_t hi, uint64_t *count);

/*
 * Writes the primes of [lo, hi) in strictly increasing order to out_dev: the
 * output of Fig. 1 (all primes of the range) as Fig. 4 produces it, every
 * index left unmarked in either array in value order, here a contiguous
 * array instead of the linked list of Sec. 4.  out_dev is device memory
 * owned by the caller, elem_bytes = 4 for uint32 or 8 for uint64,
 * little-endian, contiguous.  *n_out (required) receives the count.  If the
 * count exceeds cap, nothing is guaranteed to be written and *n_out holds the
 * required count; a synchronous call then returns SIEVE_E_CAPACITY, a
 * stream-ordered one returns SIEVE_OK and the caller sees *n_out > cap after
 * the stream synchronizes.  elem_bytes = 4 needs hi - 1 <= 2^32 - 1, else
 * SIEVE_E_DTYPE.
 */
int sieve_list(sieve_ctx *ctx, uint64_t lo, uint64_t hi, void *out_dev, uint64_t cap,
               int elem_bytes, uint64_t *n_out, void *stream);

/*
 * Batched count over n ranges lo[i], hi[i] (host arrays) in one persistent
 * launch: the segments of every range (Sec. 2.2) are the work units of one
 * pool of workers (Sec. 2.3, Fig. 4's worker loop).  counts[i] (host)
 * receives the prime count of range i.  Any invalid range fails the whole
 * call before launch.
 */
int sieve_count_batch(sieve_ctx *ctx, const uint64_t *lo, const uint64_t *hi, uint64_t n,
                      uint64_t *counts, void *stream);

/*
 * Mixed batch (Sec. 2.2-2.3 as for sieve_count_batch; listed ranges produce
 * Fig. 4's output as sieve_list does).  For range i (host arrays): mode[i] =
 * 0 counts, 1 also lists the primes into out_dev at element offset off[i]
 * with capacity cap[i]
 * (elements of elem_bytes).  counts[i] (host) receives every range's count;
 * status[i] (host) receives SIEVE_OK or, for a list range that does not fit,
 * SIEVE_E_CAPACITY (its count is still reported; other ranges are not
 * affected).  The call returns SIEVE_OK when every range was processed even
 * if some status[i] is SIEVE_E_CAPACITY.  off/cap may be NULL when no range
 * lists.  List outputs of different ranges must not overlap.
 */
int sieve_list_batch(sieve_ctx *ctx, const uint64_t *lo, const uint64_t *hi,
                     const uint8_t *mode, uint64_t n, void *out_dev, const uint64_t *off,
                     const uint64_t *cap, int elem_bytes, uint64_t *counts, int32_t *status,
                     void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * batched count as sieve_count_batch, with every piece of job scratch (job
 * header, range and visit tables, counters, per-range counts and status) in
 * one fixed device array of SIEVE_STATIC_SCRATCH_BYTES per GPU, held by the
 * library until the process ends.  The call makes no device or host
 * allocation: it uses the context's resident base primes (which must already
 * cover isqrt(hi - 1) of every range, else SIEVE_E_RANGE; they are not
 * grown), plans into fixed host arrays, copies the plan into the scratch,
 * launches the sieve kernels on `stream` (NULL: the context stream) and
 * waits for them; counts[i] (host) then holds the number of primes in
 * [lo[i], hi[i]).  Every range runs the per-tile marking path: no bucket
 * sieve and no split tiles (their scratch grows with the job), so the
 * results equal sieve_count_batch's and long ranges near 2^50 are slower.
 * Limit: n <= SIEVE_STATIC_MAX_RANGES, else SIEVE_E_LIMIT before any device
 * work.  All calls on one GPU share its scratch array, so calls that overlap
 * on the same GPU (from several threads or contexts) race; the library
 * serialises the calls of one process with a lock.
 */
#define SIEVE_STATIC_MAX_RANGES 1024
#define SIEVE_STATIC_SCRATCH_BYTES 168448
int sieve_count_batch_static(sieve_ctx *ctx, const uint64_t *lo, const uint64_t *hi, uint64_t n,
                             uint64_t *counts, void *stream);

/*
 * Windows beyond the 64-bit calls' domain.  Sec. 6 names ranges past 2^64 as
 * the step after this method; these calls take the same wheel sieve there.
 * A value is a sieve_u128 (lo = bits 0..63, hi = bits 64..127).  A window
 * [lo, hi) must satisfy 2^40 <= lo <= hi and hi - lo <= SIEVE_WIDE_MAX_SPAN,
 * else SIEVE_E_INVAL (ranges below 2^40 belong to the 64-bit calls).  The
 * window is sieved in offsets from its base W = lo - lo mod 6: bit i of
 * plane A_r stands for W + 6i + r (Sec. 2.1 with the segment base W), each
 * base prime P starts from (W - 1) mod P through Table 1 (Sec. 3) or at P*P
 * when that lies past W (Sec. 2.4), and the survivors are counted or listed
 * as W + offset.  Base primes: every prime below 2^32 resident plus an
 * extension list of 64-bit primes from 2^32 up to the extension limit; a
 * window needs isqrt(hi - 1) within them, else SIEVE_E_RANGE.  A window
 * whose bucket entries would exceed bucket_mem_mb runs as equal pieces of
 * whole tiles.  These calls wait for the context's earlier stream-ordered
 * jobs, run on `stream` (NULL: the context stream) and return when done.
 */
typedef struct sieve_u128 {
    uint64_t lo, hi;
} sieve_u128;

#define SIEVE_WIDE_MIN_LO ((uint64_t)1 << 40)
#define SIEVE_WIDE_MAX_SPAN ((uint64_t)1 << 40)
#define SIEVE_WIDE_MAX_BASE ((uint64_t)1 << 36)

/*
 * Makes the base primes cover `limit` <= SIEVE_WIDE_MAX_BASE (else
 * SIEVE_E_INVAL): below 2^32 this is sieve_base_primes(limit); above, every
 * prime below 2^32 becomes resident and the primes in [2^32, limit] are
 * produced by this library's own 64-bit list path into the extension list
 * (8 bytes each on the device).  A smaller limit than the current one does
 * nothing.  *n_out (optional) receives resident plus extension primes.
 */
int sieve_base_primes_wide(sieve_ctx *ctx, uint64_t limit, uint64_t *n_out);

/* Current extension limit (0 when there is no extension list). */
int sieve_ext_limit(const sieve_ctx *ctx, uint64_t *limit);

/*
 * Number of primes in the window [*lo, *hi) into *count (host); lo, hi and
 * count are host pointers.
 */
int sieve_count_wide(sieve_ctx *ctx, const sieve_u128 *lo, const sieve_u128 *hi, uint64_t *count,
                     void *stream);

/*
 * Writes the primes of the window [*lo, *hi) in strictly increasing order
 * to out_dev (device memory owned by the caller, cap 16-byte elements, each
 * a sieve_u128); *n_out (host, required) receives the count.  If the count
 * exceeds cap nothing is guaranteed to be written, *n_out holds the required
 * count and the call returns SIEVE_E_CAPACITY.  out_dev may be NULL with
 * cap 0 to ask for the count only.
 */
int sieve_list_wide(sieve_ctx *ctx, const sieve_u128 *lo, const sieve_u128 *hi, sieve_u128 *out_dev,
                    uint64_t cap, uint64_t *n_out, void *stream);

/*
 * A rigorous upper bound on the number of primes in [lo, hi), used for
 * output sizing and admission: the minimum of (values coprime to 6 in the
 * range + 2) and the Brun-Titchmarsh bound 2y/ln y (y = hi - lo > 1) of
 * Montgomery and Vaughan (Mathematika 20, 1973), rounded up.
 */
uint64_t sieve_list_bound(uint64_t lo, uint64_t hi);

/*
 * Table 1 (Sec. 3) for one prime, evaluated by the library's own wheel
 * start-offset code compiled for the host: for a prime p >= 5, a segment
 * whose index 0 stands for the values base + 1 and base + 5 (base a
 * multiple of 6) and a first value M >= 1, *id1 and *id5 receive the indices
 * in A_one / A_five of the first multiple of p that is >= M.  Requires
 * base <= M < base + 2^22 (M lies within one tile of the base, as in the
 * kernels) and p < 2^32; otherwise SIEVE_E_INVAL.
 * Host-only, no device work.
 */
int sieve_wheel_start(uint64_t p, uint64_t base, uint64_t M, int64_t *id1, int64_t *id5);

/*
 * Tile plan of one range for a given segment size (host-only): *ntiles
 * receives the number of tiles, *base the value base of tile 0 (a multiple
 * of 6), *last_words the plane words of the last tile.
 */
int sieve_plan_range(uint64_t lo, uint64_t hi, uint32_t segment_bytes, uint64_t *ntiles,
                     uint64_t *base, uint32_t *last_words);

/*
 * Event timing of the job phases, for measurement: when on, every
 * non-graph job records the duration of its sieve kernel, of its
 * finalize + compaction kernels and of its bucket-sieve kernels (count,
 * scan, fill), with HIP events on the stream the kernels run on.
 * sieve_get_timing returns the sums in milliseconds and the number of jobs
 * timed; sieve_set_timing resets them.
 */
int sieve_set_timing(sieve_ctx *ctx, int on);
int sieve_get_timing(const sieve_ctx *ctx, double *sieve_ms, double *post_ms, double *bucket_ms,
                     uint64_t *jobs);

/* ------------------------------------------------------------------------
 * Incremental generation (Sec. 2.4: the sieve keeps producing primes from
 * where it stopped, and the Sieve Data Store of Sec. 4 grows as the squares
 * of new primes are reached).  A generator hands out the primes >= start in
 * increasing order, n at a time, with no upper limit fixed in advance.  It
 * sieves blocks of whole tiles ahead of its cursor into a device staging
 * buffer it owns and extends the context's base primes as needed.
 * ------------------------------------------------------------------------ */
typedef struct sieve_gen sieve_gen;

/* Creates a generator on ctx starting at value `start`, handing out elements
 * of elem_bytes (4: its value domain ends at 2^32; 8: at SIEVE_MAX_HI).
 * start beyond the domain end is SIEVE_E_INVAL.  The generator borrows ctx:
 * ctx must outlive it and calls on the two must not overlap. */
int sieve_gen_create(sieve_ctx *ctx, uint64_t start, int elem_bytes, sieve_gen **gen);

/* Writes the next n primes of the generator in increasing order to out_dev
 * (device memory owned by the caller, room for n elements) and advances past
 * them.  *n_out receives the number written: n, or fewer once the end of the
 * value domain is reached (later calls write 0).  Synchronous on `stream`
 * (NULL: the context stream). */
int sieve_gen_next(sieve_gen *gen, uint64_t n, void *out_dev, uint64_t *n_out, void *stream);

/* *next receives the generator's position: every prime below it has been
 * handed out and none at or above it (the start value before the first
 * prime; the domain end once exhausted). */
int sieve_gen_position(const sieve_gen *gen, uint64_t *next);

/* Frees the generator (NULL is accepted); the context is not affected. */
int sieve_gen_destroy(sieve_gen *gen);

/* ------------------------------------------------------------------------
 * Streaming output to the host and to files (the Prime Number Data Store of
 * Sec. 4, written out to files as Sec. 6 proposes).  The range is cut into
 * pieces whose rigorous prime bound (sieve_list_bound) is at most
 * piece_elems (0: 2^24 elements; at least 256); piece k+1 is sieved on the
 * context stream while piece k is copied to the host on a second stream and
 * piece k-1 is consumed by a host task.  The context keeps two device and
 * two pinned host buffers of piece_elems elements between calls.  Base
 * primes must cover isqrt(hi - 1) as for sieve_list.
 * ------------------------------------------------------------------------ */

/* Lists the primes of [lo, hi) in increasing order into out_host (host
 * memory owned by the caller, pageable or pinned; pinned memory is written by
 * DMA directly).  *n_out receives the count.  If it exceeds cap the call
 * returns SIEVE_E_CAPACITY, *n_out holds the required count and the contents
 * of out_host are unspecified.  elem_bytes 4 needs hi - 1 <= 2^32 - 1. */
int sieve_list_host(sieve_ctx *ctx, uint64_t lo, uint64_t hi, void *out_host, uint64_t cap,
                    int elem_bytes, uint64_t piece_elems, uint64_t *n_out);

/* Writes the primes of [lo, hi) in increasing order to the files
 * "<path_prefix>.000000", "<path_prefix>.000001", ... as raw little-endian
 * elements of elem_bytes.  Every file but the last holds exactly
 * primes_per_file primes (0: 125,000,000); an empty range creates no file.
 * *n_out receives the count and *n_files the number of files created.
 * SIEVE_E_IO when a file cannot be created or written (files written so far
 * stay in place). */
int sieve_write_files(sieve_ctx *ctx, uint64_t lo, uint64_t hi, const char *path_prefix,
                      uint64_t primes_per_file, int elem_bytes, uint64_t piece_elems,
                      uint64_t *n_out, uint64_t *n_files);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of range queries.
 *
 * A server owns a context (no other call may use that context while the
 * server exists) and runs a scheduler thread.  Requests wait in FIFO order
 * until a slot is free and, for list requests, their output fits the
 * server's device output arena (the output-memory budget; a list request
 * reserves sieve_list_bound(lo, hi) elements).  Every scheduler step runs one
 * batched job over tile-aligned pieces of all active requests: each active
 * request gets up to `quantum_tiles` tiles per step (round-robin), at most
 * `step_tiles` tiles per step in total, so a long request shares the device
 * with short ones.  A request completes when its last piece finishes; its
 * result is identical to a stand-alone sieve_count / sieve_list of the range.
 * Base primes grow on demand.  Every server call is thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct sieve_server sieve_server;

typedef struct sieve_server_params {
    uint64_t out_budget_bytes; /* device output arena; default 1 GiB */
    uint32_t max_active;       /* requests on the device at once; default 1024 */
    uint32_t step_tiles;       /* tiles per scheduler step; default 16 per CU */
    uint32_t quantum_tiles;    /* tiles per request per step; default step_tiles / 16 */
    uint32_t elem_bytes;       /* list element size, 4 or 8; default 8 */
    uint32_t max_queue;        /* submitted but not admitted; default 1 << 20 */
    uint32_t overlap;          /* 1: step k + 1 is planned and enqueued while step k runs
                                  (hides host planning, costs arrivals one step of waiting);
                                  0 (default): one step on the device at a time */
    uint32_t restart_walks;    /* 1: every piece of a request starts its bucket walks afresh;
                                  0 (default): a request cut into pieces keeps its large
                                  primes' bucket walk state on the device from one piece to
                                  the next (Sec. 2.4's incremental state): 16 bytes per bucket
                                  prime, twice, while the request is active */
} sieve_server_params;

/* One finished request.  Times are nanoseconds on the server's steady clock
 * (0 = server creation): arrival (submit time or the scheduled arrival),
 * admission (first piece on the device) and completion. */
typedef struct sieve_completion {
    uint64_t tag;
    uint64_t count;       /* primes in [lo, hi) */
    uint64_t lo, hi;
    uint64_t t_arrival_ns, t_admit_ns, t_done_ns;
    int32_t status;       /* SIEVE_OK, SIEVE_E_CANCELLED, SIEVE_E_NOMEM, ... */
    int32_t mode;         /* 0 count, 1 list */
} sieve_completion;

typedef struct sieve_server_stats {
    uint64_t steps;           /* scheduler steps run */
    uint64_t tiles;           /* tiles sieved */
    uint64_t ints;            /* integers sieved */
    uint64_t completed;       /* requests completed (any status) */
    uint64_t busy_ns;         /* device time of the steps' jobs (events around each job) */
    uint64_t elapsed_ns;      /* time since creation */
    uint64_t arena_peak_bytes;
    uint64_t queued, active;  /* at the time of the call */
    uint64_t bucket_steps;    /* steps whose job used the bucket sieve */
    uint64_t overlap_steps;   /* steps enqueued while the previous step was still running */
    uint64_t resumed_walks;   /* pieces whose bucket walks resumed from the state their
                                 request's previous piece left on the device */
    uint64_t walk_bytes;      /* device memory held for resident walk state (pooled) */
} sieve_server_stats;

/* Creates a server on ctx (p == NULL: defaults).  *srv is set on success. */
int sieve_server_create(sieve_ctx *ctx, const sieve_server_params *p, sieve_server **srv);

/* Queues a request for [lo, hi); mode 0 counts, 1 lists.  `tag` identifies it
 * in completions (tags must be unique among live requests).  Never blocks;
 * SIEVE_E_BUSY when the queue is full, SIEVE_E_INVAL on a bad range. */
int sieve_submit(sieve_server *srv, uint64_t lo, uint64_t hi, int mode, uint64_t tag);

/* As sieve_submit, but the request becomes visible to the scheduler only at
 * t_arrival_ns on the server clock (an open-loop load generator). */
int sieve_submit_at(sieve_server *srv, uint64_t lo, uint64_t hi, int mode, uint64_t tag,
                    uint64_t t_arrival_ns);

/* As sieve_submit, with the list written straight into caller-owned device
 * memory instead of the server's arena (a submit that takes out and cap):
 * for mode 1, out_dev (required, aligned to elem_bytes) receives the
 * primes of [lo, hi) in increasing order, at most cap elements.  No arena
 * space is reserved and nothing is to be fetched; the completion's count is
 * the number of primes.  If that exceeds cap the request still counts every
 * piece, completes with SIEVE_E_CAPACITY and the full count, and nothing is
 * guaranteed written.  The caller keeps out_dev alive until the completion.
 * For mode 0 out_dev and cap are ignored. */
int sieve_submit_out(sieve_server *srv, uint64_t lo, uint64_t hi, int mode, void *out_dev, uint64_t cap,
                     uint64_t tag);

/* Moves up to max finished requests into buf; waits up to wait_ms for at
 * least one (0: no wait).  *n_out receives the number moved. */
int sieve_poll(sieve_server *srv, sieve_completion *buf, int max, int wait_ms, int *n_out);

/* Cancels a queued or active request: it completes with SIEVE_E_CANCELLED.
 * SIEVE_E_INVAL if no live request has that tag. */
int sieve_cancel(sieve_server *srv, uint64_t tag);

/* Copies a completed list request's primes to dst (device or host memory,
 * at most cap elements of the server's elem_bytes) and frees its arena space.
 * *n_out receives the count.  SIEVE_E_CAPACITY (nothing copied, space kept)
 * if cap is too small; SIEVE_E_INVAL for an unknown tag. */
int sieve_server_fetch(sieve_server *srv, uint64_t tag, void *dst, uint64_t cap, uint64_t *n_out);

/* Frees a completed list request's arena space without copying. */
int sieve_server_release(sieve_server *srv, uint64_t tag);

int sieve_server_get_stats(sieve_server *srv, sieve_server_stats *st);

/* Current time on the server clock (ns since creation). */
uint64_t sieve_server_now_ns(const sieve_server *srv);

/* Stops the scheduler (pending requests are dropped) and frees the server;
 * the context can be used again afterwards. */
int sieve_server_destroy(sieve_server *srv);

/* Text for a status code (static storage). */
const char *sieve_strerror(int status);

/* Last status returned by a call on ctx. */
int sieve_last_error(const sieve_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SIEVE_H */
