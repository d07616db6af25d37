/*
 * Oracle for the segmented wheel sieve -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path (the HIP library) never calls it
 * and shares no code, header, table or helper with it.
 *
 * What it computes: the primes n with lo <= n < hi (half-open range), either
 * their number or the strictly increasing list of them.  This is the plain
 * definition the paper's method reaches exactly (Fig. 1, "all prime numbers
 * from 2 through n"), so the oracle is that definition written out:
 *
 *   1. L = isqrt(hi - 1), by integer Newton iteration (no floating sqrt).
 *   2. Base primes <= L by the textbook Sieve of Eratosthenes on a byte array
 *      (Fig. 1): for i = 2 .. sqrt(L), if A[i] is still set, clear
 *      i*i, i*i+i, ... (marking starts at the square, Sec. 1.1).  2 and 3 are
 *      base primes here: the oracle has no 6k+1/6k+5 wheel at all.
 *   3. The range is cut into windows of ORACLE_WINDOW integers, one byte per
 *      integer (Sec. 2.2: contiguous segments, each owned by one worker, as
 *      in Sec. 2.3).  In each window every base prime p with p*p below the
 *      window end clears its multiples from max(p*p, first multiple >= window
 *      start) on (Sec. 1.1 and Sec. 2.4: generation starts at the square).
 *   4. Entries below 2 are cleared; the survivors are the primes.
 *   5. Windows run on POSIX threads; results are combined in window order.
 *
 * Deliberately absent: the wheel, Table 1, bit packing, presieve patterns and
 * buckets.  Those belong to the method under test, not to its checker.
 *
 * Domain: 0 <= lo <= hi <= 2^63.  Errors are reported as negative returns.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_WINDOW ((uint64_t)1 << 21)
#define ORACLE_MAX_HI ((uint64_t)1 << 63)

/* floor(sqrt(n)) by Newton's iteration on integers. */
uint64_t oracle_isqrt(uint64_t n)
{
    if (n < 2)
        return n;
    int bits = 64 - __builtin_clzll(n);
    uint64_t x = (uint64_t)1 << ((bits + 1) / 2); /* x >= sqrt(n) */
    for (;;) {
        uint64_t y = (x + n / x) >> 1;
        if (y >= x)
            break;
        x = y;
    }
    /* Newton from above lands on floor(sqrt(n)); keep the final correction
       explicit so that the result does not rest on that argument alone.
       Compare by division so that no square can overflow 64 bits. */
    while (x > n / x)
        --x;
    while (x + 1 <= n / (x + 1))
        ++x;
    return x;
}

/* Fig. 1 on [0, L]: returns the number of primes written to *out (malloc'd). */
static int64_t base_primes(uint64_t L, uint32_t **out)
{
    *out = NULL;
    uint8_t *a = (uint8_t *)malloc(L + 1);
    if (!a)
        return -1;
    memset(a, 1, L + 1);
    a[0] = 0;
    if (L >= 1)
        a[1] = 0;
    for (uint64_t i = 2; i * i <= L; ++i)
        if (a[i])
            for (uint64_t j = i * i; j <= L; j += i)
                a[j] = 0;
    uint64_t n = 0;
    for (uint64_t i = 2; i <= L; ++i)
        n += a[i];
    uint32_t *p = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!p) {
        free(a);
        return -1;
    }
    uint64_t k = 0;
    for (uint64_t i = 2; i <= L; ++i)
        if (a[i])
            p[k++] = (uint32_t)i;
    free(a);
    *out = p;
    return (int64_t)n;
}

struct job {
    uint64_t lo, hi;          /* the whole range */
    const uint32_t *primes;   /* base primes, ascending */
    uint64_t np;
    uint64_t nwin;
    uint64_t next;            /* next window index, shared */
    pthread_mutex_t lock;
    uint64_t *win_count;      /* per window */
    void **win_list;          /* per window (list mode), malloc'd */
    int elem_bytes;           /* 0 = count only, 4 or 8 = list */
    int failed;
};

/* Sieve one window [w, we) into buf (one byte per integer). */
static void sieve_window(const struct job *jb, uint64_t w, uint64_t we, uint8_t *buf)
{
    memset(buf, 1, (size_t)(we - w));
    for (uint64_t k = 0; k < jb->np; ++k) {
        uint64_t p = jb->primes[k];
        uint64_t s = p * p;
        if (s >= we)
            break;
        if (s < w)
            s = ((w + p - 1) / p) * p; /* first multiple of p >= w */
        for (uint64_t j = s; j < we; j += p)
            buf[j - w] = 0;
    }
    for (uint64_t n = w; n < we && n < 2; ++n)
        buf[n - w] = 0;
}

static void *worker(void *arg)
{
    struct job *jb = (struct job *)arg;
    uint8_t *buf = NULL;
    uint64_t cap = 0;
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        uint64_t i = jb->next++;
        int stop = jb->failed;
        pthread_mutex_unlock(&jb->lock);
        if (i >= jb->nwin || stop)
            break;
        uint64_t w = jb->lo + i * ORACLE_WINDOW;
        uint64_t we = jb->hi - w < ORACLE_WINDOW ? jb->hi : w + ORACLE_WINDOW;
        if (we - w > cap) {
            free(buf);
            cap = we - w;
            buf = (uint8_t *)malloc((size_t)cap);
            if (!buf) {
                pthread_mutex_lock(&jb->lock);
                jb->failed = 1;
                pthread_mutex_unlock(&jb->lock);
                break;
            }
        }
        sieve_window(jb, w, we, buf);
        uint64_t c = 0;
        for (uint64_t j = 0; j < we - w; ++j)
            c += buf[j];
        jb->win_count[i] = c;
        if (jb->elem_bytes) {
            void *l = malloc((size_t)((c ? c : 1) * (uint64_t)jb->elem_bytes));
            if (!l) {
                pthread_mutex_lock(&jb->lock);
                jb->failed = 1;
                pthread_mutex_unlock(&jb->lock);
                break;
            }
            uint64_t k = 0;
            for (uint64_t j = 0; j < we - w; ++j) {
                if (!buf[j])
                    continue;
                if (jb->elem_bytes == 4)
                    ((uint32_t *)l)[k++] = (uint32_t)(w + j);
                else
                    ((uint64_t *)l)[k++] = w + j;
            }
            jb->win_list[i] = l;
        }
    }
    free(buf);
    return NULL;
}

/* Runs the windows of [lo, hi).  Returns the prime count or a negative error.
   In list mode the concatenated list is written to out when it fits in cap. */
static int64_t run(uint64_t lo, uint64_t hi, int nthreads, int elem_bytes, void *out, uint64_t cap)
{
    if (lo > hi || hi > ORACLE_MAX_HI)
        return -1;
    if (elem_bytes != 0 && elem_bytes != 4 && elem_bytes != 8)
        return -1;
    if (elem_bytes == 4 && hi > ((uint64_t)1 << 32))
        return -1;
    if (lo == hi)
        return 0;
    if (nthreads < 1)
        nthreads = 1;

    struct job jb;
    memset(&jb, 0, sizeof jb);
    jb.lo = lo;
    jb.hi = hi;
    jb.elem_bytes = elem_bytes;
    jb.nwin = (hi - lo + ORACLE_WINDOW - 1) / ORACLE_WINDOW;
    uint32_t *primes = NULL;
    int64_t np = base_primes(oracle_isqrt(hi - 1), &primes);
    if (np < 0)
        return -2;
    jb.primes = primes;
    jb.np = (uint64_t)np;
    jb.win_count = (uint64_t *)calloc(jb.nwin, sizeof(uint64_t));
    jb.win_list = elem_bytes ? (void **)calloc(jb.nwin, sizeof(void *)) : NULL;
    if (!jb.win_count || (elem_bytes && !jb.win_list)) {
        free(primes);
        free(jb.win_count);
        free(jb.win_list);
        return -2;
    }
    pthread_mutex_init(&jb.lock, NULL);

    if ((uint64_t)nthreads > jb.nwin)
        nthreads = (int)jb.nwin;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0;
    for (int t = 0; th && t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, worker, &jb) == 0)
            ++started;
    if (started == 0)
        worker(&jb);
    for (int t = 0; t < started; ++t)
        pthread_join(th[t], NULL);
    free(th);

    int64_t total = jb.failed ? -2 : 0;
    if (!jb.failed)
        for (uint64_t i = 0; i < jb.nwin; ++i)
            total += (int64_t)jb.win_count[i];
    if (elem_bytes && total >= 0 && (uint64_t)total <= cap && out) {
        uint64_t off = 0;
        for (uint64_t i = 0; i < jb.nwin; ++i) {
            memcpy((char *)out + off * (uint64_t)elem_bytes, jb.win_list[i],
                   (size_t)(jb.win_count[i] * (uint64_t)elem_bytes));
            off += jb.win_count[i];
        }
    }
    if (jb.win_list)
        for (uint64_t i = 0; i < jb.nwin; ++i)
            free(jb.win_list[i]);
    free(jb.win_list);
    free(jb.win_count);
    free(primes);
    pthread_mutex_destroy(&jb.lock);
    return total;
}

/* Number of primes in [lo, hi); negative on invalid input or allocation failure. */
int64_t oracle_count(uint64_t lo, uint64_t hi, int nthreads)
{
    return run(lo, hi, nthreads, 0, NULL, 0);
}

/* Primes of [lo, hi) in increasing order as little-endian u32 (elem_bytes 4,
   needs hi <= 2^32) or u64 (elem_bytes 8).  Returns the count; the list is
   written to out only when count <= cap. */
int64_t oracle_list(uint64_t lo, uint64_t hi, void *out, uint64_t cap, int elem_bytes, int nthreads)
{
    if (elem_bytes != 4 && elem_bytes != 8)
        return -1;
    return run(lo, hi, nthreads, elem_bytes, out, cap);
}

/* Primes <= limit from the plain byte sieve of Fig. 1 (no segmentation). */
int64_t oracle_simple_primes(uint64_t limit, uint32_t *out, uint64_t cap)
{
    if (limit >= ((uint64_t)1 << 32))
        return -1;
    uint32_t *p = NULL;
    int64_t n = base_primes(limit, &p);
    if (n < 0)
        return -2;
    if ((uint64_t)n <= cap && out)
        memcpy(out, p, (size_t)n * sizeof(uint32_t));
    free(p);
    return n;
}

/* ------------------------------------------------------------------------
 * Ranges beyond 64 bits (the paper's next step, Sec. 6: numbers past the
 * 64-bit integers).  The same plain definition, with values held as
 * unsigned __int128: base primes are all primes <= isqrt(hi - 1) (listed by
 * the 64-bit sieve above, which needs isqrt(hi - 1) < 2^40), and every
 * window of ORACLE_WINDOW integers clears the multiples of each base prime p
 * from max(p*p, first multiple >= window start) on.  Values are passed and
 * returned as pairs of uint64 (low half first).
 * ------------------------------------------------------------------------ */
typedef unsigned __int128 u128;

static u128 make128(uint64_t lo, uint64_t hi) { return ((u128)hi << 64) | lo; }

/* floor(sqrt(n)) by Newton's iteration on 128-bit integers. */
static u128 isqrt128(u128 n)
{
    if (n < 2)
        return n;
    int bits = 0;
    for (u128 t = n; t; t >>= 1)
        ++bits;
    u128 x = (u128)1 << ((bits + 1) / 2); /* x >= sqrt(n) */
    for (;;) {
        u128 y = (x + n / x) >> 1;
        if (y >= x)
            break;
        x = y;
    }
    while (x > n / x)
        --x;
    while (x + 1 <= n / (x + 1))
        ++x;
    return x;
}

/* The base primes of the last call, kept for the next one with the same
   bound (listing them is most of a small window's cost). */
static pthread_mutex_t wide_lock = PTHREAD_MUTEX_INITIALIZER;
static uint64_t *wide_primes = NULL;
static uint64_t wide_np = 0, wide_bound = 0;

struct wjob {
    u128 lo, hi;
    const uint64_t *primes;
    uint64_t np, nwin, next;
    pthread_mutex_t lock;
    uint64_t *win_count;
    uint64_t **win_list; /* list mode: pairs (lo half, hi half) */
    int list, failed;
};

static void *wide_worker(void *arg)
{
    struct wjob *jb = (struct wjob *)arg;
    uint8_t *buf = (uint8_t *)malloc(ORACLE_WINDOW);
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        uint64_t i = jb->next++;
        int stop = jb->failed || !buf;
        if (!buf)
            jb->failed = 1;
        pthread_mutex_unlock(&jb->lock);
        if (i >= jb->nwin || stop)
            break;
        u128 w = jb->lo + (u128)i * ORACLE_WINDOW;
        u128 we = jb->hi - w < ORACLE_WINDOW ? jb->hi : w + ORACLE_WINDOW;
        uint64_t len = (uint64_t)(we - w);
        memset(buf, 1, len);
        for (uint64_t k = 0; k < jb->np; ++k) {
            u128 p = jb->primes[k];
            u128 s = p * p;
            if (s >= we)
                break;
            if (s < w)
                s = w + (p - w % p) % p; /* first multiple of p >= w */
            for (u128 j = s; j < we; j += p)
                buf[(uint64_t)(j - w)] = 0;
        }
        for (uint64_t j = 0; j < len && w + j < 2; ++j)
            buf[j] = 0;
        uint64_t c = 0;
        for (uint64_t j = 0; j < len; ++j)
            c += buf[j];
        jb->win_count[i] = c;
        if (jb->list) {
            uint64_t *l = (uint64_t *)malloc((size_t)((c ? c : 1) * 2 * sizeof(uint64_t)));
            if (!l) {
                pthread_mutex_lock(&jb->lock);
                jb->failed = 1;
                pthread_mutex_unlock(&jb->lock);
                break;
            }
            uint64_t q = 0;
            for (uint64_t j = 0; j < len; ++j) {
                if (!buf[j])
                    continue;
                u128 v = w + j;
                l[q++] = (uint64_t)v;
                l[q++] = (uint64_t)(v >> 64);
            }
            jb->win_list[i] = l;
        }
    }
    free(buf);
    return NULL;
}

/* Number of primes in [lo, hi) (or, with out, their list as uint64 pairs,
   written when the count fits in cap).  hi - lo < 2^63, isqrt(hi - 1) < 2^40.
   Negative on invalid input or allocation failure. */
int64_t oracle_wide(uint64_t lo_lo, uint64_t lo_hi, uint64_t hi_lo, uint64_t hi_hi, uint64_t *out, uint64_t cap,
                    int nthreads)
{
    const u128 lo = make128(lo_lo, lo_hi), hi = make128(hi_lo, hi_hi);
    if (lo > hi || hi - lo >= ((u128)1 << 63))
        return -1;
    if (lo == hi)
        return 0;
    const u128 L = hi > 1 ? isqrt128(hi - 1) : 0;
    if (L >= ((u128)1 << 40))
        return -1;
    if (nthreads < 1)
        nthreads = 1;

    pthread_mutex_lock(&wide_lock);
    if (!wide_primes || wide_bound != (uint64_t)L) {
        free(wide_primes);
        wide_primes = NULL;
        wide_np = 0;
        int64_t n = oracle_count(0, (uint64_t)L + 1, nthreads);
        uint64_t *p = n >= 0 ? (uint64_t *)malloc((size_t)((n ? n : 1) * sizeof(uint64_t))) : NULL;
        if (!p || oracle_list(0, (uint64_t)L + 1, p, (uint64_t)n, 8, nthreads) != n) {
            free(p);
            pthread_mutex_unlock(&wide_lock);
            return -2;
        }
        wide_primes = p;
        wide_np = (uint64_t)n;
        wide_bound = (uint64_t)L;
    }

    struct wjob jb;
    memset(&jb, 0, sizeof jb);
    jb.lo = lo;
    jb.hi = hi;
    jb.primes = wide_primes;
    jb.np = wide_np;
    jb.list = out != NULL;
    jb.nwin = (uint64_t)((hi - lo + ORACLE_WINDOW - 1) / ORACLE_WINDOW);
    jb.win_count = (uint64_t *)calloc(jb.nwin, sizeof(uint64_t));
    jb.win_list = jb.list ? (uint64_t **)calloc(jb.nwin, sizeof(uint64_t *)) : NULL;
    if (!jb.win_count || (jb.list && !jb.win_list)) {
        free(jb.win_count);
        free(jb.win_list);
        pthread_mutex_unlock(&wide_lock);
        return -2;
    }
    pthread_mutex_init(&jb.lock, NULL);
    if ((uint64_t)nthreads > jb.nwin)
        nthreads = (int)jb.nwin;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0;
    for (int t = 0; th && t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, wide_worker, &jb) == 0)
            ++started;
    if (started == 0)
        wide_worker(&jb);
    for (int t = 0; t < started; ++t)
        pthread_join(th[t], NULL);
    free(th);

    int64_t total = jb.failed ? -2 : 0;
    if (!jb.failed)
        for (uint64_t i = 0; i < jb.nwin; ++i)
            total += (int64_t)jb.win_count[i];
    if (jb.list && total >= 0 && (uint64_t)total <= cap) {
        uint64_t off = 0;
        for (uint64_t i = 0; i < jb.nwin; ++i) {
            memcpy(out + 2 * off, jb.win_list[i], (size_t)(jb.win_count[i] * 2 * sizeof(uint64_t)));
            off += jb.win_count[i];
        }
    }
    if (jb.win_list)
        for (uint64_t i = 0; i < jb.nwin; ++i)
            free(jb.win_list[i]);
    free(jb.win_list);
    free(jb.win_count);
    pthread_mutex_destroy(&jb.lock);
    pthread_mutex_unlock(&wide_lock);
    return total;
}
