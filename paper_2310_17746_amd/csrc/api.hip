// Host runtime and C ABI of libsieve (declared in include/sieve.h).
//
// Owns the context: the resident base primes (the paper's Sieve Data Store,
// Sec. 4) with their per-prime constants, the presieve pattern tables, the
// marking work items, grow-only device scratch, pinned staging, a stream and
// captured graphs.  Every count / list / batch call is planned here (ranges
// cut into tiles of 192 * PW integers, Sec. 2.2) and executed as one job:
// zero -> [bucket fill] -> sieve (persistent) -> segment sums -> finalize ->
// segment scan -> compact; a job whose bucket entries would exceed the
// budget runs as a sequence of jobs over tile-aligned pieces.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "sieve.h"
#include "runtime.h"
#include "sieve_internal.h"
#include "wheel.h"

namespace sieve {
hipError_t set_sieve_lds_limit(uint32_t bytes);
hipError_t launch_zero(const JobHeader *job, unsigned long long *counters, unsigned long long *counts,
                       uint32_t *bcount, uint32_t *gbm, uint32_t *garrive, unsigned long long *tally, hipStream_t s);
hipError_t launch_bucket(const BucketArgs &a, int pass, uint32_t cus, hipStream_t s);
hipError_t launch_bucket_scan(const BucketScanArgs &a, hipStream_t s);
hipError_t launch_sieve(const SieveArgs &a, uint32_t nt, uint32_t wg_per_cu, uint32_t grid, bool u24, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs &a, uint32_t grid, hipStream_t s);
hipError_t launch_seg(const SegArgs &a, int pass, uint32_t grid, hipStream_t s);
hipError_t launch_compact(const CompactArgs &a, uint32_t grid, hipStream_t s);
}  // namespace sieve

using namespace sieve;
using sieve::rt::DevBuf;
using sieve::rt::WalkSpec;

namespace {

// Presieve groups: consecutive primes, each group's period (their product)
// below 2^19 bits.
const uint32_t kGroupPrimes[kMaxGroups][4] = {
    {5, 7, 11, 13}, {17, 19, 23, 0}, {29, 31, 37, 0}, {41, 43, 47, 0}, {53, 59, 61, 0}, {67, 71, 73, 0}};

constexpr uint32_t kFinalizeGrid = 256;

uint64_t isqrt_host(uint64_t n)
{
    if (n < 2)
        return n;
    uint64_t x = (uint64_t)std::sqrt((double)n);
    while (x > n / x)
        --x;
    while (x + 1 <= n / (x + 1))
        ++x;
    return x;
}

// Primes 5..limit by a host Eratosthenes (Fig. 1).  Used only to bootstrap
// the device list path with the primes up to isqrt(limit).
std::vector<uint32_t> host_small_primes(uint64_t limit)
{
    std::vector<uint32_t> out;
    if (limit < 5)
        return out;
    std::vector<uint8_t> a(limit + 1, 1);
    for (uint64_t i = 2; i * i <= limit; ++i)
        if (a[i])
            for (uint64_t j = i * i; j <= limit; j += i)
                a[j] = 0;
    for (uint64_t i = 5; i <= limit; ++i)
        if (a[i])
            out.push_back((uint32_t)i);
    return out;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed device scratch of sieve_count_batch_static, the entry point for
// callers that cannot allocate.  It holds one job of at most
// kStaticMaxRanges count-only ranges: the job header, the range and visit
// tables, the job counters and the per-range counts and status.  Every GPU
// the library runs on holds its own copy for the life of the process; host
// code reaches it only through the address hipGetSymbolAddress returns on
// that device (kept in the context as static_scratch), never by the
// array's name.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct StaticLayout {
    static constexpr size_t ranges = align256(sizeof(JobHeader));
    static constexpr size_t visit = align256(ranges + sizeof(RangeDesc) * kStaticMaxRanges);
    static constexpr size_t counters = align256(visit + sizeof(VisitEntry) * kStaticMaxRanges);
    static constexpr size_t counts = align256(counters + sizeof(unsigned long long) * kNumCounters);
    static constexpr size_t status = align256(counts + sizeof(unsigned long long) * kStaticMaxRanges);
    static constexpr size_t total = align256(status + sizeof(int32_t) * kStaticMaxRanges);
};

static_assert(StaticLayout::total == SIEVE_STATIC_SCRATCH_BYTES, "sieve.h states the scratch size");

static __device__ __align__(256) unsigned char scratch[StaticLayout::total];

// Host side of the static path: the plan is built in these arrays (no heap
// allocation) under g_static_mu, then copied into the device scratch.
std::mutex g_static_mu;
JobHeader g_static_job;
RangeDesc g_static_ranges[kStaticMaxRanges];
VisitEntry g_static_visit[kStaticMaxRanges];
uint32_t g_static_order[kStaticMaxRanges];

}  // namespace

namespace {

int set_err(sieve_ctx *c, int e)
{
    if (c)
        c->last_error = e;
    return e;
}

int hip_status(hipError_t e)
{
    if (e == hipSuccess)
        return SIEVE_OK;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? SIEVE_E_NOMEM : SIEVE_E_DEVICE;
}

void fill_defaults(sieve_params &p)
{
    // Defaults for MI355X: one 1024-thread workgroup per CU with a 152 KiB
    // tile (nearly all of the 160 KiB of LDS), so that the 128 VGPRs of four
    // waves per SIMD hold the primes' carried state; work items of ~64 hits.
    if (!p.segment_bytes)
        p.segment_bytes = 152 * 1024;
    if (!p.block_threads)
        p.block_threads = 1024;
    if (!p.presieve_groups)
        p.presieve_groups = kMaxGroups;
    if (!p.split_hits)
        p.split_hits = 64;
    if (!p.wg_per_cu)
        p.wg_per_cu = std::max<uint32_t>(1, std::min<uint32_t>(4, (160 * 1024) / p.segment_bytes));
    if (!p.bucket_mem_mb)
        p.bucket_mem_mb = 16384;  // 16 GiB of the 288 GiB HBM
    if (!p.dense_hits)
        p.dense_hits = 512;
}

int validate_params(const sieve_params &p, uint32_t lds_max)
{
    if (p.segment_bytes < 8192 || p.segment_bytes % 4096 || p.segment_bytes > lds_max ||
        p.segment_bytes > 256 * 1024)
        return SIEVE_E_INVAL;
    if (p.block_threads != 256 && p.block_threads != 512 && p.block_threads != 1024)
        return SIEVE_E_INVAL;
    if (p.presieve_groups > kMaxGroups && p.presieve_groups != SIEVE_PRESIEVE_NONE)
        return SIEVE_E_INVAL;
    if (p.split_hits < 8)
        return SIEVE_E_INVAL;
    if (p.wg_per_cu < 1 || p.wg_per_cu > 16)
        return SIEVE_E_INVAL;
    if (p.bucket_slices > SIEVE_BUCKET_TINY || p.cofactor_skip > SIEVE_SKIP_SPLIT)
        return SIEVE_E_INVAL;
    if (p.visit_order > SIEVE_VISIT_SHUFFLED)
        return SIEVE_E_INVAL;
    if (p.strip_tiles > kMaxStrip)
        return SIEVE_E_INVAL;
    return SIEVE_OK;
}

// Builds the presieve tables and uploads them.  The first `ng` groups hold
// their patterns; the rest get an all-zero table (period 64) so that the
// kernel applies every group unconditionally.
int build_presieve(sieve_ctx *c, uint32_t ng)
{
    std::vector<uint2> tab;
    c->ngroups = ng;
    c->restore1 = c->restore5 = 0;
    for (uint32_t g = 0; g < (uint32_t)kMaxGroups; ++g) {
        const bool on = g < ng;
        uint32_t P = 1;
        if (on)
            for (int i = 0; i < 4 && kGroupPrimes[g][i]; ++i)
                P *= kGroupPrimes[g][i];
        else
            P = 64;
        const uint32_t nw = (P + 64 + 31) / 32 + 1;
        PsGroup &G = c->groups[g];
        G.period = P;
        G.offset = (uint32_t)tab.size();
        G.step = (32u * c->prm.block_threads) % P;
        tab.resize(tab.size() + nw, make_uint2(0, 0));
        if (!on)
            continue;
        for (uint32_t t = 0; t < nw * 32; ++t) {
            const uint64_t tt = t % P;
            const uint64_t v1 = 6 * tt + 1, v5 = 6 * tt + 5;
            bool c1 = false, c5 = false;
            for (int i = 0; i < 4 && kGroupPrimes[g][i]; ++i) {
                c1 |= v1 % kGroupPrimes[g][i] == 0;
                c5 |= v5 % kGroupPrimes[g][i] == 0;
            }
            if (c1)
                tab[G.offset + t / 32].x |= 1u << (t % 32);
            if (c5)
                tab[G.offset + t / 32].y |= 1u << (t % 32);
        }
        for (int i = 0; i < 4 && kGroupPrimes[g][i]; ++i) {
            const uint32_t p = kGroupPrimes[g][i];
            if (p % 6 == 1)
                c->restore1 |= 1u << ((p - 1) / 6);
            else
                c->restore5 |= 1u << ((p - 5) / 6);
        }
    }
    if (!c->d_pstab.reserve(tab.size()))
        return SIEVE_E_NOMEM;
    return hip_status(hipMemcpy(c->d_pstab.p, tab.data(), tab.size() * sizeof(uint2), hipMemcpyHostToDevice));
}

// Installs c->h_primes as the resident base primes: per-prime constants, the
// pi index and the marking work items.
int install_primes(sieve_ctx *c, uint64_t limit)
{
    const std::vector<uint32_t> &P = c->h_primes;
    const size_t n = P.size();
    std::vector<PrimeConst> prm(std::max<size_t>(n, 1), PrimeConst{0, 0, 0, 0});
    for (size_t k = 0; k < n; ++k)
        prm[k] = make_prime_const(P[k]);
    const size_t np = limit / 64 + 2;
    std::vector<uint32_t> pidx(np);
    size_t k = 0;
    for (size_t s = 0; s < np; ++s) {
        while (k < n && P[k] <= 64 * s)
            ++k;
        pidx[s] = (uint32_t)k;
    }
    // Presieved primes are never marked in LDS.
    uint32_t maxps = 0;
    for (uint32_t g = 0; g < c->ngroups; ++g)
        for (int i = 0; i < 4 && kGroupPrimes[g][i]; ++i)
            maxps = std::max(maxps, kGroupPrimes[g][i]);
    uint32_t fm = 0;
    while (fm < n && P[fm] <= maxps)
        ++fm;
    // Work items: a prime with more than split_hits hits per plane per tile
    // is split over g lanes; lane j takes hits j, j + g, j + 2g, ...
    const uint64_t plane_bits = (uint64_t)(c->prm.segment_bytes / 8) * 32;
    std::vector<uint2> items;
    std::vector<uint32_t> prefix(1, 0);
    // A prime with at least dense_hits hits per plane is split over a
    // multiple of 32 lanes: a lane's hits are then 32k P bits = kP words
    // apart and share one bit position (fixed-mask marking).
    uint32_t ks = fm, kd = fm;
    while (ks < n) {
        const uint64_t hits = plane_bits / P[ks];
        uint64_t g;
        if (c->prm.dense_hits != SIEVE_DENSE_NEVER && hits >= c->prm.dense_hits && kd == ks) {
            g = 32 * std::max<uint64_t>(1, hits / (32ull * c->prm.split_hits));
            g = std::min<uint64_t>(g, 0xFFE0);
            if (g % 5 == 0)
                g -= 32;  // a lane's cofactors then run through every residue mod 5
            kd = ks + 1;
        } else {
            g = plane_bits / ((uint64_t)P[ks] * c->prm.split_hits);
            if (g <= 1)
                break;
            g = std::min<uint64_t>(g, 0xFFFF);
            if (g % 5 == 0)
                --g;  // a lane's cofactors then run through every residue mod 5
        }
        for (uint32_t j = 0; j < g; ++j)
            items.push_back(make_uint2(ks, (j << 16) | (uint32_t)g));
        prefix.push_back((uint32_t)items.size());
        ++ks;
    }
    if (items.empty())
        items.push_back(make_uint2(0, 0));
    // {P, dlt}: the A_five multiples of P lie dlt indices after the A_one
    // ones (P (P + 4) or P (P + 2) after P * P)
    std::vector<uint2> prd(std::max<size_t>(n, 1), make_uint2(0, 0));
    for (size_t k = 0; k < n; ++k)
        prd[k] = make_uint2(P[k], P[k] % 6 == 1 ? 2 * (P[k] - 1) / 3 : (P[k] - 2) / 3);
    if (!c->d_prm.reserve(prm.size(), &c->gen) || !c->d_prd.reserve(prd.size(), &c->gen) ||
        !c->d_pidx.reserve(pidx.size(), &c->gen) || !c->d_items.reserve(items.size(), &c->gen) ||
        !c->d_item_prefix.reserve(prefix.size(), &c->gen))
        return SIEVE_E_NOMEM;
    hipError_t e = hipMemcpy(c->d_prm.p, prm.data(), prm.size() * sizeof(PrimeConst), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->d_prd.p, prd.data(), prd.size() * sizeof(uint2), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->d_pidx.p, pidx.data(), pidx.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->d_items.p, items.data(), items.size() * sizeof(uint2), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->d_item_prefix.p, prefix.data(), prefix.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return hip_status(e);
    c->inv_prefix.assign(n + 1, 0.0);
    for (size_t j = 0; j < n; ++j)
        c->inv_prefix[j + 1] = c->inv_prefix[j] + 1.0 / P[j];
    // Bucket sieve: primes at least the threshold (default four plane lengths,
    // where a prime hits a given tile with probability below 1/2).
    const uint64_t thr = c->prm.bucket_threshold ? (uint64_t)c->prm.bucket_threshold : 4 * plane_bits;
    uint32_t kl = (uint32_t)n;
    if (c->prm.bucket_threshold != SIEVE_BUCKET_NEVER)
        kl = (uint32_t)(std::lower_bound(P.begin(), P.end(), (uint32_t)std::min<uint64_t>(thr, 0xFFFFFFFFull)) -
                        P.begin());
    c->k_large = std::max(kl, ks);
    c->limit = limit;
    c->h_pidx = std::move(pidx);
    c->first_mark = fm;
    c->k_split = ks;
    c->k_dense = kd;
    c->gen++;  // kernel arguments changed: a captured graph is stale
    return SIEVE_OK;
}

// Tile plan of [lo, hi): tile 0 starts at base = lo - lo % 6; the plane-1
// index count decides the words (plane 5 never has more indices).
void plan_range(uint64_t lo, uint64_t hi, uint32_t pw, uint64_t &ntiles, uint64_t &base, uint32_t &last_words)
{
    base = lo - lo % 6;
    ntiles = 0;
    last_words = 0;
    if (hi <= base + 1)
        return;
    const uint64_t n1 = (hi - base - 1 + 5) / 6;
    const uint64_t words = (n1 + 31) / 32;
    ntiles = (words + pw - 1) / pw;
    last_words = (uint32_t)(words - (ntiles - 1) * pw);
}

uint32_t strip_tiles(const sieve_ctx *c, uint64_t job_tiles)
{
    if (c->prm.strip_tiles)
        return std::min<uint32_t>(c->prm.strip_tiles, kMaxStrip);
    const uint64_t wgs = (uint64_t)c->cus * c->prm.wg_per_cu;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(kMaxStrip, job_tiles / (16 * wgs)));
}

void set_strips(RangeDesc &d, uint32_t S)
{
    d.strip = d.nparts > 1 ? 1u : std::max<uint32_t>(1, std::min<uint32_t>(S, d.ntiles));
    d.nstrips = (d.ntiles + d.strip - 1) / d.strip;
}

// Sieve work units of a range: its strips, or every part of every tile of a
// split range.
uint64_t range_units(const RangeDesc &d)
{
    return d.nparts > 1 ? (uint64_t)d.ntiles * d.nparts : d.nstrips;
}

struct Plan {
    std::vector<RangeDesc> ranges;
    uint64_t nlist = 0;  // ranges in list mode
    uint64_t ntiles = 0, nchunks = 0, nunits = 0, nseg = 0;
    uint64_t best = 0;  // bucket entries of the estimated layout
    uint32_t bwin = 0;  // most tiles in one bucket window
    uint64_t nvisit = 0, gtiles = 0;  // sieve work units; tiles of split ranges
};

// Number of base primes <= x, for x <= c->limit: the pi index gives the
// count up to 64 floor(x / 64) and a short scan adds the primes above it (a
// binary search over all base primes costs a cache miss per step).
uint32_t primes_upto(const sieve_ctx *c, uint64_t x)
{
    const std::vector<uint32_t> &P = c->h_primes;
    size_t k = c->h_pidx[x / 64];
    while (k < P.size() && P[k] <= x)
        ++k;
    return (uint32_t)k;
}

int make_plan(const sieve_ctx *c, uint64_t n, const uint64_t *lo, const uint64_t *hi, const uint8_t *mode,
              const uint64_t *off, const uint64_t *cap, int elem_bytes, Plan &pl)
{
    const uint32_t pw = c->prm.segment_bytes / 8;
    pl.ranges.resize(n);
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t a = lo[i], b = hi[i];
        if (a > b || b > SIEVE_MAX_HI)
            return SIEVE_E_INVAL;
        const uint64_t root = b > 4 ? isqrt_host(b - 1) : 0;  // largest prime that marks
        if (root > c->limit)
            return SIEVE_E_RANGE;
        const bool lst = mode && mode[i];
        if (lst && elem_bytes == 4 && b > a && b - 1 > 0xFFFFFFFFull)
            return SIEVE_E_DTYPE;
        RangeDesc &d = pl.ranges[i];
        memset(&d, 0, sizeof d);
        d.lo = a;
        d.hi = b;
        uint64_t nt;
        plan_range(a, b, pw, nt, d.base, d.last_words);
        if (nt > 0xFFFFFFFFull)
            return SIEVE_E_INVAL;
        d.ntiles = (uint32_t)nt;
        d.tile0 = pl.ntiles;
        pl.ntiles += nt;
        // Base primes with p * p < hi; on multi-tile ranges the ones from
        // k_large on go through the bucket sieve.
        d.nact = b > 4 ? primes_upto(c, root) : 0u;
        // A range takes the bucket sieve when it spans several tiles and its
        // large primes are many: each then costs one start per tile window
        // instead of one per tile, and only its actual hits are walked.
        // (An explicit threshold applies to every multi-tile range.)
        const uint32_t min_large = c->prm.bucket_threshold ? 1u : kBucketMinPrimes;
        d.kbig = (nt >= 2 && d.nact >= c->k_large + min_large) ? c->k_large : d.nact;
        d.bwins = (uint32_t)((nt + kBucketWindow - 1) / kBucketWindow);
        d.bunits = d.kbig < d.nact ? ((d.nact - d.kbig + kBucketThreads - 1) / kBucketThreads) * d.bwins : 0;
        d.bunit0 = pl.nunits;
        pl.nunits += d.bunits;
        if (d.bunits) {
            pl.bwin = std::max(pl.bwin, (uint32_t)std::min<uint64_t>(nt, kBucketWindow));
            // Expected entries per tile: each large prime p hits a plane of
            // nbits bits nbits/p times on average; reserve that plus a
            // margin of 8 standard deviations (the count is a sum of nearly
            // independent rare events) and 64.
            const double nbits = 32.0 * pw;
            const double E = 2.0 * nbits * (c->inv_prefix[d.nact] - c->inv_prefix[d.kbig]);
            const double capd = E + 8.0 * std::sqrt(E) + 64.0;
            d.bcap = c->prm.bucket_slices == SIEVE_BUCKET_TINY ? 1u : (uint32_t)std::min(capd, 4.0e9);
            d.bbase = pl.best;
            pl.best += (uint64_t)d.bcap * nt;
        }
        d.nparts = 1;  // split tiles are chosen below, once the job's size is known
        d.mode = lst ? 1u : 0u;
        if (lst) {
            d.out_off = off ? off[i] : 0;
            d.cap = cap ? cap[i] : 0;
            const uint64_t nch =
                nt ? (nt - 1) * (pw / kChunkWords) + (d.last_words + kChunkWords - 1) / kChunkWords : 0;
            if (nch > 0xFFFFFFFFull)
                return SIEVE_E_INVAL;
            d.nchunks = (uint32_t)nch;
            d.chunk0 = pl.nchunks;
            pl.nchunks += nch;
            pl.nlist++;
            d.nseg = (uint32_t)((nch + kSegChunks - 1) / kSegChunks);
        }
        // every range carries the running segment index, so that seg0 + nseg
        // never decreases along the table (count ranges add no segment)
        if (pl.nseg + d.nseg > 0xFFFFFFFFull)
            return SIEVE_E_INVAL;
        d.seg0 = (uint32_t)pl.nseg;
        pl.nseg += d.nseg;
    }
    // Split tiles.  A tile's own loop starts min(nact, kbig) primes; one whose
    // loop is far longer than a resident workgroup's share of the whole job
    // would finish last, so its primes beyond the split items go to parts of
    // C = max(kPartPrimes, share) primes, each on its own workgroup (part 0
    // also takes the items); their marks meet in a global copy of the planes.
    double starts = 0;
    for (uint64_t i = 0; i < n; ++i)
        starts += (double)pl.ranges[i].ntiles * std::min(pl.ranges[i].nact, pl.ranges[i].kbig);
    const double share = starts / ((double)c->cus * c->prm.wg_per_cu);
    const uint32_t C = (uint32_t)std::min(std::max((double)kPartPrimes, share), 2.0e9);
    for (uint64_t i = 0; i < n; ++i) {
        RangeDesc &d = pl.ranges[i];
        const uint32_t n_loop = std::min(d.nact, d.kbig);
        if (d.ntiles && n_loop > c->k_split && (uint64_t)(n_loop - c->k_split) > 2ull * C) {
            if (pl.gtiles + d.ntiles > 0xFFFFFFFFull)
                return SIEVE_E_INVAL;
            d.nparts = (uint32_t)(((uint64_t)n_loop - c->k_split + C - 1) / C);
            d.part_primes = C;
            d.gtile0 = (uint32_t)pl.gtiles;
            pl.gtiles += d.ntiles;
        }
    }
    // Strips: a workgroup sieves S consecutive tiles of a range and carries
    // each prime's next hit from tile to tile.  S is about a sixteenth of a
    // resident workgroup's share of the job's tiles (so the dynamic hand-out
    // of strips still balances), at most kMaxStrip.
    const uint32_t S = strip_tiles(c, pl.ntiles);
    for (uint64_t i = 0; i < n; ++i) {
        RangeDesc &d = pl.ranges[i];
        set_strips(d, S);
        pl.nvisit += range_units(d);
    }
    return SIEVE_OK;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct BlobLayout {
    size_t ranges, visit, links, total;
};

BlobLayout blob_layout(uint64_t nranges)
{
    BlobLayout L;
    const uint64_t n = std::max<uint64_t>(nranges, 1);
    L.ranges = align_up(sizeof(JobHeader), 256);
    L.visit = align_up(L.ranges + sizeof(RangeDesc) * n, 256);
    L.links = align_up(L.visit + sizeof(VisitEntry) * n, 256);
    L.total = align_up(L.links + sizeof(WalkLink) * n, 256);
    return L;
}

uint64_t grow(uint64_t cur, uint64_t need, uint64_t floor_)
{
    if (need <= cur)
        return cur;
    return std::max(std::max(need, floor_), cur + cur / 2);
}

// Makes the scratch hold a job of the given size.  Capacities only grow; any
// reallocation bumps c->gen so that captured graphs are re-made.
int ensure_capacity(sieve_ctx *c, uint64_t nranges, uint64_t nchunks, uint64_t ntiles, uint64_t gtiles)
{
    bool changed = false;
    if (nranges > c->cap_ranges || nchunks > c->cap_chunks || ntiles > c->cap_tiles || gtiles > c->cap_gtiles) {
        // Buffers are about to be replaced: earlier stream-ordered jobs, and
        // their pending copies into the host slots, finish first.
        if (hipDeviceSynchronize() != hipSuccess) {
            (void)hipGetLastError();
            return SIEVE_E_DEVICE;
        }
    }
    if (nranges > c->cap_ranges || !c->d_blob.p) {
        c->cap_ranges = grow(c->cap_ranges, nranges, 64);
        const BlobLayout L = blob_layout(c->cap_ranges);
        c->d_blob.release();
        c->d_counts.release();
        c->d_status.release();
        if (!c->d_blob.reserve(L.total) || !c->d_counts.reserve(c->cap_ranges) ||
            !c->d_status.reserve(c->cap_ranges))
            return SIEVE_E_NOMEM;
        for (auto &sl : c->slot) {
            if (sl.blob)
                (void)hipHostFree(sl.blob);
            if (sl.counts)
                (void)hipHostFree(sl.counts);
            if (sl.status)
                (void)hipHostFree(sl.status);
            sl.blob = nullptr;
            sl.counts = nullptr;
            sl.status = nullptr;
            if (hipHostMalloc((void **)&sl.blob, L.total, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void **)&sl.counts, c->cap_ranges * sizeof(unsigned long long),
                              hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void **)&sl.status, c->cap_ranges * sizeof(int32_t), hipHostMallocDefault) !=
                    hipSuccess) {
                (void)hipGetLastError();
                return SIEVE_E_NOMEM;
            }
        }
        c->h_blob_n = L.total;
        changed = true;
    }
    if (nchunks > c->cap_chunks || !c->d_bitmap.p) {
        c->cap_chunks = grow(c->cap_chunks, nchunks, 64);
        c->d_bitmap.release();
        c->d_chunk_counts.release();
        c->d_chunk_vbase.release();
        c->d_chunk_off.release();
        c->d_seg_sum.release();
        c->d_seg_base.release();
        // segments: at most one per chunk (every segment holds at least one)
        if (!c->d_bitmap.reserve(c->cap_chunks * kChunkWords) || !c->d_chunk_counts.reserve(c->cap_chunks) ||
            !c->d_chunk_vbase.reserve(c->cap_chunks) || !c->d_chunk_off.reserve(c->cap_chunks) ||
            !c->d_seg_sum.reserve(c->cap_chunks) || !c->d_seg_base.reserve(c->cap_chunks))
            return SIEVE_E_NOMEM;
        changed = true;
    }
    if (ntiles > c->cap_tiles || !c->d_bcount.p) {
        c->cap_tiles = grow(c->cap_tiles, ntiles, 1024);
        c->d_bcount.release();
        c->d_bcursor.release();
        c->d_boff.release();
        if (!c->d_bcount.reserve(c->cap_tiles) || !c->d_bcursor.reserve(c->cap_tiles) ||
            !c->d_boff.reserve(c->cap_tiles + 1))
            return SIEVE_E_NOMEM;
        changed = true;
    }
    if (gtiles > c->cap_gtiles || !c->d_garrive.p) {
        c->cap_gtiles = grow(c->cap_gtiles, gtiles, 16);
        c->d_gbm.release();
        c->d_garrive.release();
        if (!c->d_gbm.reserve(c->cap_gtiles * 2 * (c->prm.segment_bytes / 8)) ||
            !c->d_garrive.reserve(c->cap_gtiles))
            return SIEVE_E_NOMEM;
        changed = true;
    }
    if (!c->d_bdata.p) {
        c->cap_bdata = 1024;
        if (!c->d_bdata.reserve(c->cap_bdata))
            return SIEVE_E_NOMEM;
        changed = true;
    }
#ifdef SIEVE_MARK_COUNT
    if (!c->d_tally.p) {
        if (!c->d_tally.reserve(4) ||
            hipHostMalloc((void **)&c->h_tally, 4 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return SIEVE_E_NOMEM;
        }
        changed = true;
    }
#endif
    if (!c->d_counters.p) {
        if (!c->d_counters.reserve(kNumCounters))
            return SIEVE_E_NOMEM;
        if (hipHostMalloc((void **)&c->slot[0].flag, 2 * sizeof(unsigned long long), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&c->slot[1].flag, 2 * sizeof(unsigned long long), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&c->h_btotal, sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return SIEVE_E_NOMEM;
        }
        changed = true;
    }
    if (changed)
        c->gen++;
    return SIEVE_OK;
}

// Where the sieve kernel skips marks whose cofactor is a multiple of 5 (the
// presieve has cleared them): SieveArgs::skip5.  By default the split items
// skip them, and the fixed-mask (dense) items too in the launch shapes of
// four waves per SIMD, whose time goes to LDS operations; the shape of six
// waves per SIMD is bound by VALU issue, where the skip's setup costs more
// than the ORs it saves.
uint32_t skip5_mode(const sieve_ctx *c)
{
    if (c->ngroups < 1 || c->prm.cofactor_skip == SIEVE_SKIP_NONE)
        return 0;
    if (c->prm.cofactor_skip == SIEVE_SKIP_ALL)
        return 1;
    if (c->prm.cofactor_skip == SIEVE_SKIP_SPLIT)
        return 2;
    const bool six = c->prm.block_threads < 1024 && (c->prm.block_threads / 64) * c->prm.wg_per_cu >= 24;
    return six ? 2u : 3u;
}

enum Phase { kPhaseWhole = 0, kPhaseBucketCount = 1, kPhaseRest = 2, kPhaseDirect = 3 };

// Enqueues one phase of the job kernels on stream s; also used under graph
// capture.  All job-specific values are read by the kernels from the device
// blob, whose layout depends only on the capacities.
//   whole:         zero, sieve, finalize, compact       (jobs without buckets)
//   direct:        zero, estimated bucket fill, sieve, finalize, compact
//   bucket count:  zero, exact bucket count, bucket scan
//   rest:          exact bucket fill, sieve, finalize, compact
// With lists false (a job with no list range, launched directly) the segment
// scans and the compaction, which would find no chunk, are not launched;
// a captured graph always holds them, since it replays for any job.
hipError_t enqueue_phase(sieve_ctx *c, hipStream_t s, int phase, bool timed, bool lists)
{
    const BlobLayout L = blob_layout(c->cap_ranges);
    const JobHeader *job = (const JobHeader *)c->d_blob.p;
    const RangeDesc *ranges = (const RangeDesc *)(c->d_blob.p + L.ranges);
    const uint32_t pw = c->prm.segment_bytes / 8;
    hipError_t e = hipSuccess;
    BucketArgs b;
    memset(&b, 0, sizeof b);
    b.job = job;
    b.ranges = ranges;
    b.prm = c->d_prm.p;
    b.bcount = c->d_bcount.p;
    b.bcursor = c->d_bcursor.p;
    b.boff = c->d_boff.p;
    b.bdata = c->d_bdata.p;
    b.counters = c->d_counters.p;
    b.skip5 = (c->ngroups >= 1 && c->prm.cofactor_skip != SIEVE_SKIP_NONE) ? 1u : 0u;
    b.nbits = 32 * pw;
    b.span = 192ull * pw;
    b.span_rcp = UINT64_MAX / b.span;
    b.win = c->bucket_win ? c->bucket_win : kBucketWindow;
    b.tally = c->d_tally.p;  // allocated in the debug build only
    b.links = (const WalkLink *)(c->d_blob.p + L.links);
    const uint32_t bcus = (uint32_t)c->cus;
    if (phase != kPhaseRest) {
        if (timed && phase == kPhaseBucketCount && (e = hipEventRecord(c->ev[3], s)) != hipSuccess)
            return e;
        // per-tile counts (exact layout) or cursors (estimated layout) start at 0
        uint32_t *bzero = phase == kPhaseDirect ? c->d_bcursor.p : c->d_bcount.p;
        if ((e = launch_zero(job, c->d_counters.p, c->d_counts.p, bzero, c->d_gbm.p, c->d_garrive.p, c->d_tally.p,
                             s)) != hipSuccess)
            return e;
    }
    if (phase == kPhaseBucketCount) {
        if ((e = launch_bucket(b, 0, bcus, s)) != hipSuccess)
            return e;
        BucketScanArgs sc;
        sc.job = job;
        sc.bcount = c->d_bcount.p;
        sc.boff = c->d_boff.p;
        sc.bcursor = c->d_bcursor.p;
        if ((e = launch_bucket_scan(sc, s)) != hipSuccess)
            return e;
        if (timed && (e = hipEventRecord(c->ev[4], s)) != hipSuccess)
            return e;
        return hipSuccess;
    }
    if (phase == kPhaseRest || phase == kPhaseDirect) {
        if (timed && (e = hipEventRecord(c->ev[5], s)) != hipSuccess)
            return e;
        if ((e = launch_bucket(b, phase == kPhaseRest ? 1 : 2, bcus, s)) != hipSuccess)
            return e;
    }
    SieveArgs a;
    memset(&a, 0, sizeof a);
    a.job = job;
    a.ranges = ranges;
    a.visit = (const VisitEntry *)(c->d_blob.p + L.visit);
    a.gbm = c->d_gbm.p;
    a.garrive = c->d_garrive.p;
    a.counters = c->d_counters.p;
    a.counts = c->d_counts.p;
    a.prm = c->d_prm.p;
    a.prd = c->d_prd.p;
    a.pidx = c->d_pidx.p;
    a.pidx_len = (uint32_t)(c->limit / 64 + 2);
    a.nprimes = (uint32_t)c->h_primes.size();
    a.first_mark = c->first_mark;
    a.k_split = c->k_split;
    a.k_dense = c->k_dense;
    a.items = c->d_items.p;
    a.item_prefix = c->d_item_prefix.p;
    a.ps_tab = c->d_pstab.p;
    for (int g = 0; g < kMaxGroups; ++g)
        a.groups[g] = c->groups[g];
    a.ngroups = c->ngroups;
    a.restore1 = c->restore1;
    a.restore5 = c->restore5;
    a.pw = pw;
    a.skip5 = skip5_mode(c);
    a.bitmap = c->d_bitmap.p;
    a.chunk_counts = c->d_chunk_counts.p;
    a.bdata = c->d_bdata.p;
    a.boff = c->d_boff.p;
    a.bcount = c->d_bcount.p;
    a.bcursor = c->d_bcursor.p;
    a.tally = c->d_tally.p;
    if (timed && (e = hipEventRecord(c->ev[0], s)) != hipSuccess)
        return e;
    e = launch_sieve(a, c->prm.block_threads, c->prm.wg_per_cu, (uint32_t)c->cus * c->prm.wg_per_cu,
                     c->sieve_u24 != 0, s);
    if (e != hipSuccess)
        return e;
    if (timed && (e = hipEventRecord(c->ev[1], s)) != hipSuccess)
        return e;
    SegArgs g;
    g.job = job;
    g.ranges = ranges;
    g.chunk_counts = c->d_chunk_counts.p;
    g.seg_sum = c->d_seg_sum.p;
    g.seg_base = c->d_seg_base.p;
    g.chunk_off = c->d_chunk_off.p;
    g.chunk_vbase = c->d_chunk_vbase.p;
    if (lists && (e = launch_seg(g, 0, (uint32_t)c->cus * 2, s)) != hipSuccess)
        return e;
    FinalizeArgs f;
    f.job = job;
    f.ranges = ranges;
    f.counts = c->d_counts.p;
    f.status = c->d_status.p;
    f.seg_sum = c->d_seg_sum.p;
    f.seg_base = c->d_seg_base.p;
    if ((e = launch_finalize(f, kFinalizeGrid, s)) != hipSuccess)
        return e;
    if (lists && (e = launch_seg(g, 1, (uint32_t)c->cus * 2, s)) != hipSuccess)
        return e;
    CompactArgs k;
    k.job = job;
    k.chunk_vbase = c->d_chunk_vbase.p;
    k.bitmap = c->d_bitmap.p;
    k.chunk_off = c->d_chunk_off.p;
    k.wbase_lo = k.wbase_hi = 0;
    if (lists && (e = launch_compact(k, (uint32_t)c->cus * 4, s)) != hipSuccess)
        return e;
    if (timed && (e = hipEventRecord(c->ev[2], s)) != hipSuccess)
        return e;
    return hipSuccess;
}

hipError_t capture_graph(sieve_ctx *c, int phase)
{
    if (c->graph[phase]) {
        (void)hipGraphExecDestroy(c->graph[phase]);
        c->graph[phase] = nullptr;
    }
    if (c->graph_src[phase]) {
        (void)hipGraphDestroy(c->graph_src[phase]);
        c->graph_src[phase] = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return e;
    hipError_t e2 = enqueue_phase(c, c->stream, phase, false, true);
    e = hipStreamEndCapture(c->stream, &c->graph_src[phase]);
    if (e2 != hipSuccess)
        return e2;
    if (e != hipSuccess)
        return e;
    e = hipGraphInstantiate(&c->graph[phase], c->graph_src[phase], nullptr, nullptr, 0);
    if (e != hipSuccess)
        return e;
    c->graph_gen[phase] = c->gen;
    return hipSuccess;
}

// Runs one phase on stream s, directly or by replaying its graph.
hipError_t run_phase(sieve_ctx *c, hipStream_t s, int phase, bool use_graph)
{
    if (!use_graph)
        return enqueue_phase(c, s, phase, c->timing != 0, ((const JobHeader *)c->h_blob)->nlist != 0);
    hipError_t e;
    if (!c->graph[phase] || c->graph_gen[phase] != c->gen) {
        // Capture on the context stream once the work before it is done.
        if (s != c->stream && (e = hipStreamSynchronize(s)) != hipSuccess)
            return e;
        if ((e = capture_graph(c, phase)) != hipSuccess)
            return e;
    }
    return hipGraphLaunch(c->graph[phase], s);
}

// Results of a stream-ordered job: a host function on the stream copies
// them from the job's pinned slot into the caller's arrays.
struct AsyncResult {
    sieve_ctx *c;
    const unsigned long long *counts_src;
    const int32_t *status_src;
    const unsigned long long *flag;
    uint64_t *counts;
    int32_t *status;
    uint64_t n;
};

void deliver_results(void *arg)
{
    AsyncResult *r = (AsyncResult *)arg;
    for (uint64_t i = 0; i < r->n; ++i) {
        if (r->counts)
            r->counts[i] = r->counts_src[i];
        if (r->status)
            r->status[i] = r->status_src[i];
    }
    if (r->flag[0])
        r->c->last_error = SIEVE_E_DEVICE;  // a kernel refused to run (see its error flag)
    delete r;
}

// Runs one job: plan, upload, kernels (graph or direct), results.
// counts/status (host, n entries) receive per-range results.  With async_ok
// a job that needs no host decision mid-way (no bucket sieve, no timing)
// returns once enqueued; its results are written when the stream gets there.
// links (host, n entries, or NULL): the ranges' bucket walk links.
int run_job_once(sieve_ctx *c, uint64_t n, const uint64_t *lo, const uint64_t *hi, const uint8_t *mode,
                 const uint64_t *off, const uint64_t *cap, int elem_bytes, void *out, uint64_t *counts,
                 int32_t *status, hipStream_t stream, bool use_graph, Plan &pl, bool async_ok,
                 const WalkLink *links = nullptr)
{
    int st;
    const uint64_t nlist = pl.nlist;
    st = ensure_capacity(c, n, pl.nchunks, pl.ntiles, pl.gtiles);
    if (st != SIEVE_OK)
        return st;
    hipStream_t s = stream ? stream : c->stream;
    // This job's host slot: the job before last used it; wait until that
    // job's copies out of it are done.
    c->cur_slot ^= 1;
    {
        sieve_ctx::HostSlot &sl = c->slot[c->cur_slot];
        if (sl.used && hipEventSynchronize(sl.done) != hipSuccess) {
            (void)hipGetLastError();
            return SIEVE_E_DEVICE;
        }
        c->h_blob = sl.blob;
        c->h_counts = sl.counts;
        c->h_status = sl.status;
        c->h_flag = sl.flag;
    }
    // The scratch is shared: a job on another stream than the last one
    // waits for it on the device.
    if (c->last_valid && c->last_stream != s && hipStreamWaitEvent(s, c->last_ev, 0) != hipSuccess) {
        (void)hipGetLastError();
        return SIEVE_E_DEVICE;
    }
    const BlobLayout L = blob_layout(c->cap_ranges);
    JobHeader *h = (JobHeader *)c->h_blob;
    memset(h, 0, sizeof *h);
    h->ntiles = pl.ntiles;
    h->nchunks = pl.nchunks;
    h->nunits = pl.nunits;
    h->nseg = pl.nseg;
    h->nvisit = pl.nvisit;
    h->gtiles = pl.gtiles;
    h->gwords = pl.gtiles * 2 * (c->prm.segment_bytes / 8);
    h->bmode = 1;
    h->nranges = (uint32_t)n;
    h->nlist = (uint32_t)nlist;
    h->out = out;
    h->elem_bytes = elem_bytes;
    h->links = links && n ? 1u : 0u;
    if (h->links)
        memcpy(c->h_blob + L.links, links, n * sizeof(WalkLink));
    if (n) {
        memcpy(c->h_blob + L.ranges, pl.ranges.data(), n * sizeof(RangeDesc));
        // Visit order: most Table 1 starts per work unit first (a tile of
        // an unsplit range starts min(nact, kbig) primes, a part of a split
        // tile about part_primes), ties in storage order.
        std::vector<uint32_t> ord(n);
        std::vector<uint32_t> key(n);
        for (uint64_t i = 0; i < n; ++i) {
            ord[i] = (uint32_t)i;
            const RangeDesc &d = pl.ranges[i];
            key[i] = d.nparts > 1 ? d.part_primes : std::min(d.nact, d.kbig);
        }
        std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) { return key[x] > key[y]; });
        if (c->prm.visit_order == SIEVE_VISIT_REVERSED) {
            std::reverse(ord.begin(), ord.end());
        } else if (c->prm.visit_order == SIEVE_VISIT_SHUFFLED) {
            // Fisher-Yates with a fixed 64-bit LCG (Knuth's MMIX constants)
            uint64_t x = 0x9E3779B97F4A7C15ull;
            for (uint64_t i = n; i > 1; --i) {
                x = x * 6364136223846793005ull + 1442695040888963407ull;
                std::swap(ord[i - 1], ord[(x >> 33) % i]);
            }
        }
        VisitEntry *v = (VisitEntry *)(c->h_blob + L.visit);
        uint64_t pos = 0;
        for (uint64_t j = 0; j < n; ++j) {
            v[j].vstart = pos;
            v[j].range = ord[j];
            v[j].pad = 0;
            pos += range_units(pl.ranges[ord[j]]);
        }
    }
    hipError_t e = hipMemcpyAsync(c->d_blob.p, c->h_blob, L.ranges + n * sizeof(RangeDesc),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n)
        e = hipMemcpyAsync(c->d_blob.p + L.visit, c->h_blob + L.visit, n * sizeof(VisitEntry),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && h->links)
        e = hipMemcpyAsync(c->d_blob.p + L.links, c->h_blob + L.links, n * sizeof(WalkLink),
                           hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return hip_status(e);
    const bool buckets = pl.nunits != 0;
    if (buckets)
        c->bucket_jobs++;
    {
        // 24-bit start arithmetic when every range's primes are below 2^24 - 8
        uint64_t top = 0;
        for (uint64_t i = 0; i < n; ++i)
            top = std::max(top, pl.ranges[i].hi);
        const uint32_t u24 = (top < 2 || isqrt_host(top - 1) < (1u << 24) - 8) ? 1u : 0u;
        if (u24 != c->sieve_u24) {
            c->sieve_u24 = u24;
            c->gen++;
        }
    }
    if (buckets) {
        // LDS bins for the largest window of the job, in power-of-two steps
        // so that captured graphs (which hold the size) are seldom re-made
        uint32_t w = 64;
        while (w < pl.bwin)
            w <<= 1;
        w = std::min(w, kBucketWindow);
        if (w != c->bucket_win) {
            c->bucket_win = w;
            c->gen++;
        }
    }
    // Results back to the host: per-range counts and status, and the flags.
    auto finish = [&]() -> hipError_t {
        hipError_t f = hipSuccess;
        if (n) {
            f = hipMemcpyAsync(c->h_counts, c->d_counts.p, n * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                               s);
            if (f == hipSuccess)
                f = hipMemcpyAsync(c->h_status, c->d_status.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        }
        if (f == hipSuccess)
            f = hipMemcpyAsync(c->h_flag, c->d_counters.p + kErrorFlag, 2 * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s);
#ifdef SIEVE_MARK_COUNT
        if (f == hipSuccess)
            f = hipMemcpyAsync(c->h_tally, c->d_tally.p, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
#endif
        if (f == hipSuccess)
            f = hipStreamSynchronize(s);
        return f;
    };
    // Marks the end of this job on s: the slot it used and the context's
    // latest work.
    auto fence = [&]() -> hipError_t {
        sieve_ctx::HostSlot &sl = c->slot[c->cur_slot];
        hipError_t f = hipEventRecord(sl.done, s);
        if (f == hipSuccess)
            f = hipEventRecord(c->last_ev, s);
        if (f == hipSuccess) {
            sl.used = true;
            c->last_stream = s;
            c->last_valid = true;
        }
        return f;
    };
    if (!buckets && async_ok && !c->timing) {
        // Stream-ordered: results copied to the slot, then handed to the
        // caller by a host function on the stream.
        e = run_phase(c, s, kPhaseWhole, use_graph);
        if (e == hipSuccess && n)
            e = hipMemcpyAsync(c->h_counts, c->d_counts.p, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && n)
            e = hipMemcpyAsync(c->h_status, c->d_status.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->h_flag, c->d_counters.p + kErrorFlag, 2 * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s);
        AsyncResult *r = nullptr;
        if (e == hipSuccess) {
            r = new (std::nothrow) AsyncResult{c, c->h_counts, c->h_status, c->h_flag, counts, status, n};
            if (!r)
                e = hipErrorOutOfMemory;
        }
        if (e == hipSuccess) {
            e = hipLaunchHostFunc(s, deliver_results, r);
            if (e != hipSuccess)
                delete r;
        }
        if (e == hipSuccess)
            e = fence();
        return e == hipSuccess ? SIEVE_OK : hip_status(e);
    }
    if (!buckets) {
        e = run_phase(c, s, kPhaseWhole, use_graph);
        if (e == hipSuccess)
            e = finish();
    } else {
        // Estimated layout first: one pass, no host round trip.
        if (c->prm.bucket_slices == SIEVE_BUCKET_EXACT)
            pl.best = 0;
        if (pl.best > c->cap_bdata) {
            c->cap_bdata = grow(c->cap_bdata, pl.best, 1024);
            c->d_bdata.release();
            if (!c->d_bdata.reserve(c->cap_bdata))
                return SIEVE_E_NOMEM;
            c->gen++;
        }
        const bool exact = c->prm.bucket_slices == SIEVE_BUCKET_EXACT;
        if (!exact) {
            e = run_phase(c, s, kPhaseDirect, use_graph);
            if (e == hipSuccess)
                e = finish();
        }
        if (e == hipSuccess && (exact || c->h_flag[1])) {
            // A slice overflowed: run the job again with the exact layout.
            c->bucket_fallbacks++;
            h->bmode = 2;
            e = hipMemcpyAsync(c->d_blob.p, c->h_blob, sizeof(JobHeader), hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = run_phase(c, s, kPhaseBucketCount, use_graph);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->h_btotal, c->d_boff.p + pl.ntiles, sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipStreamSynchronize(s);
            if (e == hipSuccess && *c->h_btotal > c->cap_bdata) {
                c->cap_bdata = grow(c->cap_bdata, *c->h_btotal, 1024);
                c->d_bdata.release();
                if (!c->d_bdata.reserve(c->cap_bdata))
                    return SIEVE_E_NOMEM;
                c->gen++;
            }
            if (e == hipSuccess)
                e = run_phase(c, s, kPhaseRest, use_graph);
            if (e == hipSuccess)
                e = finish();
        }
    }
    if (e == hipSuccess)
        e = fence();
    if (e != hipSuccess)
        return hip_status(e);
    if (c->h_flag[0])
        return SIEVE_E_DEVICE;  // a kernel refused to run (see its error flag)
#ifdef SIEVE_MARK_COUNT
    for (int q = 0; q < 4; ++q)
        c->tally_total[q] += c->h_tally[q];
#endif
    if (c->timing && !use_graph) {
        float ta = 0, tb = 0, bc = 0, bf = 0;
        if (hipEventElapsedTime(&ta, c->ev[0], c->ev[1]) == hipSuccess &&
            hipEventElapsedTime(&tb, c->ev[1], c->ev[2]) == hipSuccess) {
            c->t_sieve_ms += ta;
            c->t_post_ms += tb;
            c->t_jobs++;
        }
        if (buckets && hipEventElapsedTime(&bf, c->ev[5], c->ev[0]) == hipSuccess)
            c->t_bucket_ms += bf;
        if (buckets && h->bmode == 2 && hipEventElapsedTime(&bc, c->ev[3], c->ev[4]) == hipSuccess)
            c->t_bucket_ms += bc;
    }
    for (uint64_t i = 0; i < n; ++i) {
        if (counts)
            counts[i] = c->h_counts[i];
        if (status)
            status[i] = c->h_status[i];
    }
    return SIEVE_OK;
}

// Runs a job within the bucket-memory budget.  When the estimated bucket
// entries of the whole job exceed it, the ranges are cut at tile boundaries
// of their own plan into pieces (each piece tiles exactly like that part of
// the range) and the pieces run as a sequence of jobs, at most one piece of
// a range per job.  Counts add up; a list range's pieces write consecutively
// (offset and capacity advance by the primes already written), and once a
// piece does not fit, the rest of that range is only counted and the range
// reports SIEVE_E_CAPACITY with its full count.
//
// ws (host, n entries, or NULL) links ranges to earlier pieces of the same
// long ranges (serving): a range that takes the bucket sieve resumes the
// walks ws[i].src holds and stores its own end state in ws[i].dst; the
// outputs ws[i].saved and ws[i].resumed say what it did.
int run_job(sieve_ctx *c, uint64_t n, const uint64_t *lo, const uint64_t *hi, const uint8_t *mode,
            const uint64_t *off, const uint64_t *cap, int elem_bytes, void *out, uint64_t *counts,
            int32_t *status, hipStream_t stream, bool use_graph, bool async_ok = false, WalkSpec *ws = nullptr)
{
    Plan pl;
    int st = make_plan(c, n, lo, hi, mode, off, cap, elem_bytes, pl);
    if (st != SIEVE_OK)
        return st;
    for (uint64_t i = 0; ws && i < n; ++i)
        ws[i].saved = ws[i].resumed = 0;
    const uint64_t budget = c->bucket_budget;
    if (pl.best <= budget) {
        std::vector<WalkLink> links;
        if (ws) {
            links.assign(n, WalkLink{nullptr, nullptr, 0, 0});
            for (uint64_t i = 0; i < n; ++i) {
                const RangeDesc &d = pl.ranges[i];
                if (d.kbig >= d.nact || d.ntiles >= 0x80000000u)
                    continue;  // no bucket primes (or tiles past the states' reach)
                const uint32_t nb = d.nact - d.kbig;
                if (ws[i].src && ws[i].nsrc) {
                    links[i].src = ws[i].src;
                    links[i].nsrc = std::min(ws[i].nsrc, nb);
                    ws[i].resumed = 1;
                }
                if (ws[i].dst && nb <= ws[i].dcap) {
                    links[i].dst = ws[i].dst;
                    ws[i].saved = nb;
                }
            }
        }
        return run_job_once(c, n, lo, hi, mode, off, cap, elem_bytes, out, counts, status, stream, use_graph, pl,
                            async_ok, ws ? links.data() : nullptr);
    }
    const uint64_t span = (uint64_t)kValsPerWord * (c->prm.segment_bytes / 8);
    std::vector<RangeDesc> d0 = pl.ranges;  // the whole ranges' plans
    std::vector<uint64_t> cur(lo, lo + n), acc(n, 0), tot(n, 0), per(n);
    std::vector<int32_t> rst(n, SIEVE_OK);
    for (uint64_t i = 0; i < n; ++i)
        per[i] = d0[i].bunits ? std::max<uint64_t>(1, budget / std::max<uint32_t>(d0[i].bcap, 1)) : UINT64_MAX;
    std::vector<uint64_t> glo, ghi, goff, gcap, gcnt, gidx;
    std::vector<uint8_t> gmode;
    std::vector<int32_t> gst;
    uint64_t next = 0;  // first range that may still have work
    for (;;) {
        while (next < n && cur[next] >= hi[next])
            ++next;
        if (next == n)
            break;
        glo.clear(), ghi.clear(), goff.clear(), gcap.clear(), gidx.clear(), gmode.clear();
        uint64_t used = 0;
        for (uint64_t i = next; i < n; ++i) {
            if (cur[i] >= hi[i])
                continue;
            const RangeDesc &d = d0[i];
            uint64_t e = hi[i];
            uint64_t tiles = d.ntiles;
            if (per[i] != UINT64_MAX) {
                // tile k of the range covers [base + k span, base + (k + 1) span)
                const uint64_t k0 = cur[i] <= d.base ? 0 : (cur[i] - d.base) / span;
                tiles = std::min<uint64_t>(per[i], d.ntiles - k0);
                if (k0 + tiles < d.ntiles)
                    e = d.base + (k0 + tiles) * span;
            }
            const uint64_t need = d.bunits ? (uint64_t)d.bcap * tiles : 0;
            if (!glo.empty() && used + need > budget)
                break;
            used += need;
            const bool lst = mode && mode[i] && rst[i] == SIEVE_OK;
            glo.push_back(cur[i]);
            ghi.push_back(e);
            gmode.push_back(lst ? 1 : 0);
            goff.push_back(lst ? off[i] + acc[i] : 0);
            gcap.push_back(lst ? cap[i] - acc[i] : 0);
            gidx.push_back(i);
        }
        const uint64_t m = glo.size();
        gcnt.assign(m, 0);
        gst.assign(m, SIEVE_OK);
        Plan gp;
        st = make_plan(c, m, glo.data(), ghi.data(), gmode.data(), goff.data(), gcap.data(), elem_bytes, gp);
        if (st == SIEVE_OK)
            st = run_job_once(c, m, glo.data(), ghi.data(), gmode.data(), goff.data(), gcap.data(), elem_bytes,
                              out, gcnt.data(), gst.data(), stream, use_graph, gp, false);
        if (st != SIEVE_OK)
            return st;
        for (uint64_t g = 0; g < m; ++g) {
            const uint64_t i = gidx[g];
            tot[i] += gcnt[g];
            if (gmode[g]) {
                if (gst[g] == SIEVE_OK)
                    acc[i] += gcnt[g];
                else
                    rst[i] = gst[g];
            }
            cur[i] = ghi[g];
        }
    }
    for (uint64_t i = 0; i < n; ++i) {
        if (counts)
            counts[i] = tot[i];
        if (status)
            status[i] = rst[i];
    }
    return SIEVE_OK;
}

// Base primes: host sieve up to isqrt(limit) (at least 2^16), then the
// device list path produces the rest straight into the resident set.
int grow_base_primes(sieve_ctx *c, uint64_t limit)
{
    const uint64_t h = std::min<uint64_t>(limit, std::max<uint64_t>(isqrt_host(limit), 1u << 16));
    if (c->limit < h) {
        c->h_primes = host_small_primes(h);
        int st = install_primes(c, h);
        if (st != SIEVE_OK)
            return st;
    }
    if (limit <= c->limit)
        return SIEVE_OK;
    const uint64_t lo = c->limit + 1, hi = limit + 1;
    const uint64_t bound = sieve_list_bound(lo, hi);
    uint32_t *d_out = nullptr;
    if (hipMalloc((void **)&d_out, std::max<uint64_t>(bound, 1) * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return SIEVE_E_NOMEM;
    }
    const uint8_t mode = 1;
    const uint64_t off = 0;
    uint64_t cnt = 0;
    int32_t rs = 0;
    int st = run_job(c, 1, &lo, &hi, &mode, &off, &bound, 4, d_out, &cnt, &rs, nullptr, false);
    if (st == SIEVE_OK && rs != SIEVE_OK)
        st = rs;
    if (st == SIEVE_OK) {
        const size_t old = c->h_primes.size();
        c->h_primes.resize(old + cnt);
        hipError_t e = hipMemcpy(c->h_primes.data() + old, d_out, cnt * sizeof(uint32_t), hipMemcpyDeviceToHost);
        st = hip_status(e);
        if (st == SIEVE_OK)
            st = install_primes(c, limit);
    }
    (void)hipFree(d_out);
    return st;
}

void destroy_ctx(sieve_ctx *c)
{
    if (!c)
        return;
    for (int g = 0; g < 4; ++g) {
        if (c->graph[g])
            (void)hipGraphExecDestroy(c->graph[g]);
        if (c->graph_src[g])
            (void)hipGraphDestroy(c->graph_src[g]);
    }
    c->d_bcount.release();
    c->d_bcursor.release();
    c->d_bdata.release();
    c->d_boff.release();
    if (c->h_btotal)
        (void)hipHostFree(c->h_btotal);
    c->d_prm.release();
    c->d_prd.release();
    c->d_pidx.release();
    c->d_items.release();
    c->d_item_prefix.release();
    c->d_pstab.release();
    c->d_ext.release();
    c->d_wr.release();
    c->d_blob.release();
    c->d_counters.release();
    c->d_counts.release();
    c->d_status.release();
    c->d_bitmap.release();
    c->d_chunk_counts.release();
    c->d_chunk_vbase.release();
    c->d_chunk_off.release();
    c->d_seg_sum.release();
    c->d_seg_base.release();
    for (auto &sl : c->slot) {
        if (sl.blob)
            (void)hipHostFree(sl.blob);
        if (sl.counts)
            (void)hipHostFree(sl.counts);
        if (sl.status)
            (void)hipHostFree(sl.status);
        if (sl.flag)
            (void)hipHostFree(sl.flag);
        if (sl.done)
            (void)hipEventDestroy(sl.done);
    }
    if (c->last_ev)
        (void)hipEventDestroy(c->last_ev);
    c->d_tally.release();
    if (c->h_tally)
        (void)hipHostFree(c->h_tally);
    for (auto &ev : c->ev)
        if (ev)
            (void)hipEventDestroy(ev);
    for (int i = 0; i < 2; ++i) {
        c->d_piece[i].release();
        if (c->h_piece[i])
            (void)hipHostFree(c->h_piece[i]);
        if (c->piece_ev[i])
            (void)hipEventDestroy(c->piece_ev[i]);
    }
    if (c->copy_stream)
        (void)hipStreamDestroy(c->copy_stream);
    if (c->stream)
        (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // namespace

namespace sieve {
namespace rt {
int set_err(sieve_ctx *c, int e) { return ::set_err(c, e); }
int hip_status(hipError_t e) { return ::hip_status(e); }
uint64_t isqrt_host(uint64_t n) { return ::isqrt_host(n); }
void plan_range(uint64_t lo, uint64_t hi, uint32_t pw, uint64_t &ntiles, uint64_t &base, uint32_t &last_words)
{
    ::plan_range(lo, hi, pw, ntiles, base, last_words);
}
int run_job(sieve_ctx *c, uint64_t n, const uint64_t *lo, const uint64_t *hi, const uint8_t *mode,
            const uint64_t *off, const uint64_t *cap, int elem_bytes, void *out, uint64_t *counts, int32_t *status,
            hipStream_t stream, bool use_graph, bool async_ok, WalkSpec *ws)
{
    return ::run_job(c, n, lo, hi, mode, off, cap, elem_bytes, out, counts, status, stream, use_graph, async_ok, ws);
}
int grow_base_primes(sieve_ctx *c, uint64_t limit) { return ::grow_base_primes(c, limit); }
int ensure_capacity(sieve_ctx *c, uint64_t nranges, uint64_t nchunks, uint64_t ntiles, uint64_t gtiles)
{
    return ::ensure_capacity(c, nranges, nchunks, ntiles, gtiles);
}
size_t blob_ranges_offset() { return blob_layout(1).ranges; }
uint32_t primes_upto(const sieve_ctx *c, uint64_t x) { return ::primes_upto(c, x); }
}  // namespace rt
}  // namespace sieve

extern "C" {

const char *sieve_strerror(int s)
{
    switch (s) {
    case SIEVE_OK:
        return "ok";
    case SIEVE_E_INVAL:
        return "invalid argument";
    case SIEVE_E_RANGE:
        return "base primes do not cover isqrt(hi - 1)";
    case SIEVE_E_CAPACITY:
        return "output capacity too small";
    case SIEVE_E_DTYPE:
        return "element size not 4/8, or uint32 output for values >= 2^32";
    case SIEVE_E_NOMEM:
        return "out of memory";
    case SIEVE_E_DEVICE:
        return "HIP device error";
    case SIEVE_E_BUSY:
        return "busy";
    case SIEVE_E_CANCELLED:
        return "cancelled";
    case SIEVE_E_IO:
        return "file I/O error";
    case SIEVE_E_LIMIT:
        return "request exceeds the fixed scratch of the allocation-free call";
    default:
        return "unknown status";
    }
}

int sieve_last_error(const sieve_ctx *ctx) { return ctx ? ctx->last_error : SIEVE_E_INVAL; }

int sieve_default_params(sieve_params *p)
{
    if (!p)
        return SIEVE_E_INVAL;
    memset(p, 0, sizeof *p);
    fill_defaults(*p);
    return SIEVE_OK;
}

int sieve_create(sieve_ctx **out, int device, const sieve_params *p)
{
    if (!out)
        return SIEVE_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return SIEVE_E_DEVICE;
    }
    if (device < 0 || device >= ndev)
        return SIEVE_E_INVAL;
    hipDeviceProp_t prop;
    if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess) {
        (void)hipGetLastError();
        return SIEVE_E_DEVICE;
    }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return SIEVE_E_DEVICE;  // the kernels are built for gfx950 only
    sieve_ctx *c = new (std::nothrow) sieve_ctx();
    if (!c)
        return SIEVE_E_NOMEM;
    c->device = device;
    c->cus = prop.multiProcessorCount;
    // CDNA4 gives a workgroup up to 160 KiB of LDS; the sieve kernel's own
    // static LDS (tile bookkeeping, under 1 KiB) comes out of the same budget.
    c->lds_max = 156 * 1024;
    sieve_params q;
    memset(&q, 0, sizeof q);
    if (p)
        q = *p;
    fill_defaults(q);
    int st = validate_params(q, c->lds_max);
    if (st != SIEVE_OK) {
        destroy_ctx(c);
        return st;
    }
    c->prm = q;
    c->bucket_budget = (uint64_t)q.bucket_mem_mb * (1u << 20) / sizeof(uint32_t);
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        set_sieve_lds_limit(q.segment_bytes) != hipSuccess) {
        (void)hipGetLastError();
        destroy_ctx(c);
        return SIEVE_E_DEVICE;
    }
    for (auto &ev : c->ev)
        if (hipEventCreate(&ev) != hipSuccess) {
            (void)hipGetLastError();
            destroy_ctx(c);
            return SIEVE_E_DEVICE;
        }
    if (hipEventCreateWithFlags(&c->slot[0].done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->slot[1].done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->last_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        destroy_ctx(c);
        return SIEVE_E_DEVICE;
    }
    {
        // This device's copy of the fixed scratch array (the device is
        // current here); host code uses only this address for it.
        void *sp = nullptr;
        if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
            (void)hipGetLastError();
            destroy_ctx(c);
            return SIEVE_E_DEVICE;
        }
        c->static_scratch = (unsigned char *)sp;
    }
    st = build_presieve(c, q.presieve_groups == SIEVE_PRESIEVE_NONE ? 0 : q.presieve_groups);
    if (st == SIEVE_OK)
        st = install_primes(c, 0);
    if (st == SIEVE_OK)
        st = ensure_capacity(c, 1, 1, 1, 1);
    if (st != SIEVE_OK) {
        destroy_ctx(c);
        return st;
    }
    *out = c;
    return SIEVE_OK;
}

int sieve_destroy(sieve_ctx *ctx)
{
    if (ctx) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
    }
    destroy_ctx(ctx);
    return SIEVE_OK;
}

int sieve_get_params(const sieve_ctx *ctx, sieve_params *p)
{
    if (!ctx || !p)
        return SIEVE_E_INVAL;
    *p = ctx->prm;
    return SIEVE_OK;
}

int sieve_base_primes(sieve_ctx *ctx, uint64_t limit, uint64_t *n_out)
{
    if (!ctx)
        return SIEVE_E_INVAL;
    if (limit >= (1ull << 32))
        return set_err(ctx, SIEVE_E_INVAL);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return set_err(ctx, hip_status(hipErrorInvalidDevice));
    int st = SIEVE_OK;
    if (limit > ctx->limit)
        st = grow_base_primes(ctx, limit);
    if (st == SIEVE_OK && n_out)
        *n_out = ctx->h_primes.size();
    return set_err(ctx, st);
}

int sieve_base_limit(const sieve_ctx *ctx, uint64_t *limit)
{
    if (!ctx || !limit)
        return SIEVE_E_INVAL;
    *limit = ctx->limit;
    return SIEVE_OK;
}

int sieve_count(sieve_ctx *ctx, uint64_t lo, uint64_t hi, uint64_t *count)
{
    if (!ctx || !count)
        return set_err(ctx, SIEVE_E_INVAL);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return set_err(ctx, SIEVE_E_DEVICE);
    int32_t rs = 0;
    int st = run_job(ctx, 1, &lo, &hi, nullptr, nullptr, nullptr, 8, nullptr, count, &rs, nullptr, false);
    return set_err(ctx, st);
}

int sieve_list(sieve_ctx *ctx, uint64_t lo, uint64_t hi, void *out_dev, uint64_t cap, int elem_bytes,
               uint64_t *n_out, void *stream)
{
    if (!ctx || !n_out)
        return set_err(ctx, SIEVE_E_INVAL);
    if (elem_bytes != 4 && elem_bytes != 8)
        return set_err(ctx, SIEVE_E_DTYPE);
    if (!out_dev && cap)
        return set_err(ctx, SIEVE_E_INVAL);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return set_err(ctx, SIEVE_E_DEVICE);
    const uint8_t mode = 1;
    const uint64_t off = 0;
    int32_t rs = 0;
    // A NULL output with cap 0 only asks for the count.
    void *out = out_dev ? out_dev : (void *)ctx->d_chunk_off.p;
    if (stream) {
        // Stream-ordered: *n_out is written when the stream reaches the end
        // of the job (a capacity shortfall then shows as *n_out > cap).
        return set_err(ctx, run_job(ctx, 1, &lo, &hi, &mode, &off, &cap, elem_bytes, out, n_out, nullptr,
                                    (hipStream_t)stream, false, true));
    }
    int st = run_job(ctx, 1, &lo, &hi, &mode, &off, &cap, elem_bytes, out, n_out, &rs, nullptr, false);
    if (st == SIEVE_OK && rs != SIEVE_OK)
        st = rs;
    return set_err(ctx, st);
}

int sieve_count_batch(sieve_ctx *ctx, const uint64_t *lo, const uint64_t *hi, uint64_t n, uint64_t *counts,
                      void *stream)
{
    if (!ctx || (n && (!lo || !hi || !counts)) || n > 0xFFFFFFFFull)
        return set_err(ctx, SIEVE_E_INVAL);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return set_err(ctx, SIEVE_E_DEVICE);
    if (n == 0)
        return set_err(ctx, SIEVE_OK);
    int st = run_job(ctx, n, lo, hi, nullptr, nullptr, nullptr, 8, nullptr, counts, nullptr,
                     (hipStream_t)stream, ctx->prm.use_graph != 0, stream != nullptr);
    return set_err(ctx, st);
}

int sieve_list_batch(sieve_ctx *ctx, const uint64_t *lo, const uint64_t *hi, const uint8_t *mode, uint64_t n,
                     void *out_dev, const uint64_t *off, const uint64_t *cap, int elem_bytes, uint64_t *counts,
                     int32_t *status, void *stream)
{
    if (!ctx || (n && (!lo || !hi || !mode || !counts || !status)) || n > 0xFFFFFFFFull)
        return set_err(ctx, SIEVE_E_INVAL);
    if (elem_bytes != 4 && elem_bytes != 8)
        return set_err(ctx, SIEVE_E_DTYPE);
    bool any = false;
    for (uint64_t i = 0; i < n; ++i)
        any |= mode[i] != 0;
    if (any && (!out_dev || !off || !cap))
        return set_err(ctx, SIEVE_E_INVAL);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return set_err(ctx, SIEVE_E_DEVICE);
    if (n == 0)
        return set_err(ctx, SIEVE_OK);
    int st = run_job(ctx, n, lo, hi, mode, off, cap, elem_bytes, out_dev, counts, status, (hipStream_t)stream,
                     ctx->prm.use_graph != 0, stream != nullptr);
    return set_err(ctx, st);
}

int sieve_count_batch_static(sieve_ctx *ctx, const uint64_t *lo, const uint64_t *hi, uint64_t n,
                             uint64_t *counts, void *stream)
{
    if (!ctx || (n && (!lo || !hi || !counts)))
        return set_err(ctx, SIEVE_E_INVAL);
    if (n > kStaticMaxRanges)
        return set_err(ctx, SIEVE_E_LIMIT);
    if (!ctx->static_scratch)
        return set_err(ctx, SIEVE_E_DEVICE);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return set_err(ctx, SIEVE_E_DEVICE);
    if (n == 0)
        return set_err(ctx, SIEVE_OK);
    std::lock_guard<std::mutex> lk(g_static_mu);
    const uint32_t pw = ctx->prm.segment_bytes / 8;
    JobHeader &h = g_static_job;
    memset(&h, 0, sizeof h);
    uint64_t top = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t a = lo[i], b = hi[i];
        if (a > b || b > SIEVE_MAX_HI)
            return set_err(ctx, SIEVE_E_INVAL);
        const uint64_t root = b > 4 ? isqrt_host(b - 1) : 0;
        if (root > ctx->limit)
            return set_err(ctx, SIEVE_E_RANGE);
        RangeDesc &d = g_static_ranges[i];
        memset(&d, 0, sizeof d);
        d.lo = a;
        d.hi = b;
        uint64_t nt;
        plan_range(a, b, pw, nt, d.base, d.last_words);
        if (nt > 0xFFFFFFFFull)
            return set_err(ctx, SIEVE_E_INVAL);
        d.ntiles = (uint32_t)nt;
        d.tile0 = h.ntiles;
        h.ntiles += nt;
        d.nact = b > 4 ? primes_upto(ctx, root) : 0u;
        d.kbig = d.nact;  // every prime in the per-tile loop: no bucket scratch
        d.nparts = 1;     // no split tiles: no global plane copies
        top = std::max(top, b);
    }
    const uint32_t S = strip_tiles(ctx, h.ntiles);
    for (uint64_t i = 0; i < n; ++i) {
        set_strips(g_static_ranges[i], S);
        h.nvisit += range_units(g_static_ranges[i]);
    }
    h.nranges = (uint32_t)n;
    h.elem_bytes = 8;
    // Visit order: most Table 1 starts per tile first (ties by index).
    for (uint64_t i = 0; i < n; ++i)
        g_static_order[i] = (uint32_t)i;
    std::sort(g_static_order, g_static_order + n, [](uint32_t x, uint32_t y) {
        const uint32_t kx = g_static_ranges[x].nact, ky = g_static_ranges[y].nact;
        return kx != ky ? kx > ky : x < y;
    });
    uint64_t pos = 0;
    for (uint64_t j = 0; j < n; ++j) {
        g_static_visit[j].vstart = pos;
        g_static_visit[j].range = g_static_order[j];
        g_static_visit[j].pad = 0;
        pos += range_units(g_static_ranges[g_static_order[j]]);
    }
    unsigned char *const sp = ctx->static_scratch;  // this device's array
    const JobHeader *job = (const JobHeader *)sp;
    const RangeDesc *ranges = (const RangeDesc *)(sp + StaticLayout::ranges);
    unsigned long long *counters = (unsigned long long *)(sp + StaticLayout::counters);
    unsigned long long *dcounts = (unsigned long long *)(sp + StaticLayout::counts);
    int32_t *dstatus = (int32_t *)(sp + StaticLayout::status);
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    hipError_t e = hipMemcpyAsync(sp, &h, sizeof h, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sp + StaticLayout::ranges, g_static_ranges, n * sizeof(RangeDesc),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sp + StaticLayout::visit, g_static_visit, n * sizeof(VisitEntry),
                           hipMemcpyHostToDevice, s);
    // counters and counts start at zero (a kernel clears them)
    if (e == hipSuccess)
        e = launch_zero(job, counters, dcounts, nullptr, nullptr, nullptr, nullptr, s);
    if (e == hipSuccess) {
        SieveArgs a;
        memset(&a, 0, sizeof a);
        a.job = job;
        a.ranges = ranges;
        a.visit = (const VisitEntry *)(sp + StaticLayout::visit);
        a.counters = counters;
        a.counts = dcounts;
        a.prm = ctx->d_prm.p;
        a.prd = ctx->d_prd.p;
        a.pidx = ctx->d_pidx.p;
        a.pidx_len = (uint32_t)(ctx->limit / 64 + 2);
        a.nprimes = (uint32_t)ctx->h_primes.size();
        a.first_mark = ctx->first_mark;
        a.k_split = ctx->k_split;
        a.k_dense = ctx->k_dense;
        a.items = ctx->d_items.p;
        a.item_prefix = ctx->d_item_prefix.p;
        a.ps_tab = ctx->d_pstab.p;
        for (int g = 0; g < kMaxGroups; ++g)
            a.groups[g] = ctx->groups[g];
        a.ngroups = ctx->ngroups;
        a.restore1 = ctx->restore1;
        a.restore5 = ctx->restore5;
        a.pw = pw;
        a.skip5 = skip5_mode(ctx);
        const bool u24 = top < 2 || isqrt_host(top - 1) < (1u << 24) - 8;
        e = launch_sieve(a, ctx->prm.block_threads, ctx->prm.wg_per_cu, (uint32_t)ctx->cus * ctx->prm.wg_per_cu,
                         u24, s);
    }
    if (e == hipSuccess) {
        FinalizeArgs f;
        memset(&f, 0, sizeof f);
        f.job = job;
        f.ranges = ranges;
        f.counts = dcounts;
        f.status = dstatus;
        e = launch_finalize(f, kFinalizeGrid, s);
    }
    unsigned long long flag = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts, dcounts, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&flag, counters + kErrorFlag, sizeof flag, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return set_err(ctx, hip_status(e));
    return set_err(ctx, flag ? SIEVE_E_DEVICE : SIEVE_OK);
}

uint64_t sieve_list_bound(uint64_t lo, uint64_t hi)
{
    if (hi <= lo)
        return 0;
    // Values coprime to 6 in [lo, hi), plus 2 and 3.
    auto cop = [](uint64_t x) -> uint64_t {  // #{1 <= m < x : gcd(m, 6) = 1}
        if (x == 0)
            return 0;
        const uint64_t n = x - 1, q = n / 6, s = n % 6;
        return 2 * q + (s >= 1) + (s >= 5);
    };
    uint64_t b = cop(hi) - cop(lo) + 2;
    const uint64_t y = hi - lo;
    if (y > 1) {
        // Brun-Titchmarsh (Montgomery-Vaughan): pi(x + y) - pi(x) < 2y / ln y.
        const double bt = 2.0 * (double)y / std::log((double)y);
        if (bt < 1.8e19) {
            const uint64_t b2 = (uint64_t)std::ceil(bt * (1.0 + 1e-9)) + 1;
            if (b2 < b)
                b = b2;
        }
    }
    return b;
}

int sieve_wheel_start(uint64_t p, uint64_t base, uint64_t M, int64_t *id1, int64_t *id5)
{
    if (!id1 || !id5 || p < 5 || (p % 6 != 1 && p % 6 != 5) || base % 6 || M < 1 || M < base ||
        M - base >= (1ull << 22) || p >= (1ull << 32))
        return SIEVE_E_INVAL;
    // The same remainder path as the kernels (invariant reciprocal).
    uint32_t a, b;
    const uint32_t rem = mod_invariant(M - 1, (uint32_t)p, UINT64_MAX / p, p < 0x80000000ull);
    wheel_start((uint32_t)p, (uint32_t)(p / 6), base, M, rem, a, b);
    *id1 = a;
    *id5 = b;
    return SIEVE_OK;
}

int sieve_plan_range(uint64_t lo, uint64_t hi, uint32_t segment_bytes, uint64_t *ntiles, uint64_t *base,
                     uint32_t *last_words)
{
    if (!ntiles || !base || !last_words || lo > hi || hi > SIEVE_MAX_HI || segment_bytes < 8192 ||
        segment_bytes % 4096)
        return SIEVE_E_INVAL;
    plan_range(lo, hi, segment_bytes / 8, *ntiles, *base, *last_words);
    return SIEVE_OK;
}

#ifdef SIEVE_MARK_COUNT
int sieve_debug_tally(sieve_ctx *ctx, uint64_t *out, int reset)
{
    if (!ctx || !out)
        return SIEVE_E_INVAL;
    for (int q = 0; q < 4; ++q) {
        out[q] = ctx->tally_total[q];
        if (reset)
            ctx->tally_total[q] = 0;
    }
    return SIEVE_OK;
}
#endif

int sieve_set_timing(sieve_ctx *ctx, int on)
{
    if (!ctx)
        return SIEVE_E_INVAL;
    ctx->timing = on;
    ctx->t_sieve_ms = ctx->t_post_ms = ctx->t_bucket_ms = 0;
    ctx->t_jobs = 0;
    return SIEVE_OK;
}

int sieve_get_timing(const sieve_ctx *ctx, double *sieve_ms, double *post_ms, double *bucket_ms, uint64_t *jobs)
{
    if (!ctx || !sieve_ms || !post_ms || !bucket_ms || !jobs)
        return SIEVE_E_INVAL;
    *sieve_ms = ctx->t_sieve_ms;
    *post_ms = ctx->t_post_ms;
    *bucket_ms = ctx->t_bucket_ms;
    *jobs = ctx->t_jobs;
    return SIEVE_OK;
}

}  // extern "C"
