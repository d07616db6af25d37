// Windows beyond the 64-bit domain (Sec. 6 names ranges past 2^64 as the
// step after this method).
//
// A window [lo, hi) with 2^40 <= lo and hi - lo <= 2^40 is sieved in offsets
// from its base W = lo - lo mod 6: bit i of plane A_r stands for W + 6i + r
// (Sec. 2.1 with the segment base W), so the tile plan, the bitmap and chunk
// layout, the chunk-offset scan and the compaction are the 64-bit path's,
// applied to offsets.  Three steps see absolute values:
//   * the residues (W - 1) mod P of the base primes (one 128-bit reduction
//     per prime per window), from which Table 1 (Sec. 3) gives each prime's
//     first multiples at or past W, or P*P when that lies past W (Sec. 2.4);
//   * the presieve phases (W / 6) mod period of the pattern groups;
//   * the output, W + offset as 128-bit values.
// lo >= 2^40 keeps every prime marked in LDS (at most 4 plane lengths,
// below 2^22) below W, so the first multiple at or past W is never the prime
// itself; those primes start there with no square test (from W instead of
// P * P they only mark composites twice).  It also keeps 1, 2, 3 and the
// presieved primes out of every window.
//
// Work split by prime size:
//   * 5..73: the presieve pattern tables, which initialise each tile's planes;
//   * up to 4 plane lengths: LDS marks tile by tile, each start from the
//     window residue plus the tile's offset (one 64-by-32-bit reduction);
//     the smallest of them split over several lanes as in the 64-bit path;
//   * the next resident primes, with at least two hits in the window (P
//     below a plane's bits over the whole window): the bucket sieve of the
//     64-bit path in its exact layout, its walks started from the window
//     residue, and each tile ORs its entries into LDS;
//   * the sparse rest, resident primes below 2^32 and the 64-bit extension
//     primes: one thread per prime walks its few multiples in the window
//     and sets them in the window's bitmap in HBM with 64-bit atomic ORs (a
//     bucket walk costs each prime two passes of setup, which pays off only
//     from about two hits on).
// Each tile then merges its planes with the bitmap words, keeps the values of
// [lo, hi) that no prime marked, writes them back as prime bits (lists) and
// counts them per chunk.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "sieve.h"
#include "runtime.h"
#include "sieve_internal.h"
#include "wheel.h"

namespace sieve {

hipError_t launch_finalize(const FinalizeArgs &a, uint32_t grid, hipStream_t s);
hipError_t launch_seg(const SegArgs &a, int pass, uint32_t grid, hipStream_t s);
hipError_t launch_compact_wide(const CompactArgs &a, uint32_t grid, hipStream_t s);
hipError_t launch_zero(const JobHeader *job, unsigned long long *counters, unsigned long long *counts,
                       uint32_t *bcount, uint32_t *gbm, uint32_t *garrive, unsigned long long *tally, hipStream_t s);
hipError_t launch_bucket(const BucketArgs &a, int pass, uint32_t cus, hipStream_t s);
hipError_t launch_bucket_scan(const BucketScanArgs &a, hipStream_t s);

namespace {

constexpr uint32_t kWave = 64;
constexpr uint32_t kWideThreads = 1024;      // tile kernel
constexpr uint32_t kLargeThreads = 256;      // large-prime kernel
constexpr uint32_t kMaxTileChunks = 64;      // bitmap chunks per tile (pw <= 32768)
constexpr uint64_t kExtSample = 4096;        // extension primes per host sample
constexpr uint64_t kMidPlanes = 4;           // LDS-marked primes: up to this many plane lengths

struct WideArgs {
    uint64_t wlo, whi;          // W, the window base (a multiple of 6)
    uint64_t wm1_lo, wm1_hi;    // W - 1
    uint64_t lo_rel, hi_rel;    // [lo - W, hi - W)
    uint64_t nwords;            // plane words of all tiles
    uint32_t pw, ntiles, last_words;
    uint32_t list;              // 1: write prime bits back for the compaction
    const PrimeConst *prm;      // resident primes >= 5, ascending
    const uint2 *items;         // split work items {prime index, (j << 16) | g}
    const uint32_t *item_prefix;
    uint32_t first_mark;        // first prime index after the presieved ones
    uint32_t k_split;           // primes [first_mark, k_split) are split into items
    uint32_t n_mid;             // primes [first_mark, n_mid) are marked in LDS
    uint32_t n_act;             // resident primes with P * P < hi
    uint32_t k_atomic;          // resident primes [k_atomic, n_act) walk the window with atomics
    const uint32_t *wr;         // (W - 1) mod P by prime index, for indices < n_mid
    const uint64_t *ext;        // extension primes with P * P < hi
    uint64_t n_ext;
    const uint32_t *bdata;      // bucket entries of the resident large primes (bit | plane << 31),
    const unsigned long long *boff;  // tile t's at [boff[t], boff[t + 1]); NULL: no buckets
    const uint2 *ps_tab;
    PsGroup groups[kMaxGroups];
    uint32_t wphase[kMaxGroups];  // (W / 6) mod period
    uint32_t wstep[kMaxGroups];   // (32 kWideThreads) mod period
    unsigned long long *bitmap;   // nchunks * kChunkWords words, zeroed first
    uint32_t *chunk_counts;
    unsigned long long *counts;   // counts[0]: primes of the window (count mode)
};

__device__ inline uint32_t wave_sum(uint32_t x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        x += __shfl_xor(x, d, kWave);
    return x;
}

// Spreads the 32 bits of x to the even bit positions of a 64-bit word
// (interleaving by binary magic numbers).
__device__ inline uint64_t spread_even(uint32_t x)
{
    uint64_t v = x;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

// (h 2^64 + l) mod P for 5 <= P < 2^32 with m = floor((2^64 - 1) / P):
// Horner over 32-bit limbs, each step reducing a value below 2^64.
__device__ inline uint64_t mod128_small(uint64_t h, uint64_t l, uint32_t P, uint64_t m)
{
    uint64_t r = mod_invariant(h, P, m, false);
    r = mod_invariant((r << 32) | (l >> 32), P, m, false);
    return mod_invariant((r << 32) | (l & 0xFFFFFFFFull), P, m, false);
}

// The same for 2^32 <= P < 2^36: Horner over 16-bit limbs (r 2^16 + limb
// stays below 2^52).
__device__ inline uint64_t mod128_wide(uint64_t h, uint64_t l, uint64_t P)
{
    uint64_t r = h % P;
#pragma unroll
    for (int s = 48; s >= 0; s -= 16)
        r = ((r << 16) | ((l >> s) & 0xFFFFull)) % P;
    return r;
}

// Table 1 in 64-bit arithmetic for one prime P < 2^36 and the window base W
// as the first value: rem = (W - 1) mod P, Q = W - 1 - rem is the greatest
// multiple of P below W, and dp = (Q - W) + 6(R + 1) = 6R + 5 - rem lies in
// [1, P + 4].  The results are the indices (>= 0, below P) of the first
// multiples of P at or past W in A_one and A_five.
__device__ inline void first_hits_wide(uint64_t P, uint64_t rem, uint64_t &id1, uint64_t &id5)
{
    const uint64_t R = P / 6;
    const bool p5 = P - 6 * R == 5;
    const uint64_t dp = 6 * R + 5 - rem;
    const uint64_t i0 = dp / 6;  // = idx0 + R + 1
    const uint32_t q = (uint32_t)(dp - 6 * i0);
    const uint64_t t1 = p5 ? kTable1_id1_p5 : kTable1_id1_p1;
    const uint64_t t5 = p5 ? kTable1_id5_p5 : kTable1_id5_p1;
    const uint32_t e1 = (uint32_t)(t1 >> (8u * q));
    const uint32_t e5 = (uint32_t)(t5 >> (8u * q));
    id1 = i0 + (e1 & 7u) * R + ((e1 >> 3) & 7u) - 1u;
    id5 = i0 + (e5 & 7u) * R + ((e5 >> 3) & 7u) - 1u;
}

// Zeroes the window's bitmap (nwords, even) and the job counters.
__global__ void k_wide_clear(unsigned long long *bitmap, uint64_t nwords, unsigned long long *counters,
                             unsigned long long *counts)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    if (g < kNumCounters)
        counters[g] = 0;
    if (g == 0)
        counts[0] = 0;
    ulonglong2 *b2 = (ulonglong2 *)bitmap;
    for (uint64_t i = g; i < nwords / 2; i += stride)
        b2[i] = make_ulonglong2(0, 0);
}

// (W - 1) mod P of the primes marked in LDS.
__global__ void k_wide_prep(WideArgs a, uint32_t *wr)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t k = a.first_mark + blockIdx.x * blockDim.x + threadIdx.x; k < a.n_mid; k += stride) {
        const PrimeConst pc = a.prm[k];
        wr[k] = (uint32_t)mod128_small(a.wm1_hi, a.wm1_lo, pc.p, prime_recip(pc));
    }
}

// Primes with a few hits in the whole window at most (resident ones from
// k_atomic on, then the extension list): every multiple in the window, ORed
// into the bitmap (bit 2i: A_one index i, bit 2i + 1: A_five index i, of
// word i / 32).  Marks past hi are dropped by the tile kernel's range mask.
__global__ void __launch_bounds__(kLargeThreads) k_wide_large(WideArgs a)
{
    const uint64_t nres = a.n_act > a.k_atomic ? a.n_act - a.k_atomic : 0;
    const uint64_t n = nres + a.n_ext;
    const uint64_t nbits = 32ull * a.nwords;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        uint64_t P, rem;
        if (j < nres) {
            const PrimeConst pc = a.prm[a.k_atomic + j];
            P = pc.p;
            rem = mod128_small(a.wm1_hi, a.wm1_lo, pc.p, prime_recip(pc));
        } else {
            P = a.ext[j - nres];
            rem = mod128_wide(a.wm1_hi, a.wm1_lo, P);
        }
        uint64_t i1, i5;
        const uint64_t p2h = __umul64hi(P, P), p2l = P * P;
        if (p2h > a.whi || (p2h == a.whi && p2l > a.wlo)) {
            // P * P (= 1 mod 6) lies past W, below hi: marking starts there in
            // A_one, and at P (P + 4) or P (P + 2) in A_five
            i1 = (p2l - a.wlo - 1) / 6;
            i5 = i1 + (P % 6 == 1 ? 2 * (P - 1) / 3 : (P - 2) / 3);
        } else {
            first_hits_wide(P, rem, i1, i5);
        }
        for (uint64_t i = i1; i < nbits; i += P)
            atomicOr(&a.bitmap[i >> 5], 1ull << (2 * (i & 31)));
        for (uint64_t i = i5; i < nbits; i += P)
            atomicOr(&a.bitmap[i >> 5], 2ull << (2 * (i & 31)));
    }
}

// Mask of the bits of bitmap word gw whose values (offsets from W) lie in
// [lo, hi): bit b stands for 192 gw + 3b + 1 + (b & 1).
__device__ inline uint64_t range_mask(uint64_t gw, uint64_t lo, uint64_t hi)
{
    const uint64_t v0 = 192 * gw;
    if (v0 + 1 >= lo && v0 + 191 < hi)
        return ~0ull;
    uint64_t m = 0;
    for (uint32_t b = 0; b < 64; ++b) {
        const uint64_t v = v0 + 3 * b + 1 + (b & 1);
        if (v >= lo && v < hi)
            m |= 1ull << b;
    }
    return m;
}

// One tile at a time per workgroup: presieve, LDS marks of the primes up to
// the plane length, merge with the large primes' bitmap words.
__global__ void __launch_bounds__(kWideThreads) k_wide_tile(WideArgs a)
{
    extern __shared__ uint32_t planes[];  // A_one words [0, pw), A_five words [pw, 2 pw)
    __shared__ uint32_t s_chunk[kMaxTileChunks];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t pw = a.pw;
    uint32_t *const pl1 = planes;
    uint32_t *const pl5 = planes + pw;
    const uint32_t ks = a.n_mid < a.k_split ? a.n_mid : a.k_split;
    const uint32_t n_items = ks > a.first_mark ? a.item_prefix[ks - a.first_mark] : 0u;
    const uint32_t kp0 = a.k_split > a.first_mark ? a.k_split : a.first_mark;
    const uint32_t n_plain = a.n_mid > kp0 ? a.n_mid - kp0 : 0u;
    const uint32_t n_work = n_items + n_plain;
    const uint32_t tile_chunks = pw / kChunkWords;

    for (uint32_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const uint32_t nw = t + 1 == a.ntiles ? a.last_words : pw;
        const uint32_t nb = 32 * nw;
        const uint64_t T0 = (uint64_t)t * 32 * pw;  // index of the tile's first bit
        if (tid < kMaxTileChunks)
            s_chunk[tid] = 0;

        // Presieve: the OR of the groups' patterns initialises both planes.
        {
            uint32_t o[kMaxGroups];
#pragma unroll
            for (int g = 0; g < kMaxGroups; ++g) {
                const uint32_t per = a.groups[g].period;
                o[g] = (uint32_t)((a.wphase[g] + (T0 + 32ull * tid) % per) % per);
            }
            for (uint32_t w = tid; w < nw; w += kWideThreads) {
                uint32_t c1 = 0, c5 = 0;
#pragma unroll
                for (int g = 0; g < kMaxGroups; ++g) {
                    const uint2 *tb = a.ps_tab + a.groups[g].offset + (o[g] >> 5);
                    const uint2 x = tb[0], y = tb[1];
                    const uint32_t sft = o[g] & 31;
                    c1 |= __builtin_amdgcn_alignbit(y.x, x.x, sft);
                    c5 |= __builtin_amdgcn_alignbit(y.y, x.y, sft);
                    o[g] += a.wstep[g];
                    o[g] = o[g] >= a.groups[g].period ? o[g] - a.groups[g].period : o[g];
                }
                pl1[w] = c1;
                pl5[w] = c5;
            }
        }
        __syncthreads();

        // Primes up to the plane length: Table 1 starts from
        // (B - 1) mod P = ((W - 1) mod P + (B - W) mod P) mod P, B the
        // tile's value base; a split prime's lane j takes hits j, j + g, ...
        {
            const uint64_t x = 6 * T0;  // B - W, below 2^62
            const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
            for (uint32_t v = tid; v < n_work; v += kWideThreads) {
                uint32_t kp, j, g;
                if (v < n_items) {
                    const uint2 it = a.items[v];
                    kp = it.x;
                    j = it.y >> 16;
                    g = it.y & 0xFFFFu;
                } else {
                    kp = kp0 + (v - n_items);
                    j = 0;
                    g = 1;
                }
                const PrimeConst pc = a.prm[kp];
                const uint32_t P = pc.p;
                const bool p5 = (pc.m_hi & kP5Flag) != 0;
                uint32_t rem = a.wr[kp] + mod_narrow(xl, xh, P, pc.m_lo, pc.m_hi & ~kP5Flag);
                rem = rem >= P ? rem - P : rem;
                uint32_t id1, id5;
                table1_ids(P + (p5 ? 0u : 4u) - rem, pc.r & 0x1FFFFFFFu, p5, id1, id5);
                const uint32_t step = g * P;
                for (uint32_t i = id1 + j * P; i < nb; i += step)
                    atomicOr(&pl1[i >> 5], 1u << (i & 31));
                for (uint32_t i = id5 + j * P; i < nb; i += step)
                    atomicOr(&pl5[i >> 5], 1u << (i & 31));
            }
        }

        // Bucket entries of the resident large primes (entries past the
        // last tile's words are dropped).
        if (a.boff) {
            const unsigned long long e0 = a.boff[t], e1 = a.boff[t + 1];
            for (unsigned long long e = e0 + tid; e < e1; e += kWideThreads) {
                const uint32_t v = a.bdata[e];
                const uint32_t bit = v & 0x7FFFFFFFu;
                if (bit < nb)
                    atomicOr(&(v >> 31 ? pl5 : pl1)[bit >> 5], 1u << (bit & 31));
            }
        }
        __syncthreads();

        // Merge with the extension primes' marks, keep [lo, hi), count per chunk.
        // The loop bound is uniform so that every lane takes part in the
        // wave sums; 64 consecutive words lie in one chunk.
        for (uint32_t w0 = 0; w0 < nw; w0 += kWideThreads) {
            const uint32_t w = w0 + tid;
            uint32_t cnt = 0;
            if (w < nw) {
                const uint64_t gw = (uint64_t)t * pw + w;
                const uint64_t comp = spread_even(pl1[w]) | (spread_even(pl5[w]) << 1) | a.bitmap[gw];
                const uint64_t pm = ~comp & range_mask(gw, a.lo_rel, a.hi_rel);
                if (a.list)
                    a.bitmap[gw] = pm;
                cnt = (uint32_t)__popcll(pm);
            }
            cnt = wave_sum(cnt);
            if (lane == 0 && w < nw)
                atomicAdd(&s_chunk[w / kChunkWords], cnt);
        }
        __syncthreads();
        const uint32_t nch = (nw + kChunkWords - 1) / kChunkWords;
        if (a.list) {
            if (tid < nch)
                a.chunk_counts[(uint64_t)t * tile_chunks + tid] = s_chunk[tid];
        } else if (tid < kWave) {
            uint32_t c = tid < nch ? s_chunk[tid] : 0u;
            c = wave_sum(c);
            if (tid == 0)
                atomicAdd(&a.counts[0], (unsigned long long)c);
        }
        __syncthreads();  // the planes and s_chunk are reused by the next tile
    }
}

using u128 = unsigned __int128;

u128 to_u128(const sieve_u128 &x) { return ((u128)x.hi << 64) | x.lo; }

// floor(sqrt(n)) for any 128-bit n: a long double estimate (clamped below
// 2^64, since the root of n near 2^128 rounds up to 2^64), corrected by
// exact products; (s + 1)^2 is formed only while s + 1 < 2^64.
uint64_t isqrt_u128(u128 n)
{
    if (n < 2)
        return (uint64_t)n;
    const long double r = sqrtl((long double)n);
    uint64_t s = r >= 18446744073709551615.0L ? UINT64_MAX : (uint64_t)r;
    while ((u128)s * s > n)
        --s;
    while (s < UINT64_MAX && (u128)(s + 1) * (s + 1) <= n)
        ++s;
    return s;
}

// Extension primes <= x: the host sample finds the block, one short copy
// from the device finishes the count.
int ext_upto(sieve_ctx *c, uint64_t x, uint64_t &n)
{
    n = 0;
    if (!c->n_ext || x < c->h_ext_sample[0])
        return SIEVE_OK;
    const size_t b = (size_t)(std::upper_bound(c->h_ext_sample.begin(), c->h_ext_sample.end(), x) -
                              c->h_ext_sample.begin()) - 1;
    const uint64_t i0 = b * kExtSample;
    const uint64_t i1 = std::min<uint64_t>(c->n_ext, i0 + kExtSample);
    std::vector<uint64_t> blk(i1 - i0);
    hipError_t e = hipMemcpy(blk.data(), c->d_ext.p + i0, blk.size() * sizeof(uint64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return rt::hip_status(e);
    n = i0 + (uint64_t)(std::upper_bound(blk.begin(), blk.end(), x) - blk.begin());
    return SIEVE_OK;
}

// Base primes of a window ending at H: resident ones up to isqrt(H - 1)
// (n_act) and extension ones (n_ext).  The resident store ends below 2^32;
// 2^32 itself is not prime, so the extension list is needed from
// isqrt(H - 1) = 2^32 + 1 on.
int window_primes(sieve_ctx *c, u128 H, uint64_t &root, uint32_t &n_act, uint64_t &n_ext)
{
    root = isqrt_u128(H - 1);
    constexpr uint64_t kResTop = 0xFFFFFFFFull;
    const uint64_t res_need = std::min<uint64_t>(root, kResTop);
    const bool need_ext = root > kResTop + 1;
    if (c->limit < res_need || (need_ext && c->ext_limit < root))
        return SIEVE_E_RANGE;
    n_act = rt::primes_upto(c, res_need);
    n_ext = 0;
    return need_ext ? ext_upto(c, root, n_ext) : SIEVE_OK;
}

// Resident primes marked in LDS tile by tile: up to kMidPlanes plane lengths
// (the larger ones go through the buckets).  Measured on the count of
// [2^64, 2^64 + 10^10) and of 10^9: 1, 2, 4, 8 and 16 plane lengths give
// 25.3 / 3.79, 24.7 / 3.71, 24.4 / 3.71, 24.9 / 3.84 and 24.7 / 4.16 ms.  A
// window of few tiles keeps most CUs out of the tile kernel, so there the
// cut-off shrinks with the tiles per CU.
uint32_t mid_primes(const sieve_ctx *c, uint64_t root, uint64_t nt)
{
    const uint32_t pw = c->prm.segment_bytes / 8;
    const uint64_t planes = std::max<uint64_t>(1, std::min<uint64_t>(kMidPlanes, kMidPlanes * nt / c->cus));
    return std::max(rt::primes_upto(c, std::min<uint64_t>(root, planes * 32ull * pw)), c->first_mark);
}

// End of the bucketed resident primes for a window of nwords plane words:
// primes below its plane bits, which hit it at least twice (measured: a
// cut-off at 1, 2, 4 or 8 hits gives 26.3, 24.6, 25.6 and 27.8 ms for the
// count of [2^64, 2^64 + 10^10)).
uint32_t bucket_end(const sieve_ctx *c, uint64_t root, uint64_t nwords)
{
    const uint64_t top = std::min<uint64_t>(std::min<uint64_t>(root, 0xFFFFFFFFull), 32ull * nwords);
    return top > c->limit ? (uint32_t)c->h_primes.size() : rt::primes_upto(c, top);
}

// One window piece [L, H) (validated by the caller): count, or list into out.
int wide_piece(sieve_ctx *c, u128 L, u128 H, bool list, U128 *out, uint64_t cap, uint64_t &count, hipStream_t s)
{
    count = 0;
    const u128 W = L - L % 6;
    const uint64_t lo_rel = (uint64_t)(L - W), hi_rel = (uint64_t)(H - W);
    const uint32_t pw = c->prm.segment_bytes / 8;
    uint64_t nt, base;
    uint32_t last_words;
    rt::plan_range(lo_rel, hi_rel, pw, nt, base, last_words);
    if (nt == 0)
        return SIEVE_OK;
    if (nt > 0xFFFFFFFFull || pw > kMaxTileChunks * kChunkWords)
        return SIEVE_E_INVAL;
    uint64_t root, n_ext;
    uint32_t n_act;
    int st = window_primes(c, H, root, n_act, n_ext);
    if (st != SIEVE_OK)
        return st;
    const uint32_t n_mid = std::min(mid_primes(c, root, nt), std::max(n_act, c->first_mark));
    const uint64_t nwords_all = (nt - 1) * pw + last_words;
    const uint32_t n_big = std::max(n_mid, bucket_end(c, root, nwords_all));
    const bool buckets = n_big > n_mid;  // resident primes bucketed past the LDS-marked ones
    const uint64_t nwords = (nt - 1) * pw + last_words;
    const uint64_t nch = (nt - 1) * (pw / kChunkWords) + (last_words + kChunkWords - 1) / kChunkWords;
    const uint64_t nseg = (nch + kSegChunks - 1) / kSegChunks;
    st = rt::ensure_capacity(c, 1, nch, nt, 0);
    if (st != SIEVE_OK)
        return st;
    if (!c->d_wr.reserve(std::max<uint32_t>(n_mid, 1)))
        return SIEVE_E_NOMEM;

    WideArgs a;
    memset(&a, 0, sizeof a);
    a.wlo = (uint64_t)W;
    a.whi = (uint64_t)(W >> 64);
    a.wm1_lo = (uint64_t)(W - 1);
    a.wm1_hi = (uint64_t)((W - 1) >> 64);
    a.lo_rel = lo_rel;
    a.hi_rel = hi_rel;
    a.nwords = nwords;
    a.pw = pw;
    a.ntiles = (uint32_t)nt;
    a.last_words = last_words;
    a.list = list ? 1u : 0u;
    a.prm = c->d_prm.p;
    a.items = c->d_items.p;
    a.item_prefix = c->d_item_prefix.p;
    a.first_mark = c->first_mark;
    a.k_split = c->k_split;
    a.n_mid = n_mid;
    a.n_act = std::max(n_act, n_big);
    a.k_atomic = n_big;
    a.wr = c->d_wr.p;
    a.ext = c->d_ext.p;
    a.n_ext = n_ext;
    a.ps_tab = c->d_pstab.p;
    const u128 w6 = W / 6;
    for (int g = 0; g < kMaxGroups; ++g) {
        a.groups[g] = c->groups[g];
        a.wphase[g] = (uint32_t)(w6 % c->groups[g].period);
        a.wstep[g] = (32u * kWideThreads) % c->groups[g].period;
    }
    a.bitmap = c->d_bitmap.p;
    a.chunk_counts = c->d_chunk_counts.p;
    a.counts = c->d_counts.p;

    // Job blob for the shared bucket / finalize / scan / compaction kernels:
    // one range in offsets from W.
    JobHeader h;
    memset(&h, 0, sizeof h);
    RangeDesc d;
    memset(&d, 0, sizeof d);
    d.lo = lo_rel;
    d.hi = hi_rel;
    d.base = 0;
    d.ntiles = (uint32_t)nt;
    d.last_words = last_words;
    d.mode = list ? 1u : 0u;
    d.nact = n_big;  // the bucket sieve takes primes [kbig, nact)
    d.kbig = n_mid;
    d.bwins = (uint32_t)((nt + kBucketWindow - 1) / kBucketWindow);
    d.bunits = buckets ? ((n_big - n_mid + kBucketThreads - 1) / kBucketThreads) * d.bwins : 0;
    if (list) {
        d.nchunks = (uint32_t)nch;
        d.nseg = (uint32_t)nseg;
        d.cap = cap;
    }
    d.nparts = 1;
    d.strip = 1;
    d.nstrips = (uint32_t)nt;
    h.ntiles = nt;
    h.nchunks = list ? nch : 0;
    h.nseg = list ? nseg : 0;
    h.nunits = d.bunits;
    h.bmode = 2;
    h.nranges = 1;
    h.nlist = list ? 1u : 0u;
    h.out = out;
    h.elem_bytes = (int32_t)sizeof(U128);
    h.wide = 1;
    const size_t roff = rt::blob_ranges_offset();
    const JobHeader *job = (const JobHeader *)c->d_blob.p;
    const RangeDesc *ranges = (const RangeDesc *)(c->d_blob.p + roff);
    hipError_t e = hipMemcpyAsync(c->d_blob.p, &h, sizeof h, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_blob.p + roff, &d, sizeof d, hipMemcpyHostToDevice, s);
    const uint32_t cus = (uint32_t)c->cus;
    const uint64_t bm_words = nch * kChunkWords;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_wide_clear, dim3(cus * 4), dim3(256), 0, s, a.bitmap, bm_words, c->d_counters.p,
                           a.counts);
        e = hipGetLastError();
    }
    if (e == hipSuccess && buckets) {
        // Exact bucket layout: count the hits per tile, scan, then fill.
        BucketArgs b;
        memset(&b, 0, sizeof b);
        b.job = job;
        b.ranges = ranges;
        b.prm = c->d_prm.p;
        b.bcount = c->d_bcount.p;
        b.bcursor = c->d_bcursor.p;
        b.boff = c->d_boff.p;
        b.counters = c->d_counters.p;
        b.skip5 = (c->ngroups >= 1 && c->prm.cofactor_skip != SIEVE_SKIP_NONE) ? 1u : 0u;
        b.nbits = 32 * pw;
        b.span = 192ull * pw;
        b.span_rcp = UINT64_MAX / b.span;
        uint32_t win = 64;
        while (win < std::min<uint64_t>(nt, kBucketWindow))
            win <<= 1;
        b.win = std::min(win, kBucketWindow);
        b.wide = 1;
        b.w5 = (uint32_t)(W % 5);
        b.wlo = a.wlo;
        b.whi = a.whi;
        b.wm1_lo = a.wm1_lo;
        b.wm1_hi = a.wm1_hi;
        e = launch_zero(job, c->d_counters.p, c->d_counts.p, c->d_bcount.p, c->d_gbm.p, c->d_garrive.p, nullptr, s);
        if (e == hipSuccess)
            e = launch_bucket(b, 0, cus, s);
        BucketScanArgs sc;
        sc.job = job;
        sc.bcount = c->d_bcount.p;
        sc.boff = c->d_boff.p;
        sc.bcursor = c->d_bcursor.p;
        if (e == hipSuccess)
            e = launch_bucket_scan(sc, s);
        unsigned long long total = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&total, c->d_boff.p + nt, sizeof total, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e == hipSuccess && total > c->cap_bdata) {
            c->cap_bdata = std::max<uint64_t>(total, c->cap_bdata + c->cap_bdata / 2);
            c->d_bdata.release();
            c->gen++;  // captured graphs hold the old address
            if (!c->d_bdata.reserve(c->cap_bdata))
                return SIEVE_E_NOMEM;
        }
        b.bdata = c->d_bdata.p;
        if (e == hipSuccess)
            e = launch_bucket(b, 1, cus, s);
        a.bdata = c->d_bdata.p;
        a.boff = c->d_boff.p;
    }
    if (e == hipSuccess && a.n_mid > a.first_mark) {
        hipLaunchKernelGGL(k_wide_prep, dim3(std::min<uint32_t>(cus * 4, (a.n_mid + 255) / 256)), dim3(256), 0, s,
                           a, c->d_wr.p);
        e = hipGetLastError();
    }
    const uint64_t n_large = (uint64_t)(a.n_act - a.k_atomic) + n_ext;
    if (e == hipSuccess && n_large) {
        const uint64_t blocks = std::min<uint64_t>((n_large + kLargeThreads - 1) / kLargeThreads, cus * 32ull);
        hipLaunchKernelGGL(k_wide_large, dim3((uint32_t)blocks), dim3(kLargeThreads), 0, s, a);
        e = hipGetLastError();
    }
    const size_t lds = (size_t)pw * 8;
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_wide_tile, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_wide_tile, dim3((uint32_t)std::min<uint64_t>(nt, cus)), dim3(kWideThreads), lds, s, a);
        e = hipGetLastError();
    }
    SegArgs g;
    g.job = job;
    g.ranges = ranges;
    g.chunk_counts = c->d_chunk_counts.p;
    g.seg_sum = c->d_seg_sum.p;
    g.seg_base = c->d_seg_base.p;
    g.chunk_off = c->d_chunk_off.p;
    g.chunk_vbase = c->d_chunk_vbase.p;
    if (e == hipSuccess && list)
        e = launch_seg(g, 0, cus * 2, s);
    FinalizeArgs f;
    f.job = job;
    f.ranges = ranges;
    f.counts = c->d_counts.p;
    f.status = c->d_status.p;
    f.seg_sum = c->d_seg_sum.p;
    f.seg_base = c->d_seg_base.p;
    if (e == hipSuccess)
        e = launch_finalize(f, 1, s);
    if (e == hipSuccess && list)
        e = launch_seg(g, 1, cus * 2, s);
    CompactArgs k;
    k.job = job;
    k.chunk_vbase = c->d_chunk_vbase.p;
    k.bitmap = c->d_bitmap.p;
    k.chunk_off = c->d_chunk_off.p;
    k.wbase_lo = a.wlo;
    k.wbase_hi = a.whi;
    if (e == hipSuccess && list)
        e = launch_compact_wide(k, cus * 4, s);
    unsigned long long res[2] = {0, 0};
    int32_t status = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&res[0], c->d_counts.p, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&status, c->d_status.p, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&res[1], c->d_counters.p + kErrorFlag, sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return rt::hip_status(e);
    if (res[1])
        return SIEVE_E_DEVICE;
    count = res[0];
    return status;
}

// One wide window: count (list false) or list into out.  A window whose
// bucket entries would exceed the context's bucket memory runs as pieces of
// whole tiles, each sieved from its own base; counts add up and list pieces
// follow each other in the output.
int wide_job(sieve_ctx *c, const sieve_u128 &lo128, const sieve_u128 &hi128, bool list, U128 *out, uint64_t cap,
             uint64_t *count, hipStream_t stream)
{
    const u128 L = to_u128(lo128), H = to_u128(hi128);
    if (L < (u128)SIEVE_WIDE_MIN_LO || H < L || H - L > (u128)SIEVE_WIDE_MAX_SPAN)
        return SIEVE_E_INVAL;
    *count = 0;
    if (H == L)
        return SIEVE_OK;
    uint64_t root, n_ext;
    uint32_t n_act;
    int st = window_primes(c, H, root, n_act, n_ext);
    if (st != SIEVE_OK)
        return st;
    hipStream_t s = stream ? stream : c->stream;
    // The scratch is shared with the context's stream-ordered jobs.
    if (c->last_valid && hipEventSynchronize(c->last_ev) != hipSuccess) {
        (void)hipGetLastError();
        return SIEVE_E_DEVICE;
    }
    // Tiles per piece from the expected bucket entries per tile: each
    // resident prime p past the LDS-marked ones hits a plane of nbits bits
    // nbits / p times, plus a margin of 8 standard deviations.
    const uint32_t pw = c->prm.segment_bytes / 8;
    const u128 span = (u128)192 * pw;
    const u128 W = L - L % 6;
    const uint64_t nt_all = (uint64_t)((H - W + span - 1) / span);
    const uint32_t n_mid = std::min(mid_primes(c, root, nt_all), std::max(n_act, c->first_mark));
    const uint32_t n_big = std::max(n_mid, bucket_end(c, root, nt_all * pw));
    uint64_t tiles = nt_all;
    if (n_big > n_mid) {
        // pieces of equal size: each costs a pass over every bucketed prime
        const double E = 2.0 * 32.0 * pw * (c->inv_prefix[n_big] - c->inv_prefix[n_mid]);
        const double per_tile = E + 8.0 * std::sqrt(E) + 64.0;
        const uint64_t fit = std::max<uint64_t>(1, (uint64_t)((double)c->bucket_budget / per_tile));
        const uint64_t pieces = (nt_all + fit - 1) / fit;
        tiles = (nt_all + pieces - 1) / pieces;
    }
    uint64_t total = 0;
    bool over = false;
    u128 a = L;
    for (uint64_t k = 0; a < H; ++k) {
        u128 b = W + (u128)(k + 1) * tiles * span;
        if (b > H)
            b = H;
        const bool lst = list && !over;
        uint64_t n = 0;
        st = wide_piece(c, a, b, lst, lst ? out + total : nullptr, lst ? cap - total : 0, n, s);
        if (st == SIEVE_E_CAPACITY) {
            over = true;  // keep counting the rest for the required size
            st = SIEVE_OK;
        }
        if (st != SIEVE_OK)
            return st;
        total += n;
        a = b;
    }
    if (hipEventRecord(c->last_ev, s) != hipSuccess) {
        (void)hipGetLastError();
        return SIEVE_E_DEVICE;
    }
    c->last_stream = s;
    c->last_valid = true;
    *count = total;
    return over ? SIEVE_E_CAPACITY : SIEVE_OK;
}

}  // namespace
}  // namespace sieve

using namespace sieve;

extern "C" {

int sieve_base_primes_wide(sieve_ctx *ctx, uint64_t limit, uint64_t *n_out)
{
    if (!ctx)
        return SIEVE_E_INVAL;
    if (limit > SIEVE_WIDE_MAX_BASE)
        return rt::set_err(ctx, SIEVE_E_INVAL);
    constexpr uint64_t kResTop = 0xFFFFFFFFull;
    int st = sieve_base_primes(ctx, std::min(limit, kResTop), nullptr);
    if (st == SIEVE_OK && limit > kResTop && limit > ctx->ext_limit) {
        if (hipSetDevice(ctx->device) != hipSuccess)
            return rt::set_err(ctx, SIEVE_E_DEVICE);
        // The 64-bit list path writes the primes of [2^32, limit] straight
        // into a new extension list.
        const uint64_t lo = kResTop + 1, hi = limit + 1;
        const uint64_t bound = sieve_list_bound(lo, hi);
        rt::DevBuf<uint64_t> buf;
        if (!buf.reserve(bound))
            return rt::set_err(ctx, SIEVE_E_NOMEM);
        const uint8_t mode = 1;
        const uint64_t off = 0;
        uint64_t cnt = 0;
        int32_t rs = 0;
        st = rt::run_job(ctx, 1, &lo, &hi, &mode, &off, &bound, 8, buf.p, &cnt, &rs, nullptr, false);
        if (st == SIEVE_OK)
            st = rs;
        std::vector<uint64_t> sample;
        if (st == SIEVE_OK && cnt) {
            sample.resize((cnt + kExtSample - 1) / kExtSample);
            hipError_t e = hipMemcpy2D(sample.data(), sizeof(uint64_t), buf.p, kExtSample * sizeof(uint64_t),
                                       sizeof(uint64_t), sample.size(), hipMemcpyDeviceToHost);
            st = rt::hip_status(e);
        }
        if (st != SIEVE_OK) {
            buf.release();
            return rt::set_err(ctx, st);
        }
        ctx->d_ext.release();
        ctx->d_ext = buf;
        ctx->n_ext = cnt;
        ctx->ext_limit = limit;
        ctx->h_ext_sample = std::move(sample);
    }
    if (st == SIEVE_OK && n_out)
        *n_out = ctx->h_primes.size() + ctx->n_ext;
    return rt::set_err(ctx, st);
}

int sieve_ext_limit(const sieve_ctx *ctx, uint64_t *limit)
{
    if (!ctx || !limit)
        return SIEVE_E_INVAL;
    *limit = ctx->ext_limit;
    return SIEVE_OK;
}

int sieve_count_wide(sieve_ctx *ctx, const sieve_u128 *lo, const sieve_u128 *hi, uint64_t *count, void *stream)
{
    if (!ctx || !lo || !hi || !count)
        return rt::set_err(ctx, SIEVE_E_INVAL);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return rt::set_err(ctx, SIEVE_E_DEVICE);
    return rt::set_err(ctx, wide_job(ctx, *lo, *hi, false, nullptr, 0, count, (hipStream_t)stream));
}

int sieve_list_wide(sieve_ctx *ctx, const sieve_u128 *lo, const sieve_u128 *hi, sieve_u128 *out_dev, uint64_t cap,
                    uint64_t *n_out, void *stream)
{
    if (!ctx || !lo || !hi || !n_out || (!out_dev && cap))
        return rt::set_err(ctx, SIEVE_E_INVAL);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return rt::set_err(ctx, SIEVE_E_DEVICE);
    return rt::set_err(ctx, wide_job(ctx, *lo, *hi, true, (U128 *)out_dev, cap, n_out, (hipStream_t)stream));
}

}  // extern "C"
