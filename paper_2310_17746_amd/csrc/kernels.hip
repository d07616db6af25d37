// Device kernels of the segmented wheel sieve (gfx950, wave64).
//
// k_zero       clears the job's counters, counts, bucket cursors and the
//              split tiles' global planes (a kernel, so that the whole job
//              can be captured in a graph).
// k_bucket     bucket sieve for the large primes of multi-tile ranges: walks
//              each prime's hits tile by tile and bins them per tile (count,
//              scan and fill passes for the exact layout; one fill pass into
//              estimated per-tile slices otherwise).
// k_sieve      one persistent launch over every tile of a job.  Per tile, in
//              LDS: presieve init, Table 1 starts + marking of the remaining
//              base primes, the tile's bucket entries, edge masks, then either
//              a popcount into the range's count or a value-ordered bitmap +
//              per-chunk counts.  A split tile's parts run on several
//              workgroups and meet in a global copy of the planes.
// k_seg_sum    per scan segment (4096 chunks of a list range): chunk-count sum.
// k_finalize   per range: adds 2 and 3 when in range, scans the segment sums
//              of list ranges into segment output bases, sets count and status.
// k_seg_scan   per scan segment: each chunk's output offset and value base.
// k_compact    per bitmap chunk: popcount, block prefix, LDS staging and
//              coalesced stores of the primes as uint32 or uint64.
#include <atomic>

#include "sieve_internal.h"
#include "wheel.h"

namespace sieve {

namespace {

constexpr uint32_t kWave = 64;

__device__ inline uint64_t isqrt_dev(uint64_t x)
{
    if (x < 2)
        return x;
    uint64_t s = (uint64_t)sqrt((double)x);
    while (s * s > x)
        --s;
    while ((s + 1) * (s + 1) <= x)
        ++s;
    return s;
}

__device__ inline uint32_t wave_sum(uint32_t x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        x += __shfl_xor(x, d, kWave);
    return x;
}

__device__ inline uint32_t wave_incl_scan(uint32_t x, uint32_t lane)
{
#pragma unroll
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= d)
            x += y;
    }
    return x;
}

// Spreads the 32 bits of x to the even bit positions of a 64-bit word
// (interleaving by binary magic numbers, as in S. E. Anderson's
// "Bit Twiddling Hacks").
__device__ inline uint64_t spread32(uint32_t x)
{
    uint64_t v = x;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

// The two planes live at LDS byte address 0: A_one words at bytes [0, 4PW),
// A_five words at [4PW, 8PW).  Marks address LDS through this computed byte
// address (the kernel checks that its dynamic LDS starts at 0).  Keeping the
// planes apart lets the marks of one plane use every LDS bank.
typedef __attribute__((address_space(3))) uint32_t lds_u32;

__device__ __forceinline__ void lds_or(uint32_t byte_addr, uint32_t mask)
{
    __atomic_fetch_or((lds_u32 *)(size_t)byte_addr, mask, __ATOMIC_RELAXED);
}

// Marking tally of the debug build (SIEVE_MARK_COUNT), per thread: the hits
// the marking loops visit (whether they issue the OR or skip it because the
// cofactor is a multiple of 5, which the presieve has cleared), the ORs
// issued, the hits skipped, and the runs whose first hit is not a multiple of
// its prime at or past the prime's square.  In the product build the struct
// is empty and every call compiles to nothing.
struct MarkTally {
#ifdef SIEVE_MARK_COUNT
    unsigned long long hits = 0, issued = 0, skipped = 0, bad = 0;
    __device__ __forceinline__ void op() { ++issued; }
    __device__ __forceinline__ uint64_t run(uint32_t start, uint32_t step, uint32_t end)
    {
        const uint64_t h = start < end ? ((uint64_t)end - start + step - 1) / step : 0;
        hits += h;
        return h;
    }
    __device__ __forceinline__ void skip(uint64_t n) { skipped += n; }
    __device__ __forceinline__ void check(uint64_t B, uint32_t i, uint32_t r, uint32_t P)
    {
        const uint64_t v = B + 6ull * i + r;
        if (v % P != 0 || v < (uint64_t)P * P)
            ++bad;
    }
#else
    __device__ __forceinline__ void op() {}
    __device__ __forceinline__ uint64_t run(uint32_t, uint32_t, uint32_t) { return 0; }
    __device__ __forceinline__ void skip(uint64_t) {}
    __device__ __forceinline__ void check(uint64_t, uint32_t, uint32_t, uint32_t) {}
#endif
};

#ifdef SIEVE_MARK_COUNT
// Adds a thread's tally to the job's four counters (wavefront sums first).
__device__ inline void tally_flush(const MarkTally &t, unsigned long long *out)
{
    unsigned long long v[4] = {t.hits, t.issued, t.skipped, t.bad};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        for (int d = 32; d >= 1; d >>= 1)
            v[q] += __shfl_xor(v[q], d, 64);
        if ((threadIdx.x & 63) == 0 && v[q])
            atomicAdd(&out[q], v[q]);
    }
}
#endif

__device__ __forceinline__ void lds_or(uint32_t byte_addr, uint32_t mask, MarkTally &t)
{
    t.op();
    lds_or(byte_addr, mask);
}

// Sets the composite bits start, start + step, ... below end of the plane
// bit array (A_one bits from 0, A_five bits from 32 pw) and returns the first
// index at or past end, where the next tile's hits continue.  The paper
// strides by P indices in each array (Sec. 3: adding P to the index adds 6P
// to the value and keeps the residue mod 6).
__device__ __forceinline__ uint32_t mark_run(uint32_t i, uint32_t step, uint32_t end, MarkTally &t)
{
    if (i >= end)
        return i;
    (void)t.run(i, step, end);
    if (step < (end >> 2)) {
        const uint32_t lim = end - 3 * step;  // i < lim keeps i + 3*step < end
        while (i < lim) {
            // Keep one induction variable in a register (an empty asm operand
            // stops the compiler from splitting it into several).
            asm volatile("" : "+v"(i));
            const uint32_t i1 = i + step, i2 = i1 + step, i3 = i2 + step;
            lds_or((i >> 3) & ~3u, 1u << (i & 31), t);
            lds_or((i1 >> 3) & ~3u, 1u << (i1 & 31), t);
            lds_or((i2 >> 3) & ~3u, 1u << (i2 & 31), t);
            lds_or((i3 >> 3) & ~3u, 1u << (i3 & 31), t);
            i = i3 + step;
        }
    }
    for (; i < end; i += step)
        lds_or((i >> 3) & ~3u, 1u << (i & 31), t);
    return i;
}

// As mark_plane for a step that is a multiple of 32 bits: every hit then
// sits at the same bit of its word, so the mask is fixed and the LDS byte
// address advances by step / 8.  One add per mark.
__device__ __forceinline__ void mark_plane_fixed(uint32_t start, uint32_t step, uint32_t nbits, MarkTally &t)
{
    if (start >= nbits)
        return;
    (void)t.run(start, step, nbits);
    const uint32_t mask = 1u << (start & 31);
    const uint32_t end = nbits >> 3;  // nbits is a whole number of words
    const uint32_t sb = step >> 3;
    uint32_t a = (start >> 3) & ~3u;
    if (sb < (end >> 2)) {
        const uint32_t lim = end - 3 * sb;  // a < lim keeps a + 3*sb < end
        while (a < lim) {
            asm volatile("" : "+v"(a));
            lds_or(a, mask, t);
            lds_or(a + sb, mask, t);
            lds_or(a + 2 * sb, mask, t);
            lds_or(a + 3 * sb, mask, t);
            a += 4 * sb;
        }
    }
    for (; a < end; a += sb)
        lds_or(a, mask, t);
}

// As mark_plane_fixed, skipping hit n when n = s (mod 5): the lane's hits
// n = 0, 1, 2, ... have cofactors running through the residues mod 5 with
// period 5 (its step is g P bits with g prime to 5), and the skipped ones are
// multiples of 5, already cleared by the presieve.  Four ORs per period of
// five hits, at byte offsets fixed for the lane.  s in 0..4.
__device__ __forceinline__ void mark_plane_fixed_skip5(uint32_t start, uint32_t step, uint32_t nbits, uint32_t s,
                                                       MarkTally &t)
{
    if (start >= nbits)
        return;
    {
        const uint64_t h = t.run(start, step, nbits);
        t.skip(h > s ? (h - s - 1) / 5 + 1 : 0);
    }
    const uint32_t mask = 1u << (start & 31);
    const uint32_t end = nbits >> 3;  // nbits is a whole number of words
    const uint32_t sb = step >> 3;
    uint32_t a = (start >> 3) & ~3u;
    if (sb < end / 5) {
        const uint32_t s2 = sb + sb, s3 = s2 + sb, s4 = s3 + sb, s5 = s4 + sb;
        const uint32_t o0 = s == 0 ? sb : 0u;
        const uint32_t o1 = s <= 1 ? s2 : sb;
        const uint32_t o2 = s <= 2 ? s3 : s2;
        const uint32_t o3 = s <= 3 ? s4 : s3;
        const uint32_t lim = end - 4 * sb;  // a < lim keeps a + 4*sb < end
        while (a < lim) {
            asm volatile("" : "+v"(a));
            lds_or(a + o0, mask, t);
            lds_or(a + o1, mask, t);
            lds_or(a + o2, mask, t);
            lds_or(a + o3, mask, t);
            a += s5;
        }
    }
    // The rest, hit by hit: a whole period when the loop ran (it stops with
    // a + 4 sb >= end), else every hit (with sb = floor(end / 5) and end not
    // a multiple of 5 there can be six).
    for (uint32_t n = 0; a < end; a += sb, n = n == 4 ? 0u : n + 1u)
        if (n != s)
            lds_or(a, mask, t);
}

// As mark_plane, for a lane whose hits n = 0, 1, 2, ... have cofactors
// running through the residues mod 5 with period 5, skipping hit n when
// n = s (mod 5): those values are multiples of 5, already cleared by the
// presieve, so a fifth of the LDS operations is saved.  s in 0..4.
__device__ __forceinline__ void mark_plane_skip5(uint32_t base, uint64_t start, uint32_t step, uint32_t nbits,
                                                 uint32_t s, MarkTally &t)
{
    if (start >= nbits)
        return;
    {
        // hits n = s, s + 5, ... of the run are skipped
        const uint64_t h = t.run((uint32_t)start, step, nbits);
        t.skip(h > s ? (h - s - 1) / 5 + 1 : 0);
    }
    uint32_t i = (uint32_t)start;
    if (step < nbits / 5) {
        // kept offsets of one period of five hits
        const uint32_t s2 = step + step, s3 = s2 + step, s4 = s3 + step;
        const uint32_t o0 = s == 0 ? step : 0u;
        const uint32_t o1 = s <= 1 ? s2 : step;
        const uint32_t o2 = s <= 2 ? s3 : s2;
        const uint32_t o3 = s <= 3 ? s4 : s3;
        const uint32_t lim = nbits - 4 * step;  // i < lim keeps i + 4*step < nbits
        while (i < lim) {
            asm volatile("" : "+v"(i));
            const uint32_t i0 = i + o0, i1 = i + o1, i2 = i + o2, i3 = i + o3;
            lds_or(((i0 >> 3) & ~3u) + base, 1u << (i0 & 31), t);
            lds_or(((i1 >> 3) & ~3u) + base, 1u << (i1 & 31), t);
            lds_or(((i2 >> 3) & ~3u) + base, 1u << (i2 & 31), t);
            lds_or(((i3 >> 3) & ~3u) + base, 1u << (i3 & 31), t);
            i += 5 * step;
        }
    }
    // The rest, hit by hit (as in mark_plane_fixed_skip5: up to six when
    // the loop did not run).
    for (uint32_t n = 0; i < nbits; i += step, n = n == 4 ? 0u : n + 1u)
        if (n != s)
            lds_or(((i >> 3) & ~3u) + base, 1u << (i & 31), t);
}

// Residue mod 5 of the cofactor m of the value B + 6*id + r = m * P, from
// B mod 5 and P^-1 mod 5 (6 = 1 mod 5).
__device__ __forceinline__ uint32_t cofactor_mod5(uint32_t b5, uint32_t id, uint32_t r, uint32_t inv5)
{
    return ((b5 + id % 5u + r) * inv5) % 5u;
}

}  // namespace

// Bookkeeping of one strip and its current tile, kept in LDS after the two
// planes so that the planes start at LDS address 0 (a mark's address is then
// (i >> 3) & ~3).
struct TileShared {
    uint32_t range;
    uint32_t k0, k1;    // the strip: tiles [k0, k1) of the range
    uint32_t part;      // split tiles: this workgroup's part
    uint32_t ok;        // a work unit was taken
    uint32_t nact;
    uint32_t sqb, sqe;  // isqrt(tile base), isqrt(tile end - 1), clamped to 32 bits
    uint32_t psoff[kMaxGroups];
    uint32_t red[1024 / 64];
    uint32_t chunk[64];
    uint32_t last;  // split tiles: this workgroup finished the tile's last part
};

// Primes per thread whose next hits stay in registers from one tile of a
// strip to the next (Sec. 2.4: each prime keeps its place and the sieve goes
// on from there), for W waves per SIMD: four leave 128 VGPRs per lane, six
// (three 512-thread workgroups per CU) 80.
template <int W>
constexpr int reg_primes()
{
    return W <= 4 ? 32 : 8;
}

// First hit of prime pc in plane A_one, as an index relative to the base B of
// the first tile of a strip (sqb = isqrt(B), sqe = isqrt(first tile end - 1)).
// When P*P lies before that tile's end this is the Table 1 start.  Otherwise
// marking starts at the square itself (Sec. 1.1), and P*P = 1 (mod 6) is the
// first hit in A_one.  Indices past 2^32 - 1 saturate there; a strip spans
// far fewer.  (The A_five hits follow from it, at a fixed offset; see below.)
template <bool U24>
__device__ __forceinline__ uint32_t strip_start(const PrimeConst &pc, uint32_t sqb, uint32_t sqe, uint64_t B,
                                                bool narrow)
{
    uint32_t id1, id5;
    if (pc.p <= sqe) {
        if (U24)
            tile_start_u24(pc, sqb, B - 1, (uint32_t)B, narrow, id1, id5);
        else
            tile_start(pc, sqb, B - 1, (uint32_t)B, narrow, id1, id5);
        return id1;
    }
    const uint64_t P = pc.p;
    const uint64_t i1 = (P * P - B - 1) / 6;  // P*P lies past the tile, so it is > B; 6 | P*P - 1
    return i1 > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)i1;
}

// The multiples of P that fall in A_five are the A_one multiples shifted by
// dlt indices: P*P is the first hit of A_one, and the next multiple coprime
// to 6, P (P + 4) for P = 1 (mod 6) or P (P + 2) for P = 5 (mod 6), the
// first of A_five, dlt = 2 (P - 1) / 3 or (P - 2) / 3 indices later.  So for
// a tile with base B, given the first A_one hit id1:
//  - while the square lies at or past B (P > isqrt(B)) the first A_five hit
//    is id1 + dlt (none in the tile when id1 is past it already);
//  - once the square lies before B both progressions run through the whole
//    tile, id1 < P, and the first A_five hit is (id1 + dlt) mod P, which can
//    lie in the tile when id1 does not.

// W: waves per SIMD the kernel is compiled for (4: one 1024-thread or two
// 512-thread workgroups per CU; 6: three 512-thread workgroups).
// U24: every active prime of the job is below 2^24 - 8, so the Table 1
// starts and the per-item products use the full-rate 24-bit multiplier.
//
// One work unit is a strip of consecutive tiles of one range (or one part of
// a split tile).  The workgroup sieves the strip's tiles in order; the first
// min(n, K * NT) primes after the split items keep their next hit in
// registers (K per thread) and so need one Table 1 start per strip instead
// of one per tile; the primes beyond them start afresh in every tile.
//
// The planes are all zero whenever a tile begins (the count pass clears
// every word it reads), so a tile's presieve patterns, marks and bucket
// entries are all ORed in during one phase, with no barrier between them;
// one barrier separates marking from counting and one ends the tile.
template <int NT, int W, bool U24>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(W))) k_sieve(SieveArgs a)
{
    constexpr int K = reg_primes<W>();
    extern __shared__ uint32_t lds[];
    MarkTally tally;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    const uint32_t pw = a.pw;
    uint32_t *pl1 = lds;  // A_one words
    uint32_t *pl5 = lds + pw;  // A_five words
    const uint32_t base5 = 4 * pw;  // LDS byte address of A_five
    const uint32_t nbits_full = 32u * pw;  // bits per plane of a whole tile
    TileShared &sh = *reinterpret_cast<TileShared *>(lds + 2 * pw);
    const uint64_t nvisit = a.job->nvisit;
    const uint32_t nranges = a.job->nranges;
    if ((uint32_t)(size_t)(__attribute__((address_space(3))) void *)lds != 0) {
        // Marks assume the planes at LDS address 0; report and do nothing.
        if (tid == 0 && blockIdx.x == 0)
            atomicOr(&a.counters[kErrorFlag], 1ull);
        return;
    }
    for (uint32_t w = tid; w < 2 * pw; w += NT)
        lds[w] = 0;

    for (;;) {
        if (tid == 0) {
            const unsigned long long t = atomicAdd(&a.counters[kTileCounter], 1ull);
            sh.ok = 0;
            if (t < nvisit) {
                // t is a visit position: the last visit entry starting at or
                // before it names the range (entries of empty ranges share
                // their successor's start, so the last one has units).
                uint32_t lo = 0, hi = nranges;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (a.visit[mid].vstart <= t)
                        lo = mid;
                    else
                        hi = mid;
                }
                const uint32_t r = a.visit[lo].range;
                const RangeDesc &d = a.ranges[r];
                const uint64_t u = t - a.visit[lo].vstart;
                uint32_t k0, k1, part = 0;
                if (d.nparts > 1) {
                    // unit u of a split range: tile u / nparts, part u mod nparts
                    k0 = (uint32_t)(u / d.nparts);
                    part = (uint32_t)(u - (uint64_t)k0 * d.nparts);
                    k1 = k0 + 1;
                } else {
                    k0 = (uint32_t)u * d.strip;
                    k1 = d.ntiles - k0 < d.strip ? d.ntiles : k0 + d.strip;
                }
                sh.range = r;
                sh.k0 = k0;
                sh.k1 = k1;
                sh.part = part;
                sh.ok = 1;
            }
        }
        if (tid < 64)
            sh.chunk[tid] = 0;
        __syncthreads();
        if (!sh.ok) {
#ifdef SIEVE_MARK_COUNT
            if (a.tally)
                tally_flush(tally, a.tally);
#endif
            break;
        }
        const uint32_t rix = sh.range;
        const RangeDesc &d = a.ranges[rix];
        const uint32_t k0 = sh.k0, k1 = sh.k1, part = sh.part;
        const bool split = d.nparts > 1;
        // Primes after the split items that this unit's per-tile loop takes:
        // up to the bucket sieve's first prime; part 0 of a split tile takes
        // the first part_primes of them (the later parts take the rest).
        const uint32_t kcap = d.nact < d.kbig ? d.nact : d.kbig;
        uint32_t n_rest = kcap > a.k_split ? kcap - a.k_split : 0;
        if (split && n_rest > d.part_primes)
            n_rest = d.part_primes;
        const uint32_t kr0 = a.k_split;
        const uint32_t kr1 = kr0 + (n_rest < (uint32_t)(K * NT) ? n_rest : (uint32_t)(K * NT));
        uint32_t id1[K];  // carried next A_one hit of primes kr0 + tid + j NT

        for (uint32_t k = k0; k < k1; ++k) {
            const uint64_t t = d.tile0 + k;  // storage index of the tile
            const bool first = (k == 0);
            const bool last = (k + 1 == d.ntiles);
            const uint32_t nwords = last ? d.last_words : pw;
            const uint64_t B = d.base + (uint64_t)k * kValsPerWord * pw;  // tile value base, multiple of 6
            const uint64_t tend = B + kValsPerWord * nwords;
            const uint32_t nbits = nwords * 32;
            // Primes p with p * p < tile end (Sec. 4: only primes up to the
            // square root sieve anything); pidx over-counts by the few primes
            // in the last 64-wide step, which mark nothing.  Every thread
            // takes these tile values itself (they are uniform).
            const uint64_t se = isqrt_dev(tend - 1);
            const uint64_t sb = isqrt_dev(B);
            const uint32_t sqe = se > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)se;
            const uint32_t sqb = sb > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)sb;
            uint64_t ps = (se + 63) / 64;
            if (ps >= a.pidx_len)
                ps = a.pidx_len - 1;
            const uint32_t nact_t = a.pidx[ps];

            if (part == 0) {
                // ---- presieve: OR of the repeating composite patterns ---------
                {
                    // Every group is always applied; a disabled group has an all-zero
                    // table, so the loop has no data-dependent branches.
                    const uint64_t b6 = B / 6;
                    uint32_t o[kMaxGroups];
#pragma unroll
                    for (int g = 0; g < kMaxGroups; ++g)
                        o[g] = (uint32_t)((b6 % a.groups[g].period + 32ull * tid) % a.groups[g].period);
                    for (uint32_t w = tid; w < nwords; w += NT) {
                        uint2 x[kMaxGroups], y[kMaxGroups];
#pragma unroll
                        for (int g = 0; g < kMaxGroups; ++g) {
                            const uint2 *tb = a.ps_tab + a.groups[g].offset + (o[g] >> 5);
                            x[g] = tb[0];
                            y[g] = tb[1];
                        }
                        uint2 c = make_uint2(0, 0);
#pragma unroll
                        for (int g = 0; g < kMaxGroups; ++g) {
                            const uint32_t sft = o[g] & 31;
                            c.x |= __builtin_amdgcn_alignbit(y[g].x, x[g].x, sft);
                            c.y |= __builtin_amdgcn_alignbit(y[g].y, x[g].y, sft);
                            o[g] += a.groups[g].step;
                            o[g] = o[g] >= a.groups[g].period ? o[g] - a.groups[g].period : o[g];
                        }
                        lds_or(4u * w, c.x);
                        lds_or(base5 + 4u * w, c.y);
                    }
                }

                // ---- marking: Table 1 starts, stride P in each plane -------------
                {
                    // Primes from d.kbig on come from this tile's bucket instead.
                    const uint32_t n_act = nact_t < d.kbig ? nact_t : d.kbig;
                    const uint32_t ks = n_act < a.k_split ? n_act : a.k_split;
                    const uint32_t n_items = ks > a.first_mark ? a.item_prefix[ks - a.first_mark] : 0;
                    const uint32_t kd = n_act < a.k_dense ? n_act : a.k_dense;
                    const uint32_t n_dense = kd > a.first_mark ? a.item_prefix[kd - a.first_mark] : 0;
                    // primes past the registers' share start afresh in this tile
                    const uint32_t kf1 = n_act < kr0 + n_rest ? n_act : kr0 + n_rest;
                    const uint32_t n_fresh = kf1 > kr1 ? kf1 - kr1 : 0;
                    const uint32_t n_work = n_items + n_fresh;
                    // Every active prime is below 2^31 when the tile ends below 2^62.
                    const bool narrow = tend <= (1ull << 62);
                    const uint32_t b5 = (uint32_t)(B % 5);
                    const uint64_t Bm1 = B - 1;
                    const uint32_t B32 = (uint32_t)B;
                    // Plane A_five is addressed as bits [32 pw, 32 pw + nbits) of one
                    // array that starts with A_one, so a mark needs no base add.
                    const uint32_t off5 = 32u * pw;
                    // Two work units per thread per pass, their loads issued
                    // together (an item, then its prime's constants).
                    constexpr uint32_t kQ = 2;
                    for (uint32_t vb = tid; vb < n_work; vb += kQ * NT) {
                        uint32_t kps[kQ], js[kQ], gs[kQ];
#pragma unroll
                        for (uint32_t q = 0; q < kQ; ++q) {
                            const uint32_t v = vb + q * NT;
                            if (v < n_items) {
                                const uint2 it = a.items[v];
                                kps[q] = it.x;
                                js[q] = it.y >> 16;
                                gs[q] = it.y & 0xFFFFu;
                            } else {
                                kps[q] = kr1 + (v - n_items);
                                js[q] = 0;
                                gs[q] = 1;
                            }
                        }
                        PrimeConst pcs[kQ];
#pragma unroll
                        for (uint32_t q = 0; q < kQ; ++q)
                            if (vb + q * NT < n_work)
                                pcs[q] = a.prm[kps[q]];
#pragma unroll
                        for (uint32_t q = 0; q < kQ; ++q) {
                            const uint32_t v = vb + q * NT;
                            const PrimeConst &pc = pcs[q];
                            if (v >= n_work || pc.p > sqe)
                                continue;  // past the work, or P * P >= tile end: nothing to mark
                            const uint32_t j = js[q], g = gs[q];
                            uint32_t id1t, id5t;
                            uint32_t step, off;
                            if (U24) {
                                tile_start_u24(pc, sqb, Bm1, B32, narrow, id1t, id5t);
                                step = __umul24(g, pc.p & 0xFFFFFFu);  // g, j < 2^16
                                off = __umul24(j, pc.p & 0xFFFFFFu);
                            } else {
                                tile_start(pc, sqb, Bm1, B32, narrow, id1t, id5t);
                                step = g * pc.p;
                                off = j * pc.p;
                            }
                            if (id1t + off < nbits)
                                tally.check(B, id1t + off, 1, pc.p);
                            if (id5t + off < nbits)
                                tally.check(B, id5t + off, 5, pc.p);
                            if (v < n_dense && a.skip5 != 1 && a.skip5 != 3) {
                                // g is a multiple of 32: fixed-mask marking
                                mark_plane_fixed(id1t + off, step, nbits, tally);
                                mark_plane_fixed(id5t + off + off5, step, nbits + off5, tally);
                            } else if (v < n_dense) {
                                // fixed-mask marking without the multiples of 5
                                // (g is a multiple of 32 and prime to 5)
                                const uint32_t inv5 = pc.r >> 29;
                                const uint32_t ginv = inv_mod5(g);
                                const uint32_t c1 = (cofactor_mod5(b5, id1t, 1, inv5) + j) % 5u;
                                const uint32_t c5 = (cofactor_mod5(b5, id5t, 0, inv5) + j) % 5u;
                                mark_plane_fixed_skip5(id1t + off, step, nbits, ((5u - c1) * ginv) % 5u, tally);
                                mark_plane_fixed_skip5(id5t + off + off5, step, nbits + off5, ((5u - c5) * ginv) % 5u,
                                                       tally);
                            } else if (a.skip5 == 1 || (a.skip5 >= 2 && v < n_items)) {
                                // hit n of this lane has cofactor m0 + 6(j + n g) = c + n g (mod 5);
                                // it is a multiple of 5 when n = -c / g (mod 5)
                                const uint32_t inv5 = pc.r >> 29;
                                const uint32_t ginv = inv_mod5(g);
                                const uint32_t c1 = (cofactor_mod5(b5, id1t, 1, inv5) + j) % 5u;
                                const uint32_t c5 = (cofactor_mod5(b5, id5t, 0, inv5) + j) % 5u;
                                mark_plane_skip5(0, id1t + off, step, nbits, ((5u - c1) * ginv) % 5u, tally);
                                mark_plane_skip5(0, id5t + off + off5, step, nbits + off5, ((5u - c5) * ginv) % 5u,
                                                 tally);
                            } else {
                                (void)mark_run(id1t + off, step, nbits, tally);
                                (void)mark_run(id5t + off + off5, step, nbits + off5, tally);
                            }
                        }
                    }
                    // Register-carried primes kr0 + tid + j NT: their starts are
                    // taken once, in the strip's first tile; afterwards each
                    // continues from its last hit, shifted by one tile.
                    {
                        const bool init = k == k0;
                        // The slot index is opaque per tile, so that the compiler
                        // does not hoist the K slots' addresses out of the tile
                        // loop (they would stay live in 4 K registers).
                        uint32_t kb = kr0 + tid;
                        asm volatile("" : "+v"(kb));
                        uint2 pn = kb < kr1 ? a.prd[kb] : make_uint2(0, 0);
#pragma unroll
                        for (int jj = 0; jj < K; ++jj) {
                            const uint32_t kp = kb + (uint32_t)jj * NT;
                            const uint32_t p = pn.x, dlt = pn.y;
                            const uint32_t kn = kp + NT;
                            if (jj + 1 < K)
                                pn = kn < kr1 ? a.prd[kn] : make_uint2(0, 0);
                            uint32_t x1 = id1[jj];
                            if (init) {
                                x1 = 0xFFFFFFFFu;
                                if (kp < kr1)
                                    x1 = strip_start<U24>(a.prm[kp], sqb, sqe, B, narrow);
                            }
                            // (p = 0 past kr1: the index there stays saturated, no mark)
                            if (p <= sqb) {
                                // square before the tile: x1 < P; (x1 + dlt) mod P
                                // without overflowing 32 bits
                                const uint32_t x5 = x1 >= p - dlt ? x1 - (p - dlt) : x1 + dlt;
                                if (x5 < nbits) {
                                    tally.check(B, x5, 5, p);
                                    (void)mark_run(x5 + off5, p, nbits + off5, tally);
                                }
                                if (x1 < nbits) {
                                    tally.check(B, x1, 1, p);
                                    x1 = mark_run(x1, p, nbits, tally);
                                }
                            } else if (x1 < nbits) {
                                // the square lies in this tile: both progressions start there
                                tally.check(B, x1, 1, p);
                                if (x1 + dlt < nbits)
                                    tally.check(B, x1 + dlt, 5, p);
                                (void)mark_run(x1 + dlt + off5, p, nbits + off5, tally);
                                x1 = mark_run(x1, p, nbits, tally);
                            }
                            id1[jj] = x1 - nbits_full;
                        }
                    }
                    // Bucket entries of this tile: one mark each (entries past
                    // the last tile's words mark nothing of the range).
                    if (d.kbig < d.nact) {
                        const bool est = a.job->bmode == 1;
                        const uint64_t e0 = est ? d.bbase + (uint64_t)k * d.bcap : a.boff[t];
                        uint64_t ne = est ? a.bcursor[t] : a.bcount[t];
                        if (est && ne > d.bcap)
                            ne = d.bcap;  // overflowed slice: the job is run again exactly
                        for (uint64_t e = tid; e < ne; e += NT) {
                            const uint32_t v = a.bdata[e0 + e];
                            const uint32_t bit = v & 0x7FFFFFFFu;
                            if (bit < nbits)
                                lds_or(((bit >> 3) & ~3u) + ((v >> 31) ? base5 : 0u), 1u << (bit & 31), tally);
                        }
                    }
                }
                __syncthreads();

            } else {
                // ---- a later part of a split tile: primes k_split + [part C,
                // (part + 1) C) with C = d.part_primes, marked straight into the
                // tile's global planes (they are large: few hits each).  This
                // workgroup's own planes stay zero.
                const uint32_t n_act = nact_t < d.kbig ? nact_t : d.kbig;
                const uint32_t n_rest_t = n_act > a.k_split ? n_act - a.k_split : 0;
                const uint32_t C = d.part_primes;
                const uint32_t r0 = part * C;
                const uint32_t r1 = n_rest_t < r0 + C ? n_rest_t : r0 + C;
                const bool narrow = tend <= (1ull << 62);
                const uint64_t Bm1 = B - 1;
                const uint32_t B32 = (uint32_t)B;
                uint32_t *const g1 = a.gbm + ((uint64_t)d.gtile0 + k) * 2 * pw;
                uint32_t *const g5 = g1 + pw;
                // Four primes per thread per pass, their constants loaded
                // together: the table of a high tile lies beyond L2, so the
                // loads' latency, not the arithmetic, bounds this loop.
                constexpr uint32_t kQ = 4;
                for (uint32_t rb = r0 + tid; rb < r1; rb += kQ * NT) {
                    PrimeConst pcs[kQ];
#pragma unroll
                    for (uint32_t q = 0; q < kQ; ++q)
                        if (rb + q * NT < r1)
                            pcs[q] = a.prm[a.k_split + rb + q * NT];
#pragma unroll
                    for (uint32_t q = 0; q < kQ; ++q) {
                        const PrimeConst &pc = pcs[q];
                        if (rb + q * NT >= r1 || pc.p > sqe)
                            continue;  // past the part, or P * P >= tile end
                        uint32_t id1t, id5t;
                        if (U24)
                            tile_start_u24(pc, sqb, Bm1, B32, narrow, id1t, id5t);
                        else
                            tile_start(pc, sqb, Bm1, B32, narrow, id1t, id5t);
                        // i < nbits < 2^20 and P < 2^32 - 2^20: i + P does not wrap
                        if (id1t < nbits)
                            tally.check(B, id1t, 1, pc.p);
                        if (id5t < nbits)
                            tally.check(B, id5t, 5, pc.p);
                        (void)tally.run(id1t, pc.p, nbits);
                        (void)tally.run(id5t, pc.p, nbits);
                        for (uint32_t i = id1t; i < nbits; i += pc.p) {
                            tally.op();
                            atomicOr(&g1[i >> 5], 1u << (i & 31));
                        }
                        for (uint32_t i = id5t; i < nbits; i += pc.p) {
                            tally.op();
                            atomicOr(&g5[i >> 5], 1u << (i & 31));
                        }
                    }
                }
            }

            // ---- split tiles: the parts meet in the global planes; the
            // workgroup that finishes the last part counts or lists the tile
            if (split) {
                uint32_t *const g1 = a.gbm + ((uint64_t)d.gtile0 + k) * 2 * pw;
                if (part == 0)
                    for (uint32_t w = tid; w < nwords; w += NT) {
                        const uint32_t c1 = pl1[w], c5 = pl5[w];
                        if (c1)
                            atomicOr(&g1[w], c1);
                        if (c5)
                            atomicOr(&g1[pw + w], c5);
                        pl1[w] = 0;
                        pl5[w] = 0;
                    }
                __threadfence();  // this workgroup's marks are done before it arrives
                __syncthreads();
                if (tid == 0)
                    sh.last = atomicAdd(&a.garrive[(uint64_t)d.gtile0 + k], 1u) + 1u == d.nparts ? 1u : 0u;
                __syncthreads();
                if (sh.last == 0) {
                    __syncthreads();
                    continue;  // another part's workgroup finishes the tile
                }
                __threadfence();
                for (uint32_t w = tid; w < nwords; w += NT) {
                    pl1[w] = __hip_atomic_load(&g1[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    pl5[w] = __hip_atomic_load(&g1[pw + w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __syncthreads();
            }

            // ---- edges, then count or bitmap; every word read is cleared ------
            uint32_t head1 = 0, head5 = 0, tail1 = 0, tail5 = 0;
            if (first) {
                if (B + 1 < d.lo || B == 0)
                    head1 = 1;  // below lo, or the value 1
                if (B + 5 < d.lo)
                    head5 = 1;
            }
            if (last) {
                const uint64_t base_i = 32ull * (nwords - 1);
                const uint64_t n1 = d.hi > B + 1 ? (d.hi - B - 1 + 5) / 6 : 0;
                const uint64_t n5 = d.hi > B + 5 ? (d.hi - B - 5 + 5) / 6 : 0;
                const uint64_t r1 = n1 > base_i ? n1 - base_i : 0;
                const uint64_t r5 = n5 > base_i ? n5 - base_i : 0;
                tail1 = r1 >= 32 ? 0u : (~0u << r1);
                tail5 = r5 >= 32 ? 0u : (~0u << r5);
            }
            const bool list = d.mode != 0;
            const uint32_t nw_pad = list ? ((nwords + kChunkWords - 1) / kChunkWords) * kChunkWords : nwords;
            const uint64_t wbase = list ? (d.chunk0 + k * (pw / kChunkWords)) * kChunkWords : 0;
            uint32_t cnt = 0;
            for (uint32_t w = tid; w < nw_pad; w += NT) {
                uint32_t p1 = 0, p5 = 0;
                if (w < nwords) {
                    uint32_t c1 = pl1[w], c5 = pl5[w];
                    pl1[w] = 0;
                    pl5[w] = 0;
                    if (w == 0 && B < 74) {
                        // The presieved primes themselves (5..73) lie in word 0
                        // of any tile based below 74: the patterns marked them.
                        c1 &= ~(a.restore1 >> (B / 6));
                        c5 &= ~(a.restore5 >> (B / 6));
                    }
                    if (w == 0) {
                        c1 |= head1;
                        c5 |= head5;
                    }
                    if (w == nwords - 1) {
                        c1 |= tail1;
                        c5 |= tail5;
                    }
                    p1 = ~c1;
                    p5 = ~c5;
                }
                const uint32_t c = __popc(p1) + __popc(p5);
                if (list) {
                    a.bitmap[wbase + w] = spread32(p1) | (spread32(p5) << 1);
                    const uint32_t ws = wave_sum(c);
                    if (lane == 0)
                        atomicAdd(&sh.chunk[w / kChunkWords], ws);
                } else {
                    cnt += c;
                }
            }
            if (list) {
                __syncthreads();
                const uint32_t nch = nw_pad / kChunkWords;
                const uint64_t cbase = d.chunk0 + k * (pw / kChunkWords);
                if (tid < nch) {
                    a.chunk_counts[cbase + tid] = sh.chunk[tid];
                    sh.chunk[tid] = 0;  // for the strip's next tile
                }
            } else {
                cnt = wave_sum(cnt);
                if (lane == 0)
                    sh.red[wave] = cnt;
                __syncthreads();
                if (tid == 0) {
                    uint32_t tot = 0;
                    for (uint32_t i = 0; i < NT / kWave; ++i)
                        tot += sh.red[i];
                    atomicAdd(&a.counts[rix], (unsigned long long)tot);
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Bucket sieve.  For a range of several tiles, a prime far above the plane
// length hits a given tile with small probability, so instead of a Table 1
// start per (tile, prime) it gets one start per range and its hits are
// walked tile by tile: each hit advances by (P div nbits) tiles and
// (P mod nbits) bits.  Hits are binned per tile in LDS windows of
// kBucketWindow tiles.  Two layouts:
//  - estimated (PASS 2): every tile of a range has a slice sized from the
//    expected hit count plus a wide margin; the fill pass reserves with one
//    global atomic per (workgroup, tile) and flags a slice that would
//    overflow (the job is then run again with the exact layout);
//  - exact: the count pass (PASS 0) adds the per-tile totals, a scan gives
//    offsets, and the fill pass (PASS 1) writes into them.
// Entries are bit | plane << 31.
// ---------------------------------------------------------------------------
namespace {

struct HitWalk {
    uint32_t t1, b1, t5, b5;  // next hit (tile, bit) per plane; t >= the window's end when done
    uint32_t qp, rp;          // P div nbits, P mod nbits
    uint32_t c1, c5;          // residue mod 5 of the next hit's cofactor (5: not tracked)
};

// Next hit of one plane: P indices further, i.e. 6P in value, so the
// cofactor grows by 6 = 1 (mod 5).
__device__ inline void walk_step(uint32_t &t, uint32_t &b, uint32_t &c, const HitWalk &w, uint32_t nbits)
{
    b += w.rp;
    t += w.qp;
    if (b >= nbits) {
        b -= nbits;
        t += 1;
    }
    // c -> c + 1 mod 5, and 5 stays 5: a nibble table indexed by c, without
    // branches (0..5 -> 1, 2, 3, 4, 0, 5)
    c = (0x504321u >> (c << 2)) & 0xFu;
}

// Wide windows: the first hits of prime P (below 2^32) in plane order at or
// past the window offset x0 (a multiple of 6; the value W + x0), as indices
// from x0, and that value mod 5.  With P * P at or before W + x0 the first
// value is W + x0 itself: rem = (W + x0 - 1) mod P from the 128-bit W - 1 by
// 32-bit limbs, and Table 1 in 64-bit arithmetic (the packed R of a prime
// above 3.2e9 and the 32-bit start formula do not hold there).  Otherwise
// P * P lies in the window at offset x2 = P * P - W: its A_one index from x0
// is (x2 - x0 - 1) / 6 and A_five follows by P (P + 4) or P (P + 2).
__device__ inline bool wide_first_hits(const BucketArgs &a, uint32_t P, uint64_t m, uint64_t x0, uint64_t xend,
                                       uint64_t &id1, uint64_t &id5)
{
    const uint64_t P2 = (uint64_t)P * P;
    const uint64_t blo = a.wlo + x0;
    const uint64_t bhi = a.whi + (blo < x0 ? 1u : 0u);  // W + x0, 128-bit
    if (bhi != 0 || P2 <= blo) {
        uint64_t r = mod_invariant(a.wm1_hi, P, m, false);
        r = mod_invariant((r << 32) | (a.wm1_lo >> 32), P, m, false);
        r = mod_invariant((r << 32) | (a.wm1_lo & 0xFFFFFFFFull), P, m, false);
        r += mod_invariant(x0, P, m, false);
        const uint64_t rem = r >= P ? r - P : r;  // (W + x0 - 1) mod P
        const uint64_t R = P / 6u;
        const bool p5 = P - 6u * (uint32_t)R == 5u;
        const uint64_t dp = 6 * R + 5 - rem;
        const uint64_t i0 = dp / 6;
        const uint32_t q = (uint32_t)(dp - 6 * i0);
        const uint32_t e1 = (uint32_t)((p5 ? kTable1_id1_p5 : kTable1_id1_p1) >> (8u * q));
        const uint32_t e5 = (uint32_t)((p5 ? kTable1_id5_p5 : kTable1_id5_p1) >> (8u * q));
        id1 = i0 + (e1 & 7u) * R + ((e1 >> 3) & 7u) - 1u;
        id5 = i0 + (e5 & 7u) * R + ((e5 >> 3) & 7u) - 1u;
        return true;
    }
    const uint64_t x2 = P2 - a.wlo;  // P * P - W, with W below 2^64 here
    if (x2 >= xend)
        return false;
    id1 = (x2 - x0 - 1) / 6;
    id5 = id1 + (P % 6u == 1u ? 2ull * (P - 1) / 3 : (P - 2ull) / 3);
    return true;
}

// First hits of prime k at or past tile w0 of range d, as tile indices
// relative to the range's tile 0 (a first hit past wend keeps its true tile
// on the 64-bit path; the wide path caps it at wend).  t = wend for a
// prime that is not active there (k >= nact, or its square past wend).
template <bool WIDE>
__device__ inline HitWalk walk_init(const BucketArgs &a, const RangeDesc &d, uint32_t k, uint32_t w0,
                                    uint32_t wend)
{
    HitWalk w;
    w.t1 = w.t5 = wend;
    w.b1 = w.b5 = 0;
    w.qp = w.rp = 0;
    w.c1 = w.c5 = 5;
    if (k >= d.nact)
        return w;
    if constexpr (WIDE) {
        const PrimeConst pc = a.prm[k];
        const uint32_t P = pc.p;
        const uint64_t x0 = (uint64_t)w0 * a.span, xend = (uint64_t)wend * a.span;
        uint64_t id1, id5;
        if (!wide_first_hits(a, P, prime_recip(pc), x0, xend, id1, id5))
            return w;
        // tiles from w0 (the square case's indices count from x0 as well)
        if (a.skip5) {
            const uint32_t b5 = (uint32_t)((a.w5 + x0 % 5u) % 5u);
            const uint32_t inv5 = inv_mod5(P % 5u);
            w.c1 = ((b5 + (uint32_t)(id1 % 5u) + 1u) * inv5) % 5u;
            w.c5 = ((b5 + (uint32_t)(id5 % 5u)) * inv5) % 5u;
        }
        w.qp = P / a.nbits;
        w.rp = P - w.qp * a.nbits;
        const uint64_t t1 = w0 + id1 / a.nbits, t5 = w0 + id5 / a.nbits;
        w.t1 = t1 < wend ? (uint32_t)t1 : wend;
        w.b1 = (uint32_t)(id1 % a.nbits);
        w.t5 = t5 < wend ? (uint32_t)t5 : wend;
        w.b5 = (uint32_t)(id5 % a.nbits);
        return w;
    }
    const PrimeConst pc = a.prm[k];
    const uint64_t P = pc.p;
    const uint64_t P2 = P * P;
    const uint64_t wbase = d.base + (uint64_t)w0 * a.span;  // uniform
    const uint64_t rend = d.base + (uint64_t)wend * a.span;
    const uint32_t R = pc.r & 0x1FFFFFFFu, inv5 = pc.r >> 29;
    uint32_t id1, id5, bt5;
    uint64_t tM;
    if (P2 <= wbase) {
        // The usual case: the first value is the window base itself, so the
        // walk starts in tile w0 with rem = (wbase - 1) mod P.
        const uint64_t x = wbase - 1;
        const uint32_t rem = rend <= (1ull << 62)
                                 ? mod_narrow((uint32_t)x, (uint32_t)(x >> 32), pc.p, pc.m_lo, pc.m_hi & ~kP5Flag)
                                 : mod_invariant(x, pc.p, prime_recip(pc), false);
        wheel_start(pc.p, R, wbase, wbase, rem, id1, id5);
        tM = w0;
        bt5 = (uint32_t)(wbase % 5);
    } else {
        // P^2 lies beyond the window base: its tile, by the reciprocal of the
        // tile span, and rem = (P^2 - 1) mod P = P - 1.
        if (P2 >= rend)
            return w;
        const uint64_t x = P2 - d.base;
        tM = mulhi64(x, a.span_rcp);
        if (x - tM * a.span >= a.span)
            ++tM;
        const uint64_t Bt = d.base + tM * a.span;
        wheel_start(pc.p, R, Bt, P2, pc.p - 1u, id1, id5);
        bt5 = (uint32_t)(Bt % 5);
    }
    if (a.skip5) {
        w.c1 = cofactor_mod5(bt5, id1, 1, inv5);
        w.c5 = cofactor_mod5(bt5, id5, 0, inv5);
    }
    w.qp = pc.p / a.nbits;
    w.rp = pc.p - w.qp * a.nbits;
    // The true tiles, also past wend: where a walk ends is kept for the
    // range's next piece.
    const uint64_t t1 = tM + id1 / a.nbits, t5 = tM + id5 / a.nbits;
    w.t1 = t1 < 0xFFFFFFFFull ? (uint32_t)t1 : 0xFFFFFFFFu;
    w.b1 = id1 % a.nbits;
    w.t5 = t5 < 0xFFFFFFFFull ? (uint32_t)t5 : 0xFFFFFFFFu;
    w.b5 = id5 % a.nbits;
    return w;
}

// A walk resumed from the state a previous piece of the range left.
__device__ inline HitWalk walk_resume(const WalkState &st, uint32_t P, uint32_t nbits)
{
    HitWalk w;
    w.t1 = st.t1;
    w.b1 = st.bc1 & 0x0FFFFFFFu;
    w.c1 = st.bc1 >> 28;
    w.t5 = st.t5;
    w.b5 = st.bc5 & 0x0FFFFFFFu;
    w.c5 = st.bc5 >> 28;
    w.qp = P / nbits;
    w.rp = P - w.qp * nbits;
    return w;
}

// Where a finished walk goes on: the tiles relative to the one after wend.
__device__ inline WalkState walk_state(const HitWalk &w, uint32_t wend)
{
    WalkState st;
    st.t1 = w.t1 - wend;
    st.bc1 = w.b1 | (w.c1 << 28);
    st.t5 = w.t5 - wend;
    st.bc5 = w.b5 | (w.c5 << 28);
    return st;
}

// Range of unit u: the last range whose first unit is <= u.  Searches from
// range r0, which must satisfy ranges[r0].bunit0 <= u: exponential steps,
// then bisection of the bracket.
__device__ inline uint32_t find_unit_range(const RangeDesc *ranges, uint32_t nranges, uint32_t r0, uint64_t u)
{
    uint32_t lo = r0, step = 1;
    while (lo + step < nranges && ranges[lo + step].bunit0 <= u) {
        lo += step;
        step <<= 1;
    }
    uint32_t hi = lo + step < nranges ? lo + step : nranges;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ranges[mid].bunit0 <= u)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

}  // namespace

// LDS (dynamic, a.win bins): fill passes hold the 64-bit slice base of
// every tile of the window, then the per-tile counts, which the fill walk
// reuses as slot cursors, then kBucketKeep hits per thread from the count
// walk (window tile << 21 | plane << 20 | bit: the window has at most 2^11
// tiles and a plane at most 2^20 bits), which the fill replays instead of
// walking again when the thread had no more hits than that.
static_assert(kBucketWindow <= (1u << 11), "kept hits hold the window tile in 11 bits");

template <int PASS, bool WIDE>
__global__ void __launch_bounds__(kBucketThreads) k_bucket(BucketArgs a)
{
    extern __shared__ unsigned long long s_bucket[];
    unsigned long long *s_base = s_bucket;
    uint32_t *s_cnt = (uint32_t *)(s_bucket + (PASS ? a.win : 0));
    uint32_t *s_keep = s_cnt + a.win;  // fill passes: kBucketKeep x kBucketThreads
    const uint32_t tid = threadIdx.x;
    const uint64_t nunits = a.job->nunits;
    const uint32_t nranges = a.job->nranges;
    const uint32_t nbits = a.nbits;
    MarkTally tally;

    // Walk links (serving pieces of one long range), read once per launch.
    const WalkLink *const links = (!WIDE && a.job->links != 0) ? a.links : nullptr;

    uint32_t r = 0;
    uint64_t r_end = 0;  // one past the last unit of range r
    for (uint64_t u = blockIdx.x; u < nunits; u += gridDim.x) {
        if (u >= r_end) {
            r = find_unit_range(a.ranges, nranges, r, u);
            r_end = a.ranges[r].bunit0 + a.ranges[r].bunits;
        }
        const RangeDesc &d = a.ranges[r];
        // unit = (prime block, tile window) of range r
        const uint32_t ur = (uint32_t)(u - d.bunit0);
        const uint32_t blk = ur / d.bwins, win = ur - blk * d.bwins;
        const uint32_t w0 = win * kBucketWindow;
        const uint32_t wend = (d.ntiles - w0) < kBucketWindow ? d.ntiles : w0 + kBucketWindow;
        const uint32_t k = d.kbig + blk * kBucketThreads + tid;
        // A range linked to its previous piece: the first window's walks of
        // the primes that piece left a state for resume from it.
        const WalkLink *const link = links ? &links[r] : nullptr;
        HitWalk w;
        if (link && w0 == 0 && link->src && k < d.nact && k - d.kbig < link->nsrc)
            w = walk_resume(link->src[k - d.kbig], a.prm[k].p, nbits);
        else
            w = walk_init<WIDE>(a, d, k, w0, wend);
#ifdef SIEVE_MARK_COUNT
        // hits past the range's last plane word are binned but never applied
        const uint32_t lastbits = 32u * d.last_words;
        auto covered = [&](uint32_t tt, uint32_t bb) { return tt + 1 < d.ntiles || bb < lastbits; };
        if (PASS != 0 && k < d.nact) {
            const uint32_t P = a.prm[k].p;
            if (w.t1 < wend && covered(w.t1, w.b1))
                tally.check(d.base + (uint64_t)w.t1 * a.span, w.b1, 1, P);
            if (w.t5 < wend && covered(w.t5, w.b5))
                tally.check(d.base + (uint64_t)w.t5 * a.span, w.b5, 5, P);
        }
#endif
        for (uint32_t i = tid; i < wend - w0; i += kBucketThreads)
            s_cnt[i] = 0;
        __syncthreads();
        if (PASS == 0) {
            while (w.t1 < wend) {
                if (w.c1)
                    atomicAdd(&s_cnt[w.t1 - w0], 1u);
                walk_step(w.t1, w.b1, w.c1, w, nbits);
            }
            while (w.t5 < wend) {
                if (w.c5)
                    atomicAdd(&s_cnt[w.t5 - w0], 1u);
                walk_step(w.t5, w.b5, w.c5, w, nbits);
            }
            __syncthreads();
            for (uint32_t i = tid; i < wend - w0; i += kBucketThreads)
                if (s_cnt[i])
                    atomicAdd(&a.bcount[d.tile0 + w0 + i], s_cnt[i]);
        } else {
            uint32_t nk = 0;  // this thread's hits (the first kBucketKeep are kept)
            HitWalk c = w;    // count first, without moving the walk
            {
                while (c.t1 < wend) {
#ifdef SIEVE_MARK_COUNT
                    if (covered(c.t1, c.b1)) {
                        tally.hits++;
                        tally.skipped += c.c1 == 0;
                    }
#endif
                    if (c.c1) {
                        atomicAdd(&s_cnt[c.t1 - w0], 1u);
                        if (nk < kBucketKeep)
                            s_keep[nk * kBucketThreads + tid] = ((c.t1 - w0) << 21) | c.b1;
                        ++nk;
                    }
                    walk_step(c.t1, c.b1, c.c1, c, nbits);
                }
                while (c.t5 < wend) {
#ifdef SIEVE_MARK_COUNT
                    if (covered(c.t5, c.b5)) {
                        tally.hits++;
                        tally.skipped += c.c5 == 0;
                    }
#endif
                    if (c.c5) {
                        atomicAdd(&s_cnt[c.t5 - w0], 1u);
                        if (nk < kBucketKeep)
                            s_keep[nk * kBucketThreads + tid] = ((c.t5 - w0) << 21) | (1u << 20) | c.b5;
                        ++nk;
                    }
                    walk_step(c.t5, c.b5, c.c5, c, nbits);
                }
            }
            // The range's last window: the walk's end state for the next piece.
            if (link && link->dst && wend == d.ntiles && k < d.nact)
                link->dst[k - d.kbig] = walk_state(c, wend);
            __syncthreads();
            for (uint32_t i = tid; i < wend - w0; i += kBucketThreads) {
                const uint32_t n = s_cnt[i];
                s_cnt[i] = 0;  // now the slot cursor of tile i
                if (n) {
                    const uint64_t g = d.tile0 + w0 + i;
                    const uint32_t at = atomicAdd(&a.bcursor[g], n);
                    if (PASS == 1) {
                        s_base[i] = a.boff[g] + at;
                    } else if (at + n <= d.bcap) {
                        s_base[i] = d.bbase + (uint64_t)(w0 + i) * d.bcap + at;
                    } else {
                        s_base[i] = ~0ull;  // slice full: flag it, write nothing
                        atomicOr(&a.counters[kOverflowFlag], 1ull);
                    }
                }
            }
            __syncthreads();
            if (nk <= kBucketKeep) {
                // replay the kept hits
                for (uint32_t i = 0; i < nk; ++i) {
                    const uint32_t v = s_keep[i * kBucketThreads + tid];
                    const uint32_t tw = v >> 21;
                    const uint32_t slot = atomicAdd(&s_cnt[tw], 1u);
                    const unsigned long long b0 = s_base[tw];
                    if (b0 != ~0ull)
                        a.bdata[b0 + slot] = (v & 0xFFFFFu) | ((v << 11) & 0x80000000u);
                }
            } else {
                while (w.t1 < wend) {
                    if (w.c1) {
                        const uint32_t slot = atomicAdd(&s_cnt[w.t1 - w0], 1u);
                        const unsigned long long b0 = s_base[w.t1 - w0];
                        if (b0 != ~0ull)
                            a.bdata[b0 + slot] = w.b1;
                    }
                    walk_step(w.t1, w.b1, w.c1, w, nbits);
                }
                while (w.t5 < wend) {
                    if (w.c5) {
                        const uint32_t slot = atomicAdd(&s_cnt[w.t5 - w0], 1u);
                        const unsigned long long b0 = s_base[w.t5 - w0];
                        if (b0 != ~0ull)
                            a.bdata[b0 + slot] = w.b5 | 0x80000000u;
                    }
                    walk_step(w.t5, w.b5, w.c5, w, nbits);
                }
            }
        }
        __syncthreads();
    }
#ifdef SIEVE_MARK_COUNT
    if (PASS != 0 && a.tally)
        tally_flush(tally, a.tally);
#else
    (void)tally;
#endif
}

// Exclusive scan of the per-tile bucket counts (one workgroup); also clears
// the fill-pass cursors.
__global__ void __launch_bounds__(kFinalizeThreads) k_bucket_scan(BucketScanArgs a)
{
    __shared__ uint32_t s_w[kFinalizeThreads / kWave];
    __shared__ unsigned long long s_carry;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    const uint64_t n = a.job->ntiles;
    if (tid == 0)
        s_carry = 0;
    __syncthreads();
    for (uint64_t b0 = 0; b0 < n; b0 += kFinalizeThreads) {
        const uint64_t i = b0 + tid;
        const uint32_t c = i < n ? a.bcount[i] : 0u;
        const uint32_t incl = wave_incl_scan(c, lane);
        if (lane == kWave - 1)
            s_w[wave] = incl;
        __syncthreads();
        uint32_t woff = 0, btot = 0;
        for (uint32_t q = 0; q < kFinalizeThreads / kWave; ++q) {
            woff += q < wave ? s_w[q] : 0u;
            btot += s_w[q];
        }
        if (i < n) {
            a.boff[i] = s_carry + woff + incl - c;
            a.bcursor[i] = 0;
        }
        __syncthreads();
        if (tid == 0)
            s_carry += btot;
        __syncthreads();
    }
    if (tid == 0)
        a.boff[n] = s_carry;
}

// Range of scan segment `sg`: the first range whose segments end after it
// (count ranges hold no segment and never satisfy the test first).
__device__ inline uint32_t seg_range(const RangeDesc *ranges, uint32_t nranges, uint64_t sg)
{
    uint32_t lo = 0, hi = nranges;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)ranges[mid].seg0 + ranges[mid].nseg > sg)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Sum of the chunk counts of every scan segment (4 chunks per thread).
__global__ void __launch_bounds__(kFinalizeThreads) k_seg_sum(SegArgs a)
{
    __shared__ unsigned long long s_w[kFinalizeThreads / kWave];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    const uint64_t nseg = a.job->nseg;
    const uint32_t nranges = a.job->nranges;
    for (uint64_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const RangeDesc &d = a.ranges[seg_range(a.ranges, nranges, sg)];
        const uint64_t c0 = d.chunk0 + (sg - d.seg0) * kSegChunks;
        const uint64_t c1 = d.chunk0 + d.nchunks;
        unsigned long long v = 0;
#pragma unroll
        for (uint32_t q = 0; q < kSegChunks / kFinalizeThreads; ++q) {
            const uint64_t c = c0 + q * kFinalizeThreads + tid;
            v += c < c1 ? a.chunk_counts[c] : 0u;
        }
        for (int o = kWave / 2; o > 0; o >>= 1)
            v += __shfl_xor(v, o);
        if (lane == 0)
            s_w[wave] = v;
        __syncthreads();
        if (tid == 0) {
            unsigned long long t = 0;
            for (uint32_t q = 0; q < kFinalizeThreads / kWave; ++q)
                t += s_w[q];
            a.seg_sum[sg] = t;
        }
        __syncthreads();
    }
}

// Per range: the primes 2 and 3, the count and capacity status, and for list
// ranges the output base of each scan segment (an exclusive scan of the
// segment sums; ~0 for every segment of a range that does not fit).
__global__ void __launch_bounds__(kFinalizeThreads) k_finalize(FinalizeArgs a)
{
    __shared__ unsigned long long s_w[kFinalizeThreads / kWave];
    __shared__ unsigned long long s_carry;
    __shared__ uint32_t s_over;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    const uint32_t nranges = a.job->nranges;

    for (uint32_t r = blockIdx.x; r < nranges; r += gridDim.x) {
        const RangeDesc &d = a.ranges[r];
        // 2 and 3 lie outside the wheel (Sec. 2.1) and are reported when in
        // range (a wide window's bounds are offsets from a base above both).
        const bool abs_vals = a.job->wide == 0;
        const uint32_t has2 = (abs_vals && d.lo <= 2 && 2 < d.hi) ? 1u : 0u;
        const uint32_t has3 = (abs_vals && d.lo <= 3 && 3 < d.hi) ? 1u : 0u;
        const uint32_t sp = has2 + has3;
        if (d.mode == 0) {
            if (tid == 0) {
                a.counts[r] += sp;
                a.status[r] = 0;
            }
            continue;
        }
        if (tid == 0)
            s_carry = 0;
        __syncthreads();
        for (uint32_t b0 = 0; b0 < d.nseg; b0 += kFinalizeThreads) {
            const uint32_t i = b0 + tid;
            const unsigned long long v = i < d.nseg ? a.seg_sum[d.seg0 + i] : 0ull;
            // inclusive wave scan (64-bit)
            unsigned long long incl = v;
            for (uint32_t o = 1; o < kWave; o <<= 1) {
                const unsigned long long t = __shfl_up(incl, o);
                if (lane >= o)
                    incl += t;
            }
            if (lane == kWave - 1)
                s_w[wave] = incl;
            __syncthreads();
            unsigned long long woff = 0, btot = 0;
            for (uint32_t q = 0; q < kFinalizeThreads / kWave; ++q) {
                woff += q < wave ? s_w[q] : 0ull;
                btot += s_w[q];
            }
            if (i < d.nseg)
                a.seg_base[d.seg0 + i] = d.out_off + sp + s_carry + woff + incl - v;
            __syncthreads();
            if (tid == 0)
                s_carry += btot;
            __syncthreads();
        }
        if (tid == 0) {
            const unsigned long long total = s_carry + sp;
            a.counts[r] = total;
            s_over = total > d.cap ? 1u : 0u;
            if (total > d.cap) {
                a.status[r] = -3;  // SIEVE_E_CAPACITY
            } else {
                a.status[r] = 0;
                uint64_t pos = d.out_off;
                if (a.job->elem_bytes == 4) {
                    uint32_t *o = (uint32_t *)a.job->out;
                    if (has2)
                        o[pos++] = 2;
                    if (has3)
                        o[pos++] = 3;
                } else {
                    uint64_t *o = (uint64_t *)a.job->out;
                    if (has2)
                        o[pos++] = 2;
                    if (has3)
                        o[pos++] = 3;
                }
            }
        }
        __syncthreads();
        if (s_over)  // the compaction writes nothing for a range that does not fit
            for (uint32_t i = tid; i < d.nseg; i += kFinalizeThreads)
                a.seg_base[d.seg0 + i] = ~0ull;
        __syncthreads();
    }
}

// Output offset and value base of every chunk: the segment's base plus an
// exclusive scan of the chunk counts inside the segment (4 per thread).
__global__ void __launch_bounds__(kFinalizeThreads) k_seg_scan(SegArgs a)
{
    constexpr uint32_t kQ = kSegChunks / kFinalizeThreads;
    __shared__ uint32_t s_w[kFinalizeThreads / kWave];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    const uint64_t nseg = a.job->nseg;
    const uint32_t nranges = a.job->nranges;
    for (uint64_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const RangeDesc &d = a.ranges[seg_range(a.ranges, nranges, sg)];
        const uint64_t base = a.seg_base[sg];
        const uint64_t cs = d.chunk0 + (sg - d.seg0) * kSegChunks;  // segment's first chunk
        const uint64_t c1 = d.chunk0 + d.nchunks;
        const uint64_t cf = cs + (uint64_t)tid * kQ;  // this thread's first chunk
        uint32_t cnt[kQ];
        uint32_t tsum = 0;
#pragma unroll
        for (uint32_t q = 0; q < kQ; ++q) {
            cnt[q] = cf + q < c1 ? a.chunk_counts[cf + q] : 0u;
            tsum += cnt[q];
        }
        const uint32_t incl = wave_incl_scan(tsum, lane);
        if (lane == kWave - 1)
            s_w[wave] = incl;
        __syncthreads();
        uint32_t woff = 0;
        for (uint32_t q = 0; q < kFinalizeThreads / kWave; ++q)
            woff += q < wave ? s_w[q] : 0u;
        uint64_t run = woff + incl - tsum;  // primes before this thread's first chunk
#pragma unroll
        for (uint32_t q = 0; q < kQ; ++q) {
            const uint64_t c = cf + q;
            if (c < c1) {
                a.chunk_off[c] = base == ~0ull ? ~0ull : base + run;
                // chunk i of the range covers kChunkVals values from base + i kChunkVals
                a.chunk_vbase[c] = d.base + (uint64_t)kChunkVals * (c - d.chunk0);
            }
            run += cnt[q];
        }
        __syncthreads();
    }
}

// Workgroup barrier for LDS hand-offs only: waits for this wave's LDS
// operations, not for its global stores (a full __syncthreads also drains the
// stores, which would serialise the compaction on write latency).
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Hand-off of LDS data between lanes of one wavefront: its LDS operations
// complete, and the compiler moves no memory access across it.
__device__ __forceinline__ void wave_lds_fence()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Stores output element i for value offset v from the chunk bases: the
// value itself, or for 128-bit elements the window base plus v (one 16-byte
// store).
template <typename T>
__device__ __forceinline__ void put_out(__attribute__((address_space(1))) T *out, uint64_t i, uint64_t v,
                                        const CompactArgs &)
{
    out[i] = (T)v;
}

template <>
__device__ __forceinline__ void put_out<U128>(__attribute__((address_space(1))) U128 *out, uint64_t i, uint64_t v,
                                              const CompactArgs &a)
{
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    const uint64_t lo = a.wbase_lo + v;
    const uint64_t hi = a.wbase_hi + (lo < v ? 1u : 0u);
    ((__attribute__((address_space(1))) u64x2 *)out)[i] = u64x2{lo, hi};
}

template <typename T>
__global__ void __launch_bounds__(kCompactThreads) k_compact(CompactArgs a)
{
    constexpr uint32_t kW = kCompactThreads / kWave;
    constexpr uint32_t kU = 2;  // contiguous chunks per workgroup iteration
    // one staging window per wavefront: value offsets from the chunk's value
    // base (below kChunkVals, so 32 bits suffice for either element type)
    __shared__ uint32_t s_stage[kW][kStagePerWave];
    // per iteration parity: per-wave totals of each chunk, and each chunk's
    // output offset and value base
    __shared__ uint32_t s_wt[2][kU][kW];
    __shared__ unsigned long long s_meta[2][2][kU];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    if (a.job->elem_bytes != (int32_t)sizeof(T))
        return;
    const uint64_t nchunks = a.job->nchunks;
    // The output pointer, uniform and in the global address space, so that
    // the stores are global (not flat) stores.  (readfirstlane returns a
    // signed int: each half goes through uint32_t so that widening never
    // sign-extends.)
    const uint64_t op = (uint64_t)(size_t)a.job->out;
    const uint32_t op_hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(op >> 32));
    const uint32_t op_lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)op);
    __attribute__((address_space(1))) T *const out =
        (__attribute__((address_space(1))) T *)(size_t)(((uint64_t)op_hi << 32) | op_lo);

    // Each iteration takes kU contiguous chunks.  Their loads are issued
    // together at the top; the stores of all kU chunks stay in flight until
    // the next iteration's loads are waited for.  The wavefront scans of all
    // kU chunks come first and one workgroup barrier then publishes every
    // per-wave total; staging and storing touch only the wave's own window.
    // The totals and the chunk metadata alternate between two buffers by
    // iteration: a buffer is written again two iterations later, after the
    // barrier of the iteration in between, which every wave reaches only
    // after it has read that buffer.
    uint32_t ip = 0;
    for (uint64_t c0 = (uint64_t)blockIdx.x * kU; c0 < nchunks; c0 += (uint64_t)gridDim.x * kU, ip ^= 1u) {
        uint64_t mu[kU];
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u)
            mu[u] = c0 + u < nchunks ? a.bitmap[(c0 + u) * kChunkWords + tid] : 0ull;
        if (tid < kU) {
            const uint64_t c = c0 + tid;
            // ~0: past the end, or the range does not fit (nothing is written)
            s_meta[ip][0][tid] = c < nchunks ? a.chunk_off[c] : ~0ull;
            s_meta[ip][1][tid] = c < nchunks ? a.chunk_vbase[c] : 0ull;
        }
        // Consume the bitmap words here, before any store of this iteration:
        // the vector memory counter completes in order, so a later wait for
        // them would also wait for this iteration's stores.
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u)
            asm volatile("" : "+v"(mu[u]));
        uint32_t cnts[kU], incls[kU];
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u) {
            cnts[u] = __popcll(mu[u]);
            incls[u] = wave_incl_scan(cnts[u], lane);
            if (lane == kWave - 1)
                s_wt[ip][u][wave] = incls[u];
        }
        lds_barrier();
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u) {
            const uint64_t coff = s_meta[ip][0][u];
            if (coff == ~0ull)
                continue;  // the same for every thread of the block
            const uint64_t m = mu[u];
            const uint32_t cnt = cnts[u];
            const uint32_t incl = incls[u];
            const uint32_t *const wt = s_wt[ip][u];
            uint32_t woff = 0;
            for (uint32_t q = 0; q < kW; ++q)
                woff += q < wave ? wt[q] : 0u;
            const uint32_t wtot = wt[wave];
            const uint64_t obase = coff + woff;
            const uint64_t cvb = s_meta[ip][1][u];    // value base of the chunk (uniform)
            const uint32_t tb = kValsPerWord * tid;   // this word's offset in the chunk
            const uint32_t excl = incl - cnt;
            // Bit b of the word (bit 2i <-> 6i + 1, bit 2i + 1 <-> 6i + 5) is the
            // value tb + 3b + 1 + (b & 1) past the chunk base.
            if (wtot <= kStagePerWave) {
                // the usual case: the wave's primes fit one staging window;
                // the word's halves are walked with 32-bit operations
                uint32_t pos = excl;
                uint32_t h = (uint32_t)m;
                while (h) {
                    const uint32_t b = (uint32_t)__builtin_ctz(h);
                    h &= h - 1;
                    s_stage[wave][pos++] = tb + 3u * b + 1u + (b & 1u);
                }
                h = (uint32_t)(m >> 32);
                while (h) {
                    const uint32_t b = 32u + (uint32_t)__builtin_ctz(h);
                    h &= h - 1;
                    s_stage[wave][pos++] = tb + 3u * b + 1u + (b & 1u);
                }
                wave_lds_fence();  // the window is written before any lane reads it
                for (uint32_t e = lane; e < wtot; e += kWave)
                    put_out<T>(out, obase + e, cvb + s_stage[wave][e], a);
                wave_lds_fence();  // and read before the next chunk rewrites it
            } else {
                // Passes over rank windows of kStagePerWave, uniform across the wavefront.
                for (uint32_t pass = 0; pass < wtot; pass += kStagePerWave) {
                    if (excl < pass + kStagePerWave && excl + cnt > pass) {
                        uint64_t mm = m;
                        uint32_t pos = excl;
                        while (mm) {
                            const uint32_t b = (uint32_t)__builtin_ctzll(mm);
                            mm &= mm - 1;
                            if (pos >= pass && pos < pass + kStagePerWave)
                                s_stage[wave][pos - pass] = tb + 3u * b + 1u + (b & 1u);
                            ++pos;
                        }
                    }
                    wave_lds_fence();
                    const uint32_t n_in = (wtot - pass) < kStagePerWave ? (wtot - pass) : kStagePerWave;
                    for (uint32_t e = lane; e < n_in; e += kWave)
                        put_out<T>(out, obase + pass + e, cvb + s_stage[wave][e], a);
                    wave_lds_fence();
                }
            }
        }
    }
}

__global__ void k_zero(const JobHeader *job, unsigned long long *counters, unsigned long long *counts,
                       uint32_t *bcount, uint32_t *gbm, uint32_t *garrive, unsigned long long *tally)
{
    const uint32_t n = job->nranges;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (g < kNumCounters)
        counters[g] = 0;
    if (tally && g < 4)
        tally[g] = 0;
    for (uint32_t i = g; i < n; i += stride)
        counts[i] = 0;
    if (job->nunits)
        for (uint64_t i = g; i < job->ntiles; i += stride)
            bcount[i] = 0;  // count (exact layout) or cursor (estimated layout)
    for (uint64_t i = g; i < job->gwords; i += stride)
        gbm[i] = 0;
    for (uint64_t i = g; i < job->gtiles; i += stride)
        garrive[i] = 0;
}

// ---------------------------------------------------------------------------
// Host-side launch helpers (called from the runtime in api.hip).
// ---------------------------------------------------------------------------
hipError_t set_sieve_lds_limit(uint32_t segment_bytes)
{
    const int bytes = (int)(segment_bytes + sizeof(TileShared));
    const void *fns[] = {(const void *)k_sieve<256, 4, false>,  (const void *)k_sieve<256, 6, false>,
                         (const void *)k_sieve<512, 4, false>,  (const void *)k_sieve<512, 6, false>,
                         (const void *)k_sieve<1024, 4, false>, (const void *)k_sieve<256, 4, true>,
                         (const void *)k_sieve<256, 6, true>,   (const void *)k_sieve<512, 4, true>,
                         (const void *)k_sieve<512, 6, true>,   (const void *)k_sieve<1024, 4, true>};
    for (const void *f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_zero(const JobHeader *job, unsigned long long *counters, unsigned long long *counts,
                       uint32_t *bcount, uint32_t *gbm, uint32_t *garrive, unsigned long long *tally, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero, dim3(256), dim3(256), 0, s, job, counters, counts, bcount, gbm, garrive, tally);
    return hipGetLastError();
}

namespace {

// Workgroups of one bucket pass resident per CU for a given LDS size (the
// grid is exactly the resident set: the kernel strides over its units).
template <int PASS>
int bucket_residency(size_t lds)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bucket<PASS, false>, kBucketThreads, lds) != hipSuccess ||
        nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

}  // namespace

hipError_t launch_bucket(const BucketArgs &a, int pass, uint32_t cus, hipStream_t s)
{
    if (a.win < 1 || a.win > kBucketWindow || (a.win & (a.win - 1)))
        return hipErrorInvalidValue;
    const size_t lds = pass ? (size_t)a.win * (sizeof(unsigned long long) + sizeof(uint32_t)) +
                                  (size_t)kBucketKeep * kBucketThreads * sizeof(uint32_t)
                            : (size_t)a.win * sizeof(uint32_t);
    // residency per (pass, power-of-two window): queried once
    static std::atomic<int> occ[3][16];
    int w2 = 0;
    while ((1u << w2) < a.win)
        ++w2;
    int nb = occ[pass][w2].load(std::memory_order_relaxed);
    if (nb == 0) {
        nb = pass == 0 ? bucket_residency<0>(lds) : pass == 1 ? bucket_residency<1>(lds) : bucket_residency<2>(lds);
        occ[pass][w2].store(nb, std::memory_order_relaxed);
    }
    const dim3 grid(cus * (uint32_t)nb);
    if (a.wide) {
        // windows past 64 bits: the exact layout only
        if (pass == 0)
            hipLaunchKernelGGL((k_bucket<0, true>), grid, dim3(kBucketThreads), lds, s, a);
        else if (pass == 1)
            hipLaunchKernelGGL((k_bucket<1, true>), grid, dim3(kBucketThreads), lds, s, a);
        else
            return hipErrorInvalidValue;
    } else if (pass == 0) {
        hipLaunchKernelGGL((k_bucket<0, false>), grid, dim3(kBucketThreads), lds, s, a);
    } else if (pass == 1) {
        hipLaunchKernelGGL((k_bucket<1, false>), grid, dim3(kBucketThreads), lds, s, a);
    } else {
        hipLaunchKernelGGL((k_bucket<2, false>), grid, dim3(kBucketThreads), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_bucket_scan(const BucketScanArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(kFinalizeThreads), 0, s, a);
    return hipGetLastError();
}

namespace {

template <bool U24>
hipError_t launch_sieve_t(const SieveArgs &a, uint32_t nt, bool six, uint32_t grid, size_t lds, hipStream_t s)
{
    switch (nt) {
    case 256:
        if (six)
            hipLaunchKernelGGL((k_sieve<256, 6, U24>), dim3(grid), dim3(256), lds, s, a);
        else
            hipLaunchKernelGGL((k_sieve<256, 4, U24>), dim3(grid), dim3(256), lds, s, a);
        break;
    case 512:
        if (six)
            hipLaunchKernelGGL((k_sieve<512, 6, U24>), dim3(grid), dim3(512), lds, s, a);
        else
            hipLaunchKernelGGL((k_sieve<512, 4, U24>), dim3(grid), dim3(512), lds, s, a);
        break;
    case 1024:
        hipLaunchKernelGGL((k_sieve<1024, 4, U24>), dim3(grid), dim3(1024), lds, s, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

// u24: the caller guarantees that every prime a tile of the job uses is
// below 2^24 - 8 (isqrt(hi - 1) below that for every range).  wg_per_cu:
// resident workgroups per CU; with 24 or more waves per CU (six per SIMD)
// the kernel variant holding 80 VGPRs (a smaller carried state) is used.
hipError_t launch_sieve(const SieveArgs &a, uint32_t nt, uint32_t wg_per_cu, uint32_t grid, bool u24, hipStream_t s)
{
    const size_t lds = (size_t)a.pw * 8 + sizeof(TileShared);  // planes, then bookkeeping
    const bool six = nt < 1024 && (nt / 64) * wg_per_cu >= 24;
    return u24 ? launch_sieve_t<true>(a, nt, six, grid, lds, s) : launch_sieve_t<false>(a, nt, six, grid, lds, s);
}

hipError_t launch_finalize(const FinalizeArgs &a, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(kFinalizeThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_seg(const SegArgs &a, int pass, uint32_t grid, hipStream_t s)
{
    if (pass == 0)
        hipLaunchKernelGGL(k_seg_sum, dim3(grid), dim3(kFinalizeThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_seg_scan, dim3(grid), dim3(kFinalizeThreads), 0, s, a);
    return hipGetLastError();
}

// Both element types are launched; each kernel exits at once unless the job's
// element size is its own, so one launch sequence (and one graph) fits all.
hipError_t launch_compact(const CompactArgs &a, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_compact<uint32_t>, dim3(grid), dim3(kCompactThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_compact<uint64_t>, dim3(grid), dim3(kCompactThreads), 0, s, a);
    return hipGetLastError();
}

// The compaction of a wide window (16-byte elements).
hipError_t launch_compact_wide(const CompactArgs &a, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_compact<U128>, dim3(grid), dim3(kCompactThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace sieve
