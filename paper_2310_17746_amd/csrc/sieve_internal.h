// Internal layout shared by the HIP kernels and the host runtime of libsieve.
//
// Value layout (Sec. 2.1, Fig. 2): a tile with value base B (a multiple of
// 6) holds two bit planes of PW 32-bit words each in LDS (A_one words at
// bytes [0, 4PW), A_five words at [4PW, 8PW)).  Bit i of plane A_r (r = 1 or
// 5) stands for the value B + 6*i + r.  One plane word
// covers 192 consecutive integers; a tile covers 192 * PW integers.  In LDS a
// set bit means "composite / excluded" so that marking is a single LDS OR.
//
// List output goes through a value-ordered bitmap in HBM: plane word w of
// A_one and A_five are interleaved into one 64-bit word whose bit 2i is
// B + 192w + 6i + 1 and bit 2i+1 is B + 192w + 6i + 5, set when prime.
// Bitmap words are grouped in chunks of kChunkWords; chunk c of a range
// starts at value base + kChunkVals * c.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#include "wheel.h"

namespace sieve {

constexpr uint32_t kChunkWords = 512;                       // u64 bitmap words per chunk
constexpr uint64_t kValsPerWord = 192;                      // integers per plane word
constexpr uint64_t kChunkVals = kValsPerWord * kChunkWords;  // integers per chunk
constexpr int kMaxGroups = 6;                               // presieve pattern groups
constexpr uint32_t kCompactThreads = 512;                   // one bitmap word per thread
constexpr uint32_t kStagePerWave = 512;                     // compaction staging entries per wave
constexpr uint32_t kFinalizeThreads = 1024;
constexpr uint32_t kSegChunks = 4096;  // chunks per scan segment (4 per thread of 1024)
constexpr uint32_t kBucketThreads = 512;    // primes per bucket work unit
constexpr uint32_t kBucketWindow = 2048;    // tiles per bucket work unit (LDS bins)
constexpr uint32_t kBucketMinPrimes = 32768; // fewest large primes worth a bucket pass
constexpr uint32_t kBucketKeep = 4;          // hits per thread the bucket fill replays from LDS
constexpr uint32_t kPartPrimes = 262144;     // fewest primes (beyond the split items) per part of a split tile
constexpr uint32_t kStaticMaxRanges = 1024;  // ranges per call of the allocation-free batch count
constexpr uint32_t kMaxStrip = 64;           // tiles per strip (carried indices stay below 2^32 - 2^26)

// One range of a job.  Host-computed plan; read-only on the device.
struct RangeDesc {
    uint64_t lo, hi;     // [lo, hi)
    uint64_t base;       // lo - lo % 6: value base of tile 0
    uint64_t tile0;      // global index of the range's first tile
    uint64_t chunk0;     // list ranges: global index of the first bitmap chunk
    uint64_t out_off;    // list ranges: first output element
    uint64_t cap;        // list ranges: output capacity in elements
    uint32_t ntiles;     // tiles of this range (0 when it holds no wheel value)
    uint32_t last_words; // plane words of the last tile
    uint32_t mode;       // 0 count, 1 list
    uint32_t nchunks;    // list ranges: bitmap chunks
    uint32_t nact;       // resident primes p with p * p < hi
    uint32_t kbig;       // first prime index handled by the bucket sieve (nact: none)
    uint64_t bunit0;     // first bucket work unit of this range
    uint32_t bunits;     // bucket work units: prime blocks x tile windows
    uint32_t bwins;      // tile windows of kBucketWindow tiles
    uint64_t bbase;      // estimated layout: first entry of this range's buckets
    uint32_t bcap;       // estimated layout: entries reserved per tile
    uint32_t nseg;       // list ranges: scan segments of kSegChunks chunks
    uint32_t seg0;       // global index of the first segment (running count)
    uint32_t nparts;     // work units per tile: 1, or the parts of a split tile
    uint32_t gtile0;     // split ranges: first global-bitmap slot (one per tile)
    uint32_t part_primes;  // split ranges: primes beyond the split items per part
    uint32_t strip;      // tiles per strip: a workgroup sieves a strip's tiles in order and
                         // carries each prime's next hit from tile to tile (1 for split ranges)
    uint32_t nstrips;    // strips of this range: ceil(ntiles / strip)
};

// Per-job scalars, in device memory so that a captured graph can be replayed
// for a new job after only a host-to-device copy.
struct JobHeader {
    uint64_t ntiles;     // tiles over all ranges
    uint64_t nchunks;    // bitmap chunks over all list ranges
    uint64_t nunits;     // bucket work units over all ranges
    uint32_t bmode;      // bucket layout: 1 estimated per-range slices, 2 exact per-tile offsets
    uint32_t wide;       // 1: a window beyond 64 bits, in offsets from its base (no 2 or 3)
    uint32_t nranges;
    uint32_t nlist;      // list ranges
    void *out;           // caller's output buffer (list ranges)
    int32_t elem_bytes;  // 4 or 8
    uint32_t links;      // 1: BucketArgs::links holds a walk link per range
    uint64_t nseg;       // scan segments over all list ranges
    uint64_t nvisit;     // sieve work units: strips (or tiles times their parts), over all ranges
    uint64_t gtiles;     // tiles of split ranges (global-bitmap slots)
    uint64_t gwords;     // words of those slots (2 planes each)
};

// Bucket walk state kept between consecutive pieces of one long range (a
// serving request cut into steps): the pieces tile the range back to back,
// so where a prime's walk ends past one piece is where it goes on in the
// next (Sec. 2.4's incremental state, carried across jobs).  One WalkState
// per prime k, at index k - kbig: the next hit of each plane as a tile
// index relative to the piece that reads it, and the hit's bit | cofactor
// residue mod 5 << 28 (5: not tracked).
struct WalkState {
    uint32_t t1, bc1, t5, bc5;
};

// Per range of a job (when JobHeader::links is 1): the walks of bucket
// primes [kbig, kbig + nsrc) resume from src instead of a Table 1 start, and
// the walks of every bucket prime [kbig, nact) store their end state in dst,
// relative to the tile after the range's last.  Zero addresses: none.
struct WalkLink {
    WalkState *src;
    WalkState *dst;
    uint32_t nsrc;
    uint32_t pad;
};

// The order in which the sieve kernel's workgroups take tiles: ranges in
// visit order, each contributing its tiles in storage order.  vstart is the
// visit position of the range's first tile.  The host puts the ranges with
// the most Table 1 starts per tile first, so the costliest tiles are not
// left for the end of the job.
struct VisitEntry {
    uint64_t vstart;
    uint32_t range;
    uint32_t pad;
};

// Counters zeroed at the start of every job.
enum Counter { kTileCounter = 0, kChunkCounter = 1, kErrorFlag = 2, kOverflowFlag = 3, kNumCounters = 4 };

// A presieve pattern group: primes whose product is `period`.  Its table
// holds period + 64 bits per plane (bit t stands for 6t + r, set when some
// prime of the group divides it), stored as uint2 {A_one word, A_five word}
// at `offset` words into the shared table.
struct PsGroup {
    uint32_t period;
    uint32_t offset;
    uint32_t step;  // (32 * block_threads) mod period
    uint32_t pad;
};

// Kernel arguments: pointers and context-level constants only.  Everything
// that changes from job to job lives in JobHeader / RangeDesc on the device.
struct SieveArgs {
    const JobHeader *job;
    const RangeDesc *ranges;
    const VisitEntry *visit;      // nranges entries, in visit order
    unsigned long long *counters;
    unsigned long long *counts;   // per range
    const PrimeConst *prm;        // every resident prime >= 5, ascending
    const uint2 *prd;             // the same primes as {P, offset of A_five hits from A_one hits}
    const uint32_t *pidx;         // pidx[s] = number of resident primes <= 64 * s
    uint32_t pidx_len;
    uint32_t nprimes;
    uint32_t first_mark;          // first prime index marked in LDS (after the presieve)
    uint32_t k_split;             // primes [first_mark, k_split) are split into items
    uint32_t k_dense;             // primes [first_mark, k_dense) split over a multiple of 32 lanes
    const uint2 *items;           // {prime index, (j << 16) | g}
    const uint32_t *item_prefix;  // items before prime first_mark + i
    const uint2 *ps_tab;
    PsGroup groups[kMaxGroups];       // all applied; disabled ones are all-zero
    uint32_t ngroups;
    uint32_t restore1, restore5;  // bits of the presieved primes in word 0 of a tile based at 0
    uint32_t pw;                  // plane words per tile
    uint32_t skip5;               // marks with 5 | cofactor skipped (5 is presieved): 0 none, 1 every item,
                                  // 2 split items, 3 split and fixed-mask (dense) items
    unsigned long long *bitmap;   // list scratch (u64 words)
    uint32_t *chunk_counts;       // per chunk prime count
    const uint32_t *bdata;        // bucket entries: bit | plane << 31
    const unsigned long long *boff;  // exact layout, per tile: first entry
    const uint32_t *bcount;       // exact layout, per tile: entries
    const uint32_t *bcursor;      // estimated layout, per tile: entries written
    uint32_t *gbm;                // split tiles: both planes per slot (2 pw words), zeroed per job
    uint32_t *garrive;            // split tiles: parts finished, per slot, zeroed per job
    unsigned long long *tally;    // debug build only: hits, ORs issued, hits skipped, bad runs
};

// Bucket sieve (large primes of multi-tile ranges).  One work unit is a block
// of kBucketThreads primes of one range; every thread walks one prime's hits
// through the range's tiles.
struct BucketArgs {
    const JobHeader *job;
    const RangeDesc *ranges;
    const PrimeConst *prm;
    uint32_t *bcount;             // per tile (count pass: accumulated)
    uint32_t *bcursor;            // per tile (fill pass: reserved so far)
    const unsigned long long *boff;
    uint32_t *bdata;
    unsigned long long *counters; // kOverflowFlag set when an estimated slice overflows
    uint32_t skip5;               // as in SieveArgs
    uint32_t nbits;               // bits per plane per tile (32 * pw)
    uint64_t span;                // integers per tile (192 * pw)
    uint64_t span_rcp;            // floor((2^64 - 1) / span)
    uint32_t win;                 // LDS bins per workgroup: >= the tiles of every unit's window
    uint32_t pad;
    unsigned long long *tally;    // debug build only, as in SieveArgs
    const WalkLink *links;        // per range, read when JobHeader::links is 1
    // A window past 64 bits (range values are offsets from its base W):
    uint32_t wide;                // 1: starts from (W - 1) mod P, 64-bit Table 1
    uint32_t w5;                  // W mod 5
    uint64_t wlo, whi;            // W
    uint64_t wm1_lo, wm1_hi;      // W - 1
};

struct BucketScanArgs {
    const JobHeader *job;
    const uint32_t *bcount;
    unsigned long long *boff;     // ntiles + 1 entries; boff[ntiles] = total
    uint32_t *bcursor;            // zeroed here for the fill pass
};

struct FinalizeArgs {
    const JobHeader *job;
    const RangeDesc *ranges;
    unsigned long long *counts;
    int32_t *status;
    const unsigned long long *seg_sum;  // per segment: primes in its chunks
    unsigned long long *seg_base;       // per segment: first output element; ~0 when
                                        // its range does not fit
};

// Chunk-offset scan of the list ranges in segments, spread over workgroups:
// k_seg_sum adds each segment's chunk counts, k_finalize scans the segment
// sums of each range, k_seg_scan writes every chunk's output offset and value
// base from its segment's base.
struct SegArgs {
    const JobHeader *job;
    const RangeDesc *ranges;
    const uint32_t *chunk_counts;
    unsigned long long *seg_sum;
    const unsigned long long *seg_base;
    unsigned long long *chunk_off;
    unsigned long long *chunk_vbase;  // per chunk: value base of its first word
};

struct CompactArgs {
    const JobHeader *job;
    const unsigned long long *chunk_vbase;  // per chunk: value base of its first word
    const unsigned long long *bitmap;
    const unsigned long long *chunk_off;    // per chunk: first output element; ~0 when
                                            // its range does not fit (nothing is written)
    uint64_t wbase_lo, wbase_hi;            // 128-bit output: the window base added to every value
};

// A 128-bit output element (low half first), as sieve_u128 in sieve.h.
struct alignas(16) U128 {
    uint64_t lo, hi;
};

}  // namespace sieve
