// Host runtime internals shared by the C ABI (api.hip) and the serving
// engine (server.hip): the context layout and the job entry points.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

#include <hip/hip_runtime.h>

#include "sieve_internal.h"
#include "wheel.h"

namespace sieve {
namespace rt {

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    // Grows to at least `need` elements (contents are not kept).
    bool reserve(size_t need, uint64_t *gen = nullptr)
    {
        if (need <= n && p)
            return true;
        size_t m = std::max<size_t>(need, 1);
        if (p)
            m = std::max(m, n + n / 2);
        if (p)
            (void)hipFree(p);
        p = nullptr;
        n = 0;
        if (gen)
            ++*gen;
        T *q = nullptr;
        if (hipMalloc((void **)&q, m * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        p = q;
        n = m;
        return true;
    }
    void release()
    {
        if (p)
            (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

}  // namespace rt
}  // namespace sieve

struct sieve_ctx {
    int device = 0;
    int cus = 0;
    uint32_t lds_max = 0;
    sieve_params prm{};
    hipStream_t stream = nullptr;
    int last_error = SIEVE_OK;

    // Resident base primes (>= 5) and derived constants.
    uint64_t limit = 0;
    std::vector<uint32_t> h_primes;
    sieve::rt::DevBuf<sieve::PrimeConst> d_prm;
    sieve::rt::DevBuf<uint2> d_prd;  // the same primes as {P, offset of A_five hits from A_one hits}
    sieve::rt::DevBuf<uint32_t> d_pidx;
    sieve::rt::DevBuf<uint2> d_items;
    sieve::rt::DevBuf<uint32_t> d_item_prefix;
    uint32_t first_mark = 0, k_split = 0, k_dense = 0;
    uint32_t k_large = 0;  // first prime index the bucket sieve takes (multi-tile ranges)
    std::vector<double> inv_prefix;  // inv_prefix[k] = sum of 1/p over the first k primes
    std::vector<uint32_t> h_pidx;    // h_pidx[s] = number of base primes <= 64 s (s <= limit / 64 + 1)
    uint64_t bucket_fallbacks = 0;   // jobs re-run with the exact bucket layout
    uint64_t bucket_jobs = 0;        // jobs that ran the bucket sieve
    uint64_t bucket_budget = 0;      // bucket entries one job may hold (larger jobs run in pieces)
    uint32_t bucket_win = 0;         // per-tile LDS bins of the bucket kernels (kernel argument)
    uint32_t sieve_u24 = 0;          // the job's primes are below 2^24 - 8: 24-bit start arithmetic

    // Presieve tables.
    sieve::rt::DevBuf<uint2> d_pstab;
    sieve::PsGroup groups[sieve::kMaxGroups]{};
    uint32_t ngroups = 0;
    uint32_t restore1 = 0, restore5 = 0;

    // Job scratch.
    sieve::rt::DevBuf<unsigned char> d_blob;  // JobHeader | RangeDesc[]
    sieve::rt::DevBuf<unsigned long long> d_counters;
    sieve::rt::DevBuf<unsigned long long> d_counts;
    sieve::rt::DevBuf<int32_t> d_status;
    sieve::rt::DevBuf<unsigned long long> d_bitmap;
    sieve::rt::DevBuf<uint32_t> d_chunk_counts;
    sieve::rt::DevBuf<unsigned long long> d_chunk_vbase;
    sieve::rt::DevBuf<unsigned long long> d_chunk_off;
    sieve::rt::DevBuf<unsigned long long> d_seg_sum, d_seg_base;  // chunk-offset scan segments
    sieve::rt::DevBuf<uint32_t> d_gbm, d_garrive;  // split tiles: global planes, arrival counts
    // Pinned host staging, two slots used in turn by consecutive jobs: the
    // blob (JobHeader | RangeDesc[] | VisitEntry[]) before its copy to the
    // device, and the per-range counts, status and the error and overflow
    // flags after the job.  A slot's event is recorded after its last use on
    // the stream, so a stream-ordered call can return while its copies are
    // pending; the job after next waits for it before refilling the slot.
    struct HostSlot {
        unsigned char *blob = nullptr;
        unsigned long long *counts = nullptr;
        int32_t *status = nullptr;
        unsigned long long *flag = nullptr;
        hipEvent_t done = nullptr;
        bool used = false;
    };
    HostSlot slot[2];
    int cur_slot = 0;
    unsigned char *h_blob = nullptr;         // the current job's slot buffers
    unsigned long long *h_counts = nullptr;
    int32_t *h_status = nullptr;
    unsigned long long *h_flag = nullptr;
    size_t h_blob_n = 0;
    uint64_t cap_ranges = 0, cap_chunks = 0;
    // End of the context's latest job on the stream it ran on; a job on
    // another stream waits for it first (the scratch is shared).
    hipEvent_t last_ev = nullptr;
    hipStream_t last_stream = nullptr;
    bool last_valid = false;

    // Bucket sieve scratch: per-tile counts, cursors and offsets; entries.
    sieve::rt::DevBuf<uint32_t> d_bcount, d_bcursor, d_bdata;
    sieve::rt::DevBuf<unsigned long long> d_boff;
    unsigned long long *h_btotal = nullptr;  // pinned
    uint64_t cap_tiles = 0, cap_bdata = 0, cap_gtiles = 0;

    // Graphs of the job phases (0: whole job without buckets, 1: exact
    // bucket count + scan, 2: exact bucket fill + sieve + finalize + compact,
    // 3: estimated bucket fill + sieve + finalize + compact); each is valid
    // while gen == graph_gen[i].
    hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
    hipGraph_t graph_src[4] = {nullptr, nullptr, nullptr, nullptr};
    uint64_t graph_gen[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    uint64_t gen = 0;

    // Host streaming (stream.hip): two device piece buffers, two pinned
    // staging buffers, a copy stream and one event per slot, kept between
    // calls.
    sieve::rt::DevBuf<unsigned char> d_piece[2];
    unsigned char *h_piece[2] = {nullptr, nullptr};
    size_t h_piece_bytes = 0;
    hipStream_t copy_stream = nullptr;
    hipEvent_t piece_ev[2] = {nullptr, nullptr};

    // Marking tally of the debug build (SIEVE_MARK_COUNT): device counters of
    // the current job (hits, ORs issued, hits skipped, bad runs), a pinned
    // copy, and the sums over the jobs since the last reset.  Unallocated in
    // the product build.
    sieve::rt::DevBuf<unsigned long long> d_tally;
    unsigned long long *h_tally = nullptr;
    unsigned long long tally_total[4] = {0, 0, 0, 0};

    // Windows beyond 64 bits (wide.hip): extension base primes from 2^32 up
    // to ext_limit (ascending, 64-bit), every kExtSample-th of them on the
    // host for counting the ones below a bound, and the per-window residues
    // (W - 1) mod P of the primes marked in LDS.
    sieve::rt::DevBuf<uint64_t> d_ext;
    uint64_t n_ext = 0, ext_limit = 0;
    std::vector<uint64_t> h_ext_sample;
    sieve::rt::DevBuf<uint32_t> d_wr;

    // Device address of this GPU's fixed scratch array (allocation-free
    // entry point), looked up once when the context is created.
    unsigned char *static_scratch = nullptr;

    // Optional event timing of the sieve kernel and the post-processing.
    int timing = 0;
    hipEvent_t ev[6]{};
    double t_sieve_ms = 0, t_post_ms = 0, t_bucket_ms = 0;
    uint64_t t_jobs = 0;
};

namespace sieve {
namespace rt {

int set_err(sieve_ctx *c, int e);
int hip_status(hipError_t e);
uint64_t isqrt_host(uint64_t n);
// Tile plan of [lo, hi) for pw plane words per tile.
void plan_range(uint64_t lo, uint64_t hi, uint32_t pw, uint64_t &ntiles, uint64_t &base, uint32_t &last_words);

// Bucket walk state of one range of a job that continues an earlier piece of
// the same long range, which ended at the tile where this one starts, in a
// job with the same k_large.  src holds nsrc primes' states from k_large on
// (the earlier piece's end state); dst (dcap entries) receives this range's
// end state.  Device memory, owned by the caller; NULL / 0 for none.
// run_job sets `saved` to the number of states it stored in dst and
// `resumed` to 1 when the range's walks started from src (both 0 for a
// range without bucket primes, a dst too small, or a job that had to be cut
// into pieces itself).
struct WalkSpec {
    WalkState *src;
    WalkState *dst;
    uint32_t nsrc;
    uint32_t dcap;
    uint32_t saved;
    uint32_t resumed;
};

// One job over n ranges (see api.hip) on `stream` (NULL: the context stream).
// counts/status are host arrays of n entries (may be NULL).  List range i
// writes its primes from element off[i] of `out`; `out` may be NULL, and
// off[i] then is the output's device address divided by elem_bytes (so that
// ranges of one job can write to unrelated buffers).  Synchronous
// unless async_ok: then a job that needs no host decision mid-way returns
// once enqueued, and counts/status are written when the stream reaches its
// end.  ws (n entries, or NULL): bucket walk state carried between the
// pieces of long ranges (see WalkSpec).
int run_job(sieve_ctx *c, uint64_t n, const uint64_t *lo, const uint64_t *hi, const uint8_t *mode,
            const uint64_t *off, const uint64_t *cap, int elem_bytes, void *out, uint64_t *counts, int32_t *status,
            hipStream_t stream, bool use_graph, bool async_ok = false, WalkSpec *ws = nullptr);
// Makes the resident base primes cover `limit`.
int grow_base_primes(sieve_ctx *c, uint64_t limit);
// Makes the job scratch hold a job of the given size (capacities only grow).
int ensure_capacity(sieve_ctx *c, uint64_t nranges, uint64_t nchunks, uint64_t ntiles, uint64_t gtiles);
// Byte offset of the RangeDesc table in the device blob (after the JobHeader).
size_t blob_ranges_offset();
// Number of resident base primes <= x (x <= c->limit).
uint32_t primes_upto(const sieve_ctx *c, uint64_t x);

}  // namespace rt
}  // namespace sieve
