// Incremental generation and streaming output.
//
// sieve_gen_*: a generator hands out the primes from a start value onward,
// n at a time, with no upper limit fixed in advance -- the paper's
// incremental sieve (Sec. 2.4), which keeps producing primes and extends the
// Sieve Data Store (Sec. 4) as the squares of new primes are reached.  It
// sieves blocks of whole tiles ahead of its cursor into a device staging
// buffer through the ordinary list path and grows the resident base primes
// geometrically as the cursor advances.
//
// sieve_list_host / sieve_write_files: the Prime Number Data Store (Sec. 4)
// delivered to host memory or written to files (Sec. 6).  The range is cut
// into pieces with a rigorous prime bound of at most piece_elems; piece k+1
// is sieved on the context stream while piece k is copied over PCIe on a
// copy stream and piece k-1 is consumed (memcpy or fwrite) by a host task.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <functional>
#include <future>
#include <string>

#include <hip/hip_runtime.h>

#include "sieve.h"
#include "runtime.h"

using sieve::rt::DevBuf;

struct sieve_gen {
    sieve_ctx *c = nullptr;
    int elem = 8;
    uint64_t cursor = 0;    // every value below it has been sieved
    uint64_t end = 0;       // end of the value domain (exclusive)
    uint64_t position = 0;  // every prime below it has been handed out
    DevBuf<unsigned char> stage;
    uint64_t head = 0, tail = 0;  // staged primes not yet handed out: [head, tail)
    unsigned char *h_last = nullptr;  // pinned, one element
};

namespace {

constexpr uint64_t kDefaultPieceElems = 1ull << 24;
constexpr uint64_t kDefaultPrimesPerFile = 125000000ull;
constexpr uint64_t kMaxBlockPrimes = 1ull << 25;

uint64_t tile_span(const sieve_ctx *c) { return 24ull * c->prm.segment_bytes; }

// Makes the base primes cover hi - 1 with headroom, so that a generator that
// walks upward grows them O(log) times.
int cover_base(sieve_ctx *c, uint64_t hi)
{
    if (hi < 2)
        return SIEVE_OK;
    const uint64_t need = sieve::rt::isqrt_host(hi - 1);
    if (need <= c->limit)
        return SIEVE_OK;
    const uint64_t want = std::min<uint64_t>((1ull << 32) - 1, std::max<uint64_t>(2 * need, 1u << 16));
    return sieve_base_primes(c, want, nullptr);
}

int list_piece(sieve_ctx *c, uint64_t lo, uint64_t hi, void *dst, uint64_t cap, int elem, uint64_t *cnt,
               hipStream_t s)
{
    const uint8_t mode = 1;
    const uint64_t off = 0;
    int32_t rs = SIEVE_OK;
    int st = sieve::rt::run_job(c, 1, &lo, &hi, &mode, &off, &cap, elem, dst, cnt, &rs, s, false);
    if (st == SIEVE_OK && rs != SIEVE_OK)
        st = rs;
    return st;
}

// Sink of the streaming pipeline: consumes n elements that belong at element
// offset `first` of the output; called for the pieces in order.
using Sink = std::function<int(const unsigned char *p, uint64_t first, uint64_t n)>;

int ensure_pipe(sieve_ctx *c, size_t bytes, bool host)
{
    for (int i = 0; i < 2; ++i)
        if (!c->d_piece[i].reserve(bytes))
            return SIEVE_E_NOMEM;
    if (host && c->h_piece_bytes < bytes) {
        for (int i = 0; i < 2; ++i) {
            if (c->h_piece[i])
                (void)hipHostFree(c->h_piece[i]);
            c->h_piece[i] = nullptr;
        }
        c->h_piece_bytes = 0;
        for (int i = 0; i < 2; ++i)
            if (hipHostMalloc((void **)&c->h_piece[i], bytes, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                c->h_piece[i] = nullptr;
                return SIEVE_E_NOMEM;
            }
        c->h_piece_bytes = bytes;
    }
    if (!c->copy_stream && hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess)
        return SIEVE_E_DEVICE;
    for (int i = 0; i < 2; ++i)
        if (!c->piece_ev[i] && hipEventCreateWithFlags(&c->piece_ev[i], hipEventDisableTiming) != hipSuccess)
            return SIEVE_E_DEVICE;
    return SIEVE_OK;
}

// End of the piece that starts at `lo`: at most L integers, within hi, with a
// rigorous prime bound of at most E.
uint64_t piece_end(uint64_t lo, uint64_t hi, uint64_t L, uint64_t E)
{
    uint64_t e = hi - lo > L ? lo + L : hi;
    while (sieve_list_bound(lo, e) > E)
        e = lo + (e - lo) / 2;
    return e;
}

// Streams the primes of [lo, hi) piece by piece.  With `direct` the pieces
// are copied straight into that pinned host array (no sink); otherwise they
// go through the context's pinned staging buffers into `sink`.  Past `cap`
// elements the remaining pieces are only counted.
int stream_range(sieve_ctx *c, uint64_t lo, uint64_t hi, int elem, uint64_t E, unsigned char *direct,
                 uint64_t cap, const Sink &sink, uint64_t *total_out)
{
    if (E < 256)
        return SIEVE_E_INVAL;
    int st = ensure_pipe(c, E * (size_t)elem, direct == nullptr);
    if (st != SIEVE_OK)
        return st;
    hipStream_t s = c->stream;
    // Piece length: the largest 192 * 2^k integers whose bound fits E.
    uint64_t L = 192;
    while (L < (1ull << 61) && sieve_list_bound(lo, lo + 2 * L) <= E)
        L *= 2;

    std::shared_future<int> slot_done[2];
    std::shared_future<int> last;
    uint64_t total = 0;
    bool over = false;
    auto drain = [&]() {
        int r = SIEVE_OK;
        if (last.valid() && last.get() != SIEVE_OK)
            r = last.get();
        for (auto &f : slot_done)
            if (f.valid() && f.get() != SIEVE_OK && r == SIEVE_OK)
                r = f.get();
        if (hipStreamSynchronize(c->copy_stream) != hipSuccess && r == SIEVE_OK)
            r = SIEVE_E_DEVICE;
        return r;
    };

    uint64_t k = 0;
    for (uint64_t a = lo; a < hi; ++k) {
        const uint64_t b = piece_end(a, hi, L, E);
        const int slot = (int)(k & 1);
        uint64_t cnt = 0;
        if (over) {
            st = sieve::rt::run_job(c, 1, &a, &b, nullptr, nullptr, nullptr, 8, nullptr, &cnt, nullptr, s, false);
        } else {
            // The device slot is reused once the copy of piece k - 2 is done.
            if (k >= 2 && hipStreamWaitEvent(s, c->piece_ev[slot], 0) != hipSuccess)
                st = SIEVE_E_DEVICE;
            if (st == SIEVE_OK)
                st = list_piece(c, a, b, c->d_piece[slot].p, E, elem, &cnt, s);
        }
        if (st != SIEVE_OK) {
            drain();
            return st;
        }
        if (!over && total + cnt > cap)
            over = true;
        if (!over && cnt) {
            const size_t bytes = cnt * (size_t)elem;
            hipError_t e;
            if (direct) {
                e = hipMemcpyAsync(direct + total * elem, c->d_piece[slot].p, bytes, hipMemcpyDeviceToHost,
                                   c->copy_stream);
                if (e == hipSuccess)
                    e = hipEventRecord(c->piece_ev[slot], c->copy_stream);
            } else {
                // The host slot is reused once the sink of piece k - 2 is done.
                if (slot_done[slot].valid() && slot_done[slot].get() != SIEVE_OK) {
                    st = slot_done[slot].get();
                    drain();
                    return st;
                }
                e = hipMemcpyAsync(c->h_piece[slot], c->d_piece[slot].p, bytes, hipMemcpyDeviceToHost,
                                   c->copy_stream);
                if (e == hipSuccess)
                    e = hipEventRecord(c->piece_ev[slot], c->copy_stream);
                if (e == hipSuccess) {
                    std::shared_future<int> prev = last;
                    const unsigned char *src = c->h_piece[slot];
                    hipEvent_t ev = c->piece_ev[slot];
                    const int dev = c->device;
                    const uint64_t first = total;
                    last = std::async(std::launch::async, [prev, src, ev, dev, first, cnt, &sink]() -> int {
                               if (prev.valid() && prev.get() != SIEVE_OK)
                                   return prev.get();
                               (void)hipSetDevice(dev);
                               if (hipEventSynchronize(ev) != hipSuccess)
                                   return SIEVE_E_DEVICE;
                               return sink(src, first, cnt);
                           }).share();
                    slot_done[slot] = last;
                }
            }
            if (e != hipSuccess) {
                drain();
                return SIEVE_E_DEVICE;
            }
        }
        total += cnt;
        a = b;
    }
    st = drain();
    *total_out = total;
    if (st == SIEVE_OK && over)
        st = SIEVE_E_CAPACITY;
    return st;
}

bool is_pinned_host(const void *p)
{
    hipPointerAttribute_t at;
    memset(&at, 0, sizeof at);
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeHost;
}

}  // namespace

extern "C" {

int sieve_gen_create(sieve_ctx *ctx, uint64_t start, int elem_bytes, sieve_gen **gen)
{
    if (!ctx || !gen)
        return SIEVE_E_INVAL;
    if (elem_bytes != 4 && elem_bytes != 8)
        return SIEVE_E_DTYPE;
    const uint64_t end = elem_bytes == 4 ? (1ull << 32) : SIEVE_MAX_HI;
    if (start > end)
        return SIEVE_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return SIEVE_E_DEVICE;
    sieve_gen *g = new (std::nothrow) sieve_gen;
    if (!g)
        return SIEVE_E_NOMEM;
    g->c = ctx;
    g->elem = elem_bytes;
    g->cursor = g->position = start;
    g->end = end;
    if (hipHostMalloc((void **)&g->h_last, 8, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete g;
        return SIEVE_E_NOMEM;
    }
    *gen = g;
    return SIEVE_OK;
}

int sieve_gen_destroy(sieve_gen *g)
{
    if (!g)
        return SIEVE_OK;
    (void)hipSetDevice(g->c->device);
    g->stage.release();
    if (g->h_last)
        (void)hipHostFree(g->h_last);
    delete g;
    return SIEVE_OK;
}

int sieve_gen_position(const sieve_gen *g, uint64_t *next)
{
    if (!g || !next)
        return SIEVE_E_INVAL;
    *next = g->position;
    return SIEVE_OK;
}

int sieve_gen_next(sieve_gen *g, uint64_t n, void *out_dev, uint64_t *n_out, void *stream)
{
    if (!g || !n_out || (n && !out_dev))
        return SIEVE_E_INVAL;
    sieve_ctx *c = g->c;
    if (hipSetDevice(c->device) != hipSuccess)
        return sieve::rt::set_err(c, SIEVE_E_DEVICE);
    hipStream_t s = stream ? (hipStream_t)stream : c->stream;
    unsigned char *out = (unsigned char *)out_dev;
    const int el = g->elem;
    uint64_t done = 0;
    auto take = [&](uint64_t k) -> hipError_t {
        hipError_t e = hipMemcpyAsync(out + done * el, g->stage.p + g->head * el, k * el,
                                      hipMemcpyDeviceToDevice, s);
        g->head += k;
        done += k;
        return e;
    };
    hipError_t e = hipSuccess;
    if (n && g->tail > g->head)
        e = take(std::min(n, g->tail - g->head));
    int st = e == hipSuccess ? SIEVE_OK : SIEVE_E_DEVICE;
    const uint64_t span = tile_span(c);
    while (st == SIEVE_OK && done < n && g->cursor < g->end) {
        // Next block: enough integers for the missing primes at the local
        // density 1/ln x (at least one tile per CU, at most kMaxBlockPrimes
        // expected primes), rounded up to whole tiles.
        const uint64_t want = std::min(n - done, kMaxBlockPrimes);
        const double lnx = log((double)std::max<uint64_t>(g->cursor, 1000) + 1e6);
        uint64_t len = (uint64_t)(want * lnx * 1.1) + span;
        len = std::max<uint64_t>(len, (uint64_t)c->cus * span);
        uint64_t hi = g->end - g->cursor > len ? g->cursor + len : g->end;
        if (hi < g->end)
            hi = std::min(g->end, (hi + span - 1) / span * span);
        st = cover_base(c, hi);
        if (st != SIEVE_OK)
            break;
        const uint64_t bound = sieve_list_bound(g->cursor, hi);
        if (!g->stage.reserve(std::max<uint64_t>(bound, 1) * el)) {
            st = SIEVE_E_NOMEM;
            break;
        }
        uint64_t cnt = 0;
        st = list_piece(c, g->cursor, hi, g->stage.p, bound, el, &cnt, s);
        if (st != SIEVE_OK)
            break;
        g->cursor = hi;
        g->head = 0;
        g->tail = cnt;
        if (cnt && hipSuccess != take(std::min(n - done, cnt)))
            st = SIEVE_E_DEVICE;
    }
    if (st == SIEVE_OK && done) {
        // The last prime handed out is the staged element just before head.
        e = hipMemcpyAsync(g->h_last, g->stage.p + (g->head - 1) * el, el, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            st = SIEVE_E_DEVICE;
        else
            g->position = (el == 4 ? *(uint32_t *)g->h_last : *(uint64_t *)g->h_last) + 1;
    } else if (st == SIEVE_OK && hipStreamSynchronize(s) != hipSuccess) {
        st = SIEVE_E_DEVICE;
    }
    if (st == SIEVE_OK && done < n)
        g->position = g->end;  // domain exhausted: every prime below end was handed out
    *n_out = done;
    return sieve::rt::set_err(c, st);
}

int sieve_list_host(sieve_ctx *ctx, uint64_t lo, uint64_t hi, void *out_host, uint64_t cap, int elem_bytes,
                    uint64_t piece_elems, uint64_t *n_out)
{
    if (!ctx || !n_out || (cap && !out_host) || lo > hi || hi > SIEVE_MAX_HI)
        return sieve::rt::set_err(ctx, SIEVE_E_INVAL);
    if (elem_bytes != 4 && elem_bytes != 8)
        return sieve::rt::set_err(ctx, SIEVE_E_DTYPE);
    if (elem_bytes == 4 && hi > (1ull << 32))
        return sieve::rt::set_err(ctx, SIEVE_E_DTYPE);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sieve::rt::set_err(ctx, SIEVE_E_DEVICE);
    unsigned char *dst = (unsigned char *)out_host;
    unsigned char *direct = cap && is_pinned_host(out_host) ? dst : nullptr;
    const int el = elem_bytes;
    Sink sink = [dst, el](const unsigned char *p, uint64_t first, uint64_t n) -> int {
        memcpy(dst + first * el, p, n * el);
        return SIEVE_OK;
    };
    *n_out = 0;
    int st = stream_range(ctx, lo, hi, el, piece_elems ? piece_elems : kDefaultPieceElems, direct, cap, sink,
                          n_out);
    return sieve::rt::set_err(ctx, st);
}

int sieve_write_files(sieve_ctx *ctx, uint64_t lo, uint64_t hi, const char *path_prefix, uint64_t primes_per_file,
                      int elem_bytes, uint64_t piece_elems, uint64_t *n_out, uint64_t *n_files)
{
    if (!ctx || !path_prefix || !n_out || !n_files || lo > hi || hi > SIEVE_MAX_HI)
        return sieve::rt::set_err(ctx, SIEVE_E_INVAL);
    if (elem_bytes != 4 && elem_bytes != 8)
        return sieve::rt::set_err(ctx, SIEVE_E_DTYPE);
    if (elem_bytes == 4 && hi > (1ull << 32))
        return sieve::rt::set_err(ctx, SIEVE_E_DTYPE);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sieve::rt::set_err(ctx, SIEVE_E_DEVICE);
    const uint64_t ppf = primes_per_file ? primes_per_file : kDefaultPrimesPerFile;
    const int el = elem_bytes;
    // File state, touched only by the sink tasks, which run one after another.
    struct Files {
        std::string prefix;
        FILE *f = nullptr;
        uint64_t in_file = 0, count = 0;
    } fs;
    fs.prefix = path_prefix;
    Sink sink = [&fs, ppf, el](const unsigned char *p, uint64_t, uint64_t n) -> int {
        while (n) {
            if (!fs.f) {
                char suffix[32];
                snprintf(suffix, sizeof suffix, ".%06llu", (unsigned long long)fs.count);
                fs.f = fopen((fs.prefix + suffix).c_str(), "wb");
                if (!fs.f)
                    return SIEVE_E_IO;
                ++fs.count;
                fs.in_file = 0;
            }
            const uint64_t k = std::min(n, ppf - fs.in_file);
            if (fwrite(p, el, k, fs.f) != k)
                return SIEVE_E_IO;
            p += k * el;
            n -= k;
            fs.in_file += k;
            if (fs.in_file == ppf) {
                if (fclose(fs.f) != 0) {
                    fs.f = nullptr;
                    return SIEVE_E_IO;
                }
                fs.f = nullptr;
            }
        }
        return SIEVE_OK;
    };
    *n_out = 0;
    int st = stream_range(ctx, lo, hi, el, piece_elems ? piece_elems : kDefaultPieceElems, nullptr, UINT64_MAX,
                          sink, n_out);
    if (fs.f && fclose(fs.f) != 0 && st == SIEVE_OK)
        st = SIEVE_E_IO;
    *n_files = fs.count;
    return sieve::rt::set_err(ctx, st);
}

}  // extern "C"
