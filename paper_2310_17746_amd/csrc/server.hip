// Serving engine: continuous batching of range queries over one context.
//
// A scheduler thread owns the context.  Requests arrive (immediately, or at
// a scheduled time on the server clock), wait in FIFO order, and are admitted
// while slots are free and, for list requests, while their bounded output
// fits the device output arena.  Each step cuts every active request into a
// tile-aligned piece (up to quantum_tiles tiles, round-robin, step_tiles in
// all) and runs the pieces as one batched job.  Tile-aligned pieces of
// [lo, hi) are themselves ranges whose tiles coincide with the request's own
// tiles, so counts add up and list pieces concatenate in order: a request's
// result equals the stand-alone result for its range.
//
// With overlap on, steps are pipelined: step k + 1 is planned on the host
// and enqueued as a stream-ordered job while step k runs, and only then are
// step k's results applied.  A list request has at most one piece in flight
// (its next piece's output offset is the count so far); count requests take
// a piece in every step.  Off (the default), each step's job finishes before
// the next is planned, so a request that arrives during a step joins the
// next one.  Device busy time comes from events around each step's job.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sieve.h"
#include "runtime.h"

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator of byte offsets in the output arena (256-byte grains),
// with coalescing of freed neighbours.
class Arena {
public:
    void init(uint64_t size)
    {
        size_ = size;
        free_.clear();
        if (size)
            free_[0] = size;
        used_ = peak_ = 0;
    }
    bool alloc(uint64_t n, uint64_t &off)
    {
        n = (n + 255) / 256 * 256;
        if (n == 0)
            n = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const uint64_t rest = it->second - n;
                free_.erase(it);
                if (rest)
                    free_[off + n] = rest;
                used_ += n;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        n = (n + 255) / 256 * 256;
        if (n == 0)
            n = 256;
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t peak() const { return peak_; }

private:
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

// Two device buffers of bucket walk state (one read, one written by a piece)
// for one request at a time, in one allocation; pooled by the server.
struct WalkBuf {
    sieve::WalkState *p[2] = {nullptr, nullptr};
    uint32_t cap = 0;  // states per buffer
};

struct Request {
    uint64_t tag = 0, lo = 0, hi = 0;
    int mode = 0;
    uint64_t t_arr = 0, t_admit = 0;
    uint64_t ntiles = 0, base = 0;
    uint32_t last_words = 0;
    uint64_t next_tile = 0;   // first tile not yet handed to a step
    uint64_t tiles_done = 0;  // tiles of the pieces whose results are in
    uint32_t inflight = 0;    // pieces in enqueued steps
    uint32_t issued = 0;      // pieces handed out so far
    int err = SIEVE_OK;       // first failed piece's status
    void *uout = nullptr;     // caller's output (sieve_submit_out), else the arena
    bool over = false;        // caller's output too small: counting the rest only
    uint64_t count = 0;
    uint64_t off_bytes = 0, cap_elems = 0, arena_bytes = 0;
    bool has_arena = false;
    bool cancelled = false;
    // Resident bucket walk state (a request cut into several pieces): the
    // previous piece's end state is in wb->p[wcur] for wn primes from the
    // bucket sieve's first prime wkl on; wn = 0: none.
    WalkBuf *wb = nullptr;
    uint32_t wcur = 0, wn = 0, wkl = 0;
};

struct Finished {
    uint64_t off_bytes, arena_bytes, count;
};

}  // namespace

struct sieve_server {
    sieve_ctx *ctx = nullptr;
    sieve_server_params p{};
    unsigned char *arena_base = nullptr;
    Arena arena;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::multimap<uint64_t, Request *> inbox;  // by arrival time
    std::deque<Request *> pending;             // arrived, FIFO
    std::vector<Request *> active;
    std::deque<sieve_completion> done;
    std::unordered_map<uint64_t, Request *> live;  // queued or active, by tag
    std::unordered_map<uint64_t, Finished> results;
    std::vector<WalkBuf *> wfree, wall;  // walk-state buffers: free ones, all
    size_t rr = 0;
    bool stop = false;
    std::thread th;

    sieve_server_stats st{};

    uint64_t now() const
    {
        return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
    }
};

namespace {

void complete_locked(sieve_server *s, Request *r, int status, uint64_t t)
{
    sieve_completion c;
    memset(&c, 0, sizeof c);
    c.tag = r->tag;
    c.count = r->count;
    c.lo = r->lo;
    c.hi = r->hi;
    c.t_arrival_ns = r->t_arr;
    c.t_admit_ns = r->t_admit;
    c.t_done_ns = t;
    c.status = status;
    c.mode = r->mode;
    s->done.push_back(c);
    s->live.erase(r->tag);
    if (r->wb)
        s->wfree.push_back(r->wb);
    if (r->has_arena) {
        if (status == SIEVE_OK && r->mode)
            s->results[r->tag] = Finished{r->off_bytes, r->arena_bytes, r->count};
        else
            s->arena.release(r->off_bytes, r->arena_bytes);
    }
    s->st.completed++;
    delete r;
}

// One scheduler step: the pieces of one batched job, their results, and
// events around the job on the context stream.
struct Step {
    std::vector<uint64_t> lo, hi, off, cap, counts;
    std::vector<uint8_t> mode;
    std::vector<int32_t> status;
    std::vector<std::pair<Request *, uint64_t>> pieces;  // request, tiles taken
    std::vector<uint8_t> linked;  // piece continues its request's bucket walks
    std::vector<sieve::rt::WalkSpec> ws;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool in_flight = false, timed = false;
    int rc = SIEVE_OK;
    bool buckets = false;  // the step's job ran the bucket sieve
};

bool request_done(const Request *r)
{
    return r->ntiles == 0 ? r->issued > 0 : r->tiles_done >= r->ntiles;
}

// Whether r lists its next piece (a caller's buffer found too small turns
// the rest of the request into counting).
bool listing(const Request *r) { return r->mode && !r->over; }

// Whether r may take a piece in the step being planned.
bool plannable(const Request *r)
{
    if (r->cancelled || r->err != SIEVE_OK || (listing(r) && r->inflight))
        return false;
    return r->ntiles == 0 ? r->issued == 0 : r->next_tile < r->ntiles;
}

// Applies a finished step's results and completes the requests it ends.
void apply_step(sieve_server *s, Step &st)
{
    float ms = 0;
    const bool have_ms = st.timed && hipEventElapsedTime(&ms, st.ev0, st.ev1) == hipSuccess;
    const uint64_t te = s->now();
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.steps++;
    if (have_ms)
        s->st.busy_ns += (uint64_t)((double)ms * 1e6);
    if (st.buckets)
        s->st.bucket_steps++;
    for (size_t i = 0; i < st.pieces.size(); ++i) {
        Request *r = st.pieces[i].first;
        r->inflight--;
        const int stt = st.rc != SIEVE_OK ? st.rc : st.status[i];
        s->st.tiles += st.pieces[i].second;
        s->st.ints += st.hi[i] - st.lo[i];
        if (stt == SIEVE_OK || (stt == SIEVE_E_CAPACITY && r->uout)) {
            // (a piece that overflowed the caller's buffer still counted all
            // of its primes; the request goes on counting)
            r->count += st.counts[i];
            r->tiles_done += st.pieces[i].second;
            r->over = r->over || stt == SIEVE_E_CAPACITY;
        } else if (r->err == SIEVE_OK) {
            r->err = stt;
        }
        if (r->inflight)
            continue;
        int fin = 1;  // 1: not finished
        if (r->err != SIEVE_OK)
            fin = r->err;
        else if (request_done(r))
            fin = r->over ? SIEVE_E_CAPACITY : SIEVE_OK;
        else if (r->cancelled)
            fin = SIEVE_E_CANCELLED;
        if (fin != 1) {
            s->active.erase(std::find(s->active.begin(), s->active.end(), r));
            complete_locked(s, r, fin, te);
        }
    }
    st.in_flight = false;
    st.pieces.clear();
    s->cv_done.notify_all();
}

// Waits for an enqueued step and applies it.
void finish_step(sieve_server *s, Step &st)
{
    if (!st.in_flight)
        return;
    if (st.timed && hipEventSynchronize(st.ev1) != hipSuccess) {
        (void)hipGetLastError();
        if (st.rc == SIEVE_OK)
            st.rc = SIEVE_E_DEVICE;
    }
    apply_step(s, st);
}

// Walk-state buffers of at least `need` states per buffer for r: its own,
// a free pooled pair, or a new one (NULL when the device has no memory).
WalkBuf *walk_buffers(sieve_server *s, Request *r, uint32_t need)
{
    if (r->wb && r->wb->cap >= need)
        return r->wb;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (r->wb) {
            s->wfree.push_back(r->wb);  // too small: back to the pool
            r->wb = nullptr;
            r->wn = 0;
        }
        for (size_t i = 0; i < s->wfree.size(); ++i) {
            if (s->wfree[i]->cap >= need) {
                r->wb = s->wfree[i];
                s->wfree.erase(s->wfree.begin() + i);
                return r->wb;
            }
        }
    }
    WalkBuf *b = new (std::nothrow) WalkBuf();
    if (!b)
        return nullptr;
    b->cap = need + need / 4;
    if (hipMalloc((void **)&b->p[0], 2 * (size_t)b->cap * sizeof(sieve::WalkState)) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return nullptr;
    }
    b->p[1] = b->p[0] + b->cap;  // one allocation holds both buffers
    std::lock_guard<std::mutex> lk(s->mu);
    s->wall.push_back(b);
    s->st.walk_bytes += 2ull * b->cap * sizeof(sieve::WalkState);
    r->wb = b;
    return b;
}

void scheduler(sieve_server *s)
{
    sieve_ctx *c = s->ctx;
    (void)hipSetDevice(c->device);
    const uint32_t pw = c->prm.segment_bytes / 8;
    const uint64_t S = 192ull * pw;  // integers per tile
    const uint32_t eb = s->p.elem_bytes;
    Step steps[2];
    for (Step &st : steps) {
        if (hipEventCreate(&st.ev0) != hipSuccess || hipEventCreate(&st.ev1) != hipSuccess)
            (void)hipGetLastError();
    }
    int cur = 0;  // steps[cur] is planned next; steps[cur ^ 1] may be in flight

    for (;;) {
        uint64_t need_limit = 0;
        Step &st = steps[cur];
        Step &prev = steps[cur ^ 1];
        bool quit = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (s->stop) {
                    quit = true;
                    break;
                }
                const uint64_t t = s->now();
                while (!s->inbox.empty() && s->inbox.begin()->first <= t) {
                    s->pending.push_back(s->inbox.begin()->second);
                    s->inbox.erase(s->inbox.begin());
                }
                // Admission: FIFO, by free slots and output arena.
                while (!s->pending.empty() && s->active.size() < s->p.max_active) {
                    Request *r = s->pending.front();
                    if (r->cancelled) {
                        s->pending.pop_front();
                        complete_locked(s, r, SIEVE_E_CANCELLED, t);
                        continue;
                    }
                    if (r->mode && !r->uout) {
                        r->cap_elems = sieve_list_bound(r->lo, r->hi);
                        r->arena_bytes = std::max<uint64_t>(r->cap_elems * eb, 1);
                        if (r->arena_bytes > s->p.out_budget_bytes) {
                            s->pending.pop_front();
                            complete_locked(s, r, SIEVE_E_NOMEM, t);
                            continue;
                        }
                        if (!s->arena.alloc(r->arena_bytes, r->off_bytes))
                            break;  // head of line waits for memory
                        r->has_arena = true;
                    }
                    r->t_admit = t;
                    s->pending.pop_front();
                    s->active.push_back(r);
                    if (r->hi > 4)
                        need_limit = std::max(need_limit, sieve::rt::isqrt_host(r->hi - 1));
                }
                // Drop cancelled active requests that have no piece in flight.
                for (size_t i = 0; i < s->active.size();) {
                    Request *r = s->active[i];
                    if (r->cancelled && r->inflight == 0) {
                        complete_locked(s, r, SIEVE_E_CANCELLED, t);
                        s->active.erase(s->active.begin() + i);
                    } else {
                        ++i;
                    }
                }
                bool work = false;
                for (const Request *r : s->active)
                    work = work || plannable(r);
                if (work || prev.in_flight)
                    break;
                s->cv_done.notify_all();
                if (!s->inbox.empty()) {
                    const uint64_t wake = s->inbox.begin()->first;
                    s->cv_work.wait_for(lk, std::chrono::nanoseconds(wake > t ? wake - t : 0));
                } else {
                    s->cv_work.wait(lk);
                }
            }
            if (!quit) {
                // Plan one step: round-robin pieces of the plannable requests.
                st.lo.clear();
                st.hi.clear();
                st.off.clear();
                st.cap.clear();
                st.mode.clear();
                st.pieces.clear();
                st.linked.clear();
                uint64_t budget = s->p.step_tiles;
                const size_t n = s->active.size();
                for (size_t k = 0; k < n && budget; ++k) {
                    Request *r = s->active[(s->rr + k) % n];
                    if (!plannable(r))
                        continue;
                    // a request without wheel values takes one tile-less piece (2 and 3)
                    const uint64_t left = r->ntiles - r->next_tile;
                    const uint64_t take =
                        r->ntiles == 0 ? 0 : std::min<uint64_t>(std::min<uint64_t>(left, s->p.quantum_tiles), budget);
                    const uint64_t k0 = r->next_tile, k1 = k0 + take;
                    st.lo.push_back(k0 == 0 ? r->lo : r->base + k0 * S);
                    st.hi.push_back(r->ntiles == 0 || k1 == r->ntiles ? r->hi : r->base + k1 * S);
                    // list pieces write at absolute element addresses (the job's
                    // output base is NULL): the arena or the caller's buffer
                    const bool lst = listing(r);
                    const uint64_t dst = (uint64_t)(uintptr_t)(r->uout ? (unsigned char *)r->uout
                                                                       : s->arena_base + r->off_bytes);
                    st.mode.push_back((uint8_t)lst);
                    st.off.push_back(lst ? dst / eb + r->count : 0);
                    st.cap.push_back(lst ? r->cap_elems - r->count : 0);
                    st.pieces.emplace_back(r, take);
                    // A request cut into pieces continues its bucket walks
                    // from piece to piece when nothing of it is in flight
                    // (else its chain of states starts over).
                    const bool link = !s->p.restart_walks && take < r->ntiles && r->inflight == 0;
                    st.linked.push_back(link ? 1 : 0);
                    if (!link)
                        r->wn = 0;
                    r->next_tile = k1;
                    r->inflight++;
                    r->issued++;
                    budget -= take;
                }
                s->rr = n ? (s->rr + 1) % n : 0;
            }
        }
        if (quit) {
            // Let enqueued work end before the context is handed back.
            finish_step(s, prev);
            break;
        }
        const uint64_t m = st.lo.size();
        st.rc = SIEVE_OK;
        if (need_limit > c->limit) {
            // The base primes are re-installed: no step may be reading them.
            finish_step(s, prev);
            st.rc = sieve::rt::grow_base_primes(c, need_limit);
        }
        if (m) {
            st.counts.assign(m, 0);
            st.status.assign(m, 0);
            // Walk links: a linked piece of a request whose ranges reach the
            // bucket sieve reads its previous piece's end state and writes
            // its own (none after the request's last piece).
            bool any_link = false;
            st.ws.assign(m, sieve::rt::WalkSpec{nullptr, nullptr, 0, 0, 0, 0});
            for (uint64_t i = 0; i < m && st.rc == SIEVE_OK; ++i) {
                Request *r = st.pieces[i].first;
                if (!st.linked[i] || r->hi <= 4)
                    continue;
                const uint32_t nact = sieve::rt::primes_upto(c, sieve::rt::isqrt_host(r->hi - 1));
                if (nact <= c->k_large)
                    continue;  // no prime of the request reaches the bucket sieve
                WalkBuf *b = walk_buffers(s, r, nact - c->k_large);
                if (!b)
                    continue;
                sieve::rt::WalkSpec &w = st.ws[i];
                if (r->wn && r->wkl == c->k_large) {
                    w.src = b->p[r->wcur];
                    w.nsrc = r->wn;
                }
                if (r->next_tile < r->ntiles) {
                    w.dst = b->p[r->wcur ^ 1];
                    w.dcap = b->cap;
                }
                any_link = true;
            }
            const uint64_t bj = c->bucket_jobs;
            if (prev.in_flight) {
                std::lock_guard<std::mutex> lk(s->mu);
                s->st.overlap_steps++;
            }
            st.timed = st.ev0 && st.ev1 && hipEventRecord(st.ev0, c->stream) == hipSuccess;
            if (st.rc == SIEVE_OK)
                st.rc = sieve::rt::run_job(c, m, st.lo.data(), st.hi.data(), st.mode.data(), st.off.data(),
                                           st.cap.data(), (int)eb, nullptr, st.counts.data(),
                                           st.status.data(), c->stream, c->prm.use_graph != 0,
                                           s->p.overlap != 0, any_link ? st.ws.data() : nullptr);
            st.buckets = c->bucket_jobs != bj;
            // A job that ran the bucket sieve has finished when run_job
            // returns: the states it stored become the next pieces' sources.
            uint64_t resumed = 0;
            for (uint64_t i = 0; i < m; ++i) {
                if (!st.linked[i])
                    continue;
                Request *r = st.pieces[i].first;
                if (st.rc == SIEVE_OK && st.ws[i].saved) {
                    r->wcur ^= 1;
                    r->wn = st.ws[i].saved;
                    r->wkl = c->k_large;
                } else {
                    r->wn = 0;
                }
                resumed += st.rc == SIEVE_OK ? st.ws[i].resumed : 0u;
            }
            if (resumed) {
                std::lock_guard<std::mutex> lk(s->mu);
                s->st.resumed_walks += resumed;
            }
            st.timed = st.timed && hipEventRecord(st.ev1, c->stream) == hipSuccess;
            if (!st.timed)
                (void)hipStreamSynchronize(c->stream);
            st.in_flight = true;
            if (!s->p.overlap)
                finish_step(s, st);
        }
        // The previous step ends while this one waits behind it on the device.
        finish_step(s, prev);
        cur ^= 1;
    }
    for (Step &st : steps) {
        if (st.ev0)
            (void)hipEventDestroy(st.ev0);
        if (st.ev1)
            (void)hipEventDestroy(st.ev1);
    }
}

int submit(sieve_server *s, uint64_t lo, uint64_t hi, int mode, uint64_t tag, bool at, uint64_t t_arr,
           void *uout = nullptr, uint64_t ucap = 0)
{
    if (!s || lo > hi || hi > SIEVE_MAX_HI || (mode != 0 && mode != 1))
        return SIEVE_E_INVAL;
    if (mode && uout && (uintptr_t)uout % s->p.elem_bytes)
        return SIEVE_E_INVAL;
    if (mode && s->p.elem_bytes == 4 && hi > lo && hi - 1 > 0xFFFFFFFFull)
        return SIEVE_E_DTYPE;
    if (hi > 4 && sieve::rt::isqrt_host(hi - 1) >= (1ull << 32))
        return SIEVE_E_RANGE;
    Request *r = new (std::nothrow) Request();
    if (!r)
        return SIEVE_E_NOMEM;
    r->tag = tag;
    r->lo = lo;
    r->hi = hi;
    r->mode = mode;
    if (mode && uout) {
        r->uout = uout;
        r->cap_elems = ucap;
    }
    sieve::rt::plan_range(lo, hi, s->ctx->prm.segment_bytes / 8, r->ntiles, r->base, r->last_words);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->live.count(tag) || s->results.count(tag)) {
            delete r;
            return SIEVE_E_INVAL;
        }
        if (s->inbox.size() + s->pending.size() >= s->p.max_queue) {
            delete r;
            return SIEVE_E_BUSY;
        }
        r->t_arr = at ? t_arr : s->now();
        s->live[tag] = r;
        s->inbox.emplace(r->t_arr, r);
    }
    s->cv_work.notify_one();
    return SIEVE_OK;
}

}  // namespace

extern "C" {

int sieve_server_create(sieve_ctx *ctx, const sieve_server_params *p, sieve_server **out)
{
    if (!ctx || !out)
        return SIEVE_E_INVAL;
    *out = nullptr;
    sieve_server_params q;
    memset(&q, 0, sizeof q);
    if (p)
        q = *p;
    if (!q.out_budget_bytes)
        q.out_budget_bytes = 1ull << 30;
    if (!q.max_active)
        q.max_active = 1024;
    if (!q.step_tiles)
        q.step_tiles = 16u * (uint32_t)ctx->cus;
    if (!q.quantum_tiles)
        q.quantum_tiles = std::max<uint32_t>(1, q.step_tiles / 16);
    if (!q.elem_bytes)
        q.elem_bytes = 8;
    if (!q.max_queue)
        q.max_queue = 1u << 20;
    if (q.elem_bytes != 4 && q.elem_bytes != 8)
        return SIEVE_E_DTYPE;
    sieve_server *s = new (std::nothrow) sieve_server();
    if (!s)
        return SIEVE_E_NOMEM;
    s->ctx = ctx;
    s->p = q;
    if (hipSetDevice(ctx->device) != hipSuccess ||
        hipMalloc((void **)&s->arena_base, q.out_budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return SIEVE_E_NOMEM;
    }
    s->arena.init(q.out_budget_bytes);
    s->t0 = Clock::now();
    try {
        s->th = std::thread(scheduler, s);
    } catch (...) {
        (void)hipFree(s->arena_base);
        delete s;
        return SIEVE_E_NOMEM;
    }
    *out = s;
    return SIEVE_OK;
}

int sieve_submit(sieve_server *srv, uint64_t lo, uint64_t hi, int mode, uint64_t tag)
{
    return submit(srv, lo, hi, mode, tag, false, 0);
}

int sieve_submit_at(sieve_server *srv, uint64_t lo, uint64_t hi, int mode, uint64_t tag, uint64_t t_arrival_ns)
{
    return submit(srv, lo, hi, mode, tag, true, t_arrival_ns);
}

int sieve_submit_out(sieve_server *srv, uint64_t lo, uint64_t hi, int mode, void *out_dev, uint64_t cap,
                     uint64_t tag)
{
    if (mode && !out_dev)
        return SIEVE_E_INVAL;
    return submit(srv, lo, hi, mode, tag, false, 0, out_dev, cap);
}

int sieve_poll(sieve_server *srv, sieve_completion *buf, int max, int wait_ms, int *n_out)
{
    if (!srv || !n_out || max < 0 || (max && !buf))
        return SIEVE_E_INVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && wait_ms > 0)
        srv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !srv->done.empty(); });
    int n = 0;
    while (n < max && !srv->done.empty()) {
        buf[n++] = srv->done.front();
        srv->done.pop_front();
    }
    *n_out = n;
    return SIEVE_OK;
}

int sieve_cancel(sieve_server *srv, uint64_t tag)
{
    if (!srv)
        return SIEVE_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->live.find(tag);
        if (it == srv->live.end())
            return SIEVE_E_INVAL;
        Request *r = it->second;
        r->cancelled = true;
        // Not yet arrived: complete it here.
        for (auto jt = srv->inbox.begin(); jt != srv->inbox.end(); ++jt) {
            if (jt->second == r) {
                srv->inbox.erase(jt);
                complete_locked(srv, r, SIEVE_E_CANCELLED, srv->now());
                srv->cv_done.notify_all();
                return SIEVE_OK;
            }
        }
    }
    srv->cv_work.notify_one();
    return SIEVE_OK;
}

int sieve_server_fetch(sieve_server *srv, uint64_t tag, void *dst, uint64_t cap, uint64_t *n_out)
{
    if (!srv || !n_out)
        return SIEVE_E_INVAL;
    Finished f;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->results.find(tag);
        if (it == srv->results.end())
            return SIEVE_E_INVAL;
        f = it->second;
        *n_out = f.count;
        if (f.count > cap)
            return SIEVE_E_CAPACITY;
        if (f.count && !dst)
            return SIEVE_E_INVAL;
    }
    if (f.count) {
        (void)hipSetDevice(srv->ctx->device);
        if (hipMemcpy(dst, srv->arena_base + f.off_bytes, f.count * srv->p.elem_bytes, hipMemcpyDefault) !=
            hipSuccess) {
            (void)hipGetLastError();
            return SIEVE_E_DEVICE;
        }
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->results.erase(tag);
        srv->arena.release(f.off_bytes, f.arena_bytes);
    }
    srv->cv_work.notify_one();  // memory freed: admission may proceed
    return SIEVE_OK;
}

int sieve_server_release(sieve_server *srv, uint64_t tag)
{
    if (!srv)
        return SIEVE_E_INVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->results.find(tag);
    if (it == srv->results.end())
        return SIEVE_E_INVAL;
    srv->arena.release(it->second.off_bytes, it->second.arena_bytes);
    srv->results.erase(it);
    srv->cv_work.notify_one();  // memory freed: admission may proceed
    return SIEVE_OK;
}

int sieve_server_get_stats(sieve_server *srv, sieve_server_stats *st)
{
    if (!srv || !st)
        return SIEVE_E_INVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *st = srv->st;
    st->elapsed_ns = srv->now();
    st->arena_peak_bytes = srv->arena.peak();
    st->queued = srv->inbox.size() + srv->pending.size();
    st->active = srv->active.size();
    return SIEVE_OK;
}

uint64_t sieve_server_now_ns(const sieve_server *srv) { return srv ? srv->now() : 0; }

int sieve_server_destroy(sieve_server *srv)
{
    if (!srv)
        return SIEVE_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->th.joinable())
        srv->th.join();
    for (auto &kv : srv->inbox)
        delete kv.second;
    for (Request *r : srv->pending)
        delete r;
    for (Request *r : srv->active)
        delete r;
    (void)hipSetDevice(srv->ctx->device);
    for (WalkBuf *b : srv->wall) {
        (void)hipFree(b->p[0]);
        delete b;
    }
    if (srv->arena_base) {
        (void)hipSetDevice(srv->ctx->device);
        (void)hipFree(srv->arena_base);
    }
    delete srv;
    return SIEVE_OK;
}

}  // extern "C"
