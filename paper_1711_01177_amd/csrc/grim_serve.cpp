// Continuous-batching server for GRIM-Filter requests.
//
// Requests are host batches (reads + candidate locations).  At submit the
// request's arrays are copied once, into a block of a pinned host arena
// allocated when the server is created (pageable memory only when the arena is
// full), with room for its results; in-place submission uses the caller's
// pinned arrays directly.
//
// Threads.  One admission thread and one worker per slot; each of the
// n_streams streams carries the ticks of ticks_per_stream slots.
//   - The admission thread, while a slot is free, admits queued requests in
//     arrival order while their device bytes fit in what is left of the HBM
//     budget and the tick has fewer than max_tick_pairs pairs, reserves the
//     tick's device memory, and hands the tick to the slot's worker.
//   - The slot's worker stages the tick and queues it on the slot's stream:
//     H2D copies (large array slices straight from the request's pinned
//     memory, small slices packed through the slot's staging buffer, re-based
//     per-read arrays always staged), the batched filter, D2H copies (large
//     count slices straight into the request's result area) and a completion
//     notice.  When the notice arrives it retires the tick: copies the small
//     count slices and realigns each request's slice of the fused pass bits,
//     then closes the parts, frees the device memory and rings the admission
//     thread.
// Staging and retirement of different ticks run on different host threads.
// Ticks on different streams overlap on the device: one tick's inputs go up
// while another's results come down.  Two policies keep the host link busy, one
// per kind of result (both chosen by measurement on the full-size workload):
//   - counts and pass bits (both directions of the link loaded): upload turns.
//     A tick queues its input copies only when the tick before it at the gate
//     has its inputs on the device (a notice queued behind them ends the turn),
//     so uploads run one at a time at the link's full rate and the ticks reach
//     their filters and result copies staggered, instead of all streams moving
//     their data in the same direction at once.  A tick joins the gate only
//     once the ticks before it on its own stream have completed: its uploads
//     would otherwise wait behind that stream's downloads while holding the
//     turn;
//   - pass bits only (the upload direction alone loaded): no turns.
// Either way two slots per stream by default, so that a stream's next tick is
// staged and queued while its current one runs and the host retires the one
// before.
// Uploads and downloads overlap only on streams served by different copy
// engines, which the runtime assigns out of the server's control: at create the
// server times candidate streams, keeps streams of both engines when it finds
// two and puts consecutive ticks on alternate engines; when every candidate
// shares one engine, downloads of counts go by a kernel storing into the
// page-locked host memory instead (grim_copy.hip), which needs no engine.
//
// A request with more pairs than a tick has room for is admitted in parts, cut
// at read boundaries; its parts run as separate ticks on the free streams, so
// one part's H2D copy overlaps another part's filter and D2H copy, and the
// request is done when its last part has been retired.  Two parts of one
// request can share a pass-bit word at their boundary; workers merge such
// words with an atomic OR and store the words wholly inside a part.
//
// Fusing and splitting only concatenate, cut and re-base offsets, and every
// pair is computed by the same kernel from the same read and bin, so each
// request's counts and pass bits are identical to filtering it alone.
//
// The scheduler makes no HIP call itself: device memory, streams, copies, the
// filter launch and completion notices go through grim_serve::backend()
// (grim_serve_backend.h).  A tick's completion notice is a host function
// queued on its stream after its last copy; it wakes the slot's worker.
// Submissions, retired ticks and shutdown ring the admission thread's
// doorbell, the only thing it waits on, so nothing polls.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "grim.h"
#include "grim_serve_backend.h"

using grim_serve::backend;

namespace {

using Clock = std::chrono::steady_clock;

inline uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// Slices at least this large move by DMA straight from / to the request's
// block; smaller ones are packed through the slot's staging buffer.
constexpr uint64_t kDirectBytes = 256 << 10;

// memcpy split over a few threads for large copies (host staging is the
// bottleneck of served latency for big requests).
void par_memcpy(void *dst, const void *src, uint64_t n)
{
    constexpr uint64_t kChunk = 8ull << 20;
    if (n < 2 * kChunk) {
        if (n)
            std::memcpy(dst, src, n);
        return;
    }
    const int nt = (int)std::min<uint64_t>(8, n / kChunk);
    const uint64_t step = (n + nt - 1) / nt;
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) {
        const uint64_t a = t * step, b = std::min(n, a + step);
        if (a < b)
            th.emplace_back([=] {
                std::memcpy(static_cast<char *>(dst) + a, static_cast<const char *>(src) + a, b - a);
            });
    }
    std::memcpy(dst, src, std::min(n, step));
    for (auto &x : th)
        x.join();
}

// First-fit allocator over a byte range (offsets, 256-byte units).
class Pool {
public:
    explicit Pool(uint64_t size) { free_[0] = size; }
    bool alloc(uint64_t n, uint64_t *off)
    {
        n = align256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest)
                    free_[start] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        n = align256(n);
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
    uint64_t used() const { return used_; }

private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t used_ = 0;
};

enum class State { Queued, Running, Done };

// Host-side layout of one request's block: inputs, then result area.
struct ReqLayout {
    uint64_t words, read_off, read_len, read_e, cand_off, cand_bin, counts, bits, total;
};

ReqLayout req_layout(uint64_t n_words, uint64_t n_reads, uint64_t n_pairs)
{
    ReqLayout L;
    uint64_t o = 0;
    L.words = o;
    o = align256(o + n_words * 4);
    L.read_off = o;
    o = align256(o + n_reads * 8);
    L.read_len = o;
    o = align256(o + n_reads * 4);
    L.read_e = o;
    o = align256(o + n_reads * 4);
    L.cand_off = o;
    o = align256(o + (n_reads + 1) * 8);
    L.cand_bin = o;
    o = align256(o + n_pairs * 4);
    L.counts = o;
    o = align256(o + n_pairs * 4);
    L.bits = o;
    o = align256(o + ((n_pairs + 31) / 32) * 4 + 4);
    L.total = o;
    return L;
}

struct Request {
    uint64_t ticket = 0;
    uint8_t *host = nullptr;       // block with inputs and results (null when in place)
    bool pinned = false;           // block lives in the server's pinned arena
    bool in_place = false;         // caller-owned arrays used directly
    bool counts_writable = false;  // the device can store into the result counts directly
    uint64_t arena_off = 0;
    ReqLayout lay{};
    uint64_t n_words = 0, n_reads = 0, n_pairs = 0;
    uint32_t e_den = 0;
    State state = State::Queued;
    bool cancelled = false;
    int status = GRIM_OK;
    uint32_t flags = 0;
    uint64_t tick = 0;
    uint64_t next_read = 0;        // first read not yet admitted to a tick
    bool all_admitted = false;     // every read is in a tick (or the request was dropped)
    uint32_t parts_open = 0;       // admitted parts whose tick has not been retired
    Clock::time_point t_submit, t_admit, t_done;
    // views of the inputs and the result area
    const uint32_t *p_words = nullptr;
    const uint64_t *p_read_off = nullptr, *p_cand_off = nullptr;
    const uint32_t *p_read_len = nullptr, *p_read_e = nullptr, *p_cand_bin = nullptr;
    int32_t *p_counts = nullptr;
    uint32_t *p_bits = nullptr;
    uint64_t zero_off = 0;         // cand_off of a request without reads

    const uint32_t *words() const { return p_words; }
    const uint64_t *read_off() const { return p_read_off; }
    const uint32_t *read_len() const { return p_read_len; }
    const uint32_t *read_e() const { return p_read_e; }
    const uint64_t *cand_off() const { return p_cand_off ? p_cand_off : &zero_off; }
    const uint32_t *cand_bin() const { return p_cand_bin; }
    int32_t *counts() const { return p_counts; }
    uint32_t *bits() const { return p_bits; }
    void view_block()
    {
        p_words = reinterpret_cast<const uint32_t *>(host + lay.words);
        p_read_off = reinterpret_cast<const uint64_t *>(host + lay.read_off);
        p_read_len = reinterpret_cast<const uint32_t *>(host + lay.read_len);
        p_read_e = reinterpret_cast<const uint32_t *>(host + lay.read_e);
        p_cand_off = reinterpret_cast<const uint64_t *>(host + lay.cand_off);
        p_cand_bin = reinterpret_cast<const uint32_t *>(host + lay.cand_bin);
        p_counts = reinterpret_cast<int32_t *>(host + lay.counts);
        p_bits = reinterpret_cast<uint32_t *>(host + lay.bits);
    }
};

// Byte layout of one fused tick on the device (and in the staging buffer).
// The per-read arrays come first (always staged: one copy), then the packed
// words and the bin ids; the outputs are counts, pass bits and the filter's
// workspace, whose first word is the launch's status word, so that the pass
// bits and the status come back in one copy.
struct Layout {
    uint64_t read_off, cand_off, read_len, read_e, meta_bytes;  // per-read arrays
    uint64_t words, cand_bin, in_bytes;                         // inputs
    uint64_t out_base;
    uint64_t counts, bits, ws, out_bytes;  // outputs, relative to `out_base`
    uint64_t ws_bytes;
    uint64_t total;
};

Layout plan(uint64_t n_words, uint64_t n_reads, uint64_t n_pairs, uint64_t ws_bytes)
{
    Layout L;
    uint64_t o = 0;
    L.read_off = o;
    o = align256(o + n_reads * 8);
    L.cand_off = o;
    o = align256(o + (n_reads + 1) * 8);
    L.read_len = o;
    o = align256(o + n_reads * 4);
    L.read_e = o;
    o = align256(o + n_reads * 4);
    L.meta_bytes = o;
    L.words = o;
    o = align256(o + n_words * 4);
    L.cand_bin = o;
    o = align256(o + n_pairs * 4);
    L.in_bytes = o;
    L.out_base = o;
    L.counts = 0;
    L.bits = align256(n_pairs * 4);
    L.ws = L.bits + align256(((n_pairs + 31) / 32) * 4 + 4);
    L.ws_bytes = align256(ws_bytes);
    L.out_bytes = L.ws + L.ws_bytes;
    L.total = o + L.out_bytes;
    return L;
}

// One request's reads [ra, rb) (pairs [pa, pb) of the request) inside a tick.
struct Part {
    std::shared_ptr<Request> r;
    uint64_t ra = 0, rb = 0, pa = 0, pb = 0;
    uint64_t wlo = 0, nw = 0;      // the request's packed words the part's reads use
    uint64_t fused_base = 0;       // first pair of the part in the fused tick
    bool counts_direct = false;    // counts came back by direct DMA
};

// One host <-> device copy of a tick (a download by host stores when `store`).
struct CopyOp {
    void *dst;
    const void *src;
    uint64_t bytes;
    bool store = false;
};

struct Slot {
    grim_server *srv = nullptr;
    void *stream = nullptr;        // shared with ticks_per_stream - 1 other slots
    int group = 0;                 // the stream's copy-engine group (0 or 1)
    uint32_t stream_idx = 0;       // index of the stream in the server's list
    uint8_t *stage = nullptr;      // pinned, stage_bytes long, mirrors the tick layout
    // guarded by the server lock; the tick fields below are written by the
    // admission thread while busy is false and belong to the worker from the
    // hand-off until it clears busy
    bool busy = false;
    std::vector<Part> parts;
    Layout lay;
    uint64_t dev_off = 0;
    uint32_t e_den = 0;
    double turn_wait_s = 0;        // the last launch's wait for its upload turn
    // hand-off between the admission thread, the completion notice and the
    // worker (m is never held while taking the server lock or calling the backend)
    std::mutex m;
    std::condition_variable cv;
    bool job = false;              // a tick has been handed over
    bool notice = false;           // the tick's completion notice has run
    bool quit = false;
    std::thread worker;
};

}  // namespace

struct grim_server {
    const grim_index_t *idx = nullptr;
    grim_serve_cfg_t cfg{};
    int device = 0;
    uint8_t *pool_base = nullptr;
    std::unique_ptr<Pool> pool;
    uint8_t *arena = nullptr;          // pinned host arena for request blocks
    uint64_t arena_bytes = 0;
    std::unique_ptr<Pool> arena_pool;
    std::mutex arena_mu;
    std::vector<std::unique_ptr<Slot>> slots;
    uint64_t stage_bytes = 0;          // each slot's staging buffer: the largest tick layout
    std::vector<void *> streams;       // slot i queues its ticks on streams[i % n_streams]
    std::vector<int> stream_group;     // copy-engine group of each stream (0 or 1)
    uint32_t n_groups = 1;             // 2 when the streams were split between two groups
    bool store_downloads = false;      // one group: downloads by host stores, not the copy engine
    int last_group = 1;                // group of the last tick admitted
    // upload turns (taken when results include counts): ticks queue their
    // input copies one at a time, in the order they reach the gate; a turn ends
    // when the tick's inputs are on the device
    bool upload_turns = false;
    std::mutex up_mu;
    std::condition_variable up_cv;
    uint64_t up_next = 0, up_turn = 0;
    // ticks queued on each stream and not yet complete (with upload turns and
    // several ticks per stream, a tick takes a turn only once its stream is
    // free, so that its uploads never wait behind that stream's downloads
    // while they hold the turn); guarded by up_mu
    std::vector<uint32_t> stream_ticks;
    void stream_tick_done(uint32_t stream_idx);
    void upload_turn_end();

    std::mutex mu;
    std::condition_variable cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> all;
    uint64_t next_ticket = 1, next_tick = 1;
    uint64_t inflight_reqs = 0;
    bool stop = false;
    std::thread thr;

    // doorbell: rung by submissions, retired ticks and shutdown; the admission
    // thread sleeps until it changes (bell_mu is never held while taking mu)
    std::mutex bell_mu;
    std::condition_variable bell_cv;
    uint64_t bell = 0;

    // statistics
    uint64_t submitted = 0, completed = 0, cancelled = 0, failed = 0, ticks = 0, pairs_done = 0;
    uint64_t reqs_in_ticks = 0, peak_bytes = 0;
    std::vector<double> lat;
    double busy_s = 0;
    double admit_s = 0;                 // admission thread time forming ticks
    double launch_s = 0, retire_s = 0;  // worker time staging + queuing / retiring, summed
    int running_ticks = 0;
    Clock::time_point busy_since;

    void run();
    void ring();
    bool admit_tick();
    void work(Slot &s);
    int launch(Slot &s);
    void retire(Slot &s, double t_launch);
    void close_tick(Slot &s, int rc, const std::vector<uint32_t> &part_flags, double t_launch,
                    double t_retire);
    void part_closed(Request &r, Clock::time_point now);
    void drop_from_queue(const Request &r);
    void free_block(Request &r);
};

void grim_server::stream_tick_done(uint32_t stream_idx)
{
    {
        std::lock_guard<std::mutex> lk(up_mu);
        --stream_ticks[stream_idx];
    }
    up_cv.notify_all();
}

void grim_server::upload_turn_end()
{
    {
        std::lock_guard<std::mutex> lk(up_mu);
        ++up_turn;
    }
    up_cv.notify_all();
}

void grim_server::ring()
{
    {
        std::lock_guard<std::mutex> bl(bell_mu);
        ++bell;
    }
    bell_cv.notify_one();
}

namespace {

// Notice queued behind a tick's input copies: the next tick's turn to upload.
void on_upload_done(void *arg)
{
    static_cast<Slot *>(arg)->srv->upload_turn_end();
}

// Completion notice of a tick (runs on a backend thread once the tick's last
// copy has completed): wake the slot's worker.
void on_tick_done(void *arg)
{
    Slot *slot = static_cast<Slot *>(arg);
    if (slot->srv->upload_turns)
        slot->srv->stream_tick_done(slot->stream_idx);
    {
        std::lock_guard<std::mutex> lk(slot->m);
        slot->notice = true;
    }
    slot->cv.notify_one();
}

}  // namespace

namespace {

uint64_t ws_need(const grim_index_t *idx, uint64_t n_pairs)
{
    return backend().workspace_bytes(idx, n_pairs);
}

}  // namespace

void grim_server::free_block(Request &r)
{
    if (!r.host)
        return;
    if (r.pinned) {
        std::lock_guard<std::mutex> lk(arena_mu);
        arena_pool->release(r.arena_off, r.lay.total);
    } else {
        std::free(r.host);
    }
    r.host = nullptr;
}

namespace {

// Bits [bit, bit + 32) of src as one word (src readable one word past them).
inline uint32_t word_at(const uint32_t *src, uint64_t bit)
{
    const uint64_t w = bit >> 5;
    const uint32_t sh = (uint32_t)(bit & 31);
    return sh ? (src[w] >> sh) | (src[w + 1] << (32 - sh)) : src[w];
}

// Writes bits [sb, sb + n) of src to bits [db, db + n) of dst.  The bits of dst
// in that range are zero and belong to this call alone, but the first and last
// word may hold bits of a neighbouring part of the same request that another
// worker writes at the same time: those words are merged with an atomic OR, the
// words wholly inside the range are stored.  src must be readable one word past
// its last used bit.
void put_bits(uint32_t *dst, uint64_t db, const uint32_t *src, uint64_t sb, uint64_t n)
{
    const uint64_t end = db + n;
    auto merge = [&](uint64_t d, uint64_t take) {  // `take` bits at d, in one word of dst
        uint32_t x = word_at(src, sb + (d - db));
        if (take < 32)
            x &= (1u << take) - 1u;
        __atomic_fetch_or(&dst[d >> 5], x << (d & 31), __ATOMIC_RELAXED);
    };
    uint64_t d = db;
    if (n && (d & 31)) {
        const uint64_t take = std::min<uint64_t>(32 - (d & 31), n);
        merge(d, take);
        d += take;
    }
    const uint64_t whole_end = end & ~31ull;
    if (d < whole_end) {
        const uint64_t s0 = sb + (d - db);
        const uint64_t k0 = d >> 5, k1 = whole_end >> 5;
        const uint32_t sh = (uint32_t)(s0 & 31);
        const uint32_t *sp = src + (s0 >> 5);
        if (sh == 0) {
            std::memcpy(dst + k0, sp, (k1 - k0) * 4);
        } else {
            for (uint64_t k = k0; k < k1; ++k, ++sp)
                dst[k] = (sp[0] >> sh) | (sp[1] << (32 - sh));
        }
        d = whole_end;
    }
    if (d < end)
        merge(d, end - d);
}

double secs(Clock::duration d) { return std::chrono::duration<double>(d).count(); }

}  // namespace

// A part of r has been retired (or dropped): finish r once nothing of it is
// left in flight and no read waits for admission.  Called with mu held.
void grim_server::part_closed(Request &r, Clock::time_point now)
{
    if (r.parts_open)
        --r.parts_open;
    if (r.parts_open || !r.all_admitted || r.state == State::Done)
        return;
    if (r.cancelled) {
        r.status = GRIM_E_CANCELLED;
        ++cancelled;
    } else if (r.status != GRIM_OK && r.status != GRIM_E_BIN_RANGE) {
        ++failed;
    } else {
        const bool bad = (r.flags & GRIM_FLAG_BIN_RANGE) != 0;
        r.status = bad ? GRIM_E_BIN_RANGE : GRIM_OK;
        if (bad)
            ++failed;
        ++completed;
        pairs_done += r.n_pairs;
        lat.push_back(ms_between(r.t_submit, now));
    }
    r.t_done = now;
    r.state = State::Done;
    --inflight_reqs;
}

void grim_server::drop_from_queue(const Request &r)
{
    for (auto q = queue.begin(); q != queue.end(); ++q)
        if (q->get() == &r) {
            queue.erase(q);
            return;
        }
}

// Ends s's tick under the server lock (worker thread): with rc != GRIM_OK
// every part's request fails and the reads of it still queued are dropped;
// otherwise each part's flags go to its request.  Then the parts are closed,
// the tick's device memory is released, the slot is freed and the admission
// thread is rung.
void grim_server::close_tick(Slot &s, int rc, const std::vector<uint32_t> &part_flags,
                             double t_launch, double t_retire)
{
    {
        std::lock_guard<std::mutex> lk(mu);
        const auto now = Clock::now();
        for (size_t j = 0; j < s.parts.size(); ++j) {
            Request &r = *s.parts[j].r;
            if (rc != GRIM_OK) {
                if (!r.all_admitted) {
                    drop_from_queue(r);
                    r.all_admitted = true;
                }
                r.status = rc;
            } else if (j < part_flags.size()) {
                r.flags |= part_flags[j];
            }
            part_closed(r, now);
        }
        pool->release(s.dev_off, s.lay.total);
        s.parts.clear();
        s.busy = false;
        if (--running_ticks == 0)
            busy_s += secs(now - busy_since);
        launch_s += t_launch;
        retire_s += t_retire;
        cv_done.notify_all();
    }
    ring();
}

// Retires s's tick once its completion notice has run (worker thread).  The
// results go into each request's result area without the server lock: a
// request's area is written only by the workers of its parts until its last
// part is closed, and their bits meet only in shared boundary words.
void grim_server::retire(Slot &s, double t_launch)
{
    const auto t0 = Clock::now();
    const uint8_t *out = s.stage + s.lay.out_base;
    const int32_t *counts = reinterpret_cast<const int32_t *>(out + s.lay.counts);
    const uint32_t *bits = reinterpret_cast<const uint32_t *>(out + s.lay.bits);
    const uint32_t status = *reinterpret_cast<const uint32_t *>(out + s.lay.ws);
    const bool bits_only = (cfg.flags & GRIM_SERVE_PASS_BITS_ONLY) != 0;
    int rc = GRIM_OK;
    if (bits_only && (status & GRIM_FLAG_BIN_RANGE)) {
        // the counts stayed on the device: fetch this tick's to find the -1s
        uint64_t n = 0;
        for (const Part &pt : s.parts)
            n = std::max(n, pt.fused_base + (pt.pb - pt.pa));
        const uint8_t *dout = pool_base + s.dev_off + s.lay.out_base;
        if (backend().copy_d2h(s.stage + s.lay.out_base + s.lay.counts, dout + s.lay.counts,
                               n * 4, s.stream) != GRIM_OK ||
            backend().stream_sync(s.stream) != GRIM_OK)
            rc = GRIM_E_HIP;  // cannot tell which part: fail them all
    }
    std::vector<uint32_t> part_flags(s.parts.size(), 0);
    for (size_t j = 0; j < s.parts.size() && rc == GRIM_OK; ++j) {
        const Part &pt = s.parts[j];
        const Request &r = *pt.r;
        const uint64_t np = pt.pb - pt.pa;
        if (!np)
            continue;
        if (!bits_only && !pt.counts_direct)
            std::memcpy(r.counts() + pt.pa, counts + pt.fused_base, np * 4);
        put_bits(r.bits(), pt.pa, bits, pt.fused_base, np);
        if (status & GRIM_FLAG_BIN_RANGE) {  // only then look for -1 in this part
            const int32_t *c = bits_only ? counts + pt.fused_base : r.counts() + pt.pa;
            for (uint64_t k = 0; k < np; ++k)
                if (c[k] < 0) {
                    part_flags[j] = GRIM_FLAG_BIN_RANGE;
                    break;
                }
        }
    }
    close_tick(s, rc, part_flags, t_launch, secs(Clock::now() - t0));
}

// Forms one tick on a free slot and hands it to the slot's worker.  Returns
// false if nothing could be admitted.  Admission thread, mu held.
bool grim_server::admit_tick()
{
    // a free slot: on a stream with no tick running first (a tick on a busy
    // stream waits for it), then on a stream of the other copy-engine group
    // than the last tick's, so that consecutive ticks' uploads and downloads
    // can run at once
    Slot *slot = nullptr;
    int best = -1;
    for (auto &sp : slots) {
        if (sp->busy)
            continue;
        bool idle = true;
        for (auto &other : slots)
            if (other->busy && other->stream_idx == sp->stream_idx)
                idle = false;
        const int score = (idle ? 2 : 0) + (sp->group != last_group ? 1 : 0);
        if (score > best) {
            best = score;
            slot = sp.get();
        }
    }
    if (!slot || queue.empty())
        return false;
    // admission: requests in arrival order with the e_den of the first one
    // taken, within max_inflight, the tick's pair limit, the free budget and
    // the staging buffer; the request that does not fit whole contributes the
    // reads that do (at least one read when the tick would be empty and its
    // pairs exceed the pair limit) and stays queued.  A request already running
    // in n_streams - 1 parts is passed over, so that one stream always remains
    // for the requests behind it.
    std::vector<Part> take;
    uint64_t words = 0, reads = 0, pairs = 0, new_reqs = 0;
    uint32_t e_den = 0;
    const uint32_t max_parts = slots.size() > 1 ? (uint32_t)slots.size() - 1 : 1u;
    const uint64_t cap = std::min<uint64_t>(cfg.hbm_budget_bytes - pool->used(), stage_bytes);
    for (auto it = queue.begin(); it != queue.end();) {
        std::shared_ptr<Request> rp = *it;
        Request &r = *rp;
        const bool first = r.state == State::Queued;
        if (!first && r.parts_open >= max_parts) {
            ++it;
            continue;
        }
        if (take.empty())
            e_den = r.e_den;
        if (r.e_den != e_den || (first && inflight_reqs + new_reqs >= cfg.max_inflight))
            break;
        auto fits = [&](uint64_t nw, uint64_t nr, uint64_t np) {
            return plan(words + nw + 1, reads + nr, pairs + np, ws_need(idx, pairs + np)).total <=
                   cap;
        };
        const uint64_t room = cfg.max_tick_pairs > pairs ? cfg.max_tick_pairs - pairs : 0;
        const uint64_t *co = r.cand_off();
        Part pt;
        pt.r = rp;
        pt.ra = r.next_read;
        if (r.n_reads == 0) {
            if (!fits(0, 0, 0))
                break;
            pt.rb = 0;
        } else if (pt.ra == 0 && co[r.n_reads] <= room && fits(r.n_words, r.n_reads, co[r.n_reads])) {
            pt.rb = r.n_reads;  // the whole request
            pt.wlo = 0;
            pt.nw = r.n_words;
        } else {
            // reads [ra, rb) within the pair room (one read at least when the
            // tick is empty), cut further where the layout stops fitting
            const uint64_t lim = co[pt.ra] + room;
            uint64_t rb =
                (uint64_t)(std::upper_bound(co + pt.ra + 1, co + r.n_reads + 1, lim) - co) - 1;
            if (rb <= pt.ra) {
                if (!take.empty())
                    break;
                rb = pt.ra + 1;
            }
            const uint64_t *ro = r.read_off();
            const uint32_t *rl = r.read_len();
            // the packed words reads [ra, rb) span; the layout check per read
            // only when the whole range does not fit
            uint64_t lo = ~0ull, hi = 0, end = pt.ra;
            for (uint64_t i = pt.ra; i < rb; ++i) {
                lo = std::min<uint64_t>(lo, ro[i] >> 4);
                hi = std::max<uint64_t>(hi, (ro[i] + rl[i] + 15) >> 4);
            }
            if (fits(hi - lo, rb - pt.ra, co[rb] - co[pt.ra])) {
                end = rb;
            } else {
                lo = ~0ull;
                hi = 0;
                for (uint64_t i = pt.ra; i < rb; ++i) {
                    const uint64_t nlo = std::min<uint64_t>(lo, ro[i] >> 4);
                    const uint64_t nhi = std::max<uint64_t>(hi, (ro[i] + rl[i] + 15) >> 4);
                    if (!fits(nhi - nlo, i + 1 - pt.ra, co[i + 1] - co[pt.ra]))
                        break;
                    lo = nlo;
                    hi = nhi;
                    end = i + 1;
                }
            }
            if (end == pt.ra)  // not one more read fits: wait for memory
                break;
            pt.rb = end;
            pt.wlo = lo;
            pt.nw = hi - lo;
        }
        pt.pa = r.n_reads ? co[pt.ra] : 0;
        pt.pb = r.n_reads ? co[pt.rb] : 0;
        words += pt.nw;
        reads += pt.rb - pt.ra;
        pairs += pt.pb - pt.pa;
        if (first)
            ++new_reqs;
        take.push_back(pt);
        if (pt.rb == r.n_reads) {
            it = queue.erase(it);
        } else {
            // the rest of the request waits for the next tick
            break;
        }
    }
    if (take.empty())
        return false;
    Layout lay = plan(words + 1, reads, pairs, ws_need(idx, pairs));
    uint64_t off = 0;
    if (!pool->alloc(lay.total, &off)) {
        // fragmented: nothing was admitted; put the erased requests back in order
        for (auto it = take.rbegin(); it != take.rend(); ++it)
            if (it->rb == it->r->n_reads)
                queue.push_front(it->r);
        return false;
    }
    peak_bytes = std::max(peak_bytes, pool->used());
    const uint64_t tick = next_tick++;
    const auto now = Clock::now();
    for (auto &pt : take) {
        Request &r = *pt.r;
        if (r.state == State::Queued) {
            r.state = State::Running;
            r.t_admit = now;
            ++inflight_reqs;
        }
        r.tick = tick;
        r.next_read = pt.rb;
        r.all_admitted = pt.rb == r.n_reads;
        ++r.parts_open;
    }
    if (running_ticks++ == 0)
        busy_since = now;
    ++ticks;
    reqs_in_ticks += take.size();
    last_group = slot->group;
    slot->busy = true;
    slot->parts = std::move(take);
    slot->lay = lay;
    slot->dev_off = off;
    slot->e_den = e_den;
    {
        std::lock_guard<std::mutex> lk(slot->m);
        slot->job = true;
    }
    slot->cv.notify_one();
    return true;
}

namespace {

// Plans the copies of one region of a tick (inputs host to device, or outputs
// device to host), slice by slice in increasing offset order.  A slice of at
// least kDirectBytes moves by DMA between the request's own memory and the
// device; smaller slices go through the slot's stage, and staged slices less
// than 256 bytes apart (alignment gaps) are sent as one copy, so that a tick
// of small requests needs one copy each way.
struct RunCopier {
    uint8_t *dev, *stage;
    bool h2d;
    bool store = false;  // downloads by host stores where the destination allows
    std::vector<CopyOp> ops;
    uint64_t run_lo = 0, run_hi = 0;
    bool run = false;

    RunCopier(uint8_t *dev_, uint8_t *stage_, bool h2d_, bool store_ = false)
        : dev(dev_), stage(stage_), h2d(h2d_), store(store_) {}

    void add(uint64_t off, uint8_t *host, uint64_t bytes, bool writable = true)
    {
        if (h2d)
            ops.push_back({dev + off, host, bytes, false});
        else
            ops.push_back({host, dev + off, bytes, store && writable});
    }
    void flush()
    {
        if (run)
            add(run_lo, stage + run_lo, run_hi - run_lo);  // the stage is page-locked
        run = false;
    }
    // [off, off + bytes) of the stage holds the slice (to device) or receives it
    void staged(uint64_t off, uint64_t bytes)
    {
        if (!bytes)
            return;
        if (run && off >= run_hi && off - run_hi <= 256) {
            run_hi = off + bytes;
            return;
        }
        flush();
        run = true;
        run_lo = off;
        run_hi = off + bytes;
    }
    // the slice at off moves straight between `host` and the device
    void direct(uint64_t off, void *host, uint64_t bytes, bool writable = true)
    {
        flush();
        add(off, static_cast<uint8_t *>(host), bytes, writable);
    }
    // a host slice to the device: by DMA when large, else through the stage
    void put(uint64_t off, const void *src, uint64_t bytes)
    {
        if (bytes >= kDirectBytes) {
            direct(off, const_cast<void *>(src), bytes);
        } else if (bytes) {
            std::memcpy(stage + off, src, bytes);
            staged(off, bytes);
        }
    }
    // queue the planned copies on stream s
    int issue(void *s) const { return issue(s, 0, ops.size()); }
    // queue the planned copies [i0, i1) on stream s
    int issue(void *s, size_t i0, size_t i1) const
    {
        for (size_t i = i0; i < i1; ++i) {
            const CopyOp &op = ops[i];
            const int e = h2d        ? backend().copy_h2d(op.dst, op.src, op.bytes, s)
                          : op.store ? backend().store_d2h(op.dst, op.src, op.bytes, s)
                                     : backend().copy_d2h(op.dst, op.src, op.bytes, s);
            if (e != GRIM_OK)
                return GRIM_E_HIP;
        }
        return GRIM_OK;
    }
};

}  // namespace

// Stages s's tick and queues it on the slot's stream (worker thread, no server
// lock): the input copies, the filter, the result copies and last the
// completion notice.  On failure, waits for what was queued and returns the
// error.
int grim_server::launch(Slot &s)
{
    const grim_serve::Backend &be = backend();
    const Layout &lay = s.lay;
    uint8_t *h = s.stage;
    uint8_t *d = pool_base + s.dev_off;
    void *st = s.stream;
    // per-read arrays, re-based to the fused tick
    uint64_t wbase = 0, rbase = 0, pbase = 0;
    uint64_t *ro = reinterpret_cast<uint64_t *>(h + lay.read_off);
    uint64_t *coff = reinterpret_cast<uint64_t *>(h + lay.cand_off);
    uint32_t *rlen = reinterpret_cast<uint32_t *>(h + lay.read_len);
    uint32_t *re = reinterpret_cast<uint32_t *>(h + lay.read_e);
    for (Part &pt : s.parts) {
        const Request &r = *pt.r;
        const uint64_t nr = pt.rb - pt.ra;
        const uint64_t *sro = r.read_off(), *sco = r.cand_off();
        const uint64_t shift = wbase * 16, base0 = pt.wlo * 16;
        for (uint64_t i = 0; i < nr; ++i) {
            ro[rbase + i] = sro[pt.ra + i] - base0 + shift;
            coff[rbase + i] = sco[pt.ra + i] - pt.pa + pbase;
        }
        if (nr) {
            std::memcpy(rlen + rbase, r.read_len() + pt.ra, nr * 4);
            std::memcpy(re + rbase, r.read_e() + pt.ra, nr * 4);
        }
        pt.fused_base = pbase;
        wbase += pt.nw;
        rbase += nr;
        pbase += pt.pb - pt.pa;
    }
    coff[rbase] = pbase;
    RunCopier in{d, h, true};
    in.staged(lay.read_off, rbase * 8);
    in.staged(lay.cand_off, (rbase + 1) * 8);
    in.staged(lay.read_len, rbase * 4);
    in.staged(lay.read_e, rbase * 4);
    // packed words, then bin ids (no token reaches past a read's last base, so
    // nothing after the words needs to be written)
    uint64_t o = lay.words;
    for (const Part &pt : s.parts) {
        in.put(o, pt.r->words() + pt.wlo, pt.nw * 4);
        o += pt.nw * 4;
    }
    for (const Part &pt : s.parts)
        in.put(lay.cand_bin + pt.fused_base * 4, pt.r->cand_bin() + pt.pa, (pt.pb - pt.pa) * 4);
    in.flush();
    // with upload turns: wait for this tick's turn, queue the input copies and
    // the notice that ends the turn once they have run (or end it here if that
    // notice could not be queued).  When the last copy carries an eighth of the
    // tick's bytes or more, the notice goes before it, so that the next tick's
    // uploads are queued while it runs and the link does not idle through the
    // notice's latency.
    s.turn_wait_s = 0;
    size_t split = in.ops.size();
    if (upload_turns && split > 1) {
        uint64_t total = 0;
        for (const CopyOp &op : in.ops)
            total += op.bytes;
        if (in.ops.back().bytes * 8 >= total)
            split = in.ops.size() - 1;
    }
    if (upload_turns) {
        const auto t0 = Clock::now();
        std::unique_lock<std::mutex> lk(up_mu);
        up_cv.wait(lk, [&] { return stream_ticks[s.stream_idx] == 0; });
        ++stream_ticks[s.stream_idx];
        const uint64_t mine = up_next++;
        up_cv.wait(lk, [&] { return up_turn == mine; });
        s.turn_wait_s = secs(Clock::now() - t0);
    }
    int rc = in.issue(st, 0, split);
    if (upload_turns) {
        if (rc == GRIM_OK && be.notify(st, on_upload_done, &s) != GRIM_OK)
            rc = GRIM_E_HIP;
        if (rc != GRIM_OK) {
            (void)be.stream_sync(st);
            upload_turn_end();
        }
    }
    if (rc == GRIM_OK && split < in.ops.size())
        rc = in.issue(st, split, in.ops.size());
    grim_batch_t b;
    b.reads_2bit = reinterpret_cast<const uint32_t *>(d + lay.words);
    b.n_read_words = std::max<uint64_t>(wbase, 1);  // the layout holds one word more
    b.read_off = reinterpret_cast<const uint64_t *>(d + lay.read_off);
    b.read_len = reinterpret_cast<const uint32_t *>(d + lay.read_len);
    b.read_e = reinterpret_cast<const uint32_t *>(d + lay.read_e);
    b.e_den = s.e_den;
    b.max_len = cfg.max_len;
    b.cand_off = reinterpret_cast<const uint64_t *>(d + lay.cand_off);
    b.cand_bin = reinterpret_cast<const uint32_t *>(d + lay.cand_bin);
    b.n_reads = rbase;
    b.n_pairs = pbase;
    uint8_t *dout = d + lay.out_base;
    uint8_t *hout = h + lay.out_base;
    int32_t *dcounts = reinterpret_cast<int32_t *>(dout + lay.counts);
    uint32_t *dbits = reinterpret_cast<uint32_t *>(dout + lay.bits);
    if (rc == GRIM_OK)
        rc = be.filter(idx, &b, dcounts, dbits, dout + lay.ws, lay.ws_bytes, st);
    // results: large count slices straight into the request's result area, the
    // rest (small slices, then the pass bits with the status word that follows
    // them) via the stage; no counts at all when only the pass bits are
    // results; then the completion notice
    if (rc == GRIM_OK) {
        const bool bits_only = (cfg.flags & GRIM_SERVE_PASS_BITS_ONLY) != 0;
        RunCopier out{dout, hout, false, store_downloads};
        for (size_t j = 0; j < s.parts.size() && !bits_only; ++j) {
            Part &pt = s.parts[j];
            const uint64_t lo = lay.counts + pt.fused_base * 4, nb = (pt.pb - pt.pa) * 4;
            if (nb >= kDirectBytes) {
                out.direct(lo, pt.r->counts() + pt.pa, nb, pt.r->counts_writable);
                pt.counts_direct = true;
            } else {
                out.staged(lo, nb);
            }
        }
        out.staged(lay.bits, lay.ws - lay.bits + 4);
        out.flush();
        rc = out.issue(st);
        if (rc == GRIM_OK && be.notify(st, on_tick_done, &s) != GRIM_OK)  // last: may run at once
            rc = GRIM_E_HIP;
    }
    if (rc != GRIM_OK) {
        (void)be.stream_sync(st);  // the tick never completes: let what was queued finish
        if (upload_turns)
            stream_tick_done(s.stream_idx);
    }
    return rc;
}

// A slot's worker: takes each tick the admission thread hands over, launches
// it, waits for its completion notice and retires it.
void grim_server::work(Slot &s)
{
    backend().set_device(device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s.m);
            s.cv.wait(lk, [&] { return s.job || s.quit; });
            if (!s.job)
                return;
            s.job = false;
            s.notice = false;
        }
        const auto t0 = Clock::now();
        const int rc = launch(s);
        const double t_launch = secs(Clock::now() - t0) - s.turn_wait_s;
        if (rc != GRIM_OK) {
            close_tick(s, rc, {}, t_launch, 0.0);
            continue;
        }
        {
            std::unique_lock<std::mutex> lk(s.m);
            s.cv.wait(lk, [&] { return s.notice; });
        }
        retire(s, t_launch);
    }
}

// The admission thread: forms ticks while slots are free and requests wait,
// then sleeps until the doorbell rings.  Ends on shutdown once no tick runs.
void grim_server::run()
{
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        uint64_t seen;
        {
            std::lock_guard<std::mutex> bl(bell_mu);
            seen = bell;  // a ring after this point wakes the wait below
        }
        if (stop && running_ticks == 0)
            break;
        if (!stop) {
            const auto t0 = Clock::now();
            while (admit_tick()) {
            }
            admit_s += secs(Clock::now() - t0);
        }
        lk.unlock();
        {
            // a bounded sleep as well, measured on the system clock: its timed
            // wait is the one every thread checker models
            std::unique_lock<std::mutex> bl(bell_mu);
            bell_cv.wait_until(bl, std::chrono::system_clock::now() + std::chrono::milliseconds(100),
                               [&] { return bell != seen; });
        }
        lk.lock();
    }
}

namespace {

// The server's n streams.  Copies queued on streams that the runtime serves
// with one copy engine take turns, even in opposite directions, and which
// streams share an engine depends on the process's history (on MI355X:
// measured both as groups of four consecutively created streams, and as one
// stream of a newly created batch alone against all the others).  An upload
// overlaps a download (48 GB/s each way instead of 28.5 in turns) only across
// engines.  So candidate streams are created and timed: an upload on the first
// candidate with a download on the same stream (in turns by definition), then
// with a download on each other candidate; those that overlap form the other
// group.  The chosen streams alternate between the groups (as far as each has
// streams) and the others are destroyed.  Copies of `bytes` between dev and
// host (2 * bytes each).  Returns the number of groups found (1 or 2), or 0 if
// a stream could not be created.
uint32_t pick_streams(uint32_t n, uint8_t *dev, uint8_t *host, uint64_t bytes,
                      std::vector<void *> *out, std::vector<int> *group)
{
    const grim_serve::Backend &be = backend();
    const uint32_t n_cand = n > 1 && bytes ? std::max<uint32_t>(8, 2 * n) : n;
    std::vector<void *> cand;
    for (uint32_t i = 0; i < n_cand; ++i) {
        void *st = nullptr;
        if (be.stream_create(&st) != GRIM_OK) {
            for (void *c : cand)
                be.stream_destroy(c);
            return 0;
        }
        cand.push_back(st);
    }
    // best of two timings of an upload on the first candidate with a download
    // on candidate i (0 when a call failed)
    auto timed = [&](uint32_t i) {
        double best = 0;
        for (int rep = 0; rep < 2; ++rep) {
            const auto t0 = Clock::now();
            const int e1 = be.copy_h2d(dev, host, bytes, cand[0]);
            const int e2 = be.copy_d2h(host + bytes, dev + bytes, bytes, cand[i]);
            const int e3 = be.stream_sync(cand[0]);
            const int e4 = i ? be.stream_sync(cand[i]) : GRIM_OK;
            const double dt = secs(Clock::now() - t0);
            if (e1 || e2 || e3 || e4)
                return 0.0;
            best = rep == 0 ? dt : std::min(best, dt);
        }
        return best;
    };
    std::vector<int> cg(n_cand, 0);
    uint32_t groups = 1;
    if (n_cand > n) {
        (void)timed(0);  // warm-up
        const double serial = timed(0);
        for (uint32_t i = 1; i < n_cand && serial > 0; ++i) {
            const double t = timed(i);
            if (t > 0 && t < 0.8 * serial) {
                cg[i] = 1;
                groups = 2;
            }
        }
    }
    std::vector<bool> used(n_cand, false);
    for (uint32_t k = 0; k < n; ++k) {
        const int want = (int)(k % 2) % (int)groups;
        uint32_t pick = n_cand;
        for (uint32_t i = 0; i < n_cand && pick == n_cand; ++i)
            if (!used[i] && cg[i] == want)
                pick = i;
        for (uint32_t i = 0; i < n_cand && pick == n_cand; ++i)
            if (!used[i])
                pick = i;
        used[pick] = true;
        out->push_back(cand[pick]);
        group->push_back(cg[pick]);
    }
    for (uint32_t i = 0; i < n_cand; ++i)
        if (!used[i])
            be.stream_destroy(cand[i]);
    return groups;
}

// Frees what grim_serve_create has set up so far (no thread started yet).
void free_server_parts(grim_server *s)
{
    const grim_serve::Backend &be = backend();
    for (auto &sl : s->slots)
        be.pinned_free(sl->stage);
    for (void *st : s->streams)
        be.stream_destroy(st);
    be.pinned_free(s->arena);
    be.device_free(s->pool_base);
}

}  // namespace

extern "C" int grim_serve_create(const grim_index_t *idx, const grim_serve_cfg_t *cfg,
                                 grim_server_t **out)
{
    if (!idx || !out)
        return GRIM_E_INVALID;
    grim_serve_cfg_t c = cfg ? *cfg : grim_serve_cfg_t{};
    if (!c.hbm_budget_bytes)
        c.hbm_budget_bytes = 1ull << 30;
    if (!c.max_inflight)
        c.max_inflight = 1024;
    if (!c.n_streams)
        c.n_streams = 3;
    if (!c.max_tick_pairs)
        c.max_tick_pairs = 8u << 20;
    if (!c.max_len)
        c.max_len = 1024;
    const bool bits_only = (c.flags & GRIM_SERVE_PASS_BITS_ONLY) != 0;
    if (!c.ticks_per_stream)
        c.ticks_per_stream = 2;
    const uint32_t dl_flags = GRIM_SERVE_STORE_DOWNLOADS | GRIM_SERVE_ENGINE_DOWNLOADS;
    if (c.max_len > GRIM_MAX_READ_LEN || c.n_streams > 16 || c.ticks_per_stream > 4 ||
        (c.flags & ~(GRIM_SERVE_PASS_BITS_ONLY | dl_flags)) || (c.flags & dl_flags) == dl_flags)
        return GRIM_E_INVALID;
    const grim_serve::Backend &be = backend();
    int dev = 0;
    if (be.current_device(&dev) != GRIM_OK || dev != be.index_device(idx))
        return GRIM_E_INVALID;
    auto s = std::make_unique<grim_server>();
    s->idx = idx;
    s->cfg = c;
    s->device = dev;
    s->upload_turns = !bits_only;
    if (be.device_alloc(c.hbm_budget_bytes, &s->pool_base) != GRIM_OK)
        return GRIM_E_NOMEM;
    s->pool = std::make_unique<Pool>(c.hbm_budget_bytes);
    // pinned arena for request blocks: as large as the device budget, at most 4 GiB
    s->arena_bytes = std::min<uint64_t>(std::max<uint64_t>(c.hbm_budget_bytes, 64ull << 20),
                                        4ull << 30);
    if (be.pinned_alloc(s->arena_bytes, &s->arena) != GRIM_OK) {
        s->arena = nullptr;
        s->arena_bytes = 0;
    }
    s->arena_pool = std::make_unique<Pool>(s->arena_bytes);
    // every slot's staging buffer, sized once for the largest tick it stages:
    // max(max_tick_pairs, 2^20) pairs, max(4096, pairs / 32) reads of max_len
    // bases (admission keeps every tick's layout within it; a single read that
    // alone would not fit is refused at submit)
    const uint64_t P = std::max<uint64_t>(c.max_tick_pairs, 1ull << 20);
    const uint64_t R = std::max<uint64_t>(4096, P / 32);
    const uint64_t W = R * (c.max_len / 16 + 2) + 1;
    s->stage_bytes = std::min<uint64_t>(c.hbm_budget_bytes, plan(W, R, P, ws_need(idx, P)).total);
    s->slots.resize((size_t)c.ticks_per_stream * c.n_streams);
    for (auto &sl : s->slots) {
        sl = std::make_unique<Slot>();
        sl->srv = s.get();
        if (be.pinned_alloc(s->stage_bytes, &sl->stage) != GRIM_OK) {
            sl->stage = nullptr;
            free_server_parts(s.get());
            return GRIM_E_NOMEM;
        }
    }
    // the streams, split between copy-engine groups (probed with the pool and
    // the first slot's stage, both still unused)
    const uint64_t probe = std::min<uint64_t>(16ull << 20, std::min(s->stage_bytes, c.hbm_budget_bytes) / 2) & ~255ull;
    s->n_groups = pick_streams(c.n_streams, s->pool_base, s->slots[0]->stage, probe, &s->streams,
                               &s->stream_group);
    if (!s->n_groups) {
        free_server_parts(s.get());
        return GRIM_E_HIP;
    }
    s->stream_ticks.assign(c.n_streams, 0);
    for (size_t i = 0; i < s->slots.size(); ++i) {
        s->slots[i]->stream = s->streams[i % c.n_streams];
        s->slots[i]->stream_idx = (uint32_t)(i % c.n_streams);
        s->slots[i]->group = s->stream_group[i % c.n_streams];
    }
    // with results that include counts and every stream on one copy engine,
    // downloads go by host stores so that they overlap the engine's uploads
    if (c.flags & GRIM_SERVE_STORE_DOWNLOADS)
        s->store_downloads = true;
    else if (c.flags & GRIM_SERVE_ENGINE_DOWNLOADS)
        s->store_downloads = false;
    else
        s->store_downloads = s->n_groups < 2 && !bits_only && c.n_streams > 1;
    grim_server *raw = s.release();
    for (auto &sl : raw->slots) {
        Slot *p = sl.get();
        p->worker = std::thread([raw, p] { raw->work(*p); });
    }
    raw->thr = std::thread([raw] { raw->run(); });
    *out = raw;
    return GRIM_OK;
}

namespace {

// Checks a host batch the way a solo grim_filter_batch run would need it to be
// well formed; a malformed request never reaches the device.
int validate_request(const grim_server_t *s, const grim_batch_t *b)
{
    if (!s || !b || b->e_den == 0)
        return GRIM_E_INVALID;
    if (b->max_len > s->cfg.max_len)
        return GRIM_E_UNSUPPORTED;
    const uint64_t n = b->n_reads, P = b->n_pairs;
    if ((n && (!b->read_off || !b->read_len || !b->read_e || !b->cand_off || !b->reads_2bit)) ||
        (P && !b->cand_bin) || (!n && P))
        return GRIM_E_INVALID;
    if (n) {
        if (b->cand_off[0] != 0 || b->cand_off[n] != P)
            return GRIM_E_INVALID;
        const uint64_t nbases = b->n_read_words * 16;
        for (uint64_t i = 0; i < n; ++i) {
            if (b->cand_off[i + 1] < b->cand_off[i])
                return GRIM_E_INVALID;
            if (b->read_len[i] > b->max_len || b->read_off[i] > nbases ||
                b->read_len[i] > nbases - b->read_off[i])
                return GRIM_E_READ;
        }
    }
    const uint64_t nwords = n ? b->n_read_words : 0;
    if (plan(nwords + 1, n, P, ws_need(s->idx, P)).total > s->cfg.hbm_budget_bytes)
        return GRIM_E_BUDGET;
    // a read with more candidates than a tick holds runs alone in a tick: it
    // must fit the staging buffer by itself
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t np = b->cand_off[i + 1] - b->cand_off[i];
        if (np <= s->cfg.max_tick_pairs)
            continue;
        const uint64_t nw = ((b->read_off[i] + b->read_len[i] + 15) >> 4) - (b->read_off[i] >> 4);
        if (plan(nw + 1, 1, np, ws_need(s->idx, np)).total > s->stage_bytes)
            return GRIM_E_BUDGET;
    }
    return GRIM_OK;
}

int enqueue_request(grim_server_t *s, std::shared_ptr<Request> r, uint64_t *ticket)
{
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            s->free_block(*r);
            return GRIM_E_INVALID;
        }
        r->ticket = s->next_ticket++;
        s->all[r->ticket] = r;
        s->queue.push_back(r);
        ++s->submitted;
    }
    s->ring();
    *ticket = r->ticket;
    return GRIM_OK;
}

}  // namespace

extern "C" int grim_serve_submit(grim_server_t *s, const grim_batch_t *b, uint64_t *ticket)
{
    const auto t0 = Clock::now();
    if (!ticket)
        return GRIM_E_INVALID;
    int rc = validate_request(s, b);
    if (rc)
        return rc;
    const uint64_t n = b->n_reads, P = b->n_pairs;
    const uint64_t nwords = n ? b->n_read_words : 0;
    auto r = std::make_shared<Request>();
    r->lay = req_layout(nwords, n, P);
    {
        std::lock_guard<std::mutex> lk(s->arena_mu);
        uint64_t off = 0;
        if (s->arena && s->arena_pool->alloc(r->lay.total, &off)) {
            r->host = s->arena + off;
            r->arena_off = off;
            r->pinned = true;
            r->counts_writable = true;  // the arena is page-locked
        }
    }
    if (!r->host) {
        r->host = static_cast<uint8_t *>(std::aligned_alloc(256, r->lay.total));
        if (!r->host)
            return GRIM_E_NOMEM;
    }
    r->view_block();
    uint8_t *h = r->host;
    par_memcpy(h + r->lay.words, b->reads_2bit, nwords * 4);
    if (n) {
        std::memcpy(h + r->lay.read_off, b->read_off, n * 8);
        std::memcpy(h + r->lay.read_len, b->read_len, n * 4);
        std::memcpy(h + r->lay.read_e, b->read_e, n * 4);
        std::memcpy(h + r->lay.cand_off, b->cand_off, (n + 1) * 8);
    } else {
        *reinterpret_cast<uint64_t *>(h + r->lay.cand_off) = 0;
    }
    par_memcpy(h + r->lay.cand_bin, b->cand_bin, P * 4);
    std::memset(h + r->lay.bits, 0, ((P + 31) / 32) * 4);  // parts OR their bits in
    r->e_den = b->e_den;
    r->n_words = nwords;
    r->n_reads = n;
    r->n_pairs = P;
    r->t_submit = t0;
    return enqueue_request(s, r, ticket);
}

extern "C" int grim_serve_submit_inplace(grim_server_t *s, const grim_batch_t *b, int32_t *counts,
                                         uint32_t *pass_bits, uint64_t *ticket)
{
    const auto t0 = Clock::now();
    if (!ticket)
        return GRIM_E_INVALID;
    int rc = validate_request(s, b);
    if (rc)
        return rc;
    const uint64_t n = b->n_reads, P = b->n_pairs;
    if (P && (!pass_bits || (!counts && !(s->cfg.flags & GRIM_SERVE_PASS_BITS_ONLY))))
        return GRIM_E_INVALID;
    auto r = std::make_shared<Request>();
    r->in_place = true;
    r->counts_writable = counts && backend().device_writable(counts);
    r->p_words = b->reads_2bit;
    r->p_read_off = b->read_off;
    r->p_read_len = b->read_len;
    r->p_read_e = b->read_e;
    r->p_cand_off = n ? b->cand_off : nullptr;
    r->p_cand_bin = b->cand_bin;
    r->p_counts = counts;
    r->p_bits = pass_bits;
    if (P)
        std::memset(pass_bits, 0, ((P + 31) / 32) * 4);  // parts OR their bits in
    r->e_den = b->e_den;
    r->n_words = n ? b->n_read_words : 0;
    r->n_reads = n;
    r->n_pairs = P;
    r->t_submit = t0;
    return enqueue_request(s, r, ticket);
}

// Hand a finished request's results to the caller.  Called with the server
// lock held; releases it before copying so the scheduler is not stalled.
static int finish(grim_server_t *s, std::unique_lock<std::mutex> &lk,
                  std::map<uint64_t, std::shared_ptr<Request>>::iterator it, int32_t *counts,
                  uint32_t *pass_bits, grim_req_stats_t *st)
{
    std::shared_ptr<Request> rp = it->second;
    Request &r = *rp;
    s->all.erase(it);
    lk.unlock();
    const bool bits_only = (s->cfg.flags & GRIM_SERVE_PASS_BITS_ONLY) != 0;
    if ((r.status == GRIM_OK || r.status == GRIM_E_BIN_RANGE) && r.counts()) {
        if (counts && counts != r.counts() && !bits_only)
            par_memcpy(counts, r.counts(), r.n_pairs * 4);
        if (pass_bits && pass_bits != r.bits())
            std::memcpy(pass_bits, r.bits(), ((r.n_pairs + 31) / 32) * 4);
    }
    if (st) {
        st->queue_ms = r.t_admit.time_since_epoch().count() ? ms_between(r.t_submit, r.t_admit)
                                                            : 0.0;
        st->latency_ms = ms_between(r.t_submit, r.t_done);
        st->n_pairs = r.n_pairs;
        st->tick = r.tick;
        st->flags = r.flags;
        st->status = r.status;
    }
    const int rc = r.status;
    s->free_block(r);
    return rc;
}

extern "C" int grim_serve_poll(grim_server_t *s, uint64_t ticket, int32_t *counts,
                               uint32_t *pass_bits, grim_req_stats_t *st)
{
    if (!s)
        return GRIM_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end())
        return GRIM_E_INVALID;
    if (it->second->state != State::Done)
        return GRIM_PENDING;
    return finish(s, lk, it, counts, pass_bits, st);
}

extern "C" int grim_serve_wait(grim_server_t *s, uint64_t ticket, int64_t timeout_ms,
                               int32_t *counts, uint32_t *pass_bits, grim_req_stats_t *st)
{
    if (!s)
        return GRIM_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end())
        return GRIM_E_INVALID;
    auto req = it->second;
    auto done = [&] { return req->state == State::Done; };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_until(
                 lk, std::chrono::system_clock::now() + std::chrono::milliseconds(timeout_ms), done))
        return GRIM_E_TIMEOUT;
    it = s->all.find(ticket);
    if (it == s->all.end())
        return GRIM_E_INVALID;
    return finish(s, lk, it, counts, pass_bits, st);
}

extern "C" int grim_serve_cancel(grim_server_t *s, uint64_t ticket)
{
    if (!s)
        return GRIM_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end())
        return GRIM_E_INVALID;
    Request &r = *it->second;
    if (r.state == State::Done)
        return GRIM_OK;
    r.cancelled = true;
    if (r.state == State::Queued) {
        s->drop_from_queue(r);
        r.status = GRIM_E_CANCELLED;
        r.state = State::Done;
        r.t_done = Clock::now();
        ++s->cancelled;
        s->cv_done.notify_all();
    } else if (!r.all_admitted) {
        // admitted in part: the rest never runs; done once its parts in flight retire
        s->drop_from_queue(r);
        r.all_admitted = true;
        if (r.parts_open == 0) {
            s->part_closed(r, Clock::now());
            s->cv_done.notify_all();
        }
    }
    return GRIM_OK;
}

extern "C" int grim_serve_stats(grim_server_t *s, grim_serve_stats_t *out, int reset)
{
    if (!s || !out)
        return GRIM_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->cancelled = s->cancelled;
    out->failed = s->failed;
    out->ticks = s->ticks;
    out->pairs_done = s->pairs_done;
    std::vector<double> v = s->lat;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::min<double>(v.size() - 1, std::ceil(p * v.size()) - 1);
            return v[i];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        double sum = 0;
        for (double x : v)
            sum += x;
        out->mean_ms = sum / v.size();
        out->max_ms = v.back();
    }
    double busy = s->busy_s;
    if (s->running_ticks > 0)
        busy += std::chrono::duration<double>(Clock::now() - s->busy_since).count();
    out->busy_s = busy;
    out->pairs_per_s = busy > 0 ? s->pairs_done / busy : 0.0;
    out->peak_device_bytes = s->peak_bytes;
    out->mean_requests_per_tick = s->ticks ? (double)s->reqs_in_ticks / s->ticks : 0.0;
    out->sched_admit_s = s->admit_s;
    out->stream_groups = s->n_groups;
    out->sched_launch_s = s->launch_s;
    out->sched_retire_s = s->retire_s;
    if (reset) {
        s->submitted = s->completed = s->cancelled = s->failed = s->ticks = s->pairs_done = 0;
        s->reqs_in_ticks = 0;
        s->peak_bytes = s->pool->used();
        s->lat.clear();
        s->busy_s = 0;
        s->admit_s = s->launch_s = s->retire_s = 0;
        if (s->running_ticks > 0)
            s->busy_since = Clock::now();
    }
    return GRIM_OK;
}

extern "C" void grim_serve_destroy(grim_server_t *s)
{
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto &r : s->queue) {
            r->status = GRIM_E_CANCELLED;
            r->state = State::Done;
        }
        s->queue.clear();
    }
    s->ring();
    if (s->thr.joinable())
        s->thr.join();
    // every tick has been retired: the workers wait for work; end them
    for (auto &sl : s->slots) {
        {
            std::lock_guard<std::mutex> lk(sl->m);
            sl->quit = true;
        }
        sl->cv.notify_one();
        if (sl->worker.joinable())
            sl->worker.join();
    }
    // wait until the streams (and the completion notices on them) have
    // finished before the server's memory goes
    const grim_serve::Backend &be = backend();
    for (void *st : s->streams)
        (void)be.stream_sync(st);
    for (auto &kv : s->all)
        s->free_block(*kv.second);
    s->all.clear();
    free_server_parts(s);
    delete s;
}
