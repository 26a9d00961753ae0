// The serving scheduler (grim_serve.cpp) on the CPU, against the host-memory
// backend of serve_fake_backend.cpp; built and run under ThreadSanitizer (and
// under AddressSanitizer + UBSan) by tests/test_serve_scheduler.py.
//
// Scenarios: requests from several submitting threads, copied and in place,
// split into parts and fused into ticks, cancelled concurrently from another
// thread, with one or more ticks queued per stream; the same with injected
// filter-launch failures; large requests whose slices move by DMA instead of
// through the stage; a pass-bits-only
// server with an out-of-range bin; requests refused at submit; a server
// destroyed with work queued.  After each scenario every ticket must have
// ended with an allowed status, every finished request's results must equal
// the stand-in filter run on that request alone, and the device pool must be
// back to 0 bytes in use.  Exits non-zero on the first failed check.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "grim.h"
#include "serve_fake.h"

#define CHECK(cond)                                                                      \
    do {                                                                                 \
        if (!(cond)) {                                                                   \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            std::exit(1);                                                                \
        }                                                                                \
    } while (0)

namespace {

constexpr uint64_t kBins = 5000;

struct Req {
    std::vector<uint32_t> words;
    std::vector<uint64_t> read_off, cand_off;
    std::vector<uint32_t> read_len, read_e, cand_bin;
    uint32_t e_den = 10000, max_len = 256;
    std::vector<int32_t> want_counts, out_counts;
    std::vector<uint32_t> want_bits, out_bits;
    uint32_t want_flags = 0;
    uint64_t n_pairs = 0;

    grim_batch_t batch() const
    {
        grim_batch_t b;
        b.reads_2bit = words.data();
        b.n_read_words = words.size();
        b.read_off = read_off.data();
        b.read_len = read_len.data();
        b.read_e = read_e.data();
        b.e_den = e_den;
        b.max_len = max_len;
        b.cand_off = cand_off.data();
        b.cand_bin = cand_bin.empty() ? nullptr : cand_bin.data();
        b.n_reads = read_len.size();
        b.n_pairs = n_pairs;
        return b;
    }
};

Req make_req(std::mt19937_64 &rng, uint32_t max_reads, bool bad_bin)
{
    Req q;
    const uint32_t n = (uint32_t)(rng() % (max_reads + 1));
    uint64_t pos = rng() % 17;
    q.cand_off.push_back(0);
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t L = (rng() % 10 == 0) ? (uint32_t)(rng() % 5) : 20 + (uint32_t)(rng() % 230);
        q.read_off.push_back(pos);
        q.read_len.push_back(L);
        q.read_e.push_back(rng() % 2 ? 500 : 1000);
        pos += L + rng() % 40;
        // mostly short candidate lists, sometimes long ones
        const uint64_t k = rng() % 8 == 0 ? rng() % 1500 : rng() % 12;
        for (uint64_t j = 0; j < k; ++j)
            q.cand_bin.push_back((uint32_t)(rng() % kBins));
        q.cand_off.push_back(q.cand_bin.size());
    }
    q.words.resize(pos / 16 + 2);
    for (auto &w : q.words)
        w = (uint32_t)rng();
    q.n_pairs = q.cand_bin.size();
    if (bad_bin && q.n_pairs)
        q.cand_bin[rng() % q.n_pairs] = (uint32_t)(kBins + rng() % 100);
    q.want_counts.assign(q.n_pairs ? q.n_pairs : 1, 0);
    q.want_bits.assign((q.n_pairs + 31) / 32 + 1, 0);
    grim_batch_t b = q.batch();
    fake_filter_host(&b, kBins, q.want_counts.data(), q.want_bits.data(), &q.want_flags);
    q.out_counts.assign(q.n_pairs ? q.n_pairs : 1, -77);
    q.out_bits.assign((q.n_pairs + 31) / 32 + 1, 0xdeadbeefu);
    return q;
}

struct Scenario {
    const char *name;
    grim_serve_cfg_t cfg;
    int threads, per_thread;
    uint32_t max_reads;
    uint64_t fail_every;
    int cancel_every;     // cancel every cancel_every-th ticket (0: none)
    int bad_every;        // every bad_every-th request holds an out-of-range bin (0: none)
};

void run(const Scenario &sc, grim_index_t *idx, uint64_t seed)
{
    grim_server_t *srv = nullptr;
    CHECK(grim_serve_create(idx, &sc.cfg, &srv) == GRIM_OK);
    fake_fail_filter_every(sc.fail_every);
    const bool bits_only = (sc.cfg.flags & GRIM_SERVE_PASS_BITS_ONLY) != 0;
    const int total = sc.threads * sc.per_thread;
    std::vector<Req> reqs(total);
    std::vector<uint64_t> tickets(total, 0);
    std::vector<std::atomic<int>> submitted(total);
    for (auto &s : submitted)
        s = 0;
    std::set<int> cancelled;
    std::mutex cmu;
    std::atomic<int> n_submitted{0};
    std::vector<std::thread> th;
    for (int t = 0; t < sc.threads; ++t) {
        th.emplace_back([&, t] {
            std::mt19937_64 rng(seed * 1000 + t);
            for (int i = 0; i < sc.per_thread; ++i) {
                const int k = t * sc.per_thread + i;
                reqs[k] = make_req(rng, sc.max_reads, sc.bad_every && k % sc.bad_every == 3);
                const grim_batch_t b = reqs[k].batch();
                uint64_t tk = 0;
                int rc;
                if (k % 4 == 1) {  // in place, in memory the device cannot reach
                    Req &q = reqs[k];
                    fake_mark_pageable(q.words.data(), q.words.size() * 4);
                    fake_mark_pageable(q.cand_bin.data(), q.cand_bin.size() * 4);
                    fake_mark_pageable(q.out_counts.data(), q.out_counts.size() * 4);
                    fake_mark_pageable(q.out_bits.data(), q.out_bits.size() * 4);
                }
                if (k % 2)
                    rc = grim_serve_submit_inplace(srv, &b, bits_only ? nullptr : reqs[k].out_counts.data(),
                                                   reqs[k].out_bits.data(), &tk);
                else
                    rc = grim_serve_submit(srv, &b, &tk);
                CHECK(rc == GRIM_OK);
                tickets[k] = tk;
                submitted[k].store(1, std::memory_order_release);
                ++n_submitted;
                if (rng() % 4 == 0)
                    std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
            }
        });
    }
    // concurrent cancellations of queued, running and partly admitted requests
    std::thread canceller([&] {
        if (!sc.cancel_every)
            return;
        std::mt19937_64 rng(seed + 99);
        // until shortly after the last submission, cancel submitted tickets
        // at random: they are queued, running, admitted in part or done
        for (int extra = 0; extra < 50;) {
            const int n = n_submitted.load();
            if (n == total)
                ++extra;
            if (n == 0) {
                std::this_thread::yield();
                continue;
            }
            const int k = (int)(rng() % total);
            if (k % sc.cancel_every == 0 && submitted[k].load(std::memory_order_acquire)) {
                {
                    std::lock_guard<std::mutex> lk(cmu);
                    if (cancelled.count(k))
                        continue;
                    cancelled.insert(k);
                }
                CHECK(grim_serve_cancel(srv, tickets[k]) == GRIM_OK);
            }
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    });
    for (auto &x : th)
        x.join();
    canceller.join();
    int n_ok = 0, n_hip = 0, n_cancel = 0, n_range = 0;
    for (int k = 0; k < total; ++k) {
        Req &q = reqs[k];
        std::vector<int32_t> c(q.n_pairs ? q.n_pairs : 1, -55);
        std::vector<uint32_t> b((q.n_pairs + 31) / 32 + 1, 0x12345678u);
        grim_req_stats_t st;
        const int rc = grim_serve_wait(srv, tickets[k], -1, k % 2 ? nullptr : c.data(),
                                       k % 2 ? nullptr : b.data(), &st);
        const bool was_cancelled = cancelled.count(k) != 0;
        if (rc == GRIM_E_CANCELLED) {
            CHECK(was_cancelled);
            ++n_cancel;
            continue;
        }
        if (rc == GRIM_E_HIP) {
            CHECK(sc.fail_every > 0);
            ++n_hip;
            continue;
        }
        CHECK(rc == GRIM_OK || rc == GRIM_E_BIN_RANGE);
        CHECK((rc == GRIM_E_BIN_RANGE) == ((q.want_flags & GRIM_FLAG_BIN_RANGE) != 0));
        n_range += rc == GRIM_E_BIN_RANGE;
        ++n_ok;
        const int32_t *gc = k % 2 ? q.out_counts.data() : c.data();
        const uint32_t *gb = k % 2 ? q.out_bits.data() : b.data();
        if (!bits_only)
            CHECK(std::memcmp(gc, q.want_counts.data(), q.n_pairs * 4) == 0);
        CHECK(std::memcmp(gb, q.want_bits.data(), ((q.n_pairs + 31) / 32) * 4) == 0);
        CHECK(st.n_pairs == q.n_pairs);
    }
    grim_serve_stats_t s1, s2;
    CHECK(grim_serve_stats(srv, &s1, 1) == GRIM_OK);
    CHECK(s1.submitted == (uint64_t)total);
    CHECK(s1.completed == (uint64_t)n_ok);
    CHECK(s1.cancelled == (uint64_t)n_cancel);
    CHECK(s1.failed == (uint64_t)(n_hip + n_range));
    CHECK(grim_serve_stats(srv, &s2, 0) == GRIM_OK);
    CHECK(s2.peak_device_bytes == 0);  // the pool is back to 0 bytes in use
    if (sc.fail_every)
        CHECK(n_hip > 0 && fake_filter_failures() > 0);
    if (sc.bad_every)
        CHECK(n_range > 0);
    std::printf("%s: %d requests, %d ok (%d with bad bins), %d failed launches, %d cancelled, "
                "%llu ticks, mean %.2f requests per tick\n",
                sc.name, total, n_ok, n_range, n_hip, n_cancel, (unsigned long long)s1.ticks,
                s1.mean_requests_per_tick);
    // the server goes on serving after failures and cancellations
    fake_fail_filter_every(0);
    std::mt19937_64 rng(seed + 7);
    Req q = make_req(rng, 50, false);
    const grim_batch_t b = q.batch();
    uint64_t tk = 0;
    CHECK(grim_serve_submit(srv, &b, &tk) == GRIM_OK);
    std::vector<int32_t> c(q.n_pairs ? q.n_pairs : 1);
    std::vector<uint32_t> bb((q.n_pairs + 31) / 32 + 1);
    CHECK(grim_serve_wait(srv, tk, -1, c.data(), bb.data(), nullptr) == GRIM_OK);
    CHECK(std::memcmp(bb.data(), q.want_bits.data(), ((q.n_pairs + 31) / 32) * 4) == 0);
    grim_serve_destroy(srv);
    fake_clear_pageable();  // the requests' buffers go with reqs
}

void refusals(grim_index_t *idx)
{
    grim_serve_cfg_t cfg{};
    cfg.hbm_budget_bytes = 64ull << 20;
    cfg.max_tick_pairs = 1000;
    cfg.max_len = 256;
    grim_server_t *srv = nullptr;
    CHECK(grim_serve_create(idx, &cfg, &srv) == GRIM_OK);
    std::mt19937_64 rng(5);
    // one read with more candidates than a tick's staging buffer holds
    Req q = make_req(rng, 1, false);
    while (q.read_len.empty())
        q = make_req(rng, 1, false);
    q.cand_bin.assign(3u << 20, 7);
    q.cand_off[1] = q.cand_bin.size();
    q.n_pairs = q.cand_bin.size();
    grim_batch_t b = q.batch();
    uint64_t tk = 0;
    CHECK(grim_serve_submit(srv, &b, &tk) == GRIM_E_BUDGET);
    // a read longer than the request's max_len
    Req r = make_req(rng, 20, false);
    while (r.read_len.empty() || r.read_len[0] < 10)
        r = make_req(rng, 20, false);
    b = r.batch();
    b.max_len = r.read_len[0] - 1;
    bool any_long = false;
    for (uint32_t L : r.read_len)
        any_long |= L > b.max_len;
    CHECK(any_long);
    CHECK(grim_serve_submit(srv, &b, &tk) == GRIM_E_READ);
    // inconsistent CSR offsets
    b = r.batch();
    std::vector<uint64_t> off = r.cand_off;
    off.back() += 1;
    b.cand_off = off.data();
    CHECK(grim_serve_submit(srv, &b, &tk) == GRIM_E_INVALID);
    CHECK(grim_serve_poll(srv, 123456789, nullptr, nullptr, nullptr) == GRIM_E_INVALID);
    grim_serve_destroy(srv);
    // a request larger than the whole budget
    cfg.hbm_budget_bytes = 1 << 20;
    CHECK(grim_serve_create(idx, &cfg, &srv) == GRIM_OK);
    Req big = make_req(rng, 1, false);
    while (big.read_len.empty())
        big = make_req(rng, 1, false);
    big.cand_bin.assign(1u << 20, 3);
    big.cand_off[1] = big.cand_bin.size();
    big.n_pairs = big.cand_bin.size();
    b = big.batch();
    CHECK(grim_serve_submit(srv, &b, &tk) == GRIM_E_BUDGET);
    grim_serve_destroy(srv);
    // configurations out of range
    grim_serve_cfg_t bad = cfg;
    bad.ticks_per_stream = 5;
    CHECK(grim_serve_create(idx, &bad, &srv) == GRIM_E_INVALID);
    bad = cfg;
    bad.n_streams = 17;
    CHECK(grim_serve_create(idx, &bad, &srv) == GRIM_E_INVALID);
    bad = cfg;
    bad.flags = GRIM_SERVE_STORE_DOWNLOADS | GRIM_SERVE_ENGINE_DOWNLOADS;
    CHECK(grim_serve_create(idx, &bad, &srv) == GRIM_E_INVALID);
    bad.flags = 8;
    CHECK(grim_serve_create(idx, &bad, &srv) == GRIM_E_INVALID);
    std::printf("refusals: ok\n");
}

void destroy_with_work_queued(grim_index_t *idx)
{
    grim_serve_cfg_t cfg{};
    cfg.hbm_budget_bytes = 2ull << 20;
    cfg.max_tick_pairs = 500;
    cfg.max_len = 256;
    cfg.n_streams = 2;
    grim_server_t *srv = nullptr;
    CHECK(grim_serve_create(idx, &cfg, &srv) == GRIM_OK);
    std::mt19937_64 rng(11);
    std::vector<Req> reqs;
    for (int i = 0; i < 60; ++i)
        reqs.push_back(make_req(rng, 200, false));
    for (auto &q : reqs) {
        const grim_batch_t b = q.batch();
        uint64_t tk = 0;
        CHECK(grim_serve_submit(srv, &b, &tk) == GRIM_OK);
    }
    grim_serve_destroy(srv);  // queued requests are cancelled, running ticks finish
    std::printf("destroy with work queued: ok\n");
}

}  // namespace

int main()
{
    grim_index_t *idx = fake_index(kBins, 0);
    const int64_t dev0 = fake_device_bytes();
    grim_serve_cfg_t mix{};
    mix.hbm_budget_bytes = 4ull << 20;
    mix.max_inflight = 16;
    mix.n_streams = 3;
    mix.max_tick_pairs = 3000;
    mix.max_len = 256;
    Scenario base{"mix", mix, 4, 40, 300, 0, 0, 0};
    run(base, idx, 1);
    Scenario cancels = base;
    cancels.name = "mix with cancellations, two ticks per stream";
    cancels.cancel_every = 3;
    cancels.cfg.ticks_per_stream = 2;
    run(cancels, idx, 2);
    Scenario faults = cancels;
    faults.name = "mix with failed launches and cancellations";
    faults.fail_every = 5;
    faults.bad_every = 9;
    run(faults, idx, 3);
    Scenario bits = faults;
    bits.name = "pass bits only, failed launches, bad bins";
    bits.cfg.flags = GRIM_SERVE_PASS_BITS_ONLY;
    bits.cfg.n_streams = 2;
    bits.fail_every = 7;
    run(bits, idx, 4);
    Scenario faults_shared = faults;
    faults_shared.name = "stored downloads, failed launches and cancellations";
    faults_shared.cfg.flags = GRIM_SERVE_STORE_DOWNLOADS;
    run(faults_shared, idx, 7);
    Scenario bits_shared = bits;
    bits_shared.name = "pass bits only, stored downloads, two ticks per stream";
    bits_shared.cfg.flags = GRIM_SERVE_PASS_BITS_ONLY | GRIM_SERVE_STORE_DOWNLOADS;
    bits_shared.cfg.ticks_per_stream = 2;
    run(bits_shared, idx, 8);
    Scenario wide = base;
    wide.name = "one stream, large ticks";
    wide.cfg.n_streams = 1;
    wide.cfg.max_tick_pairs = 1 << 20;
    wide.cfg.hbm_budget_bytes = 64ull << 20;
    wide.bad_every = 5;
    run(wide, idx, 5);
    Scenario big = cancels;
    big.name = "large requests: slices moved by DMA, downloads by host stores, split over three streams, three ticks each";
    big.cfg.ticks_per_stream = 3;
    big.cfg.max_tick_pairs = 100000;
    big.cfg.hbm_budget_bytes = 64ull << 20;
    big.threads = 2;
    big.per_thread = 5;
    big.max_reads = 3000;
    big.bad_every = 4;
    big.cfg.flags = GRIM_SERVE_STORE_DOWNLOADS;
    run(big, idx, 6);
    refusals(idx);
    destroy_with_work_queued(idx);
    CHECK(fake_device_bytes() == dev0);  // every server's pool was freed
    fake_index_free(idx);
    std::printf("serve scheduler: all scenarios passed\n");
    return 0;
}
