// Host-memory implementation of the serving scheduler's backend (see
// serve_fake.h): worker threads as streams, memcpy as copies, a stand-in
// filter, completion notices run by the stream's worker.
#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "../../paper_1711_01177_amd/csrc/grim_serve_backend.h"
#include "serve_fake.h"

struct grim_index {
    uint64_t n_bins;
    int device;
};

grim_index_t *fake_index(uint64_t n_bins, int device) { return new grim_index{n_bins, device}; }
void fake_index_free(grim_index_t *idx) { delete idx; }

namespace {

std::atomic<uint64_t> g_fail_every{0}, g_calls{0}, g_failures{0};
std::atomic<int64_t> g_dev_bytes{0};
thread_local int t_device = 0;

uint32_t base_at(const uint32_t *w, uint64_t pos)
{
    return (w[pos >> 4] >> (30 - 2 * (pos & 15))) & 3u;
}

class Stream {
public:
    Stream() : thr_([this] { loop(); }) {}
    ~Stream()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        thr_.join();
    }
    void push(std::function<void()> op)
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            ops_.push_back(std::move(op));
            ++pending_;
        }
        cv_.notify_all();
    }
    void sync()
    {
        std::unique_lock<std::mutex> lk(mu_);
        idle_.wait(lk, [&] { return pending_ == 0; });
    }

private:
    void loop()
    {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return stop_ || !ops_.empty(); });
            if (ops_.empty())
                return;
            std::function<void()> op = std::move(ops_.front());
            ops_.pop_front();
            lk.unlock();
            op();
            lk.lock();
            if (--pending_ == 0)
                idle_.notify_all();
        }
    }
    std::mutex mu_;
    std::condition_variable cv_, idle_;
    std::deque<std::function<void()>> ops_;
    uint64_t pending_ = 0;
    bool stop_ = false;
    std::thread thr_;
};

struct FakeBackend final : grim_serve::Backend {
    int current_device(int *dev) const override
    {
        *dev = t_device;
        return GRIM_OK;
    }
    void set_device(int dev) const override { t_device = dev; }
    int index_device(const grim_index_t *idx) const override { return idx->device; }
    int device_alloc(uint64_t bytes, uint8_t **p) const override
    {
        *p = static_cast<uint8_t *>(std::aligned_alloc(256, (bytes + 255) & ~255ull));
        if (!*p)
            return GRIM_E_NOMEM;
        g_dev_bytes += (int64_t)bytes;
        std::memset(*p, 0xA5, bytes);  // device memory starts with garbage
        dev_sizes().emplace_back(*p, bytes);
        return GRIM_OK;
    }
    void device_free(uint8_t *p) const override
    {
        if (!p)
            return;
        auto &v = dev_sizes();
        for (auto it = v.begin(); it != v.end(); ++it)
            if (it->first == p) {
                g_dev_bytes -= (int64_t)it->second;
                v.erase(it);
                break;
            }
        std::free(p);
    }
    int pinned_alloc(uint64_t bytes, uint8_t **p) const override
    {
        *p = static_cast<uint8_t *>(std::aligned_alloc(256, (bytes + 255) & ~255ull));
        return *p ? GRIM_OK : GRIM_E_NOMEM;
    }
    void pinned_free(uint8_t *p) const override { std::free(p); }
    int stream_create(void **s) const override
    {
        *s = new Stream();
        return GRIM_OK;
    }
    void stream_destroy(void *s) const override { delete static_cast<Stream *>(s); }
    int stream_sync(void *s) const override
    {
        static_cast<Stream *>(s)->sync();
        return GRIM_OK;
    }
    int copy_h2d(void *dst, const void *src, uint64_t bytes, void *s) const override
    {
        static_cast<Stream *>(s)->push([=] { std::memcpy(dst, src, bytes); });
        return GRIM_OK;
    }
    int copy_d2h(void *dst, const void *src, uint64_t bytes, void *s) const override
    {
        static_cast<Stream *>(s)->push([=] { std::memcpy(dst, src, bytes); });
        return GRIM_OK;
    }
    int store_d2h(void *dst, const void *src, uint64_t bytes, void *s) const override
    {
        return copy_d2h(dst, src, bytes, s);
    }
    bool device_writable(const void *p) const override { return !fake_pageable(p); }
    int notify(void *s, void (*fn)(void *), void *arg) const override
    {
        static_cast<Stream *>(s)->push([=] { fn(arg); });
        return GRIM_OK;
    }
    int filter(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
               uint32_t *pass_bits, void *ws, uint64_t ws_bytes, void *s) const override
    {
        const uint64_t call = ++g_calls;
        const uint64_t every = g_fail_every.load();
        if (every && call % every == 0) {
            ++g_failures;
            return GRIM_E_HIP;
        }
        if (!ws || ws_bytes < workspace_bytes(idx, b->n_pairs))
            return GRIM_E_INVALID;
        const grim_batch_t batch = *b;
        const uint64_t n_bins = idx->n_bins;
        static_cast<Stream *>(s)->push([=] {
            uint32_t flags = 0;
            fake_filter_host(&batch, n_bins, counts, pass_bits, &flags);
            *static_cast<uint32_t *>(ws) = flags;
        });
        return GRIM_OK;
    }
    uint64_t workspace_bytes(const grim_index_t *, uint64_t n_pairs) const override
    {
        return (256 + 4 * ((n_pairs + 511) / 512) + 255) & ~255ull;
    }

private:
    static std::deque<std::pair<uint8_t *, uint64_t>> &dev_sizes()
    {
        static std::deque<std::pair<uint8_t *, uint64_t>> v;  // only create/destroy touch it
        return v;
    }
};

}  // namespace

void fake_filter_host(const grim_batch_t *b, uint64_t n_bins, int32_t *counts, uint32_t *bits,
                      uint32_t *flags)
{
    const uint64_t nwords = (b->n_pairs + 31) / 32;
    for (uint64_t w = 0; w < nwords; ++w)
        bits[w] = 0;
    for (uint64_t r = 0; r < b->n_reads; ++r) {
        const uint32_t L = b->read_len[r];
        const uint64_t off = b->read_off[r];
        uint32_t h = 2166136261u;
        for (uint32_t j = 0; j < L; ++j)
            h = (h ^ base_at(b->reads_2bit, off + j)) * 16777619u;
        const uint64_t E = ((uint64_t)b->read_e[r] * L + b->e_den - 1) / b->e_den;
        for (uint64_t k = b->cand_off[r]; k < b->cand_off[r + 1]; ++k) {
            const uint32_t bin = b->cand_bin[k];
            if (bin >= n_bins) {
                counts[k] = -1;
                *flags |= GRIM_FLAG_BIN_RANGE;
                continue;
            }
            const uint32_t x = (h ^ (bin * 2654435761u)) + (uint32_t)E * 40503u;
            const int32_t c = (int32_t)(x % (L + 1u));
            counts[k] = c;
            if ((uint64_t)c * 2 >= L)
                bits[k >> 5] |= 1u << (k & 31);
        }
    }
}

namespace {
std::mutex g_pg_mu;
std::vector<std::pair<uintptr_t, uintptr_t>> g_pageable;
}  // namespace

void fake_mark_pageable(const void *p, uint64_t bytes)
{
    if (!p || !bytes)
        return;
    std::lock_guard<std::mutex> lk(g_pg_mu);
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    g_pageable.emplace_back(a, a + bytes);
}
void fake_clear_pageable(void)
{
    std::lock_guard<std::mutex> lk(g_pg_mu);
    g_pageable.clear();
}
bool fake_pageable(const void *p)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    std::lock_guard<std::mutex> lk(g_pg_mu);
    for (const auto &r : g_pageable)
        if (a >= r.first && a < r.second)
            return true;
    return false;
}

void fake_fail_filter_every(uint64_t every)
{
    g_fail_every = every;
    g_calls = 0;
}
uint64_t fake_filter_calls(void) { return g_calls.load(); }
uint64_t fake_filter_failures(void) { return g_failures.load(); }
int64_t fake_device_bytes(void) { return g_dev_bytes.load(); }

const grim_serve::Backend &grim_serve::backend()
{
    static const FakeBackend b;
    return b;
}
