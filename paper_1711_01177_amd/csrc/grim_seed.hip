// Seeding on the GPU: the k-mer position index of the reference and the
// candidate locations of a read batch (the mapper's hash-table lookup that
// precedes the filter: Kim et al., BMC Genomics 2018, Section "Introduction",
// Fig. 1, and Section "Integration with a Full Read Mapper").
//
// Index: counts of every k-mer (atomic histogram), exclusive scan into
// offsets, scatter of positions.  Candidates, in passes that each keep many
// independent memory accesses in flight:
//   1. per read: its seeds (k-mers at offsets 0, k, 2k, ...) as (read, seed)
//      items, each with its index range (first position, hit count);
//   2. a scan of the items' hit counts lays all hits out read by read;
//   3. per 64 items: the wavefront copies the items' hits, converted to bins
//      (clamp(p - o) / B), to their places (flat, all lanes busy);
//   4. per read: sort its bins (in registers up to 64, in LDS up to 2048, in
//      place in global memory beyond), keep the distinct ones up to the cap;
//   5. a scan of the list lengths and a copy pass write the CSR candidates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "grim_internal.h"

// Result buffers of freed candidate lists, kept for the next lists of the same
// seed index: a free then costs a device synchronisation (as hipFree's does)
// instead of unmapping memory, and a call that finds a buffer allocates
// nothing.  Shared by the index and its lists, so either may go first; at most
// kCachedBuffers are kept, the rest freed.
struct SeedBufferCache {
    static constexpr size_t kCachedBuffers = 2;
    int device = 0;
    std::mutex mu;
    std::vector<std::pair<uint8_t *, uint64_t>> bufs;  // (buffer, bytes)

    // a cached buffer of at least `bytes` bytes and at most twice that (plus
    // 64 MiB), or null
    uint8_t *take(uint64_t bytes, uint64_t *got)
    {
        std::lock_guard<std::mutex> lk(mu);
        size_t best = bufs.size();
        for (size_t i = 0; i < bufs.size(); ++i)
            if (bufs[i].second >= bytes && bufs[i].second <= 2 * bytes + (64ull << 20) &&
                (best == bufs.size() || bufs[i].second < bufs[best].second))
                best = i;
        if (best == bufs.size())
            return nullptr;
        uint8_t *b = bufs[best].first;
        *got = bufs[best].second;
        bufs.erase(bufs.begin() + best);
        return b;
    }
    // keep a buffer no queued work uses any more; the smallest one goes when
    // more than kCachedBuffers are held
    void give(uint8_t *b, uint64_t bytes)
    {
        uint8_t *drop = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu);
            bufs.emplace_back(b, bytes);
            if (bufs.size() > kCachedBuffers) {
                size_t small = 0;
                for (size_t i = 1; i < bufs.size(); ++i)
                    if (bufs[i].second < bufs[small].second)
                        small = i;
                drop = bufs[small].first;
                bufs.erase(bufs.begin() + small);
            }
        }
        (void)hipFree(drop);
    }
    ~SeedBufferCache()
    {
        int cur = 0;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        (void)hipSetDevice(device);
        for (auto &b : bufs)
            (void)hipFree(b.first);
        if (have)
            (void)hipSetDevice(cur);
    }
};

struct grim_seed_index {
    uint32_t k;
    int device;
    uint64_t G;
    uint64_t *d_off;   // 4^k + 1 offsets into d_pos
    uint32_t *d_pos;   // G - k + 1 positions grouped by k-mer
    // device temporaries of grim_seed_candidates, kept between calls (grown
    // when a batch needs more); calls on one seed index take turns on mu
    std::mutex mu;
    uint8_t *tmp[3] = {nullptr, nullptr, nullptr};
    uint64_t tmp_bytes[3] = {0, 0, 0};
    std::shared_ptr<SeedBufferCache> cache;
};

struct grim_candidates {
    uint64_t n_reads, n_pairs;
    uint8_t *buf;      // one allocation: the offsets, then the bins
    uint64_t buf_bytes;
    uint64_t *d_off;   // n_reads + 1
    uint32_t *d_bin;   // n_pairs (at least one element)
    std::shared_ptr<SeedBufferCache> cache;  // where buf goes when the list is freed
};

namespace grim {
namespace {

__device__ __forceinline__ uint32_t kmer_at(const uint32_t *__restrict__ w, uint64_t nw, uint64_t pos,
                                            uint32_t k)
{
    const uint64_t wi = pos >> 4;
    const uint32_t sh = (uint32_t)(pos & 15u) << 1;
    uint64_t x = (uint64_t)(wi < nw ? w[wi] : 0u) << 32;
    if (sh + 2 * k > 32)
        x |= (wi + 1 < nw ? w[wi + 1] : 0u);
    return (uint32_t)((x << sh) >> (64 - 2 * k));
}

__global__ __launch_bounds__(256) void kmer_count_kernel(const uint32_t *__restrict__ ref, uint64_t nw,
                                                         uint64_t G, uint32_t k, uint32_t *cnt)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p + k <= G; p += stride)
        atomicAdd(&cnt[kmer_at(ref, nw, p, k)], 1u);
}

__global__ __launch_bounds__(256) void kmer_fill_kernel(const uint32_t *__restrict__ ref, uint64_t nw,
                                                        uint64_t G, uint32_t k,
                                                        const uint64_t *__restrict__ off,
                                                        uint32_t *cursor, uint32_t *pos)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p + k <= G; p += stride) {
        const uint32_t km = kmer_at(ref, nw, p, k);
        pos[off[km] + atomicAdd(&cursor[km], 1u)] = (uint32_t)p;
    }
}

// ------------------------------------------------------------ scan (u64 out)
// out[i] = sum_{j<i} in[j] for i <= n, in three launches: per-block totals,
// a one-block scan of the totals, and a per-block scan plus the block base.
constexpr int kScanPerThread = 16;
constexpr int kScanPerBlock = 256 * kScanPerThread;

__device__ uint64_t block_scan_u64(uint64_t v, uint64_t *lds, uint64_t *total)
{
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint64_t incl = v;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const uint64_t y = __shfl_up(incl, s);
        if (lane >= s)
            incl += y;
    }
    if (lane == 63)
        lds[wv] = incl;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (int i = 0; i < 4; ++i) {
        if (i < wv)
            before += lds[i];
        all += lds[i];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// Per-block totals; loads strided by the block width so that every load
// instruction reads one contiguous run.
template <typename T>
__global__ __launch_bounds__(256) void scan_totals_kernel(const T *__restrict__ in, uint64_t n,
                                                          uint64_t *block_tot)
{
    __shared__ uint64_t lds[4];
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanPerBlock;
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanPerThread; ++j) {
        const uint64_t i = b0 + (uint64_t)j * 256 + threadIdx.x;
        if (i < n)
            s += in[i];
    }
    uint64_t tot;
    block_scan_u64(s, lds, &tot);
    if (threadIdx.x == 0)
        block_tot[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void scan_tot_kernel(uint64_t *sums, uint64_t n, uint64_t *total)
{
    __shared__ uint64_t part[16];
    __shared__ uint64_t carry_s;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0)
        carry_s = 0;
    __syncthreads();
    for (uint64_t base = 0; base < n; base += 1024) {
        const uint64_t i = base + t;
        const uint64_t v = i < n ? sums[i] : 0;
        uint64_t incl = v;
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) {
            const uint64_t y = __shfl_up(incl, s);
            if (lane >= s)
                incl += y;
        }
        if (lane == 63)
            part[wv] = incl;
        __syncthreads();
        uint64_t before = carry_s, all = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < wv)
                before += part[k];
            all += part[k];
        }
        if (i < n)
            sums[i] = before + incl - v;
        __syncthreads();
        if (t == 0)
            carry_s += all;
        __syncthreads();
    }
    if (t == 0)
        *total = carry_s;
}

// The block's kScanPerBlock inputs go through LDS: loaded and stored with
// contiguous runs per instruction, scanned as 16 consecutive values per thread.
template <typename T>
__global__ __launch_bounds__(256) void scan_apply_kernel(const T *__restrict__ in, uint64_t n,
                                                         const uint64_t *__restrict__ block_base,
                                                         const uint64_t *__restrict__ total,
                                                         uint64_t *__restrict__ out)
{
    __shared__ uint64_t lds[4];
    __shared__ uint64_t vals[kScanPerBlock + kScanPerBlock / 16];  // padded: one word per 16
    const int t = threadIdx.x;
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanPerBlock;
    auto slot = [](uint32_t k) { return k + (k >> 4); };
#pragma unroll
    for (int j = 0; j < kScanPerThread; ++j) {
        const uint32_t k = (uint32_t)j * 256u + (uint32_t)t;
        const uint64_t i = b0 + k;
        vals[slot(k)] = i < n ? (uint64_t)in[i] : 0ull;
    }
    __syncthreads();
    uint64_t v[kScanPerThread];
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanPerThread; ++j) {
        v[j] = vals[slot((uint32_t)t * kScanPerThread + j)];
        sum += v[j];
    }
    uint64_t tot;
    uint64_t run = block_base[blockIdx.x] + block_scan_u64(sum, lds, &tot);
#pragma unroll
    for (int j = 0; j < kScanPerThread; ++j) {
        vals[slot((uint32_t)t * kScanPerThread + j)] = run;
        run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanPerThread; ++j) {
        const uint32_t k = (uint32_t)j * 256u + (uint32_t)t;
        const uint64_t i = b0 + k;
        if (i < n)
            out[i] = vals[slot(k)];
    }
    if (blockIdx.x == 0 && t == 0)
        out[n] = *total;
}

// --------------------------------------------------------------- seeding
// Number of seeds of each read (0 for a read outside the packed buffer or, when
// max_len > 0, longer than max_len).
__global__ __launch_bounds__(256) void seed_nseeds_kernel(const uint64_t *__restrict__ read_off,
                                                          const uint32_t *__restrict__ read_len,
                                                          uint64_t n_reads, uint64_t nw, uint32_t k,
                                                          uint32_t max_len,
                                                          uint32_t *__restrict__ nseeds)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t nb = nw * 16;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_reads; r += stride) {
        const uint32_t L = read_len[r];
        const uint64_t off = read_off[r];
        const bool ok = off <= nb && L <= nb - off && L >= k && (max_len == 0 || L <= max_len);
        nseeds[r] = ok ? L / k : 0u;
    }
}

// One thread per read: its seeds' items at item_base[r] + s (index range start
// a, hit count, seed offset o = s * k in the read).
__global__ __launch_bounds__(256) void seed_items_kernel(
    const uint32_t *__restrict__ rw, uint64_t nw, const uint64_t *__restrict__ read_off,
    const uint64_t *__restrict__ item_base, uint64_t n_reads, uint32_t k,
    const uint64_t *__restrict__ idx_off, uint32_t *__restrict__ item_a,
    uint32_t *__restrict__ item_cnt, uint32_t *__restrict__ item_o)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_reads; r += stride) {
        const uint64_t i0 = item_base[r], ns = item_base[r + 1] - i0;
        const uint64_t off = read_off[r];
        for (uint64_t s = 0; s < ns; ++s) {
            const uint32_t km = kmer_at(rw, nw, off + s * k, k);
            const uint64_t a = idx_off[km];
            item_a[i0 + s] = (uint32_t)a;
            item_cnt[i0 + s] = (uint32_t)(idx_off[km + 1] - a);
            item_o[i0 + s] = (uint32_t)(s * k);
        }
    }
}

// The same items in a fixed layout, one thread per item: item i is seed
// i % S of read i / S, S = max_len / k seeds per read (a read longer than
// max_len gets no seeds).
__global__ __launch_bounds__(256) void seed_items_fixed_kernel(
    const uint32_t *__restrict__ rw, uint64_t nw, const uint64_t *__restrict__ read_off,
    const uint32_t *__restrict__ read_len, uint64_t n_items, uint32_t S, uint32_t max_len,
    uint32_t k, const uint64_t *__restrict__ idx_off, uint32_t *__restrict__ item_a,
    uint32_t *__restrict__ item_cnt, uint32_t *__restrict__ item_o)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t nb = nw * 16;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += stride) {
        const uint64_t r = i / S;
        const uint32_t sd = (uint32_t)(i - r * S);
        const uint32_t L = read_len[r];
        const uint64_t off = read_off[r];
        uint64_t a = 0, cnt = 0;
        if (off <= nb && L <= nb - off && L <= max_len && (uint64_t)(sd + 1) * k <= L) {
            const uint32_t km = kmer_at(rw, nw, off + (uint64_t)sd * k, k);
            a = idx_off[km];
            cnt = idx_off[km + 1] - a;
        }
        item_a[i] = (uint32_t)a;
        item_cnt[i] = (uint32_t)cnt;
        item_o[i] = sd * k;
    }
}

// hit_off[r] = item_off[item_base[r]] (item_base null: r * S) for r <= n_reads;
// thread 0 also clears the long-list counter.
__global__ __launch_bounds__(256) void seed_hit_off_kernel(const uint64_t *__restrict__ item_base,
                                                           uint64_t S,
                                                           const uint64_t *__restrict__ item_off,
                                                           uint64_t n_reads,
                                                           uint64_t *__restrict__ hit_off,
                                                           uint32_t *__restrict__ long_count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0)
        *long_count = 0u;
    for (uint64_t r = i0; r <= n_reads; r += stride)
        hit_off[r] = item_off[item_base ? item_base[r] : r * S];
}

// One wavefront per 64 consecutive items: every lane takes one hit at a time
// of the items' hit range (its item found by a binary search over the lanes'
// offsets), four loads in flight per lane, and writes the hit's bin at its
// place.  Works whatever the items' hit counts (a single item may hold most of
// the range).
__global__ __launch_bounds__(256) void seed_emit_kernel(
    const uint32_t *__restrict__ item_a, const uint32_t *__restrict__ item_o,
    const uint64_t *__restrict__ item_off, uint64_t n_items,
    const uint32_t *__restrict__ idx_pos, uint64_t G, uint64_t B, uint32_t *__restrict__ hb)
{
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t i0 = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * kWave;
         i0 < n_items; i0 += waves * kWave) {
        const uint32_t ns = (uint32_t)min<uint64_t>(kWave, n_items - i0);
        const uint64_t i = i0 + lane;
        const uint64_t first = item_off[i0];
        // offsets within the group fit 32 bits: a call has fewer than 2^31 hits
        const uint32_t excl = (uint32_t)((lane < (int)ns ? item_off[i] : item_off[i0 + ns]) - first);
        const uint32_t a = lane < (int)ns ? item_a[i] : 0u;
        const uint32_t o = lane < (int)ns ? item_o[i] : 0u;
        const uint32_t total = (uint32_t)(item_off[i0 + ns] - first);
        constexpr int U = 4;
        for (uint32_t e0 = 0; e0 < total; e0 += (uint32_t)U * kWave) {
            uint32_t p[U];
            int64_t po[U];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t e = e0 + (uint32_t)u * kWave + lane;
                // the item of hit e: the last item j < ns whose hits start at or before e
                int pos = 0;
#pragma unroll
                for (int step = kWave / 2; step >= 1; step >>= 1) {
                    const int cand = pos + step;
                    const uint32_t ec = __shfl(excl, cand);
                    if (cand < (int)ns && ec <= e)
                        pos = cand;
                }
                const uint32_t ap = __shfl(a, pos), ep = __shfl(excl, pos);
                po[u] = (int64_t)__shfl(o, pos);
                ok[u] = e < total;
                p[u] = ok[u] ? idx_pos[(uint64_t)ap + (e - ep)] : 0u;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (ok[u]) {
                    int64_t z = (int64_t)p[u] - po[u];
                    if (z < 0)
                        z = 0;
                    if ((uint64_t)z > G - 1)
                        z = (int64_t)(G - 1);
                    // z < G < 2^32: a 32-bit division (every bin is 0 for B >= 2^32)
                    hb[first + e0 + (uint32_t)u * kWave + lane] =
                        (B >> 32) ? 0u : (uint32_t)z / (uint32_t)B;
                }
            }
        }
    }
}

// Wavefront-scope ordering of a wavefront's own LDS traffic between steps.
__device__ __forceinline__ void seed_wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Sorting network for m keys held in x[0 .. m), ascending, P = the power of two
// >= m: bitonic merges in the form whose comparators all put the smaller key
// at the lower index (the first step of stage k pairs i with i ^ (k - 1)).
// Keys at indices >= m act as +infinity and never move down, so comparators
// that reach past m are skipped and nothing is padded.  Each comparator is
// handled by one of n_threads threads; `fence` orders the steps.
template <typename Arr, typename Fence>
__device__ __forceinline__ void sort_keys(Arr x, uint64_t m, int lane, Fence fence,
                                          int n_threads = kWave)
{
    uint64_t P = 1;
    while (P < m)
        P <<= 1;
    for (uint64_t k = 2; k <= P; k <<= 1) {
        for (uint64_t j = k >> 1; j >= 1; j >>= 1) {
            for (uint64_t c = lane; c < P / 2; c += n_threads) {
                // c-th comparator of the step: lower index lo, partner hi
                const uint64_t lo = ((c / j) * 2 * j) + (c % j);
                const uint64_t hi = j == (k >> 1) ? (lo | (k - 1)) - (lo & (k - 1)) : lo + j;
                const uint64_t a = lo < hi ? lo : hi, b = lo < hi ? hi : lo;
                if (b < m) {
                    const uint32_t va = x[a], vb = x[b];
                    if (vb < va) {
                        x[a] = vb;
                        x[b] = va;
                    }
                }
            }
            fence();
        }
    }
}

// The same network on one key per lane (m <= 64 keys; lanes >= m hold +inf),
// with the partners exchanged by cross-lane moves; only the stages up to the
// power of two P >= m run (each block of P lanes is sorted on its own, and the
// first one holds every key).
__device__ __forceinline__ uint32_t sort_lanes(uint32_t v, int lane, uint32_t m)
{
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1) {
        if ((uint32_t)(k >> 1) >= m)
            break;
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
            const int partner = j == (k >> 1) ? (lane ^ (k - 1)) : (lane ^ j);
            const uint32_t w = __shfl(v, partner);
            v = lane < partner ? min(v, w) : max(v, w);
        }
    }
    return v;
}

// Distinct keys of the sorted x[0 .. m), at most cap of them, to out[0 ..);
// returns how many (<= cap).  out may be x itself: writes never pass the
// position being read, and the last key of a chunk is carried in a register.
template <typename Src>
__device__ __forceinline__ uint64_t unique_keys(Src x, uint64_t m, uint32_t cap, uint32_t *out,
                                                int lane)
{
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t u = 0;
    uint32_t carry = 0;
    for (uint64_t base = 0; base < m && u < cap; base += kWave) {
        const uint64_t i = base + lane;
        const uint32_t v = i < m ? x[i] : 0u;
        const uint32_t prev = __shfl_up(v, 1);
        const bool first = i < m && (i == 0 || (lane == 0 ? carry : prev) != v);
        const uint64_t mk = __ballot(first);
        const uint64_t pos = u + __popcll(mk & below);
        carry = __shfl(v, kWave - 1);
        if (first && pos < cap)
            out[pos] = v;
        u += __popcll(mk);
    }
    return u < cap ? u : cap;
}

// The same network on R keys per lane (64 R keys, key e = r * 64 + lane in
// v[r], keys past the read's end +infinity): steps between keys 64 or more
// apart exchange registers of one lane, the others exchange one register
// between lanes; the first step of a stage above 64 does both (key e pairs
// with e ^ (k - 1): lane ^ 63 in register r ^ ((k - 1) >> 6)).
template <int R>
__device__ __forceinline__ void sort_regs(uint32_t (&v)[R], int lane)
{
    constexpr int P = kWave * R;
#pragma unroll
    for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
            const bool flip = j == (k >> 1);
            if (flip && k > kWave) {
                const int rm = (k - 1) >> 6;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int r2 = r ^ rm;
                    if (r < r2) {
                        const uint32_t t1 = __shfl(v[r2], lane ^ (kWave - 1));
                        const uint32_t t2 = __shfl(v[r], lane ^ (kWave - 1));
                        v[r] = min(v[r], t1);
                        v[r2] = max(v[r2], t2);
                    }
                }
            } else if (j >= kWave) {
                const int rm = j >> 6;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int r2 = r ^ rm;
                    if (r < r2) {
                        const uint32_t a = v[r], b = v[r2];
                        v[r] = min(a, b);
                        v[r2] = max(a, b);
                    }
                }
            } else {
                const int partner = flip ? (lane ^ (k - 1)) : (lane ^ j);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t w = __shfl(v[r], partner);
                    v[r] = lane < partner ? min(v[r], w) : max(v[r], w);
                }
            }
        }
    }
}

// Distinct keys of the sorted registers (key e = r * 64 + lane, m keys), at
// most cap of them, to out[0 ..); returns how many.  out may hold the keys'
// source: every key is in registers before the first store.
template <int R>
__device__ __forceinline__ uint64_t unique_regs(const uint32_t (&v)[R], uint64_t m, uint32_t cap,
                                                uint32_t *out, int lane)
{
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t u = 0;
    uint32_t carry = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t e = (uint64_t)r * kWave + lane;
        const uint32_t x = v[r];
        const uint32_t prev = __shfl_up(x, 1);
        const bool first = e < m && (e == 0 || (lane == 0 ? carry : prev) != x);
        const uint64_t mk = __ballot(first);
        const uint64_t pos = u + __popcll(mk & below);
        carry = __shfl(x, kWave - 1);
        if (first && pos < cap)
            out[pos] = x;
        u += __popcll(mk);
    }
    return u < cap ? u : cap;
}

// One read's 64 < m <= 64 R hits: loaded into registers, sorted, reduced in place.
template <int R>
__device__ __forceinline__ uint64_t sort_unique_regs(uint32_t *hits, uint64_t m, uint32_t cap,
                                                     int lane)
{
    uint32_t v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t e = (uint64_t)r * kWave + lane;
        v[r] = e < m ? hits[e] : 0xffffffffu;
    }
    sort_regs<R>(v, lane);
    return unique_regs<R>(v, m, cap, hits, lane);
}

// Per read: its hit bins hb[hit_off[r] ..+ m) reduced to the distinct ones,
// ascending, up to the cap, written back in place from hit_off[r]; their number
// to ucnt[r].  seed_sort_kernel takes kSortReads consecutive reads per
// wavefront (their hit ranges and short lists loaded together) and sorts each
// read's hits in registers: one per lane up to 64, else R = 2 .. 8 per lane
// (up to kMidCap); longer reads go to a list that seed_sort_wide_kernel works
// through one wavefront per read with 16 or 32 keys per lane (up to kWideCap)
// and seed_sort_long_kernel one workgroup per read beyond that, sorting
// kSortCap hits in LDS and longer lists in place in global memory.
constexpr uint32_t kMidCap = 512;
constexpr uint32_t kWideCap = 2048;
constexpr uint32_t kSortCap = 8192;
constexpr int kSortWaves = 4;

constexpr int kSortReads = 4;  // consecutive reads per wavefront, their loads in flight together

__global__ __launch_bounds__(kSortWaves * kWave) void seed_sort_kernel(
    const uint64_t *__restrict__ hit_off, uint64_t n_reads, uint32_t cap, uint32_t *__restrict__ hb,
    uint64_t *__restrict__ ucnt, uint32_t *__restrict__ long_list,
    uint32_t *__restrict__ long_count)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t r0 = ((uint64_t)blockIdx.x * kSortWaves + wv) * kSortReads;
    if (r0 >= n_reads)
        return;
    const int nq = (int)min<uint64_t>(kSortReads, n_reads - r0);
    // the reads' hit ranges (lanes 0 .. nq), then every short read's hits
    const uint64_t ho = lane <= nq ? hit_off[r0 + lane] : 0u;
    uint64_t h[kSortReads + 1];
#pragma unroll
    for (int q = 0; q <= kSortReads; ++q)
        h[q] = __shfl(ho, q);
    uint32_t v[kSortReads];
#pragma unroll
    for (int q = 0; q < kSortReads; ++q) {
        const uint64_t m = q < nq ? h[q + 1] - h[q] : 0u;
        v[q] = (m <= (uint64_t)kWave && lane < (int)m) ? hb[h[q] + lane] : 0xffffffffu;
    }
#pragma unroll
    for (int q = 0; q < kSortReads; ++q) {
        if (q >= nq)
            break;
        const uint64_t m = h[q + 1] - h[q];
        const uint64_t r = r0 + q;
        uint32_t *hits = hb + h[q];
        uint64_t u = 0;
        if (m > kMidCap) {
            if (lane == 0)
                long_list[atomicAdd(long_count, 1u)] = (uint32_t)r;
            continue;
        } else if (m > 128) {
            u = m > 256 ? sort_unique_regs<8>(hits, m, cap, lane)
                        : sort_unique_regs<4>(hits, m, cap, lane);
        } else if (m > (uint64_t)kWave) {
            u = sort_unique_regs<2>(hits, m, cap, lane);
        } else if (m > 0) {
            const uint32_t w[1] = {sort_lanes(v[q], lane, (uint32_t)m)};
            u = unique_regs<1>(w, m, cap, hits, lane);
        }
        if (lane == 0)
            ucnt[r] = u;
    }
}

// Reads of the long list with at most kWideCap hits, one wavefront each, 16
// or 32 keys per lane in registers.
__global__ __launch_bounds__(256) void seed_sort_wide_kernel(
    const uint64_t *__restrict__ hit_off, uint32_t cap, uint32_t *__restrict__ hb,
    uint64_t *__restrict__ ucnt, const uint32_t *__restrict__ long_list,
    const uint32_t *__restrict__ long_count)
{
    const int lane = threadIdx.x & 63;
    const uint64_t n = *long_count;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t j = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); j < n;
         j += waves) {
        const uint64_t r = long_list[j];
        const uint64_t h0 = hit_off[r], m = hit_off[r + 1] - h0;
        if (m > kWideCap)
            continue;  // seed_sort_long_kernel's
        const uint64_t u = m > 1024 ? sort_unique_regs<32>(hb + h0, m, cap, lane)
                                    : sort_unique_regs<16>(hb + h0, m, cap, lane);
        if (lane == 0)
            ucnt[r] = u;
    }
}

// Reads of the long list with more than kWideCap hits, one workgroup each.
__global__ __launch_bounds__(256) void seed_sort_long_kernel(
    const uint64_t *__restrict__ hit_off, uint32_t cap, uint32_t *__restrict__ hb,
    uint64_t *__restrict__ ucnt, const uint32_t *__restrict__ long_list,
    const uint32_t *__restrict__ long_count)
{
    __shared__ uint32_t keys[kSortCap];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint64_t n = *long_count;
    for (uint64_t j = blockIdx.x; j < n; j += gridDim.x) {
        const uint64_t r = long_list[j];
        const uint64_t h0 = hit_off[r], m = hit_off[r + 1] - h0;
        uint32_t *hits = hb + h0;
        if (m <= kWideCap)
            continue;  // seed_sort_wide_kernel's
        if (m <= kSortCap) {
            for (uint64_t i = t; i < m; i += blockDim.x)
                keys[i] = hits[i];
            __syncthreads();
            sort_keys(keys, m, t, [] { __syncthreads(); }, (int)blockDim.x);
            if (wv == 0) {
                const uint64_t u = unique_keys(keys, m, cap, hits, lane);
                if (lane == 0)
                    ucnt[r] = u;
            }
        } else {
            // in place in global memory; every step's stores are made visible
            // to the workgroup's next loads
            __threadfence();
            __syncthreads();
            sort_keys(hits, m, t, [] { __threadfence(); __syncthreads(); }, (int)blockDim.x);
            if (wv == 0) {
                const uint64_t u = unique_keys(hits, m, cap, hits, lane);
                if (lane == 0)
                    ucnt[r] = u;
            }
        }
        __syncthreads();  // keys reused by the workgroup's next read
    }
}

// Groups of 16 lanes, one read per group: its list, list[hit_off[r] ..+
// ucnt[r]), to the CSR candidates at out[cand_off[r] ..].
constexpr int kCopyGroup = 16;
constexpr int kCopyBatch = 8;

__global__ __launch_bounds__(256) void seed_compact_kernel(const uint32_t *__restrict__ list,
                                                           const uint64_t *__restrict__ hit_off,
                                                           const uint64_t *__restrict__ cand_off,
                                                           uint64_t n_reads,
                                                           uint32_t *__restrict__ out)
{
    // the group's next read's offsets load while this one is copied, and each
    // lane loads kCopyBatch values before it stores any, so that a read of up
    // to kCopyGroup * kCopyBatch bins costs one round trip
    const int sub = threadIdx.x % kCopyGroup;
    const uint64_t groups = (uint64_t)gridDim.x * (blockDim.x / kCopyGroup);
    uint64_t r = (uint64_t)blockIdx.x * (blockDim.x / kCopyGroup) + threadIdx.x / kCopyGroup;
    uint64_t src = 0, dst = 0, end = 0;
    if (r < n_reads) {
        src = hit_off[r];
        dst = cand_off[r];
        end = cand_off[r + 1];
    }
    for (; r < n_reads; r += groups) {
        const uint64_t rn = r + groups;
        uint64_t nsrc = 0, ndst = 0, nend = 0;
        if (rn < n_reads) {
            nsrc = hit_off[rn];
            ndst = cand_off[rn];
            nend = cand_off[rn + 1];
        }
        const uint64_t n = end - dst;
        for (uint64_t base = 0; base < n; base += kCopyGroup * kCopyBatch) {
            uint32_t v[kCopyBatch];
#pragma unroll
            for (int j = 0; j < kCopyBatch; ++j) {
                const uint64_t i = base + j * kCopyGroup + sub;
                v[j] = i < n ? list[src + i] : 0u;
            }
#pragma unroll
            for (int j = 0; j < kCopyBatch; ++j) {
                const uint64_t i = base + j * kCopyGroup + sub;
                if (i < n)
                    out[dst + i] = v[j];
            }
        }
        src = nsrc;
        dst = ndst;
        end = nend;
    }
}

hipError_t scan_u64(hipStream_t s, const void *in, bool in_u32, uint64_t n, uint64_t *out,
                    uint64_t *block_tmp, uint64_t *total_tmp)
{
    const uint64_t nb = (n + kScanPerBlock - 1) / kScanPerBlock;
    const uint64_t blocks = nb ? nb : 1;
    if (in_u32)
        hipLaunchKernelGGL(scan_totals_kernel<uint32_t>, dim3((uint32_t)blocks), dim3(256), 0, s,
                           static_cast<const uint32_t *>(in), n, block_tmp);
    else
        hipLaunchKernelGGL(scan_totals_kernel<uint64_t>, dim3((uint32_t)blocks), dim3(256), 0, s,
                           static_cast<const uint64_t *>(in), n, block_tmp);
    hipLaunchKernelGGL(scan_tot_kernel, dim3(1), dim3(1024), 0, s, block_tmp, blocks, total_tmp);
    if (in_u32)
        hipLaunchKernelGGL(scan_apply_kernel<uint32_t>, dim3((uint32_t)blocks), dim3(256), 0, s,
                           static_cast<const uint32_t *>(in), n, block_tmp, total_tmp, out);
    else
        hipLaunchKernelGGL(scan_apply_kernel<uint64_t>, dim3((uint32_t)blocks), dim3(256), 0, s,
                           static_cast<const uint64_t *>(in), n, block_tmp, total_tmp, out);
    return hipGetLastError();
}

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

uint64_t scan_blocks(uint64_t n) { return std::max<uint64_t>(1, (n + kScanPerBlock - 1) / kScanPerBlock); }

uint32_t grid_for(uint64_t threads, int dev)
{
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
        cu = 256;
    uint64_t g = (threads + 255) / 256;
    const uint64_t cap = (uint64_t)cu * 16;
    if (g > cap)
        g = cap;
    return (uint32_t)(g ? g : 1);
}

}  // namespace
}  // namespace grim

using namespace grim;

#define SEED_TRY(x)                 \
    do {                            \
        if ((x) != hipSuccess) {    \
            rc = GRIM_E_HIP;        \
            goto done;              \
        }                           \
    } while (0)

extern "C" int grim_seed_index_build(const uint32_t *ref_2bit, uint64_t ref_len, uint32_t k,
                                     grim_seed_index_t **out, void *stream)
{
    if (!ref_2bit || !out || ref_len == 0)
        return GRIM_E_INVALID;
    if (k < 4 || k > 15 || ref_len < k || ref_len > 0xffffffffull)
        return GRIM_E_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return GRIM_E_HIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint64_t nk = 1ull << (2 * k);
    const uint64_t nw = grim_packed_words(ref_len);
    const uint64_t npos = ref_len - k + 1;
    int rc = GRIM_OK;
    uint32_t *d_ref = nullptr, *cnt = nullptr;
    uint64_t *btmp = nullptr;
    grim_seed_index *si = new (std::nothrow) grim_seed_index();
    if (!si)
        return GRIM_E_NOMEM;
    si->k = k;
    si->device = dev;
    si->G = ref_len;
    si->d_off = nullptr;
    si->d_pos = nullptr;
    si->cache = std::shared_ptr<SeedBufferCache>(new (std::nothrow) SeedBufferCache());
    if (!si->cache) {
        delete si;
        return GRIM_E_NOMEM;
    }
    si->cache->device = dev;
    if (hipMalloc(&d_ref, nw * 4) != hipSuccess || hipMalloc(&cnt, nk * 4) != hipSuccess ||
        hipMalloc(&btmp, (scan_blocks(nk) + 1) * 8) != hipSuccess ||
        hipMalloc(&si->d_off, (nk + 1) * 8) != hipSuccess ||
        hipMalloc(&si->d_pos, npos * 4) != hipSuccess) {
        rc = GRIM_E_NOMEM;
        goto done;
    }
    SEED_TRY(hipMemcpyAsync(d_ref, ref_2bit, nw * 4, hipMemcpyHostToDevice, s));
    SEED_TRY(hipMemsetAsync(cnt, 0, nk * 4, s));
    hipLaunchKernelGGL(kmer_count_kernel, dim3(grid_for(npos, dev)), dim3(256), 0, s, d_ref, nw,
                       ref_len, k, cnt);
    SEED_TRY(hipGetLastError());
    SEED_TRY(scan_u64(s, cnt, true, nk, si->d_off, btmp, btmp + scan_blocks(nk)));
    SEED_TRY(hipMemsetAsync(cnt, 0, nk * 4, s));  // reused as per-k-mer cursor
    hipLaunchKernelGGL(kmer_fill_kernel, dim3(grid_for(npos, dev)), dim3(256), 0, s, d_ref, nw,
                       ref_len, k, si->d_off, cnt, si->d_pos);
    SEED_TRY(hipGetLastError());
    SEED_TRY(hipStreamSynchronize(s));
done:
    (void)hipFree(d_ref);
    (void)hipFree(cnt);
    (void)hipFree(btmp);
    if (rc != GRIM_OK) {
        (void)hipFree(si->d_off);
        (void)hipFree(si->d_pos);
        delete si;
        return rc;
    }
    *out = si;
    return GRIM_OK;
}

extern "C" void grim_seed_index_free(grim_seed_index_t *si)
{
    if (!si)
        return;
    (void)hipFree(si->d_off);
    (void)hipFree(si->d_pos);
    for (uint8_t *t : si->tmp)
        (void)hipFree(t);
    delete si;
}

namespace {

// Temporary i of a seed index with at least `bytes` bytes (grown by a quarter
// more than asked when it has to grow); null when the allocation fails.
uint8_t *seed_tmp(grim_seed_index *si, int i, uint64_t bytes)
{
    if (si->tmp_bytes[i] >= bytes && si->tmp[i])
        return si->tmp[i];
    (void)hipFree(si->tmp[i]);
    si->tmp[i] = nullptr;
    si->tmp_bytes[i] = 0;
    const uint64_t want = align_up(bytes + bytes / 4, 256);
    if (hipMalloc(&si->tmp[i], want) != hipSuccess) {
        si->tmp[i] = nullptr;
        return nullptr;
    }
    si->tmp_bytes[i] = want;
    return si->tmp[i];
}

}  // namespace

extern "C" int grim_seed_candidates(const grim_seed_index_t *csi, const grim_batch_t *reads,
                                    uint64_t bin_stride, uint32_t cap, grim_candidates_t **out,
                                    void *stream)
{
    if (!csi || !reads || !out || bin_stride == 0 || cap == 0)
        return GRIM_E_INVALID;
    // the index's vectors are not touched; only its cached temporaries change
    grim_seed_index *si = const_cast<grim_seed_index *>(csi);
    const uint64_t n = reads->n_reads;
    if (n && (!reads->reads_2bit || !reads->read_off || !reads->read_len))
        return GRIM_E_INVALID;
    if (n >= 0x7fffffffull)
        return GRIM_E_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != si->device)
        return GRIM_E_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int rc = GRIM_OK;
    uint32_t *nseeds = nullptr, *long_list = nullptr, *long_count = nullptr;
    uint64_t *item_base = nullptr, *hit_off = nullptr, *ucnt = nullptr, *btmp = nullptr;
    uint32_t *item_a = nullptr, *item_cnt = nullptr, *item_o = nullptr, *hb = nullptr;
    uint64_t *item_off = nullptr, *itmp = nullptr;
    uint8_t *tmp_reads = nullptr, *tmp_items = nullptr;
    uint64_t n_items = 0, total_hits = 0, n_pairs = 0;
    grim_candidates *c = new (std::nothrow) grim_candidates();
    if (!c)
        return GRIM_E_NOMEM;
    c->n_reads = n;
    c->buf = nullptr;
    c->d_off = nullptr;
    c->d_bin = nullptr;
    std::lock_guard<std::mutex> lk(si->mu);
    const uint64_t nbt = scan_blocks(n + 1) + 1;
    // fixed item layout: S = max_len / k slots per read, if max_len is given and
    // n * S stays within 2^26 items
    const uint32_t S = reads->max_len ? std::max<uint32_t>(1, reads->max_len / si->k) : 0u;
    const bool fixed = S && n * (uint64_t)S <= (1ull << 26);
    {
        // per read: seed counts, item bases, hit offsets, list lengths, the
        // long-read list and its counter, scan block sums
        const uint64_t r4 = align_up((n + 1) * 4, 256), r8 = align_up((n + 1) * 8, 256);
        const uint64_t b8 = align_up(nbt * 8, 256);
        tmp_reads = seed_tmp(si, 0, 2 * r4 + 3 * r8 + 256 + b8);
        if (!tmp_reads) {
            rc = GRIM_E_NOMEM;
            goto done;
        }
        nseeds = reinterpret_cast<uint32_t *>(tmp_reads);
        long_list = reinterpret_cast<uint32_t *>(tmp_reads + r4);
        item_base = reinterpret_cast<uint64_t *>(tmp_reads + 2 * r4);
        hit_off = reinterpret_cast<uint64_t *>(tmp_reads + 2 * r4 + r8);
        ucnt = reinterpret_cast<uint64_t *>(tmp_reads + 2 * r4 + 2 * r8);
        long_count = reinterpret_cast<uint32_t *>(tmp_reads + 2 * r4 + 3 * r8);
        btmp = reinterpret_cast<uint64_t *>(tmp_reads + 2 * r4 + 3 * r8 + 256);
    }
    // the (read, seed) items: a fixed number S = max_len / k of slots per read
    // when that stays small, else exactly each read's seeds (counted and scanned)
    if (fixed) {
        n_items = n * S;
    } else {
        if (n) {
            hipLaunchKernelGGL(seed_nseeds_kernel, dim3(grid_for(n, dev)), dim3(256), 0, s,
                               reads->read_off, reads->read_len, n, reads->n_read_words, si->k,
                               reads->max_len, nseeds);
            SEED_TRY(hipGetLastError());
        }
        SEED_TRY(scan_u64(s, nseeds, true, n, item_base, btmp, btmp + nbt - 1));
        SEED_TRY(hipMemcpyAsync(&n_items, item_base + n, 8, hipMemcpyDeviceToHost, s));
        SEED_TRY(hipStreamSynchronize(s));
    }
    {
        const uint64_t i4 = align_up((n_items + 1) * 4, 256), i8 = align_up((n_items + 1) * 8, 256);
        const uint64_t ib = align_up((scan_blocks(n_items) + 1) * 8, 256);
        tmp_items = seed_tmp(si, 1, 3 * i4 + i8 + ib);
        if (!tmp_items) {
            rc = GRIM_E_NOMEM;
            goto done;
        }
        item_a = reinterpret_cast<uint32_t *>(tmp_items);
        item_cnt = reinterpret_cast<uint32_t *>(tmp_items + i4);
        item_o = reinterpret_cast<uint32_t *>(tmp_items + 2 * i4);
        item_off = reinterpret_cast<uint64_t *>(tmp_items + 3 * i4);
        itmp = reinterpret_cast<uint64_t *>(tmp_items + 3 * i4 + i8);
    }
    if (fixed && n_items) {
        hipLaunchKernelGGL(seed_items_fixed_kernel, dim3(grid_for(n_items, dev)), dim3(256), 0, s,
                           reads->reads_2bit, reads->n_read_words, reads->read_off,
                           reads->read_len, n_items, S, reads->max_len, si->k, si->d_off, item_a,
                           item_cnt, item_o);
        SEED_TRY(hipGetLastError());
    } else if (!fixed && n) {
        hipLaunchKernelGGL(seed_items_kernel, dim3(grid_for(n, dev)), dim3(256), 0, s,
                           reads->reads_2bit, reads->n_read_words, reads->read_off, item_base, n,
                           si->k, si->d_off, item_a, item_cnt, item_o);
        SEED_TRY(hipGetLastError());
    }
    SEED_TRY(scan_u64(s, item_cnt, true, n_items, item_off, itmp,
                      itmp + scan_blocks(n_items)));
    hipLaunchKernelGGL(seed_hit_off_kernel, dim3(grid_for(n + 1, dev)), dim3(256), 0, s,
                       fixed ? nullptr : item_base, (uint64_t)S, item_off, n, hit_off, long_count);
    SEED_TRY(hipGetLastError());
    SEED_TRY(hipMemcpyAsync(&total_hits, item_off + n_items, 8, hipMemcpyDeviceToHost, s));
    SEED_TRY(hipStreamSynchronize(s));
    if (total_hits >= 0x7fffffffull) {
        rc = GRIM_E_UNSUPPORTED;
        goto done;
    }
    // every hit's bin, then the per-read lists in place; the result (offsets
    // and bins in one allocation) is no longer than the hits together
    hb = reinterpret_cast<uint32_t *>(seed_tmp(si, 2, (total_hits + 1) * 4));
    {
        const uint64_t need = align_up((n + 1) * 8, 256) + (total_hits + 1) * 4;
        c->buf = si->cache->take(need, &c->buf_bytes);
        if (!c->buf) {
            c->buf_bytes = align_up(need, 2ull << 20);
            if (hipMalloc(&c->buf, c->buf_bytes) != hipSuccess)
                c->buf = nullptr;
        }
    }
    if (!hb || !c->buf) {
        rc = GRIM_E_NOMEM;
        goto done;
    }
    c->cache = si->cache;
    c->d_off = reinterpret_cast<uint64_t *>(c->buf);
    c->d_bin = reinterpret_cast<uint32_t *>(c->buf + align_up((n + 1) * 8, 256));
    if (n) {
        if (n_items) {
            hipLaunchKernelGGL(seed_emit_kernel, dim3(grid_for(n_items, dev)), dim3(256), 0, s,
                               item_a, item_o, item_off, n_items, si->d_pos, si->G, bin_stride, hb);
            SEED_TRY(hipGetLastError());
        }
        const uint64_t per_block = (uint64_t)kSortWaves * kSortReads;
        hipLaunchKernelGGL(seed_sort_kernel, dim3((uint32_t)((n + per_block - 1) / per_block)),
                           dim3(kSortWaves * kWave), 0, s, hit_off, n, cap, hb, ucnt, long_list,
                           long_count);
        SEED_TRY(hipGetLastError());
    }
    if (n) {
        hipLaunchKernelGGL(seed_sort_wide_kernel, dim3(grid_for((uint64_t)256 * 8 * 256, dev)),
                           dim3(256), 0, s, hit_off, cap, hb, ucnt, long_list, long_count);
        SEED_TRY(hipGetLastError());
        hipLaunchKernelGGL(seed_sort_long_kernel, dim3(grid_for((uint64_t)256 * 8 * 256, dev)),
                           dim3(256), 0, s, hit_off, cap, hb, ucnt, long_list, long_count);
        SEED_TRY(hipGetLastError());
    }
    SEED_TRY(scan_u64(s, ucnt, false, n, c->d_off, btmp, btmp + nbt - 1));
    if (n) {
        hipLaunchKernelGGL(seed_compact_kernel, dim3(grid_for(n * kCopyGroup, dev)), dim3(256), 0,
                           s, hb, hit_off, c->d_off, n, c->d_bin);
        SEED_TRY(hipGetLastError());
    }
    SEED_TRY(hipMemcpyAsync(&n_pairs, c->d_off + n, 8, hipMemcpyDeviceToHost, s));
    SEED_TRY(hipStreamSynchronize(s));
    c->n_pairs = n_pairs;
done:
    if (rc != GRIM_OK) {
        (void)hipFree(c->buf);
        delete c;
        return rc;
    }
    *out = c;
    return GRIM_OK;
}

extern "C" int grim_candidates_info(const grim_candidates_t *c, uint64_t *n_reads,
                                    uint64_t *n_pairs, const uint64_t **cand_off,
                                    const uint32_t **cand_bin)
{
    if (!c)
        return GRIM_E_INVALID;
    if (n_reads)
        *n_reads = c->n_reads;
    if (n_pairs)
        *n_pairs = c->n_pairs;
    if (cand_off)
        *cand_off = c->d_off;
    if (cand_bin)
        *cand_bin = c->d_bin;
    return GRIM_OK;
}

extern "C" int grim_candidates_copy_to_host(const grim_candidates_t *c, uint64_t *cand_off,
                                            uint32_t *cand_bin)
{
    if (!c || !cand_off || (c->n_pairs && !cand_bin))
        return GRIM_E_INVALID;
    if (hipMemcpy(cand_off, c->d_off, (c->n_reads + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return GRIM_E_HIP;
    if (c->n_pairs &&
        hipMemcpy(cand_bin, c->d_bin, c->n_pairs * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return GRIM_E_HIP;
    return GRIM_OK;
}

extern "C" void grim_candidates_free(grim_candidates_t *c)
{
    if (!c)
        return;
    if (c->buf) {
        if (c->cache && hipDeviceSynchronize() == hipSuccess)
            c->cache->give(c->buf, c->buf_bytes);
        else
            (void)hipFree(c->buf);
    }
    delete c;
}
