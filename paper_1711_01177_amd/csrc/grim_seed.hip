// Seeding on the GPU: the k-mer position index of the reference and the
// candidate locations of a read batch (the mapper's hash-table lookup that
// precedes the filter: Kim et al., BMC Genomics 2018, Section "Introduction",
// Fig. 1, and Section "Integration with a Full Read Mapper").
//
// Index: counts of every k-mer (atomic histogram), exclusive scan into
// offsets, scatter of positions.  Candidates: per read, the number of hits of
// its seeds (k-mers at offsets 0, k, 2k, ...), a scan, the hit bins
// (clamp(p - o) / B), a segmented radix sort per read (hipCUB), and a per-read
// dedup + cap pass that writes the CSR candidate list.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <new>

#include "grim_internal.h"

struct grim_seed_index {
    uint32_t k;
    int device;
    uint64_t G;
    uint64_t *d_off;   // 4^k + 1 offsets into d_pos
    uint32_t *d_pos;   // G - k + 1 positions grouped by k-mer
};

struct grim_candidates {
    uint64_t n_reads, n_pairs;
    uint64_t *d_off;   // n_reads + 1
    uint32_t *d_bin;   // n_pairs (at least one element)
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

template <typename T>
__global__ __launch_bounds__(256) void scan_totals_kernel(const T *__restrict__ in, uint64_t n,
                                                          uint64_t *block_tot)
{
    __shared__ uint64_t lds[4];
    const uint64_t i0 = (uint64_t)blockIdx.x * kScanPerBlock + (uint64_t)threadIdx.x * kScanPerThread;
    uint64_t s = 0;
    for (int j = 0; j < kScanPerThread; ++j)
        if (i0 + j < n)
            s += in[i0 + j];
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

template <typename T>
__global__ __launch_bounds__(256) void scan_apply_kernel(const T *__restrict__ in, uint64_t n,
                                                         const uint64_t *__restrict__ block_base,
                                                         const uint64_t *__restrict__ total,
                                                         uint64_t *__restrict__ out)
{
    __shared__ uint64_t lds[4];
    const uint64_t i0 = (uint64_t)blockIdx.x * kScanPerBlock + (uint64_t)threadIdx.x * kScanPerThread;
    uint64_t s = 0;
    for (int j = 0; j < kScanPerThread; ++j)
        if (i0 + j < n)
            s += in[i0 + j];
    uint64_t tot;
    uint64_t run = block_base[blockIdx.x] + block_scan_u64(s, lds, &tot);
    for (int j = 0; j < kScanPerThread; ++j) {
        if (i0 + j < n) {
            out[i0 + j] = run;
            run += in[i0 + j];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        out[n] = *total;
}

// --------------------------------------------------------------- seeding
__global__ __launch_bounds__(256) void seed_count_kernel(
    const uint32_t *__restrict__ rw, uint64_t nw, const uint64_t *__restrict__ read_off,
    const uint32_t *__restrict__ read_len, uint64_t n_reads, uint32_t k,
    const uint64_t *__restrict__ idx_off, uint64_t *__restrict__ hits)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t nb = nw * 16;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_reads; r += stride) {
        const uint32_t L = read_len[r];
        const uint64_t off = read_off[r];
        uint64_t s = 0;
        if (off <= nb && L <= nb - off) {
            for (uint32_t o = 0; o + k <= L; o += k) {
                const uint32_t km = kmer_at(rw, nw, off + o, k);
                s += idx_off[km + 1] - idx_off[km];
            }
        }
        hits[r] = s;
    }
}

// One wavefront per read; its seeds are looked up 8 at a time, one group of 8
// lanes per seed, and each group copies its seed's hits (seed order, then index
// order, as the count pass assumed) to the read's hit range.
constexpr int kSeedGroup = 8;                 // lanes per seed
constexpr int kSeedsPerStep = kWave / kSeedGroup;

__global__ __launch_bounds__(256) void seed_emit_kernel(
    const uint32_t *__restrict__ rw, uint64_t nw, const uint64_t *__restrict__ read_off,
    const uint32_t *__restrict__ read_len, uint64_t n_reads, uint32_t k,
    const uint64_t *__restrict__ idx_off, const uint32_t *__restrict__ idx_pos, uint64_t G,
    uint64_t B, const uint64_t *__restrict__ hit_off, uint32_t *__restrict__ hit_bin)
{
    const int lane = threadIdx.x & 63, grp = lane / kSeedGroup, sub = lane % kSeedGroup;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t nb = nw * 16;
    for (uint64_t r = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < n_reads;
         r += waves) {
        const uint32_t L = read_len[r];
        const uint64_t off = read_off[r];
        if (off > nb || L > nb - off)
            continue;
        const uint32_t n_seeds = L >= k ? L / k : 0u;
        uint64_t dst = hit_off[r];
        for (uint32_t s0 = 0; s0 < n_seeds; s0 += kSeedsPerStep) {
            const uint32_t sd = s0 + (uint32_t)grp;
            const uint32_t o = sd * k;
            uint64_t a = 0, cnt = 0;
            if (sd < n_seeds) {
                const uint32_t km = kmer_at(rw, nw, off + o, k);
                a = idx_off[km];
                cnt = idx_off[km + 1] - a;
            }
            // exclusive prefix of the groups' hit counts (lane sub == 0 of each group)
            uint64_t incl = sub == 0 ? cnt : 0;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint64_t y = __shfl_up(incl, d);
                if (lane >= d)
                    incl += y;
            }
            const uint64_t total = __shfl(incl, kWave - 1);
            const uint64_t before = incl - (sub == 0 ? cnt : 0);
            // the group's first lane holds its exclusive offset
            const uint64_t gdst = dst + __shfl(before, grp * kSeedGroup);
            for (uint64_t h = sub; h < cnt; h += kSeedGroup) {
                int64_t z = (int64_t)idx_pos[a + h] - (int64_t)o;
                if (z < 0)
                    z = 0;
                if ((uint64_t)z > G - 1)
                    z = (int64_t)(G - 1);
                hit_bin[gdst + h] = (uint32_t)((uint64_t)z / B);
            }
            dst += total;
        }
    }
}

// one wavefront per read: number of distinct bins in the sorted segment, capped
template <bool EMIT>
__global__ __launch_bounds__(256) void unique_kernel(const uint32_t *__restrict__ sorted,
                                                     const uint64_t *__restrict__ seg_off,
                                                     uint64_t n_reads, uint32_t cap,
                                                     uint64_t *__restrict__ count,
                                                     const uint64_t *__restrict__ out_off,
                                                     uint32_t *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (uint64_t r = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < n_reads;
         r += waves) {
        const uint64_t a = seg_off[r], b = seg_off[r + 1];
        uint64_t u = 0;
        for (uint64_t base = a; base < b && u < cap; base += kWave) {
            const uint64_t i = base + lane;
            bool first = false;
            uint32_t v = 0;
            if (i < b) {
                v = sorted[i];
                first = (i == a) || (sorted[i - 1] != v);
            }
            const uint64_t m = __ballot(first);
            const uint64_t pos = u + __popcll(m & below);
            if (EMIT && first && pos < cap)
                out[out_off[r] + pos] = v;
            u += __popcll(m);
        }
        if (!EMIT && lane == 0)
            count[r] = u < cap ? u : cap;
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
    delete si;
}

extern "C" int grim_seed_candidates(const grim_seed_index_t *si, const grim_batch_t *reads,
                                    uint64_t bin_stride, uint32_t cap, grim_candidates_t **out,
                                    void *stream)
{
    if (!si || !reads || !out || bin_stride == 0 || cap == 0)
        return GRIM_E_INVALID;
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
    uint64_t *hits = nullptr, *hit_off = nullptr, *btmp = nullptr, *ucnt = nullptr;
    uint32_t *hb = nullptr, *hs = nullptr;
    void *sort_tmp = nullptr;
    uint8_t *tmp_reads = nullptr, *tmp_hits = nullptr;  // temporaries, two allocations
    size_t sort_bytes = 0;
    uint64_t total_hits = 0, n_pairs = 0;
    grim_candidates *c = new (std::nothrow) grim_candidates();
    if (!c)
        return GRIM_E_NOMEM;
    c->n_reads = n;
    c->d_off = nullptr;
    c->d_bin = nullptr;
    const uint64_t nbt = scan_blocks(n) + 1;
    {
        // per-read temporaries: hit counts, hit offsets, scan block sums, unique counts
        const uint64_t r8 = align_up((n + 1) * 8, 256), b8 = align_up(nbt * 8, 256);
        if (hipMalloc(&tmp_reads, 3 * r8 + b8) != hipSuccess ||
            hipMalloc(&c->d_off, (n + 1) * 8) != hipSuccess) {
            rc = GRIM_E_NOMEM;
            goto done;
        }
        hits = reinterpret_cast<uint64_t *>(tmp_reads);
        hit_off = reinterpret_cast<uint64_t *>(tmp_reads + r8);
        ucnt = reinterpret_cast<uint64_t *>(tmp_reads + 2 * r8);
        btmp = reinterpret_cast<uint64_t *>(tmp_reads + 3 * r8);
    }
    if (n) {
        hipLaunchKernelGGL(seed_count_kernel, dim3(grid_for(n, dev)), dim3(256), 0, s,
                           reads->reads_2bit, reads->n_read_words, reads->read_off, reads->read_len,
                           n, si->k, si->d_off, hits);
        SEED_TRY(hipGetLastError());
    }
    SEED_TRY(scan_u64(s, hits, false, n, hit_off, btmp, btmp + nbt - 1));
    SEED_TRY(hipMemcpyAsync(&total_hits, hit_off + n, 8, hipMemcpyDeviceToHost, s));
    SEED_TRY(hipStreamSynchronize(s));
    if (total_hits >= 0x7fffffffull) {
        rc = GRIM_E_UNSUPPORTED;
        goto done;
    }
    if (n) {
        // per-hit temporaries: hit bins, sorted hit bins, the sort's own storage
        SEED_TRY(hipcub::DeviceSegmentedRadixSort::SortKeys(
            nullptr, sort_bytes, static_cast<const uint32_t *>(nullptr),
            static_cast<uint32_t *>(nullptr), (int)total_hits, (int)n, hit_off, hit_off + 1, 0, 32,
            s));
    }
    {
        const uint64_t h4 = align_up((total_hits + 1) * 4, 256);
        if (hipMalloc(&tmp_hits, 2 * h4 + align_up(sort_bytes ? sort_bytes : 1, 256)) !=
            hipSuccess) {
            rc = GRIM_E_NOMEM;
            goto done;
        }
        hb = reinterpret_cast<uint32_t *>(tmp_hits);
        hs = reinterpret_cast<uint32_t *>(tmp_hits + h4);
        sort_tmp = tmp_hits + 2 * h4;
    }
    if (n) {
        hipLaunchKernelGGL(seed_emit_kernel, dim3(grid_for(n * 64, dev)), dim3(256), 0, s,
                           reads->reads_2bit, reads->n_read_words, reads->read_off,
                           reads->read_len, n, si->k, si->d_off, si->d_pos, si->G, bin_stride,
                           hit_off, hb);
        SEED_TRY(hipGetLastError());
        SEED_TRY(hipcub::DeviceSegmentedRadixSort::SortKeys(sort_tmp, sort_bytes, hb, hs,
                                                            (int)total_hits, (int)n, hit_off,
                                                            hit_off + 1, 0, 32, s));
        hipLaunchKernelGGL(unique_kernel<false>, dim3(grid_for(n * 64, dev)), dim3(256), 0, s, hs,
                           hit_off, n, cap, ucnt, nullptr, nullptr);
        SEED_TRY(hipGetLastError());
    }
    SEED_TRY(scan_u64(s, ucnt, false, n, c->d_off, btmp, btmp + nbt - 1));
    SEED_TRY(hipMemcpyAsync(&n_pairs, c->d_off + n, 8, hipMemcpyDeviceToHost, s));
    SEED_TRY(hipStreamSynchronize(s));
    if (hipMalloc(&c->d_bin, (n_pairs + 1) * 4) != hipSuccess) {
        rc = GRIM_E_NOMEM;
        goto done;
    }
    if (n) {
        hipLaunchKernelGGL(unique_kernel<true>, dim3(grid_for(n * 64, dev)), dim3(256), 0, s, hs,
                           hit_off, n, cap, nullptr, c->d_off, c->d_bin);
        SEED_TRY(hipGetLastError());
    }
    SEED_TRY(hipStreamSynchronize(s));
    c->n_pairs = n_pairs;
done:
    (void)hipFree(tmp_reads);
    (void)hipFree(tmp_hits);
    if (rc != GRIM_OK) {
        (void)hipFree(c->d_off);
        (void)hipFree(c->d_bin);
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
    (void)hipFree(c->d_off);
    (void)hipFree(c->d_bin);
    delete c;
}
