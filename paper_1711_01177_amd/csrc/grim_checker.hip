// Seed Location Checker kernels for gfx950: compaction of the seed location
// filter bitmask into the list of surviving locations.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grim_internal.h"

namespace grim {

// ------------------------------------------------- seed location checker
// Survivor compaction (Section "Integration with a Full Read Mapper": the Seed
// Location Checker reads the filter bitmask and fetches only the passing
// locations).  Three launches: per-block popcounts, one-block exclusive scan
// of the block totals, then each thread re-counts its words, takes its offset
// from a block scan and writes its passing pairs in input order.
constexpr int kCompactWpt = 4;                       // bitmask words per thread
constexpr int kCompactWpb = 256 * kCompactWpt;       // words per block

__device__ __forceinline__ uint32_t mask_word(const uint32_t *bits, uint64_t w, uint64_t n_pairs)
{
    uint32_t x = bits[w];
    const uint64_t end = (w + 1) * 32;
    if (end > n_pairs)
        x &= (n_pairs & 31) ? ((1u << (n_pairs & 31)) - 1u) : 0u;
    return x;
}

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds, uint32_t *total)
{
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const uint32_t y = __shfl_up(incl, s);
        if (lane >= s)
            incl += y;
    }
    if (lane == 63)
        lds[wv] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        if (i < wv)
            before += lds[i];
        all += lds[i];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

__global__ __launch_bounds__(256) void compact_count_kernel(const uint32_t *__restrict__ bits,
                                                            uint64_t n_words, uint64_t n_pairs,
                                                            uint64_t *__restrict__ block_sums)
{
    __shared__ uint32_t lds[4];
    const uint64_t w0 = (uint64_t)blockIdx.x * kCompactWpb + (uint64_t)threadIdx.x * kCompactWpt;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < kCompactWpt; ++j)
        if (w0 + j < n_words)
            c += __popc(mask_word(bits, w0 + j, n_pairs));
    uint32_t total;
    block_exclusive_scan(c, lds, &total);
    if (threadIdx.x == 0)
        block_sums[blockIdx.x] = total;
}

// One workgroup: in-place exclusive scan of n block totals; *n_out = sum.
__global__ __launch_bounds__(1024) void compact_scan_kernel(uint64_t *sums, uint64_t n, uint64_t *n_out)
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
        *n_out = carry_s;
}

__global__ __launch_bounds__(256) void compact_emit_kernel(
    const uint32_t *__restrict__ bits, uint64_t n_words, uint64_t n_pairs,
    const uint64_t *__restrict__ block_off, const uint64_t *__restrict__ cand_off, uint64_t n_reads,
    const uint32_t *__restrict__ cand_bin, uint64_t cap, uint64_t *__restrict__ surv_pair,
    uint32_t *__restrict__ surv_read, uint32_t *__restrict__ surv_bin)
{
    __shared__ uint32_t lds[4];
    const uint64_t w0 = (uint64_t)blockIdx.x * kCompactWpb + (uint64_t)threadIdx.x * kCompactWpt;
    uint32_t x[kCompactWpt];
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < kCompactWpt; ++j) {
        x[j] = (w0 + j < n_words) ? mask_word(bits, w0 + j, n_pairs) : 0u;
        c += __popc(x[j]);
    }
    uint32_t total;
    uint64_t pos = block_off[blockIdx.x] + block_exclusive_scan(c, lds, &total);
    if (c == 0 || n_reads == 0)
        return;
    // read of the first survivor: the last r with cand_off[r] <= pair
    uint64_t first = 0;
#pragma unroll
    for (int j = kCompactWpt - 1; j >= 0; --j)
        if (x[j])
            first = (w0 + j) * 32 + (__ffs(x[j]) - 1);
    uint64_t lo = 0, hi = n_reads - 1;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (cand_off[mid] <= first)
            lo = mid;
        else
            hi = mid - 1;
    }
    uint64_t r = lo;
#pragma unroll
    for (int j = 0; j < kCompactWpt; ++j) {
        uint32_t m = x[j];
        while (m) {
            const uint32_t b = __ffs(m) - 1;
            m &= m - 1;
            const uint64_t k = (w0 + j) * 32 + b;
            while (r + 1 < n_reads && cand_off[r + 1] <= k)
                ++r;
            if (pos < cap) {
                surv_pair[pos] = k;
                surv_read[pos] = (uint32_t)r;
                surv_bin[pos] = cand_bin[k];
            }
            ++pos;
        }
    }
}

hipError_t launch_compact(hipStream_t s, const uint32_t *bits, uint64_t n_pairs,
                          const uint64_t *cand_off, uint64_t n_reads, const uint32_t *cand_bin,
                          uint64_t cap, uint64_t *surv_pair, uint32_t *surv_read,
                          uint32_t *surv_bin, uint64_t *n_out, uint64_t *block_sums)
{
    const uint64_t n_words = (n_pairs + 31) / 32;
    const uint64_t nb = (n_words + kCompactWpb - 1) / kCompactWpb;
    if (nb == 0) {
        hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(1024), 0, s, block_sums, 0, n_out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(compact_count_kernel, dim3((uint32_t)nb), dim3(256), 0, s, bits, n_words,
                       n_pairs, block_sums);
    hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(1024), 0, s, block_sums, nb, n_out);
    hipLaunchKernelGGL(compact_emit_kernel, dim3((uint32_t)nb), dim3(256), 0, s, bits, n_words,
                       n_pairs, block_sums, cand_off, n_reads, cand_bin, cap, surv_pair, surv_read,
                       surv_bin);
    return hipGetLastError();
}

uint64_t compact_blocks(uint64_t n_pairs)
{
    const uint64_t n_words = (n_pairs + 31) / 32;
    return (n_words + kCompactWpb - 1) / kCompactWpb;
}

}  // namespace grim
