// Bin-window form of the filter (Kim et al., BMC Genomics 2018, Section
// "Mapping GRIM-Filter to 3D-Stacked Memory with PIM": the mapper sends a read
// with a range of consecutive bins; bitvectors are laid out token-major so that
// one access returns the existence bits of one token for many bins; Section
// "GRIM-Filter Parallelization": a window of w consecutive bins is processed
// together).
//
// Token-major copy of the index: row t holds bit b = "token t occurs in bin b"
// for every bin (ceil(n_bins / 64) * 2 words per row).  For a (read, window)
// each thread owns 32 consecutive bins (one word of every row) and adds, for
// every token position of the read, that token's row word into bit-sliced
// counters (ripple-carry over planes), so repeated tokens count once per
// position.  Each token costs one coalesced row segment for the whole window.
#include <hip/hip_runtime.h>

#include <cstring>

#include "grim_internal.h"

namespace grim {
namespace {

template <int Q>
__device__ __forceinline__ uint32_t win_token_at(const uint32_t *__restrict__ w, uint64_t nw,
                                                 uint64_t pos)
{
    const uint64_t wi = pos >> 4;
    const uint32_t sh = (uint32_t)(pos & 15u) << 1;
    uint64_t x = (uint64_t)(wi < nw ? w[wi] : 0u) << 32;
    if (sh + 2 * Q > 32)
        x |= (wi + 1 < nw ? w[wi + 1] : 0u);
    return (uint32_t)((x << sh) >> (64 - 2 * Q));
}

// Transpose: one wavefront per group of 64 consecutive bins.  Lane j holds word
// w of bin (64g + j)'s vector; the ballot of bit i over the lanes is the 64-bit
// row segment of token 32w + i for those 64 bins.
template <int Q>
__global__ __launch_bounds__(256) void transpose_kernel(const uint32_t *__restrict__ vec,
                                                        uint64_t n_bins, uint64_t row_words,
                                                        uint32_t *__restrict__ rows)
{
    constexpr int VW = (1 << (2 * Q)) >> 5;
    const int lane = threadIdx.x & 63;
    const uint64_t n_groups = (n_bins + 63) / 64;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t gidx = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
         gidx < n_groups; gidx += waves) {
        const uint64_t b = gidx * 64 + lane;
        for (int w = 0; w < VW; ++w) {
            const uint32_t x = b < n_bins ? vec[b * VW + w] : 0u;
#pragma unroll 8
            for (int i = 0; i < 32; ++i) {
                const uint64_t m = __ballot((x >> i) & 1u);
                if (lane == 0) {
                    uint32_t *dst = rows + (uint64_t)(32 * w + i) * row_words + gidx * 2;
                    dst[0] = (uint32_t)m;
                    dst[1] = (uint32_t)(m >> 32);
                }
            }
        }
    }
}

// One workgroup per read (reads taken from an atomic counter); the window of
// read r is bins [win_lo[r], win_lo[r] + size) with size = cand_off[r+1] -
// cand_off[r], and pair cand_off[r] + j is bin win_lo[r] + j.  Each round
// covers 128 row words (4096 bins); counts go through LDS so that the stores
// are coalesced, and each wavefront ORs the pass bits of 64 consecutive pairs
// into at most three mask words.
template <int NP>
__device__ __forceinline__ void bitsliced_add(uint32_t (&planes)[NP], int npl, uint32_t carry)
{
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        if (k >= npl || !carry)
            break;
        const uint32_t c2 = planes[k] & carry;
        planes[k] ^= carry;
        carry = c2;
    }
}

// NP: bit planes held per thread (8 covers reads of up to 2^8 + q - 2 bases).
// UN: row loads in flight per thread.
template <int Q, int NP, int UN>
__global__ __launch_bounds__(256) void window_kernel(WindowArgs a)
{
    extern __shared__ uint32_t toks[];     // the read's tokens (max_len entries)
    __shared__ int32_t stage[128 * 33];    // counts of the round, padded rows
    __shared__ uint32_t partial[NP * 128]; // planes of the odd-token half
    __shared__ uint32_t next_read;
    const int t = threadIdx.x, lane = t & 63, col = t & 127, half = t >> 7;
    for (;;) {
        if (t == 0)
            next_read = atomicAdd(a.counter, 1u);
        __syncthreads();
        const uint64_t r = next_read;
        __syncthreads();
        if (r >= a.n_reads)
            break;
        const uint64_t p0 = a.cand_off[r], p1 = a.cand_off[r + 1];
        if (p1 <= p0)
            continue;
        if (p1 > a.n_pairs) {
            if (t == 0)
                atomicOr(a.status, GRIM_FLAG_CAND_OFF);
            continue;
        }
        const uint32_t L = a.read_len[r];
        const uint64_t off = a.read_off[r];
        const uint64_t nb = a.nw * 16;
        const uint64_t lo = a.win_lo[r], size = p1 - p0;
        if (L > a.max_len || off > nb || L > nb - off) {
            for (uint64_t k = p0 + t; k < p1; k += blockDim.x)
                a.counts[k] = -1;
            if (t == 0)
                atomicOr(a.status, GRIM_FLAG_READ);
            continue;
        }
        const uint32_t ntok = L >= (uint32_t)Q ? L - Q + 1 : 0u;
        for (uint32_t i = t; i < ntok; i += blockDim.x)
            toks[i] = win_token_at<Q>(a.rw, a.nw, off + i);
        __syncthreads();
        const uint64_t E = ((uint64_t)a.read_e[r] * L + a.e_den - 1) / a.e_den;
        const int64_t T = (int64_t)ntok - (int64_t)Q * (int64_t)E;
        const uint64_t w_first = lo >> 5, w_last = (lo + size - 1) >> 5;
        // each round: 128 row words (4096 bins); the two halves of the block
        // take the even and the odd token positions, 8 row loads in flight
        for (uint64_t wb = w_first; wb <= w_last; wb += 128) {
            const uint64_t wi = wb + col;
            uint32_t planes[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k)
                planes[k] = 0u;
            if (wi <= w_last && wi < a.row_words) {
                const uint32_t *cp = a.rows + wi;
                const uint64_t rw = a.row_words;
                uint32_t i = half;
                for (; i + 2 * (UN - 1) < ntok; i += 2 * UN) {
                    uint32_t x[UN];
#pragma unroll
                    for (int u = 0; u < UN; ++u)
                        x[u] = cp[(uint64_t)toks[i + 2 * u] * rw];
#pragma unroll
                    for (int u = 0; u < UN; ++u)
                        bitsliced_add(planes, a.npl, x[u]);
                }
                for (; i < ntok; i += 2)
                    bitsliced_add(planes, a.npl, cp[(uint64_t)toks[i] * rw]);
            }
            if (half == 1) {
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (k < a.npl)
                        partial[k * 128 + col] = planes[k];
            }
            __syncthreads();
            if (half == 0) {
                // ripple-carry addition of the two bit-sliced partial sums
                uint32_t carry = 0;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    if (k < a.npl) {
                        const uint32_t x = planes[k], y = partial[k * 128 + col];
                        planes[k] = x ^ y ^ carry;
                        carry = (x & y) | (carry & (x ^ y));
                    }
                }
                for (int j = 0; j < 32; ++j) {
                    uint32_t cnt = 0;
#pragma unroll
                    for (int k = 0; k < NP; ++k)
                        if (k < a.npl)
                            cnt |= ((planes[k] >> j) & 1u) << k;
                    stage[col * 33 + j] = (int32_t)cnt;
                }
            }
            __syncthreads();
            const uint64_t bin0 = wb * 32;
            for (uint32_t e0 = 0; e0 < 128 * 32; e0 += 256) {
                const uint32_t e = e0 + t;
                const uint64_t bin = bin0 + e;
                const bool inwin = bin >= lo && bin < lo + size;
                bool pass = false;
                if (inwin) {
                    const uint64_t k = p0 + (bin - lo);
                    if (bin >= a.n_bins) {
                        a.counts[k] = -1;
                        atomicOr(a.status, GRIM_FLAG_BIN_RANGE);
                    } else {
                        const int32_t c = stage[(e >> 5) * 33 + (e & 31)];
                        a.counts[k] = c;
                        pass = (int64_t)c >= T;
                    }
                }
                uint64_t m = __ballot(pass);
                if (lane == 0 && m) {
                    const uint64_t bin_w = bin0 + e0 + (uint32_t)(t & ~63);
                    uint64_t kb;
                    if (bin_w < lo) {
                        m >>= (lo - bin_w);
                        kb = p0;
                    } else {
                        kb = p0 + (bin_w - lo);
                    }
                    const uint64_t w0 = kb >> 5;
                    const uint32_t sh = (uint32_t)(kb & 31);
                    const uint32_t part0 = (uint32_t)(m << sh);
                    const uint32_t part1 = (uint32_t)(m >> (32 - sh));
                    const uint32_t part2 = sh ? (uint32_t)(m >> (64 - sh)) : 0u;
                    if (part0)
                        atomicOr(&a.pass_bits[w0], part0);
                    if (part1)
                        atomicOr(&a.pass_bits[w0 + 1], part1);
                    if (part2)
                        atomicOr(&a.pass_bits[w0 + 2], part2);
                }
            }
            __syncthreads();  // stage and partial are rewritten next round
        }
        __syncthreads();  // toks reused by the next read
    }
}

}  // namespace

hipError_t launch_transpose(hipStream_t s, int q, const uint32_t *vec, uint64_t n_bins,
                            uint64_t row_words, uint32_t *rows, uint32_t grid)
{
    switch (q) {
    case 4: hipLaunchKernelGGL(transpose_kernel<4>, dim3(grid), dim3(256), 0, s, vec, n_bins, row_words, rows); break;
    case 5: hipLaunchKernelGGL(transpose_kernel<5>, dim3(grid), dim3(256), 0, s, vec, n_bins, row_words, rows); break;
    case 6: hipLaunchKernelGGL(transpose_kernel<6>, dim3(grid), dim3(256), 0, s, vec, n_bins, row_words, rows); break;
    case 7: hipLaunchKernelGGL(transpose_kernel<7>, dim3(grid), dim3(256), 0, s, vec, n_bins, row_words, rows); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_window(hipStream_t s, int q, uint32_t grid, size_t lds, const WindowArgs &a)
{
    WindowArgs copy = a;
    void *args[] = {&copy};
    const void *k = nullptr;
    const bool small = a.npl <= 8;
#define GRIM_WK(Q)                                                                          \
    k = small ? reinterpret_cast<const void *>(&window_kernel<Q, 8, 16>)                    \
              : reinterpret_cast<const void *>(&window_kernel<Q, 16, 8>)
    switch (q) {
    case 4: GRIM_WK(4); break;
    case 5: GRIM_WK(5); break;
    case 6: GRIM_WK(6); break;
    case 7: GRIM_WK(7); break;
    default: return hipErrorInvalidValue;
    }
#undef GRIM_WK
    return hipLaunchKernel(k, dim3(grid), dim3(256), args, lds, s);
}

}  // namespace grim
