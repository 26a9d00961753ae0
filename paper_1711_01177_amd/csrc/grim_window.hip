// Bin-window form of the filter (Kim et al., BMC Genomics 2018, Section
// "Mapping GRIM-Filter to 3D-Stacked Memory with PIM": the mapper sends a read
// with a range of consecutive bins; bitvectors are laid out token-major so that
// one access returns the existence bits of one token for many bins; Section
// "GRIM-Filter Parallelization": a window of w consecutive bins is processed
// together).
//
// Token-major copy of the index: row t holds bit b = "token t occurs in bin b"
// for every bin (ceil(n_bins / 1024) * 32 words per row, zero past the last
// bin, plus one pad word at the end of the buffer).  For a (read, window) each thread owns 32 consecutive
// bins of the window (one row word when the window starts on a multiple of 32
// bins, else two adjacent row words joined by a funnel shift) and
// adds, for every token position of the read, that token's bits into a
// bit-sliced counter (carry-save adders), so repeated tokens count once per
// position.  Each token costs one coalesced row segment for the whole window.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

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

// Transpose of 32 x 32 bits held one row per lane in each half-wavefront: on
// entry lane r holds x with bit c = M[r][c], on exit lane r holds bit c =
// M[c][r].  Stage s exchanges x with lane r ^ s and swaps the two s x s
// off-diagonal blocks of each 2s x 2s block (bit log2(s) of the row index
// trades places with bit log2(s) of the column index; the five stages commute).
__device__ __forceinline__ uint32_t transpose32(uint32_t x, uint32_t lane)
{
#define GRIM_T32_STAGE(S, M)                                                                      \
    {                                                                                            \
        const uint32_t xp = (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x1F | ((S) << 10));   \
        const bool upper = (lane & (S)) != 0;                                                    \
        const uint32_t lo = upper ? xp : x, hi = upper ? x : xp;                                 \
        const uint32_t t = ((lo >> (S)) ^ hi) & (M);                                             \
        x ^= upper ? t : (t << (S));                                                             \
    }
    GRIM_T32_STAGE(16, 0x0000FFFFu)
    GRIM_T32_STAGE(8, 0x00FF00FFu)
    GRIM_T32_STAGE(4, 0x0F0F0F0Fu)
    GRIM_T32_STAGE(2, 0x33333333u)
    GRIM_T32_STAGE(1, 0x55555555u)
#undef GRIM_T32_STAGE
    return x;
}

// Transpose: a workgroup of 16 wavefronts takes 1024 consecutive bins (16
// groups of 64, one per wavefront, lane = bin).  Each lane loads 128 bytes of
// its bin's vector at a time (32 words: tokens 1024c .. 1024c + 1023) and
// bit-transposes each word with its half-wavefront, so lane i of half h holds
// token (32w + i)'s bits for bins 32h .. 32h + 31 of its group.  Four words
// (128 rows) at a time are staged in LDS and written out as whole 128-byte row
// segments of the tile (row_words is a multiple of 32: every tile owns one
// aligned 32-word segment of every row; bins past the last one are zero).
constexpr int kTrThreads = 1024;
constexpr int kTrRowPad = 33;  // LDS row stride (words): lanes of one word hit different banks

template <int Q>
__global__ __launch_bounds__(kTrThreads) void transpose_kernel(const uint32_t *__restrict__ vec,
                                                               uint64_t n_bins, uint64_t row_words,
                                                               uint32_t *__restrict__ rows)
{
    constexpr int VW = (1 << (2 * Q)) >> 5;
    constexpr int CW = VW < 32 ? VW : 32;  // words per load pass
    __shared__ uint32_t stage[128 * kTrRowPad];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t half = lane >> 5, li = lane & 31;
    const uint64_t n_tiles = row_words / 32;
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint64_t b = (tile * 16 + wv) * 64 + lane;
        const uint4 *src = reinterpret_cast<const uint4 *>(vec + b * VW);
        for (int c = 0; c < VW / CW; ++c) {
            uint32_t x[CW];
#pragma unroll
            for (int k = 0; k < CW / 4; ++k) {
                const uint4 v = b < n_bins ? src[c * (CW / 4) + k] : make_uint4(0u, 0u, 0u, 0u);
                x[4 * k] = v.x;
                x[4 * k + 1] = v.y;
                x[4 * k + 2] = v.z;
                x[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int st = 0; st < CW / 4; ++st) {
                uint32_t y[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    y[u] = transpose32(x[4 * st + u], li);
                __syncthreads();  // the previous step's rows have been written out
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    stage[(32 * u + li) * kTrRowPad + 2 * wv + half] = y[u];
                __syncthreads();
                const uint64_t r0 = (uint64_t)(c * CW + 4 * st) * 32;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t idx = tid + j * kTrThreads;  // 128 rows x 32 words
                    const uint32_t rl = idx >> 5, ww = idx & 31;
                    rows[(r0 + rl) * row_words + tile * 32 + ww] = stage[rl * kTrRowPad + ww];
                }
            }
        }
        __syncthreads();  // stage reused by the next tile
    }
}

// Carry-save adder: a + b + c = 2*h + l, bitwise over 32 bin lanes.
__device__ __forceinline__ void csa(uint32_t &h, uint32_t &l, uint32_t a, uint32_t b, uint32_t c)
{
    const uint32_t u = a ^ b;
    h = (u & c) | (~u & a);
    l = u ^ c;
}

// Bit-sliced counter of NP planes: for every bin lane i, the count is
// ones_i + 2 twos_i + 4 fours_i + 8 eights_i + 16 * (hi planes)_i.  Sixteen
// words at a time go through a carry-save tree (Harley-Seal), so a word costs
// about three bitwise operations instead of a ripple over all planes.
template <int NP>
struct SlicedCount {
    uint32_t p[NP];  // p[0] ones, p[1] twos, p[2] fours, p[3] eights, p[4..] weight 16+

    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int k = 0; k < NP; ++k)
            p[k] = 0u;
    }
    // add one word at weight 2^k0 (ripple, branch-free)
    __device__ __forceinline__ void add(uint32_t carry, int k0 = 0)
    {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (k >= k0) {
                const uint32_t c2 = p[k] & carry;
                p[k] ^= carry;
                carry = c2;
            }
        }
    }
    __device__ __forceinline__ void add16(const uint32_t (&w)[16])
    {
        uint32_t ta, tb, fa, fb, ea, eb, s16;
        csa(ta, p[0], p[0], w[0], w[1]);
        csa(tb, p[0], p[0], w[2], w[3]);
        csa(fa, p[1], p[1], ta, tb);
        csa(ta, p[0], p[0], w[4], w[5]);
        csa(tb, p[0], p[0], w[6], w[7]);
        csa(fb, p[1], p[1], ta, tb);
        csa(ea, p[2], p[2], fa, fb);
        csa(ta, p[0], p[0], w[8], w[9]);
        csa(tb, p[0], p[0], w[10], w[11]);
        csa(fa, p[1], p[1], ta, tb);
        csa(ta, p[0], p[0], w[12], w[13]);
        csa(tb, p[0], p[0], w[14], w[15]);
        csa(fb, p[1], p[1], ta, tb);
        csa(eb, p[2], p[2], fa, fb);
        csa(s16, p[3], p[3], ea, eb);
        add(s16, 4);
    }
};

// Bins lo + 32j + i (i = 0..31) of token row `row` for virtual column j: the
// row words holding them, joined by a funnel shift.  The row buffer carries one
// pad word past its last row, so the second word is always readable; bits taken
// from beyond a row's end belong to bins >= n_bins, which the caller masks.
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

__device__ __forceinline__ uint32_t row_bins(const char *__restrict__ row, uint32_t byte_off,
                                            uint32_t sh)
{
    const u32x2_a4 v = *reinterpret_cast<const u32x2_a4 *>(row + byte_off);
    return __builtin_amdgcn_alignbit(v.y, v.x, sh);
}

// The same through a buffer resource over the whole row buffer, when its size
// fits 32-bit byte offsets: the row's offset comes from LDS and costs one add.
__device__ __forceinline__ uint32_t row_bins(__amdgpu_buffer_rsrc_t rs, uint32_t byte_off,
                                            uint32_t sh)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, byte_off, 0, 0);
    return __builtin_amdgcn_alignbit(v[1], v[0], sh);
}

// Bins lo + 32j + i of a token row when lo is a multiple of 32: one row word.
__device__ __forceinline__ uint32_t row_word(const char *__restrict__ row, uint32_t byte_off)
{
    return *reinterpret_cast<const uint32_t *>(row + byte_off);
}

__device__ __forceinline__ uint32_t row_word(__amdgpu_buffer_rsrc_t rs, uint32_t byte_off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(rs, byte_off, 0, 0);
}

// Adds the row bits of tokens [i0, i1) for one column into its counter.
// ALIGNED: the window starts on a row word (sh = 0), so a column is one word
// of each row and a wavefront's loads cover whole 256-byte runs.
template <int NP, bool OFF32, bool ALIGNED>
__device__ __forceinline__ void add_rows(SlicedCount<NP> &c, const uint32_t *toks, uint32_t i0,
                                         uint32_t i1, __amdgpu_buffer_rsrc_t rs,
                                         const char *__restrict__ rows, uint64_t row_bytes,
                                         uint32_t bo, uint32_t sh)
{
    auto load = [&](uint32_t tk) -> uint32_t {
        if (OFF32)
            return ALIGNED ? row_word(rs, tk + bo) : row_bins(rs, tk + bo, sh);
        const char *row = rows + (uint64_t)tk * row_bytes;
        return ALIGNED ? row_word(row, bo) : row_bins(row, bo, sh);
    };
    uint32_t i = i0;
    for (; i + 16 <= i1; i += 16) {
        uint32_t w[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            w[u] = load(toks[i + u]);
        c.add16(w);
    }
    for (; i < i1; ++i)
        c.add(load(toks[i]));
}

// One workgroup per read (reads taken from an atomic counter); the window of
// read r is bins [win_lo[r], win_lo[r] + size) with size = cand_off[r+1] -
// cand_off[r], and pair cand_off[r] + j is bin win_lo[r] + j.  Column j of a
// round (128 columns, 4096 bins) owns bins lo + 32(round*128 + j) + [0, 32);
// the two halves of the block take the first and the second half of the
// read's token positions, every position adding its token's row bits into the
// column's bit-sliced counter.  The halves are then added with a bit-sliced
// ripple adder, pass bits come from a bit-sliced comparison with T, and the
// counts are unpacked into LDS so that their stores are coalesced.
// NP: bit planes per counter (8 covers reads of up to 2^8 + q - 2 bases, else 16).
// OFF32: the row buffer is below 4 GiB; LDS then holds each token's row byte
// offset instead of the token.
template <int Q, int NP, bool OFF32>
__global__ __launch_bounds__(256) void window_kernel(WindowArgs a)
{
    typedef typename std::conditional<NP == 8, uint8_t, uint16_t>::type cnt_t;
    constexpr int CPW = 4 / sizeof(cnt_t);          // counts per LDS word
    constexpr int SW = 32 / CPW + 1;                // LDS words per column (padded)
    extern __shared__ uint32_t toks[];              // the read's tokens (max_len entries)
    __shared__ uint32_t stage[128 * SW];            // counts of the round
    __shared__ uint32_t partial[NP * 128];          // counter of the second half
    __shared__ uint32_t pmask[128];                 // pass bits per column
    __shared__ uint32_t next_read;
    const int t = threadIdx.x, col = t & 127, half = t >> 7;
    // GRIM_FLAG_* of skipped reads, the same in every thread, reported once
    // after the loop: a skip path must not end in a branch on the thread index
    // (if (t == 0) ... continue), which the compiler may thread across the
    // loop's back edge so that the other threads re-enter the loop at its
    // barrier without thread 0 having fetched the next read
    uint32_t skipped = 0;
    for (;;) {
        if (t == 0)
            next_read = atomicAdd(a.counter, 1u);
        __syncthreads();
        const uint64_t slot = next_read;
        __syncthreads();
        if (slot >= a.n_reads)
            break;
        const uint64_t r = a.order ? (uint64_t)a.order[slot] : slot;
        if (r >= a.n_reads) {  // an order entry naming no read: skipped
            skipped |= GRIM_FLAG_READ;
            continue;
        }
        const uint64_t p0 = a.cand_off[r], p1 = a.cand_off[r + 1];
        if (p1 <= p0)
            continue;
        if (p1 > a.n_pairs) {
            skipped |= GRIM_FLAG_CAND_OFF;
            continue;
        }
        const uint32_t L = a.read_len[r];
        const uint64_t off = a.read_off[r];
        const uint64_t nb = a.nw * 16;
        const uint64_t lo = a.win_lo[r], size = p1 - p0;
        if (L > a.max_len || off > nb || L > nb - off) {
            for (uint64_t k = p0 + t; k < p1; k += blockDim.x)
                a.counts[k] = -1;
            skipped |= GRIM_FLAG_READ;
            continue;
        }
        const uint32_t ntok = L >= (uint32_t)Q ? L - Q + 1 : 0u;
        const uint64_t row_bytes = a.row_words * 4;
        for (uint32_t i = t; i < ntok; i += blockDim.x) {
            const uint32_t tk = win_token_at<Q>(a.rw, a.nw, off + i);
            toks[i] = OFF32 ? tk * (uint32_t)row_bytes : tk;
        }
        __syncthreads();
        const uint64_t E = ((uint64_t)a.read_e[r] * L + a.e_den - 1) / a.e_den;
        const int64_t T = (int64_t)ntok - (int64_t)Q * (int64_t)E;
        // first half: tokens [0, hsplit), second: [hsplit, ntok); hsplit is a
        // multiple of 16 so that both halves start on 16-token blocks
        const uint32_t hsplit = ((ntok / 2 + 15) / 16) * 16 < ntok ? ((ntok / 2 + 15) / 16) * 16 : ntok;
        const uint32_t i0 = half ? hsplit : 0u, i1 = half ? ntok : hsplit;
        const uint64_t wv0 = lo >> 5;
        const uint32_t sh = (uint32_t)(lo & 31);
        const uint64_t n_cols = (size + 31) >> 5;
        const char *rows = reinterpret_cast<const char *>(a.rows);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint32_t *>(a.rows), (short)0, (int)(uint32_t)a.rows_bytes, 0x00020000);
        for (uint64_t vb = 0; vb < n_cols; vb += 128) {
            const uint64_t j = vb + col;
            const uint64_t wi = wv0 + j;
            SlicedCount<NP> c;
            c.clear();
            if (j < n_cols && wi < a.row_words) {
                const uint32_t bo = (uint32_t)(wi * 4);
                if (sh == 0)
                    add_rows<NP, OFF32, true>(c, toks, i0, i1, rs, rows, row_bytes, bo, sh);
                else
                    add_rows<NP, OFF32, false>(c, toks, i0, i1, rs, rows, row_bytes, bo, sh);
            }
            if (half == 1) {
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    partial[k * 128 + col] = c.p[k];
            }
            __syncthreads();
            if (half == 0) {
                // ripple-carry addition of the two halves' counters
                uint32_t carry = 0;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const uint32_t x = c.p[k], y = partial[k * 128 + col];
                    c.p[k] = x ^ y ^ carry;
                    carry = (x & y) | (carry & (x ^ y));
                }
                // bins of this column inside the window and below n_bins
                uint32_t valid = 0;
                if (j < n_cols) {
                    const uint64_t in_win = size - j * 32;
                    const uint64_t b0 = lo + j * 32;
                    const uint64_t in_idx = b0 < a.n_bins ? a.n_bins - b0 : 0;
                    const uint64_t v = in_win < in_idx ? in_win : in_idx;
                    valid = v >= 32 ? ~0u : ((1u << v) - 1u);
                }
                // count >= T, bit-sliced, from the top plane down
                uint32_t ge;
                if (T <= 0) {
                    ge = ~0u;
                } else if (T >= (int64_t)1 << NP) {
                    ge = 0u;
                } else {
                    uint32_t gt = 0u, eq = ~0u;
#pragma unroll
                    for (int k = NP - 1; k >= 0; --k) {
                        if ((T >> k) & 1) {
                            eq &= c.p[k];
                        } else {
                            gt |= eq & c.p[k];
                            eq &= ~c.p[k];
                        }
                    }
                    ge = gt | eq;
                }
                pmask[col] = ge & valid;
                // unpack: count of bin i = sum_k bit i of plane k << k
                if (NP == 8) {
#pragma unroll
                    for (int d = 0; d < 8; ++d) {
                        uint32_t acc = 0;
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const uint32_t nib = (c.p[k] >> (4 * d)) & 15u;
                            acc |= ((nib * 0x00204081u) & 0x01010101u) << k;
                        }
                        stage[col * SW + d] = acc;
                    }
                } else {
#pragma unroll
                    for (int d = 0; d < 16; ++d) {
                        uint32_t acc = 0;
#pragma unroll
                        for (int k = 0; k < NP; ++k) {
                            const uint32_t two = (c.p[k] >> (2 * d)) & 3u;
                            acc |= ((two * 0x00008001u) & 0x00010001u) << k;
                        }
                        stage[col * SW + d] = acc;
                    }
                }
            }
            __syncthreads();
            // counts: element e of the round is bin lo + 32 vb + e, pair p0 + 32 vb + e
            const uint64_t base = vb * 32;
            const cnt_t *sc = reinterpret_cast<const cnt_t *>(stage);
            bool oob = false;
            for (uint32_t e = t; e < 128 * 32; e += 256) {
                const uint64_t pe = base + e;
                if (pe < size) {
                    if (lo + pe >= a.n_bins) {
                        a.counts[p0 + pe] = -1;
                        oob = true;
                    } else {
                        a.counts[p0 + pe] = (int32_t)sc[(e >> 5) * (SW * CPW) + (e & 31)];
                    }
                }
            }
            if (oob)
                atomicOr(a.status, GRIM_FLAG_BIN_RANGE);
            // pass bits: column j's 32 bits start at pair p0 + 32 j; global word
            // g = (p0 >> 5) + vb + m takes the high part of column m - 1 and
            // the low part of column m.  Words shared with other reads (the
            // first and the last of the window) are ORed in, the rest stored.
            if (t <= 128) {
                const uint32_t ps = (uint32_t)(p0 & 31);
                const uint64_t g0 = (p0 >> 5) + vb;
                const uint64_t g_last = (p1 - 1) >> 5;
                const uint64_t g = g0 + t;
                if (g <= g_last) {
                    const uint32_t lo_part = t < 128 ? pmask[t] << ps : 0u;
                    const uint32_t hi_part = (t > 0 && ps) ? pmask[t - 1] >> (32 - ps) : 0u;
                    const uint32_t word = lo_part | hi_part;
                    const bool first = (g == (p0 >> 5)), last = (g == g_last);
                    // the word past the round's last column gets only a high part;
                    // the next round (if any) ORs its own low part in
                    const bool shared = first || last || t == 128 || (t == 0 && vb > 0);
                    if (shared) {
                        if (word)
                            atomicOr(&a.pass_bits[g], word);
                    } else {
                        a.pass_bits[g] = word;
                    }
                }
            }
            __syncthreads();  // stage, partial and pmask are rewritten next round
        }
        __syncthreads();  // toks reused by the next read
    }
    if (t == 0 && skipped)
        atomicOr(a.status, skipped);
}

}  // namespace

hipError_t launch_transpose(hipStream_t s, int q, const uint32_t *vec, uint64_t n_bins,
                            uint64_t row_words, uint32_t *rows, uint32_t grid)
{
    if (row_words % 32 != 0 || row_words * 32 < n_bins)
        return hipErrorInvalidValue;
    const dim3 blk(kTrThreads);
    switch (q) {
    case 4: hipLaunchKernelGGL(transpose_kernel<4>, dim3(grid), blk, 0, s, vec, n_bins, row_words, rows); break;
    case 5: hipLaunchKernelGGL(transpose_kernel<5>, dim3(grid), blk, 0, s, vec, n_bins, row_words, rows); break;
    case 6: hipLaunchKernelGGL(transpose_kernel<6>, dim3(grid), blk, 0, s, vec, n_bins, row_words, rows); break;
    case 7: hipLaunchKernelGGL(transpose_kernel<7>, dim3(grid), blk, 0, s, vec, n_bins, row_words, rows); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_window(hipStream_t s, int q, uint32_t cus, size_t lds, const WindowArgs &a)
{
    WindowArgs copy = a;
    void *args[] = {&copy};
    const void *k = nullptr;
    const bool small = a.npl <= 8;
    const bool off32 = a.rows_bytes < (1ull << 32);
#define GRIM_WK(Q)                                                                          \
    k = small ? (off32 ? reinterpret_cast<const void *>(&window_kernel<Q, 8, true>)         \
                       : reinterpret_cast<const void *>(&window_kernel<Q, 8, false>))       \
              : (off32 ? reinterpret_cast<const void *>(&window_kernel<Q, 16, true>)        \
                       : reinterpret_cast<const void *>(&window_kernel<Q, 16, false>))
    switch (q) {
    case 4: GRIM_WK(4); break;
    case 5: GRIM_WK(5); break;
    case 6: GRIM_WK(6); break;
    case 7: GRIM_WK(7); break;
    default: return hipErrorInvalidValue;
    }
#undef GRIM_WK
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, lds);
    if (e != hipSuccess)
        return e;
    uint64_t grid = (uint64_t)cus * (uint64_t)(per_cu > 0 ? per_cu : 1);
    if (grid > a.n_reads)
        grid = a.n_reads;
    return hipLaunchKernel(k, dim3((uint32_t)grid), dim3(256), args, lds, s);
}

// ------------------------------------------------------- processing order
// A counting sort of the reads by window-start bucket: count, exclusive scan,
// scatter.  Reads with overlapping windows then run close together in time and
// share row segments through L2; the filter's outputs do not depend on the
// order, so the order of reads within a bucket is left to the atomics.

__device__ __forceinline__ uint32_t order_bucket(uint32_t lo, uint64_t n_bins, uint32_t shift,
                                                 uint32_t n_buckets)
{
    return lo < n_bins ? lo >> shift : n_buckets - 1;
}

__global__ __launch_bounds__(256) void order_count_kernel(const uint32_t *__restrict__ win_lo,
                                                          uint32_t n, uint64_t n_bins,
                                                          uint32_t shift, uint32_t n_buckets,
                                                          uint32_t *cnt)
{
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u)
        atomicAdd(&cnt[order_bucket(win_lo[i], n_bins, shift, n_buckets)], 1u);
}

// Exclusive scan of cnt[0, n) in place by one workgroup of 1024 threads, in
// chunks of 1024 with a running carry.
__global__ __launch_bounds__(1024) void order_scan_kernel(uint32_t *cnt, uint32_t n)
{
    __shared__ uint32_t wsum[16];
    const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < n; base += 1024u) {
        const uint32_t i = base + t;
        const uint32_t v = i < n ? cnt[i] : 0u;
        uint32_t x = v;  // inclusive scan within the wavefront
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d)
                x += y;
        }
        if (lane == 63)
            wsum[wv] = x;
        __syncthreads();
        if (t < 16) {  // inclusive scan of the 16 wavefront sums
            uint32_t sw = wsum[t];
            for (uint32_t d = 1; d < 16; d <<= 1) {
                const uint32_t y = __shfl_up(sw, d, 64);
                if (t >= d)
                    sw += y;
            }
            wsum[t] = sw;
        }
        __syncthreads();
        if (i < n)
            cnt[i] = carry + (wv ? wsum[wv - 1] : 0u) + x - v;
        carry += wsum[15];
        __syncthreads();  // wsum is rewritten by the next chunk
    }
}

__global__ __launch_bounds__(256) void order_scatter_kernel(const uint32_t *__restrict__ win_lo,
                                                            uint32_t n, uint64_t n_bins,
                                                            uint32_t shift, uint32_t n_buckets,
                                                            uint32_t *cnt, uint32_t *order)
{
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        const uint32_t pos = atomicAdd(&cnt[order_bucket(win_lo[i], n_bins, shift, n_buckets)], 1u);
        order[pos] = i;
    }
}

// Buckets of 1024 bins (a quarter of a 4096-bin window), wider when needed to
// keep at most 2^16 of them, plus one for starts past the last bin.
uint32_t order_shift(uint64_t n_bins, uint32_t *n_buckets)
{
    uint32_t shift = 10;
    while (((n_bins ? n_bins - 1 : 0) >> shift) + 2 > 65536u)
        ++shift;
    *n_buckets = (uint32_t)(((n_bins ? n_bins - 1 : 0) >> shift) + 2);
    return shift;
}

hipError_t launch_window_order(hipStream_t s, uint32_t cus, const uint32_t *win_lo, uint32_t n,
                               uint64_t n_bins, uint32_t shift, uint32_t n_buckets, uint32_t *cnt,
                               uint32_t *order)
{
    const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255u) / 256u, (uint64_t)cus * 8u);
    hipLaunchKernelGGL(order_count_kernel, dim3(grid), dim3(256), 0, s, win_lo, n, n_bins, shift,
                       n_buckets, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(1024), 0, s, cnt, n_buckets);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(order_scatter_kernel, dim3(grid), dim3(256), 0, s, win_lo, n, n_bins, shift,
                       n_buckets, cnt, order);
    return hipGetLastError();
}

}  // namespace grim
