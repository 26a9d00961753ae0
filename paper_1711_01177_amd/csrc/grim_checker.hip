// Seed Location Checker kernels for gfx950: compaction of the seed location
// filter bitmask into the list of surviving locations, and the alignment check
// of the survivors (edit distance of the read within its bin's span).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

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

// Read holding pair k: the last r in [lo, hi] with off[r] <= k (off[lo] <= k).
template <typename Off>
__device__ __forceinline__ uint64_t read_of(const Off *off, uint64_t lo, uint64_t hi, uint64_t k)
{
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if ((uint64_t)off[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Offsets staged in LDS per workgroup: a workgroup covers 32768 pairs, and the
// reads they belong to (one search each for the first and the last pair) are
// looked up in LDS when there are at most kStageReads of them.
constexpr int kStageReads = 2048;

__global__ __launch_bounds__(256) void compact_emit_kernel(
    const uint32_t *__restrict__ bits, uint64_t n_words, uint64_t n_pairs,
    const uint64_t *__restrict__ block_off, const uint64_t *__restrict__ cand_off, uint64_t n_reads,
    const uint32_t *__restrict__ cand_bin, uint64_t cap, uint64_t *__restrict__ surv_pair,
    uint32_t *__restrict__ surv_read, uint32_t *__restrict__ surv_bin)
{
    __shared__ uint32_t lds[4];
    __shared__ uint64_t stage[kStageReads + 1];
    __shared__ uint64_t range[2];
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
    if (total == 0 || n_reads == 0)
        return;
    // reads of the workgroup's first and last pair
    const uint64_t p_first = (uint64_t)blockIdx.x * kCompactWpb * 32;
    const uint64_t p_end = p_first + (uint64_t)kCompactWpb * 32 < n_pairs
                               ? p_first + (uint64_t)kCompactWpb * 32 : n_pairs;
    if (threadIdx.x < 2)
        range[threadIdx.x] =
            read_of(cand_off, 0, n_reads - 1, threadIdx.x == 0 ? p_first : p_end - 1);
    __syncthreads();
    const uint64_t r_lo = range[0], r_hi = range[1];
    const bool staged = r_hi - r_lo + 1 <= (uint64_t)kStageReads;
    if (staged) {
        // offsets of reads r_lo .. r_hi + 1 (the last one bounds the walk)
        const uint64_t n_st = r_hi - r_lo + 2;
        for (uint64_t i = threadIdx.x; i < n_st; i += blockDim.x)
            stage[i] = r_lo + i <= n_reads ? cand_off[r_lo + i] : ~0ull;
    }
    __syncthreads();
    if (c == 0)
        return;
    uint64_t first = 0;
#pragma unroll
    for (int j = kCompactWpt - 1; j >= 0; --j)
        if (x[j])
            first = (w0 + j) * 32 + (__ffs(x[j]) - 1);
    // r: the read holding the current pair; nxt: where the next read starts
    uint64_t r, nxt;
    if (staged) {
        r = r_lo + read_of(stage, 0, r_hi - r_lo, first);
        nxt = stage[r - r_lo + 1];
    } else {
        r = read_of(cand_off, r_lo, r_hi, first);
        nxt = r + 1 <= n_reads ? cand_off[r + 1] : ~0ull;
    }
#pragma unroll
    for (int j = 0; j < kCompactWpt; ++j) {
        uint32_t m = x[j];
        while (m) {
            const uint32_t b = __ffs(m) - 1;
            m &= m - 1;
            const uint64_t k = (w0 + j) * 32 + b;
            while (nxt <= k && r + 1 < n_reads) {
                ++r;
                nxt = staged ? stage[r - r_lo + 1] : cand_off[r + 1];
            }
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


// ---------------------------------------------------- alignment check
// Smallest edit distance between a surviving read and any substring of its
// bin's span (free start and end in the reference), i.e. whether the
// location really holds the read within E edits.  Computed with Myers'
// bit-parallel approximate-matching recurrence (G. Myers, J. ACM 46(3), 1999)
// on one long bit vector per column: row i of the dynamic-programming
// column is bit i of a vector of 32-bit words, and the addition and the
// one-row shifts carry from word to word.  One thread per survivor; the
// vertical deltas live in registers, the read's match masks in LDS.
//
// The read fills the vector from the bottom: the rows above it match every
// base and start with vertical delta 0, so they repeat the free boundary row
// (distance 0 at every column, nothing carried out of them), and the read's
// last row is always bit 31 of the last word.  A wavefront therefore runs the
// words from the first one any of its lanes needs to the last, with no
// per-lane branching inside a column.

// 16 read bases starting at base position pos (any alignment; may start
// before the array, whose words count as 0 there and past its end), first
// base in the top bits.
__device__ __forceinline__ uint32_t read_window(const uint32_t *__restrict__ w, uint64_t nw,
                                                int64_t pos)
{
    const int64_t wi = pos >> 4;   // floor, also for negative positions
    const uint32_t sh = (uint32_t)(pos & 15) << 1;
    const uint32_t w0 = wi >= 0 && (uint64_t)wi < nw ? w[wi] : 0u;
    const uint32_t w1 = wi + 1 >= 0 && (uint64_t)(wi + 1) < nw ? w[wi + 1] : 0u;
    return (uint32_t)((((uint64_t)w0 << 32) | w1) >> (32 - sh));
}

// Bits 0, 2, ..., 30 of x gathered into bits 0..15.
__device__ __forceinline__ uint32_t even_bits(uint32_t x)
{
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    return (x | (x >> 8)) & 0x0000FFFFu;
}

// Three-input bitwise function as gfx950's v_bitop3_b32 immediate: the truth
// table of f read off f(0xF0, 0xCC, 0xAA) (operands a, b, c in that order).
template <uint32_t IMM>
__device__ __forceinline__ uint32_t bitop3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, IMM);
}
constexpr uint32_t kXorOr = ((0xF0u ^ 0xCCu) | 0xAAu) & 0xFFu;   // (a ^ b) | c
constexpr uint32_t kOrNor = (0xF0u | ~(0xCCu | 0xAAu)) & 0xFFu;  // a | ~(b | c)

// The column scan over words S..NW-1 of every lane (S is the same for the
// whole wavefront).  peq_t points at this thread's match masks (64-bit pairs
// of words, base-major, 256 threads apart); rp/wsh locate the span
// in the packed reference.  Returns the smallest distance at the read's last
// row over the span's columns (L when the span is empty).  Per column and
// word, with Pv/Mv the vertical deltas and c the carry of the addition:
//   Xv = Eq | Mv;  Xh = (((Eq & Pv) + Pv + c) ^ Pv) | Eq
//   Ph = Mv | ~(Xh | Pv);  Mh = Pv & Xh
//   Ph, Mh shifted up one row (bit 31 of the word below comes in; 0 at S)
//   Pv = Mh | ~(Xv | Ph);  Mv = Ph & Xv
// and the distance at the last row moves by bit 31 of Ph minus that of Mh.
// UNI: every lane of the wavefront that runs the scan has the same span, so
// the column loop's trip count is uniform (kept in scalar registers).
template <int NW, int S, bool UNI>
__device__ __forceinline__ int32_t column_scan(const uint64_t *peq_t, uint32_t (&pv)[NW],
                                               uint32_t (&mv)[NW], const uint32_t *rp,
                                               uint32_t wsh, uint64_t span, int32_t L)
{
    int32_t score = L, best = L;
    if (UNI)
        span = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(span >> 32)) << 32) |
               __builtin_amdgcn_readfirstlane((uint32_t)span);
    if (span == 0)
        return best;
    // Loads run ahead of their use: the two reference words of the next
    // 16-column fetch one fetch ahead, and each pair of mask words of the
    // next column as soon as the current column is done with that pair.
    // The fetches reach at most three words past the reference's last one;
    // the reference is followed by zero words there (those bases are never
    // used), so the loads are unconditional and nothing waits on them before
    // their use.
    // nxt holds the next fetch's two words in memory order (first word in the
    // low half); they swap halves only where used, so that nothing waits on
    // the load before then
    uint32_t win = (uint32_t)(((uint64_t)rp[0] << 32 | rp[1]) >> (32 - wsh));
    uint64_t nxt;
    __builtin_memcpy(&nxt, rp + 1, 8);
    uint64_t e2[NW / 2];
    {
        const uint64_t *pq = peq_t + __builtin_amdgcn_ubfe(win, 30, 2) * (NW / 2 * 256);
#pragma unroll
        for (int q = S / 2; q < NW / 2; ++q)
            e2[q] = pq[q * 256];
    }
    for (uint64_t j = 0; j < span; ++j) {
        // the next column's base (the 16-base window moves on after column 15)
        const uint32_t col = (uint32_t)j & 15;
        if (col == 15) {
            win = (uint32_t)(((nxt << 32) | (nxt >> 32)) >> (32 - wsh));
            __builtin_memcpy(&nxt, rp + (j >> 4) + 2, 8);
        }
        const uint32_t cbn = __builtin_amdgcn_ubfe(win, 30 - 2 * ((col + 1) & 15), 2);
        const uint64_t *pqn = peq_t + cbn * (NW / 2 * 256);
        uint32_t c = 0, php = 0, mhp = 0;
#pragma unroll
        for (int k = S; k < NW; ++k) {
            const uint32_t eq = (k & 1) ? (uint32_t)(e2[k / 2] >> 32) : (uint32_t)e2[k / 2];
            const uint32_t xv = eq | mv[k];
            const uint32_t sm = __builtin_addc(eq & pv[k], pv[k], c, &c);
            const uint32_t xh = bitop3<kXorOr>(sm, pv[k], eq);
            const uint32_t ph = bitop3<kOrNor>(mv[k], xh, pv[k]);
            const uint32_t mh = pv[k] & xh;
            const uint32_t phs = k == S ? ph << 1 : __builtin_amdgcn_alignbit(ph, php, 31);
            const uint32_t mhs = k == S ? mh << 1 : __builtin_amdgcn_alignbit(mh, mhp, 31);
            php = ph;
            mhp = mh;
            pv[k] = bitop3<kOrNor>(mhs, xv, phs);
            mv[k] = phs & xv;
            if (k & 1) {   // pair k / 2 is done with: load the next column's
                e2[k / 2] = pqn[(k / 2) * 256];
                __builtin_amdgcn_sched_barrier(0);   // keep the load here
            }
        }
        // +1 when bit 31 of Ph is set, -1 when that of Mh is
        score += (int32_t)(php >> 31) + ((int32_t)mhp >> 31);
        best = min(best, score);
    }
    return best;
}

// Picks the scan for the wavefront's first word s (uniform across it).
template <int NW, int S, bool UNI>
__device__ __forceinline__ int32_t column_scan_from(int s, const uint64_t *peq_t,
                                                    uint32_t (&pv)[NW], uint32_t (&mv)[NW],
                                                    const uint32_t *rp, uint32_t wsh,
                                                    uint64_t span, int32_t L)
{
    if constexpr (S + 1 < NW) {
        if (s != S)
            return column_scan_from<NW, S + 1, UNI>(s, peq_t, pv, mv, rp, wsh, span, L);
    }
    return column_scan<NW, S, UNI>(peq_t, pv, mv, rp, wsh, span, L);
}

// Each workgroup owns one contiguous range of survivors: one chunk of 1024,
// or a run of whole chunks once the list exceeds 64 times the workgroups the
// GPU holds at once (ranges start on multiples of 32, so that no two
// workgroups share a word of pass bits).  It takes its range 1024 survivors
// at a time, sorts them by the number of 32-row words of their read
// (counting sort in LDS; survivors with nothing to align first, empty slots
// of a short last chunk last) and runs the sorted list in four rounds of
// 256, thread t taking sorted slot 256 r + t: a wavefront's 64 lanes then
// mostly hold reads of one length class, and every wavefront meets short and
// long reads over the four rounds, so none waits long for the others at the
// chunk's end.  Pass bits of the chunk are gathered in LDS and stored as
// whole words.  W is the number of 64-row blocks (NW = 2 W words) the
// batch's longest read needs.
constexpr int kVerifyChunk = 1024;

template <int W>
__global__ __launch_bounds__(256) void verify_kernel(VerifyArgs a)
{
    constexpr int NW = 2 * W;
    constexpr int CH = kVerifyChunk;
    __shared__ uint16_t order[CH];
    __shared__ uint32_t cls[NW + 2];
    __shared__ uint32_t okw[CH / 32];
    // match masks of every thread's read: peq[(base * W + block) * 256 + thread],
    // block = rows 64 block .. 64 block + 63 of the bottom-aligned vector
    // (lane-interleaved, so that a wavefront's reads of one column are
    // conflict-free whatever bases its lanes see)
    __shared__ uint64_t peq[4 * W * 256];
    const int t = threadIdx.x;
    const uint64_t per = ((a.n_surv + gridDim.x - 1) / gridDim.x + 31) & ~31ull;
    const uint64_t g0 = (uint64_t)blockIdx.x * per;
    const uint64_t g1 = g0 + per < a.n_surv ? g0 + per : a.n_surv;
    for (uint64_t base = g0; base < g1; base += CH) {
        const uint32_t cnt = (uint32_t)(g1 - base < (uint64_t)CH ? g1 - base : CH);
        if (t < NW + 2)
            cls[t] = 0;
        if (t < CH / 32)
            okw[t] = 0;
        __syncthreads();
        // class of slot u 256 + t: its read's word count, 0 when there is
        // nothing to align, NW + 1 past the chunk's end
        int key[CH / 256];
        uint32_t rank[CH / 256];
#pragma unroll
        for (int u = 0; u < CH / 256; ++u) {
            const uint32_t p = u * 256 + t;
            int k = NW + 1;
            if (p < cnt) {
                k = 0;
                const uint32_t r = a.surv_read[base + p];
                if (r < a.n_reads) {
                    const uint32_t L = a.read_len[r];
                    k = L <= 32u * NW ? (int)((L + 31) >> 5) : 0;
                }
            }
            key[u] = k;
            rank[u] = atomicAdd(&cls[k], 1u);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < CH / 256; ++u) {
            uint32_t start = 0;
            for (int c = 0; c < key[u]; ++c)
                start += cls[c];
            order[start + rank[u]] = (uint16_t)(u * 256 + t);
        }
        __syncthreads();
        for (int round = 0; round < CH / 256; ++round) {
            const uint32_t slot = order[round * 256 + t];
            const uint64_t i = base + slot;
            if (slot < cnt) {
                int32_t d = -1;
                bool ok = false;
                const uint32_t r = a.surv_read[i], b = a.surv_bin[i];
                const uint64_t nb = a.nw * 16;
                const uint32_t L = r < a.n_reads ? a.read_len[r] : 0u;
                const uint64_t off = r < a.n_reads ? a.read_off[r] : 0u;
                if (r < a.n_reads && b < a.n_bins && L <= 32u * NW && off <= nb &&
                    L <= nb - off) {
                    const uint32_t E =
                        (uint32_t)(((uint64_t)a.read_e[r] * L + a.e_den - 1) / a.e_den);
                    const int pad = 32 * NW - (int)L;   // rows above the read
                    uint32_t pv[NW], mv[NW];
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        // 16 rows at a time: rows 64 w + 16 g + k (k = 0..15) hold
                        // read bases i0 + k, i0 = 64 w + 16 g - pad; rows with
                        // i0 + k < 0 match every base
                        uint32_t ma[2] = {0u, 0u}, mc[2] = {0u, 0u}, mg[2] = {0u, 0u},
                                 mt[2] = {0u, 0u}, pw[2] = {~0u, ~0u};
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const int i0 = 64 * w + 16 * g - pad;
                            const uint32_t sh = 16 * (g & 1);
                            const int half = g >> 1;
                            uint32_t xa = 0xFFFFu, xc = 0xFFFFu, xg = 0xFFFFu, xt = 0xFFFFu,
                                     pm = 0xFFFFu;
                            if (i0 > -16) {
                                pm = i0 >= 0 ? 0u : (1u << -i0) - 1u;
                                // base k in bits 2k (high bit of its code) and 2k + 1 (low bit)
                                const uint32_t rv = __builtin_bitreverse32(
                                    read_window(a.rw, a.nw, (int64_t)off + i0));
                                const uint32_t h = rv & 0x55555555u, l = (rv >> 1) & 0x55555555u;
                                xa = even_bits(~(h | l) & 0x55555555u) | pm;
                                xc = even_bits(l & ~h) | pm;
                                xg = even_bits(h & ~l) | pm;
                                xt = even_bits(h & l) | pm;
                            }
                            ma[half] |= xa << sh;
                            mc[half] |= xc << sh;
                            mg[half] |= xg << sh;
                            mt[half] |= xt << sh;
                            pw[half] &= ~(pm << sh);
                        }
                        peq[(0 * W + w) * 256 + t] = (uint64_t)ma[1] << 32 | ma[0];
                        peq[(1 * W + w) * 256 + t] = (uint64_t)mc[1] << 32 | mc[0];
                        peq[(2 * W + w) * 256 + t] = (uint64_t)mg[1] << 32 | mg[0];
                        peq[(3 * W + w) * 256 + t] = (uint64_t)mt[1] << 32 | mt[0];
                        pv[2 * w] = pw[0];
                        pv[2 * w + 1] = pw[1];
                        mv[2 * w] = mv[2 * w + 1] = 0u;
                    }
                    const uint64_t lo = (uint64_t)b * a.B;
                    uint64_t hi = lo + a.B + a.O;
                    if (hi > a.G)
                        hi = a.G;
                    // an empty read matches anywhere with no edits: no columns
                    const uint64_t span = hi > lo && L > 0 ? hi - lo : 0;
                    // the wavefront's first word: the most words any of its
                    // scanning lanes needs, counted from the bottom
                    const uint32_t n = (L + 31) >> 5;
                    int nmax = 0;
#pragma unroll
                    for (int v = 1; v <= NW; ++v)
                        nmax += __builtin_amdgcn_ballot_w64(n >= (uint32_t)v) != 0;
                    // 16 reference bases are fetched every 16 columns; their bit
                    // offset inside the first packed word is the span start's,
                    // the same at every fetch.
                    const uint32_t *rp = a.ref + (lo >> 4);
                    const uint32_t wsh = ((uint32_t)lo & 15u) << 1;
                    // one span for all scanning lanes (all but the last bin's)?
                    const uint32_t s_lo = __builtin_amdgcn_readfirstlane((uint32_t)span);
                    const uint32_t s_hi = __builtin_amdgcn_readfirstlane((uint32_t)(span >> 32));
                    const bool uni = __builtin_amdgcn_ballot_w64(
                                         span != ((uint64_t)s_hi << 32 | s_lo)) == 0;
                    const int32_t best =
                        uni ? column_scan_from<NW, 0, true>(NW - nmax, peq + t, pv, mv, rp, wsh,
                                                            span, (int32_t)L)
                            : column_scan_from<NW, 0, false>(NW - nmax, peq + t, pv, mv, rp,
                                                             wsh, span, (int32_t)L);
                    d = min<int32_t>(best, (int32_t)E + 1);
                    ok = best <= (int32_t)E;
                }
                a.dist[i] = d;
                if (ok)
                    atomicOr(&okw[slot >> 5], 1u << (slot & 31));
            }
        }
        __syncthreads();
        if (t < (int)((cnt + 31) / 32))
            a.ok_bits[(base >> 5) + t] = okw[t];
        __syncthreads();
    }
}

hipError_t launch_verify(hipStream_t s, int W, int cus, const VerifyArgs &a)
{
    VerifyArgs copy = a;
    void *args[] = {&copy};
    const void *k = nullptr;
    int wi = 0;
    switch (W) {
    case 1: k = reinterpret_cast<const void *>(&verify_kernel<1>); wi = 0; break;
    case 2: k = reinterpret_cast<const void *>(&verify_kernel<2>); wi = 1; break;
    case 4: k = reinterpret_cast<const void *>(&verify_kernel<4>); wi = 2; break;
    case 8: k = reinterpret_cast<const void *>(&verify_kernel<8>); wi = 3; break;
    default: return hipErrorInvalidValue;
    }
    // workgroups resident per CU (LDS bound), asked once per kernel and
    // process; it only sizes the grid's cap, never what is computed
    static std::atomic<int> resident[4];
    int per_cu = resident[wi].load(std::memory_order_relaxed);
    if (per_cu <= 0) {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0);
        if (e != hipSuccess)
            return e;
        if (per_cu <= 0)
            per_cu = 1;
        resident[wi].store(per_cu, std::memory_order_relaxed);
    }
    // one sorted chunk per workgroup, dispatched as resident ones finish;
    // past 64 times the resident count, each takes a run of m whole chunks
    const uint64_t chunks = (a.n_surv + kVerifyChunk - 1) / kVerifyChunk;
    const uint64_t cap = (uint64_t)per_cu * (uint64_t)(cus > 0 ? cus : 1) * 64;
    const uint64_t m = (chunks + cap - 1) / cap;
    const uint64_t grid = (chunks + m - 1) / m;
    if (grid == 0)
        return hipSuccess;
    return hipLaunchKernel(k, dim3((uint32_t)grid), dim3(256), args, 0, s);
}

}  // namespace grim
