// Chunked bin build for gfx950.
//
// Bin b holds every token whose Q bases lie inside [b*B, min(G, (b+1)*B + O))
// (Section "Genome Metadata Representation": one existence bitvector per
// overlapping bin), i.e. the token starts p with b*B <= p <= (b+1)*B + O - Q and
// p + Q <= G.  Those are S = B + O - Q + 1 consecutive starts: m = S / B whole
// blocks of B starts, then the first R = S % B starts of the next block.  With
// P_j the token set of the first R starts of block j (starts [j*B, (j+1)*B))
// and X_j that of its other starts,
//     V_b = (P_b | X_b) | ... | (P_{b+m-1} | X_{b+m-1}) | P_{b+m}.
// A workgroup takes C consecutive bins.  It sets each token of the starts
// [c0*B, (c0+C+m)*B) once, in P or X of its block in LDS (one LDS atomic per
// token; one thread per packed word of 16 starts, so the reference is read
// with coalesced dword loads), then writes the C vectors as those ORs with
// 16-byte stores that cover one contiguous run of the index.  A token start is
// touched once per chunk instead of once per bin that holds it, and no
// wavefront waits on one bin's span at a time.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grim_internal.h"

namespace grim {

namespace {

constexpr int kBuildThreads = 256;

template <int Q>
constexpr uint32_t lds_words()
{
    return Q == 7 ? 16384u : 8192u;
}

// The 16 starts p0 .. p0+15 of one packed word, all inside [lo, hi).
// For B >= 16 the word crosses at most two boundaries between the P and X
// parts of consecutive blocks: the vector offset of start i (0, 1 or 2
// vectors past the first start's) is the 2-bit field i of K.  With R = 0
// every block is all X and one block boundary moves two vectors.
template <int Q>
__device__ __forceinline__ void set_word_fast(uint32_t *__restrict__ lds, uint64_t x64, uint32_t d,
                                              uint32_t B, uint32_t R)
{
    constexpr uint32_t VW = (1u << (2 * Q)) >> 5;
    const uint32_t j = d / B, r0 = d - j * B;
    const uint32_t base = j * (2 * VW) + (r0 >= R ? VW : 0u);
    uint32_t a, b;
    if (R == 0) {
        a = b = B - r0;
    } else if (r0 < R) {
        a = R - r0;
        b = B - r0;
    } else {
        a = B - r0;
        b = B + R - r0;
    }
    const uint32_t K = (a < 16 ? 0x55555555u << (2 * a) : 0u) + (b < 16 ? 0x55555555u << (2 * b) : 0u);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t x = (uint32_t)((x64 << (2 * i)) >> 32);
        const uint32_t t = x >> (32 - 2 * Q);
        const uint32_t off = (K >> (2 * i)) & 3u;
        atomicOr(&lds[base + off * VW + (t >> 5)], 1u << (t & 31u));
    }
}

// Any stride: block and offset stepped along the word's starts, each start
// checked against [lo, hi).
template <int Q, bool GUARD>
__device__ __forceinline__ void set_word_stepped(uint32_t *__restrict__ lds, uint64_t x64,
                                                 uint64_t p0, uint64_t lo, uint64_t hi, uint32_t B,
                                                 uint32_t R)
{
    constexpr uint32_t VW = (1u << (2 * Q)) >> 5;
    const uint32_t i0 = p0 < lo ? (uint32_t)(lo - p0) : 0u;
    const uint32_t d = (uint32_t)(p0 + i0 - lo);
    uint32_t r = d % B;
    uint32_t jb = (d / B) * (2 * VW);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (GUARD && (i < (int)i0 || p0 + i >= hi))
            continue;
        const uint32_t x = (uint32_t)((x64 << (2 * i)) >> 32);
        const uint32_t t = x >> (32 - 2 * Q);
        atomicOr(&lds[jb + (r >= R ? VW : 0u) + (t >> 5)], 1u << (t & 31u));
        if (++r == B) {
            r = 0;
            jb += 2 * VW;
        }
    }
}

// n_starts = G - Q + 1 (0 when G < Q): valid token starts are [0, n_starts).
template <int Q>
__global__ __launch_bounds__(kBuildThreads) void build_chunk_kernel(
    const uint32_t *__restrict__ ref, uint64_t nw, uint64_t n_starts, uint32_t B, uint32_t m,
    uint32_t R, uint32_t C, uint64_t n_bins, uint32_t *__restrict__ out)
{
    constexpr uint32_t VW = (1u << (2 * Q)) >> 5;
    constexpr uint32_t V4 = VW / 4;
    __shared__ __align__(16) uint32_t lds[lds_words<Q>()];
    uint4 *l4 = reinterpret_cast<uint4 *>(lds);
    const uint32_t tid = threadIdx.x;
    const uint64_t n_chunks = (n_bins + C - 1) / C;
    for (uint64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
        const uint64_t c0 = ch * C;
        const uint32_t nb = (uint32_t)(n_bins - c0 < C ? n_bins - c0 : C);
        const uint32_t nblk = nb + m;
        for (uint32_t i = tid; i < nblk * 2 * V4; i += kBuildThreads)
            l4[i] = make_uint4(0u, 0u, 0u, 0u);
        __syncthreads();

        const uint64_t lo = c0 * B;
        uint64_t hi = (c0 + nblk) * B;
        if (hi > n_starts)
            hi = n_starts;
        if (lo < hi) {
            const uint64_t w_lo = lo >> 4, w_end = ((hi - 1) >> 4) + 1;
            uint64_t wi = w_lo + tid;
            uint32_t w0 = 0, w1 = 0;
            if (wi < w_end) {
                w0 = ref[wi];
                w1 = wi + 1 < nw ? ref[wi + 1] : 0u;
            }
            for (; wi < w_end; wi += kBuildThreads) {
                // Next word pair in flight while this one is set.
                const uint64_t wn = wi + kBuildThreads;
                uint32_t n0 = 0, n1 = 0;
                if (wn < w_end) {
                    n0 = ref[wn];
                    n1 = wn + 1 < nw ? ref[wn + 1] : 0u;
                }
                const uint64_t x64 = ((uint64_t)w0 << 32) | w1;
                const uint64_t p0 = wi << 4;
                if (p0 >= lo && p0 + 16 <= hi) {
                    if (B >= 16)
                        set_word_fast<Q>(lds, x64, (uint32_t)(p0 - lo), B, R);
                    else
                        set_word_stepped<Q, false>(lds, x64, p0, lo, hi, B, R);
                } else {
                    set_word_stepped<Q, true>(lds, x64, p0, lo, hi, B, R);
                }
                w0 = n0;
                w1 = n1;
            }
        }
        __syncthreads();

        uint4 *o4 = reinterpret_cast<uint4 *>(out + c0 * VW);
        for (uint32_t i = tid; i < nb * V4; i += kBuildThreads) {
            const uint32_t b = i / V4, w = i % V4;
            uint4 acc = l4[(b + m) * 2 * V4 + w];
            for (uint32_t k = 0; k < m; ++k) {
                const uint4 a = l4[(b + k) * 2 * V4 + w];
                const uint4 c = l4[(b + k) * 2 * V4 + V4 + w];
                acc.x |= a.x | c.x;
                acc.y |= a.y | c.y;
                acc.z |= a.z | c.z;
                acc.w |= a.w | c.w;
            }
            o4[i] = acc;
        }
        __syncthreads();
    }
}

template <int Q>
hipError_t launch_chunk(uint32_t cus, hipStream_t s, const uint32_t *ref, uint64_t nw, uint64_t G,
                        uint64_t B, uint64_t O, uint64_t n_bins, uint32_t *out)
{
    constexpr uint64_t VW = (1u << (2 * Q)) >> 5;
    const int64_t S = (int64_t)B + (int64_t)O - Q + 1;
    const uint64_t m = S > 0 ? (uint64_t)S / B : 0;
    const uint64_t R = S > 0 ? (uint64_t)S % B : 0;
    const uint64_t fit = lds_words<Q>() / (2 * VW);
    if (m >= fit)
        return hipErrorNotSupported;
    uint64_t C = fit - m;
    // Offsets of starts inside a chunk are 32-bit: (C + m) * B + 16 < 2^31.
    const uint64_t span_cap = ((1ull << 31) - 16) / B;
    if (span_cap <= m)
        return hipErrorNotSupported;
    if (C > span_cap - m)
        C = span_cap - m;
    const uint64_t n_starts = G >= (uint64_t)Q ? G - Q + 1 : 0;
    uint64_t grid = (n_bins + C - 1) / C;
    const uint64_t cap = (uint64_t)cus * 64;
    if (grid > cap)
        grid = cap;
    if (grid == 0)
        grid = 1;
    hipLaunchKernelGGL(build_chunk_kernel<Q>, dim3((uint32_t)grid), dim3(kBuildThreads), 0, s, ref,
                       nw, n_starts, (uint32_t)B, (uint32_t)m, (uint32_t)R, (uint32_t)C, n_bins,
                       out);
    return hipGetLastError();
}

}  // namespace

// Returns hipErrorNotSupported, launching nothing, when the bin geometry does
// not fit the chunked form (more whole blocks per bin than the LDS holds, or a
// stride so large that offsets inside a chunk leave 32 bits); the caller then
// uses the per-bin kernel.
hipError_t launch_build_chunked(int q, uint32_t cus, hipStream_t s, const uint32_t *ref,
                                uint64_t nw, uint64_t G, uint64_t B, uint64_t O, uint64_t n_bins,
                                uint32_t *out)
{
    if (B == 0 || B >= (1ull << 31) || O >= (1ull << 40))
        return hipErrorNotSupported;
    switch (q) {
    case 4: return launch_chunk<4>(cus, s, ref, nw, G, B, O, n_bins, out);
    case 5: return launch_chunk<5>(cus, s, ref, nw, G, B, O, n_bins, out);
    case 6: return launch_chunk<6>(cus, s, ref, nw, G, B, O, n_bins, out);
    case 7: return launch_chunk<7>(cus, s, ref, nw, G, B, O, n_bins, out);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace grim
