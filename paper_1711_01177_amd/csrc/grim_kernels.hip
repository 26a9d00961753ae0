// GRIM-Filter HIP kernels for gfx950 (MI355X).
//
// The filter (Kim et al., BMC Genomics 2018, Sections "GRIM-Filter Operation"
// and "Taking Errors into Account") is an integer gather + popcount: for each
// (read, candidate bin) pair, sum over the read's token positions the bin's
// existence bit of that token, then compare with T = ntok - q * ceil(e L).
//
// Decomposition used on the GPU (exact, no approximation):
//   Let m(t) be the number of positions of the read whose token is t.  Then
//     sum_i V[tok_i] = sum_t m(t) V[t] = sum_k 2^k popcount(M_k & V)
//   where M_k is the bit plane holding bit k of m(t) for every token t.  The
//   planes of one read are built once in LDS with atomic-xor carry chains (an
//   increment of a bit-sliced counter), so the per-candidate work is a few
//   AND + popcount per 16-byte slice of the candidate's vector, independent of
//   the read length, with repeated tokens counted exactly.
//
// Memory layout: bin vectors bin-major, 4^q / 8 bytes each, so one candidate
// is one contiguous 32 B .. 2 KiB run; G lanes load it with 16-byte loads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grim_internal.h"

namespace grim {

// ------------------------------------------------------------ device helpers
// Orders the LDS traffic of one wavefront across phases (build planes, read
// planes, reuse).  Waves of a workgroup never share LDS regions in these
// kernels, so wavefront scope is enough and no memory counters are drained.
__device__ __forceinline__ void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t x)
{
    return __builtin_amdgcn_readfirstlane(x);
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t x)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Token of Q bases starting at stream position pos of a packed sequence
// (16 bases per word, first base in the top bits): a funnel shift of two
// adjacent words.  Reads past the end of the buffer see zero words.
template <int Q>
__device__ __forceinline__ uint32_t token_at(const uint32_t *__restrict__ w, uint64_t nw,
                                             uint64_t pos)
{
    const uint64_t wi = pos >> 4;
    const uint32_t sh = (uint32_t)(pos & 15u) << 1;
    uint64_t x = (uint64_t)(wi < nw ? w[wi] : 0u) << 32;
    if (sh + 2 * Q > 32)
        x |= (wi + 1 < nw ? w[wi + 1] : 0u);
    return (uint32_t)((x << sh) >> (64 - 2 * Q));
}

__device__ __forceinline__ uint32_t popc_and(const uint4 &a, const uint4 &b)
{
    return __popc(a.x & b.x) + __popc(a.y & b.y) + __popc(a.z & b.z) + __popc(a.w & b.w);
}

// Build the multiplicity bit planes of one read's tokens in LDS (one wave).
// planes holds npl planes of VW words each.  Returns the number of planes in
// use (0 for a read without tokens).  npl is chosen by the host so that
// 2^npl > ntok, hence no carry can leave the last plane.
template <int Q>
__device__ int build_planes(uint32_t *planes, int npl, const uint32_t *__restrict__ rw, uint64_t nw,
                            uint64_t off, uint32_t ntok, int lane)
{
    constexpr int VW = (1 << (2 * Q)) >> 5;
    for (int i = lane; i < npl * VW; i += kWave)
        planes[i] = 0u;
    wave_fence();
    int top = 0;
    for (uint32_t i = lane; i < ntok; i += kWave) {
        const uint32_t t = token_at<Q>(rw, nw, off + i);
        const uint32_t wd = t >> 5, bit = 1u << (t & 31u);
        int k = 0;
        uint32_t old = atomicXor(&planes[wd], bit);
        while ((old & bit) && k + 1 < npl) {
            ++k;
            old = atomicXor(&planes[k * VW + wd], bit);
        }
        top = max(top, k + 1);
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
        top = max(top, __shfl_xor(top, s));
    wave_fence();
    return top;
}

__device__ __forceinline__ void flag(uint32_t *status, uint32_t f)
{
    atomicOr(status, f);
}

// ---------------------------------------------------------------- bin build
// One wavefront per bin (grid-stride): every lane takes every 64th token start
// of the bin's span and sets the token's bit in an LDS copy of the vector,
// which is then written out whole.  Bin b spans [b*B, min(G, (b+1)*B + O)).
template <int Q>
__global__ __launch_bounds__(256) void build_bins_kernel(const uint32_t *__restrict__ ref,
                                                         uint64_t nw, uint64_t G, uint64_t B,
                                                         uint64_t O, uint64_t n_bins,
                                                         uint32_t *__restrict__ out)
{
    constexpr int VW = (1 << (2 * Q)) >> 5;
    __shared__ uint32_t vec_lds[4][VW];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t *vec = vec_lds[wv];
    for (uint64_t b = (uint64_t)blockIdx.x * 4 + wv; b < n_bins; b += (uint64_t)gridDim.x * 4) {
        for (int i = lane; i < VW; i += kWave)
            vec[i] = 0u;
        wave_fence();
        const uint64_t lo = b * B;
        uint64_t hi = (b + 1) * B + O;
        if (hi > G)
            hi = G;
        for (uint64_t p = lo + lane; p + Q <= hi; p += kWave) {
            const uint32_t t = token_at<Q>(ref, nw, p);
            atomicOr(&vec[t >> 5], 1u << (t & 31u));
        }
        wave_fence();
        uint32_t *dst = out + b * VW;
        for (int i = lane; i < VW; i += kWave)
            dst[i] = vec[i];
        wave_fence();
    }
}

// ---------------------------------------------------------------- work list
// Thread i < n_tiles records the read that owns pair i * tile_pairs: the last
// read r with cand_off[r] <= i * tile_pairs.  Thread 0 also resets the status
// word and the tile counter of this launch.
__global__ __launch_bounds__(256) void worklist_kernel(const uint64_t *__restrict__ cand_off,
                                                       uint64_t n_reads, uint32_t tile_pairs,
                                                       uint32_t n_tiles, uint32_t *tile_read,
                                                       uint32_t *status, uint32_t *counter)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *status = 0u;
        *counter = 0u;
    }
    if (i >= n_tiles || n_reads == 0)
        return;
    const uint64_t p = i * tile_pairs;
    uint64_t lo = 0, hi = n_reads - 1;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (cand_off[mid] <= p)
            lo = mid;
        else
            hi = mid - 1;
    }
    tile_read[i] = (uint32_t)lo;
}

__global__ void zero_words_kernel(uint32_t *p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ----------------------------------------------------------- batched filter
// Persistent kernel.  Each wavefront repeatedly takes the next tile of
// tile_pairs consecutive pairs (atomic counter), walks the reads that own the
// tile's pairs, builds each read's planes once, and processes its candidates
// with NG = 64 / G lane groups, U candidates in flight per group.  Pass bits of
// the tile accumulate in LDS and are stored as whole words at the end of the
// tile (tiles start on multiples of 64 pairs, so no other wave writes them).
template <int Q, int G, int U>
__global__ __launch_bounds__(256) void filter_batched_kernel(FilterArgs a)
{
    constexpr int VW = (1 << (2 * Q)) >> 5;  // 32-bit words per vector
    constexpr int CH = VW / 4;               // 16-byte slices per vector
    constexpr int C = CH / G;                // slices per lane
    constexpr int NG = kWave / G;            // candidates per wave step
    static_assert(C >= 1 && CH % G == 0, "lane group wider than the vector");

    extern __shared__ uint32_t lds[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int npl = a.npl;
    const uint32_t mask_words = a.tile_pairs >> 5;
    // each wave's region: its planes, then the tile's pass-bit words rounded up
    // to whole 16-byte units, so that every region (and plane) starts 16-byte
    // aligned for the uint4 plane reads
    uint32_t *planes = lds + (size_t)wv * (npl * VW + ((mask_words + 3u) & ~3u));
    uint32_t *tmask = planes + npl * VW;
    const int g = lane / G, lg = lane % G;

    for (;;) {
        uint32_t tile = 0;
        if (lane == 0)
            tile = atomicAdd(a.tile_counter, 1u);
        tile = uniform_u32(__shfl(tile, 0));
        if (tile >= a.n_tiles)
            break;
        const uint64_t t0 = (uint64_t)tile * a.tile_pairs;
        const uint64_t t1 = min(t0 + a.tile_pairs, a.n_pairs);
        for (uint32_t i = lane; i < mask_words; i += kWave)
            tmask[i] = 0u;
        wave_fence();

        uint64_t r = a.tile_read[tile];
        r = uniform_u64(r);
        uint64_t p = t0;
        while (p < t1) {
            if (r >= a.n_reads) {  // pairs beyond the last read's range
                if (lane == 0)
                    flag(a.status, GRIM_FLAG_CAND_OFF);
                for (uint64_t k = p + lane; k < t1; k += kWave)
                    a.counts[k] = -1;
                break;
            }
            const uint64_t cb = uniform_u64(a.cand_off[r]);
            const uint64_t ce = uniform_u64(a.cand_off[r + 1]);
            if (ce <= p) {
                ++r;
                continue;
            }
            if (cb > p) {  // a gap owned by no read: cand_off is not a CSR array
                const uint64_t ge = min(cb, t1);
                if (lane == 0)
                    flag(a.status, GRIM_FLAG_CAND_OFF);
                for (uint64_t k = p + lane; k < ge; k += kWave)
                    a.counts[k] = -1;
                p = ge;
                continue;
            }
            const uint64_t pe = min(ce, t1);
            const uint32_t L = uniform_u32(a.read_len[r]);
            const uint64_t off = uniform_u64(a.read_off[r]);
            const uint64_t nbases = a.nw * 16;
            if (L > a.max_len || off > nbases || L > nbases - off) {
                if (lane == 0)
                    flag(a.status, GRIM_FLAG_READ);
                for (uint64_t k = p + lane; k < pe; k += kWave)
                    a.counts[k] = -1;
                p = pe;
                ++r;
                continue;
            }
            const uint32_t ntok = L >= (uint32_t)Q ? L - Q + 1 : 0u;
            // bin ids of the segment's first step are requested before the
            // planes are built, and every step requests the next step's ids
            // before gathering its own vectors
            constexpr int STEP = NG * U;
            auto load_ids = [&](uint64_t c) -> uint32_t {
                if constexpr (STEP <= kWave) {
                    const uint64_t kk = c + lane;
                    return (lane < STEP && kk < pe) ? a.cand_bin[kk] : 0u;
                } else {
                    return 0u;
                }
            };
            uint32_t next_ids = load_ids(p);
            const int np = build_planes<Q>(planes, npl, a.rw, a.nw, off, ntok, lane);
            const uint32_t e_num = uniform_u32(a.read_e[r]);
            const uint64_t E = ((uint64_t)e_num * L + a.e_den - 1) / a.e_den;
            const int64_t T = (int64_t)ntok - (int64_t)Q * (int64_t)E;

            // planes 0 and 1 stay in registers for the whole segment
            uint4 p0[C], p1[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int w = (c * G + lg) * 4;
                p0[c] = np > 0 ? *reinterpret_cast<const uint4 *>(planes + w) : make_uint4(0, 0, 0, 0);
                p1[c] = np > 1 ? *reinterpret_cast<const uint4 *>(planes + VW + w)
                               : make_uint4(0, 0, 0, 0);
            }

            for (uint64_t c0 = p; c0 < pe; c0 += (uint64_t)STEP) {
                uint32_t bin[U];
                bool ok[U], inr[U];
                if constexpr (STEP <= kWave) {
                    const uint32_t mine = next_ids;
                    next_ids = load_ids(c0 + STEP);
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        bin[u] = __shfl(mine, u * NG + g);
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const uint64_t kk = c0 + (uint64_t)u * NG + g;
                        bin[u] = kk < pe ? a.cand_bin[kk] : 0u;
                    }
                }
                uint4 v[U][C];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t kk = c0 + (uint64_t)u * NG + g;
                    ok[u] = kk < pe;
                    inr[u] = ok[u] && bin[u] < a.n_bins;
                    const uint4 *src = a.vec + (uint64_t)bin[u] * CH + lg;
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        v[u][c] = inr[u] ? src[c * G] : make_uint4(0, 0, 0, 0);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    uint32_t acc = 0;
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        acc += popc_and(p0[c], v[u][c]) + (popc_and(p1[c], v[u][c]) << 1);
                    for (int k = 2; k < np; ++k) {
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            const uint4 pk = *reinterpret_cast<const uint4 *>(
                                planes + k * VW + (c * G + lg) * 4);
                            acc += popc_and(pk, v[u][c]) << k;
                        }
                    }
#pragma unroll
                    for (int s = G / 2; s >= 1; s >>= 1)
                        acc += __shfl_xor(acc, s);
                    if (lg == 0 && ok[u]) {
                        const uint64_t kk = c0 + (uint64_t)u * NG + g;
                        const int32_t cnt = inr[u] ? (int32_t)acc : -1;
                        a.counts[kk] = cnt;
                        if (!inr[u])
                            flag(a.status, GRIM_FLAG_BIN_RANGE);
                        else if ((int64_t)cnt >= T)
                            atomicOr(&tmask[(kk - t0) >> 5], 1u << ((kk - t0) & 31u));
                    }
                }
            }
            wave_fence();  // planes are rebuilt by the next segment
            p = pe;
            ++r;
        }
        wave_fence();
        const uint32_t nwords = (uint32_t)((t1 - t0 + 31) >> 5);
        for (uint32_t i = lane; i < nwords; i += kWave)
            a.pass_bits[(t0 >> 5) + i] = tmask[i];
        wave_fence();
    }
}

// ------------------------------------------------------------- plain filter
// One workgroup (one wavefront) per read: build the read's planes, then walk
// its candidates NG at a time, reading every plane from LDS for every
// candidate; pass bits are set with global atomics into a pre-zeroed mask.
template <int Q>
__global__ __launch_bounds__(64) void filter_plain_kernel(FilterArgs a)
{
    constexpr int VW = (1 << (2 * Q)) >> 5;
    constexpr int CH = VW / 4;
    constexpr int G = CH < kWave ? CH : kWave;
    constexpr int C = CH / G;
    constexpr int NG = kWave / G;
    extern __shared__ uint32_t lds[];
    uint32_t *planes = lds;
    const int lane = threadIdx.x & 63;
    const int g = lane / G, lg = lane % G;
    for (uint64_t r = blockIdx.x; r < a.n_reads; r += gridDim.x) {
        const uint64_t cb = a.cand_off[r], ce = a.cand_off[r + 1];
        if (ce <= cb) {
            if (ce < cb && lane == 0)
                flag(a.status, GRIM_FLAG_CAND_OFF);
            continue;
        }
        if (ce > a.n_pairs) {
            if (lane == 0)
                flag(a.status, GRIM_FLAG_CAND_OFF);
            continue;
        }
        const uint32_t L = a.read_len[r];
        const uint64_t off = a.read_off[r];
        const uint64_t nbases = a.nw * 16;
        if (L > a.max_len || off > nbases || L > nbases - off) {
            if (lane == 0)
                flag(a.status, GRIM_FLAG_READ);
            for (uint64_t k = cb + lane; k < ce; k += kWave)
                a.counts[k] = -1;
            continue;
        }
        const uint32_t ntok = L >= (uint32_t)Q ? L - Q + 1 : 0u;
        const int np = build_planes<Q>(planes, a.npl, a.rw, a.nw, off, ntok, lane);
        const uint64_t E = ((uint64_t)a.read_e[r] * L + a.e_den - 1) / a.e_den;
        const int64_t T = (int64_t)ntok - (int64_t)Q * (int64_t)E;
        for (uint64_t c0 = cb; c0 < ce; c0 += NG) {
            const uint64_t kk = c0 + g;
            const bool ok = kk < ce;
            const uint32_t bin = ok ? a.cand_bin[kk] : 0u;
            const bool inr = ok && bin < a.n_bins;
            uint32_t acc = 0;
            if (inr) {
                const uint4 *src = a.vec + (uint64_t)bin * CH + lg;
                for (int c = 0; c < C; ++c) {
                    const uint4 v = src[c * G];
                    for (int k = 0; k < np; ++k) {
                        const uint4 pk =
                            *reinterpret_cast<const uint4 *>(planes + k * VW + (c * G + lg) * 4);
                        acc += popc_and(pk, v) << k;
                    }
                }
            }
            for (int s = G / 2; s >= 1; s >>= 1)
                acc += __shfl_xor(acc, s);
            if (lg == 0 && ok) {
                const int32_t cnt = inr ? (int32_t)acc : -1;
                a.counts[kk] = cnt;
                if (!inr)
                    flag(a.status, GRIM_FLAG_BIN_RANGE);
                else if ((int64_t)cnt >= T)
                    atomicOr(&a.pass_bits[kk >> 5], 1u << (kk & 31u));
            }
        }
        wave_fence();
    }
}

// ---------------------------------------------------------------- dispatch
#define GRIM_V(Q, G, U) {Q, G, U, reinterpret_cast<const void *>(&filter_batched_kernel<Q, G, U>)}
static const BatchedVariant kBatched[] = {
    GRIM_V(4, 2, 2),  GRIM_V(4, 2, 4),  GRIM_V(4, 2, 8),  GRIM_V(4, 1, 8),
    GRIM_V(5, 8, 1),  GRIM_V(5, 8, 2),  GRIM_V(5, 8, 4),  GRIM_V(5, 8, 8),
    GRIM_V(5, 4, 2),  GRIM_V(5, 4, 4),  GRIM_V(5, 4, 8),  GRIM_V(5, 2, 4),
    GRIM_V(6, 32, 1), GRIM_V(6, 32, 2), GRIM_V(6, 32, 4), GRIM_V(6, 32, 8),
    GRIM_V(6, 16, 2), GRIM_V(6, 16, 4), GRIM_V(6, 8, 1),  GRIM_V(6, 8, 2),
    GRIM_V(7, 64, 1), GRIM_V(7, 64, 2), GRIM_V(7, 64, 4), GRIM_V(7, 32, 1),
    GRIM_V(7, 32, 2),
};
#undef GRIM_V

const BatchedVariant *batched_variants(int *n)
{
    *n = (int)(sizeof(kBatched) / sizeof(kBatched[0]));
    return kBatched;
}

const void *plain_kernel(int q)
{
    switch (q) {
    case 4: return reinterpret_cast<const void *>(&filter_plain_kernel<4>);
    case 5: return reinterpret_cast<const void *>(&filter_plain_kernel<5>);
    case 6: return reinterpret_cast<const void *>(&filter_plain_kernel<6>);
    case 7: return reinterpret_cast<const void *>(&filter_plain_kernel<7>);
    default: return nullptr;
    }
}

hipError_t launch_build(int q, dim3 grid, hipStream_t s, const uint32_t *ref, uint64_t nw,
                        uint64_t G, uint64_t B, uint64_t O, uint64_t n_bins, uint32_t *out)
{
    switch (q) {
    case 4: hipLaunchKernelGGL(build_bins_kernel<4>, grid, dim3(256), 0, s, ref, nw, G, B, O, n_bins, out); break;
    case 5: hipLaunchKernelGGL(build_bins_kernel<5>, grid, dim3(256), 0, s, ref, nw, G, B, O, n_bins, out); break;
    case 6: hipLaunchKernelGGL(build_bins_kernel<6>, grid, dim3(256), 0, s, ref, nw, G, B, O, n_bins, out); break;
    case 7: hipLaunchKernelGGL(build_bins_kernel<7>, grid, dim3(256), 0, s, ref, nw, G, B, O, n_bins, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_worklist(hipStream_t s, const uint64_t *cand_off, uint64_t n_reads,
                           uint32_t tile_pairs, uint32_t n_tiles, uint32_t *tile_read,
                           uint32_t *status, uint32_t *counter)
{
    const uint32_t blocks = n_tiles ? (n_tiles + 255) / 256 : 1;
    hipLaunchKernelGGL(worklist_kernel, dim3(blocks), dim3(256), 0, s, cand_off, n_reads,
                       tile_pairs, n_tiles, tile_read, status, counter);
    return hipGetLastError();
}

hipError_t launch_zero(hipStream_t s, uint32_t *p, uint64_t n)
{
    uint64_t blocks = (n + 255) / 256;
    if (blocks < 1)
        blocks = 1;
    if (blocks > 65536)
        blocks = 65536;
    hipLaunchKernelGGL(zero_words_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_filter(const void *kernel, dim3 grid, dim3 block, size_t lds_bytes,
                         hipStream_t s, const FilterArgs &a)
{
    FilterArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(kernel, grid, block, args, lds_bytes, s);
}

}  // namespace grim
