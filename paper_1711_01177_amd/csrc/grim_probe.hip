// Memory-ceiling probes for the filter's access pattern (diagnostics).  The
// paper argues that the filter is bound by memory bandwidth (Section "Candidacy
// for 3D-Stacked Memory Implementations"); these kernels measure what the
// device's memory delivers for exactly the filter's accesses, without the
// filter's token work, so the filter's rate can be put beside it.
#include <hip/hip_runtime.h>

#include "grim_internal.h"

namespace grim {
namespace {

// R: 16-byte pieces per bin vector; G: lanes per vector (each loads R / G
// pieces); U: vectors in flight per lane group.  One wavefront step covers
// (64 / G) * U vectors, whose ids are loaded by one coalesced load.
template <int R, int G, int U>
__global__ __launch_bounds__(256) void probe_gather_kernel(const uint4 *__restrict__ vec,
                                                           uint64_t n_records,
                                                           const uint32_t *__restrict__ ids,
                                                           uint64_t n, int32_t *__restrict__ out)
{
    constexpr int NG = 64 / G, STEP = NG * U, W = R / G;
    static_assert(STEP <= 64 && W * G == R, "launch shape");
    const int lane = threadIdx.x & 63, g = lane / G, lg = lane % G;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t n_waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t base = wave * STEP; base < n; base += n_waves * STEP) {
        const uint32_t mine = (lane < STEP && base + lane < n) ? ids[base + lane] : ~0u;
        uint4 v[U][W];
        bool inr[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t id = __shfl(mine, u * NG + g);
            inr[u] = base + u * NG + g < n && id < n_records;
#pragma unroll
            for (int w = 0; w < W; ++w)
                v[u][w] = inr[u] ? vec[(uint64_t)id * R + w * G + lg] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint32_t acc = 0;
#pragma unroll
            for (int w = 0; w < W; ++w)
                acc += __popc(v[u][w].x) + __popc(v[u][w].y) + __popc(v[u][w].z) +
                       __popc(v[u][w].w);
#pragma unroll
            for (int s = G / 2; s >= 1; s >>= 1)
                acc += __shfl_xor(acc, s);
            const uint64_t k = base + u * NG + g;
            if (lg == 0 && k < n)
                out[k] = inr[u] ? (int32_t)acc : -1;
        }
    }
}

__global__ __launch_bounds__(256) void probe_stream_kernel(const uint4 *__restrict__ src,
                                                           uint64_t n16, uint32_t *__restrict__ sink)
{
    uint32_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 v = src[i];
        acc += v.x ^ v.y ^ v.z ^ v.w;
    }
    // a store that never happens in practice keeps the loads from being removed
    if (acc == 0x9e3779b9u)
        sink[0] = acc;
}

}  // namespace

hipError_t launch_probe_gather(hipStream_t s, uint32_t q, uint32_t grid, const void *vec,
                               uint64_t n_records, const uint32_t *ids, uint64_t n, int32_t *out)
{
    const uint4 *v = reinterpret_cast<const uint4 *>(vec);
    switch (q) {
    case 4: hipLaunchKernelGGL((probe_gather_kernel<2, 2, 2>), dim3(grid), dim3(256), 0, s, v, n_records, ids, n, out); break;
    case 5: hipLaunchKernelGGL((probe_gather_kernel<8, 8, 8>), dim3(grid), dim3(256), 0, s, v, n_records, ids, n, out); break;
    case 6: hipLaunchKernelGGL((probe_gather_kernel<32, 8, 2>), dim3(grid), dim3(256), 0, s, v, n_records, ids, n, out); break;
    case 7: hipLaunchKernelGGL((probe_gather_kernel<128, 64, 1>), dim3(grid), dim3(256), 0, s, v, n_records, ids, n, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_probe_stream(hipStream_t s, uint32_t grid, const void *src, uint64_t n16,
                               uint32_t *sink)
{
    hipLaunchKernelGGL(probe_stream_kernel, dim3(grid), dim3(256), 0, s,
                       reinterpret_cast<const uint4 *>(src), n16, sink);
    return hipGetLastError();
}

}  // namespace grim
