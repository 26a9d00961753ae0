// Device-to-host copies done by a kernel that stores straight into page-locked
// host memory (the serving runtime's downloads when its streams share one copy
// engine: stores from the CUs need no copy engine, so they overlap the
// engine's uploads).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "grim_internal.h"

namespace grim {

namespace {

constexpr int kCopyThreads = 256;

// Copies n bytes from device memory to host memory the device can write.
// Stores into host memory go over the host link, so they are made 16 bytes
// wide whatever the two ends' alignment: the first bytes up to dst's next
// 16-byte boundary and the last ones are copied bytewise; in between each
// thread assembles a 16-byte store from four 4-byte loads (src then sits on a
// 4-byte boundary whenever both ends do, the serving runtime's case) or from
// bytes otherwise.  Every thread strides the whole range.
__global__ __launch_bounds__(kCopyThreads) void copy_to_host_kernel(uint8_t *dst, const uint8_t *src,
                                                                    uint64_t n)
{
    const uint64_t tid = (uint64_t)blockIdx.x * kCopyThreads + threadIdx.x;
    const uint64_t nth = (uint64_t)gridDim.x * kCopyThreads;
    uint64_t head = (16 - (reinterpret_cast<uintptr_t>(dst) & 15)) & 15;
    if (head > n)
        head = n;
    const uint64_t n16 = (n - head) >> 4;
    const uint64_t tail = head + (n16 << 4);
    for (uint64_t i = tid; i < head; i += nth)
        dst[i] = src[i];
    uint4 *d = reinterpret_cast<uint4 *>(dst + head);
    const uint8_t *s = src + head;
    if ((reinterpret_cast<uintptr_t>(s) & 3) == 0) {
        const uint32_t *s4 = reinterpret_cast<const uint32_t *>(s);
        for (uint64_t i = tid; i < n16; i += nth)
            d[i] = make_uint4(s4[4 * i], s4[4 * i + 1], s4[4 * i + 2], s4[4 * i + 3]);
    } else {
        for (uint64_t i = tid; i < n16; i += nth) {
            uint32_t w[4];
            for (int k = 0; k < 4; ++k)
                w[k] = (uint32_t)s[16 * i + 4 * k] | ((uint32_t)s[16 * i + 4 * k + 1] << 8) |
                       ((uint32_t)s[16 * i + 4 * k + 2] << 16) | ((uint32_t)s[16 * i + 4 * k + 3] << 24);
            d[i] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
    for (uint64_t i = tail + tid; i < n; i += nth)
        dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy_to_host(hipStream_t s, void *dst, const void *src, uint64_t bytes)
{
    if (!bytes)
        return hipSuccess;
    // 16 workgroups already store at the host link's rate (55 GB/s measured,
    // 51 GB/s beside a DMA upload), and leave the other CUs to the filter
    const uint64_t blocks = std::min<uint64_t>((bytes + 16 * kCopyThreads * 8 - 1) /
                                                   (16 * kCopyThreads * 8),
                                               16);
    hipLaunchKernelGGL(copy_to_host_kernel, dim3((uint32_t)blocks), dim3(kCopyThreads), 0, s,
                       static_cast<uint8_t *>(dst), static_cast<const uint8_t *>(src), bytes);
    return hipGetLastError();
}

}  // namespace grim
