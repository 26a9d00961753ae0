// The serving scheduler's device operations on HIP (see grim_serve_backend.h):
// hipMalloc'd pool, page-locked host memory, non-blocking streams, async
// copies, the batched filter launch, and completion notices as host functions
// queued on the stream.
#include <hip/hip_runtime.h>

#include "grim_internal.h"
#include "grim_serve_backend.h"

namespace {

struct HipBackend final : grim_serve::Backend {
    int current_device(int *dev) const override
    {
        return hipGetDevice(dev) == hipSuccess ? GRIM_OK : GRIM_E_HIP;
    }
    void set_device(int dev) const override { (void)hipSetDevice(dev); }
    int index_device(const grim_index_t *idx) const override
    {
        grim_index_info_t info;
        return grim_index_info(idx, &info) == GRIM_OK ? info.device : -1;
    }
    int device_alloc(uint64_t bytes, uint8_t **p) const override
    {
        return hipMalloc(reinterpret_cast<void **>(p), bytes) == hipSuccess ? GRIM_OK
                                                                            : GRIM_E_NOMEM;
    }
    void device_free(uint8_t *p) const override
    {
        if (p)
            (void)hipFree(p);
    }
    int pinned_alloc(uint64_t bytes, uint8_t **p) const override
    {
        return hipHostMalloc(reinterpret_cast<void **>(p), bytes, hipHostMallocDefault) ==
                       hipSuccess
                   ? GRIM_OK
                   : GRIM_E_NOMEM;
    }
    void pinned_free(uint8_t *p) const override
    {
        if (p)
            (void)hipHostFree(p);
    }
    int stream_create(void **s) const override
    {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return GRIM_E_HIP;
        *s = st;
        return GRIM_OK;
    }
    void stream_destroy(void *s) const override
    {
        (void)hipStreamDestroy(static_cast<hipStream_t>(s));
    }
    int stream_sync(void *s) const override
    {
        return hipStreamSynchronize(static_cast<hipStream_t>(s)) == hipSuccess ? GRIM_OK
                                                                               : GRIM_E_HIP;
    }
    int copy_h2d(void *dst, const void *src, uint64_t bytes, void *s) const override
    {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice,
                              static_cast<hipStream_t>(s)) == hipSuccess
                   ? GRIM_OK
                   : GRIM_E_HIP;
    }
    int copy_d2h(void *dst, const void *src, uint64_t bytes, void *s) const override
    {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost,
                              static_cast<hipStream_t>(s)) == hipSuccess
                   ? GRIM_OK
                   : GRIM_E_HIP;
    }
    int store_d2h(void *dst, const void *src, uint64_t bytes, void *s) const override
    {
        return grim::launch_copy_to_host(static_cast<hipStream_t>(s), dst, src, bytes) ==
                       hipSuccess
                   ? GRIM_OK
                   : GRIM_E_HIP;
    }
    bool device_writable(const void *p) const override
    {
        hipPointerAttribute_t a;
        if (hipPointerGetAttributes(&a, p) != hipSuccess) {
            (void)hipGetLastError();  // pageable memory: clear the error
            return false;
        }
        return a.type == hipMemoryTypeHost;
    }
    int notify(void *s, void (*fn)(void *), void *arg) const override
    {
        return hipLaunchHostFunc(static_cast<hipStream_t>(s), fn, arg) == hipSuccess ? GRIM_OK
                                                                                     : GRIM_E_HIP;
    }
    int filter(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
               uint32_t *pass_bits, void *ws, uint64_t ws_bytes, void *s) const override
    {
        return grim_filter_batch(idx, b, counts, pass_bits, ws, ws_bytes, nullptr, s);
    }
    uint64_t workspace_bytes(const grim_index_t *idx, uint64_t n_pairs) const override
    {
        uint64_t b = 0;
        grim_workspace_size(idx, n_pairs, nullptr, &b);
        return b;
    }
};

}  // namespace

const grim_serve::Backend &grim_serve::backend()
{
    static const HipBackend b;
    return b;
}
