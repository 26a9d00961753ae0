// The device operations the serving scheduler (grim_serve.cpp) uses, behind
// one interface so that the scheduler itself holds no HIP call.  The library
// links the HIP implementation (grim_serve_hip.cpp); the CPU tests link the
// scheduler against a host-memory implementation instead, to run it under
// ThreadSanitizer with injected failures.
//
// Semantics every implementation provides:
//   - a stream runs the operations queued on it in order; operations on
//     different streams may run concurrently;
//   - copy_h2d / copy_d2h / filter are asynchronous on their stream;
//   - notify(s, fn, arg) calls fn(arg) once every operation queued on s before
//     it has completed (results of earlier copies are then visible to the
//     host); fn runs on a thread of the implementation, must not block and must
//     not call back into the backend;
//   - enqueueing on one stream from several threads is allowed.
#pragma once

#include <stdint.h>

#include "grim.h"

namespace grim_serve {

struct Backend {
    virtual ~Backend() = default;
    // devices and index
    virtual int current_device(int *dev) const = 0;
    virtual void set_device(int dev) const = 0;
    virtual int index_device(const grim_index_t *idx) const = 0;
    // memory: device pool and page-locked host memory
    virtual int device_alloc(uint64_t bytes, uint8_t **p) const = 0;
    virtual void device_free(uint8_t *p) const = 0;
    virtual int pinned_alloc(uint64_t bytes, uint8_t **p) const = 0;
    virtual void pinned_free(uint8_t *p) const = 0;
    // streams
    virtual int stream_create(void **s) const = 0;
    virtual void stream_destroy(void *s) const = 0;
    virtual int stream_sync(void *s) const = 0;
    virtual int copy_h2d(void *dst, const void *src, uint64_t bytes, void *s) const = 0;
    virtual int copy_d2h(void *dst, const void *src, uint64_t bytes, void *s) const = 0;
    // copy_d2h done by the device's compute units storing into host memory
    // (no copy engine); dst must be memory for which device_writable holds
    virtual int store_d2h(void *dst, const void *src, uint64_t bytes, void *s) const = 0;
    virtual bool device_writable(const void *p) const = 0;
    virtual int notify(void *s, void (*fn)(void *), void *arg) const = 0;
    // the filter (grim_filter_batch) and the workspace it needs
    virtual int filter(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
                       uint32_t *pass_bits, void *ws, uint64_t ws_bytes, void *s) const = 0;
    virtual uint64_t workspace_bytes(const grim_index_t *idx, uint64_t n_pairs) const = 0;
};

// The implementation linked into this binary.
const Backend &backend();

}  // namespace grim_serve
