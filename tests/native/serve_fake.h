// A host-memory stand-in for the device behind the serving scheduler, used to
// run grim_serve.cpp on the CPU under ThreadSanitizer (tests/native/
// serve_fake_backend.cpp implements grim_serve::backend() with it).
//
// "Device" memory is host memory; each stream is a worker thread that runs its
// queued operations in order; the filter is a stand-in function of each pair
// (the read's bases, its length and tolerance, the bin id), so that a request's
// results depend on every field the scheduler re-bases when it fuses, splits
// and copies requests, and can be recomputed from the request alone.
#pragma once

#include <stdint.h>

#include "grim.h"

// An index handle the fake backend accepts (n_bins bins on device `device`).
grim_index_t *fake_index(uint64_t n_bins, int device);
void fake_index_free(grim_index_t *idx);

// The stand-in filter over a batch in host memory: counts[n_pairs],
// pass bits (ceil(n_pairs / 32) words, written in full) and the
// GRIM_FLAG_BIN_RANGE flag for ids >= n_bins (count -1, pass 0).
void fake_filter_host(const grim_batch_t *b, uint64_t n_bins, int32_t *counts, uint32_t *bits,
                      uint32_t *flags);

// Failure injection: with every > 0, every every-th filter launch (counted
// from the call) is refused with GRIM_E_HIP, as a failed kernel launch would be.
void fake_fail_filter_every(uint64_t every);
uint64_t fake_filter_calls(void);
uint64_t fake_filter_failures(void);
// Device bytes currently allocated through the backend (pool and nothing else).
int64_t fake_device_bytes(void);
// Host ranges the "device" cannot reach (pageable memory): device_writable is
// false for them.
void fake_mark_pageable(const void *p, uint64_t bytes);
void fake_clear_pageable(void);
bool fake_pageable(const void *p);
