// Internal declarations shared by the GRIM-Filter kernels, the C ABI and the
// serving runtime.  Not installed; the public interface is include/grim.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grim.h"

namespace grim {

constexpr int kWave = 64;
constexpr uint32_t kMaxLen = GRIM_MAX_READ_LEN;  // longest read the kernels accept
constexpr uint64_t kWsHeader = 256;      // status word + tile counter, padded

// Arguments of both filter kernels (passed by value).
struct FilterArgs {
    const uint4 *vec;           // bin vectors, 4^q / 8 bytes each
    uint64_t n_bins;
    const uint32_t *rw;         // packed reads
    uint64_t nw;                // words readable at rw
    const uint64_t *read_off;
    const uint32_t *read_len;
    const uint32_t *read_e;
    uint32_t e_den;
    uint32_t max_len;
    const uint64_t *cand_off;
    const uint32_t *cand_bin;
    uint64_t n_reads;
    uint64_t n_pairs;
    int32_t *counts;
    uint32_t *pass_bits;
    uint32_t *status;
    uint32_t *tile_counter;
    const uint32_t *tile_read;
    uint32_t n_tiles;
    uint32_t tile_pairs;
    int npl;                    // multiplicity planes reserved per read
};

// Zero words kept after the packed reference for the alignment check, whose
// look-ahead fetches of reference words run up to three words past the end.
constexpr uint64_t kRefPadWords = 4;

// Arguments of the alignment-check kernel.
struct VerifyArgs {
    const uint32_t *ref;        // packed reference, kRefPadWords zero words after its end
    uint64_t ref_words;
    uint64_t G, B, O, n_bins;
    const uint32_t *rw;
    uint64_t nw;
    const uint64_t *read_off;
    const uint32_t *read_len;
    const uint32_t *read_e;
    uint32_t e_den;
    uint64_t n_reads;
    const uint32_t *surv_read;
    const uint32_t *surv_bin;
    uint64_t n_surv;
    int32_t *dist;
    uint32_t *ok_bits;
};

// Arguments of the bin-window kernel.
struct WindowArgs {
    const uint32_t *rows;       // token-major index: row t, word w = bins [32w, 32w+32)
    uint64_t row_words;
    uint64_t rows_bytes;        // readable bytes of the row buffer (rows and pad)
    uint64_t n_bins;
    const uint32_t *rw;
    uint64_t nw;
    const uint64_t *read_off;
    const uint32_t *read_len;
    const uint32_t *read_e;
    uint32_t e_den;
    uint32_t max_len;
    const uint64_t *cand_off;   // window sizes
    const uint32_t *win_lo;     // first bin of each read's window
    const uint32_t *order;      // processing order (slot -> read), or null for index order
    uint64_t n_reads, n_pairs;
    int32_t *counts;
    uint32_t *pass_bits;
    uint32_t *status;
    uint32_t *counter;
    int npl;
};

struct BatchedVariant {
    int q, g, u;
    const void *kernel;
};

const BatchedVariant *batched_variants(int *n);
const void *plain_kernel(int q);

hipError_t launch_build(int q, dim3 grid, hipStream_t s, const uint32_t *ref, uint64_t nw,
                        uint64_t G, uint64_t B, uint64_t O, uint64_t n_bins, uint32_t *out);
hipError_t launch_build_chunked(int q, uint32_t cus, hipStream_t s, const uint32_t *ref,
                                uint64_t nw, uint64_t G, uint64_t B, uint64_t O, uint64_t n_bins,
                                uint32_t *out);
hipError_t launch_worklist(hipStream_t s, const uint64_t *cand_off, uint64_t n_reads,
                           uint32_t tile_pairs, uint32_t n_tiles, uint32_t *tile_read,
                           uint32_t *status, uint32_t *counter);
hipError_t launch_zero(hipStream_t s, uint32_t *p, uint64_t n);
hipError_t launch_compact(hipStream_t s, const uint32_t *bits, uint64_t n_pairs,
                          const uint64_t *cand_off, uint64_t n_reads, const uint32_t *cand_bin,
                          uint64_t cap, uint64_t *surv_pair, uint32_t *surv_read,
                          uint32_t *surv_bin, uint64_t *n_out, uint64_t *block_sums);
uint64_t compact_blocks(uint64_t n_pairs);
hipError_t launch_verify(hipStream_t s, int W, int cus, const VerifyArgs &a);
hipError_t launch_transpose(hipStream_t s, int q, const uint32_t *vec, uint64_t n_bins,
                            uint64_t row_words, uint32_t *rows, uint32_t grid);
// Persistent grid: as many workgroups as fit on the device's cus compute units
// at once (at most one per read).
hipError_t launch_window(hipStream_t s, int q, uint32_t cus, size_t lds, const WindowArgs &a);
// Processing order for the window kernel: reads grouped by window-start bucket
// (bins [k << shift, (k + 1) << shift) form bucket k; starts >= n_bins the last
// of the n_buckets).  cnt: n_buckets words, zeroed by the caller.
uint32_t order_shift(uint64_t n_bins, uint32_t *n_buckets);
hipError_t launch_window_order(hipStream_t s, uint32_t cus, const uint32_t *win_lo, uint32_t n,
                               uint64_t n_bins, uint32_t shift, uint32_t n_buckets, uint32_t *cnt,
                               uint32_t *order);

// Memory-ceiling probes (grim_probe.hip): the batched filter's gather of bin
// vectors without its token work, and a streaming read.
hipError_t launch_probe_gather(hipStream_t s, uint32_t q, uint32_t grid, const void *vec,
                               uint64_t n_records, const uint32_t *ids, uint64_t n, int32_t *out);
hipError_t launch_probe_stream(hipStream_t s, uint32_t grid, const void *src, uint64_t n16,
                               uint32_t *sink);
hipError_t launch_filter(const void *kernel, dim3 grid, dim3 block, size_t lds_bytes,
                         hipStream_t s, const FilterArgs &a);
// Device-to-host copy by a kernel storing into page-locked host memory (dst
// must be memory the device can write; grim_copy.hip).
hipError_t launch_copy_to_host(hipStream_t s, void *dst, const void *src, uint64_t bytes);

}  // namespace grim

// The index object behind the opaque grim_index_t handle.
struct grim_index {
    uint32_t q;
    int device;
    uint64_t B, O, G, n_bins, vector_bytes, bytes;
    void *d_vec;
    uint32_t *d_ref;        // packed reference kept for alignment checks (or null),
                            // followed by kRefPadWords zero words
    uint64_t ref_words;
    uint32_t *d_rows;       // token-major copy for the bin-window form (or null)
    uint64_t row_words;
};
