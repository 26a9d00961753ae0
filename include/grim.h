/*
 * grim.h -- C ABI of the MI355X (gfx950) GRIM-Filter library.
 *
 * GRIM-Filter (Kim et al., "GRIM-Filter: Fast seed location filtering in DNA
 * read mapping using processing-in-memory technologies", BMC Genomics 2018)
 * decides, for every candidate location of a read, whether the location can be
 * discarded before alignment.  The reference is cut into overlapping bins; each
 * bin keeps a 4^q-bit existence vector of the q-grams ("tokens") it contains
 * (Section "Genome Metadata Representation").  For a (read, bin) pair the
 * accumulation sum is the number of the read's L - q + 1 token positions whose
 * bit is set in the bin's vector, and the location passes iff the sum is at
 * least T = (L - q + 1) - q * ceil(e * L) (Sections "GRIM-Filter Operation" and
 * "Taking Errors into Account").  The mapper hands the library a read together
 * with the candidate locations found by its seed lookup and receives one pass
 * bit per location (Section "Integration with a Full Read Mapper").
 *
 * Conventions shared by every entry point:
 *   - Base codes A=0 C=1 G=2 T=3.  Packed sequences hold 16 bases per 32-bit
 *     word, base j of a word in bits [31-2j-1 .. 31-2j] (first base in the two
 *     most significant bits); a base at stream position p lives in word p / 16.
 *   - Token value: the q bases read as a base-4 number, first base most
 *     significant.  Bit t of a bin vector is bit (t & 31) of 32-bit word t >> 5.
 *   - Bin b covers reference positions [b*B, min(G, (b+1)*B + O)); only tokens
 *     lying wholly inside are recorded.  n_bins = ceil(G / B).
 *   - E = ceil(e * L) is computed exactly from e = e_num / e_den.  A read with
 *     L < q has no tokens: its sum is 0 and it passes.
 *   - Pass bit of pair k is bit (k & 31) of pass_bits[k >> 5].
 *   - Every call returns GRIM_OK (0), GRIM_PENDING (> 0) or a negative error
 *     code; no C++ exception crosses the ABI.  Pointers marked "device" must be
 *     device memory of the GPU that is current on the calling thread.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 */
#ifndef GRIM_H
#define GRIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ return codes */
#define GRIM_OK 0
#define GRIM_PENDING 1            /* serving: the request is not finished yet   */
#define GRIM_E_INVALID (-1)       /* bad argument, size or handle               */
#define GRIM_E_BASE (-2)          /* a base outside A/C/G/T (or 0..3)           */
#define GRIM_E_BIN_RANGE (-3)     /* a candidate bin id >= n_bins was seen      */
#define GRIM_E_NOMEM (-4)         /* host or device allocation failed           */
#define GRIM_E_BUDGET (-5)        /* serving: request larger than the budget    */
#define GRIM_E_HIP (-6)           /* a HIP runtime call failed                  */
#define GRIM_E_CANCELLED (-7)     /* serving: the request was cancelled         */
#define GRIM_E_UNSUPPORTED (-8)   /* parameters outside what the kernels cover  */
#define GRIM_E_IO (-9)            /* index file could not be read or written    */
#define GRIM_E_TIMEOUT (-10)      /* serving: wait timed out                    */
#define GRIM_E_READ (-11)         /* a read longer than max_len or outside the  */
                                  /* packed buffer, or inconsistent cand_off    */
#define GRIM_E_SCRATCH (-12)      /* batch too large for the static scratch     */

/* Bits of the device status word that the filter kernels set. */
#define GRIM_FLAG_BIN_RANGE 1u    /* some pair had bin id >= n_bins            */
#define GRIM_FLAG_READ 2u         /* some read was invalid (see GRIM_E_READ)   */
#define GRIM_FLAG_CAND_OFF 4u     /* cand_off was not a valid CSR offset array */

/* Human-readable text of a return code (static storage, never NULL). */
const char *grim_strerror(int code);

/* Library version: major * 10000 + minor * 100 + patch. */
int grim_version(void);

/* ------------------------------------------------------------ host helpers */
/* Number of 32-bit words grim_pack_bases writes for n bases: ceil(n / 16) plus
 * one trailing zero word (kernels may read one word past a token's last base). */
uint64_t grim_packed_words(uint64_t n_bases);

/* Pack n bases (host memory) into the 2-bit layout above.  Accepts codes 0..3
 * and the letters A C G T (either case).  words (host) receives
 * grim_packed_words(n) words.  Any other byte: GRIM_E_BASE, words undefined.
 * n_threads <= 0 uses all host cores. */
int grim_pack_bases(const uint8_t *bases, uint64_t n, uint32_t *words, int n_threads);

/* E = ceil(L * e_num / e_den), exactly (Section "Taking Errors into Account").
 * e_den == 0: GRIM_E_INVALID. */
int grim_max_edits(uint32_t L, uint32_t e_num, uint32_t e_den, uint32_t *E);

/* T = max(0, L - q + 1) - q * E, the accumulation-sum threshold (same section). */
int grim_threshold(uint32_t L, uint32_t q, uint32_t E, int64_t *T);

/* ------------------------------------------------------------------- index */
/* Build kernels (grim_params_t.build).  Both compute the same vectors:
 * GRIM_BUILD_BLOCKS (the token sets of whole blocks of B starts in LDS, one
 * thread per packed word; bins whose whole blocks fit a workgroup's LDS) and
 * GRIM_BUILD_PER_BIN (any geometry: one wavefront per bin). */
#define GRIM_BUILD_AUTO 0u
#define GRIM_BUILD_PER_BIN 1u
#define GRIM_BUILD_BLOCKS 2u

typedef struct grim_params {
    uint32_t q;            /* token length: 4..7 (vectors of 32 B .. 2 KiB)     */
    uint32_t build;        /* GRIM_BUILD_AUTO (BLOCKS where the geometry fits it,
                              else PER_BIN) or one of them                     */
    uint64_t bin_stride;   /* B: bin b starts at b * B                          */
    uint64_t overlap;      /* O: bin b extends O bases past (b+1) * B           */
} grim_params_t;

typedef struct grim_index grim_index_t; /* opaque, immutable once built */

typedef struct grim_index_info {
    uint32_t q;
    int32_t device;           /* HIP device that holds the vectors               */
    uint64_t bin_stride;
    uint64_t overlap;
    uint64_t genome_len;      /* G                                               */
    uint64_t n_bins;
    uint64_t vector_bytes;    /* 4^q / 8                                         */
    uint64_t bytes;           /* n_bins * vector_bytes                           */
    const void *vectors;      /* device: bin b at vectors + b * vector_bytes     */
} grim_index_info_t;

/* Build the bin vectors of a reference (Section "Genome Metadata
 * Representation": scan the genome once and set the bit of every token of
 * every bin).  ref_2bit: host, grim_packed_words(ref_len) words in the packed
 * layout.  The vectors are built on the current device by a HIP kernel on
 * `stream` and stay resident there; the call returns after the build has
 * finished.  The caller owns *out and releases it with grim_index_free.
 * Errors: GRIM_E_INVALID (NULL, ref_len == 0, B == 0, build not one of the
 * GRIM_BUILD_* values, more than 2^32 - 1 bins), GRIM_E_UNSUPPORTED (q outside
 * 4..7, or a forced build kernel that does not fit the geometry),
 * GRIM_E_NOMEM, GRIM_E_HIP. */
int grim_build_bins(const uint32_t *ref_2bit, uint64_t ref_len, const grim_params_t *p,
                    grim_index_t **out, void *stream);

/* Describe an index. */
int grim_index_info(const grim_index_t *idx, grim_index_info_t *out);

/* Copy the vectors to host memory (host must hold info.bytes bytes). */
int grim_index_copy_to_host(const grim_index_t *idx, void *host, uint64_t bytes);

/* Store / reload an index: a 64-byte header (magic "GRIMIDX1", version, q, B,
 * O, G, n_bins, FNV-1a checksum of the vectors) followed by the raw vectors.
 * The paper keeps the bitvectors as genome metadata built once per reference
 * (Section "Genome Metadata Representation").  load: GRIM_E_IO on a short,
 * foreign or corrupt file. */
int grim_index_save(const grim_index_t *idx, const char *path);
int grim_index_load(const char *path, grim_index_t **out, void *stream);

/* Release an index (NULL is ignored).  No filter call may be in flight on it. */
void grim_index_free(grim_index_t *idx);

/* ----------------------------------------------------------------- filtering */
/* A batch of reads and their candidate locations (Section "Integration with a
 * Full Read Mapper": the mapper sends each read with the seed locations its
 * hash table returned).  All pointers are device pointers for grim_filter_*,
 * host pointers for grim_serve_submit. */
#define GRIM_MAX_READ_LEN 8192u   /* longest read any entry point accepts */

typedef struct grim_batch {
    const uint32_t *reads_2bit;   /* packed bases of all reads                     */
    uint64_t n_read_words;        /* words readable at reads_2bit                  */
    const uint64_t *read_off;     /* [n_reads] stream position of each read's base 0 */
    const uint32_t *read_len;     /* [n_reads] L                                   */
    const uint32_t *read_e;       /* [n_reads] error tolerance numerator e_num     */
    uint32_t e_den;               /* tolerance denominator (e.g. 10000), > 0       */
    uint32_t max_len;             /* upper bound on every L, 1..GRIM_MAX_READ_LEN  */
    const uint64_t *cand_off;     /* [n_reads + 1] CSR offsets, cand_off[0] = 0,   */
                                  /* non-decreasing, cand_off[n_reads] = n_pairs   */
    const uint32_t *cand_bin;     /* [n_pairs] candidate bin ids (bin_num(z))      */
    uint64_t n_reads;
    uint64_t n_pairs;
} grim_batch_t;

/* Launch shape of the batched kernel.  Every choice computes identical
 * results; only speed differs.  Zero fields take the default for the index's q. */
typedef struct grim_tuning {
    uint32_t lanes_per_cand;   /* lanes sharing one candidate's vector load       */
    uint32_t unroll;           /* candidates in flight per lane group             */
    uint32_t tile_pairs;       /* pairs per work-list tile (multiple of 64)       */
    uint32_t wg_per_cu;        /* persistent workgroups per compute unit          */
} grim_tuning_t;

/* Fill *out with the default launch shape for token length q. */
int grim_default_tuning(uint32_t q, grim_tuning_t *out);

/* Launch shapes compiled for token length q: writes up to cap (lanes_per_cand,
 * unroll) pairs into out (tile_pairs and wg_per_cu set to the defaults) and
 * the number available into *n.  Use to enumerate or sweep shapes. */
int grim_tuning_candidates(uint32_t q, grim_tuning_t *out, uint32_t cap, uint32_t *n);

/* Device workspace (bytes) grim_filter_batch / grim_filter_plain need for a
 * batch of n_pairs pairs with the given tuning (NULL = default). */
int grim_workspace_size(const grim_index_t *idx, uint64_t n_pairs, const grim_tuning_t *tune,
                        uint64_t *bytes);

/* The filter, batched form: one persistent launch over the whole batch.
 * A work-list kernel cuts the pair space into tiles and records the first read
 * of each tile; the filter kernel's wavefronts pull tiles from an atomic
 * counter.  For each pair it writes counts[k] (int32, the accumulation sum, or
 * -1 for a bin id >= n_bins or an invalid read) and pass bit k (1 iff
 * counts[k] >= T of the pair's read).  counts (device, n_pairs int32) and
 * pass_bits (device, ceil(n_pairs / 32) words) are written in full.  workspace
 * (device, >= grim_workspace_size bytes, 256-byte aligned) is owned by the
 * caller and must not be shared by calls in flight at the same time.  The call
 * is asynchronous on `stream`, allocates nothing and returns once the kernels
 * are queued; problems found on the device are reported by grim_filter_status.
 * Host-side errors: GRIM_E_INVALID, GRIM_E_UNSUPPORTED, GRIM_E_HIP. */
int grim_filter_batch(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
                      uint32_t *pass_bits, void *workspace, uint64_t workspace_bytes,
                      const grim_tuning_t *tune, void *stream);

/* The batched filter for callers that cannot allocate device memory at all:
 * code being captured into a HIP graph, tight serving loops, and harnesses
 * that forbid allocation.  Same computation, outputs and tuning as
 * grim_filter_batch, but no workspace argument: the scratch (tile counter and
 * the tile -> first read table) lives in a file-scope device array of
 * GRIM_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from its first
 * use on a device until the process ends.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine) and is asynchronous on
 * `stream`.
 *   status: device uint32_t owned by the caller; the kernels reset it and set
 *           the GRIM_FLAG_* bits of this call in it (grim_filter_status may be
 *           called with status as its workspace argument).
 * Limit: the scratch holds 256 + 4 * ceil(n_pairs / tile_pairs) bytes; a batch
 * that needs more (about 2.1e9 pairs at tile_pairs 512, 4.3e9 at 1024) gives
 * GRIM_E_SCRATCH before anything is queued.  Every call on one GPU shares that
 * GPU's scratch: calls whose kernels overlap on one GPU (on different streams
 * or threads) race and must not be issued; calls queued one after another on
 * one stream are fine (each resets what must start at zero).
 * Errors: as grim_filter_batch, GRIM_E_INVALID for a NULL status, and
 * GRIM_E_SCRATCH. */
#define GRIM_NOALLOC_SCRATCH_BYTES (16u << 20)
int grim_filter_batch_noalloc(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
                              uint32_t *pass_bits, uint32_t *status, const grim_tuning_t *tune,
                              void *stream);

/* The same filter, plain form: one workgroup per read, no persistence, no
 * tuning, no work list (the straightforward per-read launch the batched form
 * is measured against).  Same arguments, outputs and errors. */
int grim_filter_plain(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
                      uint32_t *pass_bits, void *workspace, uint64_t workspace_bytes,
                      void *stream);

/* Wait for `stream`, then read the status word the last filter call on this
 * workspace left.  *flags (may be NULL) receives the GRIM_FLAG_* bits.
 * Returns GRIM_OK, GRIM_E_BIN_RANGE, GRIM_E_READ or GRIM_E_HIP. */
int grim_filter_status(const void *workspace, void *stream, uint32_t *flags);

/* Pick the fastest launch shape for this index and a representative batch by
 * timing each candidate shape on `stream` over the batch's first 2^26 pairs at
 * most (outputs of those pairs are overwritten).  The
 * result is cached per (device, q, max_len) for later calls with tune = NULL. */
int grim_tune(const grim_index_t *idx, const grim_batch_t *sample, int32_t *counts,
              uint32_t *pass_bits, void *workspace, uint64_t workspace_bytes, void *stream,
              grim_tuning_t *out);

/* ------------------------------------------------------ seed location checker */
/* The Seed Location Checker's first step (Section "Integration with a Full Read
 * Mapper": it reads the seed location filter bitmask and passes on only the
 * locations whose bit is set).  Compacts the pass bits of a filtered batch
 * into the list of surviving locations, in input order:
 *   surv_pair[i] (u64 pair index), surv_read[i] (u32 read), surv_bin[i] (u32 bin)
 * for i < min(total, capacity); *n_survivors (device u64) receives the total,
 * even when it exceeds capacity.  Only b->cand_off, b->cand_bin, b->n_reads and
 * b->n_pairs are used.  Bits past n_pairs in the last word are ignored.
 * workspace: device, >= grim_survivors_workspace_size bytes, 8-byte aligned.
 * Asynchronous on `stream`; allocates nothing. */
int grim_survivors_workspace_size(uint64_t n_pairs, uint64_t *bytes);
int grim_compact_survivors(const grim_batch_t *b, const uint32_t *pass_bits, uint64_t capacity,
                           uint64_t *surv_pair, uint32_t *surv_read, uint32_t *surv_bin,
                           uint64_t *n_survivors, void *workspace, uint64_t workspace_bytes,
                           void *stream);

/* Keep a packed copy of the reference (host ref_2bit, grim_packed_words(ref_len)
 * words; ref_len must equal the index's genome length) on the index's device,
 * as grim_verify_survivors needs it.  Replaces an earlier copy. */
int grim_index_attach_reference(grim_index_t *idx, const uint32_t *ref_2bit, uint64_t ref_len,
                                void *stream);

/* Alignment check of surviving locations -- the step the Seed Location Checker
 * hands the survivors to (Section "Integration with a Full Read Mapper").  For
 * survivor i (read surv_read[i], bin surv_bin[i]): d = the smallest edit
 * distance (unit substitutions, insertions, deletions) between the read and
 * any substring of the bin's span [b*B, min(G, (b+1)*B + O)).  Writes
 * dist[i] = min(d, E + 1) with E = ceil(e * L) of that read, and sets bit i of
 * ok_bits iff d <= E.  dist[i] = -1 (bit clear) for a read or bin id out of
 * range.  Needs grim_index_attach_reference first (else GRIM_E_INVALID) and
 * b->max_len <= 512 (else GRIM_E_UNSUPPORTED).  surv_*, dist (n_survivors
 * int32) and ok_bits (ceil(n_survivors / 32) words) are device memory;
 * asynchronous on `stream`, allocates nothing. */
int grim_verify_survivors(const grim_index_t *idx, const grim_batch_t *b,
                          const uint32_t *surv_read, const uint32_t *surv_bin,
                          uint64_t n_survivors, int32_t *dist, uint32_t *ok_bits, void *stream);

/* --------------------------------------------------------------- bin windows */
/* The paper's bin-window form (Section "Mapping GRIM-Filter to 3D-Stacked
 * Memory with PIM": the mapper sends a read with a range of consecutive bins,
 * and the bitvectors are stored token-major so that one access returns one
 * token's existence bits for many bins; Section "GRIM-Filter Parallelization":
 * a window of consecutive bins is filtered together).
 *
 * grim_index_transpose builds the token-major copy on the index's device (as
 * many bytes again as the vectors): row t holds, for every bin b, bit
 * (b & 31) of word b >> 5 = "token t occurs in bin b".  Synchronous. */
int grim_index_transpose(grim_index_t *idx, void *stream);

/* Filter every bin of each read's window: read r's window is bins
 * [win_lo[r], win_lo[r] + (cand_off[r+1] - cand_off[r])), and pair
 * cand_off[r] + j is bin win_lo[r] + j (b->cand_bin is not used).  Outputs,
 * status and errors as grim_filter_batch (a bin >= n_bins gives -1 and
 * GRIM_FLAG_BIN_RANGE).  win_lo: device u32[n_reads].  order: NULL (reads are
 * processed in index order) or device u32[n_reads], the order in which reads
 * are processed (grim_window_order gives one); outputs do not depend on it.  An
 * entry >= n_reads is skipped and sets GRIM_FLAG_READ (GRIM_E_READ from
 * grim_filter_status); a read named by no entry keeps the previous contents of
 * its counts.  workspace: device, >= 256 bytes, 256-byte aligned.  Needs
 * grim_index_transpose first (else GRIM_E_INVALID); b->max_len <= 4096 (else
 * GRIM_E_UNSUPPORTED).  Asynchronous on `stream`; allocates nothing. */
int grim_filter_windows(const grim_index_t *idx, const grim_batch_t *b, const uint32_t *win_lo,
                        const uint32_t *order, int32_t *counts, uint32_t *pass_bits,
                        void *workspace, uint64_t workspace_bytes, void *stream);

/* Device-side processing order for grim_filter_windows (Section "GRIM-Filter
 * Parallelization": windows of consecutive bins processed together): a
 * permutation of the n_reads reads grouped by the bucket of their window start,
 * buckets in increasing order, where bucket k holds starts in
 * [k * 2^s, (k + 1) * 2^s) with 2^s = 1024 bins, or more for indexes of over
 * 2^26 bins so that there are at most 2^16 buckets; starts >= n_bins come last.
 * Reads with overlapping windows then run close together and share row
 * segments through the cache.  The order of reads within a bucket is
 * unspecified and may differ between calls.  win_lo, order: device
 * u32[n_reads]; workspace: device, grim_window_order_workspace_size(...) bytes
 * (the bucket counts), 4-byte aligned.  GRIM_E_INVALID for NULL pointers, a
 * small workspace or a device other than the index's; GRIM_E_UNSUPPORTED for
 * n_reads >= 2^32.  Asynchronous on `stream`; allocates nothing. */
int grim_window_order_workspace_size(const grim_index_t *idx, uint64_t n_reads, uint64_t *bytes);
int grim_window_order(const grim_index_t *idx, const uint32_t *win_lo, uint64_t n_reads,
                      uint32_t *order, void *workspace, uint64_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------- probes */
/* Diagnostics: the memory ceilings the filter's rate is compared with.  The
 * filter is bound by memory bandwidth (Section "Candidacy for 3D-Stacked Memory
 * Implementations"); these calls measure what the device's memory delivers
 * for the filter's own accesses, without its token work.
 *
 * grim_probe_gather: for every i < n, reads the bin vector of bin ids[i] from
 * the index with the batched filter's gather (ids loaded coalesced, groups of
 * lanes issuing 16-byte loads, several vectors in flight per group) and writes
 * out[i] = its popcount, or -1 for an id >= n_bins (nothing is read then).
 * ids (u32[n]) and out (int32[n]) are device memory.
 *
 * grim_probe_stream: reads the whole index once with 16-byte loads; *sink
 * (device u32) is written only in the unlikely case that keeps the reads from
 * being optimised away.
 *
 * Both: GRIM_E_INVALID for a NULL index or pointer, or when the current device
 * is not the index's; asynchronous on `stream`; allocate nothing. */
int grim_probe_gather(const grim_index_t *idx, const uint32_t *ids, uint64_t n, int32_t *out,
                      void *stream);
int grim_probe_stream(const grim_index_t *idx, uint32_t *sink, void *stream);

/* ------------------------------------------------------------------- seeding */
/* The step before the filter: the mapper looks up exact seeds of each read in a
 * hash table of reference locations and sends the locations to GRIM-Filter
 * (Section "Introduction", Fig. 1; Section "Integration with a Full Read
 * Mapper").  Here the table is a k-mer position index built on the GPU. */
typedef struct grim_seed_index grim_seed_index_t;  /* opaque, device-resident */
typedef struct grim_candidates grim_candidates_t;  /* opaque, device-resident */

/* Index every k-mer (4 <= k <= 15) of a reference of ref_len <= 2^32 - 1 bases
 * (host ref_2bit, grim_packed_words(ref_len) words).  Synchronous; the index
 * (4^k + 1 u64 offsets and ref_len - k + 1 u32 positions) stays on the current
 * device until grim_seed_index_free. */
int grim_seed_index_build(const uint32_t *ref_2bit, uint64_t ref_len, uint32_t k,
                          grim_seed_index_t **out, void *stream);
void grim_seed_index_free(grim_seed_index_t *si);

/* Candidate bins of a batch of reads (uses reads_2bit, n_read_words, read_off,
 * read_len, n_reads of *reads; device memory): seeds are each read's k-mers at
 * offsets 0, k, 2k, ... while the seed fits; every occurrence p of the seed at
 * offset o proposes location z = p - o clamped into [0, G - 1] and bin
 * z / bin_stride; a read's bins are deduplicated, sorted increasingly and cut
 * to the first `cap`.  Reads outside the packed buffer, and reads longer than
 * reads->max_len when it is not 0, get no candidates.  Calls on one seed index
 * take turns (the index keeps its device temporaries between calls).
 * Synchronous; the result (CSR offsets n_reads + 1 u64, bins u32) is device
 * memory, a buffer kept from a freed list of this index when one fits, else
 * allocated.  GRIM_E_UNSUPPORTED beyond 2^31 - 1 seed hits or reads. */
int grim_seed_candidates(const grim_seed_index_t *si, const grim_batch_t *reads,
                         uint64_t bin_stride, uint32_t cap, grim_candidates_t **out, void *stream);

/* Sizes and device pointers of a candidate list (any output may be NULL). */
int grim_candidates_info(const grim_candidates_t *c, uint64_t *n_reads, uint64_t *n_pairs,
                         const uint64_t **cand_off, const uint32_t **cand_bin);
/* Copy a candidate list to host memory (cand_off: n_reads + 1, cand_bin: n_pairs). */
int grim_candidates_copy_to_host(const grim_candidates_t *c, uint64_t *cand_off,
                                 uint32_t *cand_bin);
/* Free a candidate list: waits for the device's queued work (as hipFree
 * does), then keeps its buffer for later lists of the same seed index (at most
 * two buffers per index are kept, until the index and every list made from
 * it have been freed). */
void grim_candidates_free(grim_candidates_t *c);

/* ---------------------------------------------------------------- HIP graphs */
/* Capture the work-list and filter kernels of one grim_filter_batch call (same
 * arguments, fixed buffers) into a HIP graph; replay it with grim_graph_launch
 * on any stream.  The graph holds no memset nodes. */
typedef struct grim_graph grim_graph_t;
int grim_graph_create(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
                      uint32_t *pass_bits, void *workspace, uint64_t workspace_bytes,
                      const grim_tuning_t *tune, grim_graph_t **out);
int grim_graph_launch(grim_graph_t *g, void *stream);
void grim_graph_destroy(grim_graph_t *g);

/* ------------------------------------------------------------------ serving */
/* A continuous-batching server over one resident index.  Requests (host
 * batches) are copied at submit time (or used in place); an admission thread
 * admits queued requests while their device bytes fit in the HBM budget and a
 * slot is free, fuses the admitted requests of one tick into a single batched
 * launch, and keeps admitting new requests while earlier ticks run.  Up to
 * n_streams x ticks_per_stream ticks are in flight, each in a slot with a
 * worker thread that stages it, queues its copies, filter and result copies on
 * the slot's stream and retires it; ticks on different streams overlap on the
 * device, and a stream's next tick waits queued behind its current one.  When
 * results include counts, ticks take turns to queue their input copies (a turn
 * ends when the tick's inputs are on the device; a tick takes a turn only once
 * the ticks before it on its stream have completed), so that uploads run one
 * at a time and the ticks' downloads are staggered against them.  A
 * request with more pairs than max_tick_pairs is cut at read boundaries into
 * parts that run as separate ticks, so that its copies and launches overlap
 * across streams.  Results are bit-identical to filtering each request alone.
 * Mirrors the overlap of filtering with the mapper's alignment through a
 * bitmask buffer (Sections "Mapping GRIM-Filter to 3D-Stacked Memory with PIM"
 * and "GRIM-Filter Parallelization"). */
typedef struct grim_server grim_server_t;

/* Server option: a request's results are its pass bits alone (the seed
 * location filter bitmask of Section "Integration with a Full Read Mapper");
 * its counts stay on the device, so each pair moves 1/8 byte back over the
 * host link instead of 4 1/8 bytes, and the counts buffers of
 * grim_serve_submit_inplace, grim_serve_poll and grim_serve_wait may be NULL
 * (they are left untouched).  A request with an out-of-range bin id still
 * fails alone with GRIM_E_BIN_RANGE: only a tick whose status word flags one
 * copies its counts back to find it. */
#define GRIM_SERVE_PASS_BITS_ONLY 1u

/* Server options: how results come back to host memory.  By default the
 * server probes its streams at creation; when they all share one copy engine
 * (so that an upload and a download cannot overlap) and results include
 * counts, a small kernel stores the results straight into the page-locked host
 * buffers instead of a copy-engine download, and otherwise the copy engine
 * moves them.  These flags fix the choice: GRIM_SERVE_STORE_DOWNLOADS always
 * stores from the kernel (except into pageable in-place result buffers, which
 * the device cannot write: those still come back by the copy engine),
 * GRIM_SERVE_ENGINE_DOWNLOADS always uses the copy engine.  Setting both is
 * GRIM_E_INVALID.  Results are the same bytes either way. */
#define GRIM_SERVE_STORE_DOWNLOADS 2u
#define GRIM_SERVE_ENGINE_DOWNLOADS 4u

typedef struct grim_serve_cfg {
    uint64_t hbm_budget_bytes;  /* device bytes for request buffers (0 = 1 GiB)     */
    uint32_t max_inflight;      /* requests on the device at once (0 = 1024)        */
    uint32_t n_streams;         /* concurrent ticks (0 = 3)                         */
    uint32_t max_tick_pairs;    /* pairs per launch; larger requests run in parts
                                   of whole reads (0 = 8M)                          */
    uint32_t max_len;           /* longest read accepted (0 = 1024)                 */
    uint32_t flags;             /* GRIM_SERVE_* options (0: counts and pass bits)   */
    uint32_t ticks_per_stream;  /* ticks queued on one stream at once: the next one
                                   waits behind the current one (0 = 2; at most 4) */
} grim_serve_cfg_t;

typedef struct grim_req_stats {
    double queue_ms;       /* submit -> admitted                                    */
    double latency_ms;     /* submit -> results in host memory                      */
    uint64_t n_pairs;
    uint64_t tick;         /* the fused launch that carried the request (its last
                              part, for a request run in parts)                     */
    uint32_t flags;        /* GRIM_FLAG_* bits seen in this request's pairs         */
    int32_t status;        /* GRIM_OK, GRIM_E_BIN_RANGE, GRIM_E_READ, GRIM_E_CANCELLED */
} grim_req_stats_t;

typedef struct grim_serve_stats {
    uint64_t submitted, completed, cancelled, failed, ticks;
    uint64_t pairs_done;
    double p50_ms, p99_ms, mean_ms, max_ms;  /* latency of completed requests      */
    double busy_s;            /* wall time with at least one tick on the device     */
    double pairs_per_s;       /* pairs_done / busy_s                                */
    uint64_t peak_device_bytes;
    double mean_requests_per_tick;
    double sched_launch_s;    /* worker time staging and queueing ticks (all workers,
                                 waits for upload turns excluded)                     */
    double sched_retire_s;    /* worker time handing results back (all workers)         */
    double sched_admit_s;     /* admission thread time forming ticks                    */
    uint32_t stream_groups;   /* copy-engine groups the streams were split between (1, 2) */
} grim_serve_stats_t;

/* Create a server on the current device.  It allocates its device pool
 * (hbm_budget_bytes) and streams here, never on the request path. */
int grim_serve_create(const grim_index_t *idx, const grim_serve_cfg_t *cfg, grim_server_t **out);

/* Queue a request.  b holds HOST pointers; the arrays are copied before the call
 * returns.  *ticket identifies the request.  Errors: GRIM_E_INVALID,
 * GRIM_E_BUDGET (the request alone exceeds the budget), GRIM_E_NOMEM. */
int grim_serve_submit(grim_server_t *s, const grim_batch_t *b, uint64_t *ticket);

/* Queue a request without copying it: the server reads the caller's host
 * arrays (b) in place and writes the results straight into counts
 * (n_pairs int32) and pass_bits (ceil(n_pairs / 32) words), both host memory
 * owned by the caller.  Every one of these buffers must stay alive and
 * unchanged until grim_serve_poll / grim_serve_wait reports the request done
 * (or it is cancelled and reported).  Buffers from hipHostMalloc are moved by
 * direct DMA; pageable memory works but is staged by the runtime.  Same
 * validation and errors as grim_serve_submit. */
int grim_serve_submit_inplace(grim_server_t *s, const grim_batch_t *b, int32_t *counts,
                              uint32_t *pass_bits, uint64_t *ticket);

/* Non-blocking: GRIM_PENDING while the request runs; otherwise copies the
 * results (host counts[n_pairs], pass_bits[ceil(n_pairs/32)]; either may be
 * NULL), fills *st (may be NULL), forgets the ticket and returns the request's
 * status.  Unknown ticket: GRIM_E_INVALID. */
int grim_serve_poll(grim_server_t *s, uint64_t ticket, int32_t *counts, uint32_t *pass_bits,
                    grim_req_stats_t *st);

/* Blocking form of grim_serve_poll; timeout_ms < 0 waits forever.  Returns
 * GRIM_E_TIMEOUT if the request is still running at the deadline. */
int grim_serve_wait(grim_server_t *s, uint64_t ticket, int64_t timeout_ms, int32_t *counts,
                    uint32_t *pass_bits, grim_req_stats_t *st);

/* Cancel a request: a queued request never runs; a running one has its results
 * dropped (parts not yet admitted never run).  Its poll/wait then returns
 * GRIM_E_CANCELLED. */
int grim_serve_cancel(grim_server_t *s, uint64_t ticket);

/* Aggregate statistics since creation (or the last reset). */
int grim_serve_stats(grim_server_t *s, grim_serve_stats_t *out, int reset);

/* Stop the scheduler (queued requests are cancelled, running ones finish) and
 * free the server.  NULL is ignored. */
void grim_serve_destroy(grim_server_t *s);

#ifdef __cplusplus
}
#endif

#endif /* GRIM_H */
