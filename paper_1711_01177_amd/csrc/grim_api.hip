// C ABI of the GRIM-Filter library: index build and storage, the batched and
// plain filter launches, status, autotuning and HIP-graph capture.  Kernels
// live in grim_kernels.hip; the serving runtime in grim_serve.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "grim_internal.h"

using namespace grim;

namespace {

thread_local char g_hip_msg[256] = "";

int hip_fail(hipError_t e, const char *what)
{
    std::snprintf(g_hip_msg, sizeof(g_hip_msg), "%s: %s", what, hipGetErrorString(e));
    return GRIM_E_HIP;
}

#define HIP_TRY(x)                                  \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess)                       \
            return hip_fail(e_, #x);                \
    } while (0)

int current_device(int *dev)
{
    hipError_t e = hipGetDevice(dev);
    return e == hipSuccess ? GRIM_OK : hip_fail(e, "hipGetDevice");
}

int cu_count(int dev)
{
    static std::mutex mu;
    static std::map<int, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end())
        return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        n = 256;
    cache[dev] = n;
    return n;
}

uint64_t vector_words(uint32_t q) { return (1ull << (2 * q)) >> 5; }

// Multiplicity planes needed so that no token count of a read of up to max_len
// bases overflows: bit length of the largest token count.
int planes_for(uint32_t q, uint32_t max_len)
{
    uint32_t ntok = max_len >= q ? max_len - q + 1 : 1;
    int n = 0;
    while (ntok) {
        ++n;
        ntok >>= 1;
    }
    return n;
}

const BatchedVariant *find_variant(uint32_t q, uint32_t g, uint32_t u)
{
    int n = 0;
    const BatchedVariant *v = batched_variants(&n);
    for (int i = 0; i < n; ++i)
        if ((uint32_t)v[i].q == q && (uint32_t)v[i].g == g && (uint32_t)v[i].u == u)
            return &v[i];
    return nullptr;
}

std::mutex g_tune_mu;
std::map<std::tuple<int, uint32_t, uint32_t>, grim_tuning_t> g_tune_cache;

int resolve_tuning(const grim_index_t *idx, uint32_t max_len, const grim_tuning_t *tune,
                   grim_tuning_t *out)
{
    grim_tuning_t t;
    grim_default_tuning(idx->q, &t);
    if (!tune) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find({idx->device, idx->q, max_len});
        if (it != g_tune_cache.end())
            t = it->second;
    } else {
        if (tune->lanes_per_cand)
            t.lanes_per_cand = tune->lanes_per_cand;
        if (tune->unroll)
            t.unroll = tune->unroll;
        if (tune->tile_pairs)
            t.tile_pairs = tune->tile_pairs;
        if (tune->wg_per_cu)
            t.wg_per_cu = tune->wg_per_cu;
    }
    if (t.tile_pairs < 64 || t.tile_pairs > 4096 || t.tile_pairs % 64 != 0)
        return GRIM_E_INVALID;
    if (t.wg_per_cu < 1 || t.wg_per_cu > 32)
        return GRIM_E_INVALID;
    if (!find_variant(idx->q, t.lanes_per_cand, t.unroll))
        return GRIM_E_UNSUPPORTED;
    *out = t;
    return GRIM_OK;
}

int check_batch(const grim_index_t *idx, const grim_batch_t *b)
{
    if (!idx || !b)
        return GRIM_E_INVALID;
    if (b->e_den == 0 || b->max_len == 0 || b->max_len > kMaxLen)
        return GRIM_E_INVALID;
    if (b->n_reads >= 0xffffffffull)
        return GRIM_E_INVALID;
    if (b->n_reads == 0 && b->n_pairs != 0)
        return GRIM_E_INVALID;
    if (b->n_reads && (!b->read_off || !b->read_len || !b->read_e || !b->cand_off))
        return GRIM_E_INVALID;
    if (b->n_reads && (!b->reads_2bit || b->n_read_words == 0))
        return GRIM_E_INVALID;
    if (b->n_pairs && !b->cand_bin)
        return GRIM_E_INVALID;
    if (b->n_pairs > (0xffffffffull - 1) * 4096ull)
        return GRIM_E_INVALID;
    int dev = -1;
    int rc = current_device(&dev);
    if (rc)
        return rc;
    if (dev != idx->device)
        return GRIM_E_INVALID;
    return GRIM_OK;
}

FilterArgs make_args(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
                     uint32_t *pass_bits, void *ws)
{
    FilterArgs a;
    std::memset(&a, 0, sizeof(a));
    a.vec = reinterpret_cast<const uint4 *>(idx->d_vec);
    a.n_bins = idx->n_bins;
    a.rw = b->reads_2bit;
    a.nw = b->n_read_words;
    a.read_off = b->read_off;
    a.read_len = b->read_len;
    a.read_e = b->read_e;
    a.e_den = b->e_den;
    a.max_len = b->max_len;
    a.cand_off = b->cand_off;
    a.cand_bin = b->cand_bin;
    a.n_reads = b->n_reads;
    a.n_pairs = b->n_pairs;
    a.counts = counts;
    a.pass_bits = pass_bits;
    a.status = reinterpret_cast<uint32_t *>(ws);
    a.tile_counter = reinterpret_cast<uint32_t *>(ws) + 1;
    a.tile_read = reinterpret_cast<const uint32_t *>(reinterpret_cast<char *>(ws) + kWsHeader);
    a.npl = planes_for(idx->q, b->max_len);
    return a;
}

uint64_t ws_bytes_for(uint64_t n_pairs, uint32_t tile_pairs)
{
    const uint64_t n_tiles = (n_pairs + tile_pairs - 1) / tile_pairs;
    return (kWsHeader + 4 * n_tiles + 255) & ~255ull;
}

// Queue the work-list and batched filter kernels on `s`.
// status (may be null) replaces the workspace's status word as the word the
// kernels reset and flag.
int enqueue_batched(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
                    uint32_t *pass_bits, void *ws, uint64_t ws_bytes, const grim_tuning_t &t,
                    hipStream_t s, uint32_t *status = nullptr)
{
    const uint64_t need = ws_bytes_for(b->n_pairs, t.tile_pairs);
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
        return GRIM_E_INVALID;
    if (b->n_pairs && (!counts || !pass_bits))
        return GRIM_E_INVALID;
    FilterArgs a = make_args(idx, b, counts, pass_bits, ws);
    if (status)
        a.status = status;
    const uint64_t n_tiles = (b->n_pairs + t.tile_pairs - 1) / t.tile_pairs;
    if (n_tiles >= (1ull << 32) - (1ull << 24))  // the 32-bit tile counter must not wrap
        return GRIM_E_UNSUPPORTED;
    a.n_tiles = (uint32_t)n_tiles;
    a.tile_pairs = t.tile_pairs;
    HIP_TRY(launch_worklist(s, b->cand_off, b->n_reads, t.tile_pairs, (uint32_t)n_tiles,
                            reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(ws) + kWsHeader),
                            a.status, a.tile_counter));
    if (n_tiles == 0)
        return GRIM_OK;
    const BatchedVariant *v = find_variant(idx->q, t.lanes_per_cand, t.unroll);
    // planes, then the tile's pass-bit words rounded up to 16-byte units (the
    // kernel lays each wave's LDS region out the same way)
    const size_t per_wave =
        ((size_t)a.npl * vector_words(idx->q) + ((t.tile_pairs / 32 + 3) & ~3u)) * 4;
    int waves = 4;
    while (waves > 1 && per_wave * waves > 65536)
        --waves;
    if (per_wave > 65536)
        return GRIM_E_UNSUPPORTED;
    uint64_t grid = (uint64_t)cu_count(idx->device) * t.wg_per_cu;
    const uint64_t useful = (n_tiles + waves - 1) / waves;
    if (grid > useful)
        grid = useful;
    HIP_TRY(launch_filter(v->kernel, dim3((uint32_t)grid), dim3(64 * waves), per_wave * waves, s, a));
    return GRIM_OK;
}

}  // namespace

// --------------------------------------------------------------- basics
extern "C" const char *grim_strerror(int code)
{
    switch (code) {
    case GRIM_OK: return "ok";
    case GRIM_PENDING: return "pending";
    case GRIM_E_INVALID: return "invalid argument";
    case GRIM_E_BASE: return "base outside A/C/G/T";
    case GRIM_E_BIN_RANGE: return "candidate bin id out of range";
    case GRIM_E_NOMEM: return "out of memory";
    case GRIM_E_BUDGET: return "request exceeds the device memory budget";
    case GRIM_E_HIP: return g_hip_msg[0] ? g_hip_msg : "HIP runtime error";
    case GRIM_E_CANCELLED: return "cancelled";
    case GRIM_E_UNSUPPORTED: return "unsupported parameters";
    case GRIM_E_IO: return "index file error";
    case GRIM_E_TIMEOUT: return "timed out";
    case GRIM_E_READ: return "invalid read or candidate offsets";
    case GRIM_E_SCRATCH:
        return "batch needs more than the static scratch holds (use grim_filter_batch with a "
               "workspace)";
    default: return "unknown error";
    }
}

extern "C" int grim_version(void) { return 10000; }

// ---------------------------------------------------------------- index
extern "C" int grim_build_bins(const uint32_t *ref_2bit, uint64_t ref_len, const grim_params_t *p,
                               grim_index_t **out, void *stream)
{
    if (!ref_2bit || !p || !out || ref_len == 0 || p->bin_stride == 0 || p->build > GRIM_BUILD_BLOCKS)
        return GRIM_E_INVALID;
    if (p->q < 4 || p->q > 7)
        return GRIM_E_UNSUPPORTED;
    const uint64_t n_bins = (ref_len + p->bin_stride - 1) / p->bin_stride;
    if (n_bins > 0xffffffffull)
        return GRIM_E_INVALID;
    int dev = 0;
    int rc = current_device(&dev);
    if (rc)
        return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint64_t vb = vector_words(p->q) * 4;
    const uint64_t nw = grim_packed_words(ref_len);
    grim_index *idx = new (std::nothrow) grim_index();
    if (!idx)
        return GRIM_E_NOMEM;
    idx->d_ref = nullptr;
    idx->ref_words = 0;
    idx->d_rows = nullptr;
    idx->row_words = 0;
    idx->q = p->q;
    idx->device = dev;
    idx->B = p->bin_stride;
    idx->O = p->overlap;
    idx->G = ref_len;
    idx->n_bins = n_bins;
    idx->vector_bytes = vb;
    idx->bytes = n_bins * vb;
    if (hipMalloc(&idx->d_vec, idx->bytes) != hipSuccess) {
        delete idx;
        return GRIM_E_NOMEM;
    }
    uint32_t *d_ref = nullptr;
    if (hipMalloc(&d_ref, nw * 4) != hipSuccess) {
        (void)hipFree(idx->d_vec);
        delete idx;
        return GRIM_E_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(d_ref, ref_2bit, nw * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        // the first kernel that fits the geometry, or the one asked for
        uint32_t *vec = reinterpret_cast<uint32_t *>(idx->d_vec);
        const uint32_t cus = (uint32_t)cu_count(dev);
        const uint32_t want = p->build;
        e = hipErrorNotSupported;
        if (want == GRIM_BUILD_AUTO || want == GRIM_BUILD_BLOCKS)
            e = launch_build_chunked(p->q, cus, s, d_ref, nw, ref_len, p->bin_stride, p->overlap,
                                     n_bins, vec);
        if (e == hipErrorNotSupported && (want == GRIM_BUILD_AUTO || want == GRIM_BUILD_PER_BIN)) {
            uint64_t grid = (n_bins + 3) / 4;
            const uint64_t cap = (uint64_t)cus * 32;
            if (grid > cap)
                grid = cap;
            e = launch_build(p->q, dim3((uint32_t)grid), s, d_ref, nw, ref_len, p->bin_stride,
                             p->overlap, n_bins, vec);
        }
        if (e == hipErrorNotSupported) {  // only a forced kernel gets here
            (void)hipFree(d_ref);
            (void)hipFree(idx->d_vec);
            delete idx;
            return GRIM_E_UNSUPPORTED;
        }
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    (void)hipFree(d_ref);
    if (e != hipSuccess) {
        (void)hipFree(idx->d_vec);
        delete idx;
        return hip_fail(e, "grim_build_bins");
    }
    *out = idx;
    return GRIM_OK;
}

extern "C" int grim_index_info(const grim_index_t *idx, grim_index_info_t *out)
{
    if (!idx || !out)
        return GRIM_E_INVALID;
    out->q = idx->q;
    out->device = idx->device;
    out->bin_stride = idx->B;
    out->overlap = idx->O;
    out->genome_len = idx->G;
    out->n_bins = idx->n_bins;
    out->vector_bytes = idx->vector_bytes;
    out->bytes = idx->bytes;
    out->vectors = idx->d_vec;
    return GRIM_OK;
}

extern "C" int grim_index_copy_to_host(const grim_index_t *idx, void *host, uint64_t bytes)
{
    if (!idx || !host || bytes < idx->bytes)
        return GRIM_E_INVALID;
    HIP_TRY(hipMemcpy(host, idx->d_vec, idx->bytes, hipMemcpyDeviceToHost));
    return GRIM_OK;
}

namespace {
struct IndexFileHeader {
    char magic[8];
    uint32_t version, q;
    uint64_t B, O, G, n_bins, checksum;
    uint64_t reserved;
};
static_assert(sizeof(IndexFileHeader) == 64, "header must be 64 bytes");

uint64_t fnv1a(const uint8_t *p, uint64_t n, uint64_t h = 1469598103934665603ull)
{
    for (uint64_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}
}  // namespace

extern "C" int grim_index_save(const grim_index_t *idx, const char *path)
{
    if (!idx || !path)
        return GRIM_E_INVALID;
    std::vector<uint8_t> host;
    try {
        host.resize(idx->bytes);
    } catch (...) {
        return GRIM_E_NOMEM;
    }
    int rc = grim_index_copy_to_host(idx, host.data(), host.size());
    if (rc)
        return rc;
    IndexFileHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, "GRIMIDX1", 8);
    h.version = 1;
    h.q = idx->q;
    h.B = idx->B;
    h.O = idx->O;
    h.G = idx->G;
    h.n_bins = idx->n_bins;
    h.checksum = fnv1a(host.data(), host.size());
    FILE *f = std::fopen(path, "wb");
    if (!f)
        return GRIM_E_IO;
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 &&
              std::fwrite(host.data(), 1, host.size(), f) == host.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? GRIM_OK : GRIM_E_IO;
}

extern "C" int grim_index_load(const char *path, grim_index_t **out, void *stream)
{
    if (!path || !out)
        return GRIM_E_INVALID;
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return GRIM_E_IO;
    IndexFileHeader h;
    if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, "GRIMIDX1", 8) != 0 ||
        h.version != 1 || h.q < 4 || h.q > 7 || h.B == 0 ||
        h.n_bins != (h.G + h.B - 1) / h.B) {
        std::fclose(f);
        return GRIM_E_IO;
    }
    const uint64_t vb = vector_words(h.q) * 4;
    std::vector<uint8_t> host;
    try {
        host.resize(h.n_bins * vb);
    } catch (...) {
        std::fclose(f);
        return GRIM_E_NOMEM;
    }
    const bool ok = std::fread(host.data(), 1, host.size(), f) == host.size();
    std::fclose(f);
    if (!ok || fnv1a(host.data(), host.size()) != h.checksum)
        return GRIM_E_IO;
    int dev = 0;
    int rc = current_device(&dev);
    if (rc)
        return rc;
    grim_index *idx = new (std::nothrow) grim_index();
    if (!idx)
        return GRIM_E_NOMEM;
    idx->d_ref = nullptr;
    idx->ref_words = 0;
    idx->d_rows = nullptr;
    idx->row_words = 0;
    idx->q = h.q;
    idx->device = dev;
    idx->B = h.B;
    idx->O = h.O;
    idx->G = h.G;
    idx->n_bins = h.n_bins;
    idx->vector_bytes = vb;
    idx->bytes = host.size();
    if (hipMalloc(&idx->d_vec, idx->bytes) != hipSuccess) {
        delete idx;
        return GRIM_E_NOMEM;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(idx->d_vec, host.data(), idx->bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(idx->d_vec);
        delete idx;
        return hip_fail(e, "grim_index_load");
    }
    *out = idx;
    return GRIM_OK;
}

extern "C" void grim_index_free(grim_index_t *idx)
{
    if (!idx)
        return;
    if (idx->d_ref)
        (void)hipFree(idx->d_ref);
    if (idx->d_rows)
        (void)hipFree(idx->d_rows);
    (void)hipFree(idx->d_vec);
    delete idx;
}

// ------------------------------------------------------------ filtering
extern "C" int grim_default_tuning(uint32_t q, grim_tuning_t *out)
{
    if (!out)
        return GRIM_E_INVALID;
    // the shapes the autotuner picks on the 3.1 Gbp workloads (q = 5: 8.3e8
    // pairs, q = 6: 2.0e9 pairs); q = 4 and 7 from the parity sweeps
    grim_tuning_t t = {0, 0, 1024, 8};
    switch (q) {
    case 4: t = {2, 8, 1024, 8}; break;
    case 5: t = {4, 4, 1024, 4}; break;
    case 6: t = {8, 2, 512, 4}; break;
    case 7: t = {64, 2, 1024, 8}; break;
    default: return GRIM_E_UNSUPPORTED;
    }
    *out = t;
    return GRIM_OK;
}

extern "C" int grim_tuning_candidates(uint32_t q, grim_tuning_t *out, uint32_t cap, uint32_t *n)
{
    if (!n || (cap && !out))
        return GRIM_E_INVALID;
    grim_tuning_t d;
    if (grim_default_tuning(q, &d))
        return GRIM_E_UNSUPPORTED;
    int nv = 0;
    const BatchedVariant *v = batched_variants(&nv);
    uint32_t k = 0;
    for (int i = 0; i < nv; ++i) {
        if ((uint32_t)v[i].q != q)
            continue;
        if (k < cap)
            out[k] = grim_tuning_t{(uint32_t)v[i].g, (uint32_t)v[i].u, d.tile_pairs, d.wg_per_cu};
        ++k;
    }
    *n = k;
    return GRIM_OK;
}

extern "C" int grim_workspace_size(const grim_index_t *idx, uint64_t n_pairs,
                                   const grim_tuning_t *tune, uint64_t *bytes)
{
    if (!idx || !bytes)
        return GRIM_E_INVALID;
    grim_tuning_t t;
    int rc = resolve_tuning(idx, kMaxLen, tune, &t);
    if (rc)
        return rc;
    // the cached tuning may use a smaller tile: size for the smallest tile
    *bytes = ws_bytes_for(n_pairs, std::min<uint32_t>(t.tile_pairs, 512));
    return GRIM_OK;
}

extern "C" int grim_filter_batch(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
                                 uint32_t *pass_bits, void *workspace, uint64_t workspace_bytes,
                                 const grim_tuning_t *tune, void *stream)
{
    int rc = check_batch(idx, b);
    if (rc)
        return rc;
    grim_tuning_t t;
    rc = resolve_tuning(idx, b->max_len, tune, &t);
    if (rc)
        return rc;
    return enqueue_batched(idx, b, counts, pass_bits, workspace, workspace_bytes, t,
                           reinterpret_cast<hipStream_t>(stream));
}

// ------------------------------------------------- filter without allocation
// The scratch of grim_filter_batch_noalloc: one file-scope device array per GPU
// (tile counter, padded header, first read of each tile).  Host code never uses
// the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, and is kept in g_scratch_ptr.
static __device__ __align__(256) uint8_t scratch[GRIM_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;

int scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return GRIM_OK;
    }
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255))
        return hip_fail(hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
    *out = p;
    return GRIM_OK;
}
}  // namespace

extern "C" int grim_filter_batch_noalloc(const grim_index_t *idx, const grim_batch_t *b,
                                         int32_t *counts, uint32_t *pass_bits, uint32_t *status,
                                         const grim_tuning_t *tune, void *stream)
{
    int rc = check_batch(idx, b);
    if (rc)
        return rc;
    if (!status)
        return GRIM_E_INVALID;
    grim_tuning_t t;
    rc = resolve_tuning(idx, b->max_len, tune, &t);
    if (rc)
        return rc;
    if (ws_bytes_for(b->n_pairs, t.tile_pairs) > GRIM_NOALLOC_SCRATCH_BYTES)
        return GRIM_E_SCRATCH;
    void *ws = nullptr;
    rc = scratch_address(idx->device, &ws);  // check_batch made idx->device current
    if (rc)
        return rc;
    return enqueue_batched(idx, b, counts, pass_bits, ws, GRIM_NOALLOC_SCRATCH_BYTES, t,
                           reinterpret_cast<hipStream_t>(stream), status);
}

extern "C" int grim_filter_plain(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
                                 uint32_t *pass_bits, void *workspace, uint64_t workspace_bytes,
                                 void *stream)
{
    int rc = check_batch(idx, b);
    if (rc)
        return rc;
    if (!workspace || workspace_bytes < kWsHeader || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return GRIM_E_INVALID;
    if (b->n_pairs && (!counts || !pass_bits))
        return GRIM_E_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    FilterArgs a = make_args(idx, b, counts, pass_bits, workspace);
    HIP_TRY(launch_zero(s, a.status, 2));
    const uint64_t n_words = (b->n_pairs + 31) / 32;
    if (n_words)
        HIP_TRY(launch_zero(s, pass_bits, n_words));
    if (b->n_reads == 0)
        return GRIM_OK;
    const size_t lds = (size_t)a.npl * vector_words(idx->q) * 4;
    if (lds > 65536)
        return GRIM_E_UNSUPPORTED;
    const uint64_t grid = std::min<uint64_t>(b->n_reads, 1u << 22);
    HIP_TRY(launch_filter(plain_kernel(idx->q), dim3((uint32_t)grid), dim3(64), lds, s, a));
    return GRIM_OK;
}

extern "C" int grim_filter_status(const void *workspace, void *stream, uint32_t *flags)
{
    if (!workspace)
        return GRIM_E_INVALID;
    HIP_TRY(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
    uint32_t f = 0;
    HIP_TRY(hipMemcpy(&f, workspace, 4, hipMemcpyDeviceToHost));
    if (flags)
        *flags = f;
    if (f & GRIM_FLAG_BIN_RANGE)
        return GRIM_E_BIN_RANGE;
    if (f & (GRIM_FLAG_READ | GRIM_FLAG_CAND_OFF))
        return GRIM_E_READ;
    return GRIM_OK;
}

extern "C" int grim_tune(const grim_index_t *idx, const grim_batch_t *sample, int32_t *counts,
                         uint32_t *pass_bits, void *workspace, uint64_t workspace_bytes,
                         void *stream, grim_tuning_t *out)
{
    int rc = check_batch(idx, sample);
    if (rc)
        return rc;
    if (!out)
        return GRIM_E_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // time on a prefix of the pair space (the kernel handles any prefix of a
    // valid CSR batch): keeps a sweep over every shape to a few seconds
    grim_batch_t sub = *sample;
    if (sub.n_pairs > (1ull << 26))
        sub.n_pairs = 1ull << 26;
    sample = &sub;
    int nv = 0;
    const BatchedVariant *vars = batched_variants(&nv);
    const uint32_t tiles[] = {512, 1024, 2048};
    const uint32_t occ[] = {4, 8};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    grim_tuning_t best_t;
    grim_default_tuning(idx->q, &best_t);
    for (int i = 0; i < nv; ++i) {
        if ((uint32_t)vars[i].q != idx->q)
            continue;
        for (uint32_t tp : tiles) {
            for (uint32_t wg : occ) {
                grim_tuning_t t = {(uint32_t)vars[i].g, (uint32_t)vars[i].u, tp, wg};
                if (workspace_bytes < ws_bytes_for(sample->n_pairs, tp))
                    continue;
                if (enqueue_batched(idx, sample, counts, pass_bits, workspace, workspace_bytes, t, s))
                    continue;
                float ms[3];
                bool fine = true;
                for (int rep = 0; rep < 3 && fine; ++rep) {
                    fine = hipEventRecord(e0, s) == hipSuccess &&
                           enqueue_batched(idx, sample, counts, pass_bits, workspace,
                                           workspace_bytes, t, s) == GRIM_OK &&
                           hipEventRecord(e1, s) == hipSuccess &&
                           hipEventSynchronize(e1) == hipSuccess &&
                           hipEventElapsedTime(&ms[rep], e0, e1) == hipSuccess;
                }
                if (!fine)
                    continue;
                std::sort(ms, ms + 3);
                if (ms[1] < best) {
                    best = ms[1];
                    best_t = t;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_TRY(hipStreamSynchronize(s));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[{idx->device, idx->q, sample->max_len}] = best_t;
    }
    *out = best_t;
    return GRIM_OK;
}

// ------------------------------------------------- seed location checker
extern "C" int grim_survivors_workspace_size(uint64_t n_pairs, uint64_t *bytes)
{
    if (!bytes)
        return GRIM_E_INVALID;
    *bytes = (8 * std::max<uint64_t>(1, compact_blocks(n_pairs)) + 255) & ~255ull;
    return GRIM_OK;
}

extern "C" int grim_compact_survivors(const grim_batch_t *b, const uint32_t *pass_bits,
                                      uint64_t capacity, uint64_t *surv_pair, uint32_t *surv_read,
                                      uint32_t *surv_bin, uint64_t *n_survivors, void *workspace,
                                      uint64_t workspace_bytes, void *stream)
{
    if (!b || !n_survivors || !workspace)
        return GRIM_E_INVALID;
    if (b->n_reads == 0 && b->n_pairs != 0)
        return GRIM_E_INVALID;
    if (b->n_pairs && (!pass_bits || !b->cand_off || !b->cand_bin))
        return GRIM_E_INVALID;
    if (capacity && (!surv_pair || !surv_read || !surv_bin))
        return GRIM_E_INVALID;
    uint64_t need = 0;
    grim_survivors_workspace_size(b->n_pairs, &need);
    if (workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 7))
        return GRIM_E_INVALID;
    HIP_TRY(launch_compact(reinterpret_cast<hipStream_t>(stream), pass_bits, b->n_pairs,
                           b->cand_off, b->n_reads, b->cand_bin, capacity, surv_pair, surv_read,
                           surv_bin, n_survivors, reinterpret_cast<uint64_t *>(workspace)));
    return GRIM_OK;
}

extern "C" int grim_index_attach_reference(grim_index_t *idx, const uint32_t *ref_2bit,
                                           uint64_t ref_len, void *stream)
{
    if (!idx || !ref_2bit || ref_len != idx->G)
        return GRIM_E_INVALID;
    const uint64_t nw = grim_packed_words(ref_len);
    uint32_t *d = nullptr;
    if (hipMalloc(&d, (nw + kRefPadWords) * 4) != hipSuccess)
        return GRIM_E_NOMEM;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(d, ref_2bit, nw * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_zero(s, d + nw, kRefPadWords);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "grim_index_attach_reference");
    }
    if (idx->d_ref)
        (void)hipFree(idx->d_ref);
    idx->d_ref = d;
    idx->ref_words = nw;
    return GRIM_OK;
}

extern "C" int grim_verify_survivors(const grim_index_t *idx, const grim_batch_t *b,
                                     const uint32_t *surv_read, const uint32_t *surv_bin,
                                     uint64_t n_survivors, int32_t *dist, uint32_t *ok_bits,
                                     void *stream)
{
    int rc = check_batch(idx, b);
    if (rc)
        return rc;
    if (!idx->d_ref)
        return GRIM_E_INVALID;
    if (n_survivors && (!surv_read || !surv_bin || !dist || !ok_bits))
        return GRIM_E_INVALID;
    const int W = b->max_len <= 64 ? 1 : b->max_len <= 128 ? 2 : b->max_len <= 256 ? 4
                : b->max_len <= 512 ? 8 : 0;
    if (!W)
        return GRIM_E_UNSUPPORTED;
    if (n_survivors == 0)
        return GRIM_OK;
    VerifyArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ref = idx->d_ref;
    a.ref_words = idx->ref_words;
    a.G = idx->G;
    a.B = idx->B;
    a.O = idx->O;
    a.n_bins = idx->n_bins;
    a.rw = b->reads_2bit;
    a.nw = b->n_read_words;
    a.read_off = b->read_off;
    a.read_len = b->read_len;
    a.read_e = b->read_e;
    a.e_den = b->e_den;
    a.n_reads = b->n_reads;
    a.surv_read = surv_read;
    a.surv_bin = surv_bin;
    a.n_surv = n_survivors;
    a.dist = dist;
    a.ok_bits = ok_bits;
    HIP_TRY(launch_verify(reinterpret_cast<hipStream_t>(stream), W, cu_count(idx->device), a));
    return GRIM_OK;
}

// ---------------------------------------------------------------- bin windows
extern "C" int grim_index_transpose(grim_index_t *idx, void *stream)
{
    if (!idx)
        return GRIM_E_INVALID;
    // one 32-word (1024-bin) segment of every row per transpose tile
    const uint64_t row_words = ((idx->n_bins + 1023) / 1024) * 32;
    const uint64_t n_rows = 1ull << (2 * idx->q);
    uint32_t *rows = nullptr;
    // one pad word past the last row: the window kernel reads two adjacent
    // words of a row with one load
    if (hipMalloc(&rows, n_rows * row_words * 4 + 256) != hipSuccess)
        return GRIM_E_NOMEM;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint64_t grid = row_words / 32;
    const uint64_t cap = (uint64_t)cu_count(idx->device) * 2;
    if (grid > cap)
        grid = cap;
    hipError_t e = launch_transpose(s, idx->q, reinterpret_cast<const uint32_t *>(idx->d_vec),
                                    idx->n_bins, row_words, rows, (uint32_t)grid);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(rows);
        return hip_fail(e, "grim_index_transpose");
    }
    if (idx->d_rows)
        (void)hipFree(idx->d_rows);
    idx->d_rows = rows;
    idx->row_words = row_words;
    return GRIM_OK;
}

extern "C" int grim_filter_windows(const grim_index_t *idx, const grim_batch_t *b,
                                   const uint32_t *win_lo, const uint32_t *order, int32_t *counts,
                                   uint32_t *pass_bits, void *workspace, uint64_t workspace_bytes,
                                   void *stream)
{
    if (!idx || !b)
        return GRIM_E_INVALID;
    if (b->e_den == 0 || b->max_len == 0 || (b->n_reads == 0 && b->n_pairs != 0))
        return GRIM_E_INVALID;
    if (b->max_len > 4096)
        return GRIM_E_UNSUPPORTED;
    if (b->n_reads && (!b->read_off || !b->read_len || !b->read_e || !b->cand_off || !win_lo ||
                       !b->reads_2bit || b->n_read_words == 0))
        return GRIM_E_INVALID;
    if (b->n_pairs && (!counts || !pass_bits))
        return GRIM_E_INVALID;
    if (!idx->d_rows)
        return GRIM_E_INVALID;
    if (!workspace || workspace_bytes < kWsHeader || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return GRIM_E_INVALID;
    int dev = -1;
    int rc = current_device(&dev);
    if (rc)
        return rc;
    if (dev != idx->device)
        return GRIM_E_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    WindowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.rows = idx->d_rows;
    a.row_words = idx->row_words;
    a.rows_bytes = (1ull << (2 * idx->q)) * idx->row_words * 4 + 256;
    a.n_bins = idx->n_bins;
    a.rw = b->reads_2bit;
    a.nw = b->n_read_words;
    a.read_off = b->read_off;
    a.read_len = b->read_len;
    a.read_e = b->read_e;
    a.e_den = b->e_den;
    a.max_len = b->max_len;
    a.cand_off = b->cand_off;
    a.win_lo = win_lo;
    a.order = order;
    a.n_reads = b->n_reads;
    a.n_pairs = b->n_pairs;
    a.counts = counts;
    a.pass_bits = pass_bits;
    a.status = reinterpret_cast<uint32_t *>(workspace);
    a.counter = reinterpret_cast<uint32_t *>(workspace) + 1;
    a.npl = planes_for(idx->q, b->max_len);
    HIP_TRY(launch_zero(s, a.status, 2));
    const uint64_t n_words = (b->n_pairs + 31) / 32;
    if (n_words)
        HIP_TRY(launch_zero(s, pass_bits, n_words));
    if (b->n_reads == 0)
        return GRIM_OK;
    HIP_TRY(launch_window(s, idx->q, (uint32_t)cu_count(idx->device), (size_t)b->max_len * 4, a));
    return GRIM_OK;
}

extern "C" int grim_window_order_workspace_size(const grim_index_t *idx, uint64_t n_reads,
                                                uint64_t *bytes)
{
    (void)n_reads;
    if (!idx || !bytes)
        return GRIM_E_INVALID;
    uint32_t n_buckets = 0;
    order_shift(idx->n_bins, &n_buckets);
    *bytes = std::max<uint64_t>(256, ((uint64_t)n_buckets * 4 + 255) & ~255ull);
    return GRIM_OK;
}

extern "C" int grim_window_order(const grim_index_t *idx, const uint32_t *win_lo, uint64_t n_reads,
                                 uint32_t *order, void *workspace, uint64_t workspace_bytes,
                                 void *stream)
{
    if (!idx)
        return GRIM_E_INVALID;
    if (n_reads == 0)
        return GRIM_OK;
    if (!win_lo || !order || !workspace)
        return GRIM_E_INVALID;
    if (n_reads > 0xffffffffull)
        return GRIM_E_UNSUPPORTED;
    uint32_t n_buckets = 0;
    const uint32_t shift = order_shift(idx->n_bins, &n_buckets);
    if (workspace_bytes < (uint64_t)n_buckets * 4)
        return GRIM_E_INVALID;
    int dev = -1;
    int rc = current_device(&dev);
    if (rc)
        return rc;
    if (dev != idx->device)
        return GRIM_E_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(workspace);
    HIP_TRY(launch_zero(s, cnt, n_buckets));
    HIP_TRY(launch_window_order(s, (uint32_t)cu_count(idx->device), win_lo, (uint32_t)n_reads,
                                idx->n_bins, shift, n_buckets, cnt, order));
    return GRIM_OK;
}

// ---------------------------------------------------------------- probes
extern "C" int grim_probe_gather(const grim_index_t *idx, const uint32_t *ids, uint64_t n,
                                 int32_t *out, void *stream)
{
    if (!idx || (n && (!ids || !out)))
        return GRIM_E_INVALID;
    if (n == 0)
        return GRIM_OK;
    int dev = -1;
    int rc = current_device(&dev);
    if (rc)
        return rc;
    if (dev != idx->device)
        return GRIM_E_INVALID;
    HIP_TRY(launch_probe_gather(reinterpret_cast<hipStream_t>(stream), idx->q,
                                (uint32_t)cu_count(idx->device) * 8, idx->d_vec, idx->n_bins, ids,
                                n, out));
    return GRIM_OK;
}

extern "C" int grim_probe_stream(const grim_index_t *idx, uint32_t *sink, void *stream)
{
    if (!idx || !sink)
        return GRIM_E_INVALID;
    int dev = -1;
    int rc = current_device(&dev);
    if (rc)
        return rc;
    if (dev != idx->device)
        return GRIM_E_INVALID;
    HIP_TRY(launch_probe_stream(reinterpret_cast<hipStream_t>(stream),
                                (uint32_t)cu_count(idx->device) * 8, idx->d_vec, idx->bytes / 16,
                                sink));
    return GRIM_OK;
}

// ---------------------------------------------------------------- graphs
struct grim_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" int grim_graph_create(const grim_index_t *idx, const grim_batch_t *b, int32_t *counts,
                                 uint32_t *pass_bits, void *workspace, uint64_t workspace_bytes,
                                 const grim_tuning_t *tune, grim_graph_t **out)
{
    int rc = check_batch(idx, b);
    if (rc)
        return rc;
    if (!out)
        return GRIM_E_INVALID;
    grim_tuning_t t;
    rc = resolve_tuning(idx, b->max_len, tune, &t);
    if (rc)
        return rc;
    hipStream_t s;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    rc = enqueue_batched(idx, b, counts, pass_bits, workspace, workspace_bytes, t, s);
    e = hipStreamEndCapture(s, &graph);
    (void)hipStreamDestroy(s);
    if (rc) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess)
        return hip_fail(e, "hipStreamEndCapture");
    grim_graph *g = new (std::nothrow) grim_graph();
    if (!g) {
        (void)hipGraphDestroy(graph);
        return GRIM_E_NOMEM;
    }
    g->graph = graph;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = g;
    return GRIM_OK;
}

extern "C" int grim_graph_launch(grim_graph_t *g, void *stream)
{
    if (!g)
        return GRIM_E_INVALID;
    HIP_TRY(hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)));
    return GRIM_OK;
}

extern "C" void grim_graph_destroy(grim_graph_t *g)
{
    if (!g)
        return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}
