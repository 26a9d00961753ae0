/*
 * Seeded synthetic inputs for the GRIM-Filter library and its oracle.
 *
 * This module produces references, reads and candidate lists only.  It holds
 * none of the filter's arithmetic (no tokens, bin vectors, thresholds or
 * packing): both the oracle and the HIP library consume what it writes.
 *
 * Every random number is a pure function of (seed, stream, counter) through a
 * keyed splitmix64 hash (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014; finaliser constants of Vigna's public
 * splitmix64), so work can be split over threads with no change in output.
 * Base codes: A=0 C=1 G=2 T=3, one byte each.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

static inline uint64_t sm_mix(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* keyed counter hash: independent stream of values for each (seed, stream) */
static inline uint64_t crng(uint64_t seed, uint64_t stream, uint64_t i)
{
    return sm_mix(sm_mix(sm_mix(seed) ^ (stream * 0xd1b54a32d192ed03ULL)) ^ i);
}

/* sequential splitmix64 stream seeded from one counter value */
static inline uint64_t sm_next(uint64_t *s)
{
    *s += 0x9e3779b97f4a7c15ULL;
    uint64_t z = *s;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }
static inline uint64_t below(uint64_t x, uint64_t n) { return (uint64_t)(((__uint128_t)x * n) >> 64); }

/* ---------------------------------------------------------------- threads */
typedef void (*range_fn)(void *ctx, uint64_t lo, uint64_t hi);
typedef struct {
    range_fn fn;
    void *ctx;
    uint64_t lo, hi;
} job_t;

static void *job_run(void *p)
{
    job_t *j = (job_t *)p;
    if (j->hi > j->lo)
        j->fn(j->ctx, j->lo, j->hi);
    return NULL;
}

static void parallel_for(range_fn fn, void *ctx, uint64_t n, int n_threads)
{
    if (n_threads <= 0) {
        long c = sysconf(_SC_NPROCESSORS_ONLN);
        n_threads = c > 0 ? (int)c : 1;
    }
    if (n_threads > 64)
        n_threads = 64;
    if ((uint64_t)n_threads > n)
        n_threads = n > 0 ? (int)n : 1;
    if (n_threads <= 1) {
        if (n)
            fn(ctx, 0, n);
        return;
    }
    pthread_t th[64];
    job_t jobs[64];
    int created[64];
    uint64_t step = (n + n_threads - 1) / n_threads;
    for (int t = 0; t < n_threads; t++) {
        uint64_t lo = (uint64_t)t * step, hi = lo + step;
        if (lo > n)
            lo = n;
        if (hi > n)
            hi = n;
        jobs[t] = (job_t){fn, ctx, lo, hi};
        created[t] = pthread_create(&th[t], NULL, job_run, &jobs[t]) == 0;
        if (!created[t])
            job_run(&jobs[t]);
    }
    for (int t = 0; t < n_threads; t++)
        if (created[t])
            pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------- reference */
typedef struct {
    uint64_t seed, G;
    double repeat_frac, id_lo, id_hi;
    uint32_t n_families, rep_len;
    uint8_t *out;
} ref_ctx;

static void ref_background(void *p, uint64_t lo, uint64_t hi)
{
    ref_ctx *c = (ref_ctx *)p;
    for (uint64_t blk = lo; blk < hi; blk++) {
        uint64_t h = crng(c->seed, 1, blk);
        uint64_t base = blk * 32;
        for (int j = 0; j < 32 && base + j < c->G; j++)
            c->out[base + j] = (uint8_t)((h >> (2 * j)) & 3);
    }
}

static void ref_repeats(void *p, uint64_t lo, uint64_t hi)
{
    ref_ctx *c = (ref_ctx *)p;
    const uint64_t clen = 2ull * c->rep_len; /* consensus stretch, room for deletions */
    for (uint64_t s = lo; s < hi; s++) {
        if (u01(crng(c->seed, 2, s)) >= c->repeat_frac)
            continue;
        uint64_t st = crng(c->seed, 3, s);
        uint64_t fam = below(sm_next(&st), c->n_families);
        double ident = c->id_lo + (c->id_hi - c->id_lo) * u01(sm_next(&st));
        uint8_t *dst = c->out + s * c->rep_len;
        uint64_t j = 0; /* consensus position */
        uint32_t i = 0;
        while (i < c->rep_len) {
            uint8_t cons = (uint8_t)(crng(c->seed, 4, fam * clen + (j % clen)) & 3);
            if (u01(sm_next(&st)) >= 1.0 - ident) {
                dst[i++] = cons;
                j++;
                continue;
            }
            uint64_t r = sm_next(&st);
            double kind = u01(r);
            if (kind < 0.9) { /* substitution */
                dst[i++] = (uint8_t)((cons + 1 + below(sm_next(&st), 3)) & 3);
                j++;
            } else {
                uint32_t len = 1 + (uint32_t)below(sm_next(&st), 3);
                if (kind < 0.95) { /* insertion of 1-3 random bases */
                    for (uint32_t k = 0; k < len && i < c->rep_len; k++)
                        dst[i++] = (uint8_t)(sm_next(&st) & 3);
                } else { /* deletion of 1-3 consensus bases */
                    j += len;
                }
            }
        }
    }
}

/* Reference of G bases: iid uniform ACGT, then a fraction repeat_frac of the
 * rep_len-long slots of the genome overwritten by a mutated copy of one of
 * n_families random consensus elements.  A copy keeps each consensus base with
 * probability `identity` (uniform in [id_lo, id_hi] per copy); the other
 * positions are edited: 90 % substitutions, 5 % insertions and 5 % deletions
 * of 1-3 bases. */
void synth_reference(uint64_t seed, uint64_t G, double repeat_frac, uint32_t n_families,
                     uint32_t rep_len, double id_lo, double id_hi, int n_threads, uint8_t *out)
{
    ref_ctx c = {seed, G, repeat_frac, id_lo, id_hi, n_families ? n_families : 1,
                 rep_len ? rep_len : 1, out};
    parallel_for(ref_background, &c, (G + 31) / 32, n_threads);
    if (repeat_frac > 0.0 && rep_len > 0)
        parallel_for(ref_repeats, &c, G / c.rep_len, n_threads);
}

/* ----------------------------------------------------------------- reads */
/* Per-read length and error-tolerance numerator, each drawn uniformly from the
 * given choices. */
void synth_read_meta(uint64_t seed, uint64_t n_reads, const uint32_t *len_choices, uint32_t n_len,
                     const uint32_t *e_choices, uint32_t n_e, uint32_t *read_len, uint32_t *read_e)
{
    for (uint64_t r = 0; r < n_reads; r++) {
        uint64_t st = crng(seed, 10, r);
        read_len[r] = len_choices[below(sm_next(&st), n_len)];
        read_e[r] = e_choices[below(sm_next(&st), n_e)];
    }
}

typedef struct {
    uint64_t seed, G;
    const uint8_t *ref;
    const uint32_t *read_len, *read_e;
    uint32_t e_den;
    const uint64_t *read_off;
    uint8_t *codes;
    uint64_t *read_z;
    uint32_t *read_span, *read_edits;
} reads_ctx;

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : x > y;
}

static void reads_work(void *p, uint64_t lo, uint64_t hi)
{
    reads_ctx *c = (reads_ctx *)p;
    uint32_t pos[4096];
    uint8_t kind[4096];
    for (uint64_t r = lo; r < hi; r++) {
        uint64_t st = crng(c->seed, 11, r);
        uint32_t L = c->read_len[r];
        /* planted edit budget: floor(L * e), drawn uniformly in 0..budget */
        uint32_t kmax = (uint32_t)(((uint64_t)L * c->read_e[r]) / c->e_den);
        if (kmax > 4096)
            kmax = 4096;
        uint32_t k = (uint32_t)below(sm_next(&st), (uint64_t)kmax + 1);
        uint64_t room = c->G > (uint64_t)L + kmax ? c->G - L - kmax : 1;
        uint64_t z = below(sm_next(&st), room);
        for (uint32_t e = 0; e < k; e++) {
            pos[e] = (uint32_t)below(sm_next(&st), L ? L : 1);
        }
        qsort(pos, k, sizeof(uint32_t), cmp_u32);
        for (uint32_t e = 0; e < k; e++)
            kind[e] = (uint8_t)below(sm_next(&st), 3); /* 0 sub, 1 ins, 2 del */
        uint8_t *dst = c->codes + c->read_off[r];
        uint64_t j = z;
        uint32_t e = 0, i = 0;
        while (i < L) {
            if (e < k && pos[e] == i) {
                uint8_t kd = kind[e++];
                if (kd == 0) {
                    uint8_t b = j < c->G ? c->ref[j] : 0;
                    dst[i++] = (uint8_t)((b + 1 + below(sm_next(&st), 3)) & 3);
                    j++;
                } else if (kd == 1) {
                    dst[i++] = (uint8_t)(sm_next(&st) & 3);
                } else {
                    j++;
                }
                continue;
            }
            dst[i++] = j < c->G ? c->ref[j] : 0;
            j++;
        }
        if (c->read_z)
            c->read_z[r] = z;
        if (c->read_span)
            c->read_span[r] = (uint32_t)(j - z);
        if (c->read_edits)
            c->read_edits[r] = k;
    }
}

/* Reads sampled from the reference: read r starts at a uniform origin z and
 * carries k planted edits, k uniform in 0..floor(L * read_e/e_den), each a
 * substitution, insertion or deletion with probability 1/3 at a uniform read
 * position.  Bases go to codes[read_off[r] ..+ read_len[r]).  read_z, read_span
 * (reference bases consumed) and read_edits record the ground truth; any of
 * them may be NULL. */
void synth_read_seqs(uint64_t seed, const uint8_t *ref, uint64_t G, uint64_t n_reads,
                     const uint32_t *read_len, const uint32_t *read_e, uint32_t e_den,
                     const uint64_t *read_off, int n_threads, uint8_t *codes, uint64_t *read_z,
                     uint32_t *read_span, uint32_t *read_edits)
{
    reads_ctx c = {seed, G, ref, read_len, read_e, e_den ? e_den : 1, read_off, codes,
                   read_z, read_span, read_edits};
    parallel_for(reads_work, &c, n_reads, n_threads);
}

/* ------------------------------------------------------------ candidates */
/* Candidate counts drawn from a Zipf(s) law on {1..kmax} by inverse CDF. */
void synth_cand_counts_zipf(uint64_t seed, uint64_t n_reads, double s, uint32_t kmax, uint32_t *k)
{
    double *cdf = (double *)malloc(sizeof(double) * kmax);
    double acc = 0.0;
    for (uint32_t i = 0; i < kmax; i++) {
        acc += pow((double)(i + 1), -s);
        cdf[i] = acc;
    }
    for (uint64_t r = 0; r < n_reads; r++) {
        double u = u01(crng(seed, 20, r)) * acc;
        uint32_t lo = 0, hi = kmax - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi) / 2;
            if (cdf[mid] < u)
                lo = mid + 1;
            else
                hi = mid;
        }
        k[r] = lo + 1;
    }
    free(cdf);
}

/* Candidate counts uniform on {lo..hi}. */
void synth_cand_counts_uniform(uint64_t seed, uint64_t n_reads, uint32_t lo, uint32_t hi, uint32_t *k)
{
    for (uint64_t r = 0; r < n_reads; r++)
        k[r] = lo + (uint32_t)below(crng(seed, 21, r), (uint64_t)(hi - lo) + 1);
}

typedef struct {
    uint64_t seed, B, n_bins;
    const uint64_t *cand_off, *read_z;
    uint32_t *cand_bin;
    uint64_t *true_pair;
} cand_ctx;

static void cand_work(void *p, uint64_t lo, uint64_t hi)
{
    cand_ctx *c = (cand_ctx *)p;
    for (uint64_t r = lo; r < hi; r++) {
        uint64_t a = c->cand_off[r], b = c->cand_off[r + 1];
        uint64_t st = crng(c->seed, 22, r);
        if (b == a) {
            if (c->true_pair)
                c->true_pair[r] = UINT64_MAX;
            continue;
        }
        uint64_t tb = c->read_z[r] / c->B;
        if (tb >= c->n_bins)
            tb = c->n_bins - 1;
        uint64_t slot = a + below(sm_next(&st), b - a);
        for (uint64_t k = a; k < b; k++) {
            if (k == slot) {
                c->cand_bin[k] = (uint32_t)tb;
                continue;
            }
            uint64_t x;
            do {
                x = below(sm_next(&st), c->n_bins);
            } while (x == tb && c->n_bins > 1);
            c->cand_bin[k] = (uint32_t)x;
        }
        if (c->true_pair)
            c->true_pair[r] = slot;
    }
}

/* Candidate bins per read: the read's true bin (origin / B) at a random slot
 * of its list, every other slot a uniform random bin other than the true one.
 * true_pair[r] receives the pair index of the true bin (UINT64_MAX when the
 * read has no candidates); it may be NULL. */
void synth_cand_fill_random(uint64_t seed, uint64_t n_reads, const uint64_t *cand_off,
                            const uint64_t *read_z, uint64_t B, uint64_t n_bins, int n_threads,
                            uint32_t *cand_bin, uint64_t *true_pair)
{
    cand_ctx c = {seed, B, n_bins, cand_off, read_z, cand_bin, true_pair};
    parallel_for(cand_work, &c, n_reads, n_threads);
}

/* ---------------------------------------------- k-mer seeding (mapper stand-in) */
static inline int64_t kmer_at(const uint8_t *s, uint32_t k)
{
    uint64_t v = 0;
    for (uint32_t j = 0; j < k; j++)
        v = (v << 2) | s[j];
    return (int64_t)v;
}

/* Occurrence counts of every k-mer (k <= 15) of the reference: cnt has 4^k
 * entries. */
void synth_kmer_count(const uint8_t *ref, uint64_t G, uint32_t k, uint32_t *cnt)
{
    for (uint64_t p = 0; p + k <= G; p++)
        cnt[kmer_at(ref + p, k)]++;
}

/* Position lists of every k-mer: fill[] starts as the exclusive prefix sum of
 * the counts and is advanced in place; pos receives G - k + 1 positions
 * grouped by k-mer, increasing within each group. */
void synth_kmer_fill(const uint8_t *ref, uint64_t G, uint32_t k, uint64_t *fill, uint32_t *pos)
{
    for (uint64_t p = 0; p + k <= G; p++)
        pos[fill[kmer_at(ref + p, k)]++] = (uint32_t)p;
}

/* Candidate bins of each read from exact k-mer seeds at read offsets 0, k, 2k,
 * ... (while the seed fits): every reference hit p of the seed at offset o
 * proposes location z = p - o (clamped into the genome) and bin z / B.  Bins
 * are deduplicated per read, kept in increasing order and capped at `cap`.
 * With cand_bin == NULL only the per-read counts n_out[r] are produced;
 * otherwise the bins are written at cand_off[r]. */
typedef struct {
    const uint8_t *ref, *codes;
    uint64_t G, B;
    uint32_t k, cap;
    const uint64_t *kmer_off;
    const uint32_t *kmer_pos;
    const uint64_t *read_off;
    const uint32_t *read_len;
    const uint64_t *cand_off;
    uint32_t *n_out, *cand_bin;
} seed_ctx;

static void seed_work(void *p, uint64_t lo, uint64_t hi)
{
    seed_ctx *c = (seed_ctx *)p;
    size_t capb = 1 << 16;
    uint32_t *buf = (uint32_t *)malloc(capb * sizeof(uint32_t));
    for (uint64_t r = lo; r < hi; r++) {
        const uint8_t *rd = c->codes + c->read_off[r];
        uint32_t L = c->read_len[r];
        size_t n = 0;
        for (uint32_t o = 0; o + c->k <= L; o += c->k) {
            int64_t km = kmer_at(rd + o, c->k);
            for (uint64_t h = c->kmer_off[km]; h < c->kmer_off[km + 1]; h++) {
                int64_t z = (int64_t)c->kmer_pos[h] - (int64_t)o;
                if (z < 0)
                    z = 0;
                if ((uint64_t)z >= c->G)
                    z = (int64_t)c->G - 1;
                if (n == capb) {
                    capb *= 2;
                    buf = (uint32_t *)realloc(buf, capb * sizeof(uint32_t));
                }
                buf[n++] = (uint32_t)((uint64_t)z / c->B);
            }
        }
        qsort(buf, n, sizeof(uint32_t), cmp_u32);
        size_t u = 0;
        for (size_t i = 0; i < n; i++)
            if (u == 0 || buf[u - 1] != buf[i])
                buf[u++] = buf[i];
        if (u > c->cap)
            u = c->cap;
        if (c->cand_bin)
            memcpy(c->cand_bin + c->cand_off[r], buf, u * sizeof(uint32_t));
        else
            c->n_out[r] = (uint32_t)u;
    }
    free(buf);
}

void synth_seed_candidates(const uint8_t *ref, uint64_t G, uint32_t k, const uint64_t *kmer_off,
                           const uint32_t *kmer_pos, const uint8_t *codes, const uint64_t *read_off,
                           const uint32_t *read_len, uint64_t n_reads, uint64_t B, uint32_t cap,
                           int n_threads, uint32_t *n_out, const uint64_t *cand_off, uint32_t *cand_bin)
{
    seed_ctx c = {ref, codes, G, B, k, cap, kmer_off, kmer_pos, read_off, read_len, cand_off,
                  n_out, cand_bin};
    parallel_for(seed_work, &c, n_reads, n_threads);
}
