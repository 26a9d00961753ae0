/*
 * Checks of the C ABI's host helpers (2-bit packing, exact tolerance
 * arithmetic), written to run under AddressSanitizer and UndefinedBehavior-
 * Sanitizer.  Built and run by tests/test_sanitizers.py together with
 * grim_host.cpp; exits non-zero on the first failed check.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "grim.h"

static int failures = 0;

#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

static uint64_t next_u64(void)
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* code of base j of a packed stream: 16 bases per word, first in the top bits */
static unsigned unpacked(const uint32_t *w, uint64_t j)
{
    return (w[j / 16] >> (30 - 2 * (j % 16))) & 3u;
}

static void check_pack(uint64_t n, int threads, int letters)
{
    static const char L[4] = {'A', 'C', 'G', 'T'};
    static const char l[4] = {'a', 'c', 'g', 't'};
    uint8_t *b = malloc(n ? n : 1);
    unsigned char *want = malloc(n ? n : 1);
    const uint64_t nw = grim_packed_words(n);
    CHECK(nw == (n + 15) / 16 + 1);
    /* exactly nw words: ASan reports any write past them */
    uint32_t *w = malloc(nw * sizeof(uint32_t));
    for (uint64_t i = 0; i < n; ++i) {
        const unsigned c = (unsigned)(next_u64() & 3u);
        want[i] = (unsigned char)c;
        b[i] = letters == 0 ? (uint8_t)c : letters == 1 ? (uint8_t)L[c] : (uint8_t)l[c];
    }
    CHECK(grim_pack_bases(b, n, w, threads) == GRIM_OK);
    for (uint64_t i = 0; i < n; ++i)
        CHECK(unpacked(w, i) == want[i]);
    for (uint64_t i = n; i < nw * 16; ++i)  /* padding bases are zero */
        CHECK(unpacked(w, i) == 0);
    if (n) {
        b[next_u64() % n] = 'N';
        CHECK(grim_pack_bases(b, n, w, threads) == GRIM_E_BASE);
    }
    free(w);
    free(want);
    free(b);
}

int main(void)
{
    for (uint64_t n = 0; n < 70; ++n)
        for (int letters = 0; letters < 3; ++letters)
            check_pack(n, 1, letters);
    const uint64_t big[] = {1u << 20, (1u << 20) + 7, 3000001};
    for (int i = 0; i < 3; ++i)
        for (int t = 0; t <= 8; t += 4)
            check_pack(big[i], t, i % 3);
    CHECK(grim_pack_bases(NULL, 5, (uint32_t *)&failures, 1) == GRIM_E_INVALID);
    CHECK(grim_pack_bases((const uint8_t *)"A", 1, NULL, 1) == GRIM_E_INVALID);

    /* E = ceil(L * e_num / e_den) exactly: E * den >= L * num > (E - 1) * den */
    for (int k = 0; k < 200000; ++k) {
        const uint32_t L = (uint32_t)(next_u64() % 100000);
        const uint32_t den = 1 + (uint32_t)(next_u64() % 1000000);
        const uint32_t num = (uint32_t)(next_u64() % (2ull * den + 1));
        uint32_t E = 0;
        CHECK(grim_max_edits(L, num, den, &E) == GRIM_OK);
        const uint64_t prod = (uint64_t)L * num;
        CHECK((uint64_t)E * den >= prod);
        CHECK(E == 0 || (uint64_t)(E - 1) * den < prod);
        const uint32_t q = 4 + (uint32_t)(next_u64() % 4);
        int64_t T = 0;
        CHECK(grim_threshold(L, q, E, &T) == GRIM_OK);
        const int64_t ntok = L >= q ? (int64_t)L - q + 1 : 0;
        CHECK(T == ntok - (int64_t)q * E);
    }
    uint32_t E = 0;
    CHECK(grim_max_edits(100, 7, 100, &E) == GRIM_OK && E == 7); /* binary64 would give 8 */
    CHECK(grim_max_edits(10, 1, 0, &E) == GRIM_E_INVALID);
    CHECK(grim_max_edits(10, 1, 2, NULL) == GRIM_E_INVALID);
    CHECK(grim_threshold(10, 0, 1, NULL) == GRIM_E_INVALID);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host helpers: all checks passed\n");
    return 0;
}
