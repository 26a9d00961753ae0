// Host-side helpers of the C ABI: 2-bit packing of bases and the exact
// tolerance arithmetic of Section "Taking Errors into Account".  Plain C++ with
// no HIP dependency, so that the same file also builds on its own for the
// sanitizer tests.
#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "grim.h"

extern "C" uint64_t grim_packed_words(uint64_t n_bases) { return (n_bases + 15) / 16 + 1; }

extern "C" int grim_pack_bases(const uint8_t *bases, uint64_t n, uint32_t *words, int n_threads)
{
    if ((!bases && n) || !words)
        return GRIM_E_INVALID;
    uint8_t lut[256];
    std::memset(lut, 0xff, sizeof(lut));
    for (int c = 0; c < 4; ++c)
        lut[c] = (uint8_t)c;
    lut['A'] = lut['a'] = 0;
    lut['C'] = lut['c'] = 1;
    lut['G'] = lut['g'] = 2;
    lut['T'] = lut['t'] = 3;
    const uint64_t nw = grim_packed_words(n);
    if (n_threads <= 0)
        n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
    n_threads = (int)std::min<uint64_t>((uint64_t)n_threads, std::max<uint64_t>(1, nw / 65536 + 1));
    std::vector<int> bad(n_threads, 0);
    auto work = [&](int tid) {
        const uint64_t step = (nw + n_threads - 1) / n_threads;
        const uint64_t w0 = tid * step, w1 = std::min(nw, w0 + step);
        for (uint64_t w = w0; w < w1; ++w) {
            uint32_t x = 0;
            const uint64_t p0 = w * 16;
            for (int j = 0; j < 16; ++j) {
                const uint64_t p = p0 + j;
                if (p >= n)
                    break;
                const uint8_t c = lut[bases[p]];
                if (c > 3) {
                    bad[tid] = 1;
                    return;
                }
                x |= (uint32_t)c << (30 - 2 * j);
            }
            words[w] = x;
        }
    };
    if (n_threads == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (int t = 0; t < n_threads; ++t)
            th.emplace_back(work, t);
        for (auto &x : th)
            x.join();
    }
    for (int b : bad)
        if (b)
            return GRIM_E_BASE;
    return GRIM_OK;
}

extern "C" int grim_max_edits(uint32_t L, uint32_t e_num, uint32_t e_den, uint32_t *E)
{
    if (!E || e_den == 0)
        return GRIM_E_INVALID;
    *E = (uint32_t)(((uint64_t)e_num * L + e_den - 1) / e_den);
    return GRIM_OK;
}

extern "C" int grim_threshold(uint32_t L, uint32_t q, uint32_t E, int64_t *T)
{
    if (!T || q == 0)
        return GRIM_E_INVALID;
    const int64_t ntok = L >= q ? (int64_t)L - q + 1 : 0;
    *T = ntok - (int64_t)q * E;
    return GRIM_OK;
}
