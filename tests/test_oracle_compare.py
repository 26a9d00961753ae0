"""The chunked, threaded comparison driver around the oracle (CPU only): it
must report zero mismatches for the oracle's own results, find every planted
count or pass-bit difference at its pair index wherever the chunks fall, and
cover exactly the requested read range."""
import numpy as np
import pytest

import grim_synth as gs
import oracle


@pytest.fixture(scope="module")
def case():
    w = gs.make_workload("batched", scale=0.0004)
    oidx = oracle.build_index(w["ref"], w["B"], w["O"], w["q"], n_threads=4)
    c, p, bad = oracle.filter_batch(oidx, w["q"], w["codes"], w["read_off"], w["read_len"],
                                    w["read_e"], w["e_den"], w["cand_off"], w["cand_bin"],
                                    n_threads=4)
    assert bad == 0
    return w, oidx, c, oracle.pack_bitmask(p)


def run(case, counts, bits, **kw):
    w, oidx = case[0], case[1]
    return oracle.filter_compare(oidx, w["q"], w["codes"], w["read_off"], w["read_len"],
                                 w["read_e"], w["e_den"], w["cand_off"], w["cand_bin"], counts,
                                 bits, **kw)


@pytest.mark.parametrize("chunk", [1, 777, 1 << 22])
@pytest.mark.parametrize("threads", [1, 5])
def test_identical_results_compare_clean(case, chunk, threads):
    w, _, c, b = case
    res = run(case, c, b, n_threads=threads, chunk_pairs=chunk)
    assert res["pairs"] == int(w["cand_off"][-1])
    assert res["count_mismatches"] == 0 and res["bit_mismatches"] == 0 and not res["first"]


@pytest.mark.parametrize("chunk", [13, 4096])
def test_planted_differences_are_found(case, chunk):
    w, _, c, b = case
    n = c.size
    c2, b2 = c.copy(), b.copy()
    bad_counts = [0, 5, n // 3, n - 1]
    bad_bits = [1, 8, 31, 32, n // 2 + 3, n - 2]
    for k in bad_counts:
        c2[k] += 1
    for k in bad_bits:
        b2[k >> 5] ^= np.uint32(1 << (k & 31))
    res = run(case, c2, b2, n_threads=3, chunk_pairs=chunk)
    assert res["count_mismatches"] == len(bad_counts)
    assert res["bit_mismatches"] == len(bad_bits)
    assert set(res["first"]) <= set(bad_counts) | set(bad_bits)
    assert len(res["first"]) == 8


def test_read_range(case):
    w, _, c, b = case
    off = w["cand_off"]
    r0, r1 = 17, w["read_len"].size - 23
    c2 = c.copy()
    c2[:int(off[r0])] = -9          # outside the range: not looked at
    c2[int(off[r1]):] = -9
    res = run(case, c2, b, r_begin=r0, r_end=r1, n_threads=2, chunk_pairs=1000)
    assert res["pairs"] == int(off[r1]) - int(off[r0]) and res["reads"] == r1 - r0
    assert res["count_mismatches"] == 0 and res["bit_mismatches"] == 0
