"""Planted-mistake check of the oracle's pins (CPU only).

Each mutant is a copy of oracle/oracle.c with one plausible mistake (a dropped
term, a wrong comparison, an off-by-one, a transposed index).  The copy is
compiled into a temporary library and the pin suite must reject it.
"""
import os

import pytest

import oracle
from tests import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "token_base_order_reversed": ("t = t * 4 + codes[j];", "t = t * 4 + codes[q - 1 - j];"),
    "bin_overlap_dropped": ("uint64_t hi = (b + 1) * B + O;", "uint64_t hi = (b + 1) * B;"),
    "bin_start_shifted": ("uint64_t lo = b * B;", "uint64_t lo = b * B + 1;"),
    "bin_last_token_dropped": ("for (uint64_t p = lo; p + q <= hi; p++)",
                               "for (uint64_t p = lo; p + q < hi; p++)"),
    "bit_order_within_byte": ("vec[t >> 3] |= (uint8_t)(1u << (t & 7));",
                              "vec[t >> 3] |= (uint8_t)(1u << (7 - (t & 7)));"),
    "edits_floor_not_ceil": ("return (uint32_t)((num + e_den - 1) / e_den);",
                             "return (uint32_t)(num / e_den);"),
    "edits_ceil_overshoot": ("return (uint32_t)((num + e_den - 1) / e_den);",
                             "return (uint32_t)((num + e_den) / e_den);"),
    "tokens_off_by_one": ("int64_t n = (int64_t)L - ((int64_t)q - 1);",
                          "int64_t n = (int64_t)L - (int64_t)q;"),
    "threshold_q_minus_one_per_error": ("return oracle_num_tokens(L, q) - (int64_t)q * (int64_t)E;",
                                        "return oracle_num_tokens(L, q) - ((int64_t)q - 1) * (int64_t)E;"),
    "threshold_sign": ("return oracle_num_tokens(L, q) - (int64_t)q * (int64_t)E;",
                       "return oracle_num_tokens(L, q) + (int64_t)q * (int64_t)E;"),
    "pass_strict_greater": ("pass[k] = (sum >= T) ? 1 : 0;", "pass[k] = (sum > T) ? 1 : 0;"),
    "sum_drops_last_token": ("for (int64_t i = 0; i < ntok; i++) {",
                             "for (int64_t i = 0; i + 1 < ntok; i++) {"),
    "sum_ignores_repeats": ("sum += bit;                                      /* step 4 */",
                            "if (i > 0 && t == oracle_token(read + i - 1, q)) bit = 0;\n"
                            "        sum += bit;"),
    "bins_floor": ("return (G + B - 1) / B;", "return G / B;"),
    "bitmask_msb_first": ("words[k >> 5] |= 1u << (k & 31);",
                          "words[k >> 5] |= 1u << (31 - (k & 31));"),
    "survivor_read_off_by_one": ("surv_read[n] = (uint32_t)r;", "surv_read[n] = (uint32_t)(r + 1);"),
    "survivor_bit_inverted": ("if (!((words[k >> 5] >> (k & 31)) & 1u))", "if (((words[k >> 5] >> (k & 31)) & 1u))"),
    "verify_span_without_overlap": ("uint64_t hi = B * (b + 1) + O;", "uint64_t hi = B * (b + 1);"),
    "verify_free_start_dropped": ("row[j] = 0;                                   /* D[0][j] = 0 */",
                                  "row[j] = (int32_t)j;"),
    "verify_substitution_free": ("int32_t sub = diag + (read[i - 1] != ref[lo + j - 1] ? 1 : 0);",
                                 "int32_t sub = diag;"),
    "verify_last_column_only": ("    int32_t m = row[0];\n    for (uint64_t j = 1; j <= n; j++)\n        if (row[j] < m)\n            m = row[j];",
                                "    int32_t m = row[n];"),
    "seed_no_clamp_low": ("                if (z < 0)\n                    z = 0;", "                if (z < 0)\n                    z = -z;"),
    "seed_step_one": ("for (uint32_t o = 0; o + k <= L; o += k) {", "for (uint32_t o = 0; o + k <= L; o += 1) {"),
    "seed_no_dedup": ("            if (i > 0 && buf[i] == buf[i - 1])\n                continue;", ""),
    "bin_wrong_vector": ("const uint8_t *vec = index + b * nbytes;     /* step 2 */",
                         "const uint8_t *vec = index + (b ^ 1) % n_bins * nbytes;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation site for {name} not found exactly once"
    src = tmp_path / "oracle_mut.c"
    src.write_text(text.replace(old, new))
    lib = str(tmp_path / "liboracle_mut.so")
    oracle.build(str(src), lib)
    orc = oracle.Oracle(lib)
    caught = []
    for check in oracle_pins.ALL_CHECKS:
        try:
            check(orc)
        except AssertionError:
            caught.append(check.__name__)
            break
    assert caught, f"no pin rejects mutant {name}"
