"""Pins for the GRIM-Filter oracle: checks against what the paper and plain
mathematics fix, independent of the oracle's own code.

Each check takes an ``oracle.Oracle`` instance so that the same suite can be
run against copies of the oracle with planted mistakes (tests/test_oracle_mutants.py).
Paper: Kim et al., BMC Genomics 2018 (GRIM-Filter).
"""
import json
import math
import os
import random
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BASES = "ACGT"


def enc(s):
    return np.array([BASES.index(c) for c in s], dtype=np.uint8)


def dec(codes):
    return "".join(BASES[int(c)] for c in codes)


def brute_count(ref_s, lo, hi, read_s, q):
    """Number of token positions of the read whose q-gram occurs as a substring
    of ref[lo, hi) -- plain string search, no bitvector involved."""
    seg = ref_s[lo:hi]
    n = max(0, len(read_s) - q + 1)
    return sum(1 for i in range(n) if read_s[i:i + q] in seg)


def exact_E(L, e_num, e_den):
    """ceil(e * L) in exact rational arithmetic (Section 'Taking Errors into Account')."""
    return math.ceil(Fraction(e_num, e_den) * L)


def banded_edit_distance(a, b, band):
    """Levenshtein distance of strings a, b restricted to |i - j| <= band; returns
    band + 1 when the distance exceeds the band."""
    INF = band + 1
    n, m = len(a), len(b)
    if abs(n - m) > band:
        return INF
    prev = {j: j for j in range(0, min(m, band) + 1)}
    for i in range(1, n + 1):
        cur = {}
        for j in range(max(0, i - band), min(m, i + band) + 1):
            best = INF
            if j == 0:
                best = i
            else:
                if j - 1 in prev:
                    best = min(best, prev[j - 1] + (a[i - 1] != b[j - 1]))
                if j - 1 in cur:
                    best = min(best, cur[j - 1] + 1)
            if j in prev:
                best = min(best, prev[j] + 1)
            cur[j] = min(best, INF)
        prev = cur
    return min(prev.get(m, INF), INF)


def run_filter(orc, ref_codes, B, O, q, reads, e_nums, cands, e_den=10000):
    """Build the whole index of ref and run the oracle filter on a list of reads
    (code arrays) with per-read candidate bin lists."""
    idx = orc.build_index(ref_codes, B, O, q)
    lens = np.array([len(r) for r in reads], dtype=np.uint32)
    off = np.zeros(len(reads), dtype=np.uint64)
    if len(reads) > 1:
        off[1:] = np.cumsum(lens[:-1])
    codes = np.concatenate([np.asarray(r, dtype=np.uint8) for r in reads]) if reads else \
        np.zeros(0, np.uint8)
    if codes.size == 0:
        codes = np.zeros(1, np.uint8)
    coff = np.zeros(len(reads) + 1, dtype=np.uint64)
    coff[1:] = np.cumsum([len(c) for c in cands])
    cb = np.array([b for c in cands for b in c], dtype=np.uint32)
    if cb.size == 0:
        cb = np.zeros(1, np.uint32)
    return orc.filter_batch(idx, q, codes, off, lens, np.asarray(e_nums, np.uint32), e_den, coff, cb)


# ----------------------------------------------------------------------------
def check_golden_hand_vectors(orc):
    """Hand-derived bin vectors, sums and decisions (tests/golden/hand_vectors.json)."""
    with open(os.path.join(GOLDEN, "hand_vectors.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        ref = enc(case["ref"])
        q, B, O = case["q"], case["B"], case["O"]
        assert orc.num_bins(ref.size, B) == len(case["bins"]), case["name"]
        for b in case["bins"]:
            vec = orc.build_bin(ref, B, O, q, b["b"])
            assert vec.tobytes().hex() == b["bytes_hex"], (case["name"], b["b"], vec.tobytes().hex())
            for tok, bit in zip(b["tokens"], b["bits"]):
                assert orc.token(enc(tok), q) == bit, (tok, bit)
        nb = len(case["bins"])
        for rd in case["reads"]:
            codes = enc(rd["read"])
            L = len(rd["read"])
            assert orc.max_edits(L, rd["e_num"], rd["e_den"]) == rd["E"], rd
            assert orc.threshold(L, q, rd["E"]) == rd["T"], rd
            counts, passed, bad = run_filter(orc, ref, B, O, q, [codes], [rd["e_num"]],
                                             [list(range(nb))], e_den=rd["e_den"])
            assert bad == 0
            assert counts.tolist() == rd["counts"], (case["name"], rd["read"], counts.tolist())
            assert passed.tolist() == rd["pass"], (case["name"], rd["read"], passed.tolist())


def check_all_a_example(orc):
    """Section 'Determining the Accumulation Sum Threshold': an all-A read against a
    location that is all G except a single AAAAA gets one hit per token position
    (multiplicity counted), i.e. the sum equals the read's token count."""
    q = 5
    for L, expect in ((104, 100), (100, 96)):
        seg = "G" * 100 + "AAAAA" + "G" * 95  # one bin of 200 bp
        ref = enc(seg)
        read = enc("A" * L)
        counts, passed, _ = run_filter(orc, ref, 200, 0, q, [read], [500], [[0]])
        assert counts[0] == expect, (L, counts[0])
        assert passed[0] == 1
        # the read's tokens are all the single distinct token AAAAA
        assert brute_count(seg, 0, 200, "A" * L, q) == expect


def check_single_edit_token_loss(orc):
    """Fig. 5b caption (Section 'Taking Errors into Account'): relative to the
    perfect-match sum, one substitution or deletion removes q tokens and one
    insertion removes q - 1 (the new tokens being absent from the bin).  The
    bin X uses only A, C, G, and substituted or inserted bases are T, so every
    token touching such an edit is absent; deletions are redrawn until the q - 1
    junction tokens are absent (checked by substring search)."""
    rng = random.Random(7)
    for q in (4, 5):
        for kind in range(3):
            done = tries = 0
            while done < 8 and tries < 500:
                tries += 1
                X = "".join(rng.choice("ACG") for _ in range(60))
                ntok = len(X) - q + 1
                i = rng.randrange(q + 2, len(X) - q - 2)
                if kind == 0:
                    Y, expect = X[:i] + "T" + X[i + 1:], ntok - q
                elif kind == 1:
                    Y, expect = X[:i] + "T" + X[i:], ntok - (q - 1)
                else:
                    Y, expect = X[:i] + X[i + 1:], ntok - q
                if brute_count(X, 0, len(X), Y, q) != expect:
                    continue  # a junction token of a deletion occurs in X; draw again
                counts, _, _ = run_filter(orc, enc(X), len(X), 0, q, [enc(Y)], [0], [[0]])
                assert counts[0] == expect, (q, kind, counts[0], expect)
                done += 1
            assert done == 8, (q, kind)


def check_threshold_boundary(orc):
    """Section 'Taking Errors into Account': the threshold is the token count
    minus q per tolerated error, E = ceil(e L), and a location passes when the
    sum is greater than or equal to it.  A read with k substitutions at least q
    apart, each introducing a base absent from the bin, has sum ntok - q k
    exactly, so it must pass for k <= E and fail for k = E + 1."""
    rng = random.Random(11)
    cases = [(5, 150, 500), (5, 100, 500), (6, 250, 500), (5, 120, 1000), (4, 90, 700),
             (5, 250, 1000), (6, 150, 1000)]
    for q, L, e_num in cases:
        E = exact_E(L, e_num, 10000)
        ntok = L - q + 1
        for k in (E, E + 1):
            X = "".join(rng.choice("ACG") for _ in range(L))
            step = (L - 2 * q) // max(1, k)
            assert step >= q, "read too short for the construction"
            Y = list(X)
            for j in range(k):
                Y[q + j * step] = "T"
            Y = "".join(Y)
            assert brute_count(X, 0, L, Y, q) == ntok - q * k
            counts, passed, _ = run_filter(orc, enc(X), L, 0, q, [enc(Y)], [e_num], [[0]])
            assert counts[0] == ntok - q * k
            assert passed[0] == (1 if k <= E else 0), (q, L, e_num, k, E, counts[0])


def check_max_edits_exact(orc):
    """E = ceil(e L) with e a fraction: 0.07 x 100 is exactly 7 (binary64 gives 8)."""
    assert math.ceil(0.07 * 100) == 8  # the binary64 trap the integer rule avoids
    assert orc.max_edits(100, 700, 10000) == 7
    rng = random.Random(3)
    for _ in range(3000):
        L = rng.randrange(0, 2000)
        den = rng.choice([10, 100, 1000, 10000, 7, 9973])
        num = rng.randrange(0, den + 1)
        assert orc.max_edits(L, num, den) == exact_E(L, num, den), (L, num, den)


def check_threshold_table(orc):
    """Threshold values for the workloads' (q, e, L), from the closed form in exact
    rational arithmetic: T = (L - q + 1) - q * ceil(e L)."""
    table = {
        5: {(500, 100): 71, (500, 150): 106, (500, 250): 181,
            (1000, 100): 46, (1000, 150): 71, (1000, 250): 121},
        6: {(500, 100): 65, (500, 150): 97, (500, 250): 167,
            (1000, 100): 35, (1000, 150): 55, (1000, 250): 95},
    }
    for q, rows in table.items():
        for (e_num, L), T in rows.items():
            E = exact_E(L, e_num, 10000)
            assert (L - q + 1) - q * E == T
            assert orc.threshold(L, q, orc.max_edits(L, e_num, 10000)) == T, (q, e_num, L)
    # reads shorter than a token have no tokens; their threshold is -q E
    assert orc.num_tokens(3, 5) == 0 and orc.threshold(3, 5, 1) == -5
    assert orc.num_tokens(5, 5) == 1


def check_self_match(orc):
    """A read copied from inside a bin's span finds every one of its tokens."""
    rng = np.random.default_rng(5)
    for q in (3, 4, 5, 6):
        ref = rng.integers(0, 4, 3000).astype(np.uint8)
        B, O = 200, 160
        reads, cands = [], []
        for _ in range(50):
            b = int(rng.integers(0, ref.size // B - 1))
            L = int(rng.integers(q, 150))
            st = b * B + int(rng.integers(0, B + O - L + 1))
            reads.append(ref[st:st + L].copy())
            cands.append([b])
        counts, passed, _ = run_filter(orc, ref, B, O, q, reads, [0] * len(reads), cands)
        for r, c, p in zip(reads, counts, passed):
            assert c == r.size - q + 1 and p == 1


def check_bruteforce_small(orc):
    """Sums equal a plain substring-search count on random small genomes, and each
    bin vector has exactly as many set bits as its span has distinct q-grams."""
    rng = random.Random(13)
    for trial in range(60):
        q = rng.randrange(2, 8)
        G = rng.randrange(30, 400)
        alpha = BASES if trial % 3 else "AC"  # low-complexity genomes too
        ref_s = "".join(rng.choice(alpha) for _ in range(G))
        B = rng.randrange(5, 60)
        O = rng.randrange(0, 40)
        ref = enc(ref_s)
        nb = orc.num_bins(G, B)
        assert nb == -(-G // B)
        idx = orc.build_index(ref, B, O, q)
        for b in range(nb):
            lo, hi = b * B, min(G, (b + 1) * B + O)
            distinct = {ref_s[p:p + q] for p in range(lo, max(lo, hi - q + 1))}
            pop = int(np.unpackbits(idx[b]).sum())
            assert pop == len(distinct), (trial, b)
            assert pop <= min(4 ** q, max(0, hi - lo - q + 1))
        reads, cands, truth = [], [], []
        for _ in range(12):
            L = rng.randrange(0, 40)
            if rng.random() < 0.5 and G > L:
                st = rng.randrange(0, G - L + 1)
                rs = list(ref_s[st:st + L])
                for _ in range(rng.randrange(0, 3)):
                    if rs:
                        rs[rng.randrange(len(rs))] = rng.choice(BASES)
                rs = "".join(rs)
            else:
                rs = "".join(rng.choice(alpha) for _ in range(L))
            cb = [rng.randrange(nb) for _ in range(rng.randrange(0, 6))]
            reads.append(enc(rs) if rs else np.zeros(0, np.uint8))
            cands.append(cb)
            truth.append([brute_count(ref_s, b * B, min(G, (b + 1) * B + O), rs, q) for b in cb])
        counts, passed, bad = run_filter(orc, ref, B, O, q, reads, [0] * len(reads), cands)
        assert bad == 0
        flat = [c for t in truth for c in t]
        assert counts.tolist() == flat, (trial, counts.tolist(), flat)
        k = 0
        for rs, t in zip(reads, truth):
            ntok = max(0, len(rs) - q + 1)
            for c in t:
                assert 0 <= c <= ntok
                assert passed[k] == (1 if c >= ntok else 0)  # e = 0: T = ntok
                k += 1


def check_zero_false_reject(orc):
    """Section 'GRIM-Filter Operation': no location that truly holds the read
    within the error tolerance is rejected.  Planted reads whose banded edit
    distance to their source is at most E must pass in their true bin, given
    bins overlapping by at least L + E bases."""
    import grim_synth as gs
    rng_ref = gs.reference(101, 20_000, 0.3, 5, 300, 0.85, 0.98, 1)
    ref_s = dec(rng_ref)
    q, B = 5, 200
    for lengths, e_nums in (([100], [500]), ([150], [1000]), ([100, 150, 250], [500, 1000])):
        rd = gs.reads(202 + len(lengths), rng_ref, 400, lengths, e_nums, 10000, 1)
        Lmax = max(lengths)
        O = Lmax + exact_E(Lmax, max(e_nums), 10000)
        reads, cands, checked = [], [], []
        for r in range(400):
            L = int(rd["read_len"][r])
            off = int(rd["read_off"][r])
            codes = rd["codes"][off:off + L]
            z, span = int(rd["read_z"][r]), int(rd["read_span"][r])
            E = exact_E(L, int(rd["read_e"][r]), 10000)
            d = banded_edit_distance(dec(codes), ref_s[z:z + span], E)
            reads.append(codes)
            cands.append([z // B])
            checked.append(d <= E)
        assert sum(checked) == 400  # the generator plants at most floor(e L) edits
        counts, passed, _ = run_filter(orc, rng_ref, B, O, q, reads, list(rd["read_e"]), cands)
        for r in range(400):
            L = int(rd["read_len"][r])
            E = exact_E(L, int(rd["read_e"][r]), 10000)
            assert passed[r] == 1, (r, counts[r], L - q + 1 - q * E)


def check_monotone_overlap(orc):
    """Widening every bin (larger O) never lowers a sum: a bin's token set only grows."""
    rng = np.random.default_rng(17)
    ref = rng.integers(0, 4, 5000).astype(np.uint8)
    reads = [rng.integers(0, 4, 80).astype(np.uint8) for _ in range(30)]
    reads += [ref[s:s + 100].copy() for s in rng.integers(0, 4800, 30)]
    cands = [list(rng.integers(0, 25, 8)) for _ in reads]
    prev = None
    for O in (0, 20, 60, 120, 300):
        counts, _, _ = run_filter(orc, ref, 200, O, 5, reads, [0] * len(reads), cands)
        if prev is not None:
            assert np.all(counts >= prev)
        prev = counts


def check_footprint(orc):
    """Section 'Memory Footprint': 4^n bits per bin, times the number of bins.
    The paper's setting (n = 5, 450 x 2^16 bins) gives about 3.8 GB."""
    assert orc.vector_bytes(5) * 8 == 4 ** 5
    paper = orc.vector_bytes(5) * 450 * 2 ** 16
    assert abs(paper / 1e9 - 3.8) < 0.05
    assert orc.num_bins(3_100_000_000, 200) * orc.vector_bytes(5) == 1_984_000_000
    assert orc.num_bins(3_100_000_000, 1000) * orc.vector_bytes(6) == 1_587_200_000


def check_edges(orc):
    """Out-of-range bins give -1 / reject; the last bin is cut at the genome end;
    empty candidate lists are allowed."""
    ref_s = "ACGTTGCAACGGTACCATGA"
    ref = enc(ref_s)
    G, B, O, q = len(ref_s), 8, 4, 3
    nb = orc.num_bins(G, B)
    assert nb == 3
    last = orc.build_bin(ref, B, O, q, nb - 1)
    seg = ref_s[16:20]
    assert int(np.unpackbits(last).sum()) == len({seg[i:i + 3] for i in range(2)})
    reads = [enc("ACGTT"), enc("CATGA"), enc("GG")]
    counts, passed, bad = run_filter(orc, ref, B, O, q, reads, [0, 0, 0], [[0, 3, 99], [], [2]])
    assert bad == 2
    assert counts.tolist() == [3, -1, -1, 0]
    assert passed.tolist() == [1, 0, 0, 1]


def check_bitmask_packing(orc):
    """One bit per location in input order: bit k is bit k & 31 of word k >> 5."""
    passed = np.zeros(70, dtype=np.uint8)
    passed[[0, 5, 31, 32, 63, 64, 69]] = 1
    w = orc.pack_bitmask(passed)
    assert w.tolist() == [(1 << 0) | (1 << 5) | (1 << 31), (1 << 0) | (1 << 31), (1 << 0) | (1 << 5)]


def check_survivor_list(orc):
    """Seed Location Checker (Section 'Integration with a Full Read Mapper'): the
    passing locations, in input order, with their read and bin -- hand example."""
    passed = np.zeros(70, dtype=np.uint8)
    passed[[0, 5, 31, 32, 63, 64, 69]] = 1
    words = orc.pack_bitmask(passed)
    cand_off = np.array([0, 3, 3, 40, 70], dtype=np.uint64)   # read 1 has no candidates
    cand_bin = np.arange(70, dtype=np.uint32) * 3 + 1
    sp, sr, sb = orc.survivors(words, 70, cand_off, cand_bin)
    assert sp.tolist() == [0, 5, 31, 32, 63, 64, 69]
    assert sr.tolist() == [0, 2, 2, 2, 3, 3, 3]
    assert sb.tolist() == [1, 16, 94, 97, 190, 193, 208]
    sp, sr, sb = orc.survivors(orc.pack_bitmask(np.zeros(70, np.uint8)), 70, cand_off, cand_bin)
    assert sp.size == 0


def levenshtein(a, b):
    """Plain Levenshtein distance (full table)."""
    prev = list(range(len(b) + 1))
    for i in range(1, len(a) + 1):
        cur = [i] + [0] * len(b)
        for j in range(1, len(b) + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (a[i - 1] != b[j - 1]))
        prev = cur
    return prev[-1]


def check_edit_distance_in_bin(orc):
    """Verification distance: the minimum, over every substring of the bin's
    span, of the Levenshtein distance to the read -- by brute force over all
    substrings on small cases, plus hand values."""
    assert orc.edit_distance_in_bin(enc("AAACGTAAA"), 100, 0, 0, enc("ACGT")) == 0
    assert orc.edit_distance_in_bin(enc("AAAGTAAA"), 100, 0, 0, enc("ACGT")) == 1
    assert orc.edit_distance_in_bin(enc("TTTT"), 100, 0, 0, enc("ACGT")) == 3
    assert orc.edit_distance_in_bin(enc("TTTT"), 100, 0, 0, enc("")) == 0
    assert orc.edit_distance_in_bin(enc("ACCGT"), 100, 0, 0, enc("ACGT")) == 1
    rng = random.Random(19)
    for _ in range(120):
        G = rng.randrange(1, 40)
        ref_s = "".join(rng.choice("ACGT") for _ in range(G))
        B = rng.randrange(3, 20)
        O = rng.randrange(0, 10)
        b = rng.randrange(0, -(-G // B))
        lo, hi = b * B, min(G, (b + 1) * B + O)
        seg = ref_s[lo:hi]
        if rng.random() < 0.5 and len(seg) > 2:
            a = rng.randrange(0, len(seg) - 1)
            r = list(seg[a:a + rng.randrange(1, len(seg) - a + 1)])
            for _ in range(rng.randrange(0, 3)):
                r[rng.randrange(len(r))] = rng.choice("ACGT")
            read = "".join(r)
        else:
            read = "".join(rng.choice("ACGT") for _ in range(rng.randrange(0, 12)))
        want = min(levenshtein(read, seg[x:y]) for x in range(len(seg) + 1)
                   for y in range(x, len(seg) + 1))
        got = orc.edit_distance_in_bin(enc(ref_s), B, O, b, enc(read))
        assert got == want, (ref_s, B, O, b, read, got, want)


def check_seed_candidates(orc):
    """Seeding before the filter (Section 'Introduction', Fig. 1): bins of the
    locations of exact k-mer seeds at read offsets 0, k, 2k, ... -- against a
    plain substring scan of the reference, with dedup, order and cap."""
    rng = random.Random(23)
    for trial in range(40):
        G = rng.randrange(20, 600)
        alpha = "ACGT" if trial % 4 else "AC"
        ref_s = "".join(rng.choice(alpha) for _ in range(G))
        k = rng.randrange(2, 7)
        B = rng.randrange(3, 50)
        cap = rng.choice([1, 3, 1000])
        reads = []
        for _ in range(8):
            if rng.random() < 0.6 and G > 30:
                st = rng.randrange(0, G - 25)
                r = list(ref_s[st:st + rng.randrange(0, 25)])
                if r and rng.random() < 0.5:
                    r[rng.randrange(len(r))] = rng.choice("ACGT")
                reads.append("".join(r))
            else:
                reads.append("".join(rng.choice(alpha) for _ in range(rng.randrange(0, 20))))
        want = []
        for rs in reads:
            bins = set()
            for o in range(0, len(rs) - k + 1, k):
                seed = rs[o:o + k]
                for p in range(0, G - k + 1):
                    if ref_s[p:p + k] == seed:
                        z = min(max(p - o, 0), G - 1)
                        bins.add(z // B)
            want.append(sorted(bins)[:cap])
        codes = np.concatenate([enc(r) for r in reads] + [np.zeros(0, np.uint8)])
        lens = np.array([len(r) for r in reads], dtype=np.uint32)
        offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
        off, bins = orc.seed_candidates(enc(ref_s), k, codes, offs, lens, B, cap)
        got = [bins[int(off[i]):int(off[i + 1])].tolist() for i in range(len(reads))]
        assert got == want, (trial, got, want)


ALL_CHECKS = [
    check_golden_hand_vectors,
    check_all_a_example,
    check_single_edit_token_loss,
    check_threshold_boundary,
    check_max_edits_exact,
    check_threshold_table,
    check_self_match,
    check_bruteforce_small,
    check_zero_false_reject,
    check_monotone_overlap,
    check_footprint,
    check_edges,
    check_bitmask_packing,
    check_survivor_list,
    check_edit_distance_in_bin,
    check_seed_candidates,
]
