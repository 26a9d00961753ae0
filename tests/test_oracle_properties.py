"""Randomised properties of the oracle (CPU only), over small references and
reads drawn by hypothesis: the accumulation sum of a (read, bin) pair equals a
count done without bitvectors, stays within [0, number of tokens], never drops
when the bins' overlap grows, and a read copied from inside a bin's span finds
every one of its tokens (the filter's steps in Section "GRIM-Filter Operation";
bins in Section "Genome Metadata Representation")."""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle

BASES = st.integers(min_value=0, max_value=3)


def substring_count(ref, lo, hi, read, q):
    """Token positions of the read whose q-gram occurs wholly inside ref[lo:hi]."""
    span = bytes(ref[lo:hi])
    n = 0
    for i in range(len(read) - q + 1):
        if bytes(read[i:i + q]) in span:
            n += 1
    return n


@st.composite
def case(draw):
    q = draw(st.integers(min_value=2, max_value=6))
    ref = np.array(draw(st.lists(BASES, min_size=q, max_size=300)), dtype=np.uint8)
    B = draw(st.integers(min_value=1, max_value=60))
    O = draw(st.integers(min_value=0, max_value=40))
    n_bins = (ref.size + B - 1) // B
    b = draw(st.integers(min_value=0, max_value=n_bins - 1))
    read = np.array(draw(st.lists(BASES, min_size=0, max_size=80)), dtype=np.uint8)
    return q, ref, B, O, b, read


@settings(max_examples=300, deadline=None)
@given(case())
def test_sum_equals_substring_count(c):
    q, ref, B, O, b, read = c
    vec = oracle.build_bin(ref, B, O, q, b)
    s = oracle.count(vec, q, read)
    lo, hi = b * B, min(ref.size, (b + 1) * B + O)
    assert s == substring_count(ref, lo, hi, read, q)
    assert 0 <= s <= max(0, read.size - q + 1)


@settings(max_examples=200, deadline=None)
@given(case(), st.integers(min_value=1, max_value=50))
def test_sum_monotone_in_overlap(c, extra):
    q, ref, B, O, b, read = c
    s0 = oracle.count(oracle.build_bin(ref, B, O, q, b), q, read)
    s1 = oracle.count(oracle.build_bin(ref, B, O + extra, q, b), q, read)
    assert s1 >= s0


@settings(max_examples=200, deadline=None)
@given(case(), st.data())
def test_read_from_inside_the_span_finds_every_token(c, data):
    q, ref, B, O, b, _ = c
    lo, hi = b * B, min(ref.size, (b + 1) * B + O)
    if hi - lo < q:
        return
    a = data.draw(st.integers(min_value=lo, max_value=hi - q))
    e = data.draw(st.integers(min_value=a + q, max_value=hi))
    read = ref[a:e]
    s = oracle.count(oracle.build_bin(ref, B, O, q, b), q, read)
    assert s == read.size - q + 1
