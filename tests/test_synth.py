"""The seeded generators: deterministic, thread-count independent, and shaped
as the workloads describe (CPU only)."""
import numpy as np

import grim_synth as gs


def test_reference_thread_invariant():
    a = gs.reference(9, 200_003, 0.45, 50, 300, 0.85, 0.98, n_threads=1)
    b = gs.reference(9, 200_003, 0.45, 50, 300, 0.85, 0.98, n_threads=7)
    assert np.array_equal(a, b)
    assert a.max() <= 3
    c = gs.reference(10, 200_003, 0.45, 50, 300, 0.85, 0.98, n_threads=7)
    assert not np.array_equal(a, c)


def test_repeats_are_planted():
    # with repeats the genome holds many near-copies of a few families: far more
    # repeated 16-mers than an iid genome of the same size
    iid = gs.reference(4, 300_000, 0.0, 1, 300, 0.85, 0.98)
    rep = gs.reference(4, 300_000, 0.45, 20, 300, 0.85, 0.98)

    def dup16(x):
        k = np.zeros(x.size - 15, dtype=np.uint64)
        for j in range(16):
            k = k * np.uint64(4) + x[j:x.size - 15 + j].astype(np.uint64)
        return k.size - np.unique(k).size

    assert dup16(rep) > 50 * max(1, dup16(iid))


def test_reads_and_candidates():
    ref = gs.reference(1, 100_000)
    rd = gs.reads(3, ref, 5000, [100, 150, 250], [500, 1000], n_threads=3)
    rd2 = gs.reads(3, ref, 5000, [100, 150, 250], [500, 1000], n_threads=1)
    for k in rd:
        assert np.array_equal(rd[k], rd2[k]), k
    assert set(np.unique(rd["read_len"])) == {100, 150, 250}
    budget = rd["read_len"].astype(np.int64) * rd["read_e"] // gs.E_DEN
    assert np.all(rd["read_edits"] <= budget)
    assert np.all(rd["read_z"] + rd["read_span"] <= ref.size)
    k = gs.cand_counts_zipf(4, 200_000, 1.2, 4096)
    assert k.min() >= 1 and k.max() <= 4096
    assert 6 <= np.median(k) <= 10          # Zipf(1.2) on 1..4096: median 8
    assert 150 < k.mean() < 270             # mean about 209
    off = gs.offsets_from_counts(k[:5000])
    cb, tp = gs.cand_random(5, off, rd["read_z"], 200, 500)
    assert cb.max() < 500
    assert np.array_equal(cb[tp.astype(np.int64)], (rd["read_z"] // 200).astype(np.uint32))


def test_seeded_candidates_contain_true_bin():
    w = gs.make_workload("mid", scale=0.002)
    off, cb = w["cand_off"], w["cand_bin"]
    hits = 0
    for r in range(w["read_len"].size):
        bins = cb[off[r]:off[r + 1]]
        if (w["read_z"][r] // w["B"]) in bins:
            hits += 1
    assert hits / w["read_len"].size > 0.9
    assert np.all(np.diff(off.astype(np.int64)) <= 4096)
