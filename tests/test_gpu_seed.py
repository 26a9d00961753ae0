"""Seeding on the GPU (candidate generation before the filter) against the
oracle, and the seeded candidates fed through the filter."""
import numpy as np
import pytest

import grim_synth as gs
import oracle
from tests.gpu_helpers import assert_same, gpu_index, gpu_run, lib, oracle_run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,G,n_reads,cap", [(12, 2_000_000, 3000, 4096), (8, 300_000, 2000, 37),
                                             (5, 50_000, 500, 4096), (4, 60_000, 300, 4096),
                                             (4, 60_000, 300, 100)])
def test_seed_candidates_match_oracle(k, G, n_reads, cap):
    """Reads of 5-150 bases; at k = 5 most reads collect 500-2000 hits (sorted
    in LDS), at k = 4 several thousand (sorted in global memory); the caps cut
    long lists."""
    g = lib()
    ref = gs.reference(17, G, 0.2, 20, 300, 0.85, 0.98)
    rd = gs.reads(18, ref, n_reads, [100, 150, 37, 5], [500])
    B = 200
    batch = g.Batch(rd["codes"], rd["read_off"], rd["read_len"], rd["read_e"], gs.E_DEN,
                    np.zeros(n_reads + 1, np.uint64), np.zeros(0, np.uint32))
    si = g.SeedIndex(ref, k)
    cands = g.grim_seed_candidates(si, batch, B, cap)
    off, bins = cands.to_host()
    w_off, w_bins = oracle.seed_candidates(ref, k, rd["codes"], rd["read_off"], rd["read_len"], B, cap)
    assert np.array_equal(off, w_off)
    assert np.array_equal(bins, w_bins)


def test_seeded_mid_workload_filters_like_oracle():
    """mid recipe (12-mer seeds, 200-bp bins) at 1 %: GPU seeding -> GPU filter,
    against oracle seeding -> oracle filter."""
    g = lib()
    w = gs.make_workload("mid", scale=0.01)
    batch = g.Batch.from_workload(w)
    si = g.SeedIndex(w["ref"], 12)
    cands = g.grim_seed_candidates(si, batch, w["B"], 4096)
    off, bins = cands.to_host()
    w_off, w_bins = oracle.seed_candidates(w["ref"], 12, w["codes"], w["read_off"], w["read_len"],
                                           w["B"], 4096)
    assert np.array_equal(off, w_off) and np.array_equal(bins, w_bins)
    # the generator's host seeding gives the same lists
    assert np.array_equal(off, w["cand_off"]) and np.array_equal(bins, w["cand_bin"])
    idx = gpu_index(w)
    fb = g.batch_with_candidates(batch, cands)
    out = gpu_run(idx, w, batch=fb)
    assert out[2] == 0
    assert_same(out, oracle_run(w), "seeded mid")


def test_seed_candidates_hit_count_edges():
    """Hit lists of every size class: a poly-A stretch makes the all-A seed hit
    tens of thousands of times (a list sorted in global memory), reads with
    hit counts on both sides of every class boundary (64 one per lane, 128 /
    256 / 512 two to eight per lane, 1024 / 2048 sixteen or thirty-two per lane
    in one wavefront, 8192 in a workgroup's LDS, beyond in global memory), and
    reads without any hit; every list against the oracle."""
    g = lib()
    k, B = 12, 100
    ref = gs.reference(23, 1_400_000)
    ref[100_000:130_000] = 0                      # 30,000 A: the all-A 12-mer hits 29,989 times
    reads = [np.zeros(100, np.uint8), np.zeros(24, np.uint8), ref[5_000:5_100].copy(),
             np.full(30, 3, np.uint8), ref[60_000:60_011].copy()]
    # reads made of copies of one 12-mer planted n times in the reference
    rng = np.random.default_rng(3)
    p_next = 140_000
    for n_copies in (64, 65, 128, 129, 256, 257, 512, 513, 1024, 1025, 2048, 2049, 8192, 8193):
        kmer = rng.integers(0, 4, 12).astype(np.uint8)
        kmer[0] = 1                               # not the all-A k-mer
        for p0 in range(p_next, p_next + 13 * n_copies, 13):
            ref[p0:p0 + 12] = kmer
        p_next += 13 * n_copies + 1000
        reads.append(np.concatenate([kmer, np.full(3, 2, np.uint8)]))
    assert p_next < ref.size
    codes = np.concatenate(reads)
    lens = np.array([len(r) for r in reads], np.uint32)
    offs = np.zeros(len(reads), np.uint64)
    offs[1:] = np.cumsum(lens[:-1])
    batch = g.Batch(codes, offs, lens, np.zeros(len(reads), np.uint32), gs.E_DEN,
                    np.zeros(len(reads) + 1, np.uint64), np.zeros(0, np.uint32))
    si = g.SeedIndex(ref, k)
    for cap in (4096, 50):
        cands = g.grim_seed_candidates(si, batch, B, cap)
        off, bins = cands.to_host()
        w_off, w_bins = oracle.seed_candidates(ref, k, codes, offs, lens, B, cap)
        assert np.array_equal(off, w_off)
        assert np.array_equal(bins, w_bins)


def test_seed_candidates_item_layouts():
    """Every item layout gives the oracle's lists: a fixed number of seed slots
    per read (max_len / k, used while reads x slots stays within 2^26) in
    wavefront groups (max_len 150: 12 slots) or one read at a time (max_len
    1000: 83 slots), and the counted layout (max_len = 8192 over 100,000 reads
    exceeds 2^26 slots); a read longer than max_len gets no candidates."""
    g = lib()
    k, B, n = 12, 200, 100_000
    ref = gs.reference(31, 2_000_000, 0.2, 20, 300, 0.85, 0.98)
    rd = gs.reads(32, ref, n, [100, 150, 37], [500])
    w_off, w_bins = oracle.seed_candidates(ref, k, rd["codes"], rd["read_off"], rd["read_len"], B,
                                           4096)
    si = g.SeedIndex(ref, k)
    for max_len in (150, 1000, 8192):
        batch = g.Batch(rd["codes"], rd["read_off"], rd["read_len"], rd["read_e"], gs.E_DEN,
                        np.zeros(n + 1, np.uint64), np.zeros(0, np.uint32), max_len=max_len)
        off, bins = g.grim_seed_candidates(si, batch, B, 4096).to_host()
        assert np.array_equal(off, w_off), max_len
        assert np.array_equal(bins, w_bins), max_len
    # max_len below some reads' length: those reads get no candidates
    batch = g.Batch(rd["codes"], rd["read_off"], rd["read_len"], rd["read_e"], gs.E_DEN,
                    np.zeros(n + 1, np.uint64), np.zeros(0, np.uint32), max_len=120)
    off, bins = g.grim_seed_candidates(si, batch, B, 4096).to_host()
    cnt, w_cnt = np.diff(off.astype(np.int64)), np.diff(w_off.astype(np.int64))
    long_reads = rd["read_len"] > 120
    assert np.all(cnt[long_reads] == 0)
    assert np.array_equal(cnt[~long_reads], w_cnt[~long_reads])


def test_seed_candidate_buffers_kept_and_reused():
    """Freed lists' buffers serve the next lists of the same seed index: lists
    made after a free (larger, equal and smaller batches) equal the oracle's,
    and a list that outlives its seed index stays readable until it is freed."""
    g = lib()
    k, B = 12, 200
    ref = gs.reference(41, 1_000_000, 0.2, 20, 300, 0.85, 0.98)
    rd = gs.reads(42, ref, 20_000, [100, 150], [500])

    def batch(n):
        o_end = int(rd["read_off"][n - 1]) + int(rd["read_len"][n - 1])
        return (rd["codes"][:o_end], rd["read_off"][:n], rd["read_len"][:n],
                g.Batch(rd["codes"][:o_end], rd["read_off"][:n], rd["read_len"][:n],
                        np.zeros(n, np.uint32), gs.E_DEN, np.zeros(n + 1, np.uint64),
                        np.zeros(0, np.uint32)))

    si = g.SeedIndex(ref, k)
    kept = []
    for n in (20_000, 20_000, 5_000, 20_000, 700, 12_000):
        codes, offs, lens, b = batch(n)
        c = g.grim_seed_candidates(si, b, B, 4096)
        off, bins = c.to_host()
        w_off, w_bins = oracle.seed_candidates(ref, k, codes, offs, lens, B, 4096)
        assert np.array_equal(off, w_off) and np.array_equal(bins, w_bins), n
        if n == 700:
            kept.append((c, w_off, w_bins))   # lives past the index
        else:
            c.free()
    si.free()
    c, w_off, w_bins = kept[0]
    off, bins = c.to_host()
    assert np.array_equal(off, w_off) and np.array_equal(bins, w_bins)
    c.free()
