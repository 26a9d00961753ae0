"""Seeding on the GPU (candidate generation before the filter) against the
oracle, and the seeded candidates fed through the filter."""
import numpy as np
import pytest

import grim_synth as gs
import oracle
from tests.gpu_helpers import assert_same, gpu_index, gpu_run, lib, oracle_run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,G,n_reads,cap", [(12, 2_000_000, 3000, 4096), (8, 300_000, 2000, 37),
                                             (5, 50_000, 500, 4096)])
def test_seed_candidates_match_oracle(k, G, n_reads, cap):
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
