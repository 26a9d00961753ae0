"""Seed Location Checker on the GPU: survivor compaction against the oracle."""
import numpy as np
import pytest

import grim_synth as gs
import oracle
from tests.gpu_helpers import gpu_index, gpu_run, lib, oracle_run

pytestmark = pytest.mark.gpu


def _compact(g, w, bits_np, capacity=None):
    import torch
    batch = g.Batch.from_workload(w)
    bits = torch.from_numpy(np.ascontiguousarray(bits_np).view(np.int32)).cuda()
    sp, sr, sb, total = g.grim_compact_survivors(batch, bits, capacity)
    torch.cuda.synchronize()
    return sp.cpu().numpy().astype(np.uint64), sr.cpu().numpy().view(np.uint32), \
        sb.cpu().numpy().view(np.uint32), total


@pytest.mark.parametrize("name,scale", [("tiny", 1.0), ("batched", 0.002), ("mid", 0.01)])
def test_survivors_match_oracle(name, scale):
    g = lib()
    w = gs.make_workload(name, scale=scale)
    oc, ob, bad, _ = oracle_run(w)
    idx = gpu_index(w)
    c, b, rc, _ = gpu_run(idx, w)
    assert np.array_equal(b, ob)
    sp, sr, sb, total = _compact(g, w, b)
    op, orr, obin = oracle.survivors(ob, oc.size, w["cand_off"], w["cand_bin"])
    assert total == op.size
    assert np.array_equal(sp, op) and np.array_equal(sr, orr) and np.array_equal(sb, obin)


def test_survivors_edges():
    g = lib()
    ref = gs.reference(4, 200_000)
    rng = np.random.default_rng(2)
    n_reads = 300
    k = rng.integers(0, 9, n_reads).astype(np.uint32)
    k[[0, 5, 6, 7]] = 0                                    # reads without candidates
    off = gs.offsets_from_counts(k)
    n = int(off[-1])
    assert n % 32 != 0
    w = dict(codes=np.zeros(n_reads * 10, np.uint8), read_off=np.arange(n_reads, dtype=np.uint64) * 10,
             read_len=np.full(n_reads, 10, np.uint32), read_e=np.zeros(n_reads, np.uint32),
             e_den=10000, cand_off=off, cand_bin=rng.integers(0, 1000, n).astype(np.uint32))
    nw = (n + 31) // 32
    for pattern in ("none", "all", "random"):
        if pattern == "none":
            p = np.zeros(n, np.uint8)
        elif pattern == "all":
            p = np.ones(n, np.uint8)
        else:
            p = (rng.random(n) < 0.3).astype(np.uint8)
        words = oracle.pack_bitmask(p)
        dirty = words.copy()
        dirty[-1] |= np.uint32(~((1 << (n & 31)) - 1) & 0xFFFFFFFF)  # garbage past n_pairs
        want = oracle.survivors(words, n, off, w["cand_bin"])
        sp, sr, sb, total = _compact(g, w, dirty)
        assert total == want[0].size
        assert np.array_equal(sp, want[0]) and np.array_equal(sr, want[1]) and \
            np.array_equal(sb, want[2])
        if total > 3:
            cap = total // 2
            sp2, sr2, sb2, total2 = _compact(g, w, words, capacity=cap)
            assert total2 == total and sp2.size == cap
            assert np.array_equal(sp2, want[0][:cap]) and np.array_equal(sr2, want[1][:cap])
    # empty batch
    w0 = dict(codes=np.zeros(1, np.uint8), read_off=np.zeros(0, np.uint64),
              read_len=np.zeros(0, np.uint32), read_e=np.zeros(0, np.uint32), e_den=10000,
              cand_off=np.zeros(1, np.uint64), cand_bin=np.zeros(0, np.uint32))
    sp, sr, sb, total = _compact(g, w0, np.zeros(1, np.uint32))
    assert total == 0
