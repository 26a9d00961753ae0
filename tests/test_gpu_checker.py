"""Seed Location Checker on the GPU: survivor compaction against the oracle."""
import numpy as np
import pytest

import grim_synth as gs
import oracle
from tests.gpu_helpers import custom_workload, gpu_index, gpu_run, lib, oracle_run

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


def test_survivors_many_reads_per_block():
    """Workgroups of the emit pass cover 32768 pairs; stretches of reads with
    0-2 candidates put more reads in one workgroup than its staged offsets hold
    (then the reads are searched in global memory), stretches of long candidate
    lists few; both against the oracle, for sparse and dense pass patterns."""
    g = lib()
    rng = np.random.default_rng(9)
    parts = [rng.integers(0, 3, 60_000), rng.integers(100, 4097, 60),
             rng.integers(0, 2, 40_000), np.zeros(5000, np.int64), rng.integers(0, 40, 3000)]
    k = np.concatenate(parts).astype(np.uint32)
    n_reads = k.size
    off = gs.offsets_from_counts(k)
    n = int(off[-1])
    w = dict(codes=np.zeros(n_reads * 10, np.uint8),
             read_off=np.arange(n_reads, dtype=np.uint64) * 10,
             read_len=np.full(n_reads, 10, np.uint32), read_e=np.zeros(n_reads, np.uint32),
             e_den=10000, cand_off=off, cand_bin=rng.integers(0, 1 << 30, n).astype(np.uint32))
    for density in (0.015, 0.5):
        p = (rng.random(n) < density).astype(np.uint8)
        words = oracle.pack_bitmask(p)
        want = oracle.survivors(words, n, off, w["cand_bin"])
        sp, sr, sb, total = _compact(g, w, words)
        assert total == want[0].size
        assert np.array_equal(sp, want[0]) and np.array_equal(sr, want[1]) and \
            np.array_equal(sb, want[2]), density


def _verify_gpu(g, idx, w, surv_read, surv_bin, max_len=None):
    import torch
    batch = g.Batch.from_workload(w, max_len=max_len)
    sr = torch.from_numpy(np.ascontiguousarray(surv_read, dtype=np.uint32).view(np.int32)).cuda()
    sb = torch.from_numpy(np.ascontiguousarray(surv_bin, dtype=np.uint32).view(np.int32)).cuda()
    dist, ok = g.grim_verify_survivors(idx, batch, sr, sb, len(surv_read))
    torch.cuda.synchronize()
    return dist.cpu().numpy(), ok.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("name,scale", [("tiny", 1.0), ("batched", 0.002)])
def test_verify_survivors_match_oracle(name, scale):
    import torch
    g = lib()
    w = gs.make_workload(name, scale=scale)
    idx = gpu_index(w)
    idx.attach_reference(w["ref"])
    batch = g.Batch.from_workload(w)
    c, bits = g.alloc_outputs(batch.n_pairs)
    ws = g.alloc_workspace(idx, batch.n_pairs)
    g.grim_filter_batch(idx, batch, c, bits, ws)
    sp, sr, sb, total = g.grim_compact_survivors(batch, bits)
    dist, ok = g.grim_verify_survivors(idx, batch, sr, sb, total)
    torch.cuda.synchronize()
    srn = sr.cpu().numpy().view(np.uint32)
    sbn = sb.cpu().numpy().view(np.uint32)
    want = oracle.verify(w["ref"], w["B"], w["O"], w["codes"], w["read_off"], w["read_len"],
                         w["read_e"], w["e_den"], srn, sbn)
    got = dist.cpu().numpy()
    assert np.array_equal(got, want), np.nonzero(got != want)[0][:5]
    E = (w["read_e"].astype(np.int64) * w["read_len"] + w["e_den"] - 1) // w["e_den"]
    okb = ok.cpu().numpy().view(np.uint32)
    okn = (okb[np.arange(total) >> 5] >> (np.arange(total) & 31)) & 1
    assert np.array_equal(okn.astype(bool), want <= E[srn])
    # every read's true location survives and verifies (planted edits <= E)
    spn = sp.cpu().numpy()
    true_set = set(w["true_pair"].tolist())
    verified_true = sum(1 for k, o in zip(spn.tolist(), okn.tolist()) if k in true_set and o)
    assert verified_true == len(true_set)


def test_verify_edges():
    g = lib()
    ref = gs.reference(8, 60_000, 0.3, 5, 300, 0.85, 0.98)
    q, B, O = 5, 200, 600
    nb = (ref.size + B - 1) // B
    rng = np.random.default_rng(4)
    reads, cands = [], []
    for L in (0, 1, 5, 63, 64, 65, 128, 129, 256, 300, 512):
        st = int(rng.integers(0, ref.size - L - 1))
        r = ref[st:st + L].copy()
        if L > 10:
            for _ in range(3):
                r[int(rng.integers(0, L))] = int(rng.integers(0, 4))
        reads.append(r)
        cands.append([st // B, int(rng.integers(0, nb)), nb - 1])
    e = [1000] * len(reads)
    w = custom_workload(ref, q, B, O, reads, cands, e)
    idx = g.grim_build_bins(ref, q, B, O)
    idx.attach_reference(ref)
    off = w["cand_off"]
    surv_read = np.repeat(np.arange(len(reads), dtype=np.uint32), np.diff(off.astype(np.int64)))
    surv_bin = w["cand_bin"].copy()
    surv_bin[4] = nb + 3  # out of range -> -1
    for max_len in (512,):
        dist, okb = _verify_gpu(g, idx, w, surv_read, surv_bin, max_len=max_len)
        want = oracle.verify(ref, B, O, w["codes"], w["read_off"], w["read_len"], w["read_e"],
                             w["e_den"], surv_read, np.where(surv_bin < nb, surv_bin, 0))
        want[4] = -1
        assert np.array_equal(dist, want), (dist, want)
    # short batches use the narrower kernels (1 and 2 blocks of 64 rows)
    for Lmax in (64, 128):
        sel = [i for i, r in enumerate(reads) if len(r) <= Lmax]
        w2 = custom_workload(ref, q, B, O, [reads[i] for i in sel], [cands[i] for i in sel],
                             [e[i] for i in sel])
        off2 = w2["cand_off"]
        sr2 = np.repeat(np.arange(len(sel), dtype=np.uint32), np.diff(off2.astype(np.int64)))
        dist, _ = _verify_gpu(g, idx, w2, sr2, w2["cand_bin"], max_len=Lmax)
        want = oracle.verify(ref, B, O, w2["codes"], w2["read_off"], w2["read_len"],
                             w2["read_e"], w2["e_den"], sr2, w2["cand_bin"])
        assert np.array_equal(dist, want)
    # reads longer than 512 are not supported by the alignment check
    with pytest.raises(g.GrimError) as ex:
        _verify_gpu(g, idx, w, surv_read, surv_bin, max_len=600)
    assert ex.value.code == g.GRIM_E_UNSUPPORTED


@pytest.mark.parametrize("n_surv,max_len", [(2_500_037, 256), (70_000_037, 256),
                                            (2_500_037, 512)])
def test_verify_many_chunks(n_surv, max_len):
    """Long survivor lists for the alignment check: 2.5M (plus 37) survivors
    give some 2,400 sorted chunks of 1024, one per workgroup, and a ragged
    last one; 70M (plus 37) exceed 64 times the resident workgroups, so that
    each workgroup takes a run of chunks.  Survivors are drawn from 40,000
    distinct read/bin pairs so that the oracle runs once per distinct pair;
    read lengths 0-200 mixed at random, a few read ids and bin ids out of
    range (distance -1, not verified), every distance and pass bit compared.
    With max_len 512 the reads are 0-400 bases and the 8-block kernel runs
    (its column scan compiled for each of 16 first words)."""
    import torch
    g = lib()
    rng = np.random.default_rng(77)
    ref = gs.reference(21, 200_000, 0.3, 5, 200, 0.85, 0.98)
    q, B, O = 4, 8, 4
    nb = (ref.size + B - 1) // B
    n_reads = 4000
    reads, cands, es, origin = [], [], [], []
    for _ in range(n_reads):
        L = int(rng.integers(0, 201 if max_len == 256 else 401))
        st = int(rng.integers(0, ref.size - L))
        origin.append(st)
        r = ref[st:st + L].copy()
        for _ in range(int(rng.integers(0, 4))):
            if L:
                r[int(rng.integers(0, L))] = int(rng.integers(0, 4))
        reads.append(r)
        cands.append([])
        es.append(int(rng.choice([0, 500, 1000, 2500])))
    w = custom_workload(ref, q, B, O, reads, cands, es)
    n_pairs = 40_000
    pr = rng.integers(0, n_reads, n_pairs).astype(np.uint32)
    pb = rng.integers(0, nb, n_pairs).astype(np.uint32)
    # a third of the pairs at the read's own bin, so that many verify
    near = rng.random(n_pairs) < 1 / 3
    pb[near] = np.array(origin, dtype=np.int64)[pr[near]] // B
    want_pair = oracle.verify(ref, B, O, w["codes"], w["read_off"], w["read_len"], w["read_e"],
                              w["e_den"], pr, pb)
    k = rng.integers(0, n_pairs, n_surv, dtype=np.int32)
    sr = pr[k].copy()
    sb = pb[k].copy()
    want = want_pair[k].copy()
    bad_r = rng.choice(n_surv, 50, replace=False)
    bad_b = rng.choice(n_surv, 50, replace=False)
    sr[bad_r] = n_reads + 5
    sb[bad_b] = nb + 1
    want[bad_r] = -1
    want[bad_b] = -1
    idx = g.grim_build_bins(ref, q, B, O)
    idx.attach_reference(ref)
    dist, okb = _verify_gpu(g, idx, w, sr, sb, max_len=max_len)
    assert np.array_equal(dist, want), np.nonzero(dist != want)[0][:5]
    E = ((w["read_e"].astype(np.int64) * w["read_len"] + w["e_den"] - 1) // w["e_den"])
    E = np.append(E, 0).astype(np.int32)   # index n_reads: the out-of-range read ids
    want_ok = (want >= 0) & (want <= E[np.minimum(sr, n_reads)])
    okn = np.unpackbits(okb.view(np.uint8), bitorder="little")[:n_surv]
    assert np.array_equal(okn.astype(bool), want_ok)
    assert okb.size == (n_surv + 31) // 32
    assert okb[-1] >> (n_surv & 31) == 0


@pytest.mark.parametrize("G", [1, 5, 15, 16, 17, 33, 40])
def test_verify_tiny_references(G):
    """References of one to three packed words: every bin's span ends at the
    reference's end, so the alignment check's look-ahead fetches of reference
    words past the end are all clamped.  Reads of 0-70 bases (some longer
    than the reference), every bin, two strides, against the oracle."""
    g = lib()
    rng = np.random.default_rng(300 + G)
    ref = rng.integers(0, 4, G).astype(np.uint8)
    for B, O in ((4, 3), (16, 20)):
        q = 4
        nb = (G + B - 1) // B
        reads, cands = [], []
        for L in (0, 1, 3, 4, 9, 16, 31, 32, 33, 64, 70):
            r = rng.integers(0, 4, L).astype(np.uint8)
            if 0 < L <= G:                       # some reads copied from the reference
                st = int(rng.integers(0, G - L + 1))
                r = ref[st:st + L].copy()
            reads.append(r)
            cands.append(list(range(nb)))
        w = custom_workload(ref, q, B, O, reads, cands, [500] * len(reads))
        idx = g.grim_build_bins(ref, q, B, O)
        idx.attach_reference(ref)
        off = w["cand_off"].astype(np.int64)
        sr = np.repeat(np.arange(len(reads), dtype=np.uint32), np.diff(off))
        sb = w["cand_bin"].copy()
        dist, _ = _verify_gpu(g, idx, w, sr, sb, max_len=128)
        want = oracle.verify(ref, B, O, w["codes"], w["read_off"], w["read_len"], w["read_e"],
                             w["e_den"], sr, sb)
        assert np.array_equal(dist, want), (G, B, O, dist, want)
