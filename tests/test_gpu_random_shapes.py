"""Parity over randomly drawn small shapes (fixed seeds, so every run checks the
same cases): token sizes 4-7, bin strides from 1 to 600 bases and overlaps up
to 400, references with and without repeat families, read lengths from 1 to
400 (reads shorter than a token included), tolerances from 0 to 25 %, and
candidate lists that are empty, repeat bins, hold the read's true bin or run
past the last bin.  Each case goes through the index build, the batched and
the plain kernels, the survivor list and the alignment check, all compared
with the oracle bit for bit."""
import sys

import numpy as np
import pytest

import grim_synth as gs
import oracle
from tests.gpu_helpers import assert_same, custom_workload, gpu_run, lib, oracle_run

pytestmark = pytest.mark.gpu

E_NUMS = (0, 300, 500, 1000, 2500)  # parts per 10,000


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_case(seed):
    rng = np.random.default_rng(1000 + seed)
    q = int(rng.integers(4, 8))
    G = int(rng.integers(2_000, 120_000))
    B = int(rng.integers(1, 20)) if seed % 5 == 0 else int(rng.integers(20, 600))
    O = int(rng.integers(0, 400))
    ref = gs.reference(7 + seed, G, 0.3 if seed % 2 else 0.0, 5, 200, 0.85, 0.98)
    n_bins = (G + B - 1) // B
    n_reads = int(rng.integers(1, 160))
    reads, cands, e_nums = [], [], []
    for _ in range(n_reads):
        L = int(rng.integers(1, 12)) if rng.random() < 0.1 else int(rng.integers(12, 401))
        L = min(L, G)
        z = int(rng.integers(0, G - L + 1))
        if rng.random() < 0.8:
            r = ref[z:z + L].copy()
            for _ in range(int(rng.integers(0, max(1, L // 20) + 1))):
                r[int(rng.integers(0, L))] = int(rng.integers(0, 4))
        else:
            r = rng.integers(0, 4, L).astype(np.uint8)
        reads.append(r)
        k = int(rng.integers(0, 25))
        c = [int(b) for b in rng.integers(0, n_bins, k)]
        if k and rng.random() < 0.7:
            c[int(rng.integers(0, k))] = z // B              # the read's own bin
        if k > 2 and rng.random() < 0.3:
            c[1] = c[0]                                      # a repeated bin
        if k and rng.random() < 0.01:
            c[-1] = n_bins + int(rng.integers(0, 5))         # past the last bin
        cands.append(c)
        e_nums.append(int(rng.choice(E_NUMS)))
    return custom_workload(ref, q, B, O, reads, cands, e_nums)


@pytest.mark.parametrize("seed", range(40))
def test_random_shape(seed):
    import torch
    g = lib()
    w = make_case(seed)
    n_pairs = int(w["cand_off"][-1])
    say("random shape", seed, "q", w["q"], "B", w["B"], "O", w["O"], "G", w["ref"].size,
        "reads", w["read_len"].size, "pairs", n_pairs)
    oc, ob, bad, oidx = oracle_run(w, n_threads=4)
    idx = g.grim_build_bins(w["ref"], w["q"], w["B"], w["O"])
    assert np.array_equal(idx.to_host(), oidx), "index"
    for mode in ("batched", "plain"):
        out = gpu_run(idx, w, mode)
        assert_same(out, (oc, ob, bad), f"seed {seed} {mode}")
        assert (out[2] == g.GRIM_E_BIN_RANGE) == (bad > 0), (mode, out[2], bad)
        if bad:
            assert out[3] & g.GRIM_FLAG_BIN_RANGE
    # survivor list and alignment check of the survivors
    batch = g.Batch.from_workload(w)
    bits = torch.from_numpy(np.ascontiguousarray(ob).view(np.int32)).cuda()
    sp, sr, sb, total = g.grim_compact_survivors(batch, bits)
    op, orr, obin = oracle.survivors(ob, n_pairs, w["cand_off"], w["cand_bin"])
    assert total == op.size
    assert np.array_equal(sp.cpu().numpy().astype(np.uint64), op)
    srn = sr.cpu().numpy().view(np.uint32)
    sbn = sb.cpu().numpy().view(np.uint32)
    assert np.array_equal(srn, orr) and np.array_equal(sbn, obin)
    if total:
        idx.attach_reference(w["ref"])
        dist, ok = g.grim_verify_survivors(idx, batch, sr, sb, total)
        torch.cuda.synchronize()
        want = oracle.verify(w["ref"], w["B"], w["O"], w["codes"], w["read_off"], w["read_len"],
                             w["read_e"], w["e_den"], srn, sbn)
        got = dist.cpu().numpy()
        assert np.array_equal(got, want), np.nonzero(got != want)[0][:5]
        E = (w["read_e"].astype(np.int64) * w["read_len"] + w["e_den"] - 1) // w["e_den"]
        okb = ok.cpu().numpy().view(np.uint32)
        okn = (okb[np.arange(total) >> 5] >> (np.arange(total) & 31)) & 1
        assert np.array_equal(okn.astype(bool), want <= E[srn])


@pytest.mark.parametrize("seed", range(40))
def test_random_shape_windows_and_seeding(seed):
    """The same cases through the bin-window form (a random window of 1-300
    consecutive bins per read, some running past the last bin) and through
    device seeding (k = 4-12, caps from 1 to 4096), against the oracle."""
    from tests.test_gpu_window import run_windows, window_workload
    g = lib()
    w = make_case(seed)
    rng = np.random.default_rng(5000 + seed)
    q, B, O, ref = w["q"], w["B"], w["O"], w["ref"]
    n_bins = (ref.size + B - 1) // B
    n_reads = w["read_len"].size
    reads = [w["codes"][int(o):int(o) + int(L)] for o, L in zip(w["read_off"], w["read_len"])]
    sizes = rng.integers(1, 301, n_reads)
    win_lo = rng.integers(0, n_bins, n_reads)
    say("random windows", seed, "q", q, "B", B, "bins", n_bins, "pairs", int(sizes.sum()))
    ww = window_workload(ref, q, B, O, reads, w["read_e"], win_lo, sizes)
    oc, ob, bad, _ = oracle_run(ww, n_threads=4)
    idx = g.grim_build_bins(ref, q, B, O)
    idx.transpose()
    out = run_windows(g, idx, ww, win_lo)
    assert_same(out, (oc, ob, bad), f"windows seed {seed}")
    # seeding
    k = int(rng.integers(4, 13))
    cap = int(rng.choice([1, 7, 64, 4096]))
    say("random seeding", seed, "k", k, "cap", cap)
    batch = g.Batch(w["codes"], w["read_off"], w["read_len"], w["read_e"], w["e_den"],
                    np.zeros(n_reads + 1, np.uint64), np.zeros(0, np.uint32))
    si = g.SeedIndex(ref, k)
    off, bins = g.grim_seed_candidates(si, batch, B, cap).to_host()
    w_off, w_bins = oracle.seed_candidates(ref, k, w["codes"], w["read_off"], w["read_len"], B, cap)
    assert np.array_equal(off, w_off) and np.array_equal(bins, w_bins)
