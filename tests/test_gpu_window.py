"""Bin-window form on the GPU: every bin of each read's window, from the
token-major copy of the index, against the oracle on the same (read, bin)
pairs written out as explicit candidates."""
import numpy as np
import pytest

import grim_synth as gs
import oracle
from tests.gpu_helpers import assert_same, custom_workload, gpu_run, lib, oracle_run

pytestmark = pytest.mark.gpu


def run_windows(g, idx, w, win_lo, max_len=None, order=None):
    import torch
    b = g.Batch.from_workload(w, max_len=max_len)
    n = b.n_pairs
    counts, bits = g.alloc_outputs(n)
    counts.fill_(-9)
    ws = torch.zeros(256, dtype=torch.uint8, device="cuda")
    wl = torch.from_numpy(np.ascontiguousarray(win_lo, dtype=np.uint32).view(np.int32)).cuda()
    if isinstance(order, str) and order == "sorted":
        order = g.grim_window_order(idx, wl)
    elif order is not None:
        order = torch.from_numpy(np.ascontiguousarray(order, dtype=np.uint32).view(np.int32)).cuda()
    g.grim_filter_windows(idx, b, wl, counts, bits, ws, order=order)
    rc, flags = g.grim_filter_status(ws)
    torch.cuda.synchronize()
    return (counts.cpu().numpy()[:n].copy(),
            bits.cpu().numpy().view(np.uint32)[:(n + 31) // 32].copy(), rc, flags)


def window_workload(ref, q, B, O, reads, e_nums, win_lo, sizes):
    cands = [list(range(int(lo), int(lo) + int(sz))) for lo, sz in zip(win_lo, sizes)]
    return custom_workload(ref, q, B, O, reads, cands, e_nums)


@pytest.mark.parametrize("q,B,O", [(4, 100, 60), (5, 200, 105), (6, 400, 263), (7, 300, 60)])
def test_windows_match_oracle(q, B, O):
    g = lib()
    ref = gs.reference(41 + q, 1_500_000, 0.3, 30, 300, 0.85, 0.98)
    nb = (ref.size + B - 1) // B
    rng = np.random.default_rng(q)
    rd = gs.reads(42 + q, ref, 60, [100, 150, 250, 31], [500, 1000])
    reads = [rd["codes"][int(o):int(o) + int(L)] for o, L in zip(rd["read_off"], rd["read_len"])]
    sizes = rng.choice([1, 31, 32, 33, 64, 100, 4096, 10_000], size=60)
    win_lo = [max(0, int(z) // B - int(s) // 2) for z, s in zip(rd["read_z"], sizes)]
    win_lo[0] = nb - 10                       # runs past the last bin
    sizes[0] = 40
    win_lo[1] = 0
    w = window_workload(ref, q, B, O, reads, rd["read_e"], win_lo, sizes)
    idx = g.grim_build_bins(ref, q, B, O)
    idx.transpose()
    out = run_windows(g, idx, w, win_lo)
    orc = oracle_run(w)
    assert out[2] == g.GRIM_E_BIN_RANGE and orc[2] >= 30   # window 0 runs 30 bins past the end
    assert_same(out, orc, f"windows q{q}")
    # the batched kernel agrees on the same explicit pairs
    assert_same(gpu_run(idx, w), orc, f"batched q{q}")


def test_windows_long_reads_and_empty():
    g = lib()
    ref = gs.reference(50, 400_000)
    q, B, O = 5, 200, 4200
    reads = [np.zeros(4096, np.uint8), ref[1000:5000], ref[9000:9003], np.zeros(0, np.uint8),
             ref[3000:3100]]
    win_lo = [0, 3, 10, 20, 1999]
    sizes = [300, 50, 7, 5, 0]
    w = window_workload(ref, q, B, O, reads, [500] * 5, win_lo, sizes)
    idx = g.grim_build_bins(ref, q, B, O)
    idx.transpose()
    out = run_windows(g, idx, w, win_lo, max_len=4096)
    assert out[2] == 0
    assert_same(out, oracle_run(w), "long reads")
    with pytest.raises(g.GrimError) as e:
        run_windows(g, idx, w, win_lo, max_len=5000)
    assert e.value.code == g.GRIM_E_UNSUPPORTED


@pytest.mark.parametrize("q,G,B", [(4, 250_000, 97), (5, 250_000, 97), (6, 250_000, 200),
                                   (7, 60_001, 50)])
def test_transpose_layout(q, G, B):
    """Row t, bit b of the token-major copy = bit t of bin b's vector: a window
    over every bin for a read that is just token t, for every token (q <= 5) or
    tokens sampled across every 1024-token load pass (q = 6, 7); bin counts span
    several 1024-bin transpose tiles with a ragged last one."""
    g = lib()
    ref = gs.reference(51 + q, G)
    idx = g.grim_build_bins(ref, q, B, 30)
    idx.transpose()
    vec = idx.to_host()
    bits = np.unpackbits(vec, axis=1, bitorder="little")  # (n_bins, 4^q)
    nb = idx.n_bins
    n_tok = 4 ** q
    if q <= 5:
        toks = np.arange(n_tok)
    else:
        rng = np.random.default_rng(q)
        edges = [0, 31, 32, 127, 128, 1023, 1024, n_tok - 1]
        toks = np.unique(np.concatenate([edges, rng.integers(0, n_tok, 300)]))
    reads = [np.array([(int(t) >> (2 * (q - 1 - j))) & 3 for j in range(q)], np.uint8)
             for t in toks]
    k = len(toks)
    w = window_workload(ref, q, B, 30, reads, [0] * k, [0] * k, [nb] * k)
    out = run_windows(g, idx, w, [0] * k)
    got = out[0].reshape(k, nb)
    assert np.array_equal(got, bits[:, toks].T.astype(np.int32))


def test_windows_token_blocks_and_many_reads():
    """Token counts around the 16-token blocks of the counter (ntok 0 ... 70,
    including reads shorter than q), windows of every alignment (a quarter of
    them on multiples of 32 bins) and size up to 9,000 bins, and more reads
    than the persistent grid has workgroups."""
    g = lib()
    q, B, O = 5, 150, 110
    ref = gs.reference(61, 1_200_000, 0.3, 30, 300, 0.85, 0.98)
    nb = (ref.size + B - 1) // B
    rng = np.random.default_rng(62)
    n = 2500
    ntoks = np.concatenate([np.arange(0, 71), rng.integers(0, 250, size=n - 71)])
    lens = np.maximum(ntoks + q - 1, 1)
    lens[:3] = [1, 3, 4]                      # shorter than q: no tokens
    reads, e_nums = [], []
    for i, L in enumerate(lens):
        z = int(rng.integers(0, ref.size - L))
        reads.append(ref[z:z + L].copy())
        e_nums.append(int(rng.choice([0, 300, 500, 1000])))
    sizes = rng.choice([1, 5, 31, 32, 33, 63, 64, 65, 127, 128, 129, 4095, 4096, 4097, 9000],
                       size=n)
    win_lo = rng.integers(0, nb, size=n)
    win_lo[::4] = (win_lo[::4] // 32) * 32      # windows on a row word: the one-word path
    win_lo[::16] = (win_lo[::16] // 1024) * 1024
    w = window_workload(ref, q, B, O, reads, e_nums, win_lo, sizes)
    idx = g.grim_build_bins(ref, q, B, O)
    idx.transpose()
    out = run_windows(g, idx, w, win_lo)
    orc = oracle_run(w)
    assert out[2] == (g.GRIM_E_BIN_RANGE if orc[2] else 0)
    assert_same(out, orc, "token blocks")


@pytest.mark.skip(reason="checks the first device-side window order (a library sort: the stable "
                         "argsort of the window starts), whose first GPU run stopped responding "
                         "with no cause found; that code is gone, and the bucket order that "
                         "replaced it is tested by test_window_bucket_order")
def test_window_order_and_ordered_filter():
    """grim_window_order is the stable argsort of the window starts; filtering in
    that order, or in any other permutation, gives the same outputs as index
    order; an order entry past the last read is skipped and flagged."""
    import torch
    g = lib()
    q, B, O = 5, 200, 105
    ref = gs.reference(71, 1_000_000, 0.3, 30, 300, 0.85, 0.98)
    nb = (ref.size + B - 1) // B
    rng = np.random.default_rng(72)
    rd = gs.reads(73, ref, 700, [100, 150, 250], [500, 1000])
    reads = [rd["codes"][int(o):int(o) + int(L)] for o, L in zip(rd["read_off"], rd["read_len"])]
    n = len(reads)
    sizes = rng.choice([1, 33, 500, 2048], size=n)
    win_lo = np.minimum(rd["read_z"] // B, nb - 1).astype(np.int64) - sizes // 2
    win_lo = np.clip(win_lo, 0, nb - 1)
    win_lo[:50] = rng.integers(0, 40, size=50)       # many equal and near-equal keys
    win_lo[50:60] = 7
    w = window_workload(ref, q, B, O, reads, rd["read_e"], win_lo, sizes)
    idx = g.grim_build_bins(ref, q, B, O)
    idx.transpose()
    wl = torch.from_numpy(win_lo.astype(np.uint32).view(np.int32)).cuda()
    order = g.grim_window_order(idx, wl)
    torch.cuda.synchronize()
    got = order.cpu().numpy().view(np.uint32)[:n]
    assert np.array_equal(got, np.argsort(win_lo, kind="stable").astype(np.uint32))
    base = run_windows(g, idx, w, win_lo)
    orc = oracle_run(w)
    assert_same(base, orc, "index order")
    assert_same(run_windows(g, idx, w, win_lo, order="sorted"), orc, "sorted order")
    assert_same(run_windows(g, idx, w, win_lo, order=rng.permutation(n)), orc, "random order")
    # one slot names a read that does not exist: that slot is skipped and
    # flagged, the read it replaced keeps its initial counts, the rest is exact
    bad = np.arange(n)
    bad[5] = n + 3
    c, b, rc, flags = run_windows(g, idx, w, win_lo, order=bad)
    assert rc == g.GRIM_E_READ
    p0, p1 = int(w["cand_off"][5]), int(w["cand_off"][6])
    assert np.all(c[p0:p1] == -9)
    keep = np.ones(c.size, bool)
    keep[p0:p1] = False
    assert np.array_equal(c[keep], orc[0][keep])


def test_window_bucket_order():
    """grim_window_order is a permutation of the reads with their window-start
    buckets (1024 bins each, starts past the last bin last) non-decreasing;
    filtering in that order, in a random order or in index order gives the
    oracle's outputs; an order entry naming no read is skipped and flagged, and
    the read it replaced keeps the previous contents of its counts."""
    import torch
    g = lib()
    q, B, O = 5, 40, 21
    ref = gs.reference(81, 1_000_000, 0.3, 30, 300, 0.85, 0.98)
    nb = (ref.size + B - 1) // B                # 25,000 bins: 25 buckets
    rng = np.random.default_rng(82)
    rd = gs.reads(83, ref, 900, [100, 150, 250], [500, 1000])
    reads = [rd["codes"][int(o):int(o) + int(L)] for o, L in zip(rd["read_off"], rd["read_len"])]
    n = len(reads)
    sizes = rng.choice([1, 33, 500, 2048], size=n)
    win_lo = np.clip(np.minimum(rd["read_z"] // B, nb - 1).astype(np.int64) - sizes // 2, 0, nb - 1)
    win_lo[:200] = rng.integers(0, 40, size=200)     # one crowded bucket
    win_lo[200:210] = 7
    win_lo[210:214] = [nb, nb + 5, nb + 3000, nb + 10_000_000]  # windows past the last bin
    w = window_workload(ref, q, B, O, reads, rd["read_e"], win_lo, sizes)
    idx = g.grim_build_bins(ref, q, B, O)
    idx.transpose()
    wl = torch.from_numpy(win_lo.astype(np.uint32).view(np.int32)).cuda()
    bucket = np.where(win_lo < nb, win_lo >> 10, ((nb - 1) >> 10) + 1)
    for _ in range(2):                          # twice: the bucket counts start from zero
        order = g.grim_window_order(idx, wl)
        torch.cuda.synchronize()
        got = order.cpu().numpy().view(np.uint32)[:n].astype(np.int64)
        assert np.array_equal(np.sort(got), np.arange(n))
        assert np.all(np.diff(bucket[got]) >= 0)
    orc = oracle_run(w)
    base = run_windows(g, idx, w, win_lo)
    assert base[2] == g.GRIM_E_BIN_RANGE and orc[2]
    assert_same(base, orc, "index order")
    assert_same(run_windows(g, idx, w, win_lo, order="sorted"), orc, "bucket order")
    assert_same(run_windows(g, idx, w, win_lo, order=rng.permutation(n)), orc, "random order")
    bad = np.arange(n)
    bad[5] = n + 3
    c, b, rc, flags = run_windows(g, idx, w, win_lo, order=bad)
    assert flags & g.GRIM_FLAG_READ and not base[3] & g.GRIM_FLAG_READ
    assert rc == g.GRIM_E_BIN_RANGE             # reported before GRIM_E_READ
    p0, p1 = int(w["cand_off"][5]), int(w["cand_off"][6])
    assert p1 > p0 and np.all(c[p0:p1] == -9)
    keep = np.ones(c.size, bool)
    keep[p0:p1] = False
    assert np.array_equal(c[keep], orc[0][keep])


def test_windows_invalid_reads_skipped():
    """Reads longer than max_len are skipped with counts -1, no pass bits and
    GRIM_FLAG_READ, from index order and from a processing order alike; the
    other reads' outputs are the oracle's."""
    g = lib()
    ref = gs.reference(91, 400_000)
    q, B, O = 5, 200, 105
    reads = [ref[1000:1300], ref[2000:2150], ref[3000:3100], ref[5000:5400], ref[7000:7180]]
    win_lo = [3, 10, 20, 1999, 40]
    sizes = [50, 70, 33, 5, 64]
    w = window_workload(ref, q, B, O, reads, [500] * 5, win_lo, sizes)
    idx = g.grim_build_bins(ref, q, B, O)
    idx.transpose()
    orc = oracle_run(w)
    bad = np.zeros(w["cand_off"][-1], bool)
    for r in (0, 3):                            # 300 and 400 bases, over max_len = 200
        bad[int(w["cand_off"][r]):int(w["cand_off"][r + 1])] = True
    for order in (None, [4, 3, 2, 1, 0]):
        c, b, rc, flags = run_windows(g, idx, w, win_lo, max_len=200, order=order)
        assert rc == g.GRIM_E_READ and flags & g.GRIM_FLAG_READ
        assert np.all(c[bad] == -1) and np.array_equal(c[~bad], orc[0][~bad])
        bits = np.unpackbits(b.view(np.uint8), bitorder="little")[:bad.size].astype(bool)
        want = np.unpackbits(orc[1].view(np.uint8), bitorder="little")[:bad.size].astype(bool)
        assert not bits[bad].any() and np.array_equal(bits[~bad], want[~bad])
