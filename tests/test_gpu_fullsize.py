"""Full-size workloads in the launch configuration bench.py times (autotuned
shape, HIP-graph replay).  mid is compared with the oracle element by element;
batched (8.3e8 pairs) and large (2.0e9 pairs) are compared on sampled pairs,
one pair at a time, plus properties checked over every pair on the device."""
import gc
import sys

import numpy as np
import pytest

import grim_synth as gs
import oracle
from tests.gpu_helpers import assert_same, lib

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_like_bench(w):
    """Index build, resident inputs, autotune, one graph replay -- as bench.py."""
    import torch
    g = lib()
    idx = g.grim_build_bins(w["ref"], w["q"], w["B"], w["O"])
    batch = g.Batch.from_workload(w, max_len=int(w["read_len"].max()))
    counts, bits = g.alloc_outputs(batch.n_pairs)
    ws = g.alloc_workspace(idx, batch.n_pairs)
    tune = g.grim_tune(idx, batch, counts, bits, ws)
    counts.fill_(-5)
    graph = g.grim_graph_create(idx, batch, counts, bits, ws, tune)
    graph.launch()
    rc, flags = g.grim_filter_status(ws)
    torch.cuda.synchronize()
    return g, idx, batch, counts, bits, ws, tune, rc, flags


def per_pair(values, cand_off, device):
    """Expand a per-read array to one value per pair (device tensor)."""
    import torch
    k = torch.from_numpy(np.diff(cand_off.astype(np.int64))).to(device)
    v = torch.from_numpy(np.ascontiguousarray(values)).to(device)
    return torch.repeat_interleave(v, k)


def check_properties(w, counts, bits, chunk=1 << 28):
    """Over every pair: 0 <= count <= ntok, pass bit == (count >= T);
    every read's true bin passes (no true location rejected)."""
    import torch
    dev = counts.device
    q = w["q"]
    L = w["read_len"].astype(np.int64)
    E = (w["read_e"].astype(np.int64) * L + w["e_den"] - 1) // w["e_den"]
    ntok = np.maximum(L - q + 1, 0)
    T = ntok - q * E
    n = int(w["cand_off"][-1])
    off = w["cand_off"].astype(np.int64)
    r0 = 0
    while r0 < L.size:
        p0 = int(off[r0])
        r1 = int(np.searchsorted(off, p0 + chunk, side="right")) - 1
        r1 = max(r1, r0 + 1)
        r1 = min(r1, L.size)
        p1 = int(off[r1])
        if p1 > p0:
            c = counts[p0:p1].to(torch.int64)
            nt = per_pair(ntok[r0:r1], off[r0:r1 + 1], dev)
            tt = per_pair(T[r0:r1], off[r0:r1 + 1], dev)
            assert bool((c >= 0).all()) and bool((c <= nt).all())
            ks = torch.arange(p0, p1, device=dev, dtype=torch.int64)
            words = bits[(ks >> 5)].to(torch.int64) & 0xFFFFFFFF
            b = (words >> (ks & 31)) & 1
            assert torch.equal(b, (c >= tt).to(torch.int64))
            del c, nt, tt, ks, words, b
        r0 = r1
    tp = w["true_pair"]
    ok = tp != np.iinfo(np.uint64).max
    tpi = torch.from_numpy(tp[ok].astype(np.int64)).to(dev)
    tc = counts.index_select(0, tpi).cpu().numpy().astype(np.int64)
    assert np.all(tc >= T[ok]), "a true location was rejected"
    return n


def sampled_oracle(w, counts, bits, n_samples, seed):
    import torch
    rng = np.random.default_rng(seed)
    n = int(w["cand_off"][-1])
    ks = np.sort(rng.choice(n, size=n_samples, replace=False))
    dev = counts.device
    gc_ = counts.index_select(0, torch.from_numpy(ks.astype(np.int64)).to(dev)).cpu().numpy()
    gw = bits.index_select(0, torch.from_numpy((ks >> 5).astype(np.int64)).to(dev)).cpu().numpy()
    gb = (gw.view(np.uint32) >> (ks & 31).astype(np.uint32)) & 1
    reads = np.searchsorted(w["cand_off"], ks, side="right") - 1
    for k, r, c, b in zip(ks, reads, gc_, gb):
        vec = oracle.build_bin(w["ref"], w["B"], w["O"], w["q"], int(w["cand_bin"][k]))
        o, L = int(w["read_off"][r]), int(w["read_len"][r])
        oc = oracle.count(vec, w["q"], w["codes"][o:o + L])
        T = oracle.threshold(L, w["q"], oracle.max_edits(L, int(w["read_e"][r]), w["e_den"]))
        assert oc == c, (int(k), int(r), int(c), oc)
        assert int(oc >= T) == int(b), (int(k), int(r))


def sampled_index(w, idx, n_samples, seed):
    """Sampled bin vectors (plus the first and last bin) against the oracle."""
    rng = np.random.default_rng(seed)
    bins = np.concatenate([np.unique(rng.integers(0, idx.n_bins, n_samples)), [0, idx.n_bins - 1]])
    host_rows = idx.to_host()[bins]
    for b, row in zip(bins, host_rows):
        assert np.array_equal(row, oracle.build_bin(w["ref"], w["B"], w["O"], w["q"], int(b))), b


def test_mid_fullsize_exact():
    import torch
    say("mid full size")
    w = gs.make_workload("mid")
    g, idx, batch, counts, bits, ws, tune, rc, flags = run_like_bench(w)
    assert rc == 0, (rc, flags)
    say("mid pairs", batch.n_pairs, "tuning", tune.as_dict())
    oidx = oracle.build_index(w["ref"], w["B"], w["O"], w["q"], n_threads=16)
    assert np.array_equal(idx.to_host(), oidx)
    oc, op, bad = oracle.filter_batch(oidx, w["q"], w["codes"], w["read_off"], w["read_len"],
                                      w["read_e"], w["e_den"], w["cand_off"], w["cand_bin"],
                                      n_threads=16)
    n = batch.n_pairs
    out = (counts.cpu().numpy()[:n], bits.cpu().numpy().view(np.uint32)[:(n + 31) // 32], rc, flags)
    assert_same(out, (oc, oracle.pack_bitmask(op), bad), "mid full")
    del g, idx, batch, counts, bits, ws
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["batched", "large"])
def test_fullsize_sampled_and_properties(name):
    import torch
    say(name, "full size")
    w = gs.make_workload(name)
    g, idx, batch, counts, bits, ws, tune, rc, flags = run_like_bench(w)
    assert rc == 0, (rc, flags)
    say(name, "pairs", batch.n_pairs, "tuning", tune.as_dict())
    sampled_index(w, idx, 300, 1)
    sampled_oracle(w, counts, bits, 1500, 2)
    say(name, "sampled pairs ok")
    check_properties(w, counts, bits)
    say(name, "properties ok")
    # the plain per-read kernel gives the same bits at full size
    c2, b2 = g.alloc_outputs(batch.n_pairs)
    g.grim_filter_plain(idx, batch, c2, b2, ws)
    torch.cuda.synchronize()
    n = batch.n_pairs
    assert torch.equal(c2[:n], counts[:n])
    assert torch.equal(b2[:(n + 31) // 32], bits[:(n + 31) // 32])
    del c2, b2
    if name == "batched":
        check_checker(g, w, idx, batch, counts, bits)
        say(name, "seed location checker ok")
    del g, idx, batch, counts, bits, ws
    gc.collect()
    torch.cuda.empty_cache()


def check_checker(g, w, idx, batch, counts, bits, n_samples=2000, n_align=300, seed=3):
    """Survivor list and alignment check at full size: the list holds exactly the
    passing pairs in order (count, order, sampled read and bin ids), and sampled
    survivors' capped distances equal the oracle's."""
    import torch
    n = batch.n_pairs
    words = bits[:(n + 31) // 32].view(torch.uint8).to(torch.int32)
    pop = int(torch.sum((words[:, None] >> torch.arange(8, device=bits.device,
                                                        dtype=torch.int32)[None, :]) & 1).item())
    del words
    sp, sr, sb, total = g.grim_compact_survivors(batch, bits, capacity=pop)
    assert total == pop and sp.numel() == pop
    assert bool((sp[1:] > sp[:-1]).all())
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(total, size=min(n_samples, total), replace=False))
    ti = torch.from_numpy(pick.astype(np.int64)).to(sp.device)
    kp = sp.index_select(0, ti).cpu().numpy().astype(np.int64)
    kr = sr.index_select(0, ti).cpu().numpy().view(np.uint32)
    kb = sb.index_select(0, ti).cpu().numpy().view(np.uint32)
    bw = bits.index_select(0, torch.from_numpy(kp >> 5).to(bits.device)).cpu().numpy().view(np.uint32)
    assert np.all((bw >> (kp & 31).astype(np.uint32)) & 1)
    assert np.array_equal(kr, (np.searchsorted(w["cand_off"], kp, side="right") - 1).astype(np.uint32))
    assert np.array_equal(kb, w["cand_bin"][kp])
    idx.attach_reference(w["ref"])
    dist, okb = g.grim_verify_survivors(idx, batch, sr, sb, total)
    torch.cuda.synchronize()
    sj = np.sort(rng.choice(pick.size, size=min(n_align, pick.size), replace=False))
    sel = pick[sj]
    gd = dist.index_select(0, torch.from_numpy(sel.astype(np.int64)).to(dist.device)).cpu().numpy()
    gok = okb.index_select(0, torch.from_numpy((sel >> 5).astype(np.int64)).to(okb.device)) \
        .cpu().numpy().view(np.uint32)
    for j, (i, jj) in enumerate(zip(sel, sj)):
        r, b = int(kr[jj]), int(kb[jj])
        o, L = int(w["read_off"][r]), int(w["read_len"][r])
        E = oracle.max_edits(L, int(w["read_e"][r]), w["e_den"])
        d = oracle.edit_distance_in_bin(w["ref"], w["B"], w["O"], b, w["codes"][o:o + L])
        assert int(gd[j]) == min(d, E + 1), (int(i), r, b)
        assert int((gok[j] >> (int(i) & 31)) & 1) == int(d <= E)
    del sp, sr, sb, dist, okb


def test_fullsize_windows_sampled_and_properties():
    """The bin-window leg as bench.py runs it: the batched 3.1 Gbp index, its
    token-major copy, the first 200,000 reads each against the 4096 bins centred
    on its true bin.  Sampled pairs against the oracle one by one; over every
    pair, 0 <= count <= ntok and pass == (count >= T); every true bin passes."""
    import torch
    g = lib()
    w = gs.make_workload("batched")
    idx = g.grim_build_bins(w["ref"], w["q"], w["B"], w["O"])
    idx.transpose()
    n_reads, wbins = 200_000, 4096
    nb = idx.n_bins
    tb = (w["read_z"][:n_reads] // w["B"]).astype(np.int64)
    lo = np.clip(tb - wbins // 2, 0, nb - wbins).astype(np.int64)
    off = np.arange(n_reads + 1, dtype=np.uint64) * wbins
    o_end = int(w["read_off"][n_reads - 1]) + int(w["read_len"][n_reads - 1])
    wb = g.Batch(w["codes"][:o_end], w["read_off"][:n_reads], w["read_len"][:n_reads],
                 w["read_e"][:n_reads], w["e_den"], off, np.zeros(1, np.uint32),
                 max_len=int(w["read_len"].max()))
    n = wb.n_pairs
    counts, bits = g.alloc_outputs(n)
    ws = torch.zeros(256, dtype=torch.uint8, device="cuda")
    wl = torch.from_numpy(lo.astype(np.uint32).view(np.int32)).cuda()
    g.grim_filter_windows(idx, wb, wl, counts, bits, ws)
    rc, flags = g.grim_filter_status(ws)
    torch.cuda.synchronize()
    assert rc == 0, (rc, flags)
    say("windows", n, "pairs")
    # sampled pairs one by one
    rng = np.random.default_rng(7)
    ks = np.sort(rng.choice(n, size=1500, replace=False))
    gc_ = counts.index_select(0, torch.from_numpy(ks.astype(np.int64)).cuda()).cpu().numpy()
    gw = bits.index_select(0, torch.from_numpy((ks >> 5).astype(np.int64)).cuda()).cpu().numpy()
    gb = (gw.view(np.uint32) >> (ks & 31).astype(np.uint32)) & 1
    q = w["q"]
    for k, c, b in zip(ks, gc_, gb):
        r, j = int(k) // wbins, int(k) % wbins
        vec = oracle.build_bin(w["ref"], w["B"], w["O"], q, int(lo[r]) + j)
        o, L = int(w["read_off"][r]), int(w["read_len"][r])
        oc = oracle.count(vec, q, w["codes"][o:o + L])
        T = oracle.threshold(L, q, oracle.max_edits(L, int(w["read_e"][r]), w["e_den"]))
        assert oc == c, (int(k), int(c), oc)
        assert int(oc >= T) == int(b), int(k)
    say("windows sampled pairs ok")
    # every pair: bounds and pass bit; the true bin passes
    L = w["read_len"][:n_reads].astype(np.int64)
    E = (w["read_e"][:n_reads].astype(np.int64) * L + w["e_den"] - 1) // w["e_den"]
    ntok = np.maximum(L - q + 1, 0)
    T = ntok - q * E
    c = counts[:n].view(n_reads, wbins).to(torch.int64)
    nt = torch.from_numpy(ntok).cuda()[:, None]
    tt = torch.from_numpy(T).cuda()[:, None]
    assert bool((c >= 0).all()) and bool((c <= nt).all())
    ks = torch.arange(n, device="cuda", dtype=torch.int64)
    b = ((bits[:(n + 31) // 32].to(torch.int64) & 0xFFFFFFFF)[ks >> 5] >> (ks & 31)) & 1
    assert torch.equal(b.view(n_reads, wbins), (c >= tt).to(torch.int64))
    del ks, b
    col = torch.from_numpy(tb - lo).cuda()
    tc = c.gather(1, col[:, None])[:, 0]
    assert bool((tc >= tt[:, 0]).all()), "a true bin was rejected"
    del c, counts, bits, idx
    gc.collect()
    torch.cuda.empty_cache()
