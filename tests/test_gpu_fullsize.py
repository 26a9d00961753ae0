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
    del g, idx, batch, counts, bits, ws, c2, b2
    gc.collect()
    torch.cuda.empty_cache()
