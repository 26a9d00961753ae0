"""Full-size workloads in the launch configuration bench.py times (autotuned
shape, HIP-graph replay), compared with the oracle on every pair.

mid (1M reads, seeded candidates), batched (3.1 Gbp, 8.3e8 pairs) and large
(3.1 Gbp, q = 6, 2.0e9 pairs): every count and every pass bit against the
oracle, the whole index against the oracle's vectors.  The comparison runs on
the host's cores in shards (each shard is its own test, so that progress shows
while it runs).  At full batched size also the survivor list, sampled alignment
distances, the bin-window leg and requests served on the full index."""
import gc
import math
import sys

import numpy as np
import pytest

import bench
import grim_synth as gs
import oracle
from tests.gpu_helpers import assert_same, lib

pytestmark = pytest.mark.gpu

N_THREADS = gs.default_threads()
SHARDS = {"batched": 4, "large": 12}


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
    bits.fill_(-1)
    graph = g.grim_graph_create(idx, batch, counts, bits, ws, tune)
    graph.launch()
    rc, flags = g.grim_filter_status(ws)
    torch.cuda.synchronize()
    return g, idx, batch, counts, bits, ws, tune, rc, flags


def test_mid_fullsize_exact():
    import torch
    say("mid full size")
    w = gs.make_workload("mid")
    g, idx, batch, counts, bits, ws, tune, rc, flags = run_like_bench(w)
    assert rc == 0, (rc, flags)
    say("mid pairs", batch.n_pairs, "tuning", tune.as_dict())
    oidx = oracle.build_index(w["ref"], w["B"], w["O"], w["q"], n_threads=N_THREADS)
    assert np.array_equal(idx.to_host(), oidx)
    oc, op, bad = oracle.filter_batch(oidx, w["q"], w["codes"], w["read_off"], w["read_len"],
                                      w["read_e"], w["e_den"], w["cand_off"], w["cand_bin"],
                                      n_threads=N_THREADS)
    n = batch.n_pairs
    out = (counts.cpu().numpy()[:n], bits.cpu().numpy().view(np.uint32)[:(n + 31) // 32], rc, flags)
    assert_same(out, (oc, oracle.pack_bitmask(op), bad), "mid full")
    del g, idx, batch, counts, bits, ws
    gc.collect()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module", params=["batched", "large"])
def full(request):
    """One full-size workload run as bench.py runs it; results copied to the host."""
    import torch
    name = request.param
    w = gs.make_workload(name, n_threads=N_THREADS)
    g, idx, batch, counts, bits, ws, tune, rc, flags = run_like_bench(w)
    n = batch.n_pairs
    say(name, "pairs", n, "tuning", tune.as_dict(), "status", rc, flags)
    st = dict(name=name, w=w, g=g, idx=idx, batch=batch, counts=counts, bits=bits, ws=ws,
              tune=tune, rc=rc, flags=flags, n=n,
              host_counts=counts[:n].cpu().numpy().copy(),
              host_bits=bits[:(n + 31) // 32].cpu().numpy().view(np.uint32).copy(),
              oidx=None, seen=0, mismatches=0, shards_done=set())
    yield st
    say(name, "every pair compared:", st["seen"], "pairs,", st["mismatches"], "mismatches")
    st.clear()
    del g, idx, batch, counts, bits, ws
    gc.collect()
    torch.cuda.empty_cache()


def oracle_index(st):
    if st["oidx"] is None:
        w = st["w"]
        st["oidx"] = oracle.build_index(w["ref"], w["B"], w["O"], w["q"], n_threads=N_THREADS)
    return st["oidx"]


def test_fullsize_status_and_index(full):
    assert full["rc"] == 0, (full["rc"], full["flags"])
    host = full["idx"].to_host()
    assert np.array_equal(host, oracle_index(full)), "bin vectors differ from the oracle"


@pytest.mark.parametrize("shard", range(max(SHARDS.values())))
def test_fullsize_every_pair(full, shard):
    """Shard `shard` of the reads (cut at read boundaries, equal pair counts):
    the oracle's count and pass bit of every pair against the GPU's."""
    S = SHARDS[full["name"]]
    if shard >= S:
        pytest.skip(f"{full['name']} uses {S} shards")
    w = full["w"]
    off = w["cand_off"]
    n, n_reads = full["n"], w["read_len"].size
    cuts = [int(np.searchsorted(off, (n * s) // S, side="left")) for s in range(S)] + [n_reads]
    r0, r1 = cuts[shard], cuts[shard + 1]
    res = oracle.filter_compare(oracle_index(full), w["q"], w["codes"], w["read_off"],
                                w["read_len"], w["read_e"], w["e_den"], off, w["cand_bin"],
                                full["host_counts"], full["host_bits"], r_begin=r0, r_end=r1,
                                n_threads=N_THREADS)
    full["seen"] += res["pairs"]
    full["mismatches"] += res["count_mismatches"] + res["bit_mismatches"]
    full["shards_done"].add(shard)
    say(full["name"], "shard", shard, res)
    assert res["pairs"] == int(off[r1]) - int(off[r0])
    assert res["out_of_range"] == 0
    assert res["count_mismatches"] == 0 and res["bit_mismatches"] == 0, res
    if len(full["shards_done"]) == S:
        # every pair of the batch has been compared
        assert full["seen"] == n, (full["seen"], n)
    if shard == S - 1:
        # bits past the last pair are 0
        if n % 32:
            assert int(full["host_bits"][-1]) >> (n % 32) == 0


def test_fullsize_plain_identical(full):
    """The plain per-read kernel gives the same counts and bits at full size."""
    import torch
    g, n = full["g"], full["n"]
    c2, b2 = g.alloc_outputs(n)
    g.grim_filter_plain(full["idx"], full["batch"], c2, b2, full["ws"])
    torch.cuda.synchronize()
    assert torch.equal(c2[:n], full["counts"][:n])
    assert torch.equal(b2[:(n + 31) // 32], full["bits"][:(n + 31) // 32])
    del c2, b2


def test_fullsize_true_bins_pass(full):
    """No true location is rejected (the zero-false-reject property, over every read)."""
    w = full["w"]
    q = w["q"]
    L = w["read_len"].astype(np.int64)
    E = (w["read_e"].astype(np.int64) * L + w["e_den"] - 1) // w["e_den"]
    T = np.maximum(L - q + 1, 0) - q * E
    tp = w["true_pair"].astype(np.int64)
    assert np.all(full["host_counts"][tp] >= T), "a true location was rejected"
    assert np.all((full["host_bits"][tp >> 5] >> (tp & 31).astype(np.uint32)) & 1)


def test_fullsize_checker(full):
    """Survivor list and alignment check at full size: the list holds exactly
    the passing pairs in order (all of them, against the oracle's list built
    from the oracle-verified pass bits), and sampled survivors' capped
    distances equal the oracle's."""
    import torch
    g, w, idx, batch, bits, n = full["g"], full["w"], full["idx"], full["batch"], full["bits"], full["n"]
    wp, wr, wb = oracle.survivors(full["host_bits"], n, w["cand_off"], w["cand_bin"])
    sp, sr, sb, total = g.grim_compact_survivors(batch, bits, capacity=int(wp.size))
    assert total == wp.size
    assert np.array_equal(sp[:total].cpu().numpy().astype(np.uint64), wp)
    assert np.array_equal(sr[:total].cpu().numpy().view(np.uint32), wr)
    assert np.array_equal(sb[:total].cpu().numpy().view(np.uint32), wb)
    idx.attach_reference(w["ref"])
    dist, okb = g.grim_verify_survivors(idx, batch, sr, sb, total)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    sel = np.sort(rng.choice(total, size=min(300, total), replace=False))
    gd = dist.index_select(0, torch.from_numpy(sel.astype(np.int64)).to(dist.device)).cpu().numpy()
    gok = okb.index_select(0, torch.from_numpy((sel >> 5).astype(np.int64)).to(okb.device)) \
        .cpu().numpy().view(np.uint32)
    for j, i in enumerate(sel):
        r, b = int(wr[i]), int(wb[i])
        o, L = int(w["read_off"][r]), int(w["read_len"][r])
        E = oracle.max_edits(L, int(w["read_e"][r]), w["e_den"])
        d = oracle.edit_distance_in_bin(w["ref"], w["B"], w["O"], b, w["codes"][o:o + L])
        assert int(gd[j]) == min(d, E + 1), (int(i), r, b)
        assert int((gok[j] >> (int(i) & 31)) & 1) == int(d <= E)
    del sp, sr, sb, dist, okb


def test_fullsize_served_requests(full):
    """Requests of the serving workload on the full 3.1 Gbp index: log-uniform
    sizes of 1..65,536 reads (one of exactly 65,536), mixed 100/150/250-bp
    reads with e = 0.05 and Zipf candidates, served in place from pinned
    buffers with the serving leg's settings (3 streams, ticks of 8M pairs, so
    the largest requests run in parts), every count and pass bit against the
    oracle."""
    if full["name"] != "batched":
        pytest.skip("the serving workload uses the batched index")
    g, w = full["g"], full["w"]
    sw = gs.make_workload("serve", ref=w["ref"], scale=1.0, read_scale=0.05, n_threads=N_THREADS)
    n_reads = sw["read_len"].size
    rng = np.random.default_rng(41)
    sizes = [65536] + [int(max(1, round(math.exp(rng.uniform(0, math.log(65536))))))
                       for _ in range(23)]
    reqs = []
    for size in sizes:
        r0 = int(rng.integers(0, n_reads - size + 1))
        r1 = r0 + size
        o0 = int(sw["read_off"][r0])
        o1 = int(sw["read_off"][r1 - 1]) + int(sw["read_len"][r1 - 1])
        c0, c1 = int(sw["cand_off"][r0]), int(sw["cand_off"][r1])
        hb = g.HostBatch(sw["codes"][o0:o1], sw["read_off"][r0:r1] - o0, sw["read_len"][r0:r1],
                         sw["read_e"][r0:r1], sw["e_den"], sw["cand_off"][r0:r1 + 1] - c0,
                         sw["cand_bin"][c0:c1], max_len=250, pinned=True)
        reqs.append((r0, r1, hb))
    srv = g.Server(full["idx"], hbm_budget_bytes=4 << 30, max_inflight=1024, n_streams=3,
                   max_tick_pairs=8 << 20, max_len=256)
    tickets = [srv.submit_inplace(hb) for _, _, hb in reqs]
    oidx = oracle_index(full)
    pairs = 0
    for (r0, r1, hb), t in zip(reqs, tickets):
        rc, c, b, st = srv.wait(t)
        assert rc == 0, rc
        c0, c1 = int(sw["cand_off"][r0]), int(sw["cand_off"][r1])
        res = oracle.filter_compare(oidx, sw["q"], sw["codes"], sw["read_off"][r0:r1],
                                    sw["read_len"][r0:r1], sw["read_e"][r0:r1], sw["e_den"],
                                    sw["cand_off"][r0:r1 + 1] - c0, sw["cand_bin"][c0:c1], c, b,
                                    n_threads=N_THREADS)
        assert res["pairs"] == c1 - c0
        assert res["count_mismatches"] == 0 and res["bit_mismatches"] == 0, (r1 - r0, res)
        pairs += res["pairs"]
    s = srv.stats()
    say("served on the full index:", len(reqs), "requests,", pairs, "pairs, ticks", s["ticks"],
        "p99", s["p99_ms"])
    assert s["completed"] == len(reqs)
    # the largest request has more pairs than a tick holds, so it ran in parts
    assert reqs[0][2].n_pairs > 8 << 20
    srv.destroy()


def test_fullsize_windows_sampled_and_properties(full):
    """The bin-window leg as bench.py runs it: the batched 3.1 Gbp index, its
    token-major copy, the first 200,000 reads each against a 4096-bin window
    around its true bin that starts on a multiple of 1024 bins.  Sampled pairs against the oracle one by one; over every
    pair, 0 <= count <= ntok and pass == (count >= T); every true bin passes."""
    import torch
    if full["name"] != "batched":
        pytest.skip("the bin-window leg runs on the batched index")
    g, w, idx = full["g"], full["w"], full["idx"]
    idx.transpose()
    n_reads, wbins = 200_000, 4096
    nb = idx.n_bins
    tb = (w["read_z"][:n_reads] // w["B"]).astype(np.int64)
    lo = bench.window_lo(tb, nb, wbins, 1024).astype(np.int64)
    assert np.all((tb >= lo) & (tb - lo < wbins))  # the gather index below stays in range
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
    del c, counts, bits
