"""Benchmark of the MI355X GRIM-Filter hot path.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config batched] [--scale 1.0]

One step = one batched filter pass (work-list kernel + persistent filter
kernel, replayed from a HIP graph) over the whole synthetic batch, inputs
already resident in HBM.  Prints one JSON line on stdout; progress goes to
stderr.  Default workload: 3.1 Gbp synthetic reference with 45 % repeats,
q = 5, 200-bp bins (15.5M bins, 1.98 GB of bin vectors), 4M reads of
100/150/250 bp with e in {0.05, 0.10}, Zipf(1.2) candidate counts capped at
4096 (about 8.4e8 (read, bin) pairs).
"""
import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_pair(q):
    """Bytes the method must move per (read, bin) pair: the bin vector
    (4^q / 8), the 4-byte bin id, the 4-byte count and the 1/8-byte pass bit."""
    return (4 ** q) / 8 + 4 + 4 + 1 / 8


def algorithmic_bytes_per_read(w):
    """Per-read inputs: packed bases, read offset (8), length (4), tolerance (4),
    candidate offset (8)."""
    return float(np.mean(np.ceil(w["read_len"] / 4.0))) + 8 + 4 + 4 + 8


CONFIG_TEXT = {
    "tiny": "1 Mbp uniform reference, q=5, 200-bp bins; 10k x 100-bp reads (e=0.05); 64 candidates per read",
    "mid": "100 Mbp reference with 10% repeats, q=5, 200-bp bins; 1M x 100-bp reads (e=0.05); 12-mer seeded candidates",
    "batched": "3.1 Gbp reference with 45% repeats, q=5, 200-bp bins; 4M reads of 100/150/250 bp, e in {0.05,0.10}; Zipf(1.2) candidates <= 4096",
    "large": "3.1 Gbp reference with 45% repeats, q=6, 1000-bp bins; 2M x 250-bp reads (e=0.05); uniform 1-2048 candidates",
}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, target_pairs, n_threads, idx=None):
    """Time the oracle filter on the first reads of the workload (about
    target_pairs pairs) on the host cores."""
    import oracle
    t0 = time.time()
    if idx is None:
        idx = oracle.build_index(w["ref"], w["B"], w["O"], w["q"], n_threads=n_threads)
    t_build = time.time() - t0
    r1 = int(np.searchsorted(w["cand_off"], target_pairs, side="left"))
    r1 = max(1, min(r1, w["read_len"].size))
    sub_off = w["cand_off"][:r1 + 1]
    n_pairs = int(sub_off[-1])
    t0 = time.perf_counter()
    c, p, bad = oracle.filter_batch(idx, w["q"], w["codes"], w["read_off"][:r1], w["read_len"][:r1],
                                    w["read_e"][:r1], w["e_den"], sub_off,
                                    w["cand_bin"][:n_pairs], n_threads=n_threads)
    dt = time.perf_counter() - t0
    return dict(pairs=n_pairs, reads=r1, seconds=dt, build_seconds=t_build,
                pairs_per_s=n_pairs / dt), (c, p), idx


def cpu_baseline_leg(w, counts, bits, n_threads, cpu_pairs=0):
    """The oracle on the host cores (the CPU baseline, and the parity check of
    the timed launch): the oracle's index is built (untimed), then the oracle
    filter runs over every pair of the workload (or the first reads' pairs,
    about cpu_pairs of them), n_threads threads taking chunks of about 4M pairs,
    and every count and pass bit is compared with the GPU's (device tensors
    counts and bits).  A single-thread run over about 2e7 pairs follows.
    Returns (cpu_baseline dict, parity dict)."""
    import oracle
    n_pairs = int(w["cand_off"][-1])
    n_reads = int(w["read_len"].size)
    t0 = time.time()
    oidx = oracle.build_index(w["ref"], w["B"], w["O"], w["q"], n_threads=n_threads)
    t_build = time.time() - t0
    r1 = n_reads
    if cpu_pairs and cpu_pairs < n_pairs:
        r1 = max(1, int(np.searchsorted(w["cand_off"], int(cpu_pairs), side="left")))
    host_counts = counts[:n_pairs].cpu().numpy()
    host_bits = bits[:(n_pairs + 31) // 32].cpu().numpy().view(np.uint32)
    tc = time.perf_counter()
    res = oracle.filter_compare(oidx, w["q"], w["codes"], w["read_off"], w["read_len"],
                                w["read_e"], w["e_den"], w["cand_off"], w["cand_bin"],
                                host_counts, host_bits, r_end=r1, n_threads=n_threads)
    dt = time.perf_counter() - tc
    del host_counts, host_bits
    parity = dict(pairs=res["pairs"], reads=res["reads"], count_mismatches=res["count_mismatches"],
                  bit_mismatches=res["bit_mismatches"], first_mismatches=res["first"],
                  every_pair=res["pairs"] == n_pairs,
                  note="every count and pass bit of the timed launch against the oracle")
    c1, _, _ = cpu_baseline(w, int(2e7), 1, idx=oidx)
    cpu = {"value": res["pairs"] / dt, "unit": "candidate locations/s", "cores": n_threads,
           "kind": "oracle",
           "sample": f"reads [0, {r1}) of the workload ({res['pairs']} pairs), filter phase "
                     f"only (index build {t_build:.1f}s excluded), {dt:.1f}s on {n_threads} "
                     f"threads taking chunks of about 4M pairs",
           "single_thread_value": c1["pairs_per_s"],
           "single_thread_sample": f"first {c1['reads']} reads ({c1['pairs']} pairs), "
                                   f"{c1['seconds']:.1f}s on 1 thread",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    log(f"[bench] cpu oracle: {cpu['value']:.3e} pairs/s on {n_threads} threads ({dt:.1f}s); "
        f"parity over {res['pairs']} pairs: {res['count_mismatches']} count and "
        f"{res['bit_mismatches']} pass-bit mismatches (total {time.time() - t0:.1f}s)")
    return cpu, parity


def link_probe(torch, n_bytes=256 << 20, reps=5, pairs=4):
    """Host link rates (GB/s) with page-locked buffers: one direction at a
    time, then both at once on two streams (best of reps).  Copies on two
    streams do not always run on different copy engines (then the two
    directions take turns at the one-way rate), so both-at-once is tried on
    `pairs` freshly created stream pairs and the best is kept, with every
    pair's rate listed."""
    h = torch.empty(n_bytes, dtype=torch.uint8, pin_memory=True)
    h2 = torch.empty(n_bytes, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(n_bytes, dtype=torch.uint8, device="cuda")
    d2 = torch.empty(n_bytes, dtype=torch.uint8, device="cuda")

    def best(fn):
        fn()
        t = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        return n_bytes / min(t) / 1e9

    s1 = torch.cuda.Stream()

    def up(s=s1):
        with torch.cuda.stream(s):
            d.copy_(h, non_blocking=True)

    def down(s=s1):
        with torch.cuda.stream(s):
            h.copy_(d, non_blocking=True)

    both = []
    for _ in range(pairs):
        a, b = torch.cuda.Stream(), torch.cuda.Stream()

        def fn(a=a, b=b):
            up(a)
            with torch.cuda.stream(b):
                h2.copy_(d2, non_blocking=True)
        both.append(best(fn))
    out = dict(h2d_gbs=best(up), d2h_gbs=best(down), both_each_gbs=max(both),
               both_each_gbs_per_stream_pair=both)
    del h, h2, d, d2
    return out


def serving_leg(g, idx, w, rng, loads=(0.25, 0.5, 0.75, 0.9), n_requests=10_000, pool=256,
                max_reads=65536, inplace=True, tick_pairs=8 << 20, n_streams=3,
                max_inflight=1024, fixed_rates=None, bits_only=False, expect=None,
                ticks_per_stream=0):
    """Served latency.  A pool of `pool` requests of log-uniform size
    (1..max_reads reads) is cut from the workload.  First the server's capacity
    is measured closed-loop (a burst of requests submitted at once); then, for
    each offered load rho, n_requests requests arrive as a Poisson process at
    rho x capacity, each one a pool entry drawn at random among those not in
    flight, and the server's p50/p99 latency (submit -> results in host memory)
    is recorded.  inplace=True submits pinned request buffers without copying
    (results land in the request's pinned output buffers, so a buffer is in
    flight at most once at a time); False uses the copying submission.  Ticks
    hold at most tick_pairs pairs, so larger requests run in parts; n_streams
    ticks (and at most max_inflight requests) are in flight at once.  fixed_rates (pairs per second)
    replaces the loads relative to capacity by absolute arrival rates, so that
    server configurations can be compared at the same offered traffic.
    bits_only=True serves the pass bits alone (counts stay on the device).
    expect = (counts, pass-bit words) of the whole workload as host arrays:
    with in-place submission every request's results are compared with them."""
    n_reads = w["read_len"].size
    reqs, spans = [], []
    for _ in range(pool):
        size = int(min(n_reads, max(1, round(math.exp(rng.uniform(0, math.log(max_reads)))))))
        r0 = int(rng.integers(0, n_reads - size + 1))
        r1 = r0 + size
        o0 = int(w["read_off"][r0])
        o1 = int(w["read_off"][r1 - 1]) + int(w["read_len"][r1 - 1])
        c0, c1 = int(w["cand_off"][r0]), int(w["cand_off"][r1])
        reqs.append(g.HostBatch(w["codes"][o0:o1], w["read_off"][r0:r1] - o0, w["read_len"][r0:r1],
                                w["read_e"][r0:r1], w["e_den"], w["cand_off"][r0:r1 + 1] - c0,
                                w["cand_bin"][c0:c1], max_len=250, pinned=inplace))
        spans.append((r0, r1))
    mean_pairs = float(np.mean([hb.n_pairs for hb in reqs]))
    srv = g.Server(idx, hbm_budget_bytes=4 << 30, max_inflight=max_inflight, n_streams=n_streams,
                   max_tick_pairs=tick_pairs, max_len=256, pass_bits_only=bits_only,
                   ticks_per_stream=ticks_per_stream)
    submit = srv.submit_inplace if inplace else srv.submit

    def finish(rc, ticket):
        if rc != 0:
            raise RuntimeError(f"serving request {ticket} failed: {rc}")

    def drain(tickets):
        for t in tickets:
            finish(srv.wait(t)[0], t)

    # warm-up over the whole pool (first use of every buffer), then closed-loop
    # capacity: the whole pool submitted at once (each buffer is in flight at
    # most once at a time), six times; pairs over the median wall time
    drain([submit(hb) for hb in reqs])
    srv.stats(reset=True)
    walls = []
    for _ in range(6):
        t0 = time.perf_counter()
        drain([submit(hb) for hb in reqs])
        walls.append(time.perf_counter() - t0)
    capacity = sum(hb.n_pairs for hb in reqs) / float(np.median(walls))
    cap_stats = srv.stats(reset=True)
    # host thread time during the bursts, against their wall time: the
    # workers' mean occupancy (staging, queuing, retiring) and the admission
    # thread's
    workers = n_streams * (ticks_per_stream or 2)  # 2: the server's default
    worker_busy = (cap_stats["sched_launch_s"] + cap_stats["sched_retire_s"]) / \
        max(1e-9, workers * sum(walls))
    admit_busy = cap_stats["sched_admit_s"] / max(1e-9, sum(walls))
    checked = None
    if expect is not None and inplace and not bits_only:
        # every pool request's results, as the capacity bursts left them, against
        # the timed batched launch's results for the same pairs (which the CPU
        # baseline leg compares with the oracle pair by pair)
        ec, eb = expect
        checked = dict(requests=0, pairs=0, count_mismatches=0, bit_mismatches=0,
                       largest_request_reads=max(r1 - r0 for r0, r1 in spans))
        for (r0, r1), hb in zip(spans, reqs):
            c0, c1 = int(w["cand_off"][r0]), int(w["cand_off"][r1])
            n = c1 - c0
            want_bits = np.unpackbits(eb.view(np.uint8)[c0 >> 3:(c1 + 7) >> 3],
                                      bitorder="little")[c0 & 7:(c0 & 7) + n]
            got_bits = np.unpackbits(hb.out_bits.view(np.uint8), bitorder="little")[:n]
            checked["requests"] += 1
            checked["pairs"] += n
            checked["count_mismatches"] += int(np.count_nonzero(hb.out_counts[:n] != ec[c0:c1]))
            checked["bit_mismatches"] += int(np.count_nonzero(got_bits != want_bits))
        log(f"[bench] served results against the batched launch: {checked}")
    # bytes each request moves over the host link: inputs one way, counts and
    # pass bits (the tick's bits via the stage, then ORed in) back
    n_pairs_all = sum(hb.n_pairs for hb in reqs)
    up_bytes = sum(hb.words.size * 4 + hb.n_reads * 24 + 8 + hb.n_pairs * 4 for hb in reqs)
    down_bytes = sum((0 if bits_only else hb.n_pairs * 4) + ((hb.n_pairs + 31) // 32) * 4
                     for hb in reqs)
    out = dict(mode=("in place, pinned buffers" if inplace else "copying submission") +
               (", pass bits only" if bits_only else ""),
               pool_requests=pool, mean_pairs_per_request=mean_pairs,
               max_tick_pairs=tick_pairs, n_streams=n_streams, max_inflight=max_inflight,
               ticks_per_stream=ticks_per_stream or 2,
               capacity_burst_s=walls,
               capacity_pairs_per_s=capacity,
               capacity_ticks=cap_stats["ticks"],
               capacity_worker_busy=worker_busy,
               capacity_admission_busy=admit_busy,
               stream_groups=cap_stats["stream_groups"],
               results_checked=checked,
               link_bytes_per_pair=dict(up=up_bytes / n_pairs_all, down=down_bytes / n_pairs_all),
               points=[])
    points = [(rho, rho * capacity) for rho in loads] if fixed_rates is None else \
        [(r / capacity, r) for r in fixed_rates]
    for rho, pair_rate in points:
        rate = pair_rate / mean_pairs               # requests per second
        gaps = rng.exponential(1.0 / rate, size=n_requests)
        free = list(range(pool))
        flying = {}                                 # ticket -> pool entry
        late = 0
        t_start = time.perf_counter()
        t_next = t_start
        for i in range(n_requests):
            t_next += gaps[i]
            # reap finished requests while waiting for the next arrival
            while True:
                for t in list(flying):
                    rc = srv.poll(t)[0]
                    if rc != g.GRIM_PENDING:
                        finish(rc, t)
                        free.append(flying.pop(t))
                d = t_next - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(min(d, 2e-4))
            if not free:                            # every pool entry in flight
                t = next(iter(flying))
                finish(srv.wait(t)[0], t)
                free.append(flying.pop(t))
                late += 1
            j = int(rng.integers(len(free)))
            free[j], free[-1] = free[-1], free[j]
            k = free.pop()
            flying[submit(reqs[k])] = k
        drain(list(flying))
        wall = time.perf_counter() - t_start
        st = srv.stats(reset=True)
        out["points"].append(dict(offered_load=rho, offered_rps=rate, requests=n_requests,
                                  wall_s=wall, p50_ms=st["p50_ms"], p99_ms=st["p99_ms"],
                                  mean_ms=st["mean_ms"], max_ms=st["max_ms"],
                                  pairs_per_s=st["pairs_done"] / wall,
                                  mean_requests_per_tick=st["mean_requests_per_tick"],
                                  sched_launch_s=st["sched_launch_s"],
                                  sched_retire_s=st["sched_retire_s"],
                                  sched_admit_s=st["sched_admit_s"],
                                  ticks=st["ticks"],
                                  arrivals_delayed_by_full_pool=late))
    srv.destroy()
    mid = next(p for p in out["points"] if p["offered_load"] == 0.5) \
        if any(p["offered_load"] == 0.5 for p in out["points"]) else out["points"][0]
    out["p50_ms"], out["p99_ms"] = mid["p50_ms"], mid["p99_ms"]
    return out


def seeding_leg(g, torch, stream):
    """The step before the filter, on the mid recipe (100 Mbp reference with 10 %
    repeats, 1M reads of 100 bp, exact 12-mer seeds at read offsets 0, 12, ...,
    200-bp bins, <= 4096 bins per read): k-mer index and candidate lists on the
    GPU, then the filter and the survivor list on those candidates.  Reports
    the share of reads whose true bin is among their candidates."""
    import grim_synth as gs
    t0 = time.time()
    wm = gs.WORKLOADS["mid"]
    ref = gs.make_reference("mid")
    rd = gs.reads(gs.SEEDS["reads"], ref, wm["n_reads"], wm["lengths"], wm["e_nums"], gs.E_DEN)
    n = int(rd["read_len"].size)
    rb = g.Batch(rd["codes"], rd["read_off"], rd["read_len"], rd["read_e"], gs.E_DEN,
                 np.zeros(n + 1, np.uint64), np.zeros(0, np.uint32), max_len=int(wm["lengths"][0]))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    si = g.SeedIndex(ref, 12)
    e1.record(stream)
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    cands = g.grim_seed_candidates(si, rb, wm["B"], 4096)
    e0.record(stream)
    for _ in range(3):
        g.grim_seed_candidates(si, rb, wm["B"], 4096).free()
    e1.record(stream)
    torch.cuda.synchronize()
    cand_ms = e0.elapsed_time(e1) / 3
    off, bins = cands.to_host()
    # true bin among the read's candidates: pairs keyed (read, bin) are sorted
    tb = (rd["read_z"] // wm["B"]).astype(np.int64)
    reads_of = np.repeat(np.arange(n, dtype=np.int64), np.diff(off.astype(np.int64)))
    keys = (reads_of << 32) | bins.astype(np.int64)
    want = (np.arange(n, dtype=np.int64) << 32) | tb
    at = np.minimum(np.searchsorted(keys, want), max(0, keys.size - 1))
    found = int(np.count_nonzero(keys[at] == want)) if keys.size else 0
    del reads_of, keys, want, at
    # the filter and the checker on the seeded candidates
    idx = g.grim_build_bins(ref, wm["q"], wm["B"], wm["O"])
    fb = g.batch_with_candidates(rb, cands)
    np_ = fb.n_pairs
    c, bb = g.alloc_outputs(np_)
    ws = g.alloc_workspace(idx, np_)
    g.grim_filter_batch(idx, fb, c, bb, ws)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(5):
        g.grim_filter_batch(idx, fb, c, bb, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    filt_ms = e0.elapsed_time(e1) / 5
    rc, _ = g.grim_filter_status(ws)
    sp, sr, sb, total = g.grim_compact_survivors(fb, bb)
    out = dict(recipe="mid: 100 Mbp, 10 % repeats, 1M x 100 bp, exact 12-mer seeds, 200-bp bins",
               index_build_ms=build_ms, candidates_ms=cand_ms,
               reads_per_s=n / (cand_ms * 1e-3), pairs=int(np_),
               true_bin_found=found / n, filter_ms=filt_ms, filter_status=rc,
               survivors=int(total),
               note="seeding calls are synchronous and include the library's temporary "
                    "allocations; the candidate lists equal the host generator's (bench.py "
                    "--config mid, tests/test_gpu_seed.py)")
    log(f"[bench] seeding (mid recipe): index {build_ms:.1f} ms, candidates {cand_ms:.2f} ms for "
        f"{n} reads -> {np_} pairs, true bin found for {100 * found / n:.2f} % of reads; filter "
        f"{filt_ms:.3f} ms, {total} survivors ({time.time() - t0:.1f}s)")
    del sp, sr, sb, c, bb, ws, fb
    cands.free()
    si.free()
    idx.free()
    return out


def window_lo(tb, n_bins, window_bins=4096, align=1024):
    """First bin of each read's window: window_bins bins around its true bin
    tb, starting on a multiple of `align` bins (1: no alignment), inside the
    index.  A window that would run past the last bin starts at
    n_bins - window_bins instead (unaligned); the true bin is always inside."""
    tb = np.asarray(tb, dtype=np.int64)
    lo = np.maximum(tb - window_bins // 2, 0)
    lo = (lo // align) * align
    last = max(0, n_bins - window_bins)
    lo = np.where(lo > last, last, lo)
    assert np.all((tb >= lo) & (tb < lo + window_bins)), "a true bin outside its window"
    return lo.astype(np.uint32)


def window_leg(g, idx, w, torch, stream, rng, window_bins=4096, n_reads=200_000, align=1024):
    """The bin-window form: each of n_reads reads against the window_bins
    consecutive bins around its true bin, from the token-major index copy.  The
    mapper's windows start on multiples of `align` bins (a 4096-bin window then
    covers exactly four 128-byte lines of every token row); the same windows
    unaligned are timed as well.  Compared with the batched random-gather
    kernel on the same explicit pairs (identical outputs checked) and timed
    with HIP events."""
    n_reads = min(n_reads, w["read_len"].size)
    n_bins = idx.n_bins
    tb = (w["read_z"][:n_reads] // w["B"]).astype(np.int64)
    lo = window_lo(tb, n_bins, window_bins, align)
    lo_unaligned = window_lo(tb, n_bins, window_bins, 1)
    assert np.all((tb >= lo) & (tb < lo.astype(np.int64) + window_bins))
    off = np.arange(n_reads + 1, dtype=np.uint64) * window_bins
    o_end = int(w["read_off"][n_reads - 1]) + int(w["read_len"][n_reads - 1])
    t0 = time.time()
    idx.transpose()
    torch.cuda.synchronize()
    t_transpose = time.time() - t0
    wb = g.Batch(w["codes"][:o_end], w["read_off"][:n_reads], w["read_len"][:n_reads],
                 w["read_e"][:n_reads], w["e_den"], off, np.zeros(1, np.uint32),
                 max_len=int(w["read_len"].max()))
    n = wb.n_pairs
    wl = torch.from_numpy(lo.view(np.int32)).cuda()
    c1, b1 = g.alloc_outputs(n)
    ws = torch.zeros(256, dtype=torch.uint8, device="cuda")
    g.grim_filter_windows(idx, wb, wl, c1, b1, ws)
    rc, _ = g.grim_filter_status(ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        g.grim_filter_windows(idx, wb, wl, c1, b1, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    # the same reads with windows that start anywhere (row segments then span
    # five 128-byte lines)
    wlu = torch.from_numpy(lo_unaligned.view(np.int32)).cuda()
    cu, bu = g.alloc_outputs(n)
    g.grim_filter_windows(idx, wb, wlu, cu, bu, ws)
    rc_unaligned, _ = g.grim_filter_status(ws)
    e0.record(stream)
    for _ in range(5):
        g.grim_filter_windows(idx, wb, wlu, cu, bu, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_unaligned = e0.elapsed_time(e1) / 5
    del cu, bu, wlu
    # the same reads submitted sorted by window start (a caller's choice, made on
    # the host outside the timing): concurrent workgroups then share row
    # segments through L2; outputs equal the index-order ones per (read, bin)
    perm = np.argsort(lo, kind="stable")
    lens = w["read_len"][:n_reads][perm].astype(np.int64)
    starts = w["read_off"][:n_reads][perm].astype(np.int64)
    pos = np.zeros(n_reads, np.int64)
    pos[1:] = np.cumsum(lens[:-1])
    gather = np.repeat(starts - pos, lens) + np.arange(int(lens.sum()))
    sb = g.Batch(w["codes"][gather], pos.astype(np.uint64), lens.astype(np.uint32),
                 w["read_e"][:n_reads][perm], w["e_den"], off, np.zeros(1, np.uint32),
                 max_len=int(w["read_len"].max()))
    del gather
    swl = torch.from_numpy(lo[perm].view(np.int32)).cuda()
    cs, bs = g.alloc_outputs(n)
    g.grim_filter_windows(idx, sb, swl, cs, bs, ws)
    rc_sorted, _ = g.grim_filter_status(ws)
    e0.record(stream)
    for _ in range(5):
        g.grim_filter_windows(idx, sb, swl, cs, bs, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_sorted = e0.elapsed_time(e1) / 5
    tperm = torch.from_numpy(perm).cuda()
    same_sorted = bool(torch.equal(cs[:n].view(n_reads, window_bins),
                                   c1[:n].view(n_reads, window_bins)[tperm]))
    del cs, bs, sb, swl, tperm
    # the reads in index order, processed in the device-side order (reads
    # grouped by window-start bucket): the order and the filter timed together
    co, bo = g.alloc_outputs(n)
    order_ws = torch.empty(g.grim_window_order_workspace_size(idx, n_reads), dtype=torch.uint8,
                           device="cuda")
    order = torch.empty(n_reads, dtype=torch.int32, device="cuda")
    g.grim_window_order(idx, wl, order=order, workspace=order_ws)
    g.grim_filter_windows(idx, wb, wl, co, bo, ws, order=order)
    rc_order, _ = g.grim_filter_status(ws)
    e0.record(stream)
    for _ in range(5):
        g.grim_window_order(idx, wl, order=order, workspace=order_ws)
        g.grim_filter_windows(idx, wb, wl, co, bo, ws, order=order)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_order = e0.elapsed_time(e1) / 5
    e0.record(stream)
    for _ in range(5):
        g.grim_window_order(idx, wl, order=order, workspace=order_ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_order_only = e0.elapsed_time(e1) / 5
    same_order = bool(torch.equal(co[:n], c1[:n]) and
                      torch.equal(bo[:(n + 31) // 32], b1[:(n + 31) // 32]))
    del co, bo, order, order_ws
    # the same pairs as explicit candidates through the batched kernel
    cb = (lo.astype(np.int64)[:, None] + np.arange(window_bins)[None, :]).astype(np.uint32).ravel()
    eb = g.Batch(w["codes"][:o_end], w["read_off"][:n_reads], w["read_len"][:n_reads],
                 w["read_e"][:n_reads], w["e_den"], off, cb, max_len=int(w["read_len"].max()))
    del cb
    c2, b2 = g.alloc_outputs(n)
    ws2 = g.alloc_workspace(idx, n)
    g.grim_filter_batch(idx, eb, c2, b2, ws2)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(3):
        g.grim_filter_batch(idx, eb, c2, b2, ws2)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_batched = e0.elapsed_time(e1) / 3
    same = bool(torch.equal(c1[:n], c2[:n]) and torch.equal(b1[:(n + 31) // 32], b2[:(n + 31) // 32]))
    ntok = float(np.mean(np.maximum(w["read_len"][:n_reads].astype(np.int64) - w["q"] + 1, 0)))
    row_bytes = ntok * window_bins / 8 + window_bins * (4 + 1 / 8)
    out = dict(window_bins=window_bins, window_align_bins=align, reads=n_reads, pairs=n, ms=ms,
               pairs_per_s=n / (ms * 1e-3),
               status=rc, identical=same, batched_same_pairs_ms=ms_batched,
               speedup_vs_batched_same_pairs=ms_batched / ms, transpose_s=t_transpose,
               algorithmic_bytes_per_window=row_bytes,
               algorithmic_gbs=n_reads * row_bytes / (ms * 1e-3) / 1e9,
               unaligned=dict(ms=ms_unaligned, pairs_per_s=n / (ms_unaligned * 1e-3),
                              status=rc_unaligned,
                              algorithmic_gbs=n_reads * row_bytes / (ms_unaligned * 1e-3) / 1e9),
               device_order=dict(note="index-order reads processed in the order of "
                                      "grim_window_order (reads grouped by window-start "
                                      "bucket); order + filter timed together",
                                 ms=ms_order, order_ms=ms_order_only,
                                 pairs_per_s=n / (ms_order * 1e-3), status=rc_order,
                                 identical=same_order),
               presorted=dict(note="the same reads submitted sorted by window start "
                                   "(host argsort outside the timing)",
                              ms=ms_sorted, pairs_per_s=n / (ms_sorted * 1e-3),
                              status=rc_sorted, identical_per_read_bin=same_sorted))
    del c1, b1, c2, b2, ws2, wb, eb
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="batched", choices=sorted(CONFIG_TEXT))
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=10_000,
                    help="requests offered per serving load point")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-kernel comparison")
    ap.add_argument("--no-tune", action="store_true", help="use the default launch shape")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches instead of HIP-graph replays (for counter runs)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (counter calibration)")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--cpu-pairs", type=float, default=0,
                    help="compare only the first reads' pairs (about this many) with the oracle "
                         "(0: every pair)")
    ap.add_argument("--no-window", action="store_true", help="skip the bin-window leg")
    ap.add_argument("--no-seed", action="store_true",
                    help="skip the GPU seeding leg (mid recipe) of the default workload")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the memory-ceiling probes (gather and streaming read)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the filter would shard by replicating the "
              "index and splitting reads across GPUs, with no exchange, and runs on several "
              "GPUs are not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import grim_synth as gs
    import paper_1711_01177_amd as g

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    rng = np.random.default_rng(2024)
    n_threads = gs.default_threads()

    t0 = time.time()
    w = gs.make_workload(args.config, scale=args.scale, n_threads=n_threads)
    n_pairs = int(w["cand_off"][-1])
    n_reads = int(w["read_len"].size)
    log(f"[bench] workload {args.config} x{args.scale}: G={w['ref'].size} reads={n_reads} "
        f"pairs={n_pairs} ({time.time() - t0:.1f}s)")

    t0 = time.time()
    idx = g.grim_build_bins(w["ref"], w["q"], w["B"], w["O"])
    torch.cuda.synchronize()
    log(f"[bench] index: {idx.n_bins} bins, {idx.bytes / 1e9:.3f} GB ({time.time() - t0:.1f}s)")
    t0 = time.time()
    max_len_batch = int(w["read_len"].max())
    batch = g.Batch.from_workload(w, max_len=max_len_batch)
    counts, bits = g.alloc_outputs(n_pairs)
    torch.cuda.synchronize()
    log(f"[bench] inputs resident ({time.time() - t0:.1f}s)")

    seeding = None
    if args.config == "mid":
        # the candidates of this recipe come from exact 12-mer seeds: do that step
        # on the GPU too and check it gives the same lists as the host generator
        t0 = time.time()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        si = g.SeedIndex(w["ref"], 12)
        ev1.record()
        torch.cuda.synchronize()
        build_ms = ev0.elapsed_time(ev1)
        cands = g.grim_seed_candidates(si, batch, w["B"], 4096)
        ev0.record()
        for _ in range(3):
            c2 = g.grim_seed_candidates(si, batch, w["B"], 4096)
            c2.free()
        ev1.record()
        torch.cuda.synchronize()
        cand_ms = ev0.elapsed_time(ev1) / 3
        off_d, bins_d = cands.to_host()
        same = bool(np.array_equal(off_d, w["cand_off"]) and np.array_equal(bins_d, w["cand_bin"]))
        seeding = dict(k=12, index_build_ms=build_ms, candidates_ms=cand_ms,
                       reads_per_s=n_reads / (cand_ms * 1e-3), pairs=int(cands.n_pairs),
                       identical_to_host_seeding=same,
                       note="synchronous calls; include the library's temporary allocations")
        log(f"[bench] GPU seeding: index {build_ms:.1f} ms, candidates {cand_ms:.1f} ms for "
            f"{n_reads} reads -> {cands.n_pairs} pairs, identical={same} ({time.time() - t0:.1f}s)")
        cands.free()
        si.free()

    tune = None
    if args.lanes or args.unroll or args.tile or args.wg:
        tune = g.tuning(args.lanes, args.unroll, args.tile, args.wg)
    ws = g.alloc_workspace(idx, n_pairs, tune)
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {n} bytes")
        del src, dst
    if not args.no_tune and tune is None:
        t0 = time.time()
        tune = g.grim_tune(idx, batch, counts, bits, ws)
        log(f"[bench] tuned {tune.as_dict()} ({time.time() - t0:.1f}s)")
    eff = tune if tune is not None else g.grim_default_tuning(w["q"])

    # correctness of the timed configuration before timing it
    g.grim_filter_batch(idx, batch, counts, bits, ws, tune)
    rc, flags = g.grim_filter_status(ws)
    if rc != 0:
        raise RuntimeError(f"filter status {rc} flags {flags}")

    stream = torch.cuda.current_stream()
    if args.no_graph:
        def step():
            g.grim_filter_batch(idx, batch, counts, bits, ws, tune)
    else:
        graph = g.grim_graph_create(idx, batch, counts, bits, ws, tune)

        def step():
            graph.launch()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    step_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms = float(np.mean(step_ms))
    rc, flags = g.grim_filter_status(ws)
    if rc != 0:
        raise RuntimeError(f"filter status {rc} flags {flags}")
    log(f"[bench] {'eager' if args.no_graph else 'graph'} steps: mean {ms:.3f} ms  min {min(step_ms):.3f}  max {max(step_ms):.3f}  "
        f"wall {wall * 1e3 / args.steps:.3f} ms/step")

    # eager launches (no graph) for comparison
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(3):
        g.grim_filter_batch(idx, batch, counts, bits, ws, tune)
    e1.record(stream)
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / 3

    q = w["q"]
    bpp = algorithmic_bytes_per_pair(q)
    bpr = algorithmic_bytes_per_read(w)
    alg_bytes = n_pairs * bpp + n_reads * bpr
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    pairs_per_s = n_pairs / (ms * 1e-3)

    # memory ceilings of the same accesses: the filter's gather without its
    # token work (same bin ids, 4-byte result per pair), and a streaming read
    probes = None
    if not args.no_probe:
        pout = torch.empty(max(1, n_pairs), dtype=torch.int32, device="cuda")
        g.grim_probe_gather(idx, batch.cand_bin, pout, n=n_pairs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            g.grim_probe_gather(idx, batch.cand_bin, pout, n=n_pairs)
        e1.record(stream)
        torch.cuda.synchronize()
        gms = e0.elapsed_time(e1) / 5
        del pout
        sink = torch.zeros(1, dtype=torch.int32, device="cuda")
        g.grim_probe_stream(idx, sink)
        e0.record(stream)
        for _ in range(5):
            g.grim_probe_stream(idx, sink)
        e1.record(stream)
        torch.cuda.synchronize()
        sms = e0.elapsed_time(e1) / 5
        vb = idx.bytes // idx.n_bins
        gather_gbs = n_pairs * (vb + 8) / (gms * 1e-3) / 1e9
        probes = dict(gather_ms=gms, gather_gbs=gather_gbs, gather_bytes_per_pair=vb + 8,
                      stream_read_gbs=idx.bytes / (sms * 1e-3) / 1e9,
                      filter_time_over_gather=ms / gms)
        log(f"[bench] probes: gather of the same bin ids {gms:.3f} ms ({gather_gbs:.0f} GB/s), "
            f"streaming read {probes['stream_read_gbs']:.0f} GB/s; filter / gather time "
            f"{ms / gms:.3f}")

    plain = None
    if not args.no_plain:
        c2, b2 = g.alloc_outputs(n_pairs)
        g.grim_filter_plain(idx, batch, c2, b2, ws)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(2):
            g.grim_filter_plain(idx, batch, c2, b2, ws)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / 2
        same = bool(torch.equal(c2[:n_pairs], counts[:n_pairs]) and
                    torch.equal(b2[:(n_pairs + 31) // 32], bits[:(n_pairs + 31) // 32]))
        plain = dict(ms=pms, pairs_per_s=n_pairs / (pms * 1e-3), batched_speedup=pms / ms,
                     identical_to_batched=same)
        log(f"[bench] plain per-read kernel: {pms:.3f} ms ({pms / ms:.2f}x slower), identical={same}")
        del c2, b2

    # seed location checker: compact the pass bits into the survivor list
    sp, sr, sb, total = g.grim_compact_survivors(batch, bits)
    torch.cuda.synchronize()
    ref_total = int(torch.sum(torch.bitwise_and(
        bits[:(n_pairs + 31) // 32].view(torch.uint8).to(torch.int32)[:, None] >>
        torch.arange(8, device="cuda", dtype=torch.int32)[None, :], 1)).item())
    # time the library call alone: outputs and workspace allocated once, no
    # read-back of the total inside the timed region
    cout = (torch.empty(max(1, total), dtype=torch.int64, device="cuda"),
            torch.empty(max(1, total), dtype=torch.int32, device="cuda"),
            torch.empty(max(1, total), dtype=torch.int32, device="cuda"),
            torch.zeros(1, dtype=torch.int64, device="cuda"))
    cws = torch.empty(g.grim_survivors_workspace_size(n_pairs), dtype=torch.uint8, device="cuda")
    e0.record(stream)
    for _ in range(5):
        g.grim_compact_survivors(batch, bits, out=cout, workspace=cws, read_total=False)
    e1.record(stream)
    torch.cuda.synchronize()
    cms = e0.elapsed_time(e1) / 5
    same_list = bool(int(cout[3].item()) == total and torch.equal(cout[1][:total], sr[:total]) and
                     torch.equal(cout[2][:total], sb[:total]))
    del cout, cws
    # pass bits read by the count and the emit pass, 16 B written and a 4-B bin id
    # read per survivor
    cbytes = 2 * n_pairs / 8 + total * (8 + 4 + 4 + 4)
    checker = dict(ms=cms, survivors=total, popcount_matches=(total == ref_total),
                   pass_rate=total / max(1, n_pairs), algorithmic_gbs=cbytes / (cms * 1e-3) / 1e9,
                   repeat_identical=same_list,
                   note="library call only (3 kernels), outputs preallocated")
    log(f"[bench] checker: {total} survivors in {cms:.3f} ms")
    if max_len_batch <= 512:
        idx.attach_reference(w["ref"])
        dist, okb = g.grim_verify_survivors(idx, batch, sr, sb, total)
        torch.cuda.synchronize()
        e0.record(stream)
        g.grim_verify_survivors(idx, batch, sr, sb, total)
        e1.record(stream)
        torch.cuda.synchronize()
        vms = e0.elapsed_time(e1)
        n_ok = int(torch.sum(torch.bitwise_and(
            okb.view(torch.uint8).to(torch.int32)[:, None] >>
            torch.arange(8, device="cuda", dtype=torch.int32)[None, :], 1)).item())
        # the paper's false negative rate (Section 5): the share of locations
        # that pass the filter but do not align within E edits
        checker.update(verify_ms=vms, verified=n_ok,
                       false_negative_rate=(total - n_ok) / max(1, total),
                       verify_survivors_per_s=total / (vms * 1e-3))
        log(f"[bench] alignment check: {n_ok}/{total} survivors within E edits, {vms:.3f} ms")
        del dist, okb
    del sp, sr, sb

    if args.config == "batched" and not args.no_seed:
        seeding = seeding_leg(g, torch, stream)

    window = None
    if args.config == "batched" and not args.no_window:
        window = window_leg(g, idx, w, torch, stream, rng)
        log(f"[bench] bin windows ({window['window_bins']} bins): {window['pairs']} pairs in "
            f"{window['ms']:.3f} ms -> {window['pairs_per_s']:.3e} pairs/s "
            f"(batched random-gather form: {pairs_per_s:.3e}); identical={window['identical']}; "
            f"reads pre-sorted by window: {window['presorted']['ms']:.3f} ms, "
            f"identical={window['presorted']['identical_per_read_bin']}; device order + filter: "
            f"{window['device_order']['ms']:.3f} ms (order {window['device_order']['order_ms']:.3f} ms), "
            f"identical={window['device_order']['identical']}")

    cpu, parity = None, None
    if not args.no_cpu:
        cpu, parity = cpu_baseline_leg(w, counts, bits, n_threads, args.cpu_pairs)

    serving = None
    if not args.no_serve:
        try:
            t0 = time.time()
            link = link_probe(torch)
            expect = (counts[:n_pairs].cpu().numpy(),
                      bits[:(n_pairs + 31) // 32].cpu().numpy().view(np.uint32))
            serving = serving_leg(g, idx, w, rng, n_requests=args.serve_requests, inplace=True,
                                  expect=expect)
            del expect
            # the link ceiling: both directions at once, the busier one decides
            link_bpp = serving["link_bytes_per_pair"]
            ceiling = link["both_each_gbs"] * 1e9 / max(link_bpp["up"], link_bpp["down"])
            serving["link"] = dict(link, ceiling_pairs_per_s=ceiling,
                                   capacity_frac_of_ceiling=serving["capacity_pairs_per_s"] / ceiling)
            log(f"[bench] host link: {link['h2d_gbs']:.1f} GB/s up, {link['d2h_gbs']:.1f} down, "
                f"{link['both_each_gbs']:.1f} each way at once -> serving ceiling {ceiling:.3e} "
                f"pairs/s ({link_bpp['up']:.2f} B up, {link_bpp['down']:.2f} B down per pair)")
            serving["copying_submission"] = serving_leg(g, idx, w, rng, loads=(0.5,),
                                                        n_requests=args.serve_requests,
                                                        inplace=False)
            for pt in serving["points"] + serving["copying_submission"]["points"]:
                log(f"[bench] serving at {pt['offered_load']:.2f} x capacity "
                    f"({pt['offered_rps']:.0f} req/s): p50 {pt['p50_ms']:.2f} ms "
                    f"p99 {pt['p99_ms']:.2f} ms, {pt['pairs_per_s']:.3e} pairs/s")
            bo = serving_leg(g, idx, w, rng, loads=(0.25, 0.5), n_requests=args.serve_requests,
                             inplace=True, bits_only=True)
            # pass bits only: the host-to-device direction alone decides
            bo_ceiling = link["h2d_gbs"] * 1e9 / bo["link_bytes_per_pair"]["up"]
            bo["link"] = dict(ceiling_pairs_per_s=bo_ceiling,
                              capacity_frac_of_ceiling=bo["capacity_pairs_per_s"] / bo_ceiling)
            serving["pass_bits_only"] = bo
            for pt in bo["points"]:
                log(f"[bench] serving pass bits only at {pt['offered_load']:.2f} x capacity "
                    f"({pt['offered_rps']:.0f} req/s): p50 {pt['p50_ms']:.2f} ms "
                    f"p99 {pt['p99_ms']:.2f} ms, {pt['pairs_per_s']:.3e} pairs/s")
            log(f"[bench] serving capacity {serving['capacity_pairs_per_s']:.3e} pairs/s in place "
                f"({100 * serving['link']['capacity_frac_of_ceiling']:.0f} % of the link ceiling), "
                f"{serving['copying_submission']['capacity_pairs_per_s']:.3e} copying, "
                f"{bo['capacity_pairs_per_s']:.3e} pass bits only "
                f"({100 * bo['link']['capacity_frac_of_ceiling']:.0f} % of its ceiling) "
                f"({time.time() - t0:.1f}s)")
        except Exception as ex:  # report, keep the throughput line
            serving = dict(error=str(ex))
            log(f"[bench] serving leg failed: {ex}")

    traffic = None
    try:
        import hashlib
        with open(args.traffic_json) as f:
            tj = json.load(f)
        rec = tj.get(f"{args.config}@{args.scale:g}")
        with open(os.path.join(ROOT, "paper_1711_01177_amd", "csrc", "grim_kernels.hip"), "rb") as f:
            src_hash = hashlib.sha1(f.read()).hexdigest()
        # the bytes a launch moves depend on the kernel and its lane/unroll shape,
        # not on the tile size or the number of workgroups per CU
        shape = [eff.lanes_per_cand, eff.unroll]
        if rec and rec["kernel_source_sha1"] == src_hash and rec["tuning"][:2] == shape:
            traffic = rec["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        traffic = None

    out = {
        "metric": "candidate locations filtered/sec and HBM GB/s (% peak); p99 latency served",
        "value": pairs_per_s,
        "unit": "candidate locations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "step_ms_median": float(np.median(step_ms)),
        "step_ms_min_max": [float(min(step_ms)), float(max(step_ms))],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded generators; no dataset)",
        "config": {"workload": f"{args.config}: {CONFIG_TEXT[args.config]}" +
                               ("" if args.scale == 1.0 else f" (scaled x{args.scale:g})"),
                   "genome_bp": int(w["ref"].size), "n_reads": n_reads, "n_pairs": n_pairs,
                   "q": q, "bin_stride": w["B"], "overlap": w["O"], "n_bins": idx.n_bins,
                   "index_bytes": idx.bytes, "tuning": eff.as_dict(), "hip_graph": not args.no_graph,
                   "autotuned": bool(not args.no_tune and not (args.lanes or args.unroll or
                                                               args.tile or args.wg))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     # counter-measured bytes of one launch over this run's step time
                     "traffic_gbs": (traffic / (ms * 1e-3) / 1e9) if traffic else None,
                     # the same gather without the filter's work, measured in this run
                     "gather_ceiling_gbs": probes["gather_gbs"] if probes else None,
                     "frac_of_gather_ceiling": (probes["gather_ms"] / ms) if probes else None,
                     "stream_read_gbs": probes["stream_read_gbs"] if probes else None,
                     "bytes_per_pair": bpp, "bytes_per_read": bpr,
                     "kernel": "filter_batched_kernel (+ worklist_kernel, in the same timing)"},
        "eager_ms_per_step": eager_ms,
        "probes": probes,
        "plain_kernel": plain,
        "seed_location_checker": checker,
        "seeding": seeding,
        "bin_window": window,
        "parity": parity,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
