"""Serving (continuous batching) on the GPU: every request's result is the same
alone and in the mix, admission respects the HBM budget, an invalid bin id
fails only its own request, cancellation works."""
import sys
import threading
import time

import numpy as np
import pytest

import grim_synth as gs
import oracle
from tests.gpu_helpers import lib

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    g = lib()
    w = gs.make_workload("serve", scale=0.003)  # 9.3 Mbp, 12k reads, Zipf candidates
    idx = g.grim_build_bins(w["ref"], w["q"], w["B"], w["O"])
    w["oidx"] = oracle.build_index(w["ref"], w["B"], w["O"], w["q"], n_threads=gs.default_threads())
    return g, w, idx


def oracle_check(w, sub, c, b):
    """A request's counts and pass bits against the oracle, pair by pair."""
    res = oracle.filter_compare(w["oidx"], w["q"], sub["codes"], sub["read_off"], sub["read_len"],
                                sub["read_e"], sub["e_den"], sub["cand_off"], sub["cand_bin"],
                                c, b, n_threads=gs.default_threads())
    assert res["pairs"] == int(sub["cand_off"][-1])
    return res["count_mismatches"] == 0 and res["bit_mismatches"] == 0


def cut(g, w, r0, r1, max_len=256):
    o0 = int(w["read_off"][r0])
    o1 = int(w["read_off"][r1 - 1]) + int(w["read_len"][r1 - 1])
    c0, c1 = int(w["cand_off"][r0]), int(w["cand_off"][r1])
    sub = dict(codes=w["codes"][o0:o1], read_off=w["read_off"][r0:r1] - o0,
               read_len=w["read_len"][r0:r1], read_e=w["read_e"][r0:r1], e_den=w["e_den"],
               cand_off=w["cand_off"][r0:r1 + 1] - c0, cand_bin=w["cand_bin"][c0:c1].copy(),
               ref=w["ref"], q=w["q"], B=w["B"], O=w["O"])
    hb = g.HostBatch(sub["codes"], sub["read_off"], sub["read_len"], sub["read_e"], sub["e_den"],
                     sub["cand_off"], sub["cand_bin"], max_len=max_len)
    return sub, hb


def alone(g, idx, sub, max_len=256):
    import torch
    b = g.Batch(sub["codes"], sub["read_off"], sub["read_len"], sub["read_e"], sub["e_den"],
                sub["cand_off"], sub["cand_bin"], max_len=max_len)
    n = b.n_pairs
    c, bits = g.alloc_outputs(n)
    ws = g.alloc_workspace(idx, n)
    g.grim_filter_batch(idx, b, c, bits, ws)
    rc, _ = g.grim_filter_status(ws)
    torch.cuda.synchronize()
    return rc, c.cpu().numpy()[:n].copy(), bits.cpu().numpy().view(np.uint32)[:(n + 31) // 32].copy()


def make_requests(g, w, n_req, seed, max_reads=1500):
    rng = np.random.default_rng(seed)
    n_reads = w["read_len"].size
    out = []
    for _ in range(n_req):
        size = int(min(n_reads, max(1, round(np.exp(rng.uniform(0, np.log(max_reads)))))))
        r0 = int(rng.integers(0, n_reads - size + 1))
        out.append(cut(g, w, r0, r0 + size))
    return out


def test_alone_vs_mix(setup):
    g, w, idx = setup
    reqs = make_requests(g, w, 80, 11)
    say("requests", len(reqs), "pairs", sum(hb.n_pairs for _, hb in reqs))
    solo = [alone(g, idx, sub) for sub, _ in reqs]
    # every solo result against the oracle
    for i, ((sub, _), (rc, c, b)) in enumerate(zip(reqs, solo)):
        assert rc == 0 and oracle_check(w, sub, c, b), f"request {i} differs from the oracle"
    srv = g.Server(idx, hbm_budget_bytes=256 << 20, max_inflight=16, n_streams=3,
                   max_tick_pairs=1 << 20, max_len=256)
    tickets = [None] * len(reqs)
    rng = np.random.default_rng(3)

    def producer(lo, hi):
        for i in range(lo, hi):
            time.sleep(float(rng.exponential(0.0005)))
            tickets[i] = srv.submit(reqs[i][1])

    th = [threading.Thread(target=producer, args=(a, a + 40)) for a in (0, 40)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i, t in enumerate(tickets):
        rc, c, b, st = srv.wait(t)
        assert rc == 0, (i, rc)
        assert np.array_equal(c, solo[i][1]), f"request {i}: counts differ in the mix"
        assert np.array_equal(b, solo[i][2]), f"request {i}: pass bits differ in the mix"
    s = srv.stats(reset=True)
    say("serve stats", s)
    assert s["completed"] == len(reqs)
    assert s["peak_device_bytes"] <= 256 << 20
    # the same requests submitted at once: they queue, so ticks fuse several
    tickets = [srv.submit(hb) for _, hb in reqs]
    for i, t in enumerate(tickets):
        rc, c, b, st = srv.wait(t)
        assert rc == 0, (i, rc)
        assert np.array_equal(c, solo[i][1]), f"request {i}: counts differ in the burst"
        assert np.array_equal(b, solo[i][2]), f"request {i}: pass bits differ in the burst"
    s = srv.stats()
    say("burst stats", s)
    assert s["completed"] == len(reqs)
    assert s["ticks"] < len(reqs), "no request was fused with another"
    assert s["peak_device_bytes"] <= 256 << 20
    srv.destroy()


def test_budget_admission_and_oversized_request(setup):
    g, w, idx = setup
    reqs = make_requests(g, w, 30, 12, max_reads=400)
    biggest = max(hb.n_pairs for _, hb in reqs)
    budget = 4 << 20  # a few MB: forces waiting for memory
    srv = g.Server(idx, hbm_budget_bytes=budget, max_inflight=8, n_streams=2,
                   max_tick_pairs=1 << 20, max_len=256)
    tickets = []
    for sub, hb in reqs:
        try:
            tickets.append((sub, srv.submit(hb)))
        except g.GrimError as e:
            assert e.code == g.GRIM_E_BUDGET
    assert tickets, "every request was larger than the budget"
    for sub, t in tickets:
        rc, c, b, st = srv.wait(t)
        assert rc == 0
        rc2, c2, b2 = alone(g, idx, sub)
        assert np.array_equal(c, c2) and np.array_equal(b, b2)
    s = srv.stats()
    assert s["peak_device_bytes"] <= budget
    # a request that cannot fit the budget at all is refused at submit
    big_sub, big_hb = cut(g, w, 0, w["read_len"].size)
    with pytest.raises(g.GrimError) as e:
        srv.submit(big_hb)
    assert e.value.code == g.GRIM_E_BUDGET
    srv.destroy()
    say("budget ok, biggest request", biggest)


def test_invalid_bin_fails_only_its_request(setup):
    g, w, idx = setup
    reqs = make_requests(g, w, 6, 13, max_reads=200)
    bad_sub, _ = reqs[2]
    bad_sub["cand_bin"][3] = idx.n_bins + 7
    reqs[2] = (bad_sub, g.HostBatch(bad_sub["codes"], bad_sub["read_off"], bad_sub["read_len"],
                                    bad_sub["read_e"], bad_sub["e_den"], bad_sub["cand_off"],
                                    bad_sub["cand_bin"], max_len=256))
    srv = g.Server(idx, hbm_budget_bytes=64 << 20, n_streams=2, max_len=256)
    ts = [srv.submit(hb) for _, hb in reqs]
    for i, t in enumerate(ts):
        rc, c, b, st = srv.wait(t)
        rc2, c2, b2 = alone(g, idx, reqs[i][0])
        assert np.array_equal(c, c2) and np.array_equal(b, b2)
        if i == 2:
            assert rc == g.GRIM_E_BIN_RANGE and c[3] == -1 and st.flags & g.GRIM_FLAG_BIN_RANGE
        else:
            assert rc == 0
    srv.destroy()


def test_cancel_and_invalid_submit(setup):
    g, w, idx = setup
    reqs = make_requests(g, w, 40, 14, max_reads=800)
    srv = g.Server(idx, hbm_budget_bytes=8 << 20, max_inflight=2, n_streams=1, max_len=256)
    ts = [srv.submit(hb) for _, hb in reqs]
    for t in ts[20:]:
        srv.cancel(t)
    n_cancel = 0
    for i, t in enumerate(ts):
        rc, c, b, st = srv.wait(t)
        if rc == g.GRIM_E_CANCELLED:
            n_cancel += 1
            assert i >= 20
        else:
            assert rc == 0
            rc2, c2, b2 = alone(g, idx, reqs[i][0])
            assert np.array_equal(c, c2)
    assert n_cancel >= 1
    # a read longer than the request's max_len is refused at submit
    sub, _ = reqs[0]
    hb = g.HostBatch(sub["codes"], sub["read_off"], sub["read_len"], sub["read_e"], sub["e_den"],
                     sub["cand_off"], sub["cand_bin"], max_len=50)
    with pytest.raises(g.GrimError) as e:
        srv.submit(hb)
    assert e.value.code == g.GRIM_E_READ
    # unknown ticket
    assert srv.poll(10 ** 9)[0] == g.GRIM_E_INVALID
    srv.destroy()


def test_mixed_tolerance_denominators(setup):
    g, w, idx = setup
    reqs = make_requests(g, w, 10, 15, max_reads=100)
    # rewrite half of the requests with e expressed per 1000 instead of per 10000
    conv = []
    for i, (sub, hb) in enumerate(reqs):
        if i % 2:
            sub = dict(sub)
            sub["read_e"] = (sub["read_e"] // 10).astype(np.uint32)
            sub["e_den"] = 1000
            hb = g.HostBatch(sub["codes"], sub["read_off"], sub["read_len"], sub["read_e"], 1000,
                             sub["cand_off"], sub["cand_bin"], max_len=256)
        conv.append((sub, hb))
    srv = g.Server(idx, hbm_budget_bytes=64 << 20, n_streams=2, max_len=256)
    ts = [srv.submit(hb) for _, hb in conv]
    for (sub, _), t in zip(conv, ts):
        rc, c, b, st = srv.wait(t)
        rc2, c2, b2 = alone(g, idx, sub)
        assert rc == 0 and np.array_equal(c, c2) and np.array_equal(b, b2)
    srv.destroy()


def test_inplace_submission_matches_alone(setup):
    """Zero-copy submission from pinned buffers: same results as solo runs,
    mixed with copying submissions in the same server."""
    g, w, idx = setup
    reqs = make_requests(g, w, 30, 16, max_reads=800)
    pinned = []
    for sub, _ in reqs:
        pinned.append(g.HostBatch(sub["codes"], sub["read_off"], sub["read_len"], sub["read_e"],
                                  sub["e_den"], sub["cand_off"], sub["cand_bin"], max_len=256,
                                  pinned=True))
    srv = g.Server(idx, hbm_budget_bytes=128 << 20, max_inflight=16, n_streams=3, max_len=256)
    tickets = []
    for i, ((sub, hb), phb) in enumerate(zip(reqs, pinned)):
        tickets.append(srv.submit_inplace(phb) if i % 3 else srv.submit(hb))
    for i, t in enumerate(tickets):
        rc, c, b, st = srv.wait(t)
        assert rc == 0
        rc2, c2, b2 = alone(g, idx, reqs[i][0])
        assert np.array_equal(c, c2), i
        assert np.array_equal(b, b2), i
        if i % 3:
            assert np.array_equal(pinned[i].out_counts[:c2.size], c2)
    srv.destroy()


def test_pageable_inplace_submission(setup):
    """In-place requests in pageable memory (staged by the runtime), alone and
    in ticks mixed with pinned ones, results downloaded by the copy engine or
    (pinned buffers only) stored by a kernel: every request equals its solo run
    and its counts land in the caller's buffer."""
    g, w, idx = setup
    reqs = make_requests(g, w, 18, 19, max_reads=800)
    solo = [alone(g, idx, sub) for sub, _ in reqs]
    pageable = [g.HostBatch(sub["codes"], sub["read_off"], sub["read_len"], sub["read_e"],
                            sub["e_den"], sub["cand_off"], sub["cand_bin"], max_len=256)
                for sub, _ in reqs]
    pinned = [g.HostBatch(sub["codes"], sub["read_off"], sub["read_len"], sub["read_e"],
                          sub["e_den"], sub["cand_off"], sub["cand_bin"], max_len=256, pinned=True)
              for sub, _ in reqs]
    mixed = [pageable[i] if i % 2 else pinned[i] for i in range(len(reqs))]
    for name, batches, downloads in (("pageable", pageable, "auto"), ("pinned", pinned, "auto"),
                                     ("mixed", mixed, "auto"), ("mixed, stored", mixed, "store")):
        srv = g.Server(idx, hbm_budget_bytes=64 << 20, max_inflight=8, n_streams=2, max_len=256,
                       downloads=downloads)
        ts = [srv.submit_inplace(hb) for hb in batches]
        for i, t in enumerate(ts):
            rc, c, b, st = srv.wait(t)
            assert rc == solo[i][0] == 0, (name, i, rc)
            assert np.array_equal(c, solo[i][1]), f"{name}: request {i} counts"
            assert np.array_equal(b, solo[i][2]), f"{name}: request {i} pass bits"
            assert np.array_equal(batches[i].out_counts[:c.size], solo[i][1])
        s = srv.stats()
        say(name, s)
        assert s["completed"] == len(reqs)
        srv.destroy()


def test_pass_bits_only(setup):
    """Servers that return pass bits alone: every request's bits equal its solo
    run, copied and in place, whole and in parts; counts are not returned and
    in-place count buffers are left as they were; a request with an
    out-of-range bin id still fails alone (its tick fetches its counts)."""
    g, w, idx = setup
    reqs = make_requests(g, w, 16, 23, max_reads=1200)
    bad_sub, _ = reqs[3]
    bad_sub["cand_bin"][len(bad_sub["cand_bin"]) // 2] = idx.n_bins + 7
    reqs[3] = (bad_sub, g.HostBatch(bad_sub["codes"], bad_sub["read_off"], bad_sub["read_len"],
                                    bad_sub["read_e"], bad_sub["e_den"], bad_sub["cand_off"],
                                    bad_sub["cand_bin"], max_len=256))
    solo = [alone(g, idx, sub) for sub, _ in reqs]
    assert solo[3][0] == g.GRIM_E_BIN_RANGE
    for tick_pairs in (0, 3000):
        pinned = [g.HostBatch(sub["codes"], sub["read_off"], sub["read_len"], sub["read_e"],
                              sub["e_den"], sub["cand_off"], sub["cand_bin"], max_len=256,
                              pinned=True) for sub, _ in reqs]
        for hb in pinned:
            hb.out_counts[:] = -5
        srv = g.Server(idx, hbm_budget_bytes=64 << 20, max_inflight=64, n_streams=3,
                       max_tick_pairs=tick_pairs, max_len=256, pass_bits_only=True)
        ts = [srv.submit_inplace(pinned[i]) if i % 2 else srv.submit(hb)
              for i, (_, hb) in enumerate(reqs)]
        for i, t in enumerate(ts):
            rc, c, b, st = srv.wait(t)
            assert c is None
            assert rc == solo[i][0], (tick_pairs, i, rc)
            assert np.array_equal(b, solo[i][2]), f"{tick_pairs}: request {i} pass bits"
            if i % 2:
                assert np.all(pinned[i].out_counts == -5)
        s = srv.stats()
        say("bits only", tick_pairs, s)
        assert s["completed"] == len(reqs)
        srv.destroy()


def test_requests_split_into_parts(setup):
    """Requests with more pairs than max_tick_pairs run in parts of whole reads
    (at 100 pairs down to single reads with more candidates than the limit):
    every request equals its solo run, in place and copied, and an invalid bin
    id fails only its own request."""
    g, w, idx = setup
    reqs = make_requests(g, w, 24, 17, max_reads=1500)
    bad_sub, _ = reqs[5]
    bad_sub["cand_bin"][len(bad_sub["cand_bin"]) - 2] = idx.n_bins + 1
    reqs[5] = (bad_sub, g.HostBatch(bad_sub["codes"], bad_sub["read_off"], bad_sub["read_len"],
                                    bad_sub["read_e"], bad_sub["e_den"], bad_sub["cand_off"],
                                    bad_sub["cand_bin"], max_len=256))
    solo = [alone(g, idx, sub) for sub, _ in reqs]
    pinned = [g.HostBatch(sub["codes"], sub["read_off"], sub["read_len"], sub["read_e"],
                          sub["e_den"], sub["cand_off"], sub["cand_bin"], max_len=256, pinned=True)
              for sub, _ in reqs]
    for tick_pairs in (3000, 100):
        srv = g.Server(idx, hbm_budget_bytes=64 << 20, max_inflight=8, n_streams=3,
                       max_tick_pairs=tick_pairs, max_len=256)
        ts = [srv.submit_inplace(pinned[i]) if i % 2 else srv.submit(hb)
              for i, (_, hb) in enumerate(reqs)]
        for i, t in enumerate(ts):
            rc, c, b, st = srv.wait(t)
            assert rc == solo[i][0], (tick_pairs, i, rc)
            assert np.array_equal(c, solo[i][1]), f"{tick_pairs}: request {i} counts"
            assert np.array_equal(b, solo[i][2]), f"{tick_pairs}: request {i} pass bits"
        s = srv.stats()
        say("split", tick_pairs, s)
        assert s["ticks"] > len(reqs), "no request was split"
        assert s["completed"] == len(reqs)
        srv.destroy()


def test_cancel_request_running_in_parts(setup):
    """A request cancelled while its parts run: the rest never runs, the ticket
    reports GRIM_E_CANCELLED, and the server goes on serving."""
    g, w, idx = setup
    sub, hb = cut(g, w, 0, 6000)
    say("pairs", hb.n_pairs)
    srv = g.Server(idx, hbm_budget_bytes=64 << 20, n_streams=1, max_tick_pairs=2000, max_len=256)
    t = srv.submit(hb)
    time.sleep(0.002)
    srv.cancel(t)
    rc, c, b, st = srv.wait(t)
    assert rc == g.GRIM_E_CANCELLED
    sub2, hb2 = cut(g, w, 100, 400)
    rc2, c2, b2, _ = srv.wait(srv.submit(hb2))
    solo = alone(g, idx, sub2)
    assert rc2 == 0 and np.array_equal(c2, solo[1]) and np.array_equal(b2, solo[2])
    s = srv.stats()
    assert s["cancelled"] == 1 and s["completed"] == 1
    srv.destroy()


@pytest.mark.parametrize("ticks_per_stream,bits_only,downloads",
                         [(1, False, "auto"), (1, False, "store"), (2, False, "engine"),
                          (2, False, "store"), (3, True, "auto"), (0, True, "store")])
def test_scheduling_policies_match_oracle(setup, ticks_per_stream, bits_only, downloads):
    """One request mix through every scheduling policy: one to three ticks per
    stream, with upload turns (counts and pass bits) and without (pass bits
    only), results downloaded by the copy engine or stored by a kernel, ticks
    small enough that requests run in parts; every request's results against
    the oracle."""
    g, w, idx = setup
    reqs = make_requests(g, w, 40, 17 + ticks_per_stream, max_reads=3000)
    srv = g.Server(idx, hbm_budget_bytes=128 << 20, max_inflight=32, n_streams=3,
                   max_tick_pairs=80_000, max_len=256, pass_bits_only=bits_only,
                   ticks_per_stream=ticks_per_stream, downloads=downloads)
    try:
        tickets = [srv.submit(hb) for _, hb in reqs]
        for i, ((sub, hb), t) in enumerate(zip(reqs, tickets)):
            rc, c, b, st = srv.wait(t)
            assert rc == 0, (i, rc)
            if bits_only:
                passed = oracle.filter_batch(w["oidx"], w["q"], sub["codes"], sub["read_off"],
                                             sub["read_len"], sub["read_e"], sub["e_den"],
                                             sub["cand_off"], sub["cand_bin"],
                                             n_threads=gs.default_threads())[1]
                assert c is None
                assert np.array_equal(b, oracle.pack_bitmask(passed)), i
            else:
                assert oracle_check(w, sub, c, b), f"request {i} differs from the oracle"
        stats = srv.stats()
        assert stats["completed"] == len(reqs) and stats["failed"] == 0
        assert stats["ticks"] > len(reqs) // 2
    finally:
        srv.destroy()
