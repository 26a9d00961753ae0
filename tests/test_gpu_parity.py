"""GPU parity: the HIP path (through the C ABI) against the oracle, element by
element, on seeded synthetic workloads.  Integer outputs: bit-exact."""
import sys

import numpy as np
import pytest

import grim_synth as gs
import oracle
from tests.gpu_helpers import assert_same, custom_workload, gpu_index, gpu_run, lib, oracle_run

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tiny():
    w = gs.make_workload("tiny")
    orc = oracle_run(w)
    return w, orc


def test_index_parity_tiny(tiny):
    w, orc = tiny
    say("index parity tiny")
    idx = gpu_index(w)
    assert idx.n_bins == orc[3].shape[0]
    assert np.array_equal(idx.to_host(), orc[3])


def build_every_kernel(g, ref, q, B, O, want):
    """Builds the index with the library's choice and with each build kernel
    forced; every kernel that takes the geometry must give the oracle's
    vectors.  Returns the kernels that took it."""
    took = []
    for build in (g.GRIM_BUILD_AUTO, g.GRIM_BUILD_PER_BIN, g.GRIM_BUILD_BLOCKS):
        try:
            idx = g.grim_build_bins(ref, q, B, O, build=build)
        except g.GrimError as e:
            assert build != g.GRIM_BUILD_AUTO and e.code == g.GRIM_E_UNSUPPORTED, (build, e)
            continue
        took.append(build)
        assert idx.n_bins == want.shape[0]
        assert np.array_equal(idx.to_host(), want), f"build kernel {build}"
    assert g.GRIM_BUILD_PER_BIN in took
    return took


@pytest.mark.parametrize("q,B,O", [(4, 97, 31), (5, 200, 105), (6, 1000, 263), (7, 333, 1)])
def test_index_parity_params(q, B, O):
    say("index parity", q, B, O)
    ref = gs.reference(77, 250_003 if q < 7 else 60_001, 0.3, 7, 300, 0.85, 0.98)
    g = lib()
    want = oracle.build_index(ref, B, O, q, n_threads=8)
    took = build_every_kernel(g, ref, q, B, O, want)
    assert g.GRIM_BUILD_BLOCKS in took


# Bin geometries at the edges of the chunked build: strides below one packed
# word, spans that end exactly on a block (R = 0, with B >= 16 and below),
# spans shorter than a token (all-zero vectors), a reference shorter than a
# token, many whole blocks per bin, two geometries whose whole blocks exceed
# the chunk's LDS (q=7 with m = 19, q=4 with m = 598), which take the
# one-wavefront-per-bin kernel, a 100 kb stride (three bins), and a stride
# beyond 2^31 (one bin; offsets inside a chunk would leave 32 bits, so the
# per-bin kernel again); the batched geometry, alone and with a genome that
# ends mid-way through a workgroup's blocks, and two more strides.  Where the
# block kernel takes a geometry, the per-bin kernel is run on it too.
@pytest.mark.parametrize("q,B,O,G", [(5, 10, 3, 3001), (4, 7, 100, 5003), (4, 3, 1, 1001),
                                     (5, 16, 0, 4099), (6, 1, 0, 301), (4, 200, 275, 3),
                                     (5, 1, 40, 777), (7, 5, 60, 2001), (5, 100, 4, 70_001),
                                     (7, 3, 60, 1999), (4, 1, 600, 2500), (5, 20, 4, 5000),
                                     (5, 20, 24, 5000), (6, 64, 5, 9000), (5, 16, 15, 4000),
                                     (5, 100_000, 50, 250_003), (4, 3_000_000_000, 0, 5000),
                                     (5, 200, 275, 100_003), (5, 160, 4, 50_000),
                                     (4, 240, 0, 30_011), (5, 200, 275, 16_619)])
def test_index_parity_edges(q, B, O, G):
    say("index parity edge", q, B, O, G)
    ref = np.random.default_rng(q * 1000 + B + G).integers(0, 4, G).astype(np.uint8)
    g = lib()
    want = oracle.build_index(ref, B, O, q, n_threads=8)
    took = build_every_kernel(g, ref, q, B, O, want)
    say("  kernels", took)


def test_index_parity_random_geometries():
    """Seeded random bin geometries (q 4-7, strides 1-3000, overlaps 0-2000,
    genomes 1-40 kb, with repeats): every build kernel that takes the geometry
    gives the oracle's vectors."""
    g = lib()
    rng = np.random.default_rng(20261203)
    kinds = {g.GRIM_BUILD_BLOCKS: 0, g.GRIM_BUILD_PER_BIN: 0}
    for case in range(24):
        q = int(rng.integers(4, 8))
        B = int(rng.choice([int(rng.integers(1, 17)), int(rng.integers(17, 400)),
                            int(rng.integers(400, 3001))]))
        O = int(rng.choice([0, int(rng.integers(0, 64)), int(rng.integers(64, 2001))]))
        G = int(rng.integers(1, 40_001))
        ref = rng.integers(0, 4, G).astype(np.uint8)
        if G > 200:  # a repeated stretch, so that bins share tokens
            a = int(rng.integers(0, G // 2))
            n = int(rng.integers(1, G // 4 + 1))
            ref[a + n:a + 2 * n] = ref[a:a + n][:max(0, min(n, G - a - n))]
        say("random geometry", case, q, B, O, G)
        want = oracle.build_index(ref, B, O, q, n_threads=8)
        for k in build_every_kernel(g, ref, q, B, O, want):
            kinds[k] = kinds.get(k, 0) + 1
    assert kinds[g.GRIM_BUILD_BLOCKS] > 0 and kinds[g.GRIM_BUILD_PER_BIN] == 24


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_filter_parity_tiny(tiny, mode):
    w, orc = tiny
    say("filter parity tiny", mode)
    idx = gpu_index(w)
    out = gpu_run(idx, w, mode)
    assert out[2] == 0 and out[3] == 0
    assert_same(out, orc, f"tiny/{mode}")


@pytest.mark.parametrize("name,scale", [("mid", 0.01), ("batched", 0.002), ("large", 0.002)])
@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_filter_parity_scaled(name, scale, mode):
    say("filter parity", name, scale, mode)
    w = gs.make_workload(name, scale=scale)
    orc = oracle_run(w)
    idx = gpu_index(w)
    out = gpu_run(idx, w, mode)
    assert out[2] == 0
    assert_same(out, orc, f"{name}/{mode}")


def _variant_workload(q):
    B, O = (200, 275) if q == 5 else (1000, 263) if q == 6 else (150, 260)
    ref = gs.reference(31 + q, 400_000, 0.45, 40, 300, 0.85, 0.98)
    rd = gs.reads(32 + q, ref, 700, [100, 150, 250, 37], [500, 1000])
    k = gs.cand_counts_zipf(33 + q, 700, 1.2, 600)
    off = gs.offsets_from_counts(k)
    cb, _ = gs.cand_random(34 + q, off, rd["read_z"], B, (ref.size + B - 1) // B)
    return dict(ref=ref, q=q, B=B, O=O, e_den=gs.E_DEN, cand_off=off, cand_bin=cb, **rd)


@pytest.mark.parametrize("q", [4, 5, 6, 7])
def test_every_launch_shape_identical(q):
    """Every (lanes per candidate, unroll, tile, occupancy) computes the same bits."""
    g = lib()
    say("variants q", q)
    w = _variant_workload(q)
    orc = oracle_run(w)
    idx = gpu_index(w)
    for cand in g.grim_tuning_candidates(q):
        G, U = cand.lanes_per_cand, cand.unroll
        for tile in (64, 512, 4096):
            for wg in (1, 8):
                t = g.tuning(G, U, tile, wg)
                out = gpu_run(idx, w, "batched", tune=t)
                assert out[2] == 0
                assert_same(out, orc, f"q{q} G{G} U{U} tile{tile} wg{wg}")


def test_edge_cases():
    g = lib()
    say("edge cases")
    rng = np.random.default_rng(5)
    ref = gs.reference(9, 1_000_000)
    q, B, O = 5, 200, 2100
    nb = (ref.size + B - 1) // B
    reads, cands = [], []

    def add(read, cand):
        reads.append(np.asarray(read, dtype=np.uint8))
        cands.append(list(cand))

    add(ref[1000:1100], [])                                   # no candidates
    add(ref[-100:], [nb - 1])                                 # last bin, 1 candidate
    add(ref[5000:5150], rng.integers(0, nb, 4096))            # 4096 candidates
    add(ref[7:10], rng.integers(0, nb, 5))                    # L < q
    add([], [0, 1, 2])                                        # L = 0
    add(ref[333:370], rng.integers(0, nb, 70))                # L = 37, unaligned
    add(ref[9000:9250], [45] * 100)                           # duplicate ids
    add(np.zeros(250, np.uint8), rng.integers(0, nb, 64))     # A^250: token multiplicity 246
    add(np.full(2000, 2, np.uint8), [0, 1, nb - 1])           # G^2000: multiplicity 1996
    add(ref[20_000:21_000], [100, 101, 99, nb - 2])           # 1000 bp
    add(ref[40_000:42_000], [200, 201, 202, 203, 9])          # 2000 bp
    for i in range(13):                                       # short tail reads
        add(ref[50_000 + i:50_000 + i + 17 + i], rng.integers(0, nb, i))
    e = [500] * len(reads)
    e[5] = 1000
    w = custom_workload(ref, q, B, O, reads, cands, e)
    assert int(w["cand_off"][-1]) % 64 != 0
    orc = oracle_run(w)
    idx = gpu_index(w)
    for mode in ("batched", "plain"):
        out = gpu_run(idx, w, mode, max_len=2000)
        assert out[2] == 0, mode
        assert_same(out, orc, f"edge/{mode}")
    # single read, single candidate
    w1 = custom_workload(ref, q, B, O, [ref[100:200]], [[0]], [500])
    for mode in ("batched", "plain"):
        out = gpu_run(idx, w1, mode)
        assert_same(out, oracle_run(w1, index=orc[3]), f"single/{mode}")


def test_empty_batch():
    g = lib()
    ref = gs.reference(9, 100_000)
    w = custom_workload(ref, 5, 200, 105, [], [], [])
    idx = gpu_index(w)
    batch = g.Batch(np.zeros(0, np.uint8), np.zeros(0, np.uint64), np.zeros(0, np.uint32),
                    np.zeros(0, np.uint32), 10000, np.zeros(1, np.uint64), np.zeros(0, np.uint32))
    for mode in ("batched", "plain"):
        c, b, rc, flags = gpu_run(idx, w, mode, batch=batch)
        assert c.size == 0 and rc == 0 and flags == 0


def test_out_of_range_bins_and_invalid_reads():
    g = lib()
    say("error flags")
    ref = gs.reference(12, 300_000)
    q, B, O = 5, 200, 105
    nb = (ref.size + B - 1) // B
    reads = [ref[1000:1100], ref[2000:2100], ref[3000:3100]]
    cands = [[5, nb, 7, nb + 1000], [1, 2, 3], [4, 0xFFFFFFFF]]
    w = custom_workload(ref, q, B, O, reads, cands, [500] * 3)
    oc, ob, bad, oidx = oracle_run(w)
    assert bad == 3
    idx = gpu_index(w)
    for mode in ("batched", "plain"):
        out = gpu_run(idx, w, mode)
        assert out[2] == g.GRIM_E_BIN_RANGE and out[3] & g.GRIM_FLAG_BIN_RANGE, mode
        assert_same(out, (oc, ob, bad), f"oob/{mode}")
    # a read longer than max_len: its pairs report -1 and the call GRIM_E_READ
    reads2 = [ref[1000:1100], ref[2000:2300], ref[3000:3100]]
    w2 = custom_workload(ref, q, B, O, reads2, [[1, 2], [3, 4, 5], [6]], [500] * 3)
    oc2, ob2, _, _ = oracle_run(w2, index=oidx)
    for mode in ("batched", "plain"):
        c, b, rc, flags = gpu_run(idx, w2, mode, max_len=250)
        assert rc == g.GRIM_E_READ and flags & g.GRIM_FLAG_READ
        assert c.tolist()[2:5] == [-1, -1, -1]
        assert c.tolist()[:2] == oc2.tolist()[:2] and c[5] == oc2[5]
        assert (b[0] >> 2) & 7 == 0


def test_graph_replays_and_determinism():
    import torch
    g = lib()
    say("graph replays")
    w = gs.make_workload("batched", scale=0.001)
    orc = oracle_run(w)
    idx = gpu_index(w)
    batch = g.Batch.from_workload(w)
    counts, bits = g.alloc_outputs(batch.n_pairs)
    ws = g.alloc_workspace(idx, batch.n_pairs)
    graph = g.grim_graph_create(idx, batch, counts, bits, ws)
    n = batch.n_pairs
    for rep in range(4):
        counts.fill_(-9)
        bits.fill_(0x5555)
        torch.cuda.synchronize()
        graph.launch()
        rc, flags = g.grim_filter_status(ws)
        assert rc == 0
        out = (counts.cpu().numpy()[:n], bits.cpu().numpy().view(np.uint32)[:(n + 31) // 32], rc, flags)
        assert_same(out, orc, f"graph replay {rep}")
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
    graph.destroy()
    a = gpu_run(idx, w)
    b = gpu_run(idx, w)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_tune_picks_a_valid_shape():
    g = lib()
    w = gs.make_workload("batched", scale=0.001)
    idx = gpu_index(w)
    batch = g.Batch.from_workload(w)
    counts, bits = g.alloc_outputs(batch.n_pairs)
    ws = g.alloc_workspace(idx, batch.n_pairs)
    t = g.grim_tune(idx, batch, counts, bits, ws)
    assert t.tile_pairs % 64 == 0 and t.lanes_per_cand in (2, 4, 8)
    out = gpu_run(idx, w)  # tune=None now uses the cached choice
    assert_same(out, oracle_run(w), "tuned")


def test_index_save_load(tmp_path):
    g = lib()
    ref = gs.reference(3, 123_457)
    idx = g.grim_build_bins(ref, 5, 200, 105)
    p = tmp_path / "i.grim"
    idx.save(p)
    idx2 = g.grim_index_load(p)
    assert np.array_equal(idx.to_host(), idx2.to_host())
    raw = bytearray(p.read_bytes())
    raw[100] ^= 1
    p.write_bytes(bytes(raw))
    with pytest.raises(g.GrimError) as e:
        g.grim_index_load(p)
    assert e.value.code == g.GRIM_E_IO
