"""The no-allocation entry point (grim_filter_batch_noalloc, scratch in a
file-scope device array) against the workspace entry point grim_filter_batch
and the oracle: two calls in a row on the same GPU, the second with a smaller
batch, then a batch too large for the scratch (refused on the host)."""
import ctypes

import numpy as np
import pytest

import grim_synth as gs
from tests.gpu_helpers import lib, oracle_run

pytestmark = pytest.mark.gpu


def run_both(g, idx, w, tune=None):
    import torch
    batch = g.Batch.from_workload(w)
    n = batch.n_pairs
    c1, b1 = g.alloc_outputs(n)
    c2, b2 = g.alloc_outputs(n)
    c1.fill_(-7)
    c2.fill_(-9)
    b1.fill_(-1)
    b2.fill_(0x5a5a5a5a)
    ws = g.alloc_workspace(idx, n, tune)
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    g.grim_filter_batch(idx, batch, c1, b1, ws, tune)
    rc1, f1 = g.grim_filter_status(ws)
    g.grim_filter_batch_noalloc(idx, batch, c2, b2, status, tune)
    rc2, f2 = g.grim_filter_status(status)
    torch.cuda.synchronize()
    return (n, rc1, f1, rc2, f2, c1[:n].cpu().numpy(), b1[:(n + 31) // 32].cpu().numpy(),
            c2[:n].cpu().numpy(), b2[:(n + 31) // 32].cpu().numpy())


@pytest.mark.parametrize("tune_args", [None, (4, 4, 64, 8)])
def test_noalloc_matches_workspace_entry_point(tune_args):
    g = lib()
    tune = g.tuning(*tune_args) if tune_args else None
    big = gs.make_workload("batched", scale=0.002)          # 6.2 Mbp, 8,000 mixed reads
    small = gs.make_workload("batched", scale=0.002, read_scale=0.0002, ref=big["ref"])
    idx = g.grim_build_bins(big["ref"], big["q"], big["B"], big["O"])
    oidx = None
    sizes = []
    for w in (big, small):
        n, rc1, f1, rc2, f2, c1, b1, c2, b2 = run_both(g, idx, w, tune)
        sizes.append(n)
        assert rc1 == rc2 == 0 and f1 == f2 == 0
        assert np.array_equal(c1, c2), "counts differ from grim_filter_batch"
        assert np.array_equal(b1, b2), "pass bits differ from grim_filter_batch"
        oc, ob, bad, oidx = oracle_run(w, index=oidx)
        assert bad == 0
        assert np.array_equal(c2, oc) and np.array_equal(b2.view(np.uint32), ob)
    assert sizes[1] < sizes[0]


def test_noalloc_flags_and_scratch_limit():
    import torch
    g = lib()
    w = gs.make_workload("tiny", scale=0.05)
    idx = g.grim_build_bins(w["ref"], w["q"], w["B"], w["O"])
    w["cand_bin"] = w["cand_bin"].copy()
    w["cand_bin"][5] = idx.n_bins + 3
    n, rc1, f1, rc2, f2, c1, b1, c2, b2 = run_both(g, idx, w)
    assert rc1 == rc2 == g.GRIM_E_BIN_RANGE and f1 == f2
    assert c2[5] == -1 and np.array_equal(c1, c2) and np.array_equal(b1, b2)
    # a batch whose tile table would not fit the scratch is refused before
    # anything is queued (the buffers are never read)
    batch = g.Batch.from_workload(w)
    tiles_max = (g.GRIM_NOALLOC_SCRATCH_BYTES - 256) // 4
    batch.c.n_pairs = (tiles_max + 1) * 64
    counts, bits = g.alloc_outputs(1)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(g.GrimError) as e:
        g.grim_filter_batch_noalloc(idx, batch, counts, bits, status, g.tuning(4, 4, 64, 4))
    assert e.value.code == g.GRIM_E_SCRATCH
    torch.cuda.synchronize()
