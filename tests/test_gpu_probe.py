"""Memory-ceiling probes: the gather probe reads exactly the bin vectors it is
given (out = popcount of each vector, -1 for an id past the last bin), for
every token length; the streaming probe runs over the whole index."""
import numpy as np
import pytest

import grim_synth as gs
from tests.gpu_helpers import lib

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("q,B,O", [(4, 50, 20), (5, 200, 105), (6, 400, 100), (7, 1000, 50)])
def test_probe_gather_reads_the_right_vectors(q, B, O):
    import torch
    g = lib()
    ref = gs.reference(90 + q, 300_000)
    idx = g.grim_build_bins(ref, q, B, O)
    nb = idx.n_bins
    rng = np.random.default_rng(q)
    n = 100_003                                   # not a multiple of any step
    ids = rng.integers(0, nb, size=n).astype(np.uint32)
    ids[::97] = nb + 5                            # out of range
    ids[-1] = nb - 1
    t_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    out = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    g.grim_probe_gather(idx, t_ids, out)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    g.grim_probe_stream(idx, sink)
    torch.cuda.synchronize()
    vec = idx.to_host()
    pops = np.unpackbits(vec, axis=1).sum(axis=1).astype(np.int64)
    got = out.cpu().numpy().astype(np.int64)
    ok = ids < nb
    assert np.array_equal(got[ok], pops[ids[ok]])
    assert np.all(got[~ok] == -1)
