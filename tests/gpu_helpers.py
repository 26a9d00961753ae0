"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded workload."""
import numpy as np

import grim_synth as gs
import oracle


def lib():
    import paper_1711_01177_amd as g
    return g


def oracle_run(w, n_threads=8, index=None):
    """Oracle counts, packed pass bits and out-of-range count for a workload."""
    if index is None:
        index = oracle.build_index(w["ref"], w["B"], w["O"], w["q"], n_threads=n_threads)
    c, p, bad = oracle.filter_batch(index, w["q"], w["codes"], w["read_off"], w["read_len"],
                                    w["read_e"], w["e_den"], w["cand_off"], w["cand_bin"],
                                    n_threads=n_threads)
    return c, oracle.pack_bitmask(p), bad, index


def gpu_index(w):
    g = lib()
    return g.grim_build_bins(w["ref"], w["q"], w["B"], w["O"])


def gpu_run(index, w, mode="batched", tune=None, max_len=None, batch=None):
    """Run the filter on the GPU; returns (counts, bits, rc, flags) as numpy."""
    import torch
    g = lib()
    if batch is None:
        batch = g.Batch.from_workload(w, max_len=max_len)
    n = batch.n_pairs
    counts, bits = g.alloc_outputs(n)
    counts.fill_(-7)
    bits.fill_(-1)
    ws = g.alloc_workspace(index, n, tune)
    if mode == "batched":
        g.grim_filter_batch(index, batch, counts, bits, ws, tune)
    elif mode == "plain":
        g.grim_filter_plain(index, batch, counts, bits, ws)
    else:
        raise ValueError(mode)
    rc, flags = g.grim_filter_status(ws)
    torch.cuda.synchronize()
    return (counts.cpu().numpy()[:n].copy(), bits.cpu().numpy().view(np.uint32)[:(n + 31) // 32].copy(),
            rc, flags)


def custom_workload(ref, q, B, O, reads, cands, e_nums, e_den=10000):
    """A workload dict from explicit reads (code arrays) and candidate lists."""
    lens = np.array([len(r) for r in reads], dtype=np.uint32)
    off = np.zeros(len(reads), dtype=np.uint64)
    if len(reads) > 1:
        off[1:] = np.cumsum(lens[:-1].astype(np.uint64))
    codes = np.concatenate([np.asarray(r, dtype=np.uint8) for r in reads]) if len(reads) else \
        np.zeros(0, np.uint8)
    coff = gs.offsets_from_counts([len(c) for c in cands])
    cb = np.array([b for c in cands for b in c], dtype=np.uint32)
    return dict(ref=ref, q=q, B=B, O=O, codes=codes, read_off=off, read_len=lens,
                read_e=np.asarray(e_nums, dtype=np.uint32), e_den=e_den, cand_off=coff,
                cand_bin=cb)


def assert_same(gpu, orc, what=""):
    gc, gb, rc, flags = gpu
    oc, ob, bad = orc[0], orc[1], orc[2]
    assert gc.shape == oc.shape, what
    diff = np.nonzero(gc != oc)[0]
    assert diff.size == 0, f"{what}: {diff.size} count mismatches, first at {diff[:5]}: " \
                           f"gpu {gc[diff[:5]]} oracle {oc[diff[:5]]}"
    wd = np.nonzero(gb != ob)[0]
    assert wd.size == 0, f"{what}: {wd.size} pass-bit word mismatches, first at {wd[:5]}"
