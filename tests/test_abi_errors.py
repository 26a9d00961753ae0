"""Argument checking of the C ABI and the index file format, on a machine
without a GPU: every call below must fail (or succeed) on its host-side checks,
before any device is touched."""
import ctypes
import os
import struct

import numpy as np
import pytest


@pytest.fixture(scope="module")
def g():
    import paper_1711_01177_amd as g
    return g


def test_null_handles_are_rejected(g):
    L = g._lib
    INV = g.GRIM_E_INVALID
    u64 = ctypes.c_uint64()
    u32 = ctypes.c_uint32()
    info = g.grim_index_info_t()
    b = g.grim_batch_t()
    assert L.grim_index_info(None, ctypes.byref(info)) == INV
    assert L.grim_index_copy_to_host(None, None, 0) == INV
    assert L.grim_index_save(None, b"/tmp/x") == INV
    assert L.grim_workspace_size(None, 10, None, ctypes.byref(u64)) == INV
    assert L.grim_filter_batch(None, ctypes.byref(b), None, None, None, 0, None, None) == INV
    assert L.grim_filter_plain(None, ctypes.byref(b), None, None, None, 0, None) == INV
    assert L.grim_filter_batch_noalloc(None, ctypes.byref(b), None, None, None, None, None) == INV
    assert g.grim_strerror(g.GRIM_E_SCRATCH).startswith("batch needs more than the static scratch")
    assert L.grim_filter_status(None, None, None) == INV
    assert L.grim_survivors_workspace_size(10, None) == INV
    assert L.grim_compact_survivors(None, None, 0, None, None, None, None, None, 0, None) == INV
    assert L.grim_index_attach_reference(None, None, 0, None) == INV
    assert L.grim_verify_survivors(None, ctypes.byref(b), None, None, 0, None, None, None) == INV
    assert L.grim_index_transpose(None, None) == INV
    assert L.grim_filter_windows(None, ctypes.byref(b), None, None, None, None, None, 0,
                                 None) == INV
    assert L.grim_graph_launch(None, None) == INV
    assert L.grim_serve_create(None, None, ctypes.byref(ctypes.c_void_p())) == INV
    assert L.grim_serve_submit(None, ctypes.byref(b), None) == INV
    assert L.grim_serve_poll(None, 1, None, None, None) == INV
    assert L.grim_serve_wait(None, 1, 0, None, None, None) == INV
    assert L.grim_serve_cancel(None, 1) == INV
    assert L.grim_serve_stats(None, None, 0) == INV
    assert L.grim_seed_index_build(None, 0, 12, None, None) == INV
    assert L.grim_seed_candidates(None, ctypes.byref(b), 200, 4096, None, None) == INV
    assert L.grim_candidates_info(None, None, None, None, None) == INV
    assert L.grim_candidates_copy_to_host(None, None, None) == INV
    assert L.grim_tuning_candidates(5, None, 4, ctypes.byref(u32)) == INV
    assert L.grim_default_tuning(5, None) == INV
    # freeing NULL handles is a no-op
    L.grim_index_free(None)
    L.grim_graph_destroy(None)
    L.grim_serve_destroy(None)
    L.grim_seed_index_free(None)
    L.grim_candidates_free(None)


def test_unsupported_parameters(g):
    L = g._lib
    words = g.grim_pack_bases(np.zeros(100, np.uint8))
    out = ctypes.c_void_p()
    for q in (3, 8):
        p = g.grim_params_t(q, 0, 200, 0)
        assert L.grim_build_bins(words.ctypes.data_as(ctypes.c_void_p), 100, ctypes.byref(p),
                                 ctypes.byref(out), None) == g.GRIM_E_UNSUPPORTED
    p = g.grim_params_t(5, 0, 0, 0)                   # stride 0
    assert L.grim_build_bins(words.ctypes.data_as(ctypes.c_void_p), 100, ctypes.byref(p),
                             ctypes.byref(out), None) == g.GRIM_E_INVALID
    p = g.grim_params_t(5, 3, 200, 0)                 # no such build kernel
    assert L.grim_build_bins(words.ctypes.data_as(ctypes.c_void_p), 100, ctypes.byref(p),
                             ctypes.byref(out), None) == g.GRIM_E_INVALID
    for k in (3, 16):
        assert L.grim_seed_index_build(words.ctypes.data_as(ctypes.c_void_p), 100, k,
                                       ctypes.byref(out), None) == g.GRIM_E_UNSUPPORTED
    t = g.grim_tuning_t()
    for q in (3, 8):
        assert L.grim_default_tuning(q, ctypes.byref(t)) == g.GRIM_E_UNSUPPORTED
    # host-only answers
    n = ctypes.c_uint32()
    assert L.grim_tuning_candidates(5, None, 0, ctypes.byref(n)) == g.GRIM_OK and n.value >= 4
    cands = (g.grim_tuning_t * n.value)()
    assert L.grim_tuning_candidates(5, cands, n.value, ctypes.byref(n)) == g.GRIM_OK
    assert all(c.tile_pairs % 64 == 0 and c.lanes_per_cand >= 1 for c in cands)
    nb = ctypes.c_uint64()
    assert L.grim_survivors_workspace_size(10 ** 6, ctypes.byref(nb)) == g.GRIM_OK and nb.value > 0


def _index_file(path, q=4, B=10, O=3, G=95, data=None, checksum=None, magic=b"GRIMIDX1",
                version=1, n_bins=None, truncate=0):
    n_bins = (G + B - 1) // B if n_bins is None else n_bins
    vb = (1 << (2 * q)) // 8
    data = bytes(range(256)) * ((n_bins * vb) // 256 + 1) if data is None else data
    data = data[:n_bins * vb]
    if checksum is None:
        h = 1469598103934665603
        for x in data:
            h = ((h ^ x) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
        checksum = h
    hdr = magic + struct.pack("<IIQQQQQQ", version, q, B, O, G, n_bins, checksum, 0)
    assert len(hdr) == 64
    blob = hdr + data
    with open(path, "wb") as f:
        f.write(blob[:len(blob) - truncate])


def test_index_file_validation(g, tmp_path):
    """The 64-byte header and the FNV-1a checksum reject damaged files before
    any device memory is touched."""
    L = g._lib
    out = ctypes.c_void_p()
    def load(p):
        return L.grim_index_load(str(p).encode(), ctypes.byref(out), None)
    assert load(tmp_path / "missing.idx") == g.GRIM_E_IO
    cases = {
        "magic": dict(magic=b"GRIMIDX2"),
        "version": dict(version=2),
        "q": dict(q=9),
        "n_bins": dict(n_bins=7),
        "checksum": dict(checksum=12345),
        "truncated": dict(truncate=5),
        "header_only": dict(truncate=320),            # 10 bins x 32 bytes of data cut
    }
    for name, kw in cases.items():
        p = tmp_path / f"{name}.idx"
        _index_file(p, **kw)
        assert load(p) == g.GRIM_E_IO, name
    assert L.grim_index_load(None, ctypes.byref(out), None) == g.GRIM_E_INVALID
