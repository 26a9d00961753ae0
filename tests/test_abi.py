"""The C-ABI library loads on a machine without a GPU, exports every entry
point include/grim.h declares, and its host-side helpers behave (CPU only;
no kernel is launched)."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grim.h")
LIB = os.path.join(ROOT, "paper_1711_01177_amd", "libgrim.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(grim_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("grim_build_bins", "grim_filter_batch", "grim_filter_plain", "grim_serve_create",
                 "grim_serve_submit", "grim_serve_poll", "grim_serve_wait", "grim_serve_cancel",
                 "grim_serve_stats", "grim_serve_destroy", "grim_strerror", "grim_max_edits"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libgrim.so not built"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(grim_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_binding_loads_and_covers_the_abi():
    import paper_1711_01177_amd as g
    assert set(declared()) == set(g.EXPORTED)
    assert g.grim_version() >= 10000
    assert g.grim_strerror(g.GRIM_E_BIN_RANGE) == "candidate bin id out of range"


def test_max_edits_and_threshold_match_oracle():
    import paper_1711_01177_amd as g
    rng = np.random.default_rng(1)
    for _ in range(2000):
        L = int(rng.integers(0, 3000))
        den = int(rng.choice([7, 100, 10000, 9973]))
        num = int(rng.integers(0, den + 1))
        E = g.grim_max_edits(L, num, den)
        assert E == oracle.max_edits(L, num, den)
        q = int(rng.integers(4, 8))
        assert g.grim_threshold(L, q, E) == oracle.threshold(L, q, E)
    with pytest.raises(g.GrimError):
        g.grim_max_edits(10, 1, 0)


def test_pack_bases_layout():
    import paper_1711_01177_amd as g
    # 17 bases: the first word holds 16, first base in the top two bits
    s = "ACGTACGTACGTACGTT"
    w = g.grim_pack_bases(np.frombuffer(s.encode(), dtype=np.uint8))
    assert w.size == g.grim_packed_words(17) == 3
    assert w[0] == 0x1B1B1B1B          # ACGT = 00 01 10 11
    assert w[1] == 0xC0000000          # T in the top bits
    assert w[2] == 0
    codes = np.array([0, 1, 2, 3] * 4 + [3], dtype=np.uint8)
    assert np.array_equal(g.grim_pack_bases(codes), w)
    rng = np.random.default_rng(2)
    big = rng.integers(0, 4, 1_000_003).astype(np.uint8)
    w1 = g.grim_pack_bases(big, n_threads=1)
    w8 = g.grim_pack_bases(big, n_threads=8)
    assert np.array_equal(w1, w8)
    # unpack in numpy and compare
    shifts = (30 - 2 * np.arange(16)).astype(np.uint32)
    un = ((w1[:-1, None] >> shifts[None, :]) & 3).astype(np.uint8).ravel()[:big.size]
    assert np.array_equal(un, big)
    with pytest.raises(g.GrimError) as e:
        g.grim_pack_bases(np.frombuffer(b"ACGN", dtype=np.uint8))
    assert e.value.code == g.GRIM_E_BASE


def test_window_order_argument_checks():
    """The window-order calls refuse a NULL index or output before touching a
    device (callable without a GPU)."""
    import ctypes
    import paper_1711_01177_amd as g
    n = ctypes.c_uint64(77)
    assert g._lib.grim_window_order_workspace_size(None, 10, ctypes.byref(n)) == g.GRIM_E_INVALID
    assert n.value == 77
    assert g._lib.grim_window_order(None, None, 10, None, None, 0, None) == g.GRIM_E_INVALID