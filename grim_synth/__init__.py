"""Seeded synthetic workloads for GRIM-Filter (shared by the oracle tests and
the HIP library's tests and benchmark).

The module produces references, reads and candidate lists as numpy arrays of
base codes (A=0 C=1 G=2 T=3); it holds none of the filter's arithmetic.  The
generators live in ``synth.c`` (keyed splitmix64 counters, multithreaded,
bit-identical for any thread count).

``make_workload(name, ...)`` builds the five workload families:

* ``tiny``    1 Mbp uniform reference, q=5, 200-bp bins, 10,000 x 100-bp reads
              (e=0.05), 64 candidates per read (true bin + 63 random bins)
* ``mid``     100 Mbp reference with 10 % planted 300-bp repeat families
              (85-98 % identity), 1M x 100-bp reads, candidates from exact
              12-mer seeds at read offsets 0, 12, ..., 84
* ``batched`` 3.1 Gbp reference with 45 % repeats, 4M reads mixing 100/150/250 bp,
              e in {0.05, 0.10}, Zipf(1.2) candidate counts capped at 4096
* ``large``   same reference, q=6, 1000-bp bins, 2M x 250-bp reads, e=0.05,
              candidate counts uniform on 1..2048
* ``serve``   the batched index and read/candidate recipe, cut into requests

``scale`` shrinks genome and read counts proportionally for tests.
"""
import ctypes
import hashlib
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libgrimsynth.so")
_DEFAULT_LIB = _LIB
_lib = None
_lock = threading.Lock()

E_DEN = 10000  # error tolerances are expressed in parts per 10,000

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


_CFLAGS = ["-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC"]


def _stamp(src, flags):
    """Hash of the source text and the compile flags a build used."""
    h = hashlib.sha1()
    with open(src, "rb") as f:
        h.update(f.read())
    h.update(" ".join(flags).encode())
    return h.hexdigest()


def build(out=None, extra_flags=()):
    """Compile synth.c into libgrimsynth.so (always recompiles).  A stamp file
    next to the library records the hash of the source and flags, so that a
    library older than its source is never loaded by default."""
    out = out or _LIB
    flags = _CFLAGS + list(extra_flags)
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *flags, _SRC, "-o", tmp, "-lpthread", "-lm"])
    os.replace(tmp, out)
    with open(out + ".stamp", "w") as f:
        f.write(_stamp(_SRC, flags))


def _current():
    try:
        with open(_LIB + ".stamp") as f:
            return os.path.exists(_LIB) and f.read().strip() == _stamp(_SRC, _CFLAGS)
    except OSError:
        return False


def use_library(path):
    """Bind the generators to another build of synth.c (e.g. a sanitizer build)."""
    global _LIB, _lib
    with _lock:
        _LIB = path
        _lib = None


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or (_LIB == _DEFAULT_LIB and not _current()):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, u32, dbl, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_int
        lib.synth_reference.argtypes = [u64, u64, dbl, u32, u32, dbl, dbl, i32, _u8p]
        lib.synth_read_meta.argtypes = [u64, u64, _u32p, u32, _u32p, u32, _u32p, _u32p]
        lib.synth_read_seqs.argtypes = [u64, _u8p, u64, u64, _u32p, _u32p, u32, _u64p, i32, _u8p,
                                        _u64p, _u32p, _u32p]
        lib.synth_cand_counts_zipf.argtypes = [u64, u64, dbl, u32, _u32p]
        lib.synth_cand_counts_uniform.argtypes = [u64, u64, u32, u32, _u32p]
        lib.synth_cand_fill_random.argtypes = [u64, u64, _u64p, _u64p, u64, u64, i32, _u32p, _u64p]
        lib.synth_kmer_count.argtypes = [_u8p, u64, u32, _u32p]
        lib.synth_kmer_fill.argtypes = [_u8p, u64, u32, _u64p, _u32p]
        lib.synth_seed_candidates.argtypes = [_u8p, u64, u32, _u64p, _u32p, _u8p, _u64p, _u32p, u64,
                                              u64, u32, i32, _u32p, _u64p, _u32p]
        for f in ("synth_reference", "synth_read_meta", "synth_read_seqs", "synth_cand_counts_zipf",
                  "synth_cand_counts_uniform", "synth_cand_fill_random", "synth_kmer_count",
                  "synth_kmer_fill", "synth_seed_candidates"):
            getattr(lib, f).restype = None
        _lib = lib
        return lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def default_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def reference(seed, G, repeat_frac=0.0, n_families=1, rep_len=300, id_lo=0.85, id_hi=0.98,
              n_threads=None):
    """Reference genome codes (uint8[G])."""
    out = np.empty(int(G), dtype=np.uint8)
    _load().synth_reference(seed, int(G), float(repeat_frac), int(n_families), int(rep_len),
                            float(id_lo), float(id_hi), n_threads or default_threads(), _p(out, _u8p))
    return out


def reads(seed, ref, n_reads, lengths, e_nums, e_den=E_DEN, n_threads=None):
    """Reads sampled from `ref` with planted edits.

    Returns dict(codes, read_off, read_len, read_e, read_z, read_span, read_edits)."""
    lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
    e_nums = np.ascontiguousarray(e_nums, dtype=np.uint32)
    lib = _load()
    rl = np.empty(n_reads, dtype=np.uint32)
    re = np.empty(n_reads, dtype=np.uint32)
    lib.synth_read_meta(seed, n_reads, _p(lengths, _u32p), lengths.size, _p(e_nums, _u32p),
                        e_nums.size, _p(rl, _u32p), _p(re, _u32p))
    off = np.zeros(n_reads + 1, dtype=np.uint64)
    np.cumsum(rl, out=off[1:])
    codes = np.empty(int(off[-1]), dtype=np.uint8)
    z = np.empty(n_reads, dtype=np.uint64)
    span = np.empty(n_reads, dtype=np.uint32)
    edits = np.empty(n_reads, dtype=np.uint32)
    lib.synth_read_seqs(seed, _p(ref, _u8p), ref.size, n_reads, _p(rl, _u32p), _p(re, _u32p), e_den,
                        _p(off, _u64p), n_threads or default_threads(), _p(codes, _u8p), _p(z, _u64p),
                        _p(span, _u32p), _p(edits, _u32p))
    return dict(codes=codes, read_off=off[:-1].copy(), read_len=rl, read_e=re, read_z=z,
                read_span=span, read_edits=edits)


def cand_counts_zipf(seed, n_reads, s=1.2, kmax=4096):
    k = np.empty(n_reads, dtype=np.uint32)
    _load().synth_cand_counts_zipf(seed, n_reads, float(s), int(kmax), _p(k, _u32p))
    return k


def cand_counts_uniform(seed, n_reads, lo, hi):
    k = np.empty(n_reads, dtype=np.uint32)
    _load().synth_cand_counts_uniform(seed, n_reads, int(lo), int(hi), _p(k, _u32p))
    return k


def offsets_from_counts(k):
    off = np.zeros(len(k) + 1, dtype=np.uint64)
    np.cumsum(np.asarray(k, dtype=np.uint64), out=off[1:])
    return off


def cand_random(seed, cand_off, read_z, B, n_bins, n_threads=None):
    """True bin (origin // B) plus uniform random bins.  Returns (cand_bin, true_pair)."""
    cand_off = np.ascontiguousarray(cand_off, dtype=np.uint64)
    read_z = np.ascontiguousarray(read_z, dtype=np.uint64)
    n_reads = cand_off.size - 1
    cb = np.empty(int(cand_off[-1]), dtype=np.uint32)
    tp = np.empty(n_reads, dtype=np.uint64)
    _load().synth_cand_fill_random(seed, n_reads, _p(cand_off, _u64p), _p(read_z, _u64p), int(B),
                                   int(n_bins), n_threads or default_threads(), _p(cb, _u32p),
                                   _p(tp, _u64p))
    return cb, tp


def kmer_index(ref, k=12):
    """CSR of the positions of every k-mer of `ref` (the mapper's seed table)."""
    lib = _load()
    cnt = np.zeros(4 ** k, dtype=np.uint32)
    lib.synth_kmer_count(_p(ref, _u8p), ref.size, k, _p(cnt, _u32p))
    off = np.zeros(4 ** k + 1, dtype=np.uint64)
    np.cumsum(cnt, out=off[1:])
    fill = off[:-1].copy()
    pos = np.empty(int(off[-1]), dtype=np.uint32)
    lib.synth_kmer_fill(_p(ref, _u8p), ref.size, k, _p(fill, _u64p), _p(pos, _u32p))
    return off, pos


def cand_seeded(ref, kidx, codes, read_off, read_len, B, k=12, cap=4096, n_threads=None):
    """Candidate bins from exact k-mer seeds at read offsets 0, k, 2k, ...

    Returns (cand_off, cand_bin)."""
    koff, kpos = kidx
    read_off = np.ascontiguousarray(read_off, dtype=np.uint64)
    read_len = np.ascontiguousarray(read_len, dtype=np.uint32)
    n = read_len.size
    lib = _load()
    nt = n_threads or default_threads()
    nout = np.empty(n, dtype=np.uint32)
    lib.synth_seed_candidates(_p(ref, _u8p), ref.size, k, _p(koff, _u64p), _p(kpos, _u32p),
                              _p(codes, _u8p), _p(read_off, _u64p), _p(read_len, _u32p), n, int(B),
                              int(cap), nt, _p(nout, _u32p), None, None)
    off = offsets_from_counts(nout)
    cb = np.empty(int(off[-1]), dtype=np.uint32)
    lib.synth_seed_candidates(_p(ref, _u8p), ref.size, k, _p(koff, _u64p), _p(kpos, _u32p),
                              _p(codes, _u8p), _p(read_off, _u64p), _p(read_len, _u32p), n, int(B),
                              int(cap), nt, None, _p(off, _u64p), _p(cb, _u32p))
    return off, cb


# Index parameters per workload.  O (extra overlap of each bin beyond its
# stride B) is chosen as L_max + E_max, where E_max = ceil(e_max * L_max) is the
# largest tolerated edit count: a true location then always lies wholly inside
# its bin, even with E_max deletions, so no true location can be rejected.
WORKLOADS = {
    # name: (G, repeat_frac, n_families, q, B, O, n_reads, lengths, e_nums, candidates)
    "tiny": dict(G=1_000_000, repeat_frac=0.0, n_families=1, q=5, B=200, O=105, n_reads=10_000,
                 lengths=[100], e_nums=[500], cand=("fixed", 64)),
    "mid": dict(G=100_000_000, repeat_frac=0.10, n_families=100, q=5, B=200, O=105,
                n_reads=1_000_000, lengths=[100], e_nums=[500], cand=("seeded", 12)),
    "batched": dict(G=3_100_000_000, repeat_frac=0.45, n_families=10_000, q=5, B=200, O=275,
                    n_reads=4_000_000, lengths=[100, 150, 250], e_nums=[500, 1000],
                    cand=("zipf", 1.2, 4096)),
    "large": dict(G=3_100_000_000, repeat_frac=0.45, n_families=10_000, q=6, B=1000, O=263,
                  n_reads=2_000_000, lengths=[250], e_nums=[500], cand=("uniform", 1, 2048)),
    "serve": dict(G=3_100_000_000, repeat_frac=0.45, n_families=10_000, q=5, B=200, O=275,
                  n_reads=4_000_000, lengths=[100, 150, 250], e_nums=[500],
                  cand=("zipf", 1.2, 4096)),
}

SEEDS = dict(reference=1, reads=3, counts=4, candidates=5, arrivals=6)


def make_reference(name, scale=1.0, seed=None, n_threads=None):
    w = WORKLOADS[name]
    G = max(10_000, int(w["G"] * scale))
    s = SEEDS["reference"] if seed is None else seed
    return reference(s, G, w["repeat_frac"], w["n_families"], 300, 0.85, 0.98, n_threads)


def make_workload(name, scale=1.0, read_scale=None, seed=None, ref=None, n_threads=None):
    """Build a complete workload.  Returns a dict with keys

    ref, q, B, O, n_bins_hint, codes, read_off, read_len, read_e, e_den, read_z,
    read_span, read_edits, cand_off, cand_bin, true_pair (None for seeded)."""
    w = WORKLOADS[name]
    read_scale = scale if read_scale is None else read_scale
    base = 0 if seed is None else int(seed) * 1000
    if ref is None:
        ref = make_reference(name, scale, None if seed is None else base + SEEDS["reference"],
                             n_threads)
    G = ref.size
    B = w["B"]
    n_bins = (G + B - 1) // B
    n_reads = max(1, int(w["n_reads"] * read_scale))
    rd = reads(base + SEEDS["reads"], ref, n_reads, w["lengths"], w["e_nums"], E_DEN, n_threads)
    kind = w["cand"]
    true_pair = None
    if kind[0] == "seeded":
        kidx = kmer_index(ref, kind[1])
        cand_off, cand_bin = cand_seeded(ref, kidx, rd["codes"], rd["read_off"], rd["read_len"], B,
                                         kind[1], 4096, n_threads)
        del kidx
    else:
        if kind[0] == "fixed":
            k = np.full(n_reads, kind[1], dtype=np.uint32)
        elif kind[0] == "zipf":
            k = cand_counts_zipf(base + SEEDS["counts"], n_reads, kind[1], kind[2])
        else:
            k = cand_counts_uniform(base + SEEDS["counts"], n_reads, kind[1], kind[2])
        cand_off = offsets_from_counts(k)
        cand_bin, true_pair = cand_random(base + SEEDS["candidates"], cand_off, rd["read_z"], B,
                                          n_bins, n_threads)
    return dict(ref=ref, q=w["q"], B=B, O=w["O"], n_bins_hint=n_bins, e_den=E_DEN,
                cand_off=cand_off, cand_bin=cand_bin, true_pair=true_pair, **rd)
