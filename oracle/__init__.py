"""GRIM-Filter oracle (test infrastructure only).

A thin ctypes wrapper over ``oracle.c``, the plain CPU implementation of the
bin-bitvector seed-location filter (Kim et al., BMC Genomics 2018, Sections
"Genome Metadata Representation", "GRIM-Filter Operation" and "Taking Errors
into Account").  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product library never does.

All sequences are numpy ``uint8`` arrays of base codes A=0 C=1 G=2 T=3.
"""
import ctypes
import hashlib
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)


_CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC"]


def _stamp(src, flags):
    """Hash of the source text and the compile flags a build used."""
    h = hashlib.sha1()
    with open(src, "rb") as f:
        h.update(f.read())
    h.update(" ".join(flags).encode())
    return h.hexdigest()


def build(src=_SRC, out=_LIB, extra_flags=()):
    """Compile oracle.c into a shared library with gcc (always recompiles).
    A stamp file next to the library records the hash of the source and flags,
    so that a library older than its source is never loaded by default."""
    flags = _CFLAGS + list(extra_flags)
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *flags, src, "-o", tmp])
    os.replace(tmp, out)
    with open(out + ".stamp", "w") as f:
        f.write(_stamp(src, flags))


def _current(src=_SRC, out=_LIB):
    try:
        with open(out + ".stamp") as f:
            return os.path.exists(out) and f.read().strip() == _stamp(src, _CFLAGS)
    except OSError:
        return False


class Oracle:
    """The oracle functions bound to one compiled copy of oracle.c."""

    def __init__(self, path=_LIB):
        lib = ctypes.CDLL(path)
        u64, u32 = ctypes.c_uint64, ctypes.c_uint32
        sig = {
            "oracle_num_bins": (u64, [u64, u64]),
            "oracle_vector_bytes": (u64, [u32]),
            "oracle_token": (u64, [_u8p, u32]),
            "oracle_build_bin": (None, [_u8p, u64, u64, u64, u32, u64, _u8p]),
            "oracle_build_index": (None, [_u8p, u64, u64, u64, u32, u64, u64, _u8p]),
            "oracle_max_edits": (u32, [u32, u32, u32]),
            "oracle_num_tokens": (ctypes.c_int64, [u32, u32]),
            "oracle_threshold": (ctypes.c_int64, [u32, u32, u32]),
            "oracle_count": (ctypes.c_int32, [_u8p, u32, _u8p, u32]),
            "oracle_filter": (u64, [_u8p, u64, u32, _u8p, _u64p, _u32p, _u32p, u32, u64, u64,
                                    _u64p, _u32p, _i32p, _u8p]),
            "oracle_pack_bitmask": (None, [_u8p, u64, _u32p]),
            "oracle_edit_distance_in_bin": (ctypes.c_int32, [_u8p, u64, u64, u64, u64, _u8p, u32,
                                                             _i32p]),
            "oracle_seed_candidates": (u64, [_u8p, u64, u32, _u8p, _u64p, _u32p, u64, u64, u32,
                                             _u32p, _u64p, _u32p]),
            "oracle_survivors": (u64, [_u32p, u64, _u64p, u64, _u32p, u64, _u64p, _u32p, _u32p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        self.lib = lib

    def num_bins(self, G, B):
        return int(self.lib.oracle_num_bins(G, B))

    def vector_bytes(self, q):
        return int(self.lib.oracle_vector_bytes(q))

    def token(self, codes, q):
        codes = _c(codes, np.uint8)
        assert codes.size >= q
        return int(self.lib.oracle_token(_ptr(codes, _u8p), q))

    def max_edits(self, L, e_num, e_den):
        return int(self.lib.oracle_max_edits(L, e_num, e_den))

    def num_tokens(self, L, q):
        return int(self.lib.oracle_num_tokens(L, q))

    def threshold(self, L, q, E):
        return int(self.lib.oracle_threshold(L, q, E))

    def build_bin(self, ref, B, O, q, b):
        ref = _c(ref, np.uint8)
        vec = np.zeros(self.vector_bytes(q), dtype=np.uint8)
        self.lib.oracle_build_bin(_ptr(ref, _u8p), ref.size, B, O, q, b, _ptr(vec, _u8p))
        return vec

    def build_index(self, ref, B, O, q, b_begin=0, b_end=None, n_threads=1):
        """Bitvectors of bins [b_begin, b_end) as a (n, vector_bytes) uint8 array.

        n_threads > 1 splits the bin range over Python threads (ctypes releases
        the GIL); every thread runs the same plain per-bin routine."""
        ref = _c(ref, np.uint8)
        G = ref.size
        if b_end is None:
            b_end = self.num_bins(G, B)
        nb = self.vector_bytes(q)
        out = np.empty((b_end - b_begin, nb), dtype=np.uint8)
        lib = self.lib

        def work(lo, hi):
            if hi > lo:
                lib.oracle_build_index(_ptr(ref, _u8p), G, B, O, q, lo, hi,
                                       ctypes.cast(out.ctypes.data + (lo - b_begin) * nb, _u8p))

        _split(work, b_begin, b_end, n_threads)
        return out

    def count(self, vec, q, read):
        vec = _c(vec, np.uint8)
        read = _c(read, np.uint8)
        return int(self.lib.oracle_count(_ptr(vec, _u8p), q, _ptr(read, _u8p), read.size))

    def filter_batch(self, index, q, read_codes, read_off, read_len, read_e_num, e_den,
                     cand_off, cand_bin, n_threads=1):
        """Run the oracle filter over every read.

        Returns (counts int32[n_pairs], pass uint8[n_pairs], n_out_of_range)."""
        index = _c(index, np.uint8)
        n_bins = index.shape[0] if index.ndim == 2 else index.size // self.vector_bytes(q)
        read_codes = _c(read_codes, np.uint8)
        read_off = _c(read_off, np.uint64)
        read_len = _c(read_len, np.uint32)
        read_e_num = _c(read_e_num, np.uint32)
        cand_off = _c(cand_off, np.uint64)
        cand_bin = _c(cand_bin, np.uint32)
        n_reads = read_len.size
        n_pairs = int(cand_off[-1]) if cand_off.size else 0
        counts = np.empty(n_pairs, dtype=np.int32)
        passed = np.empty(n_pairs, dtype=np.uint8)
        lib = self.lib
        bad = [0]
        blk = threading.Lock()

        def work(lo, hi):
            if hi > lo:
                n = lib.oracle_filter(_ptr(index, _u8p), n_bins, q, _ptr(read_codes, _u8p),
                                      _ptr(read_off, _u64p), _ptr(read_len, _u32p),
                                      _ptr(read_e_num, _u32p), e_den, lo, hi,
                                      _ptr(cand_off, _u64p), _ptr(cand_bin, _u32p),
                                      _ptr(counts, _i32p), _ptr(passed, _u8p))
                with blk:
                    bad[0] += int(n)

        _split(work, 0, n_reads, n_threads)
        return counts, passed, bad[0]

    def filter_compare(self, index, q, read_codes, read_off, read_len, read_e_num, e_den,
                       cand_off, cand_bin, counts, bits, r_begin=0, r_end=None, n_threads=1,
                       chunk_pairs=1 << 22):
        """Run the oracle filter over reads [r_begin, r_end) and compare every
        pair with given results (host arrays over the whole batch: int32
        counts[n_pairs], uint32 pass-bit words).

        The reads are cut at read boundaries into chunks of about chunk_pairs
        pairs; n_threads threads take chunks from a shared queue, each running
        the plain oracle_filter on its chunk alone, so that Zipf-skewed
        candidate counts still spread evenly.  Only the oracle's own results
        are compared with; nothing of the given results enters its arithmetic.
        Returns dict(pairs, reads, count_mismatches, bit_mismatches,
        out_of_range, first) with up to 8 mismatching pair indices in first."""
        index = _c(index, np.uint8)
        n_bins = index.shape[0] if index.ndim == 2 else index.size // self.vector_bytes(q)
        read_codes = _c(read_codes, np.uint8)
        read_off = _c(read_off, np.uint64)
        read_len = _c(read_len, np.uint32)
        read_e_num = _c(read_e_num, np.uint32)
        cand_off = _c(cand_off, np.uint64)
        cand_bin = _c(cand_bin, np.uint32)
        counts = np.ascontiguousarray(counts).view(np.int32)
        bytes_ = np.ascontiguousarray(bits).view(np.uint32).view(np.uint8)
        n_reads = read_len.size
        r_end = n_reads if r_end is None else int(r_end)
        r_begin = int(r_begin)
        # chunk boundaries: read indices where the pair offset crosses a multiple
        # of chunk_pairs (every chunk holds at least one read)
        marks = np.arange(int(cand_off[r_begin]), int(cand_off[r_end]), int(chunk_pairs),
                          dtype=np.uint64)
        cuts = np.searchsorted(cand_off[r_begin:r_end + 1], marks, side="right") - 1 + r_begin
        cuts = np.unique(np.concatenate([cuts, [r_begin, r_end]]).astype(np.int64))
        cuts = cuts[(cuts >= r_begin) & (cuts <= r_end)]
        chunks = list(zip(cuts[:-1].tolist(), cuts[1:].tolist()))
        lib = self.lib
        lock = threading.Lock()
        res = dict(pairs=0, reads=r_end - r_begin, count_mismatches=0, bit_mismatches=0,
                   out_of_range=0, first=[])
        nxt = [0]

        def work():
            while True:
                with lock:
                    if nxt[0] >= len(chunks):
                        return
                    a, b = chunks[nxt[0]]
                    nxt[0] += 1
                pa, pb = int(cand_off[a]), int(cand_off[b])
                n = pb - pa
                sub_off = cand_off[a:b + 1] - np.uint64(pa)
                oc = np.empty(max(1, n), dtype=np.int32)
                op = np.empty(max(1, n), dtype=np.uint8)
                bad = lib.oracle_filter(_ptr(index, _u8p), n_bins, q, _ptr(read_codes, _u8p),
                                        _ptr(read_off[a:b], _u64p), _ptr(read_len[a:b], _u32p),
                                        _ptr(read_e_num[a:b], _u32p), e_den, 0, b - a,
                                        _ptr(sub_off, _u64p),
                                        _ptr(cand_bin[pa:pb] if n else cand_bin, _u32p),
                                        _ptr(oc, _i32p), _ptr(op, _u8p))
                gc = counts[pa:pb]
                cm = np.nonzero(gc != oc[:n])[0]
                s = pa & 7
                gb = np.unpackbits(bytes_[pa >> 3:(pb + 7) >> 3], bitorder="little")[s:s + n]
                bm = np.nonzero(gb != op[:n])[0]
                with lock:
                    res["pairs"] += n
                    res["out_of_range"] += int(bad)
                    res["count_mismatches"] += int(cm.size)
                    res["bit_mismatches"] += int(bm.size)
                    for k in np.concatenate([cm, bm])[:8]:
                        if len(res["first"]) < 8:
                            res["first"].append(pa + int(k))

        ths = [threading.Thread(target=work) for _ in range(max(1, int(n_threads)))]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        return res

    def pack_bitmask(self, passed):
        passed = _c(passed, np.uint8)
        words = np.zeros((passed.size + 31) // 32, dtype=np.uint32)
        self.lib.oracle_pack_bitmask(_ptr(passed, _u8p), passed.size, _ptr(words, _u32p))
        return words

    def survivors(self, words, n_pairs, cand_off, cand_bin):
        """Passing locations in input order: (pair, read, bin) arrays."""
        words = _c(words, np.uint32)
        cand_off = _c(cand_off, np.uint64)
        cand_bin = _c(cand_bin if len(cand_bin) else np.zeros(1, np.uint32), np.uint32)
        n_reads = cand_off.size - 1
        cap = int(n_pairs)
        sp = np.empty(max(1, cap), dtype=np.uint64)
        sr = np.empty(max(1, cap), dtype=np.uint32)
        sb = np.empty(max(1, cap), dtype=np.uint32)
        n = int(self.lib.oracle_survivors(_ptr(words, _u32p), int(n_pairs), _ptr(cand_off, _u64p),
                                          n_reads, _ptr(cand_bin, _u32p), cap, _ptr(sp, _u64p),
                                          _ptr(sr, _u32p), _ptr(sb, _u32p)))
        return sp[:n], sr[:n], sb[:n]

    def edit_distance_in_bin(self, ref, B, O, b, read):
        """Smallest edit distance between `read` and any substring of bin b's span."""
        ref = _c(ref, np.uint8)
        L = len(read)
        read = _c(read if L else np.zeros(1, np.uint8), np.uint8)
        lo = b * B
        hi = min(ref.size, (b + 1) * B + O)
        row = np.empty(max(1, hi - lo + 1), dtype=np.int32)
        return int(self.lib.oracle_edit_distance_in_bin(_ptr(ref, _u8p), ref.size, B, O, b,
                                                        _ptr(read, _u8p), L, _ptr(row, _i32p)))

    def verify(self, ref, B, O, read_codes, read_off, read_len, read_e, e_den, surv_read,
               surv_bin):
        """Distances capped at E + 1 and verified flags for a survivor list."""
        d = np.empty(len(surv_read), dtype=np.int32)
        for i, (r, b) in enumerate(zip(surv_read, surv_bin)):
            o, L = int(read_off[r]), int(read_len[r])
            E = self.max_edits(L, int(read_e[r]), e_den)
            dist = self.edit_distance_in_bin(ref, B, O, int(b), read_codes[o:o + L])
            d[i] = min(dist, E + 1)
        return d

    def seed_candidates(self, ref, k, read_codes, read_off, read_len, B, cap):
        """Candidate bins from exact k-mer seeds: (cand_off u64[n+1], cand_bin u32)."""
        ref = _c(ref, np.uint8)
        read_codes = _c(read_codes if len(read_codes) else np.zeros(1, np.uint8), np.uint8)
        read_off = _c(read_off, np.uint64)
        read_len = _c(read_len, np.uint32)
        n = read_len.size
        cnt = np.zeros(max(1, n), dtype=np.uint32)
        self.lib.oracle_seed_candidates(_ptr(ref, _u8p), ref.size, k, _ptr(read_codes, _u8p),
                                        _ptr(read_off, _u64p), _ptr(read_len, _u32p), n, B, cap,
                                        _ptr(cnt, _u32p), None, None)
        off = np.zeros(n + 1, dtype=np.uint64)
        np.cumsum(cnt[:n], out=off[1:])
        bins = np.zeros(max(1, int(off[-1])), dtype=np.uint32)
        self.lib.oracle_seed_candidates(_ptr(ref, _u8p), ref.size, k, _ptr(read_codes, _u8p),
                                        _ptr(read_off, _u64p), _ptr(read_len, _u32p), n, B, cap,
                                        _ptr(cnt, _u32p), _ptr(off, _u64p), _ptr(bins, _u32p))
        return off, bins[:int(off[-1])]


def _default():
    global _lib
    with _lock:
        if _lib is None:
            if not _current():
                build()
            _lib = Oracle(_LIB)
        return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _fwd(name):
    def f(*args, **kw):
        return getattr(_default(), name)(*args, **kw)
    f.__name__ = name
    f.__doc__ = getattr(Oracle, name).__doc__
    return f


for _n in ("num_bins", "vector_bytes", "token", "max_edits", "num_tokens", "threshold",
           "build_bin", "build_index", "count", "filter_batch", "filter_compare", "pack_bitmask",
           "survivors",
           "edit_distance_in_bin", "verify", "seed_candidates"):
    globals()[_n] = _fwd(_n)


def _split(fn, lo, hi, n_threads):
    n_threads = max(1, int(n_threads))
    if n_threads == 1 or hi - lo < 2:
        fn(lo, hi)
        return
    step = (hi - lo + n_threads - 1) // n_threads
    ths = [threading.Thread(target=fn, args=(a, min(hi, a + step))) for a in range(lo, hi, step)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
