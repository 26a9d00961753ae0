"""Python binding of the MI355X GRIM-Filter library (libgrim.so).

Argument marshalling only: every step of the filter runs in the library's HIP
kernels.  PyTorch provides device memory and the current HIP stream.  The
functions keep the C ABI's names (include/grim.h); the few classes below own
the opaque handles.  Importing works without a GPU; calling anything that
touches the device needs one.  If libgrim.so has not been built the import
raises, and nothing falls back to another implementation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrim.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1711_01177_amd.build` "
                      "(or __graft_entry__.build())")

# PyTorch ships its own HIP runtime under the same soname as the system one
# (libamdhip64.so.7).  Loading torch first makes libgrim.so bind to that copy,
# so the process holds a single HIP runtime and device pointers and streams
# from torch are valid inside the library.
try:
    import torch as _torch_mod  # noqa: F401
except ImportError:  # host-only use (packing, ABI checks) works without torch
    _torch_mod = None

_lib = ctypes.CDLL(LIB_PATH)

GRIM_OK = 0
GRIM_PENDING = 1
GRIM_E_INVALID = -1
GRIM_E_BASE = -2
GRIM_E_BIN_RANGE = -3
GRIM_E_NOMEM = -4
GRIM_E_BUDGET = -5
GRIM_E_HIP = -6
GRIM_E_CANCELLED = -7
GRIM_E_UNSUPPORTED = -8
GRIM_E_IO = -9
GRIM_E_TIMEOUT = -10
GRIM_E_READ = -11
GRIM_E_SCRATCH = -12
GRIM_NOALLOC_SCRATCH_BYTES = 16 << 20
GRIM_FLAG_BIN_RANGE = 1
GRIM_FLAG_READ = 2
GRIM_SERVE_PASS_BITS_ONLY = 1
GRIM_BUILD_AUTO = 0
GRIM_BUILD_PER_BIN = 1
GRIM_BUILD_BLOCKS = 2
GRIM_SERVE_STORE_DOWNLOADS = 2
GRIM_SERVE_ENGINE_DOWNLOADS = 4
GRIM_FLAG_CAND_OFF = 4

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32


class GrimError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {grim_strerror(code)} ({code})" if what else
                         f"{grim_strerror(code)} ({code})")


class grim_params_t(ctypes.Structure):
    _fields_ = [("q", _u32), ("build", _u32), ("bin_stride", _u64), ("overlap", _u64)]


class grim_index_info_t(ctypes.Structure):
    _fields_ = [("q", _u32), ("device", ctypes.c_int32), ("bin_stride", _u64), ("overlap", _u64),
                ("genome_len", _u64), ("n_bins", _u64), ("vector_bytes", _u64), ("bytes", _u64),
                ("vectors", _vp)]


class grim_batch_t(ctypes.Structure):
    _fields_ = [("reads_2bit", _vp), ("n_read_words", _u64), ("read_off", _vp), ("read_len", _vp),
                ("read_e", _vp), ("e_den", _u32), ("max_len", _u32), ("cand_off", _vp),
                ("cand_bin", _vp), ("n_reads", _u64), ("n_pairs", _u64)]


class grim_tuning_t(ctypes.Structure):
    _fields_ = [("lanes_per_cand", _u32), ("unroll", _u32), ("tile_pairs", _u32),
                ("wg_per_cu", _u32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class grim_serve_cfg_t(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", _u64), ("max_inflight", _u32), ("n_streams", _u32),
                ("max_tick_pairs", _u32), ("max_len", _u32), ("flags", _u32),
                ("ticks_per_stream", _u32)]


class grim_req_stats_t(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double), ("n_pairs", _u64),
                ("tick", _u64), ("flags", _u32), ("status", ctypes.c_int32)]


class grim_serve_stats_t(ctypes.Structure):
    _fields_ = [("submitted", _u64), ("completed", _u64), ("cancelled", _u64), ("failed", _u64),
                ("ticks", _u64), ("pairs_done", _u64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("pairs_per_s", ctypes.c_double), ("peak_device_bytes", _u64),
                ("mean_requests_per_tick", ctypes.c_double), ("sched_launch_s", ctypes.c_double),
                ("sched_retire_s", ctypes.c_double), ("sched_admit_s", ctypes.c_double),
                ("stream_groups", _u32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.POINTER
_SIGS = {
    "grim_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "grim_version": (ctypes.c_int, []),
    "grim_packed_words": (_u64, [_u64]),
    "grim_pack_bases": (ctypes.c_int, [_vp, _u64, _vp, ctypes.c_int]),
    "grim_max_edits": (ctypes.c_int, [_u32, _u32, _u32, _P(_u32)]),
    "grim_threshold": (ctypes.c_int, [_u32, _u32, _u32, _P(ctypes.c_int64)]),
    "grim_build_bins": (ctypes.c_int, [_vp, _u64, _P(grim_params_t), _P(_vp), _vp]),
    "grim_index_info": (ctypes.c_int, [_vp, _P(grim_index_info_t)]),
    "grim_index_copy_to_host": (ctypes.c_int, [_vp, _vp, _u64]),
    "grim_index_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "grim_index_load": (ctypes.c_int, [ctypes.c_char_p, _P(_vp), _vp]),
    "grim_index_free": (None, [_vp]),
    "grim_default_tuning": (ctypes.c_int, [_u32, _P(grim_tuning_t)]),
    "grim_tuning_candidates": (ctypes.c_int, [_u32, _P(grim_tuning_t), _u32, _P(_u32)]),
    "grim_workspace_size": (ctypes.c_int, [_vp, _u64, _P(grim_tuning_t), _P(_u64)]),
    "grim_filter_batch": (ctypes.c_int, [_vp, _P(grim_batch_t), _vp, _vp, _vp, _u64,
                                         _P(grim_tuning_t), _vp]),
    "grim_filter_batch_noalloc": (ctypes.c_int, [_vp, _P(grim_batch_t), _vp, _vp, _vp,
                                                 _P(grim_tuning_t), _vp]),
    "grim_filter_plain": (ctypes.c_int, [_vp, _P(grim_batch_t), _vp, _vp, _vp, _u64, _vp]),
    "grim_filter_status": (ctypes.c_int, [_vp, _vp, _P(_u32)]),
    "grim_tune": (ctypes.c_int, [_vp, _P(grim_batch_t), _vp, _vp, _vp, _u64, _vp,
                                 _P(grim_tuning_t)]),
    "grim_survivors_workspace_size": (ctypes.c_int, [_u64, _P(_u64)]),
    "grim_compact_survivors": (ctypes.c_int, [_P(grim_batch_t), _vp, _u64, _vp, _vp, _vp, _vp, _vp,
                                              _u64, _vp]),
    "grim_index_attach_reference": (ctypes.c_int, [_vp, _vp, _u64, _vp]),
    "grim_verify_survivors": (ctypes.c_int, [_vp, _P(grim_batch_t), _vp, _vp, _u64, _vp, _vp,
                                             _vp]),
    "grim_index_transpose": (ctypes.c_int, [_vp, _vp]),
    "grim_filter_windows": (ctypes.c_int, [_vp, _P(grim_batch_t), _vp, _vp, _vp, _vp, _vp, _u64,
                                           _vp]),
    "grim_probe_gather": (ctypes.c_int, [_vp, _vp, _u64, _vp, _vp]),
    "grim_probe_stream": (ctypes.c_int, [_vp, _vp, _vp]),
    "grim_window_order_workspace_size": (ctypes.c_int, [_vp, _u64, _P(_u64)]),
    "grim_window_order": (ctypes.c_int, [_vp, _vp, _u64, _vp, _vp, _u64, _vp]),
    "grim_seed_index_build": (ctypes.c_int, [_vp, _u64, _u32, _P(_vp), _vp]),
    "grim_seed_index_free": (None, [_vp]),
    "grim_seed_candidates": (ctypes.c_int, [_vp, _P(grim_batch_t), _u64, _u32, _P(_vp), _vp]),
    "grim_candidates_info": (ctypes.c_int, [_vp, _P(_u64), _P(_u64), _P(_vp), _P(_vp)]),
    "grim_candidates_copy_to_host": (ctypes.c_int, [_vp, _vp, _vp]),
    "grim_candidates_free": (None, [_vp]),
    "grim_graph_create": (ctypes.c_int, [_vp, _P(grim_batch_t), _vp, _vp, _vp, _u64,
                                         _P(grim_tuning_t), _P(_vp)]),
    "grim_graph_launch": (ctypes.c_int, [_vp, _vp]),
    "grim_graph_destroy": (None, [_vp]),
    "grim_serve_create": (ctypes.c_int, [_vp, _P(grim_serve_cfg_t), _P(_vp)]),
    "grim_serve_submit": (ctypes.c_int, [_vp, _P(grim_batch_t), _P(_u64)]),
    "grim_serve_submit_inplace": (ctypes.c_int, [_vp, _P(grim_batch_t), _vp, _vp, _P(_u64)]),
    "grim_serve_poll": (ctypes.c_int, [_vp, _u64, _vp, _vp, _P(grim_req_stats_t)]),
    "grim_serve_wait": (ctypes.c_int, [_vp, _u64, ctypes.c_int64, _vp, _vp,
                                       _P(grim_req_stats_t)]),
    "grim_serve_cancel": (ctypes.c_int, [_vp, _u64]),
    "grim_serve_stats": (ctypes.c_int, [_vp, _P(grim_serve_stats_t), ctypes.c_int]),
    "grim_serve_destroy": (None, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


def grim_strerror(code):
    return _lib.grim_strerror(int(code)).decode()


def grim_version():
    return int(_lib.grim_version())


def _check(rc, what):
    if rc != GRIM_OK:
        raise GrimError(rc, what)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(int(t.data_ptr())) if t is not None else None


# ------------------------------------------------------------------ host helpers
def grim_packed_words(n_bases):
    return int(_lib.grim_packed_words(int(n_bases)))


def grim_pack_bases(bases, n_threads=0):
    """Pack base codes (0..3) or ACGT letters (uint8 array) into 2-bit words."""
    bases = np.ascontiguousarray(bases, dtype=np.uint8)
    words = np.empty(grim_packed_words(bases.size), dtype=np.uint32)
    _check(_lib.grim_pack_bases(bases.ctypes.data_as(_vp), bases.size,
                                words.ctypes.data_as(_vp), int(n_threads)), "grim_pack_bases")
    return words


def grim_max_edits(L, e_num, e_den):
    E = _u32()
    _check(_lib.grim_max_edits(int(L), int(e_num), int(e_den), ctypes.byref(E)), "grim_max_edits")
    return int(E.value)


def grim_threshold(L, q, E):
    T = ctypes.c_int64()
    _check(_lib.grim_threshold(int(L), int(q), int(E), ctypes.byref(T)), "grim_threshold")
    return int(T.value)


def grim_default_tuning(q):
    t = grim_tuning_t()
    _check(_lib.grim_default_tuning(int(q), ctypes.byref(t)), "grim_default_tuning")
    return t


def grim_tuning_candidates(q):
    """Launch shapes compiled for token length q, as grim_tuning_t list."""
    n = _u32()
    _check(_lib.grim_tuning_candidates(int(q), None, 0, ctypes.byref(n)), "grim_tuning_candidates")
    arr = (grim_tuning_t * max(1, n.value))()
    _check(_lib.grim_tuning_candidates(int(q), arr, n.value, ctypes.byref(n)),
           "grim_tuning_candidates")
    return [arr[i] for i in range(n.value)]


def tuning(lanes_per_cand=0, unroll=0, tile_pairs=0, wg_per_cu=0):
    return grim_tuning_t(lanes_per_cand, unroll, tile_pairs, wg_per_cu)


# ------------------------------------------------------------------------ index
class Index:
    """A device-resident bin-vector index (owns a grim_index_t)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle) if not isinstance(handle, ctypes.c_void_p) else handle
        self.info = grim_index_info_t()
        _check(_lib.grim_index_info(self._h, ctypes.byref(self.info)), "grim_index_info")

    @property
    def handle(self):
        return self._h

    @property
    def q(self):
        return int(self.info.q)

    @property
    def n_bins(self):
        return int(self.info.n_bins)

    @property
    def vector_bytes(self):
        return int(self.info.vector_bytes)

    @property
    def bytes(self):
        return int(self.info.bytes)

    def to_host(self):
        out = np.empty((self.n_bins, self.vector_bytes), dtype=np.uint8)
        _check(_lib.grim_index_copy_to_host(self._h, out.ctypes.data_as(_vp), out.nbytes),
               "grim_index_copy_to_host")
        return out

    def attach_reference(self, ref, stream=None):
        """Keep the packed reference on the device (for grim_verify_survivors)."""
        words = grim_pack_bases(ref)
        _check(_lib.grim_index_attach_reference(self._h, words.ctypes.data_as(_vp),
                                                int(np.asarray(ref).size), _stream(stream)),
               "grim_index_attach_reference")

    def transpose(self, stream=None):
        """Build the token-major copy used by grim_filter_windows."""
        _check(_lib.grim_index_transpose(self._h, _stream(stream)), "grim_index_transpose")

    def save(self, path):
        _check(_lib.grim_index_save(self._h, str(path).encode()), "grim_index_save")

    def free(self):
        if self._h is not None and self._h.value:
            _lib.grim_index_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def grim_build_bins(ref, q, bin_stride, overlap, stream=None, packed=False, ref_len=None,
                    build=0):
    """Build the index of a reference: codes/letters (uint8), or packed words
    (uint32, with packed=True and ref_len given).  build: GRIM_BUILD_* (0 = the
    library's choice)."""
    if packed:
        words = np.ascontiguousarray(ref, dtype=np.uint32)
        n = int(ref_len)
        if words.size < grim_packed_words(n):
            raise ValueError("packed reference shorter than grim_packed_words(ref_len)")
    else:
        words = grim_pack_bases(ref)
        n = int(np.asarray(ref).size)
    p = grim_params_t(int(q), int(build), int(bin_stride), int(overlap))
    h = ctypes.c_void_p()
    _check(_lib.grim_build_bins(words.ctypes.data_as(_vp), n, ctypes.byref(p), ctypes.byref(h),
                                _stream(stream)), "grim_build_bins")
    return Index(h)


def grim_index_load(path, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.grim_index_load(str(path).encode(), ctypes.byref(h), _stream(stream)),
           "grim_index_load")
    return Index(h)


# ------------------------------------------------------------------------ batch
class Batch:
    """Device copies of a batch (reads packed 2-bit, CSR candidates) and the
    grim_batch_t that points at them."""

    def __init__(self, codes, read_off, read_len, read_e, e_den, cand_off, cand_bin,
                 max_len=None, device="cuda", words=None):
        torch = _torch()
        read_len = np.ascontiguousarray(read_len, dtype=np.uint32)
        if words is None:
            words = grim_pack_bases(codes)
        words = np.ascontiguousarray(words, dtype=np.uint32)
        self.n_reads = int(read_len.size)
        cand_off = np.ascontiguousarray(cand_off, dtype=np.uint64)
        self.n_pairs = int(cand_off[-1]) if cand_off.size else 0
        if max_len is None:
            max_len = max(1, int(read_len.max()) if read_len.size else 1)
        self.max_len = int(max_len)
        self.e_den = int(e_den)

        def dev(a, dt):
            a = np.ascontiguousarray(a)
            if a.size == 0:
                a = np.zeros(1, dtype=a.dtype)
            return torch.from_numpy(a.view(dt)).to(device)

        self.words = dev(words, np.int32)
        self.read_off = dev(np.asarray(read_off, dtype=np.uint64), np.int64)
        self.read_len = dev(read_len, np.int32)
        self.read_e = dev(np.asarray(read_e, dtype=np.uint32), np.int32)
        self.cand_off = dev(cand_off, np.int64)
        self.cand_bin = dev(np.asarray(cand_bin, dtype=np.uint32), np.int32)
        self.n_words = int(words.size)
        self.c = grim_batch_t(_ptr(self.words), self.n_words, _ptr(self.read_off),
                              _ptr(self.read_len), _ptr(self.read_e), self.e_den, self.max_len,
                              _ptr(self.cand_off), _ptr(self.cand_bin), self.n_reads, self.n_pairs)

    @classmethod
    def from_workload(cls, w, device="cuda", max_len=None):
        return cls(w["codes"], w["read_off"], w["read_len"], w["read_e"], w["e_den"],
                   w["cand_off"], w["cand_bin"], max_len=max_len, device=device)


def alloc_outputs(n_pairs, device="cuda"):
    torch = _torch()
    counts = torch.empty(max(1, n_pairs), dtype=torch.int32, device=device)
    bits = torch.empty(max(1, (n_pairs + 31) // 32), dtype=torch.int32, device=device)
    return counts, bits


def grim_workspace_size(index, n_pairs, tune=None):
    b = _u64()
    _check(_lib.grim_workspace_size(index.handle, int(n_pairs),
                                    ctypes.byref(tune) if tune is not None else None,
                                    ctypes.byref(b)), "grim_workspace_size")
    return int(b.value)


def alloc_workspace(index, n_pairs, tune=None, device="cuda"):
    torch = _torch()
    nb = grim_workspace_size(index, n_pairs, tune)
    ws = torch.empty(nb, dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace is not 256-byte aligned")
    return ws


def grim_filter_batch(index, batch, counts, pass_bits, workspace, tune=None, stream=None):
    _check(_lib.grim_filter_batch(index.handle, ctypes.byref(batch.c), _ptr(counts),
                                  _ptr(pass_bits), _ptr(workspace), workspace.numel(),
                                  ctypes.byref(tune) if tune is not None else None,
                                  _stream(stream)), "grim_filter_batch")


def grim_filter_batch_noalloc(index, batch, counts, pass_bits, status, tune=None, stream=None):
    """The batched filter with the library's static scratch (no workspace, no
    allocation); status is a device tensor of at least 4 bytes that receives
    the call's GRIM_FLAG_* bits."""
    _check(_lib.grim_filter_batch_noalloc(index.handle, ctypes.byref(batch.c), _ptr(counts),
                                          _ptr(pass_bits), _ptr(status),
                                          ctypes.byref(tune) if tune is not None else None,
                                          _stream(stream)), "grim_filter_batch_noalloc")


def grim_filter_plain(index, batch, counts, pass_bits, workspace, stream=None):
    _check(_lib.grim_filter_plain(index.handle, ctypes.byref(batch.c), _ptr(counts),
                                  _ptr(pass_bits), _ptr(workspace), workspace.numel(),
                                  _stream(stream)), "grim_filter_plain")


def grim_filter_status(workspace, stream=None):
    """Returns (code, flags) after waiting for the stream."""
    f = _u32()
    rc = _lib.grim_filter_status(_ptr(workspace), _stream(stream), ctypes.byref(f))
    return int(rc), int(f.value)


def grim_tune(index, batch, counts, pass_bits, workspace, stream=None):
    t = grim_tuning_t()
    _check(_lib.grim_tune(index.handle, ctypes.byref(batch.c), _ptr(counts), _ptr(pass_bits),
                          _ptr(workspace), workspace.numel(), _stream(stream), ctypes.byref(t)),
           "grim_tune")
    return t


def grim_survivors_workspace_size(n_pairs):
    nb = _u64()
    _check(_lib.grim_survivors_workspace_size(int(n_pairs), ctypes.byref(nb)),
           "grim_survivors_workspace_size")
    return int(nb.value)


def grim_compact_survivors(batch, pass_bits, capacity=None, stream=None, out=None,
                           workspace=None, read_total=True):
    """Survivor list of a filtered batch: (surv_pair, surv_read, surv_bin, n_total)
    device tensors, truncated to min(total, capacity).  out = (surv_pair int64,
    surv_read int32, surv_bin int32, n int64[1]) reuses caller tensors (capacity =
    their length); read_total=False skips the host read-back of the total and
    returns the untruncated tensors with the device count tensor last."""
    torch = _torch()
    dev = pass_bits.device
    if out is not None:
        sp, sr, sb, n = out
        cap = int(sp.numel())
    else:
        cap = batch.n_pairs if capacity is None else int(capacity)
        sp = torch.empty(max(1, cap), dtype=torch.int64, device=dev)
        sr = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
        sb = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
        n = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = workspace
    if ws is None:
        ws = torch.empty(grim_survivors_workspace_size(batch.n_pairs), dtype=torch.uint8,
                         device=dev)
    _check(_lib.grim_compact_survivors(ctypes.byref(batch.c), _ptr(pass_bits), cap, _ptr(sp),
                                       _ptr(sr), _ptr(sb), _ptr(n), _ptr(ws), ws.numel(),
                                       _stream(stream)), "grim_compact_survivors")
    if not read_total:
        return sp, sr, sb, n
    total = int(n.item())
    k = min(total, cap)
    return sp[:k], sr[:k], sb[:k], total


def grim_verify_survivors(index, batch, surv_read, surv_bin, n=None, stream=None):
    """Alignment check of survivors: (dist int32[n], ok_bits int32[ceil(n/32)])."""
    torch = _torch()
    dev = surv_read.device
    n = int(surv_read.numel()) if n is None else int(n)
    dist = torch.empty(max(1, n), dtype=torch.int32, device=dev)
    ok = torch.empty(max(1, (n + 31) // 32), dtype=torch.int32, device=dev)
    _check(_lib.grim_verify_survivors(index.handle, ctypes.byref(batch.c), _ptr(surv_read),
                                      _ptr(surv_bin), n, _ptr(dist), _ptr(ok), _stream(stream)),
           "grim_verify_survivors")
    return dist[:n], ok[:(n + 31) // 32]


def grim_filter_windows(index, batch, win_lo, counts, pass_bits, workspace, stream=None,
                        order=None):
    """Bin-window filter: every bin of [win_lo[r], win_lo[r] + window size).
    order: None (index order) or a device int32/uint32 tensor of n_reads read
    ids giving the processing order (grim_window_order makes one)."""
    _check(_lib.grim_filter_windows(index.handle, ctypes.byref(batch.c), _ptr(win_lo),
                                    _ptr(order) if order is not None else None,
                                    _ptr(counts), _ptr(pass_bits), _ptr(workspace),
                                    workspace.numel(), _stream(stream)), "grim_filter_windows")


def grim_window_order_workspace_size(index, n_reads):
    n = _u64()
    _check(_lib.grim_window_order_workspace_size(index.handle, int(n_reads), ctypes.byref(n)),
           "grim_window_order_workspace_size")
    return int(n.value)


def grim_window_order(index, win_lo, order=None, workspace=None, stream=None):
    """Processing order for grim_filter_windows: the reads grouped by the
    bucket of their window start (1024-bin buckets, increasing; order within a
    bucket unspecified)."""
    import torch
    n = int(win_lo.numel())
    if order is None:
        order = torch.empty(max(1, n), dtype=torch.int32, device=win_lo.device)
    if workspace is None:
        workspace = torch.empty(grim_window_order_workspace_size(index, n), dtype=torch.uint8,
                                device=win_lo.device)
    _check(_lib.grim_window_order(index.handle, _ptr(win_lo), n, _ptr(order), _ptr(workspace),
                                  workspace.numel(), _stream(stream)), "grim_window_order")
    return order


def grim_probe_gather(index, ids, out, n=None, stream=None):
    """Gather probe: out[i] = popcount of bin ids[i]'s vector (-1 if out of
    range), read with the batched filter's access pattern (device tensors)."""
    n = int(ids.numel()) if n is None else int(n)
    _check(_lib.grim_probe_gather(index.handle, _ptr(ids), n, _ptr(out), _stream(stream)),
           "grim_probe_gather")


def grim_probe_stream(index, sink, stream=None):
    """Streaming-read probe over the whole index (sink: device int32 tensor)."""
    _check(_lib.grim_probe_stream(index.handle, _ptr(sink), _stream(stream)), "grim_probe_stream")


class SeedIndex:
    """Device k-mer position index of a reference (owns a grim_seed_index_t)."""

    def __init__(self, ref, k=12, stream=None):
        words = grim_pack_bases(ref)
        self.k = int(k)
        self.G = int(np.asarray(ref).size)
        self._h = ctypes.c_void_p()
        _check(_lib.grim_seed_index_build(words.ctypes.data_as(_vp), self.G, self.k,
                                          ctypes.byref(self._h), _stream(stream)),
               "grim_seed_index_build")

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h is not None and self._h.value:
            _lib.grim_seed_index_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Candidates:
    """A device candidate list (owns a grim_candidates_t)."""

    def __init__(self, handle):
        self._h = handle
        nr, npairs = _u64(), _u64()
        po, pb = ctypes.c_void_p(), ctypes.c_void_p()
        _check(_lib.grim_candidates_info(self._h, ctypes.byref(nr), ctypes.byref(npairs),
                                         ctypes.byref(po), ctypes.byref(pb)), "grim_candidates_info")
        self.n_reads, self.n_pairs = int(nr.value), int(npairs.value)
        self.cand_off_ptr, self.cand_bin_ptr = po.value, pb.value

    def to_host(self):
        """(cand_off u64[n_reads+1], cand_bin u32[n_pairs]) copied to the host."""
        off = np.empty(self.n_reads + 1, dtype=np.uint64)
        bins = np.empty(max(1, self.n_pairs), dtype=np.uint32)
        _check(_lib.grim_candidates_copy_to_host(self._h, off.ctypes.data_as(_vp),
                                                 bins.ctypes.data_as(_vp)),
               "grim_candidates_copy_to_host")
        return off, bins[:self.n_pairs]

    def free(self):
        if self._h is not None and self._h.value:
            _lib.grim_candidates_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def grim_seed_candidates(seed_index, batch, bin_stride, cap=4096, stream=None):
    """Candidate bins of the batch's reads from exact k-mer seeds (device)."""
    h = ctypes.c_void_p()
    _check(_lib.grim_seed_candidates(seed_index.handle, ctypes.byref(batch.c), int(bin_stride),
                                     int(cap), ctypes.byref(h), _stream(stream)),
           "grim_seed_candidates")
    return Candidates(h)


def batch_with_candidates(batch, cands):
    """A copy of `batch`'s grim_batch_t whose candidates are `cands` (device)."""
    b = Batch.__new__(Batch)
    b.__dict__.update(batch.__dict__)
    b._cands = cands
    b.n_pairs = cands.n_pairs
    b.c = grim_batch_t(batch.c.reads_2bit, batch.c.n_read_words, batch.c.read_off,
                       batch.c.read_len, batch.c.read_e, batch.c.e_den, batch.c.max_len,
                       cands.cand_off_ptr, cands.cand_bin_ptr, batch.c.n_reads, cands.n_pairs)
    return b


class Graph:
    """A captured work-list + filter launch (owns a grim_graph_t)."""

    def __init__(self, index, batch, counts, pass_bits, workspace, tune=None):
        self._h = ctypes.c_void_p()
        self._keep = (index, batch, counts, pass_bits, workspace)
        _check(_lib.grim_graph_create(index.handle, ctypes.byref(batch.c), _ptr(counts),
                                      _ptr(pass_bits), _ptr(workspace), workspace.numel(),
                                      ctypes.byref(tune) if tune is not None else None,
                                      ctypes.byref(self._h)), "grim_graph_create")

    def launch(self, stream=None):
        _check(_lib.grim_graph_launch(self._h, _stream(stream)), "grim_graph_launch")

    def destroy(self):
        if self._h is not None and self._h.value:
            _lib.grim_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def grim_graph_create(index, batch, counts, pass_bits, workspace, tune=None):
    return Graph(index, batch, counts, pass_bits, workspace, tune)


# ---------------------------------------------------------------------- serving
def _pinned_copy(a, dtype):
    """A copy of `a` in page-locked host memory (a numpy view of a pinned
    torch tensor, which owns the memory)."""
    torch = _torch()
    a = np.ascontiguousarray(a, dtype=dtype)
    t = torch.empty(max(1, a.nbytes), dtype=torch.uint8, pin_memory=True)
    v = t.numpy().view(dtype)[:a.size]
    v[...] = a
    return v, t


class HostBatch:
    """Host arrays of one request and the grim_batch_t pointing at them.

    pinned=True keeps the arrays (and the result buffers used by in-place
    submission) in page-locked memory, so the server moves them by direct DMA."""

    def __init__(self, codes, read_off, read_len, read_e, e_den, cand_off, cand_bin, max_len=None,
                 words=None, pinned=False):
        self._keep = []

        def arr(a, dtype):
            if not pinned:
                return np.ascontiguousarray(a, dtype=dtype)
            v, t = _pinned_copy(a, dtype)
            self._keep.append(t)
            return v

        self.words = arr(words if words is not None else grim_pack_bases(codes), np.uint32)
        self.read_off = arr(read_off, np.uint64)
        self.read_len = arr(read_len, np.uint32)
        self.read_e = arr(read_e, np.uint32)
        self.cand_off = arr(cand_off, np.uint64)
        self.cand_bin = arr(cand_bin if len(cand_bin) else np.zeros(1, np.uint32), np.uint32)
        n_out = int(np.asarray(cand_off)[-1]) if len(cand_off) else 0
        self.out_counts = arr(np.zeros(max(1, n_out), np.int32), np.int32)
        self.out_bits = arr(np.zeros(max(1, (n_out + 31) // 32), np.uint32), np.uint32)
        self.n_reads = int(self.read_len.size)
        self.n_pairs = int(self.cand_off[-1]) if self.cand_off.size else 0
        self.max_len = int(max_len if max_len is not None else
                           (self.read_len.max() if self.read_len.size else 1))
        self.c = grim_batch_t(self.words.ctypes.data, self.words.size, self.read_off.ctypes.data,
                              self.read_len.ctypes.data, self.read_e.ctypes.data, int(e_den),
                              self.max_len, self.cand_off.ctypes.data, self.cand_bin.ctypes.data,
                              self.n_reads, self.n_pairs)


class Server:
    """Continuous-batching server over a resident index (owns a grim_server_t).

    downloads: "auto" (the server's choice after probing its streams), "store"
    (GRIM_SERVE_STORE_DOWNLOADS) or "engine" (GRIM_SERVE_ENGINE_DOWNLOADS)."""

    _DOWNLOADS = {"auto": 0, "store": GRIM_SERVE_STORE_DOWNLOADS,
                  "engine": GRIM_SERVE_ENGINE_DOWNLOADS}

    def __init__(self, index, hbm_budget_bytes=0, max_inflight=0, n_streams=0, max_tick_pairs=0,
                 max_len=0, pass_bits_only=False, ticks_per_stream=0, downloads="auto"):
        self.index = index
        self.pass_bits_only = bool(pass_bits_only)
        if downloads not in self._DOWNLOADS:
            raise ValueError(f"downloads must be one of {sorted(self._DOWNLOADS)}")
        cfg = grim_serve_cfg_t(int(hbm_budget_bytes), int(max_inflight), int(n_streams),
                               int(max_tick_pairs), int(max_len),
                               (GRIM_SERVE_PASS_BITS_ONLY if pass_bits_only else 0) |
                               self._DOWNLOADS[downloads],
                               int(ticks_per_stream))
        self._h = ctypes.c_void_p()
        _check(_lib.grim_serve_create(index.handle, ctypes.byref(cfg), ctypes.byref(self._h)),
               "grim_serve_create")
        self._pending = {}

    def submit(self, hb):
        t = _u64()
        rc = _lib.grim_serve_submit(self._h, ctypes.byref(hb.c), ctypes.byref(t))
        if rc != GRIM_OK:
            raise GrimError(rc, "grim_serve_submit")
        self._pending[int(t.value)] = hb.n_pairs
        return int(t.value)

    def submit_inplace(self, hb):
        """Queue hb without copying; results land in hb.out_counts / hb.out_bits."""
        t = _u64()
        rc = _lib.grim_serve_submit_inplace(self._h, ctypes.byref(hb.c),
                                            hb.out_counts.ctypes.data_as(_vp),
                                            hb.out_bits.ctypes.data_as(_vp), ctypes.byref(t))
        if rc != GRIM_OK:
            raise GrimError(rc, "grim_serve_submit_inplace")
        self._pending[int(t.value)] = (hb.n_pairs, hb)
        return int(t.value)

    def _result(self, fn, ticket, *extra):
        pend = self._pending.get(ticket, 0)
        if isinstance(pend, tuple):  # in place: results are already in the batch's buffers
            n, hb = pend
            counts, bits = hb.out_counts, hb.out_bits
        else:
            n = pend
            counts = None if self.pass_bits_only else np.empty(max(1, n), dtype=np.int32)
            bits = np.empty(max(1, (n + 31) // 32), dtype=np.uint32)
        st = grim_req_stats_t()
        rc = fn(self._h, int(ticket), *extra,
                counts.ctypes.data_as(_vp) if counts is not None else None,
                bits.ctypes.data_as(_vp), ctypes.byref(st))
        if rc in (GRIM_PENDING, GRIM_E_TIMEOUT):
            return rc, None, None, None
        self._pending.pop(ticket, None)
        # with pass bits only the counts are not results (an in-place batch's
        # count buffer is left as it was)
        return rc, (None if self.pass_bits_only else counts[:n]), bits[:(n + 31) // 32], st

    def poll(self, ticket):
        return self._result(_lib.grim_serve_poll, ticket)

    def wait(self, ticket, timeout_ms=-1):
        return self._result(lambda h, t, c, b, s: _lib.grim_serve_wait(h, t, int(timeout_ms), c, b, s),
                            ticket)

    def cancel(self, ticket):
        _check(_lib.grim_serve_cancel(self._h, int(ticket)), "grim_serve_cancel")

    def stats(self, reset=False):
        s = grim_serve_stats_t()
        _check(_lib.grim_serve_stats(self._h, ctypes.byref(s), int(bool(reset))), "grim_serve_stats")
        return s.as_dict()

    def destroy(self):
        if self._h is not None and self._h.value:
            _lib.grim_serve_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
