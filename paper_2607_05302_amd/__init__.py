"""Radsort on MI355X: thin ctypes binding of libradsort.so (include/radsort.h).

Every step of the sort runs in the library's HIP kernels.  This module only
marshals arguments: device pointers and sizes from torch tensors, the current
HIP stream, and return codes into exceptions.  There is no CPU fallback: when the
library is missing, every call raises.

    import paper_2607_05302_amd as radsort
    radsort.sort_(keys, payload)            # in place, ascending, stable

Keys are read as unsigned integers of their width: torch.uint32 / torch.int32
(4 bytes) or torch.uint64 / torch.int64 (8 bytes), bit patterns taken as
unsigned.  The payload, optional, is any 4- or 8-byte integer tensor of the same
length.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libradsort.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_TIMEOUT, E_ORDER = 0, -1, -2, -3, -4, -5, -6
F_CHECK, F_TIMING, F_SHARED, F_SEQ_DRAWS, F_DEBUG_ORDER = 1, 2, 4, 8, 16
F_DEBUG_PLANT = 0x80000000  # with F_DEBUG_ORDER: marks with a wrong tag (tests the check)
MAX_ROUNDS = 64

# every function declared in include/radsort.h
ABI = [
    "radsort_sort_pairs", "radsort_sort", "radsort_workspace_bytes", "radsort_oop_sort_pairs",
    "radsort_oop_workspace_bytes", "radsort_histograms", "radsort_last_stats",
    "radsort_strerror", "radsort_state_create", "radsort_state_setup", "radsort_state_round",
    "radsort_state_finalize", "radsort_state_finalize_sequential", "radsort_state_read",
    "radsort_state_logical", "radsort_state_dims", "radsort_state_destroy",
    "radsort_sort_segments", "radsort_segments_workspace_bytes",
    "radsort_state_blocks", "radsort_state_planes", "radsort_state_count",
    "radsort_state_truncate", "radsort_state_restart", "radsort_workspace_error",
    "radsort_sort_pairs_noalloc", "radsort_msd_sort_pairs", "radsort_copy",
]
NOALLOC_SCRATCH_BYTES = 32 << 20  # RADSORT_NOALLOC_SCRATCH_BYTES
SEG_CLASSES = 32


class RadsortError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"radsort error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("block_elems", ctypes.c_uint32), ("tile_elems", ctypes.c_uint32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64),
                ("flags", ctypes.c_uint32)]


class SegTuning(ctypes.Structure):
    _fields_ = [("classes", ctypes.c_uint32), ("max_log2n", ctypes.c_uint32 * SEG_CLASSES),
                ("block_elems", ctypes.c_uint32 * SEG_CLASSES),
                ("digit_bits", ctypes.c_uint32 * SEG_CLASSES)]


class Stats(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_uint64), ("input_bytes", ctypes.c_uint64),
                ("rounds", ctypes.c_uint32), ("error_bits", ctypes.c_uint32),
                ("timed", ctypes.c_uint32), ("setup_ms", ctypes.c_float),
                ("round_ms", ctypes.c_float * MAX_ROUNDS),
                ("count_ms", ctypes.c_float * MAX_ROUNDS), ("fixup_ms", ctypes.c_float),
                ("finalize_ms", ctypes.c_float), ("total_ms", ctypes.c_float)]


_lib = None


def load(path: str | None = None):
    """Load libradsort.so; raises if it was not built (no fallback exists)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libradsort.so not found at {p}: run __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    vp, u64, i32, u32p = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32)
    op = ctypes.POINTER(Opts)
    sig = {
        "radsort_sort_pairs": (i32, [vp, vp, u64, i32, i32, i32, op, vp]),
        "radsort_msd_sort_pairs": (i32, [vp, vp, u64, i32, i32, i32, op, vp]),
        "radsort_copy": (i32, [vp, vp, u64, vp]),
        "radsort_sort_pairs_noalloc": (i32, [vp, vp, u64, i32, i32, i32, ctypes.c_uint32,
                                             ctypes.c_uint32, vp]),
        "radsort_sort": (i32, [vp, u64, i32, i32, vp]),
        "radsort_workspace_bytes": (u64, [u64, i32, i32, i32, op]),
        "radsort_oop_sort_pairs": (i32, [vp, vp, u64, i32, i32, i32, op, vp]),
        "radsort_oop_workspace_bytes": (u64, [u64, i32, i32, i32, op]),
        "radsort_workspace_error": (i32, [vp, u64, i32, i32, i32, op, i32, u32p, vp]),
        "radsort_histograms": (i32, [vp, u64, i32, i32, vp, vp]),
        "radsort_last_stats": (i32, [ctypes.POINTER(Stats)]),
        "radsort_strerror": (ctypes.c_char_p, [i32]),
        "radsort_state_create": (i32, [ctypes.POINTER(vp), vp, vp, u64, i32, i32, i32, op]),
        "radsort_state_setup": (i32, [vp, vp]),
        "radsort_state_round": (i32, [vp, vp]),
        "radsort_state_finalize": (i32, [vp, vp]),
        "radsort_state_finalize_sequential": (i32, [vp, vp]),
        "radsort_state_read": (i32, [vp, u32p, u32p, u32p, u32p, vp]),
        "radsort_state_logical": (i32, [vp, vp, vp, vp]),
        "radsort_state_dims": (i32, [vp, u32p, u32p, u32p]),
        "radsort_state_destroy": (i32, [vp]),
        "radsort_state_blocks": (i32, [vp, vp, vp, vp]),
        "radsort_state_planes": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), u32p]),
        "radsort_state_count": (i32, [vp, ctypes.POINTER(u64)]),
        "radsort_state_truncate": (i32, [vp, u64, vp]),
        "radsort_state_restart": (i32, [vp, vp]),
        "radsort_sort_segments": (i32, [vp, vp, ctypes.POINTER(u64), vp, ctypes.c_uint32, i32, i32,
                                        ctypes.POINTER(SegTuning), op, vp]),
        "radsort_segments_workspace_bytes": (u64, [ctypes.POINTER(u64), ctypes.c_uint32, i32, i32,
                                                   ctypes.POINTER(SegTuning), op]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().radsort_strerror(code).decode()


def _check(rc: int):
    if rc != OK:
        raise RadsortError(rc, strerror(rc))


def _width(t) -> int:
    import torch
    w = {torch.int32: 4, torch.uint32: 4, torch.int64: 8, torch.uint64: 8}.get(t.dtype)
    if w is None:
        raise TypeError(f"unsupported dtype {t.dtype}: need a 4- or 8-byte integer tensor")
    return w


def _stream(stream, device):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _opts(block_elems=1024, workspace=None, flags=0):
    o = Opts()
    o.block_elems = block_elems
    o.tile_elems = 0
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.flags = flags
    return o


def _validate(keys, payload):
    if not keys.is_cuda:
        raise ValueError("keys must be a device tensor")
    if not keys.is_contiguous():
        raise ValueError("keys must be contiguous")
    if payload is not None:
        if payload.device != keys.device or not payload.is_contiguous():
            raise ValueError("payload must be a contiguous tensor on the keys' device")
        if payload.numel() != keys.numel():
            raise ValueError("payload and keys differ in length")
    return _width(keys), (_width(payload) if payload is not None else 0)


def workspace_bytes(n, key_bytes=4, payload_bytes=0, digit_bits=8, block_elems=1024,
                    shared=False) -> int:
    """radsort_workspace_bytes; shared: for calls made with shared=True."""
    o = _opts(block_elems, None, F_SHARED if shared else 0)
    return int(load().radsort_workspace_bytes(n, key_bytes, payload_bytes, digit_bits,
                                              ctypes.byref(o)))


def oop_workspace_bytes(n, key_bytes=4, payload_bytes=0, digit_bits=8, block_elems=1024) -> int:
    o = _opts(block_elems)
    return int(load().radsort_oop_workspace_bytes(n, key_bytes, payload_bytes, digit_bits,
                                                  ctypes.byref(o)))


def sort_(keys, payload=None, digit_bits=8, block_elems=1024, stream=None, workspace=None,
          check=False, timing=False, shared=False, seq_draws=False):
    """Radsort in place on the current stream (radsort_sort_pairs).  shared: other
    work runs on the GPU at the same time (RADSORT_F_SHARED); seq_draws: blocks are
    drawn in the sequential algorithm's order (RADSORT_F_SEQ_DRAWS)."""
    kb, vb = _validate(keys, payload)
    o = _opts(block_elems, workspace, (F_CHECK if check else 0) | (F_TIMING if timing else 0)
              | (F_SHARED if shared else 0) | (F_SEQ_DRAWS if seq_draws else 0))
    with _device(keys):
        rc = load().radsort_sort_pairs(
            ctypes.c_void_p(keys.data_ptr()),
            ctypes.c_void_p(payload.data_ptr() if payload is not None else None),
            keys.numel(), kb, vb, digit_bits, ctypes.byref(o), _stream(stream, keys.device))
    _check(rc)
    return keys, payload


def copy_(dst, src, stream=None):
    """dst[:] = src[:] by the library's streaming copy kernel (radsort_copy); both
    contiguous device tensors of the same size in bytes."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (dst.is_contiguous() and
                                                           src.is_contiguous()):
        raise ValueError("copy_ needs contiguous tensors of equal size")
    with _device(src):
        rc = load().radsort_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                 nbytes, _stream(stream, src.device))
    _check(rc)
    return dst


def msd_sort_(keys, payload=None, digit_bits=8, block_elems=1024, stream=None, check=False,
              shared=False):
    """The MSD-first split (radsort_msd_sort_pairs): a Radsort round on the top
    digit, finalize, then every top-digit group sorted by the remaining digits as
    one batch.  Waits for the stream once, between the two phases."""
    kb, vb = _validate(keys, payload)
    o = _opts(block_elems, None, (F_CHECK if check else 0) | (F_SHARED if shared else 0))
    with _device(keys):
        rc = load().radsort_msd_sort_pairs(
            ctypes.c_void_p(keys.data_ptr()),
            ctypes.c_void_p(payload.data_ptr() if payload is not None else None),
            keys.numel(), kb, vb, digit_bits, ctypes.byref(o), _stream(stream, keys.device))
    _check(rc)
    return keys, payload


def sort_noalloc_(keys, payload=None, digit_bits=8, block_elems=1024, stream=None,
                  check=False, seq_draws=False):
    """Radsort in place with the library's static scratch as workspace
    (radsort_sort_pairs_noalloc): allocates nothing.  Calls overlapping on one GPU
    share that scratch and race."""
    kb, vb = _validate(keys, payload)
    flags = (F_CHECK if check else 0) | (F_SEQ_DRAWS if seq_draws else 0)
    with _device(keys):
        rc = load().radsort_sort_pairs_noalloc(
            ctypes.c_void_p(keys.data_ptr()),
            ctypes.c_void_p(payload.data_ptr() if payload is not None else None),
            keys.numel(), kb, vb, digit_bits, block_elems, flags, _stream(stream, keys.device))
    _check(rc)
    return keys, payload


def oop_sort_(keys, payload=None, digit_bits=8, block_elems=1024, stream=None, workspace=None,
              check=False, timing=False, shared=False):
    """The out-of-place LSD baseline of Alg. 1, in place from the caller's view."""
    kb, vb = _validate(keys, payload)
    o = _opts(block_elems, workspace, (F_CHECK if check else 0) | (F_TIMING if timing else 0)
              | (F_SHARED if shared else 0))
    with _device(keys):
        rc = load().radsort_oop_sort_pairs(
            ctypes.c_void_p(keys.data_ptr()),
            ctypes.c_void_p(payload.data_ptr() if payload is not None else None),
            keys.numel(), kb, vb, digit_bits, ctypes.byref(o), _stream(stream, keys.device))
    _check(rc)
    return keys, payload


def workspace_error(keys, payload=None, digit_bits=8, block_elems=1024, stream=None,
                    workspace=None, out_of_place=False) -> int:
    """The error bits that the last sort_ (or oop_sort_ with out_of_place) of these
    arrays with this workspace left (radsort_workspace_error): 0, or bit 0 when a
    bounded wait between workgroups gave up, bit 1 for an index out of range.
    Waits for the stream."""
    kb, vb = _validate(keys, payload)
    if workspace is None:
        raise ValueError("workspace_error needs the workspace the sort used")
    o = _opts(block_elems, workspace, 0)
    bits = ctypes.c_uint32(0)
    with _device(keys):
        rc = load().radsort_workspace_error(
            ctypes.c_void_p(workspace.data_ptr()), keys.numel(), kb, vb, digit_bits,
            ctypes.byref(o), 1 if out_of_place else 0, ctypes.byref(bits),
            _stream(stream, keys.device))
    if rc not in (0, E_TIMEOUT):
        _check(rc)
    return int(bits.value)


def seg_tuning(table):
    """A SegTuning from [(max_log2n, block_elems, digit_bits), ...] in increasing
    max_log2n, or None."""
    if not table:
        return None
    t = SegTuning()
    t.classes = len(table)
    for c, (lg, b, bits) in enumerate(table):
        t.max_log2n[c], t.block_elems[c], t.digit_bits[c] = lg, b, bits
    return t


def _offsets(offsets, device):
    import numpy as np
    import torch
    host = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    dev = torch.from_numpy(host.view(np.int64)).to(device)
    return host, dev


def segments_workspace_bytes(offsets, key_bytes=4, payload_bytes=0, tuning="auto") -> int:
    import numpy as np
    if isinstance(tuning, str):
        from .tune import load_table
        tuning = load_table(key_bytes, payload_bytes)
    host = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    t = seg_tuning(tuning)
    return int(load().radsort_segments_workspace_bytes(
        host.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), len(host) - 1, key_bytes,
        payload_bytes, ctypes.byref(t) if t else None, None))


def sort_segments_(keys, payload, offsets, tuning="auto", stream=None, workspace=None,
                   check=False, offsets_dev=None):
    """Sorts keys[offsets[i]:offsets[i+1]] (with the payload) in place for every i
    (radsort_sort_segments).  tuning: [(max_log2n, block_elems, digit_bits), ...],
    "auto" for the table the autotuner wrote for this record size (if any), or
    None for the library's default.  With a caller workspace and offsets_dev
    given, the call allocates nothing and can be captured into a graph."""
    import numpy as np
    kb, vb = _validate(keys, payload)
    if isinstance(tuning, str):
        from .tune import load_table
        tuning = load_table(kb, vb)
    host = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    if offsets_dev is None:
        host, offsets_dev = _offsets(host, keys.device)
    if int(host[-1]) > keys.numel():
        raise ValueError("offsets run past the arrays")
    t = seg_tuning(tuning)
    o = _opts(0, workspace, F_CHECK if check else 0)
    with _device(keys):
        rc = load().radsort_sort_segments(
            ctypes.c_void_p(keys.data_ptr()),
            ctypes.c_void_p(payload.data_ptr() if payload is not None else None),
            host.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
            ctypes.c_void_p(offsets_dev.data_ptr()), len(host) - 1, kb, vb,
            ctypes.byref(t) if t else None, ctypes.byref(o), _stream(stream, keys.device))
    _check(rc)
    return keys, payload


def histograms(keys, digit_bits=8, stream=None):
    """Digit histograms of every key position: int32 tensor [n_t, sigma] (as uint32 bits)."""
    import torch
    kb, _ = _validate(keys, None)
    sigma = 1 << digit_bits
    nt = (8 * kb + digit_bits - 1) // digit_bits
    out = torch.empty(nt * sigma, dtype=torch.int32, device=keys.device)
    with _device(keys):
        rc = load().radsort_histograms(ctypes.c_void_p(keys.data_ptr()), keys.numel(), kb,
                                       digit_bits, ctypes.c_void_p(out.data_ptr()),
                                       _stream(stream, keys.device))
    _check(rc)
    return out.view(nt, sigma)


def last_stats() -> dict:
    """Stats of the last sort; with timing=True it waits for that sort's events."""
    s = Stats()
    _check(load().radsort_last_stats(ctypes.byref(s)))
    out = {"workspace_bytes": s.workspace_bytes, "input_bytes": s.input_bytes,
           "rounds": s.rounds, "error_bits": s.error_bits, "timed": bool(s.timed)}
    if s.timed:
        out.update(setup_ms=s.setup_ms, round_ms=[s.round_ms[i] for i in range(s.rounds)],
                   count_ms=[s.count_ms[i] for i in range(s.rounds)],
                   fixup_ms=s.fixup_ms, finalize_ms=s.finalize_ms, total_ms=s.total_ms)
    return out


class _device:
    """Makes the tensor's device current for the duration of a call."""

    def __init__(self, t):
        self.t = t

    def __enter__(self):
        import torch
        self.ctx = torch.cuda.device(self.t.device)
        self.ctx.__enter__()

    def __exit__(self, *exc):
        self.ctx.__exit__(*exc)


class State:
    """The step interface: setup, rounds, finalize, and inspection between them."""

    def __init__(self, keys, payload=None, digit_bits=8, block_elems=1024, workspace=None,
                 seq_draws=False):
        kb, vb = _validate(keys, payload)
        self.keys, self.payload = keys, payload
        self.kb, self.vb, self.digit_bits = kb, vb, digit_bits
        o = _opts(block_elems, workspace, F_SEQ_DRAWS if seq_draws else 0)
        h = ctypes.c_void_p()
        with _device(keys):
            rc = load().radsort_state_create(
                ctypes.byref(h), ctypes.c_void_p(keys.data_ptr()),
                ctypes.c_void_p(payload.data_ptr() if payload is not None else None),
                keys.numel(), kb, vb, digit_bits, ctypes.byref(o))
        _check(rc)
        self._h = h
        npi, sigma, nt = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(load().radsort_state_dims(h, ctypes.byref(npi), ctypes.byref(sigma),
                                         ctypes.byref(nt)))
        self.npi, self.sigma, self.nt = npi.value, sigma.value, nt.value

    def _call(self, name, *args, stream=None):
        with _device(self.keys):
            rc = getattr(load(), name)(self._h, *args, _stream(stream, self.keys.device))
        _check(rc)

    def setup(self, stream=None):
        self._call("radsort_state_setup", stream=stream)

    def round(self, stream=None):
        self._call("radsort_state_round", stream=stream)

    def finalize(self, stream=None):
        self._call("radsort_state_finalize", stream=stream)

    def finalize_sequential(self, stream=None):
        self._call("radsort_state_finalize_sequential", stream=stream)

    def read(self, stream=None):
        """(pi, P_idx, P_len, f) as numpy arrays; waits for the stream."""
        import numpy as np
        pi = np.zeros(self.npi, np.uint32)
        pidx = np.zeros(self.sigma, np.uint32)
        plen = np.zeros(self.sigma, np.uint32)
        f = np.zeros(1, np.uint32)
        P = ctypes.POINTER(ctypes.c_uint32)
        self._call("radsort_state_read", pi.ctypes.data_as(P), pidx.ctypes.data_as(P),
                   plen.ctypes.data_as(P), f.ctypes.data_as(P), stream=stream)
        return pi, pidx, plen, int(f[0])

    @property
    def count(self) -> int:
        """Elements in the dataset (fewer than n after truncate)."""
        c = ctypes.c_uint64()
        _check(load().radsort_state_count(self._h, ctypes.byref(c)))
        return c.value

    def truncate(self, count: int, stream=None):
        """truncate (Alg. 8): keep the first ``count`` elements in logical order."""
        self._call("radsort_state_truncate", ctypes.c_uint64(count), stream=stream)

    def restart(self, stream=None):
        """Sort the current contents again from this state (no finalize, no setup)."""
        self._call("radsort_state_restart", stream=stream)

    def blocks(self, stream=None):
        """The block table (phys, len) of logical blocks sigma .. n_pi - 1, as new
        int32 device tensors holding uint32 values."""
        import torch
        m = self.npi - self.sigma
        phys = torch.empty(m, dtype=torch.int32, device=self.keys.device)
        ln = torch.empty(m, dtype=torch.int32, device=self.keys.device)
        self._call("radsort_state_blocks", ctypes.c_void_p(phys.data_ptr()),
                   ctypes.c_void_p(ln.data_ptr()), stream=stream)
        return phys, ln

    def planes(self):
        """(device address of T's keys, of T's payload or None, block size b)."""
        tk, tv, b = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_uint32()
        _check(load().radsort_state_planes(self._h, ctypes.byref(tk), ctypes.byref(tv),
                                           ctypes.byref(b)))
        return tk.value, tv.value, b.value

    def logical(self, stream=None):
        """The permuted representation gathered in logical order (new tensors of
        ``count`` elements)."""
        import torch
        c = self.count
        ok = torch.empty(c, dtype=self.keys.dtype, device=self.keys.device)
        ov = (torch.empty(c, dtype=self.payload.dtype, device=self.payload.device)
              if self.payload is not None else None)
        self._call("radsort_state_logical", ctypes.c_void_p(ok.data_ptr()),
                   ctypes.c_void_p(ov.data_ptr() if ov is not None else None), stream=stream)
        return ok, ov

    def close(self):
        if getattr(self, "_h", None):
            load().radsort_state_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
