"""Radsort oracle: ctypes binding of the plain sequential C implementation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never loads it, and it shares no code with the GPU library.

Every routine follows the paper "Parallel O(sqrt n) Overhead LSD Radix Sort":
setup (Alg. 4), sizeOfNextBlock (Alg. 3), sortPhase (Alg. 5), fixupPhase
(Alg. 6), finalize (Alg. 7), the driver (Alg. 2), the out-of-place round (Alg. 1)
the space formula (Sec. 3, Sec. 4), truncate (Alg. 8) and the use of the
permuted representation without finalize (Sec. 4.1).  Keys and payloads cross this binding as
uint64 arrays; narrower inputs are widened by the caller.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "radsort_oracle.c")]

# indices of the counters kept by the oracle (radsort_oracle.h)
C_ROUNDS, C_LEMMA1_EQUAL, C_FINALIZE_COPIES = 0, 1, 2
C_FIRST_ERROR = 3
NCOUNTERS = 10
COUNTER_NAMES = [
    "rounds", "lemma1_equal", "finalize_copies", "lemma1_violation",
    "lemma2_violation", "pool_overrun", "finalize_tail_overwritten",
    "finalize_count_mismatch", "finalize_home_taken",
]


def build(extra_flags=()) -> str:
    """Compile the oracle with gcc into ``liboracle.so`` (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           *extra_flags, "-o", LIB_PATH, *SOURCES]
    subprocess.run(cmd, check=True)
    return LIB_PATH


def build_variant(out_path: str, defines=()) -> str:
    """Compile a copy of the oracle with extra -D flags into ``out_path``."""
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC",
           *[f"-D{d}" for d in defines], "-o", out_path, *SOURCES]
    subprocess.run(cmd, check=True)
    return out_path


_U64P = ctypes.POINTER(ctypes.c_uint64)


def _bind(lib):
    u64, vp = ctypes.c_uint64, ctypes.c_void_p
    sig = {
        "orc_key": (u64, [u64, u64, u64, u64]),
        "orc_create": (vp, [u64, u64, u64, u64]),
        "orc_destroy": (None, [vp]),
        "orc_load": (None, [vp, _U64P, _U64P]),
        "orc_store": (None, [vp, _U64P, _U64P]),
        "orc_setup": (None, [vp]),
        "orc_sort_phase": (None, [vp, u64]),
        "orc_fixup_phase": (None, [vp]),
        "orc_round": (None, [vp, u64]),
        "orc_finalize": (None, [vp]),
        "orc_radsort": (ctypes.c_int, [_U64P, _U64P, u64, u64, u64, u64]),
        "orc_npi": (u64, [vp]),
        "orc_f": (u64, [vp]),
        "orc_i_out": (u64, [vp]),
        "orc_get_pi": (None, [vp, _U64P]),
        "orc_get_P": (None, [vp, _U64P, _U64P]),
        "orc_get_C": (None, [vp, _U64P]),
        "orc_get_counters": (None, [vp, _U64P]),
        "orc_get_logical": (u64, [vp, _U64P, _U64P]),
        "orc_check_invariant": (ctypes.c_int, [vp]),
        "orc_truncate": (ctypes.c_int, [vp, u64, ctypes.c_int64]),
        "orc_truncate_count": (ctypes.c_int, [vp, u64]),
        "orc_set_logical": (None, [vp, _U64P, _U64P]),
        "orc_n": (u64, [vp]),
        "orc_test_set_pi": (None, [vp, u64, u64]),
        "orc_test_set_P": (None, [vp, u64, u64, u64]),
        "orc_test_set_f": (None, [vp, u64]),
        "orc_oop_lsd": (ctypes.c_int, [_U64P, _U64P, u64, u64, u64, u64]),
        "orc_histograms": (None, [_U64P, u64, u64, u64, _U64P]),
        "orc_extra_bytes": (u64, [u64, u64, u64, u64, u64, u64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIBS: dict = {}


def load(path: str | None = None):
    """Load (building first if absent) the oracle library at ``path``."""
    path = path or LIB_PATH
    if path not in _LIBS:
        if path == LIB_PATH and not os.path.exists(path):
            build()
        _LIBS[path] = _bind(ctypes.CDLL(path))
    return _LIBS[path]


def _p(a):
    return None if a is None else a.ctypes.data_as(_U64P)


def _u64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint64).copy()


def key(x: int, t: int, sigma: int, nt: int, lib=None) -> int:
    """key(x, t) of Sec. 1: digit t (0 = most significant) of n_t base-sigma digits."""
    return int((lib or load()).orc_key(x, t, sigma, nt))


class Radsort:
    """Step-by-step sequential Radsort (Alg. 2) over uint64 keys and payloads."""

    def __init__(self, keys, vals=None, sigma=256, nt=4, b=1024, lib=None):
        self.lib = lib or load()
        self.n0, self.sigma, self.nt, self.b = len(keys), sigma, nt, b
        self.has_vals = vals is not None
        self._st = self.lib.orc_create(self.n0, sigma, nt, b)
        if not self._st:
            raise MemoryError("oracle state allocation failed")
        k = _u64(keys)
        v = _u64(vals) if vals is not None else np.zeros(self.n0, np.uint64)
        self.lib.orc_load(self._st, _p(k), _p(v))

    def close(self):
        if self._st:
            self.lib.orc_destroy(self._st)
            self._st = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # phases
    def setup(self):
        self.lib.orc_setup(self._st)

    def sort_phase(self, t):
        self.lib.orc_sort_phase(self._st, t)

    def fixup_phase(self):
        self.lib.orc_fixup_phase(self._st)

    def round(self, t):
        self.lib.orc_round(self._st, t)

    def finalize(self):
        self.lib.orc_finalize(self._st)

    def truncate(self, i, j):
        """Alg. 8: element j of logical block i becomes the last datum (j = -1
        leaves block i empty)."""
        if self.lib.orc_truncate(self._st, i, j) != 0:
            raise ValueError(f"truncate({i}, {j}) names no element of the dataset")

    def truncate_count(self, count):
        """Keeps the first ``count`` elements of the logical sequence."""
        if self.lib.orc_truncate_count(self._st, count) != 0:
            raise ValueError(f"count {count} exceeds the dataset ({self.n})")

    def set_logical(self, keys, vals=None):
        """Overwrites the dataset in logical order through the permuted
        representation (``vals`` None keeps the payloads)."""
        k = _u64(keys)
        v = _u64(vals) if vals is not None else None
        if len(k) != self.n or (v is not None and len(v) != self.n):
            raise ValueError("set_logical needs exactly n elements")
        self.lib.orc_set_logical(self._st, _p(k), _p(v))

    # test hooks: plant a broken state (for the pins of the invariant checker)
    def plant_pi(self, i, v):
        self.lib.orc_test_set_pi(self._st, i, v)

    def plant_P(self, k, idx, length):
        self.lib.orc_test_set_P(self._st, k, idx, length)

    def plant_f(self, f):
        self.lib.orc_test_set_f(self._st, f)

    # inspection
    @property
    def n(self):
        """Elements in the dataset (smaller than at creation after truncate)."""
        return int(self.lib.orc_n(self._st))

    @property
    def npi(self):
        return int(self.lib.orc_npi(self._st))

    @property
    def f(self):
        return int(self.lib.orc_f(self._st))

    @property
    def i_out(self):
        return int(self.lib.orc_i_out(self._st))

    def pi(self):
        out = np.zeros(self.npi, np.uint64)
        self.lib.orc_get_pi(self._st, _p(out))
        return out

    def P(self):
        idx = np.zeros(self.sigma, np.uint64)
        ln = np.zeros(self.sigma, np.uint64)
        self.lib.orc_get_P(self._st, _p(idx), _p(ln))
        return idx, ln

    def C(self):
        out = np.zeros(self.sigma, np.uint64)
        self.lib.orc_get_C(self._st, _p(out))
        return out

    def counters(self):
        out = np.zeros(NCOUNTERS, np.uint64)
        self.lib.orc_get_counters(self._st, _p(out))
        return {name: int(out[i]) for i, name in enumerate(COUNTER_NAMES)}

    def logical(self):
        k = np.zeros(self.n, np.uint64)
        v = np.zeros(self.n, np.uint64)
        cnt = int(self.lib.orc_get_logical(self._st, _p(k), _p(v)))
        return k, v, cnt

    def invariant(self):
        return int(self.lib.orc_check_invariant(self._st))

    def result(self):
        k = np.zeros(self.n, np.uint64)
        v = np.zeros(self.n, np.uint64)
        self.lib.orc_store(self._st, _p(k), _p(v))
        return k, v


def radsort(keys, vals=None, sigma=256, nt=4, b=1024, lib=None):
    """Full sequential Radsort (Alg. 2).  Returns (keys, vals) as uint64 arrays."""
    lib = lib or load()
    k = _u64(keys)
    v = _u64(vals) if vals is not None else np.zeros(len(k), np.uint64)
    rc = lib.orc_radsort(_p(k), _p(v), len(k), sigma, nt, b)
    if rc != 0:
        raise RuntimeError(f"oracle radsort failed (rc={rc})")
    return k, v


def oop_lsd(keys, vals=None, sigma=256, nt=4, rounds=None, lib=None):
    """Out-of-place LSD radix sort, Alg. 1 applied ``rounds`` times (default n_t)."""
    lib = lib or load()
    k = _u64(keys)
    v = _u64(vals) if vals is not None else np.zeros(len(k), np.uint64)
    rc = lib.orc_oop_lsd(_p(k), _p(v), len(k), sigma, nt, nt if rounds is None else rounds)
    if rc != 0:
        raise MemoryError("oracle oop_lsd allocation failed")
    return k, v


def histograms(keys, sigma=256, nt=4, lib=None):
    """Histograms of every key position: array [n_t, sigma] (the first loop of Alg. 1)."""
    lib = lib or load()
    k = _u64(keys)
    out = np.zeros(nt * sigma, np.uint64)
    lib.orc_histograms(_p(k), len(k), sigma, nt, _p(out))
    return out.reshape(nt, sigma)


def extra_bytes(n, sigma, b, elem_bytes, ptr_bytes=8, int_bytes=4, lib=None):
    """Extra storage besides A (Sec. 3 "Space"; itemised as in Sec. 4)."""
    return int((lib or load()).orc_extra_bytes(n, sigma, b, elem_bytes, ptr_bytes, int_bytes))


def digit_params(key_bytes: int, digit_bits: int):
    """sigma and n_t for integer keys of key_bytes bytes split into digit_bits digits."""
    sigma = 1 << digit_bits
    nt = (8 * key_bytes + digit_bits - 1) // digit_bits
    return sigma, nt
