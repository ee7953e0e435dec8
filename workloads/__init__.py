"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no part of the sorting method: it only draws keys.  Both the
oracle side and the GPU side receive the same bytes from here.

Generator: counter-based splitmix64 (Steele, Lea, Flood 2014): word i of stream
``seed`` is mix64(seed + (i + 1) * 0x9E3779B97F4A7C15).  uint32 keys take the
high 32 bits of the word.  The paper's workload is uniform keys from a xorshift
generator (Sec. 5.1); for uniform keys the choice of generator does not matter,
and a counter-based one is reproducible in any order and in parallel.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# seeds of the named workloads
SEED_SMALL = 0x5EED0001      # n = 2^20 uint32 + index payload
SEED_LARGE = 0x5EED0002      # n = 2^28 uint32 + index payload
SEED_SKEWED = 0x5EED0003     # uint64 skewed / structured keys


def mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def words(seed: int, n: int, start: int = 0, chunk: int = 1 << 24) -> np.ndarray:
    """n uint64 words of splitmix64 stream ``seed`` starting at counter ``start``."""
    out = np.empty(n, np.uint64)
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        idx = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            out[lo:hi] = mix64(s + idx * GAMMA)
    return out


def uniform(seed: int, n: int, key_bytes: int = 4) -> np.ndarray:
    """Uniform keys over [0, 2^(8 key_bytes))."""
    w = words(seed, n)
    if key_bytes == 4:
        return (w >> np.uint64(32)).astype(np.uint32)
    if key_bytes == 8:
        return w
    raise ValueError("key_bytes must be 4 or 8")


def index_payload(n: int, dtype=np.uint32) -> np.ndarray:
    """Payload = original index (the stability check of the workloads)."""
    return np.arange(n, dtype=dtype)


def zipf(seed: int, n: int, s: float = 1.1, distinct: int = 1 << 16,
         key_bytes: int = 8) -> np.ndarray:
    """Zipf(s) over ``distinct`` seeded values: value v_k = mix64(seed ^ k) has
    probability proportional to (k+1)^-s; drawn by inverse-CDF sampling."""
    ks = np.arange(distinct, dtype=np.uint64)
    values = mix64(np.uint64(seed) ^ ks)
    if key_bytes == 4:
        values = (values >> np.uint64(32)).astype(np.uint32)
    w = np.arange(1, distinct + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    out = np.empty(n, values.dtype)
    chunk = 1 << 24
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        u = (words(seed ^ 0xA5A5A5A5, hi - lo, start=lo) >> np.uint64(11)).astype(
            np.float64) * (1.0 / (1 << 53))
        out[lo:hi] = values[np.minimum(np.searchsorted(cdf, u, side="right"), distinct - 1)]
    return out


def all_equal(seed: int, n: int, key_bytes: int = 8) -> np.ndarray:
    v = uniform(seed, 1, key_bytes)[0]
    return np.full(n, v, dtype=v.dtype)


def presorted(seed: int, n: int, key_bytes: int = 8) -> np.ndarray:
    return np.sort(uniform(seed, n, key_bytes))


def low_bits(seed: int, n: int, bits: int = 20, key_bytes: int = 8) -> np.ndarray:
    """Keys with only the low ``bits`` bits random, the rest zero."""
    k = uniform(seed, n, key_bytes)
    return k & k.dtype.type((1 << bits) - 1)


def reverse_sorted(seed: int, n: int, key_bytes: int = 4) -> np.ndarray:
    return np.sort(uniform(seed, n, key_bytes))[::-1].copy()


def few_distinct(seed: int, n: int, distinct: int = 3, key_bytes: int = 4) -> np.ndarray:
    vals = uniform(seed ^ 0x77, distinct, key_bytes)
    pick = words(seed, n) % np.uint64(distinct)
    return vals[pick.astype(np.int64)]


def log_uniform_sizes(seed: int, count: int, lo_log2: float, hi_log2: float) -> np.ndarray:
    """``count`` sizes log-uniform in [2^lo_log2, 2^hi_log2] (batched and serving inputs)."""
    u = (words(seed, count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    return np.floor(2.0 ** (lo_log2 + u * (hi_log2 - lo_log2))).astype(np.int64)


DISTRIBUTIONS = {
    "uniform": lambda seed, n, kb: uniform(seed, n, kb),
    "zipf": lambda seed, n, kb: zipf(seed, n, key_bytes=kb),
    "equal": lambda seed, n, kb: all_equal(seed, n, kb),
    "sorted": lambda seed, n, kb: presorted(seed, n, kb),
    "reverse": lambda seed, n, kb: reverse_sorted(seed, n, kb),
    "low20": lambda seed, n, kb: low_bits(seed, n, 20, kb),
    "few": lambda seed, n, kb: few_distinct(seed, n, 3, kb),
}


def make(dist: str, seed: int, n: int, key_bytes: int = 4) -> np.ndarray:
    return DISTRIBUTIONS[dist](seed, n, key_bytes)


# ---- the same streams drawn with torch on a device ----------------------------------
# For inputs too large to draw on the host in test time (n = 2^30).  Each function
# returns the bytes of its host counterpart above, as a torch tensor (int32 /
# int64 views of the unsigned keys); a CPU test checks the equality on small n.

def _signed(u: int) -> int:
    return u - (1 << 64) if u >= 1 << 63 else u


def _shr(z, k: int):
    """Logical right shift of int64 words that hold unsigned values."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def _mix64_t(z):
    z = z ^ _shr(z, 30)
    z = z * _signed(int(_M1))
    z = z ^ _shr(z, 27)
    z = z * _signed(int(_M2))
    return z ^ _shr(z, 31)


def words_t(seed: int, n: int, device, start: int = 0, chunk: int = 1 << 26):
    """``words(seed, n, start)`` as an int64 tensor on ``device``."""
    import torch
    out = torch.empty(n, dtype=torch.int64, device=device)
    s = _signed(seed & 0xFFFFFFFFFFFFFFFF)
    g = _signed(int(GAMMA))
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        idx = torch.arange(start + lo + 1, start + hi + 1, dtype=torch.int64, device=device)
        out[lo:hi] = _mix64_t(idx * g + s)
    return out


def _high32_t(w):
    import torch
    h = _shr(w, 32)
    return torch.where(h >= 1 << 31, h - (1 << 32), h).to(torch.int32)


def uniform_t(seed: int, n: int, key_bytes: int, device, start: int = 0):
    """Keys start .. start + n - 1 of ``uniform(seed, ...)`` on ``device``."""
    w = words_t(seed, n, device, start=start)
    return _high32_t(w) if key_bytes == 4 else w


def zipf_t(seed: int, n: int, device, s: float = 1.1, distinct: int = 1 << 16,
           key_bytes: int = 8):
    import torch
    ks = torch.arange(distinct, dtype=torch.int64, device=device)
    values = _mix64_t(ks ^ _signed(seed))
    if key_bytes == 4:
        values = _high32_t(values)
    w = torch.arange(1, distinct + 1, dtype=torch.float64, device=device) ** (-s)
    cdf = torch.cumsum(w, 0)
    cdf /= cdf[-1].clone()
    out = torch.empty(n, dtype=values.dtype, device=device)
    chunk = 1 << 24
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        u = _shr(words_t(seed ^ 0xA5A5A5A5, hi - lo, device, start=lo), 11).to(
            torch.float64) * (1.0 / (1 << 53))
        pick = torch.clamp(torch.searchsorted(cdf, u, right=True), max=distinct - 1)
        out[lo:hi] = values[pick]
    return out


def make_t(dist: str, seed: int, n: int, key_bytes: int, device):
    """``make(dist, seed, n, key_bytes)`` on ``device`` for the distributions of
    the large structured inputs."""
    import torch
    if dist == "uniform":
        return uniform_t(seed, n, key_bytes, device)
    if dist == "zipf":
        return zipf_t(seed, n, device, key_bytes=key_bytes)
    if dist == "equal":
        v = uniform_t(seed, 1, key_bytes, device)
        return v.expand(n).contiguous()
    if dist == "low20":
        k = uniform_t(seed, n, key_bytes, device)
        return k & ((1 << 20) - 1)
    if dist == "sorted":
        k = uniform_t(seed, n, key_bytes, device)
        top = -(1 << 63) if key_bytes == 8 else -(1 << 31)
        return torch.sort(k ^ top).values ^ top  # unsigned order via the flipped sign bit
    raise ValueError(dist)
