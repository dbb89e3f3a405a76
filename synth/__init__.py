"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws numbers: it holds none of the sorting method's arithmetic.  Every
array is a pure function of (size, seed), so the CPU oracle and the GPU path always see
identical inputs.

The random source is SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): draw k (0-based) of the stream seeded with ``seed`` is
``mix(seed + (k + 1) * 0x9E3779B97F4A7C15)`` with the published 64-bit finaliser ``mix``.  The
k-th draw is computed directly from k, so a stream can be produced in vectorised chunks.

The paper evaluates on uniformly distributed random items and mentions six input
distributions without listing them (Section 3 and Section 5); the distributions below are
synthetic stand-ins with the shapes named for each workload.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22

__all__ = [
    "mix64", "draws64", "draws32", "uniform_u32", "gaussian_u32", "bucket_u32",
    "staggered_u32", "sorted_u32", "equal_u32", "uniform_u64", "zipf_u64",
    "index_values", "segment_sizes", "normal_f32_segments", "DISTRIBUTIONS_U32", "make_u32",
]


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser, applied in place to a uint64 array (and returned)."""
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def draws64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Draws ``start .. start+count-1`` of the SplitMix64 stream seeded with ``seed``."""
    out = np.empty(count, dtype=np.uint64)
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    for c0 in range(0, count, _CHUNK):
        c1 = min(count, c0 + _CHUNK)
        k = np.arange(start + c0 + 1, start + c1 + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            k *= _GAMMA
            k += s
        out[c0:c1] = mix64(k)
    return out


def draws32(seed: int, count: int, start: int = 0) -> np.ndarray:
    """The top 32 bits of each 64-bit draw."""
    out = np.empty(count, dtype=np.uint32)
    for c0 in range(0, count, _CHUNK):
        c1 = min(count, c0 + _CHUNK)
        out[c0:c1] = (draws64(seed, c1 - c0, start + c0) >> np.uint64(32)).astype(np.uint32)
    return out


def _unit_double(d: np.ndarray) -> np.ndarray:
    """Map 64-bit draws to doubles in [0, 1) using their top 53 bits."""
    return (d >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# --------------------------------------------------------------------------- uint32 keys

def uniform_u32(n: int, seed: int) -> np.ndarray:
    """i.i.d. uniform over [0, 2^32)."""
    return draws32(seed, n)


def gaussian_u32(n: int, seed: int) -> np.ndarray:
    """Mean of four uniform 32-bit draws (draws 4t..4t+3 for item t), an approximate Gaussian."""
    out = np.empty(n, dtype=np.uint32)
    step = _CHUNK // 4
    for c0 in range(0, n, step):
        c1 = min(n, c0 + step)
        d = draws32(seed, 4 * (c1 - c0), 4 * c0).astype(np.uint64).reshape(-1, 4)
        out[c0:c1] = (d.sum(axis=1) >> np.uint64(2)).astype(np.uint32)
    return out


def _grouped(n: int, seed: int, p: int, perm) -> np.ndarray:
    shift = 32 - int(p).bit_length() + 1  # width of one subrange is 2^(32 - log2 p)
    assert (1 << (32 - shift)) == p, "p must be a power of two"
    t = np.arange(n, dtype=np.uint64)
    g = (t * np.uint64(p)) // np.uint64(max(n, 1))
    sub = perm(g)
    low = draws32(seed, n) >> np.uint32(32 - shift)
    return ((sub << np.uint64(shift)) + low.astype(np.uint64)).astype(np.uint32)


def bucket_u32(n: int, seed: int, p: int = 64) -> np.ndarray:
    """p groups of consecutive items; group g draws uniformly inside subrange g of [0, 2^32)."""
    return _grouped(n, seed, p, lambda g: g)


def staggered_u32(n: int, seed: int, p: int = 64) -> np.ndarray:
    """Like ``bucket_u32`` but group g uses subrange 2g+1 (first half) or 2g-p (second half)."""
    half = np.uint64(p // 2)

    def perm(g):
        return np.where(g < half, np.uint64(2) * g + np.uint64(1), np.uint64(2) * g - np.uint64(p))

    return _grouped(n, seed, p, perm)


def sorted_u32(n: int, seed: int) -> np.ndarray:
    """The uniform array, pre-sorted ascending while the input is prepared."""
    return np.sort(uniform_u32(n, seed))


def equal_u32(n: int, seed: int) -> np.ndarray:
    """Every key equal to the stream's first draw."""
    return np.full(n, draws32(seed, 1)[0], dtype=np.uint32)


DISTRIBUTIONS_U32 = {
    "uniform": uniform_u32,
    "gaussian": gaussian_u32,
    "bucket": bucket_u32,
    "staggered": staggered_u32,
    "sorted": sorted_u32,
    "equal": equal_u32,
}


def make_u32(dist: str, n: int, seed: int) -> np.ndarray:
    return DISTRIBUTIONS_U32[dist](n, seed)


# --------------------------------------------------------------------------- uint64 keys

def uniform_u64(n: int, seed: int) -> np.ndarray:
    """i.i.d. uniform over [0, 2^64)."""
    return draws64(seed, n)


def zipf_u64(n: int, seed: int, s: float = 1.1, distinct: int = 1 << 20) -> np.ndarray:
    """Zipf(s) over ``distinct`` ranks by inverse CDF; rank k becomes key mix64(k).

    The finaliser is a bijection on 64-bit words, so the key multiset has exactly the rank
    multiset's tie structure while its values are spread over the whole key range.
    """
    k = np.arange(1, distinct + 1, dtype=np.float64)
    cdf = np.cumsum(k ** (-s))
    cdf /= cdf[-1]
    out = np.empty(n, dtype=np.uint64)
    for c0 in range(0, n, _CHUNK):
        c1 = min(n, c0 + _CHUNK)
        u = _unit_double(draws64(seed, c1 - c0, c0))
        rank = np.minimum(np.searchsorted(cdf, u, side="right"), distinct - 1) + 1
        out[c0:c1] = mix64(rank.astype(np.uint64))
    return out


def index_values(n: int) -> np.ndarray:
    """Values for key/value workloads: the input index of each item."""
    return np.arange(n, dtype=np.uint32)


# --------------------------------------------------------------------------- segmented f32

def segment_sizes(count: int, seed: int, lo_log2: int = 8, hi_log2: int = 20) -> np.ndarray:
    """``count`` sizes floor(2^(lo + (hi-lo)*U)), U uniform in [0, 1)."""
    u = _unit_double(draws64(seed, count))
    return np.floor(np.exp2(lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def normal_f32_segments(sizes, seed: int, dup_frac: float = 0.01,
                        zero_log2: int = 10) -> np.ndarray:
    """Concatenated float32 segments drawn N(0,1) by Box-Muller (in double, rounded to f32).

    Inside each segment, floor(dup_frac * size) positions are overwritten with copies of other
    positions of the same segment (exact duplicates), and every item independently becomes
    +0.0 or -0.0 (50/50) with probability 2^-zero_log2.  Returned as float32.
    """
    sizes = np.asarray(sizes, dtype=np.int64)
    total = int(sizes.sum())
    out = np.empty(total, dtype=np.float32)
    cursor = 0
    draw = 0
    for size in sizes.tolist():
        d = draws64(seed, 2 * size, draw)
        draw += 2 * size
        u1 = 1.0 - _unit_double(d[0::2])  # (0, 1]
        u2 = _unit_double(d[1::2])
        seg = (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).astype(np.float32)
        ndup = int(dup_frac * size)
        if ndup:
            e = draws64(seed, 2 * ndup, draw)
            draw += 2 * ndup
            dst = (e[0::2] % np.uint64(size)).astype(np.int64)
            src = (e[1::2] % np.uint64(size)).astype(np.int64)
            for a, b in zip(dst.tolist(), src.tolist()):
                seg[a] = seg[b]
        z = draws64(seed, size, draw)
        draw += size
        hit = (z >> np.uint64(64 - zero_log2)) == np.uint64(0)
        neg = (z & np.uint64(1)) == np.uint64(1)
        seg[hit & ~neg] = np.float32(0.0)
        seg[hit & neg] = np.float32(-0.0)
        out[cursor:cursor + size] = seg
        cursor += size
    return out
