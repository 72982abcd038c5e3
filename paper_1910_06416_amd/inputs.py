"""Seeded synthetic key sets.

This module only draws random inputs; it holds none of the method's
arithmetic.  Every generator uses numpy's PCG64 bit generator with an explicit
seed, so the test-suite, the benchmark and the smoke check see identical keys.

The paper measures on random 128-bit keys and names no public data set; these
generators stand in for it with uniformly random 64-bit integers and random
printable-ASCII strings.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def u64_keys(n: int, seed: int) -> np.ndarray:
    """n distinct uniformly random 64-bit keys (first occurrences kept)."""
    rng = _rng(seed)
    keys = rng.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    while True:
        _, first = np.unique(keys, return_index=True)
        if len(first) == len(keys):
            return keys
        keep = np.sort(first)
        extra = rng.integers(0, 2**64, size=n - len(keep), dtype=np.uint64, endpoint=False)
        keys = np.concatenate([keys[keep], extra])


def u64_keys_raw(n: int, seed: int) -> np.ndarray:
    """n uniformly random 64-bit keys without the distinctness pass (for
    10^9-key workloads, where that pass would sort 8 GB on the host; two of
    10^9 draws coincide with probability about 3%, so callers check)."""
    return _rng(seed).integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)


def ascii_keys(n: int, seed: int, min_len: int = 8, max_len: int = 32):
    """n distinct random strings of printable ASCII (0x21..0x7e), lengths
    uniform in [min_len, max_len] (max_len < 65536).  Returns (data uint8[],
    offsets uint64[n+1])."""
    assert 0 <= min_len <= max_len < 65536
    rng = _rng(seed)
    lens_all = np.zeros(0, dtype=np.int64)
    chars_all = np.zeros((0, max_len), dtype=np.uint8)
    while len(lens_all) < n:
        need = n - len(lens_all)
        lens = rng.integers(min_len, max_len + 1, size=need, dtype=np.int64)
        chars = rng.integers(0x21, 0x7F, size=(need, max_len), dtype=np.uint8)
        chars[np.arange(max_len)[None, :] >= lens[:, None]] = 0
        lens_all = np.concatenate([lens_all, lens])
        chars_all = np.concatenate([chars_all, chars])
        # distinct strings, first occurrences kept in draw order (the length is
        # part of the row: trailing zero bytes belong to no string)
        rows = np.concatenate([lens_all.astype("<u2").view(np.uint8).reshape(-1, 2), chars_all], axis=1)
        view = np.ascontiguousarray(rows).view(np.dtype((np.void, max_len + 2))).ravel()
        _, first = np.unique(view, return_index=True)
        keep = np.sort(first)
        lens_all, chars_all = lens_all[keep], chars_all[keep]
    lens = lens_all[:n].astype(np.uint64)
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    mask = np.arange(max_len)[None, :] < lens[:, None].astype(np.int64)
    data = chars_all[:n][mask]
    return np.ascontiguousarray(data, dtype=np.uint8), offsets


def permutation(n: int, seed: int) -> np.ndarray:
    """A uniformly random permutation of range(n) (lookup order)."""
    return _rng(seed).permutation(n).astype(np.int64)


def gather_strings(keys, order: np.ndarray):
    """Reorder a (data, offsets) string set by an index array."""
    data, offsets = keys
    lens = (offsets[1:] - offsets[:-1]).astype(np.int64)[order]
    starts = offsets[:-1].astype(np.int64)[order]
    new_off = np.zeros(len(order) + 1, dtype=np.uint64)
    np.cumsum(lens, out=new_off[1:])
    idx = np.repeat(starts - new_off[:-1].astype(np.int64), lens) + np.arange(int(new_off[-1]), dtype=np.int64)
    return np.ascontiguousarray(data[idx]), new_off


def log_uniform_sizes(count: int, seed: int, lo: float, hi: float) -> np.ndarray:
    """count integer sizes floor(exp(U(ln lo, ln hi))) (batched/served builds)."""
    u = _rng(seed).random(count)
    return np.floor(np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))).astype(np.int64)
