"""Counter-based random numbers for the synthetic workloads.

This module is a pure input generator: it produces seeded random floats and
permutations and contains none of the transfer-entropy arithmetic.  Both the
CPU oracle tests and the GPU path draw their inputs from here, so the two
sides always see bit-identical series and surrogate permutations.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used in counter mode: the i-th output of the
stream with key K is mix64(K + (i + 1) * GAMMA).  Normals come from the
Box-Muller transform evaluated in float64 and rounded once to float32
(round-to-nearest-even), so the data do not depend on numpy's own generators.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK53 = np.uint64((1 << 53) - 1)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output mixing function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def derive_key(*ids: int) -> np.uint64:
    """Fold a tuple of non-negative integers into one 64-bit stream key."""
    k = np.uint64(0x5EED5EED5EED5EED)
    with np.errstate(over="ignore"):
        for v in ids:
            k = mix64(np.uint64(k) + GAMMA * np.uint64(int(v) & 0xFFFFFFFFFFFFFFFF) + np.uint64(1))
    return np.uint64(k)


def stream_u64(key, n: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+n-1 of the counter-mode SplitMix64 stream ``key``."""
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(key) + idx * GAMMA)


def uniform01(key, n: int, start: int = 0) -> np.ndarray:
    """float64 uniforms in [0, 1) from the top 53 bits of each output."""
    return (stream_u64(key, n, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal64(key, n: int) -> np.ndarray:
    """n standard normals in float64 (Box-Muller: pairs of uniforms -> pairs of normals)."""
    m = (n + 1) // 2
    u = uniform01(key, 2 * m)
    u1 = 1.0 - u[0::2]            # (0, 1]: log is finite
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    out = np.empty(2 * m, dtype=np.float64)
    out[0::2] = r * np.cos(th)
    out[1::2] = r * np.sin(th)
    return out[:n]


def bounded(key, n_draws: int, bounds: np.ndarray) -> np.ndarray:
    """Unbiased integers in [0, bounds[i]) (Lemire's multiply-shift with rejection).

    ``bounds`` has one entry per draw; outputs are consumed from the stream in
    order, rejected values being skipped, so the result depends only on the key.
    """
    bounds = np.asarray(bounds, dtype=np.uint64)
    out = np.empty(n_draws, dtype=np.int64)
    pos = 0
    todo = np.arange(n_draws)
    while todo.size:
        raw = stream_u64(key, todo.size, pos)
        pos += todo.size
        x = raw >> np.uint64(32)                      # 32-bit draw
        s = bounds[todo]
        m = x * s                                     # < 2**64 since s < 2**32
        lo = m & np.uint64(0xFFFFFFFF)
        thresh = (np.uint64(1 << 32) - s) % s
        ok = lo >= thresh
        out[todo[ok]] = (m[ok] >> np.uint64(32)).astype(np.int64)
        todo = todo[~ok]
    return out


def permutation(key, n: int) -> np.ndarray:
    """Uniform random permutation of 0..n-1 (Fisher-Yates, swaps i <-> j, j in [0, i])."""
    perm = np.arange(n, dtype=np.int32)
    if n < 2:
        return perm
    js = bounded(key, n - 1, np.arange(n, 1, -1, dtype=np.uint64))
    for step, i in enumerate(range(n - 1, 0, -1)):
        j = js[step]
        perm[i], perm[j] = perm[j], perm[i]
    return perm


def permutations(keys: list, n: int) -> np.ndarray:
    """One independent permutation of 0..n-1 per key, as an int32 [len(keys), n] array.

    Vectorised Fisher-Yates: all permutations swap position i at the same step.
    """
    s = len(keys)
    perm = np.tile(np.arange(n, dtype=np.int32), (s, 1))
    if n < 2 or s == 0:
        return perm
    bounds = np.arange(n, 1, -1, dtype=np.uint64)
    js = np.stack([bounded(k, n - 1, bounds) for k in keys])     # [s, n-1]
    rows = np.arange(s)
    for step, i in enumerate(range(n - 1, 0, -1)):
        j = js[:, step]
        a = perm[rows, i].copy()
        perm[rows, i] = perm[rows, j]
        perm[rows, j] = a
    return perm
