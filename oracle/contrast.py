"""Contrast variables, written plainly (oracle side; TEST INFRASTRUCTURE ONLY).

AddContrastVariables (section "Package functions introduction") is cited, not defined, by the
paper.  The reading shared with the library's documentation: contrast variable c copies original
variable src(c) = draw(seed, c, 0x5352434) mod n_var, its objects permuted by a keyed 4-round
Feistel network on 2h-bit indices (2^(2h) >= n_obj) whose round r computes
F = fin(key_r + R) mod 2^h, (L, R) <- (R, L xor F), with key_r = draw(seed, c, r); an index that
lands at or beyond n_obj is mapped again until it falls below n_obj.  draw() absorbs its three
key components into SplitMix64 (Steele, Lea & Flood 2014), one finaliser step each.
"""
from __future__ import annotations

import numpy as np

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def fin(z: int) -> int:
    """SplitMix64 output function."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def draw(seed: int, a: int, b: int) -> int:
    h = fin(seed + GAMMA)
    h = fin(h + (a + 1) * GAMMA)
    return fin(h + (b + 1) * GAMMA)


def source(seed: int, c: int, n_var: int) -> int:
    return draw(seed, c, 0x5352434) % n_var


def permutation(seed: int, c: int, n_obj: int) -> np.ndarray:
    """perm[n] for n in [0, n_obj): the object contrast variable c takes at position n."""
    h = 1
    while (1 << (2 * h)) < n_obj:
        h += 1
    mask = (1 << h) - 1
    keys = [draw(seed, c, r) for r in range(4)]

    def feistel(x: int) -> int:
        left, right = x >> h, x & mask
        for r in range(4):
            f = fin(keys[r] + right) & mask
            left, right = right, left ^ f
        return (left << h) | right

    out = np.empty(n_obj, dtype=np.int64)
    for n in range(n_obj):
        j = feistel(n)
        while j >= n_obj:
            j = feistel(j)
        out[n] = j
    return out


def add_contrast(data: np.ndarray, n_contrast: int, seed: int):
    """The originals followed by the contrast variables, and each contrast variable's source."""
    n_var, n_obj = data.shape
    out = np.empty((n_var + n_contrast, n_obj), dtype=data.dtype)
    out[:n_var] = data
    src = np.empty(n_contrast, dtype=np.int64)
    for c in range(n_contrast):
        src[c] = source(seed, c, n_var)
        out[n_var + c] = data[src[c]][permutation(seed, c, n_obj)]
    return out, src
