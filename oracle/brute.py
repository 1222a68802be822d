"""Tiny-input brute force of IG^k_max in pure Python (a second, independent oracle).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.  It re-derives every step from the
paper with Python integers, dictionaries and ``math.log``, sharing no code with
``mdfs_oracle.c``: the shares and cut positions of the randomised discretisation ("Algorithm and
implementation", the range/shares paragraph), per-class voxel counts of every k-subset (the
counters N^d), pseudocounted class probabilities p^d = (N^d_v + beta^d)/(N_v + beta^0 + beta^1)
with beta^d = xi N^d / min(N^0, N^1), the voxel-weighted conditional entropy N H(y|X) =
sum_v n_v h(p_v) in nats, and IG(i | m) = N (H(y|m) - H(y|i,m)) maximised over tuples and
discretisations (equation IGmax, section "Theory") with the tie rule of the readings list
(tau = 1e-9 max(1, |max|); smallest discretisation, then smallest tuple).

Meant for a few dozen objects and variables: it is slow by design.
"""
from __future__ import annotations

import itertools
import math

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _mix(z: int) -> int:
    # SplitMix64 output function (Steele, Lea & Flood 2014)
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def draw(seed: int, disc: int, var: int, j: int) -> int:
    """The counter-based draw keyed by (seed, discretisation, variable, share index)."""
    h = _mix((seed + GAMMA) & MASK)
    for c in (disc, var, j):
        h = _mix((h + (c + 1) * GAMMA) & MASK)
    return h


def cut_positions(n: int, c: int, rng: float, seed: int, disc: int, var: int) -> list[int]:
    """c shares from U(1-range, 1+range); c-1 strictly increasing 0-based cut positions."""
    shares = [(1.0 - rng) + (2.0 * rng) * ((draw(seed, disc, var, j) >> 11) * 2.0 ** -53) for j in range(c)]
    total = 0.0
    for s in shares:
        total += s
    cuts, acc = [], 0.0
    for j in range(1, c):
        acc += shares[j - 1]
        t = min(max(math.floor((n * acc) / total), 1), n - 1)
        if cuts:
            t = max(t, cuts[-1] + 1)
        cuts.append(min(t, n - (c - j)))
    return cuts


def codes_of(x, c: int, rng: float, seed: int, disc: int, var: int) -> list[int]:
    srt = sorted(float(v) for v in x)
    thr = [srt[t] for t in cut_positions(len(srt), c, rng, seed, disc, var)]
    return [sum(1 for v in thr if float(xv) >= v) for xv in x]


def _F(counts: dict, b0: float, b1: float) -> float:
    """sum over occupied voxels of n_v h(p_v), terms added in ascending order."""
    terms = []
    for n0, n1 in counts.values():
        nv = n0 + n1
        if nv == 0:
            continue
        den = n0 + b0 + n1 + b1
        h = 0.0
        for nd, bd in ((n0, b0), (n1, b1)):
            p = (nd + bd) / den
            if p > 0.0:
                h -= p * math.log(p)
        terms.append(nv * h)
    out = 0.0
    for t in sorted(terms):
        out += t
    return out


def _counts(cols, y, vars_) -> dict:
    tab: dict = {}
    for n, yn in enumerate(y):
        key = tuple(cols[v][n] for v in vars_)
        c0, c1 = tab.get(key, (0, 0))
        tab[key] = (c0 + (yn == 0), c1 + (yn == 1))
    return tab


def max_ig(data, y, k: int, divisions: int, n_disc: int, rng: float, xi: float, seed: int,
           disc_offset: int = 0):
    """Returns (ig [p], argmax [p][k-1], disc [p]) as Python lists."""
    y = [int(v) for v in y]
    n1 = sum(y)
    n0 = len(y) - n1
    m = min(n0, n1)
    b0, b1 = xi * n0 / m, xi * n1 / m
    p = len(data)
    c = divisions + 1
    cands = [[] for _ in range(p)]
    top = [-math.inf] * p
    for r in range(n_disc):
        q = disc_offset + r
        cols = [codes_of(data[v], c, rng, seed, q, v) for v in range(p)]
        for i in range(p):
            others = [v for v in range(p) if v != i]
            for mset in itertools.combinations(others, k - 1):
                g = _F(_counts(cols, y, mset), b0, b1) - _F(_counts(cols, y, sorted(mset + (i,))), b0, b1)
                cands[i].append((g, q, mset))
                top[i] = max(top[i], g)
    ig, am, ad = [], [], []
    for i in range(p):
        mx = top[i]
        tau = 1e-9 * max(1.0, abs(mx))
        tied = [(q, mset) for g, q, mset in cands[i] if g >= mx - tau]
        q, mset = min(tied)
        ig.append(mx)
        am.append(list(mset))
        ad.append(q)
    return ig, am, ad
