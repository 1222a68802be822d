"""Seeded synthetic inputs shaped like the paper's workloads.

This module draws data only: it holds none of the method's arithmetic (no discretisation, no
counting, no entropy), so the oracle and the HIP path can both be fed from it.

The paper evaluates on Madelon (2000 objects, 500 variables: 5 base variables feeding a random
parity decision, 15 linear combinations of them, 480 noise variables; section "Madelon example"),
which is not available here.  The generators below stand in for it and for the larger
genomics-shaped sizes the method targets.  All data is float32, variable-major [n_var][n_obj];
the decision is uint8 in {0, 1}.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    data: np.ndarray              # float32 [n_var][n_obj]
    y: np.ndarray                 # uint8 [n_obj]
    k: int
    divisions: int
    n_disc: int
    range_: float
    xi: float
    seed: int
    planted: dict                 # what was planted and where

    @property
    def n_var(self) -> int:
        return self.data.shape[0]

    @property
    def n_obj(self) -> int:
        return self.data.shape[1]


def xor_small(seed: int = 1, n_obj: int = 500, n_var: int = 100, noise: float = 0.1,
              divisions: int = 2, n_disc: int = 1) -> Workload:
    """Gaussian variables; variables 0 and 1 planted as an XOR pair: y = [x0>0] xor [x1>0],
    each label flipped with probability `noise`."""
    g = np.random.default_rng(seed)
    X = g.standard_normal((n_var, n_obj)).astype(np.float32)
    y = ((X[0] > 0) ^ (X[1] > 0)).astype(np.uint8)
    flip = g.random(n_obj) < noise
    y = (y ^ flip).astype(np.uint8)
    return Workload("xor_small", X, y, 2, divisions, n_disc, 0.5, 0.25, seed,
                    {"xor_pair": [0, 1]})


def madelon_like(seed: int = 2, n_obj: int = 2000, n_base: int = 5, n_comb: int = 15,
                 n_noise: int = 480, divisions: int = 2, n_disc: int = 30, k: int = 2) -> Workload:
    """Madelon-shaped: a latent hypercube vertex z in {-1,+1}^5 per object; base features
    z + 0.5*eps (bimodal); y = a balanced random labelling of the 32 vertices (a random parity
    function); 15 random linear combinations of the base features; Gaussian noise features;
    columns shuffled, positions recorded."""
    g = np.random.default_rng(seed)
    z = g.choice([-1.0, 1.0], size=(n_obj, n_base))
    base = z + 0.5 * g.standard_normal((n_obj, n_base))
    verts = 1 << n_base
    lab = np.zeros(verts, dtype=np.uint8)
    lab[g.permutation(verts)[: verts // 2]] = 1
    vid = ((z > 0).astype(np.int64) * (1 << np.arange(n_base))).sum(axis=1)
    y = lab[vid]
    A = g.standard_normal((n_base, n_comb))
    comb = base @ A
    noise = g.standard_normal((n_obj, n_noise))
    cols = np.concatenate([base, comb, noise], axis=1)
    perm = g.permutation(cols.shape[1])
    X = cols[:, perm].T.astype(np.float32).copy()
    where = np.argsort(perm)
    return Workload("madelon_like", X, y.astype(np.uint8), k, divisions, n_disc, 0.5, 0.25, seed,
                    {"base": sorted(where[:n_base].tolist()),
                     "comb": sorted(where[n_base:n_base + n_comb].tolist())})


def parity3(seed: int = 3, n_obj: int = 2000, n_var: int = 500, divisions: int = 2,
            n_disc: int = 30) -> Workload:
    """Gaussian variables; y = [x0>0] xor [x1>0] xor [x2>0] (no label noise): invisible to pairs,
    visible to triples."""
    g = np.random.default_rng(seed)
    X = g.standard_normal((n_var, n_obj)).astype(np.float32)
    y = ((X[0] > 0) ^ (X[1] > 0) ^ (X[2] > 0)).astype(np.uint8)
    return Workload("parity3", X, y, 3, divisions, n_disc, 0.5, 0.25, seed, {"triple": [0, 1, 2]})


def genomics_like(seed: int = 4, n_obj: int = 500, n_var: int = 20000, n_pairs: int = 10,
                  n_ones: int | None = 200, noise: float = 0.1, divisions: int = 2,
                  n_disc: int = 30) -> Workload:
    """Expression-like: log-normal(0,1) variables; y with exactly `n_ones` ones, shuffled
    (balanced when None); `n_pairs` planted XOR pairs at seeded positions.  For a pair (a, b):
    s_a = +-1 uniform, s_b = s_a*(1-2y) flipped with probability `noise`, x = exp(|g| s),
    g ~ N(0,1), so each planted variable is marginally log-normal(0,1) and independent of y."""
    g = np.random.default_rng(seed)
    X = np.exp(g.standard_normal((n_var, n_obj))).astype(np.float32)
    ones = n_obj // 2 if n_ones is None else n_ones
    y = np.zeros(n_obj, dtype=np.uint8)
    y[:ones] = 1
    y = y[g.permutation(n_obj)]
    pos = g.choice(n_var, size=2 * n_pairs, replace=False)
    pairs = []
    for q in range(n_pairs):
        a, b = int(pos[2 * q]), int(pos[2 * q + 1])
        sa = g.choice([-1.0, 1.0], size=n_obj)
        sb = sa * (1.0 - 2.0 * y)
        flip = g.random(n_obj) < noise
        sb = np.where(flip, -sb, sb)
        X[a] = np.exp(np.abs(g.standard_normal(n_obj)) * sa)
        X[b] = np.exp(np.abs(g.standard_normal(n_obj)) * sb)
        pairs.append(sorted((a, b)))
    return Workload("genomics_like", X, y, 2, divisions, n_disc, 0.5, 0.25, seed, {"pairs": pairs})


def headline(seed: int = 5) -> Workload:
    """The throughput workload: k=2, N=2000 objects, p=20000 log-normal variables with 10
    planted XOR pairs, balanced y, d=3 classes, 30 random discretisations."""
    w = genomics_like(seed=seed, n_obj=2000, n_var=20000, n_pairs=10, n_ones=None)
    w.name = "headline"
    return w


def null_data(seed: int, n_obj: int, n_var: int, ones: int | None = None) -> Workload:
    """Pure noise (no planted signal), for null-distribution checks."""
    g = np.random.default_rng(seed)
    X = g.standard_normal((n_var, n_obj)).astype(np.float32)
    m = n_obj // 2 if ones is None else ones
    y = np.zeros(n_obj, dtype=np.uint8)
    y[:m] = 1
    y = y[g.permutation(n_obj)]
    return Workload("null", X, y, 2, 2, 1, 0.5, 0.25, seed, {})


WORKLOADS = {
    "xor_small": xor_small,
    "madelon_like": madelon_like,
    "parity3": parity3,
    "genomics_like": genomics_like,
    "headline": headline,
}


def serving_datasets(seed: int = 6, n_datasets: int = 32, n_range=(100, 5000), p_range=(100, 20000),
                     k3_max_vars: int = 1000):
    """Datasets of the serving trace: N and p log-uniform in the given ranges, Gaussian
    variables, y balanced in expectation from one planted XOR pair [x_a>0] xor [x_b>0] (10%
    label noise); datasets with p <= k3_max_vars also carry a second, exact XOR pair.  Every
    other dataset is capped at k3_max_vars variables so that k = 3 requests exist."""
    g = np.random.default_rng(seed)
    out = []
    for t in range(n_datasets):
        n = int(round(np.exp(g.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        p_hi = p_range[1] if t % 2 == 0 else min(p_range[1], k3_max_vars)
        p = int(round(np.exp(g.uniform(np.log(p_range[0]), np.log(p_hi)))))
        X = g.standard_normal((p, n)).astype(np.float32)
        a, b = (int(v) for v in g.choice(p, size=2, replace=False))
        y = ((X[a] > 0) ^ (X[b] > 0)).astype(np.uint8)
        y ^= (g.random(n) < 0.1).astype(np.uint8)
        if y.min() == y.max():
            y[0] ^= 1
        pairs = [sorted((a, b))]
        if p <= k3_max_vars and p >= 4:
            c, d = (int(v) for v in g.choice(np.setdiff1d(np.arange(p), [a, b]), size=2, replace=False))
            X[d] = np.abs(X[d]) * np.where((X[c] > 0) ^ (y > 0), 1.0, -1.0).astype(np.float32)
            pairs.append(sorted((c, d)))
        out.append((X, y, {"pairs": pairs}))
    return out


def serving_requests(datasets, seed: int = 6, n_requests: int = 256, rate_hz: float = 1.0,
                     k3_max_vars: int = 1000):
    """Request parameters of the serving trace: dataset uniform, k in {2, 3} (k = 3 only on
    datasets with at most k3_max_vars variables), divisions in {1, 2, 4}, 1..30 discretisations,
    Poisson arrivals at rate_hz.  Returns dicts (dataset, k, divisions, n_disc, seed, arrival)."""
    g = np.random.default_rng(seed + 1000)
    t = 0.0
    reqs = []
    for i in range(n_requests):
        t += g.exponential(1.0 / rate_hz)
        ds = int(g.integers(len(datasets)))
        p = datasets[ds][0].shape[0]
        k = int(g.choice([2, 3])) if p <= k3_max_vars else 2
        reqs.append({"dataset": ds, "k": k, "divisions": int(g.choice([1, 2, 4])),
                     "n_disc": int(g.integers(1, 31)), "seed": int(g.integers(1 << 31)), "arrival": t})
    return reqs
