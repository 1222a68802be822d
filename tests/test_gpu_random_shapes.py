"""Seeded random shapes through every engine, against the FP64 oracle.

The fixed cases of the other GPU tests pick shapes with a purpose (ragged tiles, imbalanced
classes, planted tuples).  These draw the shape itself -- object and variable counts across tile
and padding boundaries, class balance, class count, discretisations, pseudocount, range -- from a
fixed seed, for each tuple size and each engine that takes it, so that a case nobody thought of
still meets the oracle.  Pure-noise data: many near-equal gains, so the tie rule is exercised."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_1811_00631_amd import workloads

from test_gpu_k2 import assert_ig_parity, to_dev

pytestmark = pytest.mark.gpu

# (k, engines, largest n_var the oracle finishes quickly, divisions allowed)
KINDS = [
    (2, ("auto", "mfma", "mfma_fp4"), 300, (1, 2, 4)),
    (3, ("auto", "bitset"), 80, (1, 2, 4)),
    (3, ("mfma_fp4",), 140, (1, 2)),
    (4, ("auto", "bitset"), 24, (1, 2)),
    (4, ("hist",), 16, (1, 2, 4)),
    (5, ("auto", "bitset"), 14, (1,)),
    (5, ("hist",), 11, (1, 2)),
]


def _cases():
    g = np.random.default_rng(20261203)
    out = []
    for kind, (k, engines, pmax, divs) in enumerate(KINDS):
        for rep in range(5):
            n_obj = int(g.integers(k + 6, 700))
            n_var = int(g.integers(k, pmax + 1))
            ones = int(g.integers(1, n_obj))
            div = int(g.choice(divs))
            n_disc = int(g.integers(1, 4))
            xi = float(g.choice([0.1, 0.25, 1.0]))
            rng = float(g.choice([0.0, 0.5, 1.0]))
            seed = int(g.integers(0, 2**31))
            engine = engines[rep % len(engines)]
            out.append((f"k{k}_{engine}_{rep}", k, engine, n_obj, n_var, ones, div, n_disc, xi, rng, seed))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_random_shape_matches_oracle(mdfs_gpu, case):
    name, k, engine, n_obj, n_var, ones, div, n_disc, xi, rng, seed = case
    if min(ones, n_obj - ones) == 0:
        pytest.skip("one class empty")
    w = dataclasses.replace(workloads.null_data(seed, n_obj, n_var, ones=ones), divisions=div, n_disc=n_disc,
                            xi=xi, range_=rng, seed=seed)
    print(f"random {name}: N={n_obj} p={n_var} ones={ones} d={div + 1} R={n_disc} xi={xi} range={rng} "
          f"seed={seed}", flush=True)
    data, y = to_dev(w)
    got = mdfs_gpu.mdfs_max_ig(data, y, k, div, n_disc, xi, rng, seed, 0, engine=engine)
    torch.cuda.synchronize()
    got = [t.cpu().numpy() for t in got]
    ref = oracle.max_ig_all(w.data, w.y, k, div, n_disc, rng, xi, seed, n_threads=8)
    assert_ig_parity(*got, ref, name)


# The bitset engines keep EA, EB and the (L, Q) pairs (16 N bytes) at the start of their LDS
# array and address them by byte offsets of the counts; near the largest object count whose
# tables fit in LDS (the pair sweep's int8 layout bounds N at about 7000) those offsets are
# largest.  Unbalanced classes, so that both per-class tables are long.
LARGE_N = [(3, 4, 8), (4, 1, 9), (4, 2, 8), (5, 1, 8)]


@pytest.mark.parametrize("k,div,n_var", LARGE_N, ids=[f"k{k}_d{d + 1}" for k, d, _ in LARGE_N])
def test_bitset_engines_at_large_n(mdfs_gpu, k, div, n_var):
    n_obj, ones = 6800, 2900
    w = dataclasses.replace(workloads.null_data(77 + k + div, n_obj, n_var, ones=ones), divisions=div, n_disc=1,
                            xi=0.25, range_=0.5, seed=77)
    print(f"large N k={k} d={div + 1} N={n_obj} p={n_var} ones={ones}", flush=True)
    data, y = to_dev(w)
    got = mdfs_gpu.mdfs_max_ig(data, y, k, div, 1, 0.25, 0.5, 77, 0, engine="bitset")
    torch.cuda.synchronize()
    got = [t.cpu().numpy() for t in got]
    ref = oracle.max_ig_all(w.data, w.y, k, div, 1, 0.5, 0.25, 77, n_threads=8)
    assert_ig_parity(*got, ref, f"large N k={k} d={div + 1}")
