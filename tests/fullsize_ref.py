"""Oracle references of the full-size workloads for the GPU parity tests.

The FP64 oracle's IG^k_max of every variable of each full-size workload is stored under
tests/golden/fullsize_<name>.npz by tests/golden/make_fullsize.py (which calls only the oracle
and the seeded generators).  `reference` returns those values for every variable when the
regenerated inputs hash to the stored digest; otherwise it falls back to the live per-variable
oracle on a sample that includes every planted variable.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_fullsize  # noqa: E402

import oracle  # noqa: E402


def planted_vars(w) -> list[int]:
    out = set()
    for key in ("pairs",):
        for pr in w.planted.get(key, []):
            out.update(int(v) for v in pr)
    for key in ("base", "comb", "triple", "xor_pair"):
        out.update(int(v) for v in w.planted.get(key, []))
    return sorted(out)


def workload(name: str):
    gen, k = make_fullsize.FULLSIZE[name]
    return gen(), k


def reference(name: str, w, k: int, n_sample: int = 64, threads: int = 16):
    """(targets, (ig, argmax, disc), complete) for workload `name` regenerated as `w`."""
    path = make_fullsize.path_of(name)
    if os.path.exists(path):
        z = make_fullsize.load(name)
        if str(z["digest"]) == make_fullsize.data_digest(w) and int(z["k"]) == k:
            tg = np.arange(w.n_var, dtype=np.int64)
            return tg, (z["ig"], z["argmax"].astype(np.int64), z["disc"].astype(np.int64)), True
        print(f"{name}: stored reference does not match the regenerated inputs; sampling the live oracle",
              flush=True)
    g = np.random.default_rng(0)
    planted = planted_vars(w)
    rest = np.setdiff1d(np.arange(w.n_var), planted)
    n_rand = max(0, min(len(rest), n_sample - len(planted)))
    tg = np.array(sorted(planted + g.choice(rest, n_rand, replace=False).tolist()), dtype=np.int64)
    ref = oracle.max_ig(w.data, w.y, k, w.divisions, w.n_disc, w.range_, w.xi, w.seed, targets=tg,
                        n_threads=threads)
    return tg, ref, False
