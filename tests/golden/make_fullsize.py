"""Write the oracle's IG^k_max of every variable of the full-size workloads.

Run from the repository root:  python tests/golden/make_fullsize.py [name ...] [--threads T]

Each output file tests/golden/fullsize_<name>.npz holds, for every variable, the FP64 oracle's
IG_max, argmax tuple and argmax discretisation (oracle.max_ig_all, the tuple-sweep form of
equation IGmax), together with the workload parameters and a SHA-256 of the generated data and
decision, so a test can tell whether the seeded generator reproduced the same inputs.  Only the
oracle and the seeded input generators are called; nothing comes from the HIP path.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1811_00631_amd import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# name -> (generator, k); sizes are those of the benchmark workloads
FULLSIZE = {
    "madelon_like": (lambda: workloads.madelon_like(), 2),
    "madelon2_d2": (lambda: workloads.madelon_like(divisions=1, n_disc=30), 2),
    "parity3": (lambda: workloads.parity3(seed=3), 3),
    "madelon3_d2": (lambda: workloads.madelon_like(divisions=1, n_disc=30, k=3), 3),
    "genomics_like": (lambda: workloads.genomics_like(seed=4), 2),
    "headline": (lambda: workloads.headline(), 2),
}


def data_digest(w) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(w.data, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(w.y, dtype=np.uint8).tobytes())
    return h.hexdigest()


def path_of(name: str) -> str:
    return os.path.join(HERE, f"fullsize_{name}.npz")


def make(name: str, threads: int) -> None:
    gen, k = FULLSIZE[name]
    w = gen()
    t0 = time.time()
    ig, am, ad = oracle.max_ig_all(w.data, w.y, k, w.divisions, w.n_disc, w.range_, w.xi, w.seed,
                                   n_threads=threads)
    dt = time.time() - t0
    np.savez_compressed(path_of(name), ig=ig, argmax=am.astype(np.int32), disc=ad.astype(np.int32),
                        k=np.int32(k), divisions=np.int32(w.divisions), n_disc=np.int32(w.n_disc),
                        range_=np.float64(w.range_), xi=np.float64(w.xi), seed=np.int64(w.seed),
                        digest=np.array(data_digest(w)))
    print(f"{name}: N={w.n_obj} p={w.n_var} k={k} R={w.n_disc}: {dt:.0f} s on {threads} threads", flush=True)


def load(name: str) -> dict:
    with np.load(path_of(name), allow_pickle=False) as z:
        return {key: z[key] for key in z.files}


if __name__ == "__main__":
    args = sys.argv[1:]
    threads = 6
    if "--threads" in args:
        i = args.index("--threads")
        threads = int(args[i + 1])
        del args[i:i + 2]
    for name in args or list(FULLSIZE):
        make(name, threads)
