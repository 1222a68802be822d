"""Autotuner for the sweep's launch configuration.

The tunables are the count engine (k = 2: fp4 or int8 one-hot on the matrix cores; k = 3: the
matrix-core engine or bitsets; k = 4 and 5: bitsets or per-tuple histograms), the persistent grid size
(workgroups) and, for k = 2, the launch shape of the pair sweep: the super-tile side (how many
tiles' operand panels the workgroups of one XCD share in its L2: 4, 8 or 16 tiles a side) and,
with three classes, 4 or 8 waves per workgroup (64 x 64 or 64 x 32 outputs per wave).  None of
them changes any result (every call is deterministic and every grid takes all tiles), so the
tuner only times: for a problem shape it runs each valid candidate on seeded synthetic data of
that shape, takes the sweep phase time from the library's HIP events, and keeps the fastest.
Results are cached per shape bucket (N and p rounded up to powers of two, k, d, discretisations
up to 4) in memory and, if a path is given, in a JSON file.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import mdfs

GRIDS = (128, 256, 512, 1024)
SUPERTILES = (4, 8, 16)


def bucket(n_obj: int, n_var: int, k: int, divisions: int, n_disc: int) -> tuple:
    p2 = lambda x: 1 << max(0, math.ceil(math.log2(max(1, x))))
    return (p2(n_obj), p2(n_var), k, divisions, min(n_disc, 4))


def candidates(n_obj: int, k: int, divisions: int, ones: int) -> list[dict]:
    """Valid launch configurations for the shape (keyword arguments of mdfs_max_ig);
    `ones` = objects of class 1."""
    small_classes = max(ones, n_obj - ones) < 4096
    if k == 1:
        return [{"engine": "auto", "workgroups": 0, "tile": 0}]
    if k == 2:
        engines = (["mfma_fp4"] if small_classes else []) + ["mfma"]
        waves = (8, 4) if divisions == 2 else (0,)
        return [{"engine": e, "workgroups": g, "tile": mdfs.tile_code(sb, nw)}
                for e in engines for g in GRIDS for sb in SUPERTILES for nw in waves]
    if k == 3:
        engines = (["mfma_fp4"] if small_classes and divisions in (1, 2) else []) + ["bitset"]
    elif k == 4:
        engines = (["bitset"] if divisions <= 2 else []) + ["hist"]
    else:
        engines = (["bitset"] if divisions == 1 else []) + ["hist"]
    return [{"engine": e, "workgroups": g, "tile": 0} for e in engines for g in GRIDS]


class Tuner:
    def __init__(self, path: str | None = None, device: str = "cuda:0", reps: int = 2):
        self.path = path
        self.device = device
        self.reps = reps
        self.cache: dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)

    def _save(self):
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)

    def best(self, n_obj: int, n_var: int, k: int, divisions: int, n_disc: int) -> dict:
        key = json.dumps(bucket(n_obj, n_var, k, divisions, n_disc))
        if key not in self.cache:
            self.cache[key] = self.tune(n_obj, n_var, k, divisions, n_disc)
            self._save()
        return self.cache[key]

    def tune(self, n_obj: int, n_var: int, k: int, divisions: int, n_disc: int) -> dict:
        import torch

        g = np.random.default_rng(12345)
        n_disc = min(n_disc, 4)
        X = torch.from_numpy(g.standard_normal((n_var, n_obj)).astype(np.float32)).to(self.device)
        yv = np.zeros(n_obj, dtype=np.uint8)
        yv[: n_obj // 2] = 1
        y = torch.from_numpy(g.permutation(yv)).to(self.device)
        timings = []
        for cand in candidates(n_obj, k, divisions, int(yv.sum())):
            ms = []
            try:
                for rep in range(self.reps + 1):
                    mdfs.mdfs_max_ig(X, y, k, divisions, n_disc, timing=True, **cand)
                    if rep:
                        ms.append(mdfs.mdfs_phase_times()["sweep"])
            except mdfs.MdfsError as e:
                if e.code != mdfs.E_LIMIT:   # only a size limit of an engine is a skipped candidate
                    raise
                continue
            timings.append((float(np.median(ms)), cand))
        t, cand = min(timings, key=lambda x: x[0])
        return dict(cand, sweep_ms=t, tried=[dict(c, sweep_ms=m) for m, c in timings])
