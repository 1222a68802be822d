"""Plain FP64 CPU oracle of the MDFS k-tuple information-gain sweep.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the product path (``paper_1811_00631_amd``) never does.
It shares no code with the HIP implementation.

The arithmetic lives in ``mdfs_oracle.c`` (plain loops, IEEE binary64, no contraction); this
module only marshals numpy arrays through ctypes.  Every function follows the paper
"MDFS - MultiDimensional Feature Selection":

* ``discretize`` -- randomised rank-based discretisation ("Algorithm and implementation",
  the range/shares paragraph), one per discretisation index;
* ``table`` -- per-class voxel counts N^d of one k-tuple (same section);
* ``betas`` / ``F`` -- pseudocounts beta^d = xi N^d / min(N^0, N^1) and F = N*H(y|X) with
  pseudocounted voxel probabilities (the p^d and beta^d equations), natural log, voxel-weighted;
* ``max_ig`` -- IG^k_max(y; x_i) for chosen targets, straight from equation IGmax ("Theory");
* ``max_ig_all`` -- the same for every variable, organised as the tuple sweep.

``cuts`` and ``draw`` expose the readings of the discretisation that the paper leaves open.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdfs_oracle.c")
_LIB = os.path.join(_HERE, "libmdfs_oracle.so")

ERRORS = {0: "ok", -1: "bad argument", -2: "decision not binary or a class is empty",
          -3: "bad k", -4: "bad divisions", -5: "NaN in data", -6: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64, u64, dbl, ip = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
        L.mdfs_oracle_splitmix64_next.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        L.mdfs_oracle_splitmix64_next.restype = u64
        L.mdfs_oracle_draw.argtypes = [u64, i64, i64, i64]
        L.mdfs_oracle_draw.restype = u64
        L.mdfs_oracle_cuts.argtypes = [i64, ctypes.c_int, dbl, u64, i64, i64, ip]
        L.mdfs_oracle_discretize.argtypes = [ip, i64, i64, ctypes.c_int, i64, i64, dbl, u64, ip]
        L.mdfs_oracle_table.argtypes = [ip, ip, i64, ctypes.c_int, ctypes.c_int, ip, ip]
        L.mdfs_oracle_betas.argtypes = [ip, i64, dbl, ip, ip]
        L.mdfs_oracle_F.argtypes = [ip, i64, dbl, dbl]
        L.mdfs_oracle_F.restype = dbl
        L.mdfs_oracle_ig_member.argtypes = [ip, ip, i64, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int,
                                            dbl, dbl]
        L.mdfs_oracle_ig_member.restype = dbl
        L.mdfs_oracle_max_ig.argtypes = [ip, ip, i64, i64, ctypes.c_int, ctypes.c_int, i64, i64, dbl, dbl,
                                         u64, ip, i64, ip, ip, ip, ctypes.c_int]
        L.mdfs_oracle_max_ig_all.argtypes = [ip, ip, i64, i64, ctypes.c_int, ctypes.c_int, i64, i64, dbl,
                                             dbl, u64, ip, ip, ip, ctypes.c_int]
        L.mdfs_oracle_max_threads.restype = ctypes.c_int
        L.mdfs_oracle_interesting.argtypes = [ip, ip, i64, i64, ctypes.c_int, ctypes.c_int, i64, i64, dbl, dbl,
                                              u64, dbl, i64, ip, ip, ip, ip]
        L.mdfs_oracle_interesting.restype = i64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _chk(rc: int):
    if rc != 0:
        raise OracleError(rc)


def splitmix64(state: int, n: int):
    """First n outputs of the sequential SplitMix64 generator from `state`."""
    s = ctypes.c_uint64(state)
    return [lib().mdfs_oracle_splitmix64_next(ctypes.byref(s)) for _ in range(n)]


def draw(seed: int, disc: int, var: int, j: int) -> int:
    return lib().mdfs_oracle_draw(seed, disc, var, j)


def cuts(n_obj: int, divisions: int, rng: float, seed: int, disc: int, var: int) -> np.ndarray:
    t = np.zeros(divisions, dtype=np.int64)
    _chk(lib().mdfs_oracle_cuts(n_obj, divisions + 1, rng, seed, disc, var, _p(t)))
    return t


def discretize(data: np.ndarray, divisions: int, n_disc: int, rng: float, seed: int,
               disc_offset: int = 0) -> np.ndarray:
    """data: float32 [n_var][n_obj] -> codes uint8 [n_disc][n_var][n_obj]."""
    data = np.ascontiguousarray(data, dtype=np.float32)
    n_var, n_obj = data.shape
    codes = np.zeros((n_disc, n_var, n_obj), dtype=np.uint8)
    _chk(lib().mdfs_oracle_discretize(_p(data), n_obj, n_var, divisions, n_disc, disc_offset, rng,
                                      seed, _p(codes)))
    return codes


def table(codes_r: np.ndarray, y: np.ndarray, c: int, vars_) -> np.ndarray:
    """Per-class counts [2][c]*k of the tuple `vars_` from one discretisation's codes."""
    codes_r = np.ascontiguousarray(codes_r, dtype=np.uint8)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    v = np.ascontiguousarray(vars_, dtype=np.int64)
    k = len(v)
    t = np.zeros((2,) + (c,) * k, dtype=np.int64)
    _chk(lib().mdfs_oracle_table(_p(codes_r), _p(y), codes_r.shape[1], c, k, _p(v), _p(t)))
    return t


def betas(y: np.ndarray, xi: float):
    y = np.ascontiguousarray(y, dtype=np.uint8)
    b0, b1 = ctypes.c_double(), ctypes.c_double()
    _chk(lib().mdfs_oracle_betas(_p(y), len(y), xi, ctypes.byref(b0), ctypes.byref(b1)))
    return b0.value, b1.value


def F(tab: np.ndarray, beta0: float, beta1: float) -> float:
    """N * conditional entropy of a [2][...] count table (pseudocounted, nats)."""
    t = np.ascontiguousarray(tab, dtype=np.int64)
    ncell = t.size // 2
    return lib().mdfs_oracle_F(_p(t), ncell, beta0, beta1)


def ig_member(codes_r, y, c: int, vars_, member: int, beta0: float, beta1: float) -> float:
    """IG(vars_[member] | other members) under one discretisation."""
    codes_r = np.ascontiguousarray(codes_r, dtype=np.uint8)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    v = np.ascontiguousarray(vars_, dtype=np.int64)
    return lib().mdfs_oracle_ig_member(_p(codes_r), _p(y), codes_r.shape[1], c, len(v), _p(v),
                                       member, beta0, beta1)


def max_ig(data, y, k: int, divisions: int, n_disc: int, rng: float, xi: float, seed: int,
           targets=None, disc_offset: int = 0, n_threads: int = 1):
    """IG^k_max per target variable (equation IGmax).  Returns (ig f64, argmax i64 [t][k-1],
    argdisc i64)."""
    data = np.ascontiguousarray(data, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    n_var, n_obj = data.shape
    tg = np.arange(n_var, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, np.int64)
    nt = len(tg)
    ig = np.zeros(nt, dtype=np.float64)
    am = np.zeros((nt, max(k - 1, 1)), dtype=np.int64)
    ad = np.zeros(nt, dtype=np.int64)
    _chk(lib().mdfs_oracle_max_ig(_p(data), _p(y), n_obj, n_var, k, divisions, n_disc, disc_offset, rng,
                                  xi, seed, _p(tg), nt, _p(ig), _p(am), _p(ad), n_threads))
    return ig, am[:, :k - 1], ad


def max_ig_all(data, y, k: int, divisions: int, n_disc: int, rng: float, xi: float, seed: int,
               disc_offset: int = 0, n_threads: int = 1):
    """IG^k_max for every variable via the tuple sweep.  Same outputs as ``max_ig``."""
    data = np.ascontiguousarray(data, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    n_var, n_obj = data.shape
    ig = np.zeros(n_var, dtype=np.float64)
    am = np.zeros((n_var, max(k - 1, 1)), dtype=np.int64)
    ad = np.zeros(n_var, dtype=np.int64)
    _chk(lib().mdfs_oracle_max_ig_all(_p(data), _p(y), n_obj, n_var, k, divisions, n_disc, disc_offset,
                                      rng, xi, seed, _p(ig), _p(am), _p(ad), n_threads))
    return ig, am[:, :k - 1], ad


def interesting(data, y, k: int, divisions: int, n_disc: int, rng: float, xi: float, seed: int, ig_thr: float,
                disc_offset: int = 0, cap: int = 1 << 20):
    """ComputeInterestingTuples: every (variable, partner tuple, discretisation) with
    IG(variable | partners) >= ig_thr.  Returns (var [n], partners [n][k-1], disc [n], ig [n]) in
    the order discretisation, tuple (lexicographic), member."""
    data = np.ascontiguousarray(data, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    n_var, n_obj = data.shape
    var = np.zeros(cap, dtype=np.int64)
    part = np.zeros((cap, max(k - 1, 1)), dtype=np.int64)
    disc = np.zeros(cap, dtype=np.int64)
    igv = np.zeros(cap, dtype=np.float64)
    n = lib().mdfs_oracle_interesting(_p(data), _p(y), n_obj, n_var, k, divisions, n_disc, disc_offset, rng, xi,
                                      seed, float(ig_thr), cap, _p(var), _p(part), _p(disc), _p(igv))
    if n < 0:
        _chk(int(n))
    if n > cap:
        raise RuntimeError(f"{n} interesting tuples exceed the capacity {cap}")
    return var[:n], part[:n, :k - 1], disc[:n], igv[:n]


def max_threads() -> int:
    return lib().mdfs_oracle_max_threads()
