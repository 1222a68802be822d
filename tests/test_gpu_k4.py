"""k = 4 and k = 5 sweeps on the GPU through the C ABI, against the FP64 oracle: the bitset engines
(k = 4 with three classes: every cell counted directly; k = 4 and 5 with two classes: subset
counts and inclusion-exclusion) and the per-tuple histogram engine (k = 4 and 5, any class
count)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_1811_00631_amd import workloads

from test_gpu_k2 import assert_ig_parity, to_dev

pytestmark = pytest.mark.gpu


def run4(mdfs, w, n_disc=None, divisions=None, disc_offset=0, engine="auto", k=4):
    data, y = to_dev(w)
    out = mdfs.mdfs_max_ig(data, y, k, w.divisions if divisions is None else divisions,
                           w.n_disc if n_disc is None else n_disc, w.xi, w.range_, w.seed, disc_offset,
                           engine=engine)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


CASES4 = {
    "d3": lambda: workloads.xor_small(seed=61, n_obj=400, n_var=26, n_disc=2),
    "d2_imbalanced": lambda: dataclasses.replace(workloads.null_data(62, 333, 23, ones=90), divisions=1, n_disc=2),
    "d3_wide_words": lambda: workloads.xor_small(seed=63, n_obj=1100, n_var=17, n_disc=1),
    "four_vars": lambda: workloads.xor_small(seed=64, n_obj=200, n_var=4, n_disc=3),
    "tiny_n": lambda: workloads.xor_small(seed=65, n_obj=7, n_var=9, n_disc=2),
    "d2": lambda: dataclasses.replace(workloads.xor_small(seed=69, n_obj=700, n_var=31, n_disc=2), divisions=1),
    "d2_tiny_n": lambda: dataclasses.replace(workloads.xor_small(seed=60, n_obj=9, n_var=8, n_disc=2), divisions=1),
}


@pytest.mark.parametrize("name", list(CASES4))
def test_k4_matches_oracle(mdfs_gpu, name):
    w = CASES4[name]()
    print(f"k4 {name} N={w.n_obj} p={w.n_var} d={w.divisions + 1} R={w.n_disc}", flush=True)
    got = run4(mdfs_gpu, w)
    ref = oracle.max_ig_all(w.data, w.y, 4, w.divisions, w.n_disc, w.range_, w.xi, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, name)


def test_k4_finds_a_planted_parity_quadruple(mdfs_gpu):
    # y = xor of the signs of x0..x3: invisible to every triple, found by the quadruple sweep
    g = np.random.default_rng(66)
    n, p = 1200, 30
    X = g.standard_normal((p, n)).astype(np.float32)
    y = ((X[0] > 0) ^ (X[1] > 0) ^ (X[2] > 0) ^ (X[3] > 0)).astype(np.uint8)
    w = workloads.Workload("parity4", X, y, 2, 2, 1, 0.5, 0.25, 3, {})
    print("k4 planted", flush=True)
    ig, am, ad = run4(mdfs_gpu, w, divisions=1)
    top = set(np.argsort(-ig)[:4].tolist())
    assert top == {0, 1, 2, 3}
    assert am[0].tolist() == [1, 2, 3]
    assert ig[:4].min() > 10 * np.median(ig[4:])


def test_k4_collect_pass(mdfs_gpu, monkeypatch):
    w = workloads.xor_small(seed=67, n_obj=300, n_var=22, n_disc=2)
    monkeypatch.setenv("MDFS_TEST_CAP", str(3 * w.n_var))
    print("k4 collect pass", flush=True)
    got = run4(mdfs_gpu, w)
    monkeypatch.delenv("MDFS_TEST_CAP")
    ref = oracle.max_ig_all(w.data, w.y, 4, w.divisions, w.n_disc, w.range_, w.xi, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, "k4 collect pass")


def test_k4_limits(mdfs_gpu):
    # checked on the host by the C entry point before any pointer is used
    import ctypes
    lib = mdfs_gpu.load()
    null = ctypes.c_void_p(0)
    for kw, code in ((dict(divisions=4, engine="bitset"), -10), (dict(engine="mfma"), -10),
                     (dict(engine="mfma_fp4"), -10), (dict(n_var=2049), -10)):
        base = dict(n_obj=100, n_var=8, k=4, divisions=2, n_disc=1)
        base.update(kw)
        prm = mdfs_gpu.make_params(**base)
        rc = lib.mdfs_max_ig(ctypes.byref(prm), null, null, null, null, null, null, 0, null)
        assert rc == code, (kw, lib.mdfs_last_error())
    w = workloads.xor_small(seed=68, n_obj=100, n_var=8)
    data, y = to_dev(w)
    with pytest.raises(mdfs_gpu.MdfsError) as e:
        mdfs_gpu.mdfs_interesting_tuples(data, y, 4, 2, 1, 0.0)
    assert e.value.code == -3


# ------------------------------------------------------------------ the histogram engine (k = 4, 5)
CASES_H = {
    # k, workload
    "k4_d5": (4, lambda: dataclasses.replace(workloads.xor_small(seed=71, n_obj=500, n_var=17, n_disc=2), divisions=4)),
    "k4_d5_imbalanced": (4, lambda: dataclasses.replace(workloads.null_data(72, 333, 15, ones=70), divisions=4,
                                                        n_disc=2)),
    "k5_d2": (5, lambda: dataclasses.replace(workloads.xor_small(seed=73, n_obj=600, n_var=16, n_disc=2), divisions=1)),
    "k5_d3": (5, lambda: workloads.xor_small(seed=74, n_obj=450, n_var=13, n_disc=2)),
    "k5_d5": (5, lambda: dataclasses.replace(workloads.null_data(75, 700, 9, ones=300), divisions=4, n_disc=1)),
    "k5_five_vars": (5, lambda: workloads.xor_small(seed=76, n_obj=120, n_var=5, n_disc=3)),
    "k5_tiny_n": (5, lambda: dataclasses.replace(workloads.xor_small(seed=77, n_obj=9, n_var=8, n_disc=2), divisions=1)),
}


@pytest.mark.parametrize("name", list(CASES_H))
def test_hist_engine_matches_oracle(mdfs_gpu, name):
    k, make = CASES_H[name]
    w = make()
    print(f"hist {name} k={k} N={w.n_obj} p={w.n_var} d={w.divisions + 1} R={w.n_disc}", flush=True)
    got = run4(mdfs_gpu, w, k=k)
    ref = oracle.max_ig_all(w.data, w.y, k, w.divisions, w.n_disc, w.range_, w.xi, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, name)


@pytest.mark.parametrize("k,divisions", [(4, 1), (4, 2), (5, 1)])
def test_hist_engine_equals_bitset_engine(mdfs_gpu, k, divisions):
    # two count engines: identical outputs (the re-scored maxima do not depend on how the counts
    # were obtained); p spans several 64-pair chunks above the early prefixes
    w = dataclasses.replace(workloads.xor_small(seed=78, n_obj=800, n_var=30 if k == 4 else 24, n_disc=2),
                            divisions=divisions)
    print(f"hist vs bitset k={k} d={divisions + 1}", flush=True)
    a = run4(mdfs_gpu, w, engine="bitset", k=k)
    b = run4(mdfs_gpu, w, engine="hist", k=k)
    for x, z in zip(a, b):
        assert np.array_equal(x, z)


# ------------------------------------------------------------------ k = 5, two classes, bitsets
CASES_B5 = {
    "k5_d2": lambda: dataclasses.replace(workloads.xor_small(seed=81, n_obj=600, n_var=16, n_disc=2), divisions=1),
    "k5_d2_imbalanced": lambda: dataclasses.replace(workloads.null_data(82, 333, 12, ones=90), divisions=1,
                                                    n_disc=2),
    "k5_d2_wide_words": lambda: dataclasses.replace(workloads.xor_small(seed=83, n_obj=2100, n_var=9, n_disc=1),
                                                    divisions=1),
    "k5_d2_five_vars": lambda: dataclasses.replace(workloads.xor_small(seed=84, n_obj=120, n_var=5, n_disc=3),
                                                   divisions=1),
    "k5_d2_tiny_n": lambda: dataclasses.replace(workloads.xor_small(seed=85, n_obj=9, n_var=8, n_disc=2),
                                                divisions=1),
}


@pytest.mark.parametrize("name", list(CASES_B5))
def test_k5_bitset_engine_matches_oracle(mdfs_gpu, name):
    w = CASES_B5[name]()
    print(f"k5 bitset {name} N={w.n_obj} p={w.n_var} R={w.n_disc}", flush=True)
    got = run4(mdfs_gpu, w, k=5, engine="bitset")
    ref = oracle.max_ig_all(w.data, w.y, 5, w.divisions, w.n_disc, w.range_, w.xi, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, name)


def test_k5_bitset_engine_collect_pass(mdfs_gpu, monkeypatch):
    w = dataclasses.replace(workloads.xor_small(seed=86, n_obj=500, n_var=13, n_disc=2), divisions=1)
    monkeypatch.setenv("MDFS_TEST_CAP", str(3 * w.n_var))
    print("k5 bitset collect pass", flush=True)
    got = run4(mdfs_gpu, w, k=5, engine="bitset")
    monkeypatch.delenv("MDFS_TEST_CAP")
    ref = oracle.max_ig_all(w.data, w.y, 5, w.divisions, w.n_disc, w.range_, w.xi, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, "k5 bitset collect pass")


def test_hist_engine_finds_a_planted_parity_quintuple(mdfs_gpu):
    # y = xor of the signs of x0..x4: invisible to every quadruple, found by the k = 5 sweep
    g = np.random.default_rng(79)
    n, p = 2000, 14
    X = g.standard_normal((p, n)).astype(np.float32)
    y = ((X[0] > 0) ^ (X[1] > 0) ^ (X[2] > 0) ^ (X[3] > 0) ^ (X[4] > 0)).astype(np.uint8)
    w = workloads.Workload("parity5", X, y, 5, 1, 1, 0.0, 0.25, 3, {})
    for engine in ("auto", "hist"):   # two classes: "auto" is the bitset engine
        print(f"k5 planted {engine}", flush=True)
        ig, am, ad = run4(mdfs_gpu, w, k=5, divisions=1, engine=engine)
        assert set(np.argsort(-ig)[:5].tolist()) == {0, 1, 2, 3, 4}
        assert am[0].tolist() == [1, 2, 3, 4]
        assert ig[:5].min() > 10 * np.median(ig[5:])


def test_hist_engine_collect_pass_and_async(mdfs_gpu, monkeypatch):
    w = dataclasses.replace(workloads.xor_small(seed=80, n_obj=300, n_var=12, n_disc=2), divisions=4)
    monkeypatch.setenv("MDFS_TEST_CAP", str(3 * w.n_var))
    print("hist collect pass", flush=True)
    got = run4(mdfs_gpu, w)
    monkeypatch.delenv("MDFS_TEST_CAP")
    ref = oracle.max_ig_all(w.data, w.y, 4, w.divisions, w.n_disc, w.range_, w.xi, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, "hist collect pass")
    data, y = to_dev(w)
    a = mdfs_gpu.mdfs_max_ig_async(data, y, int(w.y.sum()), 5, 4, 2, w.xi, w.range_, w.seed)
    mdfs_gpu.mdfs_check_status((w.n_var, w.n_obj), 5, 4, 2)
    b = mdfs_gpu.mdfs_max_ig(data, y, 5, 4, 2, w.xi, w.range_, w.seed)
    for x, z in zip(a, b):
        assert torch.equal(x, z)
