"""k = 3 sweep on the GPU through the C ABI, against the FP64 oracle.

Two count engines: "bitset" (per-class bitsets, AND + popcount; every class count) and
"mfma_fp4" (pair one-hot x one-hot on the matrix cores; two or three classes, classes < 4096
objects),
which "auto" picks where it applies."""
import numpy as np
import pytest
import torch

import fullsize_ref
import oracle
from paper_1811_00631_amd import workloads

from test_gpu_k2 import assert_ig_parity, to_dev

pytestmark = pytest.mark.gpu


ENGINES3 = ["bitset", "mfma_fp4"]


def run3(mdfs, w, n_disc=None, xi=None, rng=None, divisions=None, disc_offset=0, engine="auto"):
    data, y = to_dev(w)
    out = mdfs.mdfs_max_ig(data, y, 3, w.divisions if divisions is None else divisions,
                           w.n_disc if n_disc is None else n_disc, w.xi if xi is None else xi,
                           w.range_ if rng is None else rng, w.seed, disc_offset, engine=engine)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


CASES3 = {
    "parity3_small": lambda: workloads.parity3(seed=3, n_obj=400, n_var=14, n_disc=2),
    "chunks_ragged": lambda: workloads.xor_small(seed=21, n_obj=301, n_var=75, n_disc=2),
    "two_classes_d2": lambda: workloads.parity3(seed=22, n_obj=257, n_var=40, divisions=1, n_disc=3),
    "imbalanced": lambda: workloads.null_data(23, 333, 30, ones=41),
    "three_vars": lambda: workloads.parity3(seed=24, n_obj=100, n_var=3, n_disc=2),
    "five_classes": lambda: workloads.parity3(seed=25, n_obj=500, n_var=26, divisions=4, n_disc=2),
    # two classes over three 128-variable blocks with a ragged last one (the two-class matrix-core
    # tile is 128 j x 128 l)
    "two_classes_tiles": lambda: workloads.parity3(seed=26, n_obj=203, n_var=261, divisions=1, n_disc=2),
}


@pytest.mark.parametrize("engine", ENGINES3)
@pytest.mark.parametrize("name", list(CASES3))
def test_k3_matches_oracle(mdfs_gpu, name, engine):
    w = CASES3[name]()
    if engine == "mfma_fp4" and w.divisions not in (1, 2):
        pytest.skip("the matrix-core k=3 engine is built for two or three classes")
    print(f"k3 {name} {engine} N={w.n_obj} p={w.n_var} R={w.n_disc} d={w.divisions + 1}", flush=True)
    got = run3(mdfs_gpu, w, engine=engine)
    ref = oracle.max_ig_all(w.data, w.y, 3, w.divisions, w.n_disc, w.range_, w.xi, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, name)


def _triple_ref(codes_r, y, c, i, n_var):
    """The oracle's tables of every triple (i, j, l), i < j < l, indexed [j][l]."""
    ref = {}
    for j in range(i + 1, n_var):
        for l in range(j + 1, n_var):
            ref[(j, l)] = oracle.table(codes_r, y, c, [i, j, l])
    return ref


# n_obj, n_var, divisions, class-1 objects, i_sel: ragged tiles of both matrix-core kernels (32 j x
# 64 l and 128 x 128 variables), several K blocks per class, the largest class the fp4 encoding
# takes (4095 objects), imbalanced classes, five classes on the bitset engine, the last i_sel
COUNT3 = [(300, 70, 2, None, 0), (257, 140, 1, 40, 0), (333, 45, 2, 60, 7), (4095 + 70, 12, 2, 4095, 0),
          (500, 29, 4, None, 0), (199, 37, 1, None, 34), (1000, 67, 2, 300, 1)]


@pytest.mark.parametrize("engine", ENGINES3)
@pytest.mark.parametrize("n_obj,n_var,div,ones,i_sel", COUNT3)
def test_k3_counts_bit_exact(mdfs_gpu, engine, n_obj, n_var, div, ones, i_sel):
    # the tables of every triple (i_sel, j, l) of one discretisation, from the count engine the
    # maximum sweep runs, equal the oracle's brute-force tables cell by cell
    if engine == "mfma_fp4" and div not in (1, 2):
        pytest.skip("the matrix-core k=3 engine is built for two or three classes")
    w = workloads.null_data(70 + n_var, n_obj, n_var, ones=ones)
    data, y = to_dev(w)
    R, disc, c = 3, 2, div + 1
    print(f"k3 counts {engine} N={n_obj} p={n_var} d={c} i={i_sel}", flush=True)
    got = mdfs_gpu.mdfs_triple_counts(data, y, disc, i_sel, div, R, 0.5, 19, engine=engine).cpu().numpy()
    codes = oracle.discretize(w.data, div, R, 0.5, 19)[disc]
    for (j, l), ref in _triple_ref(codes, w.y, c, i_sel, n_var).items():
        if not np.array_equal(got[j, l], ref):
            pytest.fail(f"triple ({i_sel},{j},{l}): gpu {got[j, l].tolist()} oracle {ref.tolist()}")


@pytest.mark.parametrize("engine", ENGINES3)
def test_k3_parity_triple_found(mdfs_gpu, engine):
    w = workloads.parity3(seed=31, n_obj=1000, n_var=40, n_disc=2)
    ig, am, _ = run3(mdfs_gpu, w, engine=engine)
    for v, others in [(0, [1, 2]), (1, [0, 2]), (2, [0, 1])]:
        assert am[v].tolist() == others
    assert ig[:3].min() > 5 * ig[3:].max()


@pytest.mark.parametrize("engine", ENGINES3)
def test_k3_screen_within_error_bound(mdfs_gpu, engine):
    w = workloads.parity3(seed=32, n_obj=600, n_var=24, n_disc=2)
    data, y = to_dev(w)
    ig32, E = mdfs_gpu.mdfs_screen_max(data, y, 3, 2, 2, 0.25, 0.5, w.seed, engine=engine)
    ig32 = ig32.cpu().numpy().astype(np.float64)
    ref, _, _ = oracle.max_ig_all(w.data, w.y, 3, 2, 2, 0.5, 0.25, w.seed, n_threads=2)
    err = np.abs(ig32 - ref)
    print(f"k=3 float32 screen: max |err| {err.max():.3g}, bound E {E:.3g}")
    assert err.max() <= E


@pytest.mark.parametrize("engine", ENGINES3)
def test_k3_deterministic_and_fused_equals_separate(mdfs_gpu, engine):
    w = workloads.parity3(seed=33, n_obj=300, n_var=30, n_disc=3)
    a = run3(mdfs_gpu, w, engine=engine)
    b = run3(mdfs_gpu, w, engine=engine)
    for x, z in zip(a, b):
        assert np.array_equal(x, z)
    sep = [run3(mdfs_gpu, w, n_disc=1, disc_offset=r, engine=engine) for r in range(3)]
    assert np.array_equal(a[0], np.stack([s[0] for s in sep]).max(axis=0))


@pytest.mark.parametrize("which,engine", [("parity3", "mfma_fp4"), ("parity3", "bitset"),
                                          ("madelon3_d2", "mfma_fp4"), ("madelon3_d2", "bitset")])
def test_k3_full_size_every_variable(mdfs_gpu, which, engine):
    # the k = 3 workloads at full size (N=2000, p=500, 30 discretisations; three classes with the
    # planted parity triple, and two classes in the shape of the paper's 3D timing), every variable
    # against the FP64 oracle stored by tests/golden/make_fullsize.py
    w, k = fullsize_ref.workload(which)
    print(f"k3 full size {which} {engine}: N={w.n_obj} p={w.n_var} R={w.n_disc} d={w.divisions + 1}", flush=True)
    ig, am, ad = run3(mdfs_gpu, w, engine=engine)
    assert np.isfinite(ig).all()
    if "triple" in w.planted:
        for v, others in [(0, [1, 2]), (1, [0, 2]), (2, [0, 1])]:
            assert am[v].tolist() == others
    tg, ref, complete = fullsize_ref.reference(which, w, k)
    print(f"  compared {len(tg)} of {w.n_var} variables ({'all, stored' if complete else 'live sample'})",
          flush=True)
    assert_ig_parity(ig[tg], am[tg], ad[tg], ref, which)


@pytest.mark.parametrize("divisions", [1, 2])
def test_k3_engines_agree_bit_for_bit_on_argmax(mdfs_gpu, divisions):
    # same float32 screen tables, same binary64 re-score: both engines must give identical
    # results (the re-scored maxima do not depend on how the counts were obtained)
    w = workloads.parity3(seed=34, n_obj=777, n_var=50 if divisions == 2 else 150, divisions=divisions, n_disc=3)
    a = run3(mdfs_gpu, w, engine="bitset")
    b = run3(mdfs_gpu, w, engine="mfma_fp4")
    for x, z in zip(a, b):
        assert np.array_equal(x, z)


def test_k3_at_the_largest_variable_count(mdfs_gpu):
    # p = 8192, the limit: the last j block of the matrix-core tile list and pair tables of
    # 2^26 entries; both engines agree on every variable and the planted triple is found
    p = 8192
    w = workloads.parity3(seed=36, n_obj=256, n_var=p, divisions=1, n_disc=1)
    print(f"k3 p={p}", flush=True)
    a = run3(mdfs_gpu, w, engine="mfma_fp4")
    b = run3(mdfs_gpu, w, engine="bitset")
    for x, z in zip(a, b):
        assert np.array_equal(x, z)
    assert set(np.argsort(-a[0])[:3].tolist()) == {0, 1, 2}
    assert a[1][0].tolist() == [1, 2]
    import ctypes
    prm = mdfs_gpu.make_params(256, p + 1, 3, 1, 1)
    null = ctypes.c_void_p(0)
    assert mdfs_gpu.load().mdfs_max_ig(ctypes.byref(prm), null, null, null, null, null, null, 0, null) == -10


def test_k3_mfma_engine_limits(mdfs_gpu):
    w = workloads.parity3(seed=35, n_obj=200, n_var=12, divisions=4, n_disc=1)
    with pytest.raises(mdfs_gpu.MdfsError) as e:
        run3(mdfs_gpu, w, engine="mfma_fp4")
    assert e.value.code == -10
    with pytest.raises(mdfs_gpu.MdfsError) as e:
        run3(mdfs_gpu, workloads.parity3(seed=35, n_obj=200, n_var=12, n_disc=1), engine="mfma")
    assert e.value.code == -10
