"""k = 2 sweep on the GPU through the C ABI, against the FP64 oracle.

Bars: discretisation codes and voxel counts bit-exact; IG_max within
1e-4 * max(|IG|, 1) of the oracle; argmax tuple and discretisation exact.  Both one-hot
encodings of the pair contraction are covered: "mfma_fp4" (E2M1, float32 accumulation; what
"auto" picks while each class has < 4096 objects) and "mfma" (int8).
"""
import dataclasses

import numpy as np
import pytest
import torch

import fullsize_ref
import oracle
from paper_1811_00631_amd import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
IG_TOL = 1e-4
ENGINES = ["mfma_fp4", "mfma"]


def to_dev(w):
    return torch.from_numpy(w.data).to(DEV), torch.from_numpy(w.y).to(DEV)


def assert_ig_parity(ig, am, ad, ref, label=""):
    ref_ig, ref_am, ref_ad = ref
    ig = np.asarray(ig, dtype=np.float64)
    err = np.abs(ig - ref_ig) / np.maximum(np.abs(ref_ig), 1.0)
    worst = int(np.argmax(err))
    assert err.max() <= IG_TOL, f"{label}: IG error {err.max():.3g} at var {worst}: {ig[worst]} vs {ref_ig[worst]}"
    bad = np.nonzero((np.asarray(am) != ref_am).any(axis=1) | (np.asarray(ad) != ref_ad))[0]
    assert len(bad) == 0, (f"{label}: argmax differs for {len(bad)} vars, first {bad[:5]}: "
                           f"gpu {np.asarray(am)[bad[:3]]} r{np.asarray(ad)[bad[:3]]} vs "
                           f"oracle {ref_am[bad[:3]]} r{ref_ad[bad[:3]]}")


def run_gpu(mdfs, w, n_disc=None, xi=None, rng=None, seed=None, divisions=None, disc_offset=0, engine="auto"):
    data, y = to_dev(w)
    out = mdfs.mdfs_max_ig(data, y, 2, w.divisions if divisions is None else divisions,
                           w.n_disc if n_disc is None else n_disc, w.xi if xi is None else xi,
                           w.range_ if rng is None else rng, w.seed if seed is None else seed, disc_offset,
                           engine=engine)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


# ------------------------------------------------------------------ discretisation
@pytest.mark.parametrize("n_obj,n_var,div,R,rng", [(500, 37, 2, 3, 0.5), (1000, 5, 1, 2, 1.0),
                                                  (129, 130, 2, 2, 0.0), (64, 3, 4, 2, 0.7),
                                                  (3, 2, 2, 1, 0.5), (16384, 3, 2, 2, 0.5),
                                                  (16383, 2, 4, 1, 1.0)])
def test_codes_bit_exact(mdfs_gpu, n_obj, n_var, div, R, rng):
    g = np.random.default_rng(n_obj + n_var)
    X = g.standard_normal((n_var, n_obj)).astype(np.float32)
    X[0, ::2] = X[0, 1]      # ties
    X[-1] = np.round(X[-1])  # few distinct values
    print(f"codes N={n_obj} p={n_var} div={div} R={rng}", flush=True)
    codes = mdfs_gpu.mdfs_discretize(torch.from_numpy(X).to(DEV), div, R, rng, 17, disc_offset=3).cpu().numpy()
    ref = oracle.discretize(X, div, R, rng, 17, disc_offset=3)
    assert np.array_equal(codes, ref)


# ------------------------------------------------------------------ counts
@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("n_obj,n_var,div,ones", [(300, 150, 2, None), (257, 131, 1, 40), (130, 70, 2, 1),
                                                  (4095 + 129, 20, 2, 4095), (333, 90, 4, None), (140, 37, 4, 9)])
def test_pair_counts_bit_exact(mdfs_gpu, engine, n_obj, n_var, div, ones):
    # the last case puts 4095 objects (the fp4 maximum) in class 1 and 129 in class 0
    w = workloads.null_data(5, n_obj, n_var, ones=ones)
    data, y = to_dev(w)
    R, disc = 2, 1
    print(f"counts {engine} N={n_obj} p={n_var} div={div}", flush=True)
    counts = mdfs_gpu.mdfs_pair_counts(data, y, disc, div, R, 0.5, 9, engine=engine).cpu().numpy()
    codes = oracle.discretize(w.data, div, R, 0.5, 9)[disc]
    c = div + 1
    for i in range(n_var):
        for j in range(i + 1, n_var):
            ref = oracle.table(codes, w.y, c, [i, j])
            if not np.array_equal(counts[i, j], ref):
                pytest.fail(f"pair ({i},{j}): gpu {counts[i, j].tolist()} oracle {ref.tolist()}")


# ------------------------------------------------------------------ IG_max, small problems vs the full oracle
CASES = {
    "xor_small_C1": lambda: workloads.xor_small(seed=1),
    "madelon_like_small": lambda: workloads.madelon_like(seed=2, n_obj=600, n_noise=50, n_disc=4),
    "two_classes_d2": lambda: workloads.xor_small(seed=3, n_obj=333, n_var=129, divisions=1, n_disc=3),
    "imbalanced": lambda: workloads.null_data(4, 401, 66, ones=37),
    "two_vars": lambda: workloads.xor_small(seed=5, n_obj=100, n_var=2),
    "tiny_n": lambda: workloads.xor_small(seed=6, n_obj=5, n_var=9, n_disc=2),
    "five_classes": lambda: workloads.xor_small(seed=7, n_obj=700, n_var=77, divisions=4, n_disc=3),
    "five_classes_imbalanced": lambda: dataclasses.replace(workloads.null_data(15, 300, 45, ones=61),
                                                           divisions=4, n_disc=2),
}


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("name", list(CASES))
def test_max_ig_matches_oracle(mdfs_gpu, name, engine):
    w = CASES[name]()
    print(f"max_ig {name} {engine} N={w.n_obj} p={w.n_var} R={w.n_disc}", flush=True)
    got = run_gpu(mdfs_gpu, w, engine=engine)
    ref = oracle.max_ig_all(w.data, w.y, 2, w.divisions, w.n_disc, w.range_, w.xi, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, name)


def test_xi_zero_and_range_zero(mdfs_gpu):
    w = workloads.xor_small(seed=8, n_obj=256, n_var=40, n_disc=3)
    got = run_gpu(mdfs_gpu, w, xi=0.0, rng=0.0)
    ref = oracle.max_ig_all(w.data, w.y, 2, 2, 3, 0.0, 0.0, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, "xi0_range0")


def test_exact_ties_follow_tie_rule(mdfs_gpu):
    # copies of the XOR partner tie exactly; range=0 makes every discretisation tie as well
    w = workloads.xor_small(seed=9, n_obj=300, n_var=10, n_disc=3)
    X = np.concatenate([w.data, w.data[[1, 1, 1]]], axis=0)
    w2 = workloads.Workload("ties", X, w.y, 2, 2, 3, 0.0, 0.25, 9, {})
    got = run_gpu(mdfs_gpu, w2)
    ref = oracle.max_ig_all(X, w.y, 2, 2, 3, 0.0, 0.25, 9, n_threads=8)
    assert_ig_parity(*got, ref, "ties")
    assert got[1][0, 0] == 1 and got[2][0] == 0


@pytest.mark.parametrize("engine", ENGINES)
def test_screen_within_error_bound(mdfs_gpu, engine):
    w = workloads.madelon_like(seed=12, n_obj=700, n_noise=60, n_disc=3)
    data, y = to_dev(w)
    ig32, E = mdfs_gpu.mdfs_screen_max(data, y, 2, 2, 3, 0.25, 0.5, w.seed, engine=engine)
    ig32 = ig32.cpu().numpy().astype(np.float64)
    ref, _, _ = oracle.max_ig_all(w.data, w.y, 2, 2, 3, 0.5, 0.25, w.seed, n_threads=8)
    err = np.abs(ig32 - ref)
    print(f"float32 screen: max |err| {err.max():.3g}, bound E {E:.3g}")
    assert 0 < E < 0.05
    assert err.max() <= E


def test_deterministic_and_fused_equals_separate(mdfs_gpu):
    w = workloads.xor_small(seed=10, n_obj=400, n_var=90, n_disc=4)
    a = run_gpu(mdfs_gpu, w)
    b = run_gpu(mdfs_gpu, w)
    for x, z in zip(a, b):
        assert np.array_equal(x, z)
    sep = [run_gpu(mdfs_gpu, w, n_disc=1, disc_offset=r) for r in range(4)]
    stack = np.stack([s[0] for s in sep])
    assert np.array_equal(a[0], stack.max(axis=0))
    for v in range(w.n_var):
        r = a[2][v]
        assert np.array_equal(sep[r][1][v], a[1][v]) and sep[r][2][v] == r


@pytest.mark.parametrize("div,n_var,engine", [(2, 1500, "mfma_fp4"), (2, 700, "mfma"), (1, 1100, "mfma_fp4"),
                                               (4, 900, "mfma_fp4")])
def test_launch_shapes_give_identical_results(mdfs_gpu, div, n_var, engine):
    # every super-tile side and wave count (and grid) takes every tile once: the outputs are
    # bit-identical to the default launch; the variable counts leave ragged super-tiles
    w = workloads.xor_small(seed=12, n_obj=700, n_var=n_var, divisions=div, n_disc=2)
    X, y = to_dev(w)
    print(f"launch shapes div={div} p={n_var} {engine}", flush=True)
    ref = [t.cpu() for t in mdfs_gpu.mdfs_max_ig(X, y, 2, div, 2, 0.25, 0.5, 3, engine=engine)]
    waves = (0, 4, 8) if div == 2 else (0,)
    for sb in (2, 4, 16):
        for nw in waves:
            for g in (0, 96):
                got = mdfs_gpu.mdfs_max_ig(X, y, 2, div, 2, 0.25, 0.5, 3, engine=engine, workgroups=g,
                                           tile=mdfs_gpu.tile_code(sb, nw))
                for a_, b_ in zip(ref, got):
                    assert torch.equal(a_, b_.cpu()), (sb, nw, g)
    if div in (1, 2):   # k = 3: the pair tables come from the pair sweep at the chosen shape
        w3 = workloads.xor_small(seed=13, n_obj=700, n_var=150, divisions=div, n_disc=2)
        X3, y3 = to_dev(w3)
        ref3 = [t.cpu() for t in mdfs_gpu.mdfs_max_ig(X3, y3, 3, div, 2, engine="mfma_fp4")]
        got3 = mdfs_gpu.mdfs_max_ig(X3, y3, 3, div, 2, engine="mfma_fp4", tile=mdfs_gpu.tile_code(2, 4))
        for a_, b_ in zip(ref3, got3):
            assert torch.equal(a_, b_.cpu())


def test_decision_errors(mdfs_gpu):
    w = workloads.xor_small(seed=11, n_obj=50, n_var=4)
    data, y = to_dev(w)
    bad = y.clone()
    bad[3] = 2
    with pytest.raises(mdfs_gpu.MdfsError) as e:
        mdfs_gpu.mdfs_max_ig(data, bad, 2, 2, 1)
    assert e.value.code == -2
    with pytest.raises(mdfs_gpu.MdfsError) as e:
        mdfs_gpu.mdfs_max_ig(data, torch.zeros_like(y), 2, 2, 1)
    assert e.value.code == -2
    d2 = data.clone()
    d2[2, 7] = float("nan")
    with pytest.raises(mdfs_gpu.MdfsError) as e:
        mdfs_gpu.mdfs_max_ig(d2, y, 2, 2, 1)
    assert e.value.code == -5


# ------------------------------------------------------------------ full size, every variable
@pytest.mark.parametrize("which,engine", [("headline", "auto"), ("headline", "mfma"), ("genomics_like", "auto"),
                                          ("madelon_like", "auto"), ("madelon2_d2", "auto")])
def test_full_size_every_variable(mdfs_gpu, which, engine):
    # the benchmark workloads at their full sizes, every variable against the FP64 oracle (stored
    # by tests/golden/make_fullsize.py; a regenerated input that does not hash to the stored digest
    # falls back to the live oracle on a sample holding every planted variable)
    w, k = fullsize_ref.workload(which)
    print(f"full-size {which} {engine}: N={w.n_obj} p={w.n_var} R={w.n_disc} d={w.divisions + 1}", flush=True)
    ig, am, ad = run_gpu(mdfs_gpu, w, engine=engine)
    assert np.isfinite(ig).all()
    for a_, b_ in w.planted.get("pairs", []):
        assert am[a_, 0] == b_ and am[b_, 0] == a_, (a_, b_, am[a_], am[b_])
    tg, ref, complete = fullsize_ref.reference(which, w, k)
    print(f"  compared {len(tg)} of {w.n_var} variables ({'all, stored' if complete else 'live sample'})",
          flush=True)
    assert_ig_parity(ig[tg], am[tg], ad[tg], ref, which)


def test_candidate_overflow_falls_back_to_collect_pass(mdfs_gpu, monkeypatch):
    # a tiny candidate buffer overflows during the sweep; the second (collect) pass with the
    # final float32 maxima must reproduce the oracle exactly
    w = workloads.xor_small(seed=13, n_obj=500, n_var=120, n_disc=5)
    monkeypatch.setenv("MDFS_TEST_CAP", str(3 * w.n_var))
    got = run_gpu(mdfs_gpu, w)
    monkeypatch.delenv("MDFS_TEST_CAP")
    ref = oracle.max_ig_all(w.data, w.y, 2, w.divisions, w.n_disc, w.range_, w.xi, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, "collect-pass")
    # and a buffer too small even for the final window is reported, not silently wrong
    monkeypatch.setenv("MDFS_TEST_CAP", "8")
    with pytest.raises(mdfs_gpu.MdfsError) as e:
        run_gpu(mdfs_gpu, w)
    assert e.value.code == -9


def test_large_classes_use_int8_and_fp4_refuses_them(mdfs_gpu):
    # 4096 objects in class 1: float32 packing n1 * 4096 + n0 would no longer be exact, so
    # "auto" must take the int8 encoding (parity shows it did) and "mfma_fp4" must refuse
    w = workloads.null_data(14, 4096 + 300, 48, ones=4096)
    print(f"large classes N={w.n_obj} p={w.n_var}", flush=True)
    got = run_gpu(mdfs_gpu, w, n_disc=2)
    ref = oracle.max_ig_all(w.data, w.y, 2, w.divisions, 2, w.range_, w.xi, w.seed, n_threads=8)
    assert_ig_parity(*got, ref, "large classes")
    with pytest.raises(mdfs_gpu.MdfsError) as e:
        run_gpu(mdfs_gpu, w, n_disc=2, engine="mfma_fp4")
    assert e.value.code == -10


@pytest.mark.parametrize("div,rng,ones,n_obj,n_var", [(2, 0.5, None, 450, 70), (1, 0.0, 60, 450, 70),
                                                     (4, 0.7, None, 450, 70), (2, 0.5, 5000, 16384, 6)])
def test_k1_matches_oracle(mdfs_gpu, div, rng, ones, n_obj, n_var):
    # the one-dimensional analysis: no tuples, binary64 F of each variable, max over discretisations
    # (the last case: the largest N, class sizes 11384 / 5000, through the class-sorted marginals)
    print(f"k1 N={n_obj} p={n_var} div={div}", flush=True)
    w = workloads.null_data(16, n_obj, n_var, ones=ones)
    X = w.data.copy()
    X[3] = (w.y * 2.0 - 1.0) + 0.3 * X[3]          # an informative variable
    data, y = torch.from_numpy(X).to(DEV), torch.from_numpy(w.y).to(DEV)
    ig, am, ad = mdfs_gpu.mdfs_max_ig(data, y, 1, div, 5, 0.25, rng, 7)
    ref_ig, _, ref_ad = oracle.max_ig_all(X, w.y, 1, div, 5, rng, 0.25, 7, n_threads=4)
    ig = ig.cpu().numpy().astype(np.float64)
    err = np.abs(ig - ref_ig) / np.maximum(np.abs(ref_ig), 1.0)    # per element
    assert err.max() <= IG_TOL, f"k=1 IG error {err.max():.3g} at var {int(np.argmax(err))}"
    assert np.array_equal(ad.cpu().numpy(), ref_ad)
    assert int(np.argmax(ig)) == 3
