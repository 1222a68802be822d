"""mdfs_max_ig_batch: several k = 2 problems with one fused persistent sweep launch, and several
k = 3, 4 or 5 problems on concurrent streams."""
import numpy as np
import pytest
import torch

from paper_1811_00631_amd import mdfs, workloads

DEV = "cuda:0"
pytestmark = pytest.mark.gpu

SHAPES = [(300, 50, 1), (1200, 700, 3), (777, 129, 2), (2500, 333, 4), (64, 9, 5), (1500, 260, 1)]


def problems(div, shapes, seed=91, ones=None):
    out = []
    for i, (n, p, R) in enumerate(shapes):
        w = workloads.xor_small(seed=seed + i, n_obj=n, n_var=p, divisions=div, n_disc=R)
        y = w.y if ones is None or ones[i] is None else _force_ones(w.y, ones[i], seed + i)
        out.append((torch.from_numpy(w.data).to(DEV), torch.from_numpy(y).to(DEV), R, 11 + i))
    return out


def _force_ones(y, k, seed):
    g = np.random.default_rng(seed)
    v = np.zeros_like(y)
    v[g.permutation(len(y))[:k]] = 1
    return v


def run_batch(probs, div, engine="auto"):
    outs, wss = mdfs.mdfs_max_ig_batch([d for d, _, _, _ in probs], [y for _, y, _, _ in probs],
                                       [int(y.sum().item()) for _, y, _, _ in probs], 2, div,
                                       [R for _, _, R, _ in probs], 0.25, 0.5, [s for _, _, _, s in probs],
                                       engine=engine)
    torch.cuda.synchronize()
    for (d, _, R, _), ws in zip(probs, wss):
        mdfs.mdfs_check_status(d.shape, 2, div, R, ws=ws, engine=engine)
    return outs


def check_equal(probs, outs, div, engine="auto"):
    for i, ((d, y, R, s), got) in enumerate(zip(probs, outs)):
        ref = mdfs.mdfs_max_ig(d, y, 2, div, R, 0.25, 0.5, s, engine=engine)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), f"problem {i}"


@pytest.mark.parametrize("div,engine", [(2, "auto"), (1, "mfma"), (4, "auto"), (2, "mfma")])
def test_batch_equals_separate_calls(div, engine):
    probs = problems(div, SHAPES)
    print(f"batch div={div} {engine}", flush=True)
    check_equal(probs, run_batch(probs, div, engine), div, engine)


def test_batch_of_one_and_twelve():
    probs = problems(2, [(400, 120, 2)])
    check_equal(probs, run_batch(probs, 2), 2)
    probs = problems(2, [(200 + 37 * i, 20 + 11 * i, 1 + i % 3) for i in range(12)], seed=140)
    print("batch of 12", flush=True)
    check_equal(probs, run_batch(probs, 2), 2)


def test_batch_overflow_goes_through_each_collect_pass(monkeypatch):
    probs = problems(2, [(500, 120, 5), (600, 150, 3)], seed=160)
    monkeypatch.setenv("MDFS_TEST_CAP", "400")
    print("batch overflow", flush=True)
    outs = run_batch(probs, 2)
    monkeypatch.delenv("MDFS_TEST_CAP")
    check_equal(probs, outs, 2)


def test_batch_rejections():
    probs = problems(2, [(300, 40, 1), (300, 40, 1)], seed=170)
    d, y = [p[0] for p in probs], [p[1] for p in probs]
    n1 = [int(v.sum().item()) for v in y]
    with pytest.raises(mdfs.MdfsError) as e:   # one problem needs the int8 encoding
        big = workloads.xor_small(seed=171, n_obj=4500, n_var=20)
        yb = torch.from_numpy(_force_ones(big.y, 4200, 3)).to(DEV)
        mdfs.mdfs_max_ig_batch(d + [torch.from_numpy(big.data).to(DEV)], y + [yb], n1 + [4200], 2, 2, [1, 1, 1])
    assert e.value.code == -10
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_max_ig_batch(d * 7, y * 7, n1 * 7, 2, 2, [1] * 14)   # 14 > 12
    assert e.value.code == -1


def test_batch_graph_capture():
    probs = problems(2, [(500, 90, 2), (800, 200, 3), (300, 60, 1)], seed=180)
    d, y = [p[0] for p in probs], [p[1] for p in probs]
    n1 = [int(v.sum().item()) for v in y]
    seeds = [p[3] for p in probs]
    args = (d, y, n1, 2, 2, [p[2] for p in probs], 0.25, 0.5, seeds)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        mdfs.mdfs_max_ig_batch(*args)   # warm-up (sets the kernels' LDS attribute)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    print("batch capture", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs, _ = mdfs.mdfs_max_ig_batch(*args)
    for rep in range(3):
        for t in d:
            t.mul_(-1.0 if rep % 2 == 0 else 1.0)   # inputs change between replays
        g.replay()
        torch.cuda.synchronize()
        check_equal(probs, outs, 2)


def _run_k(probs, k, div, engine="auto"):
    outs, wss = mdfs.mdfs_max_ig_batch([d for d, _, _, _ in probs], [y for _, y, _, _ in probs],
                                       [int(y.sum().item()) for _, y, _, _ in probs], k, div,
                                       [R for _, _, R, _ in probs], 0.25, 0.5, [s for _, _, _, s in probs],
                                       engine=engine)
    torch.cuda.synchronize()
    for (d, _, R, _), ws in zip(probs, wss):
        mdfs.mdfs_check_status(d.shape, k, div, R, ws=ws, engine=engine)
    return outs


@pytest.mark.parametrize("k,div,engine,shapes", [
    (3, 2, "auto", [(300, 40, 2), (1200, 90, 3), (777, 33, 1), (2500, 61, 2), (64, 9, 3), (1500, 70, 1)]),
    (3, 1, "bitset", [(500, 50, 2), (901, 23, 1), (333, 64, 3)]),
    (3, 4, "auto", [(400, 20, 2), (650, 31, 1)]),
    (4, 1, "auto", [(600, 24, 1), (300, 17, 2), (1000, 30, 1)]),
    (5, 1, "auto", [(500, 14, 1), (700, 11, 2)]),
])
def test_batch_of_higher_k_equals_separate_calls(k, div, engine, shapes):
    probs = problems(div, shapes, seed=300 + k)
    print(f"batch k={k} d={div + 1} {engine} n={len(probs)}", flush=True)
    outs = _run_k(probs, k, div, engine)
    for i, ((d, y, R, s), got) in enumerate(zip(probs, outs)):
        ref = mdfs.mdfs_max_ig(d, y, k, div, R, 0.25, 0.5, s, engine=engine)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), f"problem {i}"


def test_batch_of_higher_k_rejects_mixed_k_and_captures():
    probs = problems(2, [(300, 30, 2), (500, 40, 1), (200, 25, 2)], seed=310)
    d, y = [p[0] for p in probs], [p[1] for p in probs]
    n1 = [int(v.sum().item()) for v in y]
    # mixed k is refused on the host before any pointer is used
    prms = (mdfs.Params * 2)(mdfs.make_params(300, 30, 3, 2, 2), mdfs.make_params(500, 40, 4, 2, 1))
    import ctypes
    null = (ctypes.c_void_p * 2)()
    bws = torch.empty(mdfs.load().mdfs_batch_workspace_size(), dtype=torch.uint8, device=DEV)
    rc = mdfs.load().mdfs_max_ig_batch(2, prms, null, null, (ctypes.c_int64 * 2)(1, 1), null, null, null, null,
                                       (ctypes.c_size_t * 2)(), ctypes.c_void_p(bws.data_ptr()), bws.numel(), None)
    assert rc == -3
    # captured in a graph after a warm-up call (which creates the thread's side streams), replayed
    args = (d, y, n1, 3, 2, [p[2] for p in probs], 0.25, 0.5, [p[3] for p in probs])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        mdfs.mdfs_max_ig_batch(*args)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    print("batch k=3 capture", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs, _ = mdfs.mdfs_max_ig_batch(*args)
    for rep in range(3):
        for t in d:
            t.mul_(-1.0 if rep % 2 == 0 else 1.0)   # inputs change between replays
        _ = sum(float(t.sum()) for t in d)        # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        for i, ((dd, yy, R, sd), got) in enumerate(zip(probs, outs)):
            ref = mdfs.mdfs_max_ig(dd, yy, 3, 2, R, 0.25, 0.5, sd)
            for a, b in zip(ref, got):
                assert torch.equal(a, b), f"replay {rep} problem {i}"
