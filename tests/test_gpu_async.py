"""mdfs_max_ig_async (no host synchronisation) and its capture in a CUDA graph."""
import numpy as np
import pytest
import torch

from paper_1811_00631_amd import mdfs, workloads

DEV = "cuda:0"
pytestmark = pytest.mark.gpu


def dev(w):
    return torch.from_numpy(w.data).to(DEV), torch.from_numpy(w.y).to(DEV)


def sync_call(X, y, k, div, R, engine="auto"):
    return mdfs.mdfs_max_ig(X, y, k, div, R, 0.25, 0.5, 7, engine=engine)


def async_call(X, y, k, div, R, ws=None, out=None):
    n1 = int(y.sum().item())
    return mdfs.mdfs_max_ig_async(X, y, n1, k, div, R, 0.25, 0.5, 7, ws=ws, out=out)


@pytest.mark.parametrize("k,div,p,engine", [(1, 2, 50, "auto"), (2, 2, 130, "auto"), (2, 4, 70, "auto"),
                                            (2, 1, 90, "auto"), (3, 2, 40, "bitset"), (3, 2, 70, "mfma_fp4"),
                                            (3, 1, 150, "mfma_fp4"), (4, 1, 18, "auto")])
def test_async_equals_sync(k, div, p, engine):
    # the k = 3 matrix-core engine builds its tile list on the device, so the asynchronous call
    # runs it as the synchronous one does
    w = workloads.xor_small(seed=81, n_obj=600, n_var=p, divisions=div, n_disc=3)
    X, y = dev(w)
    print(f"async k={k} div={div} p={p} {engine}", flush=True)
    ref = sync_call(X, y, k, div, 3, engine=engine)
    n1 = int(y.sum().item())
    got = mdfs.mdfs_max_ig_async(X, y, n1, k, div, 3, 0.25, 0.5, 7, engine=engine)
    mdfs.mdfs_check_status(X.shape, k, div, 3, engine=engine)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)


def test_async_collect_pass_runs_on_the_device(monkeypatch):
    w = workloads.xor_small(seed=82, n_obj=500, n_var=120, n_disc=5)
    X, y = dev(w)
    print("async collect pass", flush=True)
    ref = sync_call(X, y, 2, 2, 5)
    monkeypatch.setenv("MDFS_TEST_CAP", str(3 * w.n_var))
    got = async_call(X, y, 2, 2, 5)
    mdfs.mdfs_check_status(X.shape, 2, 2, 5)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    monkeypatch.setenv("MDFS_TEST_CAP", "8")
    async_call(X, y, 2, 2, 5)
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_check_status(X.shape, 2, 2, 5)
    assert e.value.code == -9


def test_async_flags_bad_inputs_on_the_device():
    w = workloads.xor_small(seed=83, n_obj=300, n_var=20)
    X, y = dev(w)
    n1 = int(y.sum().item())
    print("async bad inputs", flush=True)
    mdfs.mdfs_max_ig_async(X, y, n1 + 1, 2, 2, 1)                  # wrong class-1 count
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_check_status(X.shape, 2, 2, 1)
    assert e.value.code == -2
    y2 = y.clone()
    y2[5] = 2
    mdfs.mdfs_max_ig_async(X, y2, n1 + (1 - int(y[5].item())), 2, 2, 1)   # a value outside {0, 1}
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_check_status(X.shape, 2, 2, 1)
    assert e.value.code == -2
    Xn = X.clone()
    Xn[3, 7] = float("nan")
    mdfs.mdfs_max_ig_async(Xn, y, n1, 2, 2, 1)
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_check_status(X.shape, 2, 2, 1)
    assert e.value.code == -5
    # the same workspace serves a correct call afterwards
    got = mdfs.mdfs_max_ig_async(X, y, n1, 2, 2, 1)
    mdfs.mdfs_check_status(X.shape, 2, 2, 1)
    ref = mdfs.mdfs_max_ig(X, y, 2, 2, 1)
    assert torch.equal(got[0], ref[0])
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_max_ig_async(X, y, 0, 2, 2, 1)                   # refused on the host
    assert e.value.code == -2


@pytest.mark.parametrize("k", [2, 3])
def test_graph_capture_replays_match_eager(k):
    # the whole call captured once; replays on changed inputs, with eager work in between,
    # each checked against an eager synchronous call on the same inputs
    w = workloads.xor_small(seed=84 + k, n_obj=500, n_var=90 if k == 2 else 40, n_disc=3)
    X, y = dev(w)
    n1 = int(y.sum().item())
    prm = mdfs.make_params(w.n_obj, w.n_var, k, 2, 3, 0, 0.5, 0.25, 7)
    ws = torch.empty(mdfs.mdfs_workspace_size(prm), dtype=torch.uint8, device=DEV)
    out = (torch.empty(w.n_var, dtype=torch.float32, device=DEV),
           torch.empty((w.n_var, k - 1), dtype=torch.int32, device=DEV),
           torch.empty(w.n_var, dtype=torch.int32, device=DEV))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        mdfs.mdfs_max_ig_async(X, y, n1, k, 2, 3, 0.25, 0.5, 7, ws=ws, out=out)   # warm-up
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    print(f"capture k={k}", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mdfs.mdfs_max_ig_async(X, y, n1, k, 2, 3, 0.25, 0.5, 7, ws=ws, out=out)
    gen = np.random.default_rng(5)
    for rep in range(3):
        new = torch.from_numpy(gen.standard_normal(w.data.shape).astype(np.float32)).to(DEV)
        new[0] = X[0]
        new[1] = X[1]                  # keep the planted pair
        X.copy_(new)
        _ = (X * 2).sum()              # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        mdfs.mdfs_check_status(X.shape, k, 2, 3, ws=ws)
        ref = mdfs.mdfs_max_ig(X.clone(), y, k, 2, 3, 0.25, 0.5, 7)
        for a, b in zip(out, ref):
            assert torch.equal(a, b), f"replay {rep}"
