"""mdfs_max_ig_noalloc (the entry point for callers that cannot allocate) against
mdfs_max_ig_async, through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1811_00631_amd import mdfs, workloads

DEV = "cuda:0"
pytestmark = pytest.mark.gpu


def _noalloc(lib, prm, data, y, n1, out, status):
    ig, am, ad = out
    return lib.mdfs_max_ig_noalloc(ctypes.byref(prm), mdfs._ptr(data), mdfs._ptr(y), int(n1), mdfs._ptr(ig),
                                   mdfs._ptr(am), mdfs._ptr(ad), mdfs._ptr(status),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("k", [2, 3])
def test_noalloc_equals_async_twice_then_smaller(mdfs_gpu, k):
    lib = mdfs.load()
    # a larger problem, then a smaller one on the same scratch array
    cases = [workloads.madelon_like(seed=81, n_obj=1500, n_noise=280 if k == 2 else 60, n_disc=6 if k == 2 else 3),
             workloads.xor_small(seed=82, n_obj=301, n_var=75 if k == 2 else 33, n_disc=2)]
    for w in cases:
        print(f"noalloc k={k} N={w.n_obj} p={w.n_var} R={w.n_disc}", flush=True)
        data, y = torch.from_numpy(w.data).to(DEV), torch.from_numpy(w.y).to(DEV)
        n1 = int(w.y.sum())
        ref = mdfs.mdfs_max_ig_async(data, y, n1, k, w.divisions, w.n_disc, w.xi, w.range_, w.seed)
        mdfs.mdfs_check_status((w.n_var, w.n_obj), k, w.divisions, w.n_disc)
        out = (torch.full((w.n_var,), -7.0, device=DEV), torch.full((w.n_var, k - 1), -7, dtype=torch.int32, device=DEV),
               torch.full((w.n_var,), -7, dtype=torch.int32, device=DEV))
        status = torch.full((1,), 123, dtype=torch.int32, device=DEV)
        prm = mdfs.make_params(w.n_obj, w.n_var, k, w.divisions, w.n_disc, 0, w.range_, w.xi, w.seed)
        rc = _noalloc(lib, prm, data, y, n1, out, status)
        assert rc == 0, lib.mdfs_last_error().decode()
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        for a, b in zip(out, ref):
            assert torch.equal(a, b)
        # the planted pair is found through the allocation-free call as well
        am = out[1].cpu().numpy()
        if k == 2 and "xor_pair" in w.planted:
            assert am[0, 0] == 1 and am[1, 0] == 0


def test_noalloc_k3_holds_fewer_discretisations_of_pair_data(mdfs_gpu):
    # N = 2000, p = 500, R = 30 at k = 3: the default chunk of pair data (12 discretisations) does
    # not fit the array, so the allocation-free call takes fewer per launch; same results
    lib = mdfs.load()
    w = workloads.parity3(seed=3)
    prm = mdfs.make_params(w.n_obj, w.n_var, 3, w.divisions, w.n_disc, 0, w.range_, w.xi, w.seed)
    assert lib.mdfs_workspace_size(ctypes.byref(prm)) > 128 << 20
    data, y = torch.from_numpy(w.data).to(DEV), torch.from_numpy(w.y).to(DEV)
    n1 = int(w.y.sum())
    print("noalloc k=3 C3 size", flush=True)
    ref = mdfs.mdfs_max_ig_async(data, y, n1, 3, w.divisions, w.n_disc, w.xi, w.range_, w.seed)
    mdfs.mdfs_check_status((w.n_var, w.n_obj), 3, w.divisions, w.n_disc)
    out = (torch.empty(w.n_var, device=DEV), torch.empty((w.n_var, 2), dtype=torch.int32, device=DEV),
           torch.empty(w.n_var, dtype=torch.int32, device=DEV))
    status = torch.full((1,), 123, dtype=torch.int32, device=DEV)
    assert _noalloc(lib, prm, data, y, n1, out, status) == 0, lib.mdfs_last_error().decode()
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    for a, b in zip(out, ref):
        assert torch.equal(a, b)


def test_noalloc_reports_device_status_and_rejects_oversize(mdfs_gpu):
    lib = mdfs.load()
    w = workloads.xor_small(seed=83, n_obj=200, n_var=20, n_disc=1)
    data, y = torch.from_numpy(w.data).to(DEV), torch.from_numpy(w.y).to(DEV)
    out = (torch.empty(20, device=DEV), torch.empty((20, 1), dtype=torch.int32, device=DEV),
           torch.empty(20, dtype=torch.int32, device=DEV))
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    prm = mdfs.make_params(200, 20, 2, 2, 1, 0, 0.5, 0.25, 1)
    # a class-1 count that disagrees with y: flagged on the device, reported through status_out
    assert _noalloc(lib, prm, data, y, int(w.y.sum()) + 1, out, status) == 0
    torch.cuda.synchronize()
    assert int(status.item()) == -2
    # NaN data: reported the same way
    d2 = data.clone()
    d2[3, 5] = float("nan")
    assert _noalloc(lib, prm, d2, y, int(w.y.sum()), out, status) == 0
    torch.cuda.synchronize()
    assert int(status.item()) == -5
    # a valid call afterwards on the same array succeeds
    assert _noalloc(lib, prm, data, y, int(w.y.sum()), out, status) == 0
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    # a problem whose workspace exceeds the array is refused before anything is enqueued
    big = mdfs.make_params(2000, 20000, 2, 2, 30, 0, 0.5, 0.25, 1)
    rc = _noalloc(lib, big, data, y, int(w.y.sum()), out, status)
    assert rc == -6 and "allocation-free" in lib.mdfs_last_error().decode()
