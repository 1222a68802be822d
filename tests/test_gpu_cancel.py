"""Cancellation through the caller's host-mapped cancel word (mdfs_params.cancel).

The word is set from the host, never by the GPU: every kernel polls it and exits normally, and the
call reports MDFS_E_CANCELLED.  A cleared word lets the same workspace serve a complete call."""
import ctypes
import threading
import time

import pytest
import torch

from paper_1811_00631_amd import mdfs, workloads

DEV = "cuda:0"
pytestmark = pytest.mark.gpu

HIP_HOST_MALLOC_MAPPED, HIP_HOST_MALLOC_COHERENT = 0x2, 0x40000000


@pytest.fixture
def cancel_word(mdfs_gpu):
    """A coherent, mapped pinned host word (hipHostMalloc), freed after the test."""
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipHostMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_uint]
    hip.hipHostFree.argtypes = [ctypes.c_void_p]
    ptr = ctypes.c_void_p()
    assert hip.hipHostMalloc(ctypes.byref(ptr), 64, HIP_HOST_MALLOC_MAPPED | HIP_HOST_MALLOC_COHERENT) == 0
    word = ctypes.cast(ptr, ctypes.POINTER(ctypes.c_uint32))
    word[0] = 0
    yield ptr.value, word
    torch.cuda.synchronize()
    hip.hipHostFree(ptr)


@pytest.mark.parametrize("k,engine,div", [(2, "auto", 2), (3, "mfma_fp4", 2), (3, "bitset", 2), (4, "bitset", 2),
                                          (4, "bitset", 1), (5, "bitset", 1), (5, "hist", 2)])
def test_cancel_before_the_call_then_a_clean_call(cancel_word, k, engine, div):
    addr, word = cancel_word
    w = workloads.xor_small(seed=90 + k, n_obj=400, n_var={2: 300, 3: 60, 4: 20, 5: 11}[k], n_disc=3)
    X, y = torch.from_numpy(w.data).to(DEV), torch.from_numpy(w.y).to(DEV)
    print(f"cancel before k={k} {engine} d={div + 1}", flush=True)
    ref = mdfs.mdfs_max_ig(X, y, k, div, 3, engine=engine)
    word[0] = 1
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_max_ig(X, y, k, div, 3, engine=engine, cancel=addr)
    assert e.value.code == mdfs.E_CANCELLED
    # asynchronous call: reported by mdfs_check_status
    mdfs.mdfs_max_ig_async(X, y, int(w.y.sum()), k, div, 3, engine=engine, cancel=addr)
    with pytest.raises(mdfs.MdfsError) as e:
        mdfs.mdfs_check_status(X.shape, k, div, 3, engine=engine)
    assert e.value.code == mdfs.E_CANCELLED
    # cleared: the same workspace gives the complete result
    word[0] = 0
    got = mdfs.mdfs_max_ig(X, y, k, div, 3, engine=engine, cancel=addr)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)


@pytest.mark.parametrize("k", [2, 3])
def test_cancel_from_another_thread_stops_a_running_call(cancel_word, k):
    # a call of a few hundred milliseconds, cancelled from another host thread shortly after it
    # starts: it returns MDFS_E_CANCELLED well before its uncancelled duration
    addr, word = cancel_word
    if k == 2:
        w = workloads.genomics_like(seed=4, n_obj=2000, n_var=20000, n_ones=None, n_disc=120)
    else:
        w = workloads.parity3(seed=3, n_obj=2000, n_var=500, n_disc=300)
    X, y = torch.from_numpy(w.data).to(DEV), torch.from_numpy(w.y).to(DEV)
    mdfs.mdfs_max_ig(X, y, k, 2, 2)          # warm-up (workspace, code objects)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = mdfs.mdfs_max_ig(X, y, k, 2, w.n_disc, cancel=addr)
    torch.cuda.synchronize()
    full = time.perf_counter() - t0
    print(f"cancel running k={k}: uncancelled call {full * 1e3:.0f} ms", flush=True)
    result = {}

    def run():
        t1 = time.perf_counter()
        try:
            mdfs.mdfs_max_ig(X, y, k, 2, w.n_disc, cancel=addr)
            result["code"] = 0
        except mdfs.MdfsError as exc:
            result["code"] = exc.code
        result["dt"] = time.perf_counter() - t1

    th = threading.Thread(target=run)
    th.start()
    time.sleep(0.15 * full)
    word[0] = 1
    th.join(timeout=60)
    assert not th.is_alive()
    print(f"  cancelled call returned {result['code']} after {result['dt'] * 1e3:.0f} ms", flush=True)
    assert result["code"] == mdfs.E_CANCELLED
    assert result["dt"] < 0.7 * full
    word[0] = 0
    got = mdfs.mdfs_max_ig(X, y, k, 2, w.n_disc, cancel=addr)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
