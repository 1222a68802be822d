"""Host logic of the serving loop (no GPU): the trace generator and first-fit admission."""
import math

import numpy as np

from paper_1811_00631_amd import workloads


def test_serving_trace_shape():
    ds = workloads.serving_datasets(seed=6, n_datasets=8)
    rq = workloads.serving_requests(ds, seed=6, n_requests=64, rate_hz=2.0)
    assert len(rq) == 64
    arr = np.array([r["arrival"] for r in rq])
    assert np.all(np.diff(arr) > 0)
    for X, y, meta in ds:
        assert 100 <= X.shape[1] <= 5000 and 100 <= X.shape[0] <= 20000
        assert set(np.unique(y)) <= {0, 1} and y.min() != y.max()
    for r in rq:
        assert r["k"] in (2, 3) and r["divisions"] in (1, 2, 4) and 1 <= r["n_disc"] <= 30
        if r["k"] == 3:
            assert ds[r["dataset"]][0].shape[0] <= 1000


def test_first_fit_admission_order():
    # the admission rule, replayed on plain numbers: take the first queued request that fits;
    # one passed over max_bypass times blocks the rest until it fits
    class Req:
        def __init__(self, i, f):
            self.id, self.footprint = i, f

    from paper_1811_00631_amd.serving import Server
    srv = Server.__new__(Server)
    srv.budget, srv.resident, srv._in_use, srv.max_bypass = 100, 10, 0, 2
    srv._bypassed = {}
    import collections
    srv._queue = collections.deque([Req(0, 95), Req(1, 30), Req(2, 50)])
    assert srv._take().id == 1          # 95 does not fit in 90, 30 does
    srv._in_use = 30
    assert srv._take().id == 2          # 50 fits in 60
    srv._in_use = 80
    srv._queue.append(Req(3, 5))
    assert srv._take() is None          # request 0 was passed over twice: it now blocks
    srv._in_use = 0
    assert srv._take() is None          # 95 > 100 - 10 resident: still waiting
    srv.resident = 0
    assert srv._take().id == 0


def test_autotune_candidates_and_buckets():
    from paper_1811_00631_amd import autotune
    c2 = autotune.candidates(2000, 2, 2, 1000)
    assert {c["engine"] for c in c2} == {"mfma_fp4", "mfma"}
    assert {c["engine"] for c in autotune.candidates(9000, 2, 2, 4500)} == {"mfma"}   # classes >= 4096
    assert {c["engine"] for c in autotune.candidates(2000, 3, 2, 1000)} == {"mfma_fp4", "bitset"}
    assert {c["engine"] for c in autotune.candidates(2000, 3, 4, 1000)} == {"bitset"}
    assert all(c["workgroups"] % 8 == 0 and 8 <= c["workgroups"] <= 4096 for c in c2)
    assert autotune.bucket(2000, 20000, 2, 2, 30) == (2048, 32768, 2, 2, 4)
    assert autotune.bucket(1025, 100, 3, 1, 1) == (2048, 128, 3, 1, 1)
