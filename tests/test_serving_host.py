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
    srv.budget, srv.resident, srv._in_use, srv.max_bypass, srv.fuse = 100, 10, 0, 2, False
    srv._bypassed, srv.max_large, srv._large = {}, None, 0
    import collections
    srv._queue = collections.deque([Req(0, 95), Req(1, 30), Req(2, 50)])
    ids = lambda g: [r.id for r in g]   # noqa: E731
    assert ids(srv._take()) == [1]      # 95 does not fit in 90, 30 does
    srv._in_use = 30
    assert ids(srv._take()) == [2]      # 50 fits in 60
    srv._in_use = 80
    srv._queue.append(Req(3, 5))
    assert srv._take() == []            # request 0 was passed over twice: it now blocks
    srv._in_use = 0
    assert srv._take() == []            # 95 > 100 - 10 resident: still waiting
    srv.resident = 0
    assert ids(srv._take()) == [0]


def test_fusion_groups_small_k2_requests():
    # small k = 2 requests with the same divisions and encoding queued behind the admitted one
    # join it (memory permitting, at most 12); others keep their place
    from paper_1811_00631_amd.serving import Dataset, Request, Server
    import collections

    srv = Server.__new__(Server)
    srv.budget, srv.resident, srv._in_use, srv.max_bypass = 1000, 0, 0, 8
    srv.fuse, srv.fuse_tuples, srv._bypassed = True, 5e8, {}
    srv.max_large, srv._large = 1, 0
    small = Dataset.__new__(Dataset)
    big = Dataset.__new__(Dataset)
    for ds, (p, n, n1) in ((small, (100, 500, 250)), (big, (20000, 2000, 1000))):
        object.__setattr__(ds, "data", np.zeros((p, n)))
        object.__setattr__(ds, "n1", n1)
    srv.datasets = {0: small, 1: big}

    def req(i, ds, k=2, div=2, fp=10):
        r = Request(dataset=ds, k=k, divisions=div, n_disc=3)
        r.id, r.footprint = i, fp
        return r
    srv._queue = collections.deque([req(0, 0), req(1, 1), req(2, 0, div=1), req(3, 0, k=3), req(4, 0)] +
                                   [req(5 + i, 0) for i in range(14)])
    g = srv._take()
    assert [r.id for r in g] == [0, 4] + list(range(5, 15))     # 12: same key, small
    assert [r.id for r in srv._queue][:3] == [1, 2, 3]           # big, other divisions, k = 3 wait
    srv._queue = collections.deque([req(20, 0, fp=600), req(21, 0, fp=500), req(22, 0, fp=300)])
    assert [r.id for r in srv._take()] == [20, 22]               # 500 no longer fits next to 600


def test_one_large_request_at_a_time():
    # with a large request running, queued large ones wait in arrival order and small ones pass;
    # express slots take small ones only; without the limit the next large one is taken
    from paper_1811_00631_amd.serving import Dataset, Request, Server
    import collections

    srv = Server.__new__(Server)
    srv.budget, srv.resident, srv._in_use, srv.max_bypass = 1000, 0, 0, 2
    srv.fuse, srv.fuse_tuples, srv._bypassed = False, 5e8, {}
    small = Dataset.__new__(Dataset)
    big = Dataset.__new__(Dataset)
    for ds, (p, n, n1) in ((small, (100, 500, 250)), (big, (20000, 2000, 1000))):
        object.__setattr__(ds, "data", np.zeros((p, n)))
        object.__setattr__(ds, "n1", n1)
    srv.datasets = {0: small, 1: big}

    def req(i, ds):
        r = Request(dataset=ds, k=2, divisions=2, n_disc=3)
        r.id, r.footprint = i, 10
        return r
    ids = lambda g: [r.id for r in g]   # noqa: E731
    srv.max_large, srv._large = 1, 0
    srv._queue = collections.deque([req(0, 1), req(1, 1), req(2, 0)])
    assert ids(srv._take(express=True)) == [2]
    assert ids(srv._take()) == [0]
    srv._large = 1                                   # request 0 runs
    srv._queue.extend([req(3, 0), req(4, 0), req(5, 0)])
    assert ids(srv._take()) == [3] and ids(srv._take()) == [4] and ids(srv._take()) == [5]
    assert srv._take() == []                         # request 1 waits for the large slot
    srv._large = 0
    assert ids(srv._take()) == [1]                   # passed over, still first among the large
    srv.max_large, srv._large = None, 1
    srv._queue = collections.deque([req(6, 1)])
    assert ids(srv._take()) == [6]


def test_autotune_candidates_and_buckets():
    from paper_1811_00631_amd import autotune
    c2 = autotune.candidates(2000, 2, 2, 1000)
    assert {c["engine"] for c in c2} == {"mfma_fp4", "mfma"}
    assert {c["engine"] for c in autotune.candidates(9000, 2, 2, 4500)} == {"mfma"}   # classes >= 4096
    assert {c["engine"] for c in autotune.candidates(2000, 3, 2, 1000)} == {"mfma_fp4", "bitset"}
    assert {c["engine"] for c in autotune.candidates(2000, 3, 4, 1000)} == {"bitset"}
    # k = 4: bitsets (two or three classes) or histograms; k = 5: bitsets (two classes) or histograms
    assert {c["engine"] for c in autotune.candidates(2000, 4, 2, 1000)} == {"bitset", "hist"}
    assert {c["engine"] for c in autotune.candidates(2000, 4, 4, 1000)} == {"hist"}
    assert {c["engine"] for c in autotune.candidates(2000, 5, 1, 1000)} == {"bitset", "hist"}
    assert {c["engine"] for c in autotune.candidates(2000, 5, 2, 1000)} == {"hist"}
    # k = 2 launch shapes: super-tiles 4, 8, 16; with three classes 8 or 4 waves too
    shapes = {(c["tile"] & 0xff, c["tile"] >> 8) for c in c2}
    assert shapes == {(sb, nw) for sb in (4, 8, 16) for nw in (8, 4)}
    assert {c["tile"] >> 8 for c in autotune.candidates(2000, 2, 1, 1000)} == {0}
    assert all(c["tile"] == 0 for c in autotune.candidates(2000, 3, 2, 1000))
    assert all(c["workgroups"] % 8 == 0 and 8 <= c["workgroups"] <= 4096 for c in c2)
    assert autotune.bucket(2000, 20000, 2, 2, 30) == (2048, 32768, 2, 2, 4)
    assert autotune.bucket(1025, 100, 3, 1, 1) == (2048, 128, 3, 1, 1)
