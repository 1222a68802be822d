"""Serving loop for feature-selection requests: continuous batching on one GPU.

Datasets are uploaded once and stay resident in HBM; a request names a dataset and the sweep
parameters (k, divisions, discretisations, pseudocount, seed).  The server admits queued
requests into free slots while their HBM footprint (the library's workspace plus the outputs)
fits the memory budget, first fit in arrival order (a request passed over too often blocks
later ones until it fits).  Each slot is a host thread with its own HIP stream; the C-ABI call
releases the GIL, so the sweeps of admitted requests run concurrently on the device.
* Every sweep (single or fused) runs the whole-GPU persistent grid by default: a request that
  runs alone is not slowed to a share of the GPU, and concurrent requests share it through the
  hardware dispatcher, which overlaps one request's host work and small kernels with another's
  sweep.  (Grids sized by request, three quarters of the GPU for large ones and an eighth to a
  quarter for small ones, measured 7% less capacity on the serving trace.)
* `express` of the slots take only small requests (at most `fuse_tuples` tuples), so small
  requests never wait behind large ones that occupy the other slots.
* At most `max_large` large requests run at a time (default 1): each fills the GPU by itself, so
  two together only stretch both latencies; queued large ones keep their arrival order and let
  small ones pass.
* Small k = 2 requests waiting behind an admitted small one (same divisions, encoding and engine,
  up to 12, memory permitting) are fused with it into one mdfs_max_ig_batch call: one persistent
  sweep launch over all their tiles.
* Encoded datasets stay resident when discretisation parameters repeat: the second request
  with the same (dataset, divisions, range, seed) has its codes computed once (mdfs_discretize)
  and kept in an LRU cache within `code_cache_bytes`; that and every later such request with at
  most as many discretisations runs mdfs_max_ig_codes on them, skipping the discretisation.
Results do not depend on the mix: every call is deterministic, the persistent grids take all of
their tiles whatever their size, and a sweep from cached codes is bit-identical to the sweep
that discretises.

Host orchestration only: every step of every sweep runs in the library's kernels.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time

import numpy as np
import torch

from . import mdfs


@dataclasses.dataclass
class Request:
    dataset: int
    k: int
    divisions: int
    n_disc: int
    pseudocount: float = 0.25
    range_: float = 0.5
    seed: int = 0
    engine: str = "auto"
    arrival: float = 0.0          # seconds after the start of a trace
    # filled by the server
    id: int = -1
    t_admit: float = math.nan
    t_done: float = math.nan
    footprint: int = 0
    result: tuple | None = None   # (ig_max, argmax, argmax_disc) as numpy arrays
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclasses.dataclass
class Dataset:
    data: torch.Tensor            # float32 [n_var][n_obj] on the device
    y: torch.Tensor               # uint8 [n_obj] on the device
    n1: int = 0                   # objects with y = 1 (counted once, at upload)

    @property
    def n_var(self) -> int:
        return self.data.shape[0]

    @property
    def n_obj(self) -> int:
        return self.data.shape[1]


def tuples_of(ds: Dataset, req: Request) -> int:
    return math.comb(ds.n_var, req.k) * req.n_disc


class Server:
    def __init__(self, device: str = "cuda:0", slots: int = 4, hbm_budget: int | None = None,
                 workgroups: int | None = None, max_bypass: int = 8, fuse: bool = True,
                 fuse_tuples: float = 5e8, express: int | None = None, code_cache_bytes: int = 2 << 30,
                 max_large: int | None = 1):
        mdfs.load()
        self.device = torch.device(device)
        self.slots = slots
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.8 * free)
        self.budget = hbm_budget
        # persistent grid of every sweep (None or 0: the whole GPU)
        self.workgroups = workgroups
        self.max_bypass = max_bypass
        self.fuse = fuse
        self.fuse_tuples = fuse_tuples   # requests up to this many tuples may be fused (and are small)
        self.express = express if express is not None else (1 if slots >= 3 else 0)
        self.max_large = max_large       # large requests running at once (None: no limit)
        self._large = 0                  # large requests running now
        self.n_fused = 0                 # requests that ran inside a fused batch
        self.code_cache_bytes = code_cache_bytes
        self._codes: collections.OrderedDict = collections.OrderedDict()   # key -> codes (LRU)
        self._code_seen: dict = {}       # discretisation key -> requests seen
        self.code_hits = 0               # requests served from cached codes
        self.datasets: dict[int, Dataset] = {}
        self.resident = 0
        self._lock = threading.Condition()
        self._queue: collections.deque[Request] = collections.deque()
        self._in_use = 0
        self._bypassed: dict[int, int] = {}
        self._next_id = 0
        self._closing = False
        self._t0 = time.perf_counter()
        self.done: list[Request] = []
        self._threads = [threading.Thread(target=self._worker, args=(s,), daemon=True) for s in range(slots)]
        self._streams = [torch.cuda.Stream(self.device) for _ in range(slots)]   # default priority
        for th in self._threads:
            th.start()

    # -------------------------------------------------------------- datasets
    def add_dataset(self, data: np.ndarray, y: np.ndarray) -> int:
        """Upload a dataset once; it stays resident until remove_dataset."""
        d = torch.from_numpy(np.ascontiguousarray(data, dtype=np.float32)).to(self.device)
        yy = torch.from_numpy(np.ascontiguousarray(y, dtype=np.uint8)).to(self.device)
        torch.cuda.synchronize(self.device)
        with self._lock:
            did = len(self.datasets)
            while did in self.datasets:
                did += 1
            self.datasets[did] = Dataset(d, yy, int(np.count_nonzero(y)))
            self.resident += d.numel() * 4 + yy.numel()
        return did

    def remove_dataset(self, did: int):
        with self._lock:
            ds = self.datasets.pop(did)
            self.resident -= ds.data.numel() * 4 + ds.y.numel()

    # -------------------------------------------------------------- requests
    def grid_of(self, req: Request) -> int:
        """Persistent workgroups of the request's sweep (0: the whole GPU)."""
        return self.workgroups or 0

    def footprint(self, req: Request) -> int:
        ds = self.datasets[req.dataset]
        prm = mdfs.make_params(ds.n_obj, ds.n_var, req.k, req.divisions, req.n_disc, 0, req.range_,
                               req.pseudocount, req.seed, req.engine, 0, self.grid_of(req))
        ws = mdfs.mdfs_workspace_size(prm)
        return ws + ds.n_var * 4 * (req.k + 1) + 4096

    def submit(self, req: Request) -> Request:
        req.footprint = self.footprint(req)
        if req.footprint + self.resident > self.budget:
            raise ValueError(f"request needs {req.footprint} bytes, more than the HBM budget allows")
        with self._lock:
            req.id = self._next_id
            self._next_id += 1
            self._queue.append(req)
            self._lock.notify_all()
        return req

    def now(self) -> float:
        return time.perf_counter() - self._t0

    def reset_clock(self):
        self._t0 = time.perf_counter()

    def fuse_key(self, req: Request):
        """Requests with equal keys can share one fused sweep launch (None: never fused)."""
        if not self.fuse or req.k != 2 or req.engine == "bitset":
            return None
        ds = self.datasets[req.dataset]
        if tuples_of(ds, req) > self.fuse_tuples:
            return None
        fp4 = max(ds.n1, ds.n_obj - ds.n1) < 4096 and req.engine != "mfma"
        return (req.divisions, fp4, req.engine)

    def _small(self, req: Request) -> bool:
        return tuples_of(self.datasets[req.dataset], req) <= self.fuse_tuples

    def _take(self, express: bool = False) -> list[Request]:
        """First queued request whose footprint fits (an express slot: first small one), and the
        fusable ones queued behind it that also fit (called with the lock held)."""
        free = self.budget - self.resident - self._in_use
        large_full = self.max_large is not None and self._large >= self.max_large
        for idx, req in enumerate(self._queue):
            if (express or large_full) and not self._small(req):
                continue
            if req.footprint <= free:
                for earlier in list(self._queue)[:idx]:
                    self._bypassed[earlier.id] = self._bypassed.get(earlier.id, 0) + 1
                del self._queue[idx]
                self._bypassed.pop(req.id, None)
                group = [req]
                key = self.fuse_key(req)
                if key is not None:
                    free -= req.footprint
                    for later in list(self._queue)[idx:]:
                        if len(group) == 12:
                            break
                        if self.fuse_key(later) == key and later.footprint <= free:
                            self._queue.remove(later)
                            self._bypassed.pop(later.id, None)
                            group.append(later)
                            free -= later.footprint
                return group
            if self._bypassed.get(req.id, 0) >= self.max_bypass:
                return []   # this one waits for memory; nobody passes it any more
        return []

    def _worker(self, slot: int):
        stream = self._streams[slot]
        express = slot < self.express
        while True:
            with self._lock:
                group = []
                while not group:
                    if self._closing and not self._queue:
                        return
                    group = self._take(express)
                    if not group:
                        self._lock.wait()
                now = self.now()
                large = len(group) == 1 and not self._small(group[0])
                self._large += large
                for req in group:
                    self._in_use += req.footprint
                    req.t_admit = now
            if len(group) == 1:
                try:
                    self._run(group[0], stream)
                except Exception as exc:   # reported on the request, the server keeps serving
                    group[0].error = f"{type(exc).__name__}: {exc}"
            else:
                self._run_fused(group, stream)
            with self._lock:
                now = self.now()
                self._large -= large
                for req in group:
                    self._in_use -= req.footprint
                    req.t_done = now
                    self.done.append(req)
                if len(group) > 1:
                    self.n_fused += len(group)
                self._lock.notify_all()

    def _cached_codes(self, req: Request, ws: torch.Tensor, stream: torch.cuda.Stream):
        """Resident codes for the request's discretisations, or None.  A discretisation key seen
        for the second time is encoded once (mdfs_discretize) and kept, LRU, within the budget."""
        ds = self.datasets[req.dataset]
        key = (req.dataset, req.divisions, req.range_, req.seed)
        with self._lock:
            hit = self._codes.get(key)
            if hit is not None and hit.shape[0] >= req.n_disc:
                self._codes.move_to_end(key)
                self.code_hits += 1
                return hit[:req.n_disc]
            self._code_seen[key] = self._code_seen.get(key, 0) + 1
            if self._code_seen[key] < 2:
                return None
        nbytes = req.n_disc * ds.n_var * ds.n_obj
        if nbytes > self.code_cache_bytes:
            return None
        codes = mdfs.mdfs_discretize(ds.data, req.divisions, req.n_disc, req.range_, req.seed, k=req.k, ws=ws,
                                     stream=stream)
        with self._lock:
            self._codes[key] = codes
            while sum(c.numel() for c in self._codes.values()) > self.code_cache_bytes:
                self._codes.popitem(last=False)
            self.code_hits += 1
        return codes

    def _run(self, req: Request, stream: torch.cuda.Stream):
        ds = self.datasets[req.dataset]
        grid = self.grid_of(req)
        with torch.cuda.stream(stream):
            prm = mdfs.make_params(ds.n_obj, ds.n_var, req.k, req.divisions, req.n_disc, 0, req.range_,
                                   req.pseudocount, req.seed, req.engine, 0, grid)
            ws = torch.empty(mdfs.mdfs_workspace_size(prm), dtype=torch.uint8, device=self.device)
            codes = self._cached_codes(req, ws, stream) if req.k >= 2 else None
            if codes is not None:
                ig, am, ad = mdfs.mdfs_max_ig_codes(codes, ds.y, req.k, req.divisions, req.pseudocount, 0,
                                                    engine=req.engine, workgroups=grid, ws=ws, stream=stream)
            else:
                ig, am, ad = mdfs.mdfs_max_ig(ds.data, ds.y, req.k, req.divisions, req.n_disc, req.pseudocount,
                                              req.range_, req.seed, 0, engine=req.engine, workgroups=grid, ws=ws,
                                              stream=stream)
            req.result = (ig.cpu().numpy(), am.cpu().numpy(), ad.cpu().numpy())
            del ws

    def _run_fused(self, group: list[Request], stream: torch.cuda.Stream):
        """One mdfs_max_ig_batch call for the group; each request gets its own status."""
        dss = [self.datasets[r.dataset] for r in group]
        try:
            with torch.cuda.stream(stream):
                outs, wss = mdfs.mdfs_max_ig_batch(
                    [d.data for d in dss], [d.y for d in dss], [d.n1 for d in dss], 2, group[0].divisions,
                    [r.n_disc for r in group], [r.pseudocount for r in group], [r.range_ for r in group],
                    [r.seed for r in group], engine=group[0].engine,
                    workgroups=self.workgroups or 0)
                for r, d, (ig, am, ad), ws in zip(group, dss, outs, wss):
                    try:
                        mdfs.mdfs_check_status((d.n_var, d.n_obj), 2, r.divisions, r.n_disc, ws=ws, engine=r.engine)
                        r.result = (ig.cpu().numpy(), am.cpu().numpy(), ad.cpu().numpy())
                    except Exception as exc:
                        r.error = f"{type(exc).__name__}: {exc}"
        except Exception as exc:   # the whole call was refused: every request reports it
            for r in group:
                r.error = f"{type(exc).__name__}: {exc}"

    def wait_all(self, n: int, timeout: float | None = None):
        """Block until n requests have finished."""
        with self._lock:
            ok = self._lock.wait_for(lambda: len(self.done) >= n, timeout)
        if not ok:
            raise TimeoutError(f"{len(self.done)} of {n} requests finished")

    def close(self):
        with self._lock:
            self._closing = True
            self._lock.notify_all()
        for th in self._threads:
            th.join()


def run_trace(server: Server, reqs: list[Request], timeout: float = 600.0) -> dict:
    """Submit requests at their arrival times (seconds from now) and wait for all of them.
    Returns latency percentiles and throughput over the makespan."""
    server.done.clear()
    server.reset_clock()
    for req in sorted(reqs, key=lambda r: r.arrival):
        delay = req.arrival - server.now()
        if delay > 0:
            time.sleep(delay)
        server.submit(req)
    server.wait_all(len(reqs), timeout)
    bad = [r for r in reqs if r.error]
    if bad:
        raise RuntimeError(f"{len(bad)} requests failed, first: {bad[0].error}")
    lat = np.array([r.latency for r in reqs])
    makespan = max(r.t_done for r in reqs) - min(r.arrival for r in reqs)
    tuples = sum(tuples_of(server.datasets[r.dataset], r) for r in reqs)
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "makespan_s": makespan, "tuples": tuples, "tuples_per_s": tuples / makespan}
