#!/usr/bin/env python
"""Throughput of the MDFS k-tuple information-gain sweep on one MI355X.

One step = one mdfs_max_ig call over the whole problem (discretise all variables under every
random discretisation, count every pair's per-class table, float32 entropy screen, binary64
re-score, per-variable max/argmax), with the data and the decision already resident in HBM.

Workload (the throughput metric's shape): k = 2, N = 2000 objects, p = 20000 log-normal
variables with 10 planted XOR pairs, balanced binary decision, 3 classes per variable,
30 random discretisations -> C(20000, 2) * 30 = 6.0e9 pair tables per step.

Prints one JSON line.  Extra keys: p50/p99 step latency, per-phase times from HIP events on the
launch stream, the roofline of the dominant kernel (the pair sweep) and the FP64 oracle timed on
the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0        # MI355X dense int8 MFMA, TOP/s
FP4_PEAK_TFLOPS = 10100.0      # MI355X dense fp4 (and fp6) MFMA, TFLOP/s
HBM_PEAK_GBS = 8000.0
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 256 CUs x 64 lanes/clk x 2.4 GHz integer VALU = 39.3 Tops/s
LDS_PEAK_GBS = 256 * 128 * 2.4e9 / 1e9   # 256 CUs x 128 bytes/clk x 2.4 GHz = 78.6 TB/s
EPILOGUE_OPS_PER_VOXEL = 18               # VALU lane-ops per voxel term of the entropy screen (estimate)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-vars", type=int, default=2000, help="variables in the oracle's sample")
    ap.add_argument("--cpu-disc", type=int, default=30, help="discretisations in the oracle's sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--autotune", action="store_true",
                    help="pick engine and persistent grid size with the autotuner (cached per shape)")
    ap.add_argument("--engine", default="auto", choices=["auto", "mfma_fp4", "mfma", "bitset"],
                    help="auto: fp4 MFMA for k=2 and for k=3 at d=2 or 3 while each class has < 4096 objects, else int8 MFMA (k=2) or bitsets")
    ap.add_argument("--graph", action="store_true",
                    help="each step replays a CUDA graph of one asynchronous call (no host synchronisation)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "sweep2_headline_traffic.json"))
    ap.add_argument("--workload", default="headline", choices=sorted(WORKLOADS),
                    help="headline is the metric's workload; the others print informational lines")
    return ap.parse_args()


def _wl(name):
    from paper_1811_00631_amd import workloads
    return {"headline": workloads.headline, "xor_small": workloads.xor_small,
            "madelon_like": workloads.madelon_like, "parity3": workloads.parity3,
            "genomics_like": workloads.genomics_like,
            "madelon4": lambda: workloads.madelon_like(divisions=1, n_disc=1, k=4),
            "madelon5": lambda: workloads.madelon_like(divisions=1, n_disc=1, k=5),
            "madelon4_d5": lambda: workloads.madelon_like(divisions=4, n_disc=1, k=4, n_noise=180),
            "madelon2_d2": lambda: workloads.madelon_like(divisions=1, n_disc=30, k=2),
            "madelon3_d2": lambda: workloads.madelon_like(divisions=1, n_disc=30, k=3)}[name]()


WORKLOADS = ["headline", "xor_small", "madelon_like", "parity3", "genomics_like", "madelon4", "madelon5",
             "madelon4_d5", "madelon2_d2", "madelon3_d2", "batch12", "batch12_k3", "serving"]
WORKLOAD_TEXT = {
    "headline": "genomics-shaped k=2: N=2000, p=20000 log-normal, 10 planted XOR pairs, balanced y, d=3, "
                "30 random discretisations (range 0.5, xi 0.25)",
    "xor_small": "k=2: N=500, p=100 Gaussian, XOR pair (0,1) with 10% label noise, d=3, 1 discretisation",
    "madelon_like": "Madelon-shaped k=2: N=2000, p=500 (5 base + 15 combinations + 480 noise), d=3, 30 discretisations",
    "parity3": "k=3: N=2000, p=500 Gaussian, parity triple (0,1,2), d=3, 30 discretisations",
    "genomics_like": "genomics-shaped k=2: N=500, p=20000 log-normal, 10 planted XOR pairs, y 200/300, d=3, "
                     "30 discretisations",
    "madelon4": "Madelon-shaped k=4: N=2000, p=500 (5 base + 15 combinations + 480 noise), d=2, 1 discretisation "
                "(the shape of the paper's 4D timing)",
    "madelon5": "Madelon-shaped k=5: N=2000, p=500 (5 base + 15 combinations + 480 noise), d=2, 1 discretisation "
                "(the shape of the paper's 5D timing)",
    "madelon4_d5": "Madelon-shaped k=4 with five classes: N=2000, p=200 (5 base + 15 combinations + 180 noise), "
                   "1 discretisation, histogram engine",
    "madelon2_d2": "Madelon-shaped k=2: N=2000, p=500, d=2, 30 discretisations (the shape of the paper's 2D timing)",
    "madelon3_d2": "Madelon-shaped k=3: N=2000, p=500, d=2, 30 discretisations (the shape of the paper's 3D timing)",
    "batch12": "12 Madelon-shaped k=2 datasets of uneven size (N 500-2000, p 200-600), d=3, 30 discretisations each: "
               "one fused persistent launch vs separate calls",
    "batch12_k3": "12 Madelon-shaped k=3 datasets of uneven size (N 500-2000, p 60-200), d=3, 30 discretisations "
                  "each: one batched call (each dataset on one of four concurrent streams) vs separate calls",
    "serving": "serving trace: 256 requests, Poisson arrivals at 0.8 x the measured batched capacity, 32 resident "
               "datasets N~logU[100,5000], p~logU[100,20000] (k=3 requests on datasets with p<=1000), "
               "k in {2,3}, d in {2,3,5}, 1-30 discretisations, Gaussian data with planted XOR pairs",
}


def _sweep_source_hash():
    import hashlib
    src = os.path.join(ROOT, "paper_1811_00631_amd", "csrc", "sweep2.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def host_threads() -> int:
    """Host threads the oracle may use: the machine's CPU share (OMP_NUM_THREADS there), else nproc."""
    return max(1, min(int(os.environ.get("OMP_NUM_THREADS", str(os.cpu_count() or 1))), os.cpu_count() or 1))


def cpu_baseline(w, k, n_vars, n_disc, ig_gpu, argmax_gpu, disc_gpu, gpu_on_sample=None):
    """The FP64 oracle timed on the host cores on a bounded sample of the same workload: the
    tuple-sweep form (threads over discretisations) on the first n_vars variables and n_disc
    discretisations, on every host thread and on one core.  Also the per-result IG error of the
    GPU outputs: against the stored oracle values of every variable (tests/golden, when the
    regenerated inputs hash to the stored digest), else against the per-variable oracle on a
    sample of variables holding every planted one; for k >= 4 (where the per-variable oracle over
    all p variables is out of reach) against the timed oracle run itself, with the GPU run on the
    same sample (`gpu_on_sample`)."""
    import numpy as np

    import oracle
    threads = min(host_threads(), n_disc)
    data = w.data[:n_vars]
    t0 = time.perf_counter()
    sample_ref = oracle.max_ig_all(data, w.y, k, w.divisions, n_disc, w.range_, w.xi, w.seed, n_threads=threads)
    dt = time.perf_counter() - t0
    tuples = math.comb(n_vars, k) * n_disc
    # one core: a quarter of the variables, two discretisations
    n1v, n1d = max(k + 1, n_vars // 4), min(2, n_disc)
    t0 = time.perf_counter()
    oracle.max_ig_all(w.data[:n1v], w.y, k, w.divisions, n1d, w.range_, w.xi, w.seed, n_threads=1)
    dt1 = time.perf_counter() - t0
    tuples1 = math.comb(n1v, k) * n1d
    out = {"value": tuples / dt, "unit": "k-tuples evaluated/sec", "cores": threads, "kind": "oracle",
           "sample": f"first {n_vars} of {w.n_var} variables, {n_disc} of {w.n_disc} discretisations, "
                     f"N={w.n_obj}, k={k}, d={w.divisions + 1}: {tuples} tuple tables in {dt:.2f} s",
           "single_core": {"value": tuples1 / dt1, "cores": 1,
                           "sample": f"first {n1v} variables, {n1d} discretisations: {tuples1} tuple tables "
                                     f"in {dt1:.2f} s"}}
    # per-result IG error of the GPU outputs (outside the timed region)
    ref, where = None, ""
    try:
        sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
        import make_fullsize
        name = {"headline": "headline", "genomics_like": "genomics_like", "madelon_like": "madelon_like",
                "parity3": "parity3", "madelon2_d2": "madelon2_d2", "madelon3_d2": "madelon3_d2"}.get(w.name_key)
        if name and os.path.exists(make_fullsize.path_of(name)):
            z = make_fullsize.load(name)
            if str(z["digest"]) == make_fullsize.data_digest(w) and int(z["k"]) == k:
                tg = np.arange(w.n_var)
                ref = (z["ig"], z["argmax"].astype(np.int64), z["disc"].astype(np.int64))
                where = "stored oracle values of every variable (tests/golden)"
    except Exception as exc:   # the stored values are optional
        print(f"# stored oracle values unavailable: {exc}", file=sys.stderr)
    if ref is None and gpu_on_sample is not None:
        ig_gpu, argmax_gpu, disc_gpu = gpu_on_sample(n_vars, n_disc)
        tg = np.arange(n_vars)
        ref = tuple(np.asarray(x) for x in sample_ref)
        where = f"the timed oracle run (first {n_vars} variables, {n_disc} discretisations) against the GPU on the same"
    if ref is None:
        g = np.random.default_rng(0)
        planted = sorted({int(v) for pr in w.planted.get("pairs", []) for v in pr} |
                         {int(v) for v in w.planted.get("triple", [])})
        rest = np.setdiff1d(np.arange(w.n_var), planted)
        tg = np.array(sorted(planted + g.choice(rest, min(len(rest), 12), replace=False).tolist()))
        ref = oracle.max_ig(w.data, w.y, k, w.divisions, w.n_disc, w.range_, w.xi, w.seed, targets=tg,
                            n_threads=host_threads())
        where = f"per-variable oracle on {len(tg)} variables (every planted one)"
    ig = np.asarray(ig_gpu, dtype=np.float64)[tg]
    err = np.abs(ig - ref[0])
    out["ig_error"] = {"max_rel_floor1": float((err / np.maximum(np.abs(ref[0]), 1.0)).max()),
                       "max_rel": float((err / np.maximum(np.abs(ref[0]), 1e-300)).max()),
                       "max_abs": float(err.max()), "tolerance": 1e-4, "vars": int(len(tg)),
                       "argmax_equal": int(((np.asarray(argmax_gpu)[tg] == ref[1]).all(axis=1) &
                                            (np.asarray(disc_gpu)[tg] == ref[2])).sum()),
                       "reference": where}
    return out


def batch_bench(args):
    """Several datasets: separate synchronous calls, separate asynchronous calls, one fused call
    (mdfs_max_ig_batch: one persistent sweep launch over all their tiles), and the fused call
    replayed as a captured graph.  Every variant's outputs are checked equal."""
    import numpy as np
    import torch

    from paper_1811_00631_amd import mdfs, workloads
    dev = torch.device("cuda:0")
    g = np.random.default_rng(12)
    k = 3 if args.workload == "batch12_k3" else 2
    lo, hi = (60, 201) if k == 3 else (200, 601)
    shapes = [(int(g.integers(500, 2001)), int(g.integers(lo, hi))) for _ in range(12)]
    ws_ = [workloads.madelon_like(seed=30 + i, n_obj=n, n_noise=p - 20) for i, (n, p) in enumerate(shapes)]
    D = [torch.from_numpy(w.data).to(dev) for w in ws_]
    Y = [torch.from_numpy(w.y).to(dev) for w in ws_]
    n1 = [int(w.y.sum()) for w in ws_]
    R = 30
    tuples = sum(math.comb(w.n_var, k) * R for w in ws_)

    def separate():
        return [mdfs.mdfs_max_ig(D[i], Y[i], k, 2, R, 0.25, 0.5, i) for i in range(12)]

    def separate_async():
        return [mdfs.mdfs_max_ig_async(D[i], Y[i], n1[i], k, 2, R, 0.25, 0.5, i,
                                       ws=torch.empty(mdfs.mdfs_workspace_size(mdfs.make_params(
                                           D[i].shape[1], D[i].shape[0], k, 2, R, 0, 0.5, 0.25, i)),
                                           dtype=torch.uint8, device=dev)) for i in range(12)]

    def fused():
        return mdfs.mdfs_max_ig_batch(D, Y, n1, k, 2, [R] * 12, 0.25, 0.5, list(range(12)))[0]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fused()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gout = fused()

    def graphed():
        graph.replay()
        return gout

    ref = separate()
    res = {}
    for name, fn in (("separate", separate), ("separate_async", separate_async), ("fused", fused), ("fused_graph", graphed)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        for a, b in zip(ref, out):
            if not all(torch.equal(u, v) for u, v in zip(a, b)):
                raise RuntimeError(f"{name}: results differ from separate calls")
        res[name] = ms
        print(f"# {name}: {ms:.3f} ms per batch of 12", file=sys.stderr, flush=True)
    line = {
        "metric": f"k-tuples evaluated/sec (12 k={k} datasets per batch, informational)",
        "value": tuples / (res["fused"] * 1e-3), "unit": "k-tuples evaluated/sec",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["fused"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp4 (E2M1 one-hot), f32 accumulate", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "shapes": shapes, "n_disc": R, "tuples_per_step": tuples},
        "ms_per_batch": res,
        "tuples_per_s": {k: tuples / (v * 1e-3) for k, v in res.items()},
    }
    print(json.dumps(line))


def serving_bench(args):
    """The serving trace: capacities (requests back to back) of the plain one-at-a-time sweep
    and of continuous batching (4 slots), then Poisson arrivals at 0.8 x the batched capacity
    served both ways."""
    import numpy as np
    from paper_1811_00631_amd import serving, workloads

    ds = workloads.serving_datasets()
    base = workloads.serving_requests(ds, n_requests=args.serve_requests)
    print(f"# serving: {len(ds)} datasets, {len(base)} requests", file=sys.stderr, flush=True)

    def make(srv, ids, rate):
        out = []
        for r in base:
            q = serving.Request(dataset=ids[r["dataset"]], k=r["k"], divisions=r["divisions"], n_disc=r["n_disc"],
                                seed=r["seed"], arrival=r["arrival"] * (1.0 / rate if rate else 0.0))
            out.append(q)
        return out

    def session(slots, rate, fuse):
        srv = serving.Server(slots=slots, fuse=fuse)
        try:
            ids = [srv.add_dataset(X, y) for X, y, _ in ds]
            # warm-up: one small request per engine path
            serving.run_trace(srv, make(srv, ids, 0)[:4], timeout=600)
            reqs = make(srv, ids, rate)
            srv.n_fused = 0
            st = serving.run_trace(srv, reqs, timeout=900)
            st["fused_requests"] = srv.n_fused
            print(f"# serving slots={slots} fuse={fuse} rate={rate}: {st}", file=sys.stderr, flush=True)
            return st, reqs
        finally:
            srv.close()

    plain_cap, _ = session(1, 0, False)                 # back to back, one at a time: the plain sweep
    batch_cap, _ = session(4, 0, True)                  # back to back: 4 slots and fused small requests
    rate = 0.8 * len(base) / batch_cap["makespan_s"]   # requests/s; base arrivals are at rate 1
    mixed, _ = session(4, rate, True)
    plain, _ = session(1, rate, False)
    line = {
        "metric": "serving: k-tuples evaluated/sec over the trace; p50/p99 request latency",
        "value": mixed["tuples_per_s"], "unit": "k-tuples evaluated/sec", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": mixed["makespan_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "mixed (fp4/int8 MFMA, bitsets)", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["serving"], "requests": len(base), "arrival_rate_hz": rate,
                   "slots": 4, "fused_requests": mixed["fused_requests"]},
        "p50_ms": mixed["p50_ms"], "p99_ms": mixed["p99_ms"],
        "plain_sweep_same_arrivals": {"tuples_per_s": plain["tuples_per_s"], "p50_ms": plain["p50_ms"],
                                      "p99_ms": plain["p99_ms"]},
        "plain_sweep_capacity_tuples_per_s": plain_cap["tuples_per_s"],
        "batched_capacity_tuples_per_s": batch_cap["tuples_per_s"],
        "total_tuples": mixed["tuples"],
    }
    print(json.dumps(line))


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); multi-GPU sharding of the tuple "
              "space is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1811_00631_amd import mdfs, workloads

    mdfs.load()
    if args.workload == "serving":
        serving_bench(args)
        return
    if args.workload in ("batch12", "batch12_k3"):
        batch_bench(args)
        return
    dev = torch.device("cuda:0")
    w = _wl(args.workload)
    w.name_key = args.workload
    data = torch.from_numpy(w.data).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    k, div, R = w.k, w.divisions, w.n_disc
    tuples = math.comb(w.n_var, k) * R

    workgroups, tile, tuned = 0, 0, None
    if args.autotune:
        from paper_1811_00631_amd import autotune
        tuned = autotune.Tuner(os.path.join(ROOT, "gpurun_out", "autotune.json")).best(w.n_obj, w.n_var, k, div, R)
        args.engine, workgroups, tile = tuned["engine"], tuned["workgroups"], tuned.get("tile", 0)
        print(f"# autotune: {tuned['engine']} x {workgroups} workgroups, tile 0x{tile:x}", file=sys.stderr,
              flush=True)

    def step():
        return mdfs.mdfs_max_ig(data, y, k, div, R, w.xi, w.range_, w.seed, engine=args.engine, timing=True,
                                workgroups=workgroups, tile=tile)

    graph = None
    if args.graph:
        # one asynchronous call captured once; a step is one replay (inputs stay in HBM)
        n1 = int(w.y.sum())
        prm = mdfs.make_params(w.n_obj, w.n_var, k, div, R, 0, w.range_, w.xi, w.seed, args.engine, 0, workgroups,
                               tile=tile)
        gws = torch.empty(mdfs.mdfs_workspace_size(prm), dtype=torch.uint8, device=dev)
        gout = (torch.empty(w.n_var, dtype=torch.float32, device=dev),
                torch.empty((w.n_var, k - 1), dtype=torch.int32, device=dev),
                torch.empty(w.n_var, dtype=torch.int32, device=dev))
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            mdfs.mdfs_max_ig_async(data, y, n1, k, div, R, w.xi, w.range_, w.seed, engine=args.engine,
                                   workgroups=workgroups, ws=gws, out=gout, tile=tile)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            mdfs.mdfs_max_ig_async(data, y, n1, k, div, R, w.xi, w.range_, w.seed, engine=args.engine,
                                   workgroups=workgroups, ws=gws, out=gout, tile=tile)
        ref = step()

        def step():   # noqa: F811
            graph.replay()
            return gout

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat, phases = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        out = step()
        if graph is not None:
            torch.cuda.synchronize()   # per-step latency; the timed region is synchronised anyway
        lat.append(time.perf_counter() - s0)
        if graph is None:
            phases.append(mdfs.mdfs_phase_times())
        print(f"# step {len(lat)}/{args.steps}: {lat[-1] * 1e3:.2f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    if graph is not None:
        mdfs.mdfs_check_status((w.n_var, w.n_obj), k, div, R, ws=gws, engine=args.engine)
        if not all(torch.equal(a, b) for a, b in zip(out, ref)):
            raise RuntimeError("graph replay differs from the synchronous call")
        # phase times come from the synchronous call (same kernels)
        step_sync = lambda: mdfs.mdfs_max_ig(data, y, k, div, R, w.xi, w.range_, w.seed, engine=args.engine,  # noqa: E731
                                             timing=True, workgroups=workgroups, tile=tile)
        step_sync()
        phases.append(mdfs.mdfs_phase_times())

    ig, am, _ = out
    if "pairs" in w.planted:
        found = f"{sum(int(am[a, 0]) == b for a, b in w.planted['pairs'])}/{len(w.planted['pairs'])}"
    elif "triple" in w.planted:
        found = f"{sum(am[v].tolist() == [u for u in w.planted['triple'] if u != v] for v in w.planted['triple'])}/3"
    elif "base" in w.planted:
        top = set(np.argsort(-ig.cpu().numpy())[:20].tolist())
        found = f"{len(top & set(w.planted['base']))}/{len(w.planted['base'])} base features in the top 20"
    elif "xor_pair" in w.planted:
        found = f"{int(int(am[0, 0]) == 1) + int(int(am[1, 0]) == 0)}/2"
    else:
        found = "n/a"

    if args.copy_calib:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    ph = {name: float(np.mean([p[name] for p in phases])) for name in phases[0]}
    sweep_ms = ph["sweep"]
    W = div
    n0, n1 = int((w.y == 0).sum()), int((w.y == 1).sum())
    fp4 = args.engine == "mfma_fp4" or (args.engine == "auto" and max(n0, n1) < 4096)
    fp4 = fp4 and (k == 2 or (k == 3 and div in (1, 2)))
    k3_mfma = k == 3 and fp4
    C = div + 1
    if k in (2, 3) and (k == 2 or k3_mfma):
        # algorithmic work: N voxel increments per tuple table, each counted as one multiply-add
        # (2 ops); the engine executes 2 N (d-1)^k ops (a one-hot contraction over every bin of
        # the first d-1, the last rebuilt from marginals)
        alg_per_unit = 2 * w.n_obj
        exe_per_unit = 2 * w.n_obj * W ** k
        achieved = tuples * alg_per_unit / (sweep_ms * 1e-3) / 1e12
        executed = tuples * exe_per_unit / (sweep_ms * 1e-3) / 1e12
        peak = FP4_PEAK_TFLOPS if fp4 else INT8_PEAK_TOPS
        unit = "TFLOP/s" if fp4 else "TOP/s"
        # the float32 entropy screen: C^k voxel terms per tuple table on the vector ALUs
        epi_rate = ALU_PEAK_TOPS * 1e12 / (C ** k * EPILOGUE_OPS_PER_VOXEL)
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                "per_unit": f"2*N = {alg_per_unit} ops per {'pair' if k == 2 else 'triple'} table "
                            f"(N voxel increments, one multiply-add each)",
                "executed": {"achieved": executed, "frac": executed / peak,
                             "per_unit": f"2*N*(d-1)^{k} = {exe_per_unit} {'fp4' if fp4 else 'int8'} MFMA ops"},
                "epilogue_ceiling": {"tuples_per_s": epi_rate,
                                     "per_unit": f"{C ** k} voxels x {EPILOGUE_OPS_PER_VOXEL} VALU lane-ops "
                                                 f"on {ALU_PEAK_TOPS:.1f} Tops/s",
                                     "frac": tuples / (sweep_ms * 1e-3) / epi_rate},
                "traffic": None,
                "kernel": (f"k_sweep2<{W}, max, {'fp4' if fp4 else 'int8'}>" if k == 2
                           else f"k_sweep3m{'1' if W == 1 else ''} (+ pair data)"),
                "units_per_launch": tuples, "kernel_ms": sweep_ms}
    elif k >= 4 and (args.engine == "hist" or C > (3 if k == 4 else 2)):
        # per-tuple histogram: N voxel increments (one LDS add each, the algorithmic work), then
        # C^k + k C^(k-1) voxel terms of the float32 screen
        ops_per_unit = 2 * w.n_obj
        achieved = tuples * ops_per_unit / (sweep_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "Tops/s (32-bit integer VALU)",
                "frac": achieved / ALU_PEAK_TOPS, "traffic": None, "kernel": f"k_sweep_hist<{C}, {k}>",
                "per_unit": f"2*N = {ops_per_unit} ops per tuple table (N voxel increments)",
                "units_per_launch": tuples, "kernel_ms": sweep_ms}
    elif k >= 4 and C == 2:
        # two classes: AND + popcount-accumulate per (subset holding m or n, 32-object word), the
        # 3 * 2^(k-2) per-lane subset counts of the prefix-wave / pair-lane engine
        words = (int((w.y == 0).sum()) + 31) // 32 + (int((w.y == 1).sum()) + 31) // 32
        ops_per_unit = 2 * 3 * 2 ** (k - 2) * words
        achieved = tuples * ops_per_unit / (sweep_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "Tops/s (32-bit integer VALU)",
                "frac": achieved / ALU_PEAK_TOPS, "traffic": None, "kernel": f"k_sweep45<{k}>",
                "per_unit": f"2*3*2^(k-2)*words = {ops_per_unit} VALU lane-ops per {k}-tuple",
                "units_per_launch": tuples, "kernel_ms": sweep_ms}
    elif k == 4:
        # AND + popcount-accumulate per (cell, 32-object word), every one of the C^4 cells counted
        words = (int((w.y == 0).sum()) + 31) // 32 + (int((w.y == 1).sum()) + 31) // 32
        ops_per_unit = 2 * (div + 1) ** 4 * words
        achieved = tuples * ops_per_unit / (sweep_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "Tops/s (32-bit integer VALU)",
                "frac": achieved / ALU_PEAK_TOPS, "traffic": None, "kernel": f"k_sweep4<{W}>",
                "per_unit": f"2*d^4*words = {ops_per_unit} VALU lane-ops per quadruple",
                "units_per_launch": tuples, "kernel_ms": sweep_ms}
    else:
        # AND + popcount-accumulate per (bin triple, 32-object word): 2 integer ops on 32 lanes
        words = (int((w.y == 0).sum()) + 31) // 32 + (int((w.y == 1).sum()) + 31) // 32
        ops_per_unit = 2 * W ** 3 * words
        achieved = tuples * ops_per_unit / (sweep_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "Tops/s (32-bit integer VALU)",
                "frac": achieved / ALU_PEAK_TOPS, "traffic": None, "kernel": f"k_sweep3<{W}> (+ pair data)",
                "per_unit": f"2*(d-1)^3*words = {ops_per_unit} VALU lane-ops per triple",
                "units_per_launch": tuples, "kernel_ms": sweep_ms}
    if k == 2 and os.path.exists(args.traffic_json):
        # counters are only valid for the kernel source and encoding they were taken on
        tr = json.load(open(args.traffic_json))
        if tr.get("sweep2_sha256") == _sweep_source_hash() and tr.get("encoding", "int8") == ("fp4" if fp4 else "int8"):
            roof["traffic"] = tr.get("bytes_per_launch")
    lds_json = os.path.join(ROOT, "profiles", "sweep2_headline_lds.json")
    if k == 2 and args.workload == "headline" and fp4 and os.path.exists(lds_json):
        # the binding resource, from the SQ counters of the same kernel source (profiles/)
        lc = json.load(open(lds_json))
        if lc.get("sweep2_sha256") == _sweep_source_hash():
            roof["binding_resource"] = lc["binding_resource"]
            roof["lds"] = {"bytes_per_launch": lc["lds_bytes_per_launch"],
                           "achieved": lc["lds_bytes_per_launch"] / (sweep_ms * 1e-3) / 1e9,
                           "peak": LDS_PEAK_GBS, "unit": "GB/s",
                           "frac": lc["lds_bytes_per_launch"] / (sweep_ms * 1e-3) / 1e9 / LDS_PEAK_GBS,
                           "busy": lc["lds_util"], "bank_conflict_share": lc["bank_conflict_share"],
                           "mfma_busy": lc["mfma_util"]}

    line = {
        "metric": "k-tuples evaluated/sec (k=2, N=2000, p=20k, 30 discretizations); p50/p99 latency",
        "value": tuples / (ms_per_step * 1e-3),
        "unit": "k-tuples evaluated/sec",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp4 (E2M1 one-hot), f32 accumulate" if fp4 else ("i8" if k == 2 else (
            "u8 codes, u32 histograms" if "hist" in roof["kernel"]
            else "u32 bitsets")),
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "k": k, "n_obj": w.n_obj, "n_var": w.n_var, "classes": div + 1, "n_disc": R,
                   "tuples_per_step": tuples,
                   "engine": args.engine, "workgroups": workgroups or "whole GPU",
                   "tile": ({"supertile": (tile & 0xff) or 8, "waves": ((tile >> 8) & 0xf) or (8 if div == 2 else 4)}
                            if k == 2 else None),
                   "autotuned": bool(tuned), "graph_replay": bool(args.graph),
                   "counts": ("fp4 MFMA, exact f32 accumulate" if fp4 else "int8 MFMA, int32 accumulate")
                   if (k == 2 or k3_mfma) else ("per-tuple LDS histograms" if k >= 4 and "hist" in roof["kernel"]
                                                else "bitset AND + popcount, int32"),
                   "entropy": "float32 screen + binary64 re-score"},
        "p50_ms": float(np.percentile(np.array(lat) * 1e3, 50)),
        "p99_ms": float(np.percentile(np.array(lat) * 1e3, 99)),
        "phase_ms": ph,
        "planted_found": found,
        "roofline": roof,
    }
    if k != 2 or args.workload != "headline":
        line["metric"] = f"k-tuples evaluated/sec (k={k} workload, informational)"
    if not args.no_cpu_baseline:
        # samples of about 10 s of oracle work on the host
        nv = min({2: args.cpu_vars, 3: 200, 4: 90, 5: 48}[k], w.n_var)

        def gpu_on_sample(n_vars, n_disc):
            o = mdfs.mdfs_max_ig(data[:n_vars].contiguous(), y, k, div, n_disc, w.xi, w.range_, w.seed,
                                 engine=args.engine)
            return [t.cpu().numpy() for t in o]

        cb = cpu_baseline(w, k, nv, min(args.cpu_disc, w.n_disc), ig.cpu().numpy(), am.cpu().numpy(),
                          out[2].cpu().numpy(), gpu_on_sample if k >= 4 else None)
        line["ig_error"] = cb.pop("ig_error")
        line["cpu_baseline"] = cb
    print(json.dumps(line))


if __name__ == "__main__":
    main()
