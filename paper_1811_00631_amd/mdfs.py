"""Python binding of libmdfs (the C ABI in include/mdfs.h): argument marshalling only.

Every step of the computation runs in the HIP kernels behind the C ABI; torch is used for
device memory (inputs, outputs, the workspace) and for the current stream.  There is no CPU
fallback: if libmdfs.so is missing, `load()` raises.

Functions mirror the C entry points:
    mdfs_workspace_size(...)            -> int
    mdfs_discretize(data, ...)          -> codes uint8 [n_disc][n_var][n_obj]
    mdfs_max_ig(data, y, ...)           -> (ig_max f32 [n_var], argmax i32 [n_var][k-1],
                                            argmax_disc i32 [n_var])
    mdfs_pair_counts(data, y, disc,...) -> counts i32 [n_var][n_var][2][c][c] (i < j filled)
    mdfs_triple_counts(data, y, disc, i_sel, ...)
                                        -> counts i32 [n_var][n_var][2][c][c][c] (i_sel < j < l)
    mdfs_screen_max(data, y, ...)       -> (ig32 f32 [n_var], error bound E)
    mdfs_chi2_df(k, divisions)          -> int
    mdfs_pvalues(ig, k, divisions, ...) -> (p float64 [n], n_eff)       (host arrays)
    mdfs_ig_lim(k, divisions, n_eff, a) -> float
    mdfs_p_adjust(p, method)            -> adjusted float64 [n]          (host arrays)
    mdfs_add_contrast(data, n, seed)    -> (data + contrast f32 [n_var+n][n_obj], src i32 [n])
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdfs.so")

MDFS_OK = 0
STATUS = {0: "MDFS_OK", -1: "MDFS_E_ARG", -2: "MDFS_E_Y", -3: "MDFS_E_K", -4: "MDFS_E_DIV",
          -5: "MDFS_E_NAN", -6: "MDFS_E_NOMEM", -7: "MDFS_E_HIP", -8: "MDFS_E_CANCELLED",
          -9: "MDFS_E_OVERFLOW", -10: "MDFS_E_LIMIT"}
E_CANCELLED, E_OVERFLOW, E_LIMIT = -8, -9, -10
ENGINES = {"auto": 0, "mfma": 1, "bitset": 2, "mfma_fp4": 3, "hist": 4}
ADJUST = {"none": 0, "holm": 1, "BH": 2, "BY": 3}


class MdfsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("n_obj", ctypes.c_int64), ("n_var", ctypes.c_int64), ("k", ctypes.c_int32),
                ("divisions", ctypes.c_int32), ("n_disc", ctypes.c_int32), ("disc_offset", ctypes.c_int32),
                ("range", ctypes.c_double), ("pseudocount", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("engine", ctypes.c_int32), ("flags", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("cancel", ctypes.c_void_p)]


_lib = None
SYMBOLS = ["mdfs_workspace_size", "mdfs_discretize", "mdfs_max_ig", "mdfs_pair_counts", "mdfs_triple_counts",
           "mdfs_screen_max", "mdfs_interesting_tuples", "mdfs_phase_times", "mdfs_last_error",
           "mdfs_chi2_df", "mdfs_pvalues", "mdfs_ig_lim", "mdfs_p_adjust", "mdfs_add_contrast",
           "mdfs_max_ig_codes", "mdfs_max_ig_async", "mdfs_check_status", "mdfs_max_ig_batch",
           "mdfs_batch_workspace_size", "mdfs_max_ig_noalloc"]
FLAG_TIMING = 1
PHASES = ["setup", "discretize", "sweep", "finalize"]


def load(path: str = LIB_PATH):
    """Load libmdfs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_1811_00631_amd.build`")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER(Params)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    L.mdfs_workspace_size.argtypes = [P]
    L.mdfs_workspace_size.restype = sz
    L.mdfs_discretize.argtypes = [P, vp, vp, vp, sz, vp]
    L.mdfs_max_ig.argtypes = [P, vp, vp, vp, vp, vp, vp, sz, vp]
    L.mdfs_max_ig_codes.argtypes = [P, vp, vp, vp, vp, vp, vp, sz, vp]
    L.mdfs_max_ig_async.argtypes = [P, vp, vp, ctypes.c_int64, vp, vp, vp, vp, sz, vp]
    L.mdfs_check_status.argtypes = [P, vp, sz, vp]
    L.mdfs_max_ig_noalloc.argtypes = [P, vp, vp, ctypes.c_int64, vp, vp, vp, vp, vp]
    L.mdfs_max_ig_noalloc.restype = ctypes.c_int
    L.mdfs_batch_workspace_size.argtypes = []
    L.mdfs_batch_workspace_size.restype = sz
    L.mdfs_max_ig_batch.argtypes = [ctypes.c_int, P, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.mdfs_max_ig_batch.restype = ctypes.c_int
    L.mdfs_pair_counts.argtypes = [P, vp, vp, ctypes.c_int32, vp, vp, sz, vp]
    L.mdfs_triple_counts.argtypes = [P, vp, vp, ctypes.c_int32, ctypes.c_int32, vp, vp, sz, vp]
    L.mdfs_screen_max.argtypes = [P, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp, sz, vp]
    L.mdfs_interesting_tuples.argtypes = [P, vp, vp, ctypes.c_double, vp, vp, vp, vp, ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_int64), vp, sz, vp]
    L.mdfs_phase_times.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int]
    L.mdfs_phase_times.restype = ctypes.c_int
    L.mdfs_last_error.restype = ctypes.c_char_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.mdfs_chi2_df.argtypes = [ctypes.c_int, ctypes.c_int]
    L.mdfs_pvalues.argtypes = [vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, vp, ctypes.c_double, vp, dp]
    L.mdfs_ig_lim.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
    L.mdfs_p_adjust.argtypes = [vp, ctypes.c_int64, ctypes.c_int, vp]
    L.mdfs_add_contrast.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, vp, vp, vp]
    for fn in ("mdfs_chi2_df", "mdfs_pvalues", "mdfs_ig_lim", "mdfs_p_adjust", "mdfs_add_contrast"):
        getattr(L, fn).restype = ctypes.c_int
    for fn in ("mdfs_discretize", "mdfs_max_ig", "mdfs_max_ig_codes", "mdfs_max_ig_async", "mdfs_check_status",
               "mdfs_pair_counts", "mdfs_triple_counts", "mdfs_screen_max", "mdfs_interesting_tuples"):
        getattr(L, fn).restype = ctypes.c_int
    _lib = L
    return L


def tile_code(supertile: int = 0, waves: int = 0) -> int:
    """The `tile` field: super-tile side (2, 4, 8, 16; 0 default) and waves per workgroup of the
    three-class pair sweep (4, 8; 0 default)."""
    return (int(supertile) & 0xff) | ((int(waves) & 0xf) << 8)


def make_params(n_obj, n_var, k=2, divisions=2, n_disc=1, disc_offset=0, range_=0.5, pseudocount=0.25,
                seed=0, engine="auto", flags=0, workgroups=0, cancel=None, tile=0) -> Params:
    """`cancel`: None, or the address (int) of a caller-owned host-mapped uint32 cancel word;
    `tile`: see tile_code."""
    return Params(int(n_obj), int(n_var), int(k), int(divisions), int(n_disc), int(disc_offset),
                  float(range_), float(pseudocount), int(seed) & ((1 << 64) - 1), ENGINES[engine], int(flags),
                  int(workgroups), int(tile), cancel)


def mdfs_phase_times() -> dict:
    """Per-phase milliseconds of the last call made with timing on (HIP events on its stream)."""
    buf = (ctypes.c_float * 8)()
    n = load().mdfs_phase_times(buf, 8)
    return {PHASES[i]: float(buf[i]) for i in range(n)}


def _check(rc: int):
    if rc != MDFS_OK:
        raise MdfsError(rc, load().mdfs_last_error().decode())


def mdfs_workspace_size(prm: Params) -> int:
    """Bytes of device workspace for `prm`; raises MdfsError on invalid parameters."""
    n = load().mdfs_workspace_size(ctypes.byref(prm))
    if n == 0:
        raise MdfsError(-1, load().mdfs_last_error().decode())
    return n


class Workspace:
    """Grow-only device workspace per device (owned by the caller side, as the C ABI asks)."""

    def __init__(self):
        self.buf = {}

    def get(self, nbytes: int, device) -> torch.Tensor:
        key = torch.device(device).index or 0
        b = self.buf.get(key)
        if b is None or b.numel() < nbytes:
            self.buf.pop(key, None)
            b = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
            self.buf[key] = b
        return b


_WS = Workspace()


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_inputs(data: torch.Tensor, y: torch.Tensor | None = None):
    if not (data.is_cuda and data.dtype == torch.float32 and data.dim() == 2):
        raise ValueError("data must be a CUDA float32 tensor [n_var][n_obj]")
    data = data.contiguous()
    if y is not None:
        if not (y.is_cuda and y.dtype == torch.uint8 and y.dim() == 1 and y.numel() == data.shape[1]):
            raise ValueError("y must be a CUDA uint8 tensor [n_obj]")
        y = y.contiguous()
    return data, y


def workspace_for(prm: Params, device) -> torch.Tensor:
    return _WS.get(mdfs_workspace_size(prm), device)


def mdfs_discretize(data: torch.Tensor, divisions: int, n_disc: int, range_: float = 0.5, seed: int = 0,
                    disc_offset: int = 0, k: int = 2, ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    data, _ = _dev_inputs(data)
    n_var, n_obj = data.shape
    prm = make_params(n_obj, n_var, k, divisions, n_disc, disc_offset, range_, 0.25, seed)
    if ws is None:
        ws = workspace_for(prm, data.device)
    strm = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream(data.device)
    codes = torch.empty((n_disc, n_var, n_obj), dtype=torch.uint8, device=data.device)
    _check(load().mdfs_discretize(ctypes.byref(prm), _ptr(data), _ptr(codes), _ptr(ws), ws.numel(), strm))
    return codes


def mdfs_max_ig(data: torch.Tensor, y: torch.Tensor, k: int, divisions: int, n_disc: int,
                pseudocount: float = 0.25, range_: float = 0.5, seed: int = 0, disc_offset: int = 0,
                engine: str = "auto", timing: bool = False, workgroups: int = 0, ws: torch.Tensor | None = None,
                stream=None, cancel=None, tile: int = 0):
    """IG_max, argmax tuple and argmax discretisation of every variable.  `ws` (a caller-owned
    uint8 device workspace of at least mdfs_workspace_size bytes) and `stream` (a torch CUDA
    stream) default to a per-device cached workspace and the current stream; `cancel` is the
    address of a caller-owned host-mapped uint32 cancel word, or None."""
    data, y = _dev_inputs(data, y)
    n_var, n_obj = data.shape
    prm = make_params(n_obj, n_var, k, divisions, n_disc, disc_offset, range_, pseudocount, seed, engine,
                      FLAG_TIMING if timing else 0, workgroups, cancel, tile)
    if ws is None:
        ws = workspace_for(prm, data.device)
    strm = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream(data.device)
    ig = torch.empty(n_var, dtype=torch.float32, device=data.device)
    am = torch.empty((n_var, k - 1), dtype=torch.int32, device=data.device)
    ad = torch.empty(n_var, dtype=torch.int32, device=data.device)
    _check(load().mdfs_max_ig(ctypes.byref(prm), _ptr(data), _ptr(y), _ptr(ig), _ptr(am), _ptr(ad), _ptr(ws),
                              ws.numel(), strm))
    return ig, am, ad


def mdfs_max_ig_async(data: torch.Tensor, y: torch.Tensor, n1: int, k: int, divisions: int, n_disc: int,
                      pseudocount: float = 0.25, range_: float = 0.5, seed: int = 0, disc_offset: int = 0,
                      engine: str = "auto", workgroups: int = 0, ws: torch.Tensor | None = None, out=None,
                      cancel=None, tile: int = 0):
    """Enqueue mdfs_max_ig on the current stream without any host synchronisation (capturable in
    a CUDA graph).  `out` = (ig, argmax, argmax_disc) preallocated tensors or None; `ws` a
    preallocated workspace or None (the cached one).  Check errors later with mdfs_check_status."""
    data, y = _dev_inputs(data, y)
    n_var, n_obj = data.shape
    prm = make_params(n_obj, n_var, k, divisions, n_disc, disc_offset, range_, pseudocount, seed, engine, 0,
                      workgroups, cancel, tile)
    if ws is None:
        ws = workspace_for(prm, data.device)
    if out is None:
        out = (torch.empty(n_var, dtype=torch.float32, device=data.device),
               torch.empty((n_var, k - 1), dtype=torch.int32, device=data.device),
               torch.empty(n_var, dtype=torch.int32, device=data.device))
    ig, am, ad = out
    _check(load().mdfs_max_ig_async(ctypes.byref(prm), _ptr(data), _ptr(y), int(n1), _ptr(ig), _ptr(am), _ptr(ad),
                                    _ptr(ws), ws.numel(), _stream(data.device)))
    return ig, am, ad


def mdfs_max_ig_noalloc(data: torch.Tensor, y: torch.Tensor, n1: int, k: int, divisions: int, n_disc: int,
                        pseudocount: float = 0.25, range_: float = 0.5, seed: int = 0, disc_offset: int = 0,
                        engine: str = "auto", workgroups: int = 0, out=None, status=None):
    """mdfs_max_ig_async with the library's own fixed device workspace: nothing is allocated by the
    call (`out` = preallocated (ig, argmax, argmax_disc) or None; `status` = a preallocated int32
    device tensor of one element that receives the device status code, or None)."""
    data, y = _dev_inputs(data, y)
    n_var, n_obj = data.shape
    prm = make_params(n_obj, n_var, k, divisions, n_disc, disc_offset, range_, pseudocount, seed, engine, 0,
                      workgroups)
    if out is None:
        out = (torch.empty(n_var, dtype=torch.float32, device=data.device),
               torch.empty((n_var, k - 1), dtype=torch.int32, device=data.device),
               torch.empty(n_var, dtype=torch.int32, device=data.device))
    ig, am, ad = out
    _check(load().mdfs_max_ig_noalloc(ctypes.byref(prm), _ptr(data), _ptr(y), int(n1), _ptr(ig), _ptr(am), _ptr(ad),
                                      _ptr(status), _stream(data.device)))
    return ig, am, ad


def mdfs_check_status(data_shape, k: int, divisions: int, n_disc: int, ws: torch.Tensor | None = None,
                disc_offset: int = 0, engine: str = "auto"):
    """Raise MdfsError if the last asynchronous call on `ws` flagged an error (synchronises)."""
    n_var, n_obj = data_shape
    prm = make_params(n_obj, n_var, k, divisions, n_disc, disc_offset, 0.5, 0.25, 0, engine)
    if ws is None:
        ws = workspace_for(prm, torch.device("cuda", torch.cuda.current_device()))
    _check(load().mdfs_check_status(ctypes.byref(prm), _ptr(ws), ws.numel(), _stream(ws.device)))


def mdfs_max_ig_batch(datas, ys, n1s, k: int, divisions: int, n_discs, pseudocount: float = 0.25,
                      range_: float = 0.5, seeds=None, engine: str = "auto", workgroups: int = 0):
    """Several problems with one k in one asynchronous call (no host synchronisation): for k = 2
    one fused persistent sweep launch, for other k the problems' calls on four concurrent
    streams; pseudocount and range_ may be one value or one per problem.  Returns
    [(ig, argmax, argmax_disc)] and the workspaces (for mdfs_check_status)."""
    n = len(datas)
    seeds = seeds if seeds is not None else [0] * n
    per = lambda v: list(v) if isinstance(v, (list, tuple)) else [v] * n   # noqa: E731
    xis, rngs = per(pseudocount), per(range_)
    PA = Params * n
    prms = PA(*[make_params(d.shape[1], d.shape[0], k, divisions, n_discs[i], 0, rngs[i], xis[i], seeds[i],
                            engine, 0, workgroups) for i, d in enumerate(datas)])
    dev = datas[0].device
    ins = [_dev_inputs(d, y) for d, y in zip(datas, ys)]
    wss = [torch.empty(mdfs_workspace_size(prms[i]), dtype=torch.uint8, device=dev) for i in range(n)]
    outs = [(torch.empty(d.shape[0], dtype=torch.float32, device=dev),
             torch.empty((d.shape[0], k - 1), dtype=torch.int32, device=dev),
             torch.empty(d.shape[0], dtype=torch.int32, device=dev)) for d, _ in ins]
    bws = torch.empty(load().mdfs_batch_workspace_size(), dtype=torch.uint8, device=dev)
    ptrs = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])   # noqa: E731
    n1a = (ctypes.c_int64 * n)(*[int(v) for v in n1s])
    wsb = (ctypes.c_size_t * n)(*[w.numel() for w in wss])
    _check(load().mdfs_max_ig_batch(n, prms, ptrs([d for d, _ in ins]), ptrs([y for _, y in ins]), n1a,
                                    ptrs([o[0] for o in outs]), ptrs([o[1] for o in outs]), ptrs([o[2] for o in outs]),
                                    ptrs(wss), wsb, _ptr(bws), bws.numel(), _stream(dev)))
    return outs, wss


def mdfs_max_ig_codes(codes: torch.Tensor, y: torch.Tensor, k: int, divisions: int, pseudocount: float = 0.25,
                      disc_offset: int = 0, engine: str = "auto", workgroups: int = 0, ws: torch.Tensor | None = None,
                      stream=None):
    """mdfs_max_ig from device codes uint8 [n_disc][n_var][n_obj] (values 0..divisions)."""
    if not (isinstance(codes, torch.Tensor) and codes.is_cuda and codes.dtype == torch.uint8 and codes.dim() == 3):
        raise ValueError("codes must be a CUDA uint8 tensor [n_disc][n_var][n_obj]")
    codes = codes.contiguous()
    n_disc, n_var, n_obj = codes.shape
    if not (y.is_cuda and y.dtype == torch.uint8 and y.dim() == 1 and y.numel() == n_obj):
        raise ValueError("y must be a CUDA uint8 tensor [n_obj]")
    y = y.contiguous()
    prm = make_params(n_obj, n_var, k, divisions, n_disc, disc_offset, 0.0, pseudocount, 0, engine, 0, workgroups)
    if ws is None:
        ws = workspace_for(prm, codes.device)
    strm = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream(codes.device)
    ig = torch.empty(n_var, dtype=torch.float32, device=codes.device)
    am = torch.empty((n_var, k - 1), dtype=torch.int32, device=codes.device)
    ad = torch.empty(n_var, dtype=torch.int32, device=codes.device)
    _check(load().mdfs_max_ig_codes(ctypes.byref(prm), _ptr(codes), _ptr(y), _ptr(ig), _ptr(am), _ptr(ad), _ptr(ws),
                                    ws.numel(), strm))
    return ig, am, ad


def mdfs_pair_counts(data: torch.Tensor, y: torch.Tensor, disc: int, divisions: int, n_disc: int,
                     range_: float = 0.5, seed: int = 0, disc_offset: int = 0, engine: str = "auto") -> torch.Tensor:
    data, y = _dev_inputs(data, y)
    n_var, n_obj = data.shape
    c = divisions + 1
    prm = make_params(n_obj, n_var, 2, divisions, n_disc, disc_offset, range_, 0.25, seed, engine)
    ws = workspace_for(prm, data.device)
    counts = torch.zeros((n_var, n_var, 2, c, c), dtype=torch.int32, device=data.device)
    _check(load().mdfs_pair_counts(ctypes.byref(prm), _ptr(data), _ptr(y), int(disc), _ptr(counts), _ptr(ws),
                                   ws.numel(), _stream(data.device)))
    return counts


def mdfs_triple_counts(data: torch.Tensor, y: torch.Tensor, disc: int, i_sel: int, divisions: int, n_disc: int,
                       range_: float = 0.5, seed: int = 0, disc_offset: int = 0,
                       engine: str = "auto") -> torch.Tensor:
    """Per-class tables [n_var][n_var][2][c][c][c] of the triples (i_sel, j, l), i_sel < j < l, of
    discretisation `disc`, from the k = 3 count engine `engine` selects."""
    data, y = _dev_inputs(data, y)
    n_var, n_obj = data.shape
    c = divisions + 1
    prm = make_params(n_obj, n_var, 3, divisions, n_disc, disc_offset, range_, 0.25, seed, engine)
    ws = workspace_for(prm, data.device)
    counts = torch.zeros((n_var, n_var, 2, c, c, c), dtype=torch.int32, device=data.device)
    _check(load().mdfs_triple_counts(ctypes.byref(prm), _ptr(data), _ptr(y), int(disc), int(i_sel), _ptr(counts),
                                     _ptr(ws), ws.numel(), _stream(data.device)))
    return counts


def mdfs_interesting_tuples(data: torch.Tensor, y: torch.Tensor, k: int, divisions: int, n_disc: int,
                            ig_thr: float, pseudocount: float = 0.25, range_: float = 0.5, seed: int = 0,
                            disc_offset: int = 0, engine: str = "auto", max_out: int = 1 << 20):
    """Every (variable, partner tuple, discretisation) with IG >= ig_thr: device tensors
    (var int32 [n], partners int32 [n][k-1], disc int32 [n], ig float64 [n]) in unspecified order.
    Raises MdfsError(E_LIMIT) if more than max_out records exist."""
    data, y = _dev_inputs(data, y)
    n_var, n_obj = data.shape
    prm = make_params(n_obj, n_var, k, divisions, n_disc, disc_offset, range_, pseudocount, seed, engine)
    ws = workspace_for(prm, data.device)
    dev = data.device
    var = torch.empty(max_out, dtype=torch.int32, device=dev)
    part = torch.empty((max_out, k - 1), dtype=torch.int32, device=dev)
    disc = torch.empty(max_out, dtype=torch.int32, device=dev)
    ig = torch.empty(max_out, dtype=torch.float64, device=dev)
    n = ctypes.c_int64(0)
    _check(load().mdfs_interesting_tuples(ctypes.byref(prm), _ptr(data), _ptr(y), float(ig_thr), _ptr(var),
                                          _ptr(part), _ptr(disc), _ptr(ig), int(max_out), ctypes.byref(n), _ptr(ws),
                                          ws.numel(), _stream(dev)))
    if n.value > max_out:
        raise MdfsError(E_LIMIT, f"{n.value} interesting tuples exceed max_out={max_out}")
    m = n.value
    return var[:m], part[:m], disc[:m], ig[:m]


def mdfs_screen_max(data: torch.Tensor, y: torch.Tensor, k: int, divisions: int, n_disc: int,
                    pseudocount: float = 0.25, range_: float = 0.5, seed: int = 0, disc_offset: int = 0,
                    engine: str = "auto"):
    data, y = _dev_inputs(data, y)
    n_var, n_obj = data.shape
    prm = make_params(n_obj, n_var, k, divisions, n_disc, disc_offset, range_, pseudocount, seed, engine)
    ws = workspace_for(prm, data.device)
    ig32 = torch.empty(n_var, dtype=torch.float32, device=data.device)
    eb = ctypes.c_double(0.0)
    _check(load().mdfs_screen_max(ctypes.byref(prm), _ptr(data), _ptr(y), _ptr(ig32), ctypes.byref(eb), _ptr(ws),
                                  ws.numel(), _stream(data.device)))
    return ig32, eb.value


# ------------------------------------------------------------------ significance (host, binary64)
def _host_f64(x) -> np.ndarray:
    if isinstance(x, torch.Tensor):
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(x, dtype=np.float64)


def mdfs_chi2_df(k: int, divisions: int) -> int:
    """Degrees of freedom of 2 IG for one tuple of irrelevant variables."""
    rc = load().mdfs_chi2_df(int(k), int(divisions))
    if rc <= 0:
        _check(rc)
    return rc


def mdfs_pvalues(ig, k: int, divisions: int, fit_mask=None, n_eff: float | None = None):
    """p-values of IG^k_max (host arrays).  fit_mask selects the variables taken as irrelevant
    for the fit of n_eff (None = all); a given n_eff is used as is.  Returns (p, n_eff)."""
    x = _host_f64(ig).ravel()
    out = np.empty_like(x)
    mask = None
    if fit_mask is not None:
        mask = np.ascontiguousarray(np.asarray(fit_mask).ravel() != 0, dtype=np.uint8)
        if mask.shape != x.shape:
            raise ValueError("fit_mask must have one entry per variable")
    ne = ctypes.c_double(0.0)
    _check(load().mdfs_pvalues(x.ctypes.data, x.size, int(k), int(divisions),
                               None if mask is None else mask.ctypes.data,
                               float(n_eff) if n_eff is not None else 0.0, out.ctypes.data, ctypes.byref(ne)))
    return out, ne.value


def mdfs_ig_lim(k: int, divisions: int, n_eff: float, alpha: float) -> float:
    """IG_lim: the IG^k_max whose p-value is alpha."""
    v = ctypes.c_double(0.0)
    _check(load().mdfs_ig_lim(int(k), int(divisions), float(n_eff), float(alpha), ctypes.byref(v)))
    return v.value


def mdfs_p_adjust(p, method: str = "BY") -> np.ndarray:
    """Adjusted p-values: "holm", "BH", "BY" or "none" (the definitions of R's p.adjust)."""
    x = _host_f64(p).ravel()
    out = np.empty_like(x)
    _check(load().mdfs_p_adjust(x.ctypes.data, x.size, ADJUST[method], out.ctypes.data))
    return out


def mdfs_add_contrast(data: torch.Tensor, n_contrast: int, seed: int = 0):
    """The originals followed by n_contrast contrast variables (device), and the source variable
    of each contrast variable (host int32 numpy array)."""
    d, _ = _dev_inputs(data)
    n_var, n_obj = d.shape
    out = torch.empty((n_var + int(n_contrast), n_obj), dtype=torch.float32, device=d.device)
    src = np.zeros(max(1, int(n_contrast)), dtype=np.int32)
    _check(load().mdfs_add_contrast(_ptr(d), n_obj, n_var, int(n_contrast), int(seed) & ((1 << 64) - 1), _ptr(out),
                                    src.ctypes.data, _stream(d.device)))
    return out, src[: int(n_contrast)]
