"""Python binding of librbc (include/rbc.h): argument marshalling only.

Every step of a search runs in the library's HIP kernels; this module passes
device pointers of torch tensors, the current HIP stream and a workspace
tensor.  The library must be built (``paper_1103_2635_amd.build.build()``);
importing the binding without it, or calling it on tensors that are not on a
GPU, raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbc.so")

L2, L1 = 0, 1
FP32, BF16, FP8_E4M3 = 0, 1, 2
EXACT, ONESHOT = 0, 1
FLAG_ONE_PASS = 1
STATS_LEN = 8
STAT_FALLBACK, STAT_NEARTIE, STAT_PAIRS, STAT_LISTS, STAT_CAND, STAT_CASCADE = 0, 1, 2, 3, 4, 5
STAT_ITEMS, STAT_SLOTS = 6, 7

_METRICS = {"l2": L2, "l1": L1, L2: L2, L1: L1}
_MODES = {"exact": EXACT, "oneshot": ONESHOT, EXACT: EXACT, ONESHOT: ONESHOT}
_PRECS = {"fp32": FP32, "bf16": BF16, "fp8": FP8_E4M3, FP32: FP32, BF16: BF16, FP8_E4M3: FP8_E4M3}

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SZ = ctypes.c_size_t


class SearchOpts(ctypes.Structure):
    _fields_ = [("precision", _I32), ("shortlist", _I32), ("splits", _I32), ("flags", _I32),
                ("dev_stats", _P), ("dev_approx_dist", _P), ("prune_eps", ctypes.c_float),
                ("reserved", _I32)]


class BuildParams(ctypes.Structure):
    _fields_ = [("mode", _I32), ("metric", _I32), ("n_r", _I64), ("s", _I64),
                ("seed", ctypes.c_uint64), ("rep_idx", _P), ("precisions", _I32),
                ("reserved", _I32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("shape", _I32), ("blocks", _I32), ("splits", _I32), ("item_queries", _I32),
                ("ms", ctypes.c_float),
                ("ms_before", ctypes.c_float), ("candidates", _I32)]


class RbcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("librbc status %d: %s" % (status, msg))
        self.status = status


_lib = None


def lib():
    """The loaded librbc (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librbc.so is not built: run paper_1103_2635_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.rbc_last_error.restype = ctypes.c_char_p
        L.bf_search_workspace_size.argtypes = [_I64, _I64, _I32, _I64, _I64, _I32, _I32, _P,
                                               ctypes.POINTER(_SZ)]
        L.bf_search.argtypes = [_P, _I64, _I64, _P, _I64, _I64, _I32, _I32, _I32, _P, _P, _P, _P,
                                _SZ, _P]
        L.rbc_build.argtypes = [_P, _I64, _I64, _I32, _P, _P, ctypes.POINTER(_P)]
        L.rbc_search_workspace_size.argtypes = [_P, _I64, _I64, _I32, _P, ctypes.POINTER(_SZ)]
        L.rbc_search.argtypes = [_P, _P, _I64, _I64, _I32, _P, _P, _P, _P, _SZ, _P]
        L.rbc_range_workspace_size.argtypes = [_P, _I64, _I64, ctypes.POINTER(_SZ)]
        L.rbc_range_count.argtypes = [_P, _P, _I64, _I64, ctypes.c_double, _P, _P, _SZ, _P]
        L.rbc_range_search.argtypes = [_P, _P, _I64, _I64, ctypes.c_double, _P, _P, _P, _P, _SZ,
                                       _P]
        L.rbc_index_info.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I32),
                                     ctypes.POINTER(_I64), ctypes.POINTER(_I32),
                                     ctypes.POINTER(_I32), ctypes.POINTER(_SZ)]
        L.rbc_index_export.argtypes = [_P, _P, _P, _P, _P]
        L.rbc_index_export_order.argtypes = [_P, _P, _P]
        L.rbc_free.argtypes = [_P]
        L.rbc_free.restype = None
        L.rbc_autotune_search.argtypes = [_P, _P, _I64, _I64, _I32, _P, _P, _P, _P, _SZ, _P,
                                          ctypes.POINTER(TuneResult)]
        L.rbc_autotune_bf.argtypes = [_P, _I64, _I64, _P, _I64, _I64, _I32, _I32, _I32, _P, _P,
                                      _P, _P, _SZ, _P, ctypes.POINTER(TuneResult)]
        L.rbc_autotune_set.argtypes = [_I32, _I32, _I32, _I32, _I32, _I32, _I32]
        L.rbc_autotune_clear.argtypes = []
        L.rbc_autotune_clear.restype = None
        L.rbc_timer_enable.argtypes = [ctypes.c_int]
        L.rbc_timer_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(_I64)]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise RbcError(rc, lib().rbc_last_error().decode())


def _stream_ptr(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _mat(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.dim() != 2:
        raise TypeError("%s must be a 2-D float32 tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be on a GPU (the library has no CPU path)" % name)
    if t.stride(1) != 1:
        raise ValueError("%s must have unit stride along rows" % name)
    return t


def _opts(precision="fp32", shortlist=0, splits=0, stats=None, approx_dist=None, prune_eps=0.0,
          one_pass=False):
    o = SearchOpts()
    o.precision = _PRECS[precision]
    o.shortlist = int(shortlist)
    o.splits = int(splits)
    o.flags = FLAG_ONE_PASS if one_pass else 0
    o.prune_eps = float(prune_eps)
    if stats is not None:
        if stats.dtype != torch.int64 or not stats.is_cuda or stats.numel() < STATS_LEN:
            raise ValueError("stats must be a GPU int64 tensor of %d counters" % STATS_LEN)
        o.dev_stats = stats.data_ptr()
    if approx_dist is not None:
        if approx_dist.dtype != torch.float32 or not approx_dist.is_cuda:
            raise ValueError("approx_dist must be a GPU float32 tensor of m x k")
        o.dev_approx_dist = approx_dist.data_ptr()
    return o


def new_stats(device="cuda"):
    """Zeroed device counters for the ``stats`` argument."""
    return torch.zeros(STATS_LEN, dtype=torch.int64, device=device)


def bf_search_workspace_size(m, n, d, k, metric="l2", ldq=None, ldx=None, **kw):
    sz = _SZ()
    o = _opts(**kw)
    _check(lib().bf_search_workspace_size(m, n, d, ldq or d, ldx or d, _METRICS[metric], k,
                                          ctypes.byref(o), ctypes.byref(sz)))
    return sz.value


def bf_search(Q, X, k, metric="l2", out=None, workspace=None, **kw):
    """BF(Q, X): the k nearest rows of X for every row of Q.

    Returns (idx int64 [m, k], dist float32 [m, k]) on Q's device, each row
    sorted by (distance, id).  Keyword options: precision ("fp32", "bf16",
    "fp8"), shortlist, splits, stats (see new_stats), approx_dist (a GPU
    float32 m x k tensor that receives the pre-re-score distances)."""
    _mat(Q, "Q")
    _mat(X, "X")
    m, d = Q.shape
    n = X.shape[0]
    if X.shape[1] != d:
        raise ValueError("Q and X have different dimensions")
    o = _opts(**kw)
    sz = _SZ()
    _check(lib().bf_search_workspace_size(m, n, d, Q.stride(0), X.stride(0), _METRICS[metric], k,
                                          ctypes.byref(o), ctypes.byref(sz)))
    if workspace is None or workspace.numel() < sz.value:
        workspace = torch.empty(max(1, sz.value), dtype=torch.uint8, device=Q.device)
    if out is None:
        out = (torch.empty((m, k), dtype=torch.int64, device=Q.device),
               torch.empty((m, k), dtype=torch.float32, device=Q.device))
    idx, dist = out
    _check(lib().bf_search(Q.data_ptr(), m, Q.stride(0), X.data_ptr(), n, X.stride(0), d,
                           _METRICS[metric], k, ctypes.byref(o), idx.data_ptr(), dist.data_ptr(),
                           workspace.data_ptr(), workspace.numel(), _stream_ptr(Q)))
    return idx, dist


class Index:
    """A built Random Ball Cover (owns device memory through librbc)."""

    def __init__(self, handle, device):
        self._h = handle
        self.device = device

    @property
    def handle(self):
        if not self._h:
            raise ValueError("index has been freed")
        return self._h

    def info(self):
        n, d, n_r, mode, metric, nb = _I64(), _I32(), _I64(), _I32(), _I32(), _SZ()
        _check(lib().rbc_index_info(self.handle, ctypes.byref(n), ctypes.byref(d),
                                    ctypes.byref(n_r), ctypes.byref(mode), ctypes.byref(metric),
                                    ctypes.byref(nb)))
        return {"n": n.value, "d": d.value, "n_r": n_r.value, "mode": mode.value,
                "metric": metric.value, "device_bytes": nb.value}

    def export(self):
        """Host copies of the index arrays (rep_idx, psi, list_off, list_ids)."""
        import numpy as np

        inf = self.info()
        n_r = inf["n_r"]
        rep = np.empty(n_r, np.int64)
        psi = np.empty(n_r, np.float64)
        off = np.empty(n_r + 1, np.int64)
        _check(lib().rbc_index_export(self.handle, rep.ctypes.data, psi.ctypes.data,
                                      off.ctypes.data, None))
        ids = np.empty(int(off[-1]), np.int64)
        _check(lib().rbc_index_export(self.handle, None, None, None, ids.ctypes.data))
        return {"rep_idx": rep, "psi": psi, "list_off": off, "list_ids": ids}

    def export_order(self):
        """Exact mode: (own distances in list order, per-list sorted flags)."""
        import numpy as np

        inf = self.info()
        own = np.empty(inf["n"], np.float32)
        srt = np.empty(inf["n_r"], np.int32)
        _check(lib().rbc_index_export_order(self.handle, own.ctypes.data, srt.ctypes.data))
        return own, srt.astype(bool)

    def free(self):
        if self._h:
            lib().rbc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def rbc_build(X, n_r, mode="exact", metric="l2", s=0, seed=0, rep_idx=None, precisions=()):
    """Build an RBC index over X (rep_idx: optional host int64 array of ids;
    precisions: low precisions ("bf16", "fp8") rbc_search may use)."""
    import numpy as np

    _mat(X, "X")
    n, d = X.shape
    p = BuildParams()
    p.mode = _MODES[mode]
    p.metric = _METRICS[metric]
    p.n_r = int(n_r)
    p.s = int(s)
    p.seed = int(seed)
    p.precisions = sum(1 << _PRECS[pr] for pr in set(precisions) if _PRECS[pr] != FP32)
    reps = None
    if rep_idx is not None:
        reps = np.ascontiguousarray(rep_idx, dtype=np.int64)
        if reps.shape != (int(n_r),):
            raise ValueError("rep_idx must hold n_r ids")
        p.rep_idx = reps.ctypes.data
    h = _P()
    _check(lib().rbc_build(X.data_ptr(), n, X.stride(0), d, ctypes.byref(p), _stream_ptr(X),
                           ctypes.byref(h)))
    return Index(h, X.device)


def rbc_search_workspace_size(index, m, k, ldq=None, **kw):
    sz = _SZ()
    o = _opts(**kw)
    _check(lib().rbc_search_workspace_size(index.handle, m, ldq or index.info()["d"], k,
                                           ctypes.byref(o), ctypes.byref(sz)))
    return sz.value


def rbc_search(index, Q, k, out=None, workspace=None, **kw):
    """Search an RBC index; returns (idx int64 [m, k], dist float32 [m, k])."""
    _mat(Q, "Q")
    m = Q.shape[0]
    o = _opts(**kw)
    sz = _SZ()
    _check(lib().rbc_search_workspace_size(index.handle, m, Q.stride(0), k, ctypes.byref(o),
                                           ctypes.byref(sz)))
    if workspace is None or workspace.numel() < sz.value:
        workspace = torch.empty(max(1, sz.value), dtype=torch.uint8, device=Q.device)
    if out is None:
        out = (torch.empty((m, k), dtype=torch.int64, device=Q.device),
               torch.empty((m, k), dtype=torch.float32, device=Q.device))
    idx, dist = out
    _check(lib().rbc_search(index.handle, Q.data_ptr(), m, Q.stride(0), k, ctypes.byref(o),
                            idx.data_ptr(), dist.data_ptr(), workspace.data_ptr(),
                            workspace.numel(), _stream_ptr(Q)))
    return idx, dist


def rbc_range_workspace_size(index, m, ldq=None):
    sz = _SZ()
    _check(lib().rbc_range_workspace_size(index.handle, m, ldq or index.info()["d"],
                                          ctypes.byref(sz)))
    return sz.value


def rbc_range_count(index, Q, radius, offsets=None, workspace=None):
    """Offsets (device int64 [m + 1]) of every query's points within radius."""
    _mat(Q, "Q")
    m = Q.shape[0]
    sz = _SZ()
    _check(lib().rbc_range_workspace_size(index.handle, m, Q.stride(0), ctypes.byref(sz)))
    if workspace is None or workspace.numel() < sz.value:
        workspace = torch.empty(max(1, sz.value), dtype=torch.uint8, device=Q.device)
    if offsets is None:
        offsets = torch.empty(m + 1, dtype=torch.int64, device=Q.device)
    _check(lib().rbc_range_count(index.handle, Q.data_ptr(), m, Q.stride(0), float(radius),
                                 offsets.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                 _stream_ptr(Q)))
    return offsets


def rbc_range_search(index, Q, radius, workspace=None):
    """All points within radius of each query: (offsets int64 [m + 1], idx
    int64 [total], dist float32 [total]); the points of query i are
    idx[offsets[i]:offsets[i + 1]] in ascending (distance, id) order."""
    _mat(Q, "Q")
    m = Q.shape[0]
    sz = _SZ()
    _check(lib().rbc_range_workspace_size(index.handle, m, Q.stride(0), ctypes.byref(sz)))
    if workspace is None or workspace.numel() < sz.value:
        workspace = torch.empty(max(1, sz.value), dtype=torch.uint8, device=Q.device)
    off = rbc_range_count(index, Q, radius, workspace=workspace)
    total = int(off[-1].item()) if m > 0 else 0
    idx = torch.empty(max(total, 1), dtype=torch.int64, device=Q.device)
    dist = torch.empty(max(total, 1), dtype=torch.float32, device=Q.device)
    _check(lib().rbc_range_search(index.handle, Q.data_ptr(), m, Q.stride(0), float(radius),
                                  off.data_ptr(), idx.data_ptr(), dist.data_ptr(),
                                  workspace.data_ptr(), workspace.numel(), _stream_ptr(Q)))
    return off, idx[:total], dist[:total]


def _tune_dict(r):
    return {"shape": r.shape, "blocks": r.blocks, "splits": r.splits,
            "item_queries": r.item_queries, "ms": r.ms,
            "ms_before": r.ms_before,
            "candidates": r.candidates}


def autotune_search(index, Q, k, **kw):
    """Time the tile shapes and stage-2 grid sizes of rbc_search(index, Q, k)
    and keep the fastest for later calls; returns the choice and its time."""
    _mat(Q, "Q")
    m = Q.shape[0]
    o = _opts(**kw)
    sz = _SZ()
    _check(lib().rbc_search_workspace_size(index.handle, m, Q.stride(0), k, ctypes.byref(o),
                                           ctypes.byref(sz)))
    ws = torch.empty(max(1, sz.value), dtype=torch.uint8, device=Q.device)
    idx = torch.empty((m, k), dtype=torch.int64, device=Q.device)
    dist = torch.empty((m, k), dtype=torch.float32, device=Q.device)
    r = TuneResult()
    _check(lib().rbc_autotune_search(index.handle, Q.data_ptr(), m, Q.stride(0), k,
                                     ctypes.byref(o), idx.data_ptr(), dist.data_ptr(),
                                     ws.data_ptr(), ws.numel(), _stream_ptr(Q), ctypes.byref(r)))
    return _tune_dict(r)


def autotune_bf(Q, X, k, metric="l2", **kw):
    """Time the tile shapes of bf_search(Q, X, k) and keep the fastest."""
    _mat(Q, "Q")
    _mat(X, "X")
    m, d = Q.shape
    n = X.shape[0]
    o = _opts(**kw)
    sz = _SZ()
    _check(lib().bf_search_workspace_size(m, n, d, Q.stride(0), X.stride(0), _METRICS[metric], k,
                                          ctypes.byref(o), ctypes.byref(sz)))
    ws = torch.empty(max(1, sz.value), dtype=torch.uint8, device=Q.device)
    idx = torch.empty((m, k), dtype=torch.int64, device=Q.device)
    dist = torch.empty((m, k), dtype=torch.float32, device=Q.device)
    r = TuneResult()
    _check(lib().rbc_autotune_bf(Q.data_ptr(), m, Q.stride(0), X.data_ptr(), n, X.stride(0), d,
                                 _METRICS[metric], k, ctypes.byref(o), idx.data_ptr(),
                                 dist.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(Q),
                                 ctypes.byref(r)))
    return _tune_dict(r)


def autotune_set(kind, d, shortlist, shape, blocks=1024, splits=0, item_queries=64):
    """Pin the tile choice of kind "bf" or "search" for (d, shortlist length)."""
    _check(lib().rbc_autotune_set({"bf": 0, "search": 1}[kind], d, shortlist, shape, blocks,
                                  splits, item_queries))


def autotune_clear():
    """Forget every tuned choice."""
    lib().rbc_autotune_clear()


def timer_enable(on=True):
    """Start (or stop) per-kernel HIP event timing inside the library."""
    _check(lib().rbc_timer_enable(1 if on else 0))


def timer_read(name):
    """(total device ms, launches) of the library kernels called ``name``."""
    ms, n = ctypes.c_double(), _I64()
    _check(lib().rbc_timer_read(name.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value
