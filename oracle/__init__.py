"""CPU FP64 oracle for the Random Ball Cover and the brute-force primitive.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the HIP library: the arithmetic lives in ``rbc_oracle.c`` (plain C, double
precision, OpenMP over queries) and this module only marshals NumPy arrays.

Every function takes float32 row-major arrays (they are converted exactly to
double inside the C code) and returns int64 ids and float64 distances ranked in
(distance, id) order.  ``metric`` is ``"l2"`` (Euclidean) or ``"l1"``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbc_oracle.c")
_LIB = os.path.join(_HERE, "librbc_oracle.so")
_lib = None

METRICS = {"l2": 0, "l1": 1}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (generic x86-64 code, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
               "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        path = build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_rho_pairs.argtypes = [P, P, I64, I32, I32, P]
        lib.orc_bf_knn.argtypes = [P, I64, P, I64, I32, I32, I32, P, P]
        lib.orc_rank.argtypes = [P, I64, P, I64, I32, I32, P, P]
        lib.orc_rbc_build_exact.argtypes = [P, I64, I32, I32, P, I64, P, P, P, P]
        lib.orc_rbc_search_exact.argtypes = [P, I64, P, I64, I32, I32, P, I64, P, P, P, I32,
                                             I32, P, P, P, P, P]
        lib.orc_rbc_search_approx.argtypes = [P, I64, P, I64, I32, I32, P, I64, P, P, P, I32,
                                              I32, ctypes.c_double, P, P, P, P, P]
        lib.orc_range_bf.argtypes = [P, I64, P, I64, I32, I32, ctypes.c_double, P, P, P]
        lib.orc_rbc_build_oneshot.argtypes = [P, I64, I32, I32, P, I64, I64, P, P]
        lib.orc_rbc_search_oneshot.argtypes = [P, I64, P, I64, I32, I32, P, I64, I64, P, I32,
                                               P, P, P]
        for f in ("orc_rho_pairs", "orc_bf_knn", "orc_rank", "orc_rbc_build_exact",
                  "orc_rbc_search_exact", "orc_rbc_search_approx", "orc_range_bf",
                  "orc_rbc_build_oneshot",
                  "orc_rbc_search_oneshot"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 2:
        raise ValueError("expected a 2-D array")
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc, name):
    if rc != 0:
        raise ValueError("%s rejected its arguments (rc=%d)" % (name, rc))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def rho_pairs(A, B, metric="l2"):
    """rho(A[i], B[i]) for each row pair."""
    A, B = _f32(A), _f32(B)
    out = np.empty(A.shape[0], np.float64)
    _check(_load().orc_rho_pairs(_p(A), _p(B), A.shape[0], A.shape[1], METRICS[metric], _p(out)),
           "rho_pairs")
    return out


def bf_knn(Q, X, k, metric="l2"):
    """BF(Q, X): the k nearest database rows of every query."""
    Q, X = _f32(Q), _f32(X)
    m, d = Q.shape
    idx = np.empty((m, k), np.int64)
    dist = np.empty((m, k), np.float64)
    _check(_load().orc_bf_knn(_p(Q), m, _p(X), X.shape[0], d, METRICS[metric], k, _p(idx),
                              _p(dist)), "bf_knn")
    return idx, dist


def rank(Q, X, ret_dist, metric="l2"):
    """Number of database points strictly closer than each returned distance."""
    Q, X = _f32(Q), _f32(X)
    ret = np.ascontiguousarray(ret_dist, dtype=np.float64)
    out = np.empty(Q.shape[0], np.int64)
    _check(_load().orc_rank(_p(Q), Q.shape[0], _p(X), X.shape[0], Q.shape[1], METRICS[metric],
                            _p(ret), _p(out)), "rank")
    return out


def rbc_build_exact(X, rep_idx, metric="l2"):
    """Exact-mode RBC: owner position of each point, radii psi, CSR lists."""
    X = _f32(X)
    reps = np.ascontiguousarray(rep_idx, dtype=np.int64)
    n, d = X.shape
    n_r = reps.shape[0]
    owner = np.empty(n, np.int32)
    psi = np.empty(n_r, np.float64)
    off = np.empty(n_r + 1, np.int64)
    ids = np.empty(n, np.int64)
    _check(_load().orc_rbc_build_exact(_p(X), n, d, METRICS[metric], _p(reps), n_r, _p(owner),
                                       _p(psi), _p(off), _p(ids)), "rbc_build_exact")
    return {"rep_idx": reps, "owner": owner, "psi": psi, "list_off": off, "list_ids": ids}


def rbc_search_exact(Q, X, index, k, metric="l2", strict=True, return_kept=False):
    """Exact RBC search: (idx, dist, ncand, nkept[, kept mask])."""
    Q, X = _f32(Q), _f32(X)
    m, d = Q.shape
    reps = index["rep_idx"]
    n_r = reps.shape[0]
    idx = np.empty((m, k), np.int64)
    dist = np.empty((m, k), np.float64)
    ncand = np.empty(m, np.int64)
    nkept = np.empty(m, np.int32)
    kept = np.empty((m, n_r), np.uint8) if return_kept else None
    _check(_load().orc_rbc_search_exact(
        _p(Q), m, _p(X), X.shape[0], d, METRICS[metric], _p(reps), n_r, _p(index["psi"]),
        _p(index["list_off"]), _p(index["list_ids"]), k, 1 if strict else 0, _p(idx), _p(dist),
        _p(ncand), _p(nkept), _p(kept)), "rbc_search_exact")
    if return_kept:
        return idx, dist, ncand, nkept, kept.astype(bool)
    return idx, dist, ncand, nkept


def rbc_search_approx(Q, X, index, k, eps, metric="l2", return_kept=False):
    """The approximate variant beside Sec. 5: both pruning bounds divided by
    (1 + eps); the answer is BF over the kept lists.  (idx, dist, ncand,
    nkept[, kept mask])."""
    Q, X = _f32(Q), _f32(X)
    m, d = Q.shape
    reps = index["rep_idx"]
    n_r = reps.shape[0]
    idx = np.empty((m, k), np.int64)
    dist = np.empty((m, k), np.float64)
    ncand = np.empty(m, np.int64)
    nkept = np.empty(m, np.int32)
    kept = np.empty((m, n_r), np.uint8) if return_kept else None
    _check(_load().orc_rbc_search_approx(
        _p(Q), m, _p(X), X.shape[0], d, METRICS[metric], _p(reps), n_r, _p(index["psi"]),
        _p(index["list_off"]), _p(index["list_ids"]), k, 1, float(eps), _p(idx), _p(dist),
        _p(ncand), _p(nkept), _p(kept)), "rbc_search_approx")
    if return_kept:
        return idx, dist, ncand, nkept, kept.astype(bool)
    return idx, dist, ncand, nkept


def range_bf(Q, X, radius, metric="l2"):
    """Range search by its definition: (offsets[m+1], ids, distances) with
    query i's points at offsets[i] .. offsets[i+1], in (distance, id) order."""
    Q, X = _f32(Q), _f32(X)
    m, d = Q.shape
    cnt = np.zeros(m + 1, np.int64)
    _check(_load().orc_range_bf(_p(Q), m, _p(X), X.shape[0], d, METRICS[metric], float(radius),
                                _p(cnt), None, None), "range_bf count")
    off = np.zeros(m + 1, np.int64)
    off[1:] = np.cumsum(cnt[:m])
    idx = np.empty(max(int(off[-1]), 1), np.int64)
    dist = np.empty(max(int(off[-1]), 1), np.float64)
    _check(_load().orc_range_bf(_p(Q), m, _p(X), X.shape[0], d, METRICS[metric], float(radius),
                                _p(off), _p(idx), _p(dist)), "range_bf fill")
    return off, idx[:off[-1]], dist[:off[-1]]


def rbc_build_oneshot(X, rep_idx, s, metric="l2"):
    """One-shot RBC: the s nearest points of each representative, and psi."""
    X = _f32(X)
    reps = np.ascontiguousarray(rep_idx, dtype=np.int64)
    n, d = X.shape
    lists = np.empty((reps.shape[0], s), np.int64)
    psi = np.empty(reps.shape[0], np.float64)
    _check(_load().orc_rbc_build_oneshot(_p(X), n, d, METRICS[metric], _p(reps), reps.shape[0],
                                         s, _p(lists), _p(psi)), "rbc_build_oneshot")
    return {"rep_idx": reps, "lists": lists, "psi": psi, "s": s}


def rbc_search_oneshot(Q, X, index, k, metric="l2"):
    """One-shot RBC search: (idx, dist, chosen representative position)."""
    Q, X = _f32(Q), _f32(X)
    m, d = Q.shape
    reps = index["rep_idx"]
    lists = np.ascontiguousarray(index["lists"], dtype=np.int64)
    idx = np.empty((m, k), np.int64)
    dist = np.empty((m, k), np.float64)
    rep = np.empty(m, np.int64)
    _check(_load().orc_rbc_search_oneshot(
        _p(Q), m, _p(X), X.shape[0], d, METRICS[metric], _p(reps), reps.shape[0], index["s"],
        _p(lists), k, _p(idx), _p(dist), _p(rep)), "rbc_search_oneshot")
    return idx, dist, rep
