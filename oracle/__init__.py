"""CPU oracle for range retrieval over graph indices -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference for every step of the GPU library's
hot path (Manohar, Kim, Blelloch, "Range Retrieval with Graph-Based
Indices"): squared-L2 distances, Definition 2.1 by enumeration, Algorithms
1-6, the average-precision (range recall) metric of Definition 2.2, and a
DiskANN/Vamana builder.  The arithmetic lives in ``rr_oracle.c``; this module
is ctypes marshalling plus the two radius rules and recall, written with
numpy on top of the oracle's own outputs.

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import this module.  The GPU library never does, and this module imports
nothing from it.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

U8, I8, F32 = 0, 1, 2
PLAIN, ES, ADAPTIVE, DOUBLING = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation pragmas)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC,
             "-lpthread", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("beam", C.c_int32), ("es_enable", C.c_int32),
                ("es_visit_limit", C.c_int32), ("es_radius", C.c_double),
                ("lam", C.c_double), ("max_beam", C.c_int64), ("metric", C.c_int32)]


L2, IP = 0, 1
_METRICS = {"l2": L2, "ip": IP}


def _metric(m) -> int:
    return _METRICS[m] if isinstance(m, str) else int(m)


class _Stats(C.Structure):
    _fields_ = [("visits", C.c_int64), ("evals", C.c_int64), ("greedy_visits", C.c_int64),
                ("greedy_evals", C.c_int64), ("count", C.c_int64), ("final_beam", C.c_int64),
                ("es_fired", C.c_int32), ("expanded", C.c_int32), ("rounds", C.c_int32),
                ("truncated", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("nq", C.c_int64), ("total", C.c_int64), ("offsets", C.POINTER(C.c_int64)),
                ("ids", C.POINTER(C.c_int32)), ("dists", C.POINTER(C.c_double)),
                ("stats", C.POINTER(_Stats))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        vp, i64, i32, dp = C.c_void_p, C.c_int64, C.c_int32, C.POINTER(C.c_double)
        lib.orc_dist.restype = C.c_double
        lib.orc_dist.argtypes = [C.c_int, vp, vp, i32, C.c_int]
        lib.orc_brute_force.argtypes = [vp, C.c_int, i64, i32, vp, i64, dp, C.c_int,
                                        C.POINTER(_Result), C.c_int]
        lib.orc_nn_dist.argtypes = [vp, C.c_int, i64, i32, vp, i64, C.c_int, dp, C.c_int]
        lib.orc_pair_dists.argtypes = [vp, C.c_int, i64, i32, vp, i64, C.c_int, dp, C.c_int]
        lib.orc_range_search.argtypes = [vp, C.c_int, i64, i32, C.POINTER(C.c_int32), i32, i32,
                                         vp, i64, dp, C.POINTER(_Params), C.c_int,
                                         C.POINTER(_Result)]
        lib.orc_es_profile.argtypes = [vp, C.c_int, i64, i32, C.POINTER(C.c_int32), i32, i32, vp,
                                       i64, dp, i64, i64, C.c_int, vp, vp, C.c_int]
        lib.orc_medoid.restype = C.c_int32
        lib.orc_medoid.argtypes = [vp, C.c_int, i64, i32]
        lib.orc_build_vamana.argtypes = [vp, C.c_int, i64, i32, i32, i32, C.c_double, i32,
                                         C.POINTER(C.c_int64), C.c_int, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32)]
        lib.orc_result_free.argtypes = [C.POINTER(_Result)]
        lib.orc_robust_prune.restype = C.c_int32
        lib.orc_robust_prune.argtypes = [vp, C.c_int, i64, i32, i32, C.POINTER(C.c_int32), i64,
                                         C.c_double, i32, C.POINTER(C.c_int32)]
        _lib = lib
    return _lib


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.uint8:
        return U8
    if a.dtype == np.int8:
        return I8
    if a.dtype == np.float32:
        return F32
    raise TypeError(f"unsupported vector dtype {a.dtype}")


def _threads(threads):
    if threads:
        return int(threads)
    return max(1, min(16, os.cpu_count() or 1))


@dataclass
class Result:
    """CSR range-search output: per query q, ids[offsets[q]:offsets[q+1]]."""
    offsets: np.ndarray
    ids: np.ndarray
    dists: np.ndarray
    stats: np.ndarray | None  # structured array of per-query counters

    @property
    def nq(self):
        return len(self.offsets) - 1

    def query(self, q):
        a, b = self.offsets[q], self.offsets[q + 1]
        return self.ids[a:b], self.dists[a:b]

    def counts(self):
        return np.diff(self.offsets)


_STATS_DTYPE = np.dtype([("visits", np.int64), ("evals", np.int64), ("greedy_visits", np.int64),
                         ("greedy_evals", np.int64), ("count", np.int64),
                         ("final_beam", np.int64), ("es_fired", np.int32),
                         ("expanded", np.int32), ("rounds", np.int32),
                         ("truncated", np.int32)])


def _take(res: _Result, with_stats: bool) -> Result:
    lib = _load()
    nq, tot = res.nq, res.total
    off = np.ctypeslib.as_array(res.offsets, shape=(nq + 1,)).copy()
    ids = np.ctypeslib.as_array(res.ids, shape=(max(tot, 1),))[:tot].copy()
    dists = np.ctypeslib.as_array(res.dists, shape=(max(tot, 1),))[:tot].copy()
    st = None
    if with_stats and nq > 0:
        raw = C.string_at(res.stats, nq * C.sizeof(_Stats))
        st = np.frombuffer(raw, dtype=_STATS_DTYPE).copy()
    lib.orc_result_free(C.byref(res))
    return Result(off, ids, dists, st)


def _c(a, dt=None):
    a = np.ascontiguousarray(a if dt is None else a.astype(dt, copy=False))
    return a


def _radius_array(radius, nq):
    r = np.asarray(radius, dtype=np.float64)
    if r.ndim == 0:
        r = np.full(nq, float(r))
    if r.shape != (nq,):
        raise ValueError("radius must be a scalar or one value per query")
    return np.ascontiguousarray(r)


def dist(a: np.ndarray, b: np.ndarray, metric="l2") -> float:
    """Squared L2 (or, with metric="ip", the negated inner product) of two
    vectors (exact for integer data, FP64 for float32)."""
    a, b = _c(a), _c(b)
    if a.dtype != b.dtype or a.shape != b.shape:
        raise ValueError("dtype/shape mismatch")
    return _load().orc_dist(_dtype_code(a), a.ctypes.data, b.ctypes.data, a.shape[-1],
                            _metric(metric))


def brute_force(base, queries, radius, threads=None, metric="l2") -> Result:
    """Definition 2.1 by enumeration: K_q = {p : d(p, q) <= r_q}."""
    base, queries = _c(base), _c(queries)
    nq = queries.shape[0]
    r = _radius_array(radius, nq)
    res = _Result()
    rc = _load().orc_brute_force(base.ctypes.data, _dtype_code(base), base.shape[0], base.shape[1],
                                 queries.ctypes.data, nq,
                                 r.ctypes.data_as(C.POINTER(C.c_double)), _threads(threads),
                                 C.byref(res), _metric(metric))
    if rc != 0:
        raise ValueError("orc_brute_force: invalid arguments")
    return _take(res, False)


def nn_dist(base, queries, threads=None, metric="l2") -> np.ndarray:
    """Distance from each query to its nearest base point."""
    base, queries = _c(base), _c(queries)
    out = np.zeros(queries.shape[0], dtype=np.float64)
    rc = _load().orc_nn_dist(base.ctypes.data, _dtype_code(base), base.shape[0], base.shape[1],
                             queries.ctypes.data, queries.shape[0], _threads(threads),
                             out.ctypes.data_as(C.POINTER(C.c_double)), _metric(metric))
    if rc != 0:
        raise ValueError("orc_nn_dist: invalid arguments")
    return out


def range_search(base, adj, entry, queries, radius, mode=PLAIN, beam=32, es_enable=False,
                 es_visit_limit=20, es_radius=0.0, lam=1.0, max_beam=1 << 20,
                 threads=None, metric="l2") -> Result:
    """Graph range search: mode PLAIN / ES / ADAPTIVE / DOUBLING (Algorithms 1-6)."""
    base, queries = _c(base), _c(queries)
    adj = _c(adj, np.int32)
    nq = queries.shape[0]
    r = _radius_array(radius, nq)
    p = _Params(int(mode), int(beam), int(bool(es_enable) or mode == ES), int(es_visit_limit),
                float(es_radius), float(lam), int(max_beam), _metric(metric))
    res = _Result()
    rc = _load().orc_range_search(base.ctypes.data, _dtype_code(base), base.shape[0],
                                  base.shape[1], adj.ctypes.data_as(C.POINTER(C.c_int32)),
                                  adj.shape[1], int(entry), queries.ctypes.data, nq,
                                  r.ctypes.data_as(C.POINTER(C.c_double)), C.byref(p),
                                  _threads(threads), C.byref(res))
    if rc != 0:
        raise ValueError("orc_range_search: invalid arguments")
    return _take(res, True)


def es_profile(base, adj, entry, queries, radius, beam, step, threads=None, metric="l2"):
    """Early-stopping metrics of the paper's appendix at visit count `step`
    of Algorithm 1 (beam `beam`, no stopping rule).  Returns (metrics[nq, 4]
    = d_visited, d_top1, d_top10, d_start; flags[nq, 2] = reached, found)."""
    base, queries = _c(base), _c(queries)
    adj = _c(adj, np.int32)
    nq = queries.shape[0]
    r = _radius_array(radius, nq)
    metrics = np.empty((nq, 4), np.float64)
    flags = np.empty((nq, 2), np.int8)
    rc = _load().orc_es_profile(base.ctypes.data, _dtype_code(base), base.shape[0], base.shape[1],
                                adj.ctypes.data_as(C.POINTER(C.c_int32)), adj.shape[1],
                                int(entry), queries.ctypes.data, nq,
                                r.ctypes.data_as(C.POINTER(C.c_double)), int(beam), int(step),
                                _threads(threads), metrics.ctypes.data, flags.ctypes.data,
                                _metric(metric))
    if rc != 0:
        raise ValueError("orc_es_profile: invalid arguments")
    return metrics, flags


def medoid(base) -> int:
    base = _c(base)
    return int(_load().orc_medoid(base.ctypes.data, _dtype_code(base), base.shape[0],
                                  base.shape[1]))


def build_vamana(base, R, L, alpha, order, passes=2, threads=None):
    """DiskANN/Vamana graph: returns (adj[n, R] int32 with -1 padding, entry)."""
    base = _c(base)
    n = base.shape[0]
    order = _c(order, np.int64)
    if order.shape != (n,) or not np.array_equal(np.sort(order), np.arange(n)):
        raise ValueError("order must be a permutation of range(n)")
    adj = np.empty((n, R), dtype=np.int32)
    entry = C.c_int32(0)
    rc = _load().orc_build_vamana(base.ctypes.data, _dtype_code(base), n, base.shape[1], int(R),
                                  int(L), float(alpha), int(passes),
                                  order.ctypes.data_as(C.POINTER(C.c_int64)), _threads(threads),
                                  adj.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(entry))
    if rc != 0:
        raise ValueError("orc_build_vamana: invalid arguments")
    return adj, int(entry.value)


def robust_prune(base, p, cand, alpha, R):
    """RobustPrune(p, cand, alpha, R) of the Vamana construction."""
    base = _c(base)
    cand = _c(np.asarray(cand), np.int32)
    out = np.empty(R, dtype=np.int32)
    k = _load().orc_robust_prune(base.ctypes.data, _dtype_code(base), base.shape[0],
                                 base.shape[1], int(p), cand.ctypes.data_as(C.POINTER(C.c_int32)),
                                 cand.size, float(alpha), int(R),
                                 out.ctypes.data_as(C.POINTER(C.c_int32)))
    if k < 0:
        raise ValueError("orc_robust_prune: invalid arguments")
    return out[:k].copy()


# ---------------------------------------------------------------------------
# metric and radius rules
# ---------------------------------------------------------------------------

def range_recall(truth: Result, found: Result) -> float:
    """Average precision of Definition 2.2: sum |K_q & K'_q| / sum |K_q|.

    Returns nan when no query has a true result (the ratio is undefined)."""
    if truth.nq != found.nq:
        raise ValueError("query count mismatch")
    hit = 0
    for q in range(truth.nq):
        t, _ = truth.query(q)
        f, _ = found.query(q)
        hit += np.intersect1d(t, f, assume_unique=True).size
    tot = int(truth.offsets[-1])
    return float("nan") if tot == 0 else hit / tot


def pair_dists(base, queries, threads=None, metric="l2") -> np.ndarray:
    """All query-base distances as an nq x n float64 matrix."""
    base, queries = _c(base), _c(queries)
    out = np.empty((queries.shape[0], base.shape[0]), dtype=np.float64)
    rc = _load().orc_pair_dists(base.ctypes.data, _dtype_code(base), base.shape[0], base.shape[1],
                                queries.ctypes.data, queries.shape[0], _threads(threads),
                                out.ctypes.data_as(C.POINTER(C.c_double)), _metric(metric))
    if rc != 0:
        raise ValueError("orc_pair_dists: invalid arguments")
    return out


def percentile_radius(base, queries, p, threads=None, metric="l2") -> float:
    """Inverted-CDF radius: the k-th smallest of all nq*n distances,
    k = ceil(p * nq * n).  Enumerates every pair (moderate inputs only)."""
    ds = pair_dists(base, queries, threads, metric).ravel()
    k = max(1, math.ceil(p * ds.size))
    return float(np.partition(ds, k - 1)[k - 1])


def empty_fraction_radius(base, queries, nonempty_frac, threads=None, metric="l2") -> float:
    """Radius that leaves at least `nonempty_frac` of queries non-empty: the
    ceil(f * nq)-th smallest per-query nearest-neighbour distance."""
    nn = np.sort(nn_dist(base, queries, threads, metric))
    k = max(1, math.ceil(nonempty_frac * len(nn)))
    return float(nn[k - 1])
