"""Python binding of the C ABI in include/rr.h (argument marshalling only).

Every step of the search runs in the HIP library ``librr.so``; PyTorch only
provides device memory (through the library's allocator callbacks) and the
stream.  Importing this module on a machine without the built library raises
instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librr.so")

RR_OK, RR_EINVAL, RR_ENOMEM, RR_EHIP, RR_EIO, RR_ESTATE, RR_EBUSY = range(7)
U8, I8, F32 = 0, 1, 2
PLAIN, ES, ADAPTIVE, DOUBLING = 0, 1, 2, 3
EXACT, BF16_RECHECK, SQ8_RERANK = 0, 1, 2
L2, IP = 0, 1

_MODES = {"plain": PLAIN, "es": ES, "adaptive": ADAPTIVE, "doubling": DOUBLING}


class RRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"[rr status {status}] {msg}")
        self.status = status


class BuildParams(C.Structure):
    _fields_ = [("R", C.c_int32), ("L", C.c_int32), ("alpha", C.c_double), ("passes", C.c_int32),
                ("threads", C.c_int32), ("seed", C.c_uint64), ("order", C.POINTER(C.c_int64)),
                ("verbose", C.c_int32)]


class SearchParams(C.Structure):
    _fields_ = [("mode", C.c_int32), ("beam", C.c_int32), ("es_enable", C.c_int32),
                ("es_visit_limit", C.c_int32), ("es_radius", C.c_double), ("lam", C.c_double),
                ("precision", C.c_int32), ("recheck_margin", C.c_double),
                ("max_results_per_query", C.c_int64), ("max_beam", C.c_int64),
                ("result_capacity", C.c_int64), ("cache_slots", C.c_int32),
                ("waves_per_group", C.c_int32), ("timing", C.c_int32)]


class QueryStats(C.Structure):
    _fields_ = [("visits", C.c_int32), ("evals", C.c_int32), ("greedy_visits", C.c_int32),
                ("greedy_evals", C.c_int32), ("count", C.c_int32), ("final_beam", C.c_int32),
                ("es_fired", C.c_int16), ("expanded", C.c_int16), ("truncated", C.c_int16),
                ("cache_overflow", C.c_int16), ("rechecked", C.c_int32), ("rounds", C.c_int32),
                ("edges", C.c_int32), ("greedy_edges", C.c_int32)]


STATS_DTYPE = np.dtype([("visits", np.int32), ("evals", np.int32), ("greedy_visits", np.int32),
                        ("greedy_evals", np.int32), ("count", np.int32),
                        ("final_beam", np.int32), ("es_fired", np.int16),
                        ("expanded", np.int16), ("truncated", np.int16),
                        ("cache_overflow", np.int16), ("rechecked", np.int32),
                        ("rounds", np.int32), ("edges", np.int32), ("greedy_edges", np.int32)])
assert STATS_DTYPE.itemsize == C.sizeof(QueryStats)


class BatchStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in
                ("nq", "total_results", "visits", "evals", "greedy_visits", "greedy_evals",
                 "rechecked", "es_fired", "expanded", "truncated", "cache_overflow",
                 "bytes_algorithmic", "bytes_beam")] + [
                (k, C.c_double) for k in ("beam_ms", "greedy_ms", "total_ms")] + [
                (k, C.c_int64) for k in ("greedy_levels", "greedy_items", "bytes_greedy")] + [
                ("greedy_kernel_ms", C.c_double), ("greedy_set_ops", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneReport(C.Structure):
    _fields_ = [("tried", C.c_int32), ("beam", C.c_int32), ("waves_per_group", C.c_int32),
                ("cache_slots", C.c_int32), ("ms", C.c_double), ("recall", C.c_double),
                ("met_target", C.c_int32), ("es_dropped", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ESTuneReport(C.Structure):
    _fields_ = [("tried", C.c_int32), ("es_enable", C.c_int32), ("es_visit_limit", C.c_int32),
                ("es_radius", C.c_double), ("ms", C.c_double), ("recall", C.c_double),
                ("met_target", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(C.Structure):
    _fields_ = [("slots", C.c_int32), ("step_budget", C.c_int32),
                ("result_capacity", C.c_int64), ("max_pending", C.c_int32),
                ("hbm_budget", C.c_int64)]


class Completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("count", C.c_int64), ("truncated", C.c_int32),
                ("ticks", C.c_int32), ("t_arrival", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("stats", QueryStats)]


class ServerInfo(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("ticks", "submitted", "admitted", "completed",
                                          "pending", "resident", "max_resident")] + [
                ("busy_s", C.c_double), ("slots", C.c_int64), ("device_bytes", C.c_int64),
                ("retried", C.c_int64), ("max_tick_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


# exported symbols and their signatures: (restype, argtypes)
_VP, _I64, _I32 = C.c_void_p, C.c_int64, C.c_int32
SIGNATURES = {
    "rr_last_error": (C.c_char_p, []),
    "rr_version": (C.c_char_p, []),
    "rr_default_build_params": (None, [C.POINTER(BuildParams)]),
    "rr_default_search_params": (None, [C.POINTER(SearchParams)]),
    "rr_index_build": (C.c_int, [_VP, C.c_int, _I64, _I32, C.POINTER(BuildParams),
                                 C.POINTER(_VP)]),
    "rr_index_from_graph": (C.c_int, [_VP, C.c_int, _I64, _I32, C.POINTER(C.c_int32), _I32,
                                      _I32, C.POINTER(_VP)]),
    "rr_index_graph": (C.c_int, [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)]),
    "rr_index_info": (C.c_int, [_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32)]),
    "rr_index_set_metric": (C.c_int, [_VP, _I32]),
    "rr_index_metric": (C.c_int, [_VP, C.POINTER(C.c_int32)]),
    "rr_index_save": (C.c_int, [_VP, C.c_char_p]),
    "rr_index_load": (C.c_int, [C.c_char_p, C.POINTER(_VP)]),
    "rr_index_to_device": (C.c_int, [_VP, C.POINTER(Allocator), _VP]),
    "rr_index_free": (None, [_VP]),
    "rr_range_search": (C.c_int, [_VP, _VP, _I64, C.c_double, _VP, C.POINTER(SearchParams),
                                  C.POINTER(Allocator), _VP, C.POINTER(_VP)]),
    "rr_range_search_noalloc": (C.c_int, [_VP, _VP, _I64, C.c_double, _VP,
                                          C.POINTER(SearchParams), _VP, _VP, _I64, _VP, _VP, _VP]),
    "rr_brute_force": (C.c_int, [_VP, _VP, _I64, C.c_double, _VP, C.POINTER(Allocator), _VP,
                                 C.POINTER(_VP)]),
    "rr_nn_dist": (C.c_int, [_VP, _VP, _I64, _VP, _VP]),
    "rr_select_radius": (C.c_int, [_VP, _VP, _I64, C.POINTER(C.c_double), _I32,
                                   C.POINTER(C.c_double), C.POINTER(Allocator), _VP]),
    "rr_probe_row_gather": (C.c_int, [_VP, _I64, C.c_uint64, _VP, _I64, C.POINTER(C.c_int64), _VP]),
    "rr_results_total": (C.c_int, [_VP, C.POINTER(C.c_int64)]),
    "rr_results_copy": (C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "rr_results_stats": (C.c_int, [_VP, C.POINTER(QueryStats), C.POINTER(BatchStats)]),
    "rr_results_level_profile": (C.c_int, [_VP, _I32, C.POINTER(C.c_int64),
                                           C.POINTER(C.c_double), C.POINTER(C.c_double),
                                           C.POINTER(C.c_int32)]),
    "rr_results_free": (None, [_VP]),
    "rr_server_create": (C.c_int, [_VP, C.POINTER(SearchParams), C.POINTER(ServerConfig),
                                   C.POINTER(Allocator), C.POINTER(_VP)]),
    "rr_server_clock": (C.c_double, [_VP]),
    "rr_server_submit": (C.c_int, [_VP, _VP, C.c_double, C.c_uint64, C.c_double]),
    "rr_server_poll": (C.c_int, [_VP, C.POINTER(Completion), _I32, C.POINTER(C.c_int32)]),
    "rr_server_result": (C.c_int, [_VP, C.c_uint64, _VP, _VP, _I64, C.POINTER(C.c_int64)]),
    "rr_server_drain": (C.c_int, [_VP, C.c_double]),
    "rr_server_info_get": (C.c_int, [_VP, C.POINTER(ServerInfo)]),
    "rr_server_destroy": (None, [_VP]),
    "rr_autotune": (C.c_int, [_VP, _VP, _I64, C.c_double, _VP, _VP, C.c_double, _I32,
                              C.POINTER(SearchParams), C.POINTER(TuneReport),
                              C.POINTER(Allocator), _VP]),
    "rr_tune_early_stop": (C.c_int, [_VP, _VP, _I64, C.c_double, _VP, _VP, C.c_double, _I32,
                                     C.POINTER(SearchParams), C.POINTER(ESTuneReport),
                                     C.POINTER(Allocator), _VP]),
    "rr_es_profile": (C.c_int, [_VP, _VP, _I64, C.c_double, _VP, _I32, _I32, _VP, _VP,
                                C.POINTER(Allocator), _VP]),
}

_lib = None


def lib():
    """Load librr.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2502_13245_amd.build_lib`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def _check(st):
    if st != RR_OK:
        raise RRError(st, lib().rr_last_error().decode())


def _dtype_code(dt) -> int:
    dt = np.dtype(dt)
    if dt == np.uint8:
        return U8
    if dt == np.int8:
        return I8
    if dt == np.float32:
        return F32
    raise TypeError(f"unsupported vector dtype {dt}")


def _metric_code(metric) -> int:
    if metric in (L2, "l2", "L2"):
        return L2
    if metric in (IP, "ip", "IP"):
        return IP
    raise ValueError(f"unknown metric {metric!r}")


# ---------------------------------------------------------------------------
# torch-backed device memory
# ---------------------------------------------------------------------------

class TorchAllocator:
    """Device memory for the library from torch's caching allocator."""

    def __init__(self, device=None):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        self.live = {}

        def _alloc(nbytes, stream, ctx):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
                p = t.data_ptr()
                self.live[p] = t
                return p
            except Exception:
                return None

        def _free(ptr, stream, ctx):
            self.live.pop(ptr, None)

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.struct = Allocator(self._alloc, self._free, None)

    def ref(self):
        return C.byref(self.struct)


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# index
# ---------------------------------------------------------------------------

class Index:
    """A proximity-graph index (host copy; on the device after to_device())."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle)
        self._alloc = None
        self.device = None
        self._dt = None

    def dtype_code(self) -> int:
        """The element type code (fixed for the index's lifetime)."""
        if self._dt is None:
            self._dt = self.info()["dtype"]
        return self._dt

    def free(self):
        """Release the host and device copies now (the index is unusable after)."""
        if self._h and self._h.value:
            lib().rr_index_free(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @staticmethod
    def build(base: np.ndarray, R=64, L=128, alpha=1.2, passes=2, threads=0, seed=0,
              order=None, verbose=False, metric="l2") -> "Index":
        """build_graph: DiskANN/Vamana construction on the host (L2 graph;
        `metric` is the distance the searches use)."""
        base = np.ascontiguousarray(base)
        bp = BuildParams()
        lib().rr_default_build_params(C.byref(bp))
        bp.R, bp.L, bp.alpha, bp.passes, bp.threads, bp.seed = R, L, alpha, passes, threads, seed
        bp.verbose = int(bool(verbose))
        if order is not None:
            order = np.ascontiguousarray(order, dtype=np.int64)
            bp.order = order.ctypes.data_as(C.POINTER(C.c_int64))
        out = C.c_void_p()
        _check(lib().rr_index_build(base.ctypes.data, _dtype_code(base.dtype), base.shape[0],
                                    base.shape[1], C.byref(bp), C.byref(out)))
        return Index(out.value).set_metric(metric)

    @staticmethod
    def from_graph(base: np.ndarray, adj: np.ndarray, entry: int, metric="l2") -> "Index":
        base = np.ascontiguousarray(base)
        adj = np.ascontiguousarray(adj, dtype=np.int32)
        out = C.c_void_p()
        _check(lib().rr_index_from_graph(base.ctypes.data, _dtype_code(base.dtype),
                                         base.shape[0], base.shape[1],
                                         adj.ctypes.data_as(C.POINTER(C.c_int32)),
                                         adj.shape[1], int(entry), C.byref(out)))
        return Index(out.value).set_metric(metric)

    def set_metric(self, metric):
        """rr_index_set_metric: "l2" (squared Euclidean) or "ip" (negated
        inner product); before to_device()."""
        _check(lib().rr_index_set_metric(self._h, _metric_code(metric)))
        return self

    @property
    def metric(self) -> str:
        m = C.c_int32()
        _check(lib().rr_index_metric(self._h, C.byref(m)))
        return ("l2", "ip")[m.value]

    @staticmethod
    def load(path: str) -> "Index":
        out = C.c_void_p()
        _check(lib().rr_index_load(path.encode(), C.byref(out)))
        return Index(out.value)

    def save(self, path: str):
        _check(lib().rr_index_save(self._h, path.encode()))

    def info(self):
        n, d, dt, R, e = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().rr_index_info(self._h, C.byref(n), C.byref(d), C.byref(dt), C.byref(R),
                                   C.byref(e)))
        return dict(n=n.value, d=d.value, dtype=dt.value, R=R.value, entry=e.value)

    def graph(self):
        inf = self.info()
        adj = np.empty((inf["n"], inf["R"]), dtype=np.int32)
        R, e = C.c_int32(), C.c_int32()
        _check(lib().rr_index_graph(self._h, adj.ctypes.data_as(C.POINTER(C.c_int32)),
                                    C.byref(R), C.byref(e)))
        return adj, e.value

    def to_device(self, device="cuda:0", stream=None):
        import torch
        torch.cuda.set_device(torch.device(device))
        self._alloc = TorchAllocator(device)
        _check(lib().rr_index_to_device(self._h, self._alloc.ref(), _stream_handle(stream)))
        self.device = device
        return self


# ---------------------------------------------------------------------------
# results
# ---------------------------------------------------------------------------

@dataclass
class Results:
    offsets: "object"   # torch int64 [nq + 1] on the device
    ids: "object"       # torch int32 [total]
    dists: "object"     # torch int32 (integer data) / float32 (float data)
    stats: np.ndarray | None
    batch: dict | None

    def numpy(self):
        return (self.offsets.cpu().numpy(), self.ids.cpu().numpy(), self.dists.cpu().numpy())


class PendingResults:
    """Handle of a search whose kernels may still run (rr_results*)."""

    def __init__(self, handle, nq, dtype, alloc, keep):
        self._h = C.c_void_p(handle)
        self.nq = nq
        self.dtype = dtype
        self._alloc = alloc
        self._keep = keep

    def __del__(self):
        try:
            if self._h and self._h.value:
                lib().rr_results_free(self._h)
                self._h = C.c_void_p(0)
        except Exception:
            pass

    def total(self) -> int:
        t = C.c_int64()
        _check(lib().rr_results_total(self._h, C.byref(t)))
        return t.value

    def fetch(self, with_stats=True, stream=None) -> Results:
        import torch
        dev = self._alloc.device
        total = self.total()
        offsets = torch.empty(self.nq + 1, dtype=torch.int64, device=dev)
        ids = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
        dists = torch.empty(max(total, 1),
                            dtype=torch.float32 if self.dtype == F32 else torch.int32,
                            device=dev)
        _check(lib().rr_results_copy(self._h, C.c_void_p(ids.data_ptr()),
                                     C.c_void_p(dists.data_ptr()),
                                     C.c_void_p(offsets.data_ptr()), _stream_handle(stream)))
        st = None
        agg = None
        if with_stats:
            st = np.zeros(self.nq, dtype=STATS_DTYPE)
            b = BatchStats()
            _check(lib().rr_results_stats(
                self._h, st.ctypes.data_as(C.POINTER(QueryStats)) if self.nq else None,
                C.byref(b)))
            agg = b.as_dict()
            agg["levels"] = self.level_profile()
        return Results(offsets, ids[:total], dists[:total], st, agg)


    def level_profile(self, max_levels=64):
        """Per level of the greedy phase: points expanded and the time spent
        expanding them and regrouping the next level (ms)."""
        items = (C.c_int64 * max_levels)()
        exp_ms = (C.c_double * max_levels)()
        reg_ms = (C.c_double * max_levels)()
        n = C.c_int32()
        _check(lib().rr_results_level_profile(self._h, max_levels, items, exp_ms, reg_ms,
                                              C.byref(n)))
        return [dict(items=items[i], expand_ms=round(exp_ms[i], 4), regroup_ms=round(reg_ms[i], 4))
                for i in range(n.value)]


def search_params(mode="adaptive", beam=32, es_enable=False, es_visit_limit=20, es_radius=0.0,
                  lam=1.0, precision=EXACT, recheck_margin=0.02, max_results_per_query=None,
                  max_beam=None, result_capacity=0, cache_slots=0, waves_per_group=0,
                  timing=False):
    sp = SearchParams()
    lib().rr_default_search_params(C.byref(sp))
    sp.mode = _MODES[mode] if isinstance(mode, str) else int(mode)
    sp.beam = int(beam)
    sp.es_enable = int(bool(es_enable))
    sp.es_visit_limit = int(es_visit_limit)
    sp.es_radius = float(es_radius)
    sp.lam = float(lam)
    sp.precision = int(precision)
    sp.recheck_margin = float(recheck_margin)
    if max_results_per_query is not None:
        sp.max_results_per_query = int(max_results_per_query)
    if max_beam is not None:
        sp.max_beam = int(max_beam)
    sp.result_capacity = int(result_capacity)
    sp.cache_slots = int(cache_slots)
    sp.waves_per_group = int(waves_per_group)
    sp.timing = int(bool(timing))
    return sp


def _radius_args(radius, nq, device):
    import torch
    if isinstance(radius, torch.Tensor):
        r = radius.to(device=device, dtype=torch.float64).contiguous()
        if r.numel() != nq:
            raise ValueError("radius tensor must have one value per query")
        return 0.0, C.c_void_p(r.data_ptr()), r
    return float(radius), None, None


def range_search_async(index: Index, queries, radius, params: SearchParams | None = None,
                       stream=None, **kw) -> PendingResults:
    """Enqueue one batched range_search (queries: torch tensor on the index's device)."""
    import torch
    if index.device is None:
        raise RRError(RR_ESTATE, "index is not on the device")
    sp = params if params is not None else search_params(**kw)
    q = queries.contiguous()
    nq = q.shape[0] if q.dim() == 2 else 0
    r0, rdev, keep = _radius_args(radius, nq, q.device)
    out = C.c_void_p()
    _check(lib().rr_range_search(index._h, C.c_void_p(q.data_ptr()), nq, r0, rdev, C.byref(sp),
                                 index._alloc.ref(), _stream_handle(stream), C.byref(out)))
    return PendingResults(out.value, nq, index.dtype_code(), index._alloc, (q, keep))


def range_search(index: Index, queries, radius, params: SearchParams | None = None, stream=None,
                 with_stats=True, **kw) -> Results:
    """range_search(queries, radius, params) -> (ids, dists, offsets) + per-query counters."""
    return range_search_async(index, queries, radius, params, stream, **kw).fetch(with_stats, stream)


def range_search_noalloc(index: Index, queries, radius, capacity, params: SearchParams | None = None,
                         stream=None, with_stats=True, **kw):
    """rr_range_search_noalloc: the library allocates nothing; the caller's
    buffers (allocated here with torch) receive the CSR result.  Returns
    (offsets, ids, dists, stats): offsets int64 [nq + 1] (complete), ids and
    dists the first `capacity` entries, stats a device tensor of nq
    rr_query_stats records as raw bytes (or None)."""
    import torch
    if index.device is None:
        raise RRError(RR_ESTATE, "index is not on the device")
    sp = params if params is not None else search_params(**kw)
    q = queries.contiguous()
    nq = q.shape[0] if q.dim() == 2 else 0
    r0, rdev, keep = _radius_args(radius, nq, q.device)
    dev = q.device
    dt = index.dtype_code()
    offsets = torch.empty(nq + 1, dtype=torch.int64, device=dev)
    ids = torch.empty(max(int(capacity), 1), dtype=torch.int32, device=dev)
    dists = torch.empty(max(int(capacity), 1), dtype=torch.float32 if dt == F32 else torch.int32,
                        device=dev)
    stats = (torch.empty(max(nq, 1) * C.sizeof(QueryStats), dtype=torch.uint8, device=dev)
             if with_stats else None)
    _check(lib().rr_range_search_noalloc(index._h, C.c_void_p(q.data_ptr()), nq, r0, rdev,
                                         C.byref(sp), C.c_void_p(ids.data_ptr()),
                                         C.c_void_p(dists.data_ptr()), int(capacity),
                                         C.c_void_p(offsets.data_ptr()),
                                         C.c_void_p(stats.data_ptr()) if stats is not None else None,
                                         _stream_handle(stream)))
    return offsets, ids, dists, stats


def stats_from_bytes(raw) -> np.ndarray:
    """Per-query counters from the raw bytes of nq rr_query_stats records."""
    return np.frombuffer(raw.cpu().numpy().tobytes(), dtype=STATS_DTYPE)


def brute_force_async(index: Index, queries, radius, stream=None) -> PendingResults:
    """Exact range search by a dense scan (ground truth), as a result handle."""
    q = queries.contiguous()
    nq = q.shape[0]
    r0, rdev, keep = _radius_args(radius, nq, q.device)
    out = C.c_void_p()
    _check(lib().rr_brute_force(index._h, C.c_void_p(q.data_ptr()), nq, r0, rdev,
                                index._alloc.ref(), _stream_handle(stream), C.byref(out)))
    return PendingResults(out.value, nq, index.dtype_code(), index._alloc, (q, keep))


def brute_force(index: Index, queries, radius, stream=None) -> Results:
    """Exact range search by a dense scan (ground truth)."""
    return brute_force_async(index, queries, radius, stream).fetch(False, stream)


def autotune(index: Index, queries, radius, truth: PendingResults, target=0.9, reps=3,
             params: SearchParams | None = None, stream=None, **kw):
    """rr_autotune: beam width for the recall target, then kernel shape.
    Returns (SearchParams, report dict)."""
    sp = params if params is not None else search_params(**kw)
    q = queries.contiguous()
    nq = q.shape[0]
    r0, rdev, keep = _radius_args(radius, nq, q.device)
    rep = TuneReport()
    _check(lib().rr_autotune(index._h, C.c_void_p(q.data_ptr()), nq, r0, rdev, truth._h,
                             float(target), int(reps), C.byref(sp), C.byref(rep),
                             index._alloc.ref(), _stream_handle(stream)))
    return sp, rep.as_dict()


def tune_early_stop(index: Index, queries, radius, truth: PendingResults, target=0.9, reps=3,
                    params: SearchParams | None = None, stream=None, **kw):
    """rr_tune_early_stop: Algorithm 5's (vl, esr) for the recall target.
    Returns (SearchParams, report dict)."""
    sp = params if params is not None else search_params(**kw)
    q = queries.contiguous()
    nq = q.shape[0]
    r0, rdev, keep = _radius_args(radius, nq, q.device)
    rep = ESTuneReport()
    _check(lib().rr_tune_early_stop(index._h, C.c_void_p(q.data_ptr()), nq, r0, rdev, truth._h,
                                    float(target), int(reps), C.byref(sp), C.byref(rep),
                                    index._alloc.ref(), _stream_handle(stream)))
    return sp, rep.as_dict()


def es_profile(index: Index, queries, radius, beam, step, stream=None):
    """rr_es_profile: (metrics[nq, 4] = d_visited, d_top1, d_top10, d_start;
    flags[nq, 2] = reached, found) at visit count `step` of a plain beam
    search of width `beam`."""
    q = queries.contiguous()
    nq = q.shape[0]
    r0, rdev, keep = _radius_args(radius, nq, q.device)
    m = np.empty((nq, 4), np.float64)
    f = np.empty((nq, 2), np.int8)
    _check(lib().rr_es_profile(index._h, C.c_void_p(q.data_ptr()), nq, r0, rdev, int(beam),
                               int(step), m.ctypes.data, f.ctypes.data, index._alloc.ref(),
                               _stream_handle(stream)))
    return m, f


def nn_dist(index: Index, queries, stream=None):
    """Squared distance from each query to its nearest base point (torch float64)."""
    import torch
    q = queries.contiguous()
    out = torch.empty(q.shape[0], dtype=torch.float64, device=q.device)
    _check(lib().rr_nn_dist(index._h, C.c_void_p(q.data_ptr()), q.shape[0],
                            C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def select_radius(index: Index, queries, p, stream=None):
    """rr_select_radius: the k-th smallest of all query-base distances,
    k = ceil(p * nq * n), for one percentile p or a list of them."""
    q = queries.contiguous()
    ps = np.atleast_1d(np.asarray(p, dtype=np.float64))
    out = np.empty(len(ps), np.float64)
    _check(lib().rr_select_radius(index._h, C.c_void_p(q.data_ptr()), q.shape[0],
                                  ps.ctypes.data_as(C.POINTER(C.c_double)), len(ps),
                                  out.ctypes.data_as(C.POINTER(C.c_double)), index._alloc.ref(),
                                  _stream_handle(stream)))
    return float(out[0]) if np.ndim(p) == 0 else out


def probe_row_gather(index: Index, gathers: int, seed: int = 1, stream=None):
    """Launch the random row-read probe (rr_probe_row_gather) on `stream`.

    Returns the device tensor of per-workgroup uint32 word sums (int64)."""
    import torch
    if index.device is None:
        raise RRError(5, "index is not on the device (to_device)")
    n_parts = (int(gathers) + 1023) // 1024
    sink = torch.zeros(max(1, n_parts), dtype=torch.int64, device=index.device)
    parts = C.c_int64(0)
    _check(lib().rr_probe_row_gather(index._h, int(gathers), C.c_uint64(int(seed) & (2**64 - 1)),
                                     C.c_void_p(sink.data_ptr()), sink.numel(), C.byref(parts),
                                     _stream_handle(stream)))
    return sink[:parts.value]


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

class Server:
    """Continuous batching over resident slots (rr_server_*).

    Requests are host vectors; results come back to host memory.  The
    library's own thread runs the ticks, so ``submit`` never waits for the
    device.
    """

    def __init__(self, index: Index, params: SearchParams | None = None, slots=1024,
                 step_budget=0, result_capacity=0, max_pending=0, hbm_budget=0):
        if index.device is None:
            raise RRError(RR_ESTATE, "index is not on the device")
        self.index = index  # the server reads the index's device memory
        inf = index.info()
        self.d = inf["d"]
        self.np_dtype = {U8: np.uint8, I8: np.int8, F32: np.float32}[inf["dtype"]]
        self.dist_dtype = np.float32 if inf["dtype"] == F32 else np.int32
        params = params or search_params()
        cfg = ServerConfig(int(slots), int(step_budget), int(result_capacity), int(max_pending),
                           int(hbm_budget))
        out = C.c_void_p()
        _check(lib().rr_server_create(index._h, C.byref(params), C.byref(cfg), None,
                                      C.byref(out)))
        self._h = out

    def close(self):
        if self._h and self._h.value:
            lib().rr_server_destroy(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def clock(self) -> float:
        return lib().rr_server_clock(self._h)

    def submit(self, query, radius: float, tag: int, t_arrival: float = -1.0) -> bool:
        """Queue one request; False if the queue is full (RR_EBUSY)."""
        q = np.ascontiguousarray(query, dtype=self.np_dtype)
        if q.size != self.d:
            raise ValueError(f"query has {q.size} values, the index has d={self.d}")
        st = lib().rr_server_submit(self._h, q.ctypes.data, float(radius), int(tag),
                                    float(t_arrival))
        if st == RR_EBUSY:
            return False
        _check(st)
        return True

    def poll(self, max_items=4096):
        buf = (Completion * max_items)()
        n = C.c_int32()
        _check(lib().rr_server_poll(self._h, buf, max_items, C.byref(n)))
        return [buf[i] for i in range(n.value)]

    def result(self, tag: int):
        """(ids, dists) of a finished request, ordered by (distance, id)."""
        cnt = C.c_int64()
        st = lib().rr_server_result(self._h, int(tag), None, None, 0, C.byref(cnt))
        if st == RR_OK:
            return np.empty(0, np.int32), np.empty(0, self.dist_dtype)
        if st != RR_ENOMEM:
            _check(st)
        ids = np.empty(cnt.value, np.int32)
        dists = np.empty(cnt.value, self.dist_dtype)
        _check(lib().rr_server_result(self._h, int(tag), ids.ctypes.data, dists.ctypes.data,
                                      cnt.value, C.byref(cnt)))
        return ids, dists

    def drain(self, timeout=-1.0):
        _check(lib().rr_server_drain(self._h, float(timeout)))

    def info(self) -> dict:
        inf = ServerInfo()
        _check(lib().rr_server_info_get(self._h, C.byref(inf)))
        return inf.as_dict()
