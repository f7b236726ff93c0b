"""Python binding of libgsmat (sparse-matrix BGP join on MI355X).

Argument marshalling only: every step of storage building, planning and the
join runs inside the C-ABI library (HIP kernels for gfx950).  The function
names are those of the C-ABI (include/gsmat.h).  The library is loaded from
this directory; if it has not been built, importing the binding fails loudly.

Streams: functions take an optional `stream` (an int hipStream_t handle).  By
default torch's current stream on the current device is used when torch has a
GPU, else the null stream.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgsmat.so")

GSMAT_OK, GSMAT_EINVAL, GSMAT_ENOMEM, GSMAT_EHIP, GSMAT_ESTATE, GSMAT_EUNSUPPORTED, GSMAT_ETOOBIG = range(7)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ESTATE", 5: "EUNSUPPORTED",
                6: "ETOOBIG"}
STEP_SCAN, STEP_INTERSECT, STEP_EXPAND, STEP_FILTER, STEP_CARTESIAN = range(5)
STEP_NAMES = {0: "SCAN", 1: "INTERSECT", 2: "EXPAND", 3: "FILTER", 4: "CARTESIAN"}
PLAN_PAPER, PLAN_DEFAULT, PLAN_ADAPTIVE = 0, 1, 2
K_COUNT, K_SCAN, K_WRITE, K_COMPACT, K_OTHER = range(5)
K_NAMES = ["count", "scan", "write", "compact", "other"]
EXPORTED = [
    "gsmat_load_triples", "gsmat_build_index", "gsmat_store_stats", "gsmat_pred_stats",
    "gsmat_export_matrix", "gsmat_store_free", "gsmat_plan", "gsmat_plan_from_stats",
    "gsmat_plan_info", "gsmat_plan_free", "gsmat_join", "gsmat_result_info",
    "gsmat_fetch_bindings", "gsmat_result_free", "gsmat_last_error", "gsmat_prof_enable",
    "gsmat_prof_read", "gsmat_prof_host", "gsmat_release_pools", "gsmat_plan_batch",
    "gsmat_join_batch", "gsmat_plan_free_many", "gsmat_result_free_many",
    "gsmat_result_rows_many", "gsmat_server_new", "gsmat_server_submit", "gsmat_server_step",
    "gsmat_server_poll", "gsmat_server_free", "gsmat_dict_new", "gsmat_dict_free",
    "gsmat_dict_load_text", "gsmat_dict_triples", "gsmat_dict_sizes", "gsmat_dict_lookup",
    "gsmat_dict_term", "gsmat_parse_bgp", "gsmat_set_hub_options", "gsmat_set_sparse_expand",
    "gsmat_autotune_batch", "gsmat_expand_strategy", "gsmat_set_batch_engine",
    "gsmat_set_batch_regions", "gsmat_batch_round_stats", "gsmat_join_noalloc",
    "gsmat_set_batch_tuning", "gsmat_get_batch_tuning", "gsmat_join_ext",
    "gsmat_join_batch_bgp",
]


class GsmatError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Pattern(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32), ("p", ctypes.c_int32), ("o", ctypes.c_int32)]


class _StepInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tp", ctypes.c_int32), ("orient", ctypes.c_int32),
                ("var", ctypes.c_int32), ("members", ctypes.c_uint32), ("pad", ctypes.c_int32),
                ("est_rows", ctypes.c_int64)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


def _load():
    if not os.path.exists(_SO):
        raise ImportError(
            f"{_SO} is missing: build the HIP library first (python __graft_entry__.py build)")
    L = ctypes.CDLL(_SO)
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.gsmat_load_triples.restype = i32
    L.gsmat_load_triples.argtypes = [vp, vp, vp, i64, i32, i32, vp, vp, pp]
    L.gsmat_set_sparse_expand.restype = i32
    L.gsmat_set_sparse_expand.argtypes = [vp, ctypes.c_double, i64]
    L.gsmat_set_batch_engine.restype = i32
    L.gsmat_set_batch_engine.argtypes = [vp, i32]
    L.gsmat_set_batch_regions.restype = i32
    L.gsmat_set_batch_regions.argtypes = [vp, i64, i64]
    L.gsmat_batch_round_stats.restype = i32
    L.gsmat_join_noalloc.restype = i32
    L.gsmat_join_noalloc.argtypes = [vp, vp, vp, i64, i64, vp, vp]
    L.gsmat_batch_round_stats.argtypes = [vp, vp, i32, vp]
    L.gsmat_autotune_batch.restype = i32
    L.gsmat_autotune_batch.argtypes = [vp, vp, i32, i64, vp, vp]
    L.gsmat_set_batch_tuning.restype = i32
    L.gsmat_set_batch_tuning.argtypes = [vp, i32, i32]
    L.gsmat_get_batch_tuning.restype = i32
    L.gsmat_get_batch_tuning.argtypes = [vp, vp, vp, vp, vp]
    L.gsmat_expand_strategy.restype = i32
    L.gsmat_expand_strategy.argtypes = [ctypes.c_double, i64, i64, i64]
    L.gsmat_set_hub_options.restype = i32
    L.gsmat_set_hub_options.argtypes = [vp, i64, i64]
    L.gsmat_build_index.restype = i32
    L.gsmat_build_index.argtypes = [vp, i32, vp]
    L.gsmat_store_stats.restype = i32
    L.gsmat_store_stats.argtypes = [vp, vp, vp, vp]
    L.gsmat_pred_stats.restype = i32
    L.gsmat_pred_stats.argtypes = [vp, i32, vp, vp, vp]
    L.gsmat_export_matrix.restype = i32
    L.gsmat_export_matrix.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.gsmat_store_free.restype = None
    L.gsmat_store_free.argtypes = [vp]
    L.gsmat_plan.restype = i32
    L.gsmat_plan.argtypes = [vp, vp, i32, i32, vp, pp]
    L.gsmat_plan_from_stats.restype = i32
    L.gsmat_plan_from_stats.argtypes = [vp, i32, i32, vp, pp]
    L.gsmat_plan_info.restype = i32
    L.gsmat_plan_info.argtypes = [vp, vp, vp, vp, i32]
    L.gsmat_plan_free.restype = None
    L.gsmat_plan_free.argtypes = [vp]
    L.gsmat_join.restype = i32
    L.gsmat_join.argtypes = [vp, vp, i64, i64, vp, pp]
    L.gsmat_join_batch_bgp.restype = i32
    L.gsmat_join_batch_bgp.argtypes = [vp, vp, vp, i32, i32, i64, i64, vp, vp, vp]
    L.gsmat_join_ext.restype = i32
    L.gsmat_join_ext.argtypes = [vp, vp, i32, vp, i32, i32, i64, i64, vp, pp]
    L.gsmat_result_info.restype = i32
    L.gsmat_result_info.argtypes = [vp, vp, vp, vp, vp, vp]
    L.gsmat_fetch_bindings.restype = i32
    L.gsmat_fetch_bindings.argtypes = [vp, i64, i64, vp, vp, vp]
    L.gsmat_result_free.restype = None
    L.gsmat_result_free.argtypes = [vp]
    L.gsmat_last_error.restype = ctypes.c_char_p
    L.gsmat_last_error.argtypes = []
    L.gsmat_prof_enable.restype = None
    L.gsmat_prof_enable.argtypes = [i32]
    L.gsmat_prof_read.restype = i32
    L.gsmat_prof_read.argtypes = [vp, vp, vp]
    L.gsmat_prof_host.restype = i32
    L.gsmat_prof_host.argtypes = [vp]
    L.gsmat_release_pools.restype = i32
    L.gsmat_release_pools.argtypes = []
    L.gsmat_plan_batch.restype = i32
    L.gsmat_plan_batch.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
    L.gsmat_join_batch.restype = i32
    L.gsmat_join_batch.argtypes = [vp, vp, i32, i64, i64, vp, vp, vp]
    L.gsmat_plan_free_many.restype = None
    L.gsmat_plan_free_many.argtypes = [vp, i32]
    L.gsmat_result_free_many.restype = None
    L.gsmat_result_free_many.argtypes = [vp, i32]
    L.gsmat_result_rows_many.restype = i32
    L.gsmat_result_rows_many.argtypes = [vp, i32, vp]
    L.gsmat_server_new.restype = i32
    L.gsmat_server_new.argtypes = [vp, i64, i64, i64, i32, vp, pp]
    L.gsmat_server_submit.restype = i32
    L.gsmat_server_submit.argtypes = [vp, vp, i64]
    L.gsmat_server_step.restype = i32
    L.gsmat_server_step.argtypes = [vp, vp, vp, vp]
    L.gsmat_server_poll.restype = i32
    L.gsmat_server_poll.argtypes = [vp, i32, vp, vp, vp, vp]
    L.gsmat_server_free.restype = None
    L.gsmat_server_free.argtypes = [vp]
    sz = ctypes.c_size_t
    L.gsmat_dict_new.restype = i32
    L.gsmat_dict_new.argtypes = [pp]
    L.gsmat_dict_free.restype = None
    L.gsmat_dict_free.argtypes = [vp]
    L.gsmat_dict_load_text.restype = i32
    L.gsmat_dict_load_text.argtypes = [vp, ctypes.c_char_p, sz, vp]
    L.gsmat_dict_triples.restype = i32
    L.gsmat_dict_triples.argtypes = [vp, vp, vp, vp]
    L.gsmat_dict_sizes.restype = i32
    L.gsmat_dict_sizes.argtypes = [vp, vp, vp]
    L.gsmat_dict_lookup.restype = i32
    L.gsmat_dict_lookup.argtypes = [vp, ctypes.c_char_p, sz, i32, vp]
    L.gsmat_dict_term.restype = i32
    L.gsmat_dict_term.argtypes = [vp, i32, i32, vp, sz, vp]
    L.gsmat_parse_bgp.restype = i32
    L.gsmat_parse_bgp.argtypes = [vp, ctypes.c_char_p, sz, vp, i32, vp, vp, vp, sz]
    return L


_lib = _load()


def lib():
    return _lib


def library_path() -> str:
    return _SO


def _check(st):
    if st != GSMAT_OK:
        raise GsmatError(st, _lib.gsmat_last_error().decode(errors="replace"))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:  # torch absent or without a GPU: the null stream
        pass
    return 0


def _stream(s):
    return ctypes.c_void_p(default_stream() if s is None else int(s))


# Live handles, closed in dependency order at interpreter exit (results and
# plans before their stores) while the HIP runtime and torch are still up.
_live_results = weakref.WeakSet()
_live_plans = weakref.WeakSet()
_live_stores = weakref.WeakSet()
_used_device = [False]


@atexit.register
def _shutdown():
    for group in (_live_results, _live_plans, _live_stores):
        for obj in list(group):
            try:
                obj.close()
            except Exception:
                pass
    if _used_device[0]:
        _lib.gsmat_release_pools()


class Store:
    def __init__(self, handle, n_vertices, n_predicates):
        self.h = handle
        self.n_vertices = n_vertices
        self.n_predicates = n_predicates
        self._alloc_keep = None
        _live_stores.add(self)
        _used_device[0] = True

    def close(self):
        if self.h:
            _lib.gsmat_store_free(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Plan:
    def __init__(self, handle):
        self.h = handle
        _live_plans.add(self)

    def close(self):
        if self.h:
            _lib.gsmat_plan_free(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Result:
    def __init__(self, handle, store):
        self.h = handle
        self.store = store  # keeps the store alive while the result lives
        _live_results.add(self)

    def close(self):
        if self.h:
            _lib.gsmat_result_free(self.h)
            self.h = None

    def __del__(self):
        self.close()


def _patterns(tps):
    t = np.ascontiguousarray(np.asarray(tps, dtype=np.int32).reshape(-1, 3))
    arr = (_Pattern * len(t))()
    for i, (s, p, o) in enumerate(t.tolist()):
        arr[i] = _Pattern(s, p, o)
    return arr, len(t)


def make_allocator(alloc_fn, free_fn):
    """Wraps Python callables alloc(bytes, stream)->int and free(ptr, bytes, stream)
    into a gsmat_allocator (kept alive by the returned object)."""
    a = ALLOC_FN(lambda b, s, c: alloc_fn(b, s) or None)
    f = FREE_FN(lambda ptr, b, s, c: free_fn(ptr, b, s))
    return _Allocator(a, f, None), (a, f)


def gsmat_load_triples(s, p, o, n_vertices, n_predicates, stream=None, allocator=None):
    s = np.ascontiguousarray(s, np.int32)
    p = np.ascontiguousarray(p, np.int32)
    o = np.ascontiguousarray(o, np.int32)
    if not (len(s) == len(p) == len(o)):
        raise ValueError("s, p, o must have the same length")
    h = ctypes.c_void_p()
    aptr = None
    keep = None
    if allocator is not None:
        struct, keep = allocator
        aptr = ctypes.cast(ctypes.pointer(struct), ctypes.c_void_p)
        keep = (keep, struct)
    _check(_lib.gsmat_load_triples(_p(s), _p(p), _p(o), len(s), n_vertices, n_predicates, aptr,
                                   _stream(stream), ctypes.byref(h)))
    st = Store(h, n_vertices, n_predicates)
    st._alloc_keep = keep
    return st


def gsmat_set_hub_options(store, min_len, max_bytes):
    _check(_lib.gsmat_set_hub_options(store.h, min_len, max_bytes))


def gsmat_build_index(store, dense_div=0, stream=None):
    _check(_lib.gsmat_build_index(store.h, dense_div, _stream(stream)))


def gsmat_store_stats(store):
    t, pr, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(_lib.gsmat_store_stats(store.h, ctypes.byref(t), ctypes.byref(pr), ctypes.byref(b)))
    return {"n_triples": t.value, "n_predicates": pr.value, "device_bytes": b.value}


def gsmat_pred_stats(store, pred):
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.gsmat_pred_stats(store.h, pred, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def gsmat_export_matrix(store, pred, orient, stream=None):
    nnz, nr, nc = gsmat_pred_stats(store, pred)
    rows = nr if orient == 0 else nc
    keys = np.empty(rows, np.int32)
    ptr = np.empty(rows + 1, np.int32)
    nbr = np.empty(nnz, np.int32)
    _check(_lib.gsmat_export_matrix(store.h, pred, orient, _p(keys), _p(ptr), _p(nbr),
                                    _stream(stream)))
    return keys, ptr, nbr


def gsmat_plan(store, tps, mode=PLAN_DEFAULT, stream=None):
    arr, n = _patterns(tps)
    h = ctypes.c_void_p()
    _check(_lib.gsmat_plan(store.h, arr, n, mode, _stream(stream), ctypes.byref(h)))
    return Plan(h)


def gsmat_plan_from_stats(tps, mode, stats):
    arr, n = _patterns(tps)
    st = np.ascontiguousarray(stats, np.int64)
    h = ctypes.c_void_p()
    _check(_lib.gsmat_plan_from_stats(arr, n, mode, _p(st), ctypes.byref(h)))
    return Plan(h)


def gsmat_plan_info(plan):
    ns, nv = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.gsmat_plan_info(plan.h, ctypes.byref(ns), ctypes.byref(nv), None, 0))
    steps = (_StepInfo * max(ns.value, 1))()
    _check(_lib.gsmat_plan_info(plan.h, ctypes.byref(ns), ctypes.byref(nv), steps, ns.value))
    out = []
    for i in range(ns.value):
        s = steps[i]
        out.append({"kind": STEP_NAMES[s.kind], "tp": s.tp, "orient": s.orient, "var": s.var,
                    "members": [b for b in range(32) if s.members >> b & 1],
                    "est_rows": s.est_rows})
    return nv.value, out


def gsmat_join(store, plan, budget_bytes=0, max_rows=-1, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.gsmat_join(store.h, plan.h, budget_bytes, max_rows, _stream(stream),
                           ctypes.byref(h)))
    return Result(h, store)


F_EQ, F_NE, F_LT, F_LE, F_GT, F_GE, F_BOUND, F_NOT_BOUND = range(8)


def gsmat_join_ext(store, pats, filters=(), n_vars=None, budget_bytes=0, max_rows=-1,
                   stream=None):
    """OPTIONAL / UNION / FILTER query: pats (n, 5) int32 rows (s, p, o, branch,
    group), filters (m, 4) int32 rows (op, a, b, branch); n_vars defaults to
    one past the largest variable named.  Returns a Result (unbound = -1)."""
    pa = np.ascontiguousarray(np.asarray(pats, dtype=np.int32).reshape(-1, 5))
    fa = np.ascontiguousarray(np.asarray(filters, dtype=np.int32).reshape(-1, 4))
    if n_vars is None:
        terms = np.concatenate([pa[:, [0, 2]].ravel(), fa[:, [1, 2]].ravel()])
        n_vars = int(-terms.min()) if len(terms) and terms.min() < 0 else 0
    h = ctypes.c_void_p()
    _check(_lib.gsmat_join_ext(store.h, _p(pa) if pa.size else None, len(pa),
                               _p(fa) if fa.size else None, len(fa), int(n_vars), budget_bytes,
                               max_rows, _stream(stream), ctypes.byref(h)))
    return Result(h, store)


def gsmat_join_noalloc(store, plan, out_ptr, out_stride, out_cap, stream=None):
    """gsmat_join into the caller's device buffer (variable v's column at
    out_ptr + 4 * v * out_stride bytes) with no device allocation; returns the
    row count.  Raises GsmatError (its `n_rows` attribute holds the row count
    when it is known)."""
    n = ctypes.c_int64(0)
    rc = _lib.gsmat_join_noalloc(store.h, plan.h, ctypes.c_void_p(int(out_ptr)), int(out_stride),
                                 int(out_cap), ctypes.byref(n), _stream(stream))
    if rc != GSMAT_OK:
        e = GsmatError(rc, _lib.gsmat_last_error().decode(errors="replace"))
        e.n_rows = int(n.value)
        raise e
    return int(n.value)


class _Handle:
    """A borrowed handle (owned by a PlanSet or ResultSet)."""

    def __init__(self, h, owner):
        self.h = h
        self.owner = owner


class PlanSet:
    """n plans held in one handle array (one call frees them all)."""

    def __init__(self, arr, n):
        self.arr = arr
        self.n = n
        _live_plans.add(self)

    def __len__(self):
        return self.n

    def __getitem__(self, i):
        h = self.arr[i]
        return _Handle(ctypes.c_void_p(h), self) if h else None

    def close(self):
        if self.arr is not None:
            _lib.gsmat_plan_free_many(self.arr, self.n)
            self.arr = None

    def __del__(self):
        self.close()


class ResultSet:
    """n results held in one handle array (one call frees them all)."""

    def __init__(self, arr, n, store):
        self.arr = arr
        self.n = n
        self.store = store
        _live_results.add(self)

    def __len__(self):
        return self.n

    def __getitem__(self, i):
        h = self.arr[i]
        return _Handle(ctypes.c_void_p(h), self) if h else None

    def rows(self):
        out = np.zeros(max(self.n, 1), np.int64)
        _check(_lib.gsmat_result_rows_many(self.arr, self.n, _p(out)))
        return out[: self.n]

    def close(self):
        if self.arr is not None:
            _lib.gsmat_result_free_many(self.arr, self.n)
            self.arr = None

    def __del__(self):
        self.close()


def pack_queries(queries):
    """(flat (N, 3) int32 patterns, per-query pattern counts) for gsmat_plan_batch."""
    ts = [np.asarray(t, dtype=np.int32).reshape(-1, 3) for t in queries]
    n_pats = np.array([len(t) for t in ts], np.int32)
    flat = np.ascontiguousarray(np.concatenate(ts) if ts else np.zeros((0, 3), np.int32))
    return flat, n_pats


def gsmat_plan_batch(store, queries, mode=PLAN_DEFAULT, stream=None, raise_on_error=True,
                     as_set=False):
    """Plans of several BGPs with one device round trip.  queries: a list of
    (n, 3) pattern arrays, or the (flat, n_pats) pair of pack_queries.
    Returns (plans, statuses): a list of Plan (None where a query was
    rejected), or with as_set one PlanSet.  With raise_on_error, the first
    failure raises after freeing the rest."""
    flat, n_pats = queries if isinstance(queries, tuple) else pack_queries(queries)
    nq = len(n_pats)
    hs = (ctypes.c_void_p * max(nq, 1))()
    st = np.zeros(max(nq, 1), np.int32)
    rc = _lib.gsmat_plan_batch(store.h, _p(flat), _p(n_pats), nq, mode, _stream(stream), hs,
                               _p(st))
    msg = _lib.gsmat_last_error().decode(errors="replace") if rc != GSMAT_OK else ""
    if rc != GSMAT_OK and raise_on_error:
        _lib.gsmat_plan_free_many(hs, nq)
        raise GsmatError(rc, msg)
    statuses = st[:nq].tolist()
    if as_set:
        return PlanSet(hs, nq), statuses
    return [Plan(ctypes.c_void_p(hs[i])) if hs[i] else None for i in range(nq)], statuses


def gsmat_join_batch(store, plans, budget_bytes=0, max_rows=-1, stream=None,
                     raise_on_error=True, as_set=False):
    """Evaluates several plans (a list of Plan, or a PlanSet) together.  Returns
    (results, statuses): a list of Result (None where a query failed), or with
    as_set one ResultSet.  With raise_on_error, the first failure raises after
    freeing the rest."""
    if isinstance(plans, PlanSet):
        nq = plans.n
        ph = plans.arr
    else:
        nq = len(plans)
        ph = (ctypes.c_void_p * max(nq, 1))(*[pl.h for pl in plans])
    hs = (ctypes.c_void_p * max(nq, 1))()
    st = np.zeros(max(nq, 1), np.int32)
    rc = _lib.gsmat_join_batch(store.h, ph, nq, budget_bytes, max_rows, _stream(stream), hs,
                               _p(st))
    msg = _lib.gsmat_last_error().decode(errors="replace") if rc != GSMAT_OK else ""
    if rc != GSMAT_OK and raise_on_error:
        _lib.gsmat_result_free_many(hs, nq)
        raise GsmatError(rc, msg)
    statuses = st[:nq].tolist()
    if as_set:
        return ResultSet(hs, nq, store), statuses
    return [Result(ctypes.c_void_p(hs[i]), store) if hs[i] else None for i in range(nq)], statuses


def gsmat_join_batch_bgp(store, queries, mode=PLAN_ADAPTIVE, budget_bytes=0, max_rows=-1,
                         stream=None, raise_on_error=True, as_set=False):
    """Plans and joins several BGPs in one call (no plan objects): queries is a
    list of (n, 3) pattern arrays or the (flat, n_pats) pair of pack_queries.
    Returns (results, statuses) as gsmat_join_batch does."""
    flat, n_pats = queries if isinstance(queries, tuple) else pack_queries(queries)
    nq = len(n_pats)
    hs = (ctypes.c_void_p * max(nq, 1))()
    st = np.zeros(max(nq, 1), np.int32)
    rc = _lib.gsmat_join_batch_bgp(store.h, _p(flat), _p(n_pats), nq, mode, budget_bytes,
                                   max_rows, _stream(stream), hs, _p(st))
    msg = _lib.gsmat_last_error().decode(errors="replace") if rc != GSMAT_OK else ""
    if rc != GSMAT_OK and raise_on_error:
        _lib.gsmat_result_free_many(hs, nq)
        raise GsmatError(rc, msg)
    statuses = st[:nq].tolist()
    if as_set:
        return ResultSet(hs, nq, store), statuses
    return [Result(ctypes.c_void_p(hs[i]), store) if hs[i] else None for i in range(nq)], statuses


class Server:
    """Continuous-batching request loop over one store (gsmat_server_*)."""

    def __init__(self, handle, store):
        self.h = handle
        self.store = store
        self.plans = {}  # tag -> plan, kept alive until its result is polled
        _live_results.add(self)

    def close(self):
        if self.h:
            _lib.gsmat_server_free(self.h)
            self.h = None
        self.plans = {}

    def __del__(self):
        self.close()


def gsmat_server_new(store, mem_budget_bytes=0, step_budget_bytes=0, max_rows=-1,
                     max_active=4096, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.gsmat_server_new(store.h, mem_budget_bytes, step_budget_bytes, max_rows,
                                 max_active, _stream(stream), ctypes.byref(h)))
    return Server(h, store)


def gsmat_server_submit(server, plan, tag):
    """plan: a Plan or a borrowed handle; it is kept alive until polled."""
    _check(_lib.gsmat_server_submit(server.h, plan.h, tag))
    server.plans[tag] = plan


def gsmat_server_step(server):
    """One admission + batched round: (active, waiting, done)."""
    a, w, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.gsmat_server_step(server.h, ctypes.byref(a), ctypes.byref(w), ctypes.byref(d)))
    return a.value, w.value, d.value


def gsmat_server_poll(server, cap=4096):
    """Finished queries: a list of (tag, Result or None, status)."""
    tags = np.zeros(max(cap, 1), np.int64)
    st = np.zeros(max(cap, 1), np.int32)
    hs = (ctypes.c_void_p * max(cap, 1))()
    n = ctypes.c_int32()
    _check(_lib.gsmat_server_poll(server.h, cap, _p(tags), hs, _p(st), ctypes.byref(n)))
    out = []
    for i in range(n.value):
        tag = int(tags[i])
        server.plans.pop(tag, None)
        out.append((tag, Result(ctypes.c_void_p(hs[i]), server.store) if hs[i] else None,
                    int(st[i])))
    return out


class Dict:
    """Host dictionary of terms (gsmat_dict_*)."""

    def __init__(self, handle):
        self.h = handle
        _live_plans.add(self)

    def close(self):
        if self.h:
            _lib.gsmat_dict_free(self.h)
            self.h = None

    def __del__(self):
        self.close()


def gsmat_dict_new():
    h = ctypes.c_void_p()
    _check(_lib.gsmat_dict_new(ctypes.byref(h)))
    return Dict(h)


def gsmat_dict_load_text(d, text):
    """Codes the text's triples; returns (s, p, o) int32 arrays."""
    b = text.encode() if isinstance(text, str) else bytes(text)
    n = ctypes.c_int64()
    _check(_lib.gsmat_dict_load_text(d.h, b, len(b), ctypes.byref(n)))
    s, p, o = (np.empty(n.value, np.int32) for _ in range(3))
    _check(_lib.gsmat_dict_triples(d.h, _p(s), _p(p), _p(o)))
    return s, p, o


def gsmat_dict_sizes(d):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.gsmat_dict_sizes(d.h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def gsmat_dict_lookup(d, term, is_predicate=False):
    b = term.encode()
    c = ctypes.c_int32()
    _check(_lib.gsmat_dict_lookup(d.h, b, len(b), int(is_predicate), ctypes.byref(c)))
    return c.value


def gsmat_dict_term(d, code, is_predicate=False):
    n = ctypes.c_size_t()
    _check(_lib.gsmat_dict_term(d.h, int(code), int(is_predicate), None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(_lib.gsmat_dict_term(d.h, int(code), int(is_predicate), buf, n.value + 1,
                                ctypes.byref(n)))
    return buf.value.decode()


def gsmat_parse_bgp(d, text):
    """(patterns (n, 3) int32, variable names)."""
    b = text.encode()
    n, nv = ctypes.c_int32(), ctypes.c_int32()
    rc = _lib.gsmat_parse_bgp(d.h, b, len(b), None, 0, ctypes.byref(n), ctypes.byref(nv), None, 0)
    if rc not in (GSMAT_OK, GSMAT_ETOOBIG):
        _check(rc)
    arr = (_Pattern * max(n.value, 1))()
    names = ctypes.create_string_buffer(len(b) + 1)
    _check(_lib.gsmat_parse_bgp(d.h, b, len(b), arr, n.value, ctypes.byref(n), ctypes.byref(nv),
                                names, len(b) + 1))
    tps = np.array([[arr[i].s, arr[i].p, arr[i].o] for i in range(n.value)], np.int32).reshape(-1, 3)
    raw = names.raw
    out, at = [], 0
    for _ in range(nv.value):
        end = raw.index(b"\0", at)
        out.append(raw[at:end].decode())
        at = end + 1
    return tps, out


def gsmat_set_sparse_expand(store, theta, min_rows=4096):
    _check(_lib.gsmat_set_sparse_expand(store.h, float(theta), int(min_rows)))


ENGINE_HOST, ENGINE_DEVICE = 0, 1


def gsmat_set_batch_engine(store, engine):
    """gsmat_join_batch's rounds: ENGINE_DEVICE (default, device-driven) or
    ENGINE_HOST (host-driven)."""
    _check(_lib.gsmat_set_batch_engine(store.h, int(engine)))


def gsmat_set_batch_regions(store, out_bytes=0, scratch_bytes=0):
    """Starting sizes of the device-driven batch's output slab and scratch
    region (0: the defaults); the store then keeps each batch's own sizes."""
    _check(_lib.gsmat_set_batch_regions(store.h, int(out_bytes), int(scratch_bytes)))


ROUND_STAT_FIELDS = ("tasks", "count_tiles", "post_tiles", "write_tiles", "split_entries",
                     "out_bytes", "candidates", "deferred")


def gsmat_batch_round_stats(store):
    """Per round of the store's last device-driven batch: a dict of the
    ROUND_STAT_FIELDS figures."""
    out = np.zeros((64, len(ROUND_STAT_FIELDS)), np.int64)
    n = ctypes.c_int32(0)
    _check(_lib.gsmat_batch_round_stats(store.h, _p(out), 64, ctypes.byref(n)))
    return [dict(zip(ROUND_STAT_FIELDS, map(int, row))) for row in out[: min(n.value, 64)]]


def gsmat_expand_strategy(theta, min_rows, n_in, n_nonempty):
    """1 when the batched join writes such an expansion over its compacted
    rows with output, 0 when it walks every input row."""
    return int(_lib.gsmat_expand_strategy(float(theta), int(min_rows), int(n_in),
                                          int(n_nonempty)))


SPARSE_CANDIDATES = (0.0, 0.25, 0.5, 0.75, 1.0)
ITEMS_CANDIDATES = (4, 8, 16)
ISECT_SEARCH, ISECT_WINDOW, ISECT_MERGE = 0, 1, 2
ISECT_NAMES = ("search", "window", "merge")


class TuneReport(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("count_items", ctypes.c_int32),
                ("intersect", ctypes.c_int32), ("theta_ms", ctypes.c_double * 5),
                ("items_ms", ctypes.c_double * 3), ("intersect_ms", ctypes.c_double * 3)]


def gsmat_set_batch_tuning(store, count_items=8, intersect=ISECT_SEARCH):
    """Count rows per thread (4, 8, 16) and sorted-list intersection strategy
    (ISECT_*) of the device-driven batched join."""
    _check(_lib.gsmat_set_batch_tuning(store.h, int(count_items), int(intersect)))


def gsmat_get_batch_tuning(store):
    theta, min_rows = ctypes.c_double(), ctypes.c_int64()
    items, isect = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.gsmat_get_batch_tuning(store.h, ctypes.byref(theta), ctypes.byref(min_rows),
                                       ctypes.byref(items), ctypes.byref(isect)))
    return {"sparse_theta": theta.value, "sparse_min_rows": min_rows.value,
            "count_items": items.value, "intersect": ISECT_NAMES[isect.value]}


def gsmat_autotune_batch(store, plans, budget_bytes=0, stream=None):
    """Tunes the batch's sparse-expansion threshold, count rows per thread and
    intersection strategy in turn, keeping the fastest of each for the store:
    a dict of the choices and each candidate's time in ms (-1: not tuned)."""
    if isinstance(plans, PlanSet):
        nq, ph = plans.n, plans.arr
    else:
        nq = len(plans)
        ph = (ctypes.c_void_p * max(nq, 1))(*[pl.h for pl in plans])
    r = TuneReport()
    _check(_lib.gsmat_autotune_batch(store.h, ph, nq, budget_bytes, _stream(stream),
                                     ctypes.byref(r)))
    return {"sparse_theta": r.theta, "count_items": r.count_items,
            "intersect": ISECT_NAMES[r.intersect],
            "candidate_ms": {
                "sparse_theta": {str(c): round(r.theta_ms[i], 3)
                                 for i, c in enumerate(SPARSE_CANDIDATES)},
                "count_items": {str(c): round(r.items_ms[i], 3)
                                for i, c in enumerate(ITEMS_CANDIDATES)},
                "intersect": {n: round(r.intersect_ms[i], 3) for i, n in enumerate(ISECT_NAMES)}}}


def gsmat_result_info(result):
    rows, nv, ns = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.gsmat_result_info(result.h, ctypes.byref(rows), ctypes.byref(nv),
                                  ctypes.byref(ns), None, None))
    si = np.zeros(max(ns.value, 1), np.int64)
    so = np.zeros(max(ns.value, 1), np.int64)
    _check(_lib.gsmat_result_info(result.h, None, None, None, _p(si), _p(so)))
    return {"rows": rows.value, "n_vars": nv.value, "step_rows_in": si[:ns.value].tolist(),
            "step_rows_out": so[:ns.value].tolist()}


def gsmat_fetch_bindings(result, row_offset=0, max_rows=None, stream=None):
    info = gsmat_result_info(result)
    rows, nv = info["rows"], info["n_vars"]
    if max_rows is None:
        max_rows = rows
    n = max(0, min(rows - min(row_offset, rows), max_rows))
    out = np.empty((n, nv), np.int32)
    written = ctypes.c_int64()
    _check(_lib.gsmat_fetch_bindings(result.h, row_offset, max_rows,
                                     _p(out) if out.size else None, ctypes.byref(written),
                                     _stream(stream)))
    return out[:written.value]


def gsmat_release_pools():
    _check(_lib.gsmat_release_pools())


def gsmat_prof_enable(class_mask=0x1F):
    """class_mask: bit K_* set to time that kernel class (0 stops)."""
    _lib.gsmat_prof_enable(int(class_mask))


def gsmat_prof_read():
    la = np.zeros(5, np.int64)
    ms = np.zeros(5, np.float64)
    by = np.zeros(5, np.float64)
    _check(_lib.gsmat_prof_read(_p(la), _p(ms), _p(by)))
    return {K_NAMES[i]: {"launches": int(la[i]), "ms": float(ms[i]), "bytes": float(by[i])}
            for i in range(5)}


def gsmat_prof_host():
    out = np.zeros(5, np.float64)
    _check(_lib.gsmat_prof_host(_p(out)))
    return {"alloc_ms": float(out[0]), "allocs": int(out[1]), "free_ms": float(out[2]),
            "sync_ms": float(out[3]), "syncs": int(out[4])}


def evaluate_batch(store, queries, mode=PLAN_ADAPTIVE, budget_bytes=0, max_rows=-1,
                   stream=None):
    """Batched plan + join + fetch: one (rows, n_vars) int32 array per BGP."""
    plans, _ = gsmat_plan_batch(store, queries, mode, stream)
    try:
        results, _ = gsmat_join_batch(store, plans, budget_bytes, max_rows, stream)
        try:
            return [gsmat_fetch_bindings(r, stream=stream) for r in results]
        finally:
            for r in results:
                r.close()
    finally:
        for pl in plans:
            pl.close()


def evaluate(store, tps, mode=PLAN_ADAPTIVE, budget_bytes=0, max_rows=-1, stream=None):
    """Plan + join + fetch: all rows of the BGP as an (rows, n_vars) int32 array."""
    pl = gsmat_plan(store, tps, mode, stream)
    try:
        r = gsmat_join(store, pl, budget_bytes, max_rows, stream)
        try:
            return gsmat_fetch_bindings(r, stream=stream)
        finally:
            r.close()
    finally:
        pl.close()
