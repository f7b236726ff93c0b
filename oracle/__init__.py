"""Oracle: plain CPU evaluation of BGPs over a triple set, for testing only.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  The product path (the
GPU library and its Python binding) never does, and shares no code with it.

Contents:
  * ``liboracle.so`` (built from ``oracle.cpp`` with g++): set semantics,
    per-pattern relations, hash/Cartesian joins, sorted output, fingerprint,
    and the per-predicate compressed matrices of the storage scheme.
  * ``brute_force``: enumeration of every assignment of the variables (tiny
    inputs only), the definition of BGP matching written out.
  * ``plan_order``: the planner's ordering rule, "connected minimal upper
    bound" (paper Sec. 6.2.1 and its Algorithm "Query Plan Generated"), read as
    its prose states it (see the reading notes in ``plan_order``).
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC,
                               "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        L.oracle_dedupe.restype = i64
        L.oracle_dedupe.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.oracle_csr.restype = i64
        L.oracle_csr.argtypes = [vp, vp, vp, i64, i32, i32, vp, vp, vp, vp]
        L.oracle_join.restype = vp
        L.oracle_join.argtypes = [vp, vp, vp, i64, vp, i32, i32, i64]
        L.oracle_result_rows.restype = i64
        L.oracle_result_rows.argtypes = [vp]
        L.oracle_result_nvars.restype = i32
        L.oracle_result_nvars.argtypes = [vp]
        L.oracle_result_copy.argtypes = [vp, vp]
        L.oracle_result_fingerprint.argtypes = [vp, vp]
        L.oracle_fingerprint_rows.argtypes = [vp, i64, i32, vp]
        L.oracle_mix64.restype = ctypes.c_uint64
        L.oracle_mix64.argtypes = [ctypes.c_uint64]
        L.oracle_result_partition.restype = i64
        L.oracle_result_partition.argtypes = [vp, i32, i32, vp]
        L.oracle_result_free.argtypes = [vp]
        L.oracle_dataset_new.restype = vp
        L.oracle_dataset_new.argtypes = [vp, vp, vp, i64]
        L.oracle_dataset_free.argtypes = [vp]
        L.oracle_join_dataset.restype = vp
        L.oracle_join_dataset.argtypes = [vp, vp, i32, i32, i64]
        L.oracle_join_dataset_omp.restype = vp
        L.oracle_join_dataset_omp.argtypes = [vp, vp, i32, i32, i64, i32]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def dedupe(s, p, o):
    """Sorted distinct (s, p, o) triples (the dataset as a set, Sec. 3.1)."""
    s, p, o = _i32(s), _i32(p), _i32(o)
    n = len(s)
    so, po, oo = (np.empty(n, np.int32) for _ in range(3))
    m = lib().oracle_dedupe(_p(s), _p(p), _p(o), n, _p(so), _p(po), _p(oo))
    return so[:m], po[:m], oo[:m]


def csr(s, p, o, pred, orient):
    """(keys, ptr, nbr) of predicate `pred`: orient 0 by subject, 1 by object."""
    s, p, o = _i32(s), _i32(p), _i32(o)
    nr = ctypes.c_int64(0)
    nnz = lib().oracle_csr(_p(s), _p(p), _p(o), len(s), pred, orient, ctypes.byref(nr),
                           None, None, None)
    keys = np.empty(nr.value, np.int32)
    ptr = np.empty(nr.value + 1, np.int32)
    nbr = np.empty(nnz, np.int32)
    lib().oracle_csr(_p(s), _p(p), _p(o), len(s), pred, orient, ctypes.byref(nr), _p(keys),
                     _p(ptr), _p(nbr))
    return keys, ptr, nbr


class Dataset:
    """The deduplicated triple set, built once for repeated oracle joins."""

    def __init__(self, s, p, o):
        s, p, o = _i32(s), _i32(p), _i32(o)
        self.h = lib().oracle_dataset_new(_p(s), _p(p), _p(o), len(s))

    def close(self):
        if self.h:
            lib().oracle_dataset_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def join(self, tps, n_vars, cap_rows=-1, fingerprint=False, partition=None):
        t = _i32(np.asarray(tps).reshape(-1, 3))
        h = lib().oracle_join_dataset(self.h, _p(t), len(t), n_vars, cap_rows)
        return _collect(h, n_vars, fingerprint, partition)

    def join_omp(self, tps, n_vars, threads, cap_rows=-1, fingerprint=False):
        """The same answer evaluated on `threads` host threads (the CPU
        baseline's multi-core form)."""
        t = _i32(np.asarray(tps).reshape(-1, 3))
        h = lib().oracle_join_dataset_omp(self.h, _p(t), len(t), n_vars, cap_rows, int(threads))
        return _collect(h, n_vars, fingerprint)


def _collect(h, n_vars, fingerprint, partition=None):
    if not h:
        raise ValueError("oracle_join rejected the input (invalid BGP or row cap exceeded)")
    try:
        if partition is not None:
            # (fingerprint, sorted rows of the hash partition h1 mod m == r)
            mod, res = partition
            fp = np.zeros(3, np.uint64)
            lib().oracle_result_fingerprint(h, _p(fp))
            k = lib().oracle_result_partition(h, mod, res, None)
            part = np.empty((k, n_vars), np.int32)
            if k and n_vars:
                lib().oracle_result_partition(h, mod, res, _p(part))
            return tuple(int(x) for x in fp), part
        if fingerprint:
            out = np.zeros(3, np.uint64)
            lib().oracle_result_fingerprint(h, _p(out))
            return tuple(int(x) for x in out)
        rows = lib().oracle_result_rows(h)
        out = np.empty((rows, n_vars), np.int32)
        if rows and n_vars:
            lib().oracle_result_copy(h, _p(out))
        return out
    finally:
        lib().oracle_result_free(h)


def join(s, p, o, tps, n_vars, cap_rows=-1, fingerprint=False, partition=None):
    """Sorted result rows (rows x n_vars int32) of the BGP `tps` ((n,3) int32).

    With fingerprint=True returns (rows, h1 sum, h2 sum) instead; with
    partition=(m, r) returns (that fingerprint, the sorted rows whose h1 is r
    modulo m).
    """
    s, p, o = _i32(s), _i32(p), _i32(o)
    t = _i32(np.asarray(tps).reshape(-1, 3))
    h = lib().oracle_join(_p(s), _p(p), _p(o), len(s), _p(t), len(t), n_vars, cap_rows)
    return _collect(h, n_vars, fingerprint, partition)


def fingerprint_rows_c(rows):
    """The C oracle's fingerprint of arbitrary rows (row-major int32)."""
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    n = rows.shape[0]
    nv = rows.shape[1] if rows.ndim == 2 else 0
    out = np.zeros(3, np.uint64)
    lib().oracle_fingerprint_rows(_p(rows) if rows.size else None, n, nv, _p(out))
    return tuple(int(x) for x in out)


def mix64(z):
    """The SplitMix64 finaliser of the C oracle."""
    return int(lib().oracle_mix64(int(z) & 0xFFFFFFFFFFFFFFFF))


def brute_force(s, p, o, tps, n_vars, V):
    """Every assignment mu in [0,V)^n_vars with (mu(s_i), p_i, mu(o_i)) in D for
    all patterns; sorted.  Tiny inputs only (V**n_vars small)."""
    D = set(zip(np.asarray(s).tolist(), np.asarray(p).tolist(), np.asarray(o).tolist()))
    tps = [tuple(int(v) for v in t) for t in np.asarray(tps).reshape(-1, 3)]

    def val(term, mu):
        return term if term >= 0 else mu[-term - 1]

    out = []
    for mu in itertools.product(range(V), repeat=n_vars):
        if all((val(a, mu), b, val(c, mu)) in D for a, b, c in tps):
            out.append(mu)
    return np.array(out, dtype=np.int32).reshape(len(out), n_vars)


def plan_order(tps, stat):
    """Order of the triple patterns under the paper's planner (Sec. 6.2.1).

    Steps as the prose gives them: (1) sort all edges by their statistic;
    (2) take the smallest edge first and put its nodes in N; (3) repeatedly take,
    in sorted order, the first remaining edge with at least one node in N, add
    its nodes to N and remove it; (4) until no edge remains.

    Readings where the text is silent or its listing disagrees with the prose:
      * ties in the sort keep the original pattern order (stable sort);
      * "a node in N" means a shared *variable*: constants do not connect
        patterns (the prose speaks of common join variables);
      * when no remaining edge shares a variable (a disconnected BGP) the first
        remaining edge in sorted order is taken (a Cartesian step).
    """
    tps = [tuple(int(v) for v in t) for t in np.asarray(tps).reshape(-1, 3)]
    n = len(tps)
    L = sorted(range(n), key=lambda i: (stat[i], i))
    order = [L.pop(0)]
    N = {x for x in (tps[order[0]][0], tps[order[0]][2]) if x < 0}
    while L:
        pick = None
        for j, e in enumerate(L):
            if any(x < 0 and x in N for x in (tps[e][0], tps[e][2])):
                pick = j
                break
        if pick is None:
            pick = 0
        e = L.pop(pick)
        order.append(e)
        N |= {x for x in (tps[e][0], tps[e][2]) if x < 0}
    return order


def _h1(rows):
    rows = np.asarray(rows)
    with np.errstate(over="ignore"):
        x = np.full(len(rows), 0x1234567, np.uint64)
        for c in range(rows.shape[1] if rows.ndim == 2 else 0):
            v = rows[:, c].astype(np.int64).astype(np.uint64) & np.uint64(0xFFFFFFFF)
            z = x ^ v
            z = z ^ (z >> np.uint64(30))
            z = z * np.uint64(0xbf58476d1ce4e5b9)
            z = z ^ (z >> np.uint64(27))
            z = z * np.uint64(0x94d049bb133111eb)
            x = z ^ (z >> np.uint64(31))
    return x


def partition_rows(rows, mod=64, residue=0):
    """The rows whose h1 (the fingerprint's first row hash) is `residue`
    modulo `mod`, sorted: the hash partition the oracle returns with
    partition=(mod, residue), for rows fetched from the GPU library."""
    rows = np.asarray(rows)
    if len(rows) == 0:
        return rows.reshape(0, rows.shape[1] if rows.ndim == 2 else 0).astype(np.int32)
    keep = rows[(_h1(rows) % np.uint64(mod)) == np.uint64(residue)]
    if keep.ndim == 2 and keep.shape[1] and len(keep):
        keep = keep[np.lexsort(keep.T[::-1])]
    return keep.astype(np.int32)


def fingerprint_rows(rows: np.ndarray):
    """The same fingerprint as the C oracle's, over rows given as an array.

    Used by the tests to fingerprint rows fetched from the GPU library."""
    rows = np.asarray(rows)
    M = np.uint64(0xFFFFFFFFFFFFFFFF)

    def mix(z):
        z = z ^ (z >> np.uint64(30))
        z = z * np.uint64(0xbf58476d1ce4e5b9)
        z = z ^ (z >> np.uint64(27))
        z = z * np.uint64(0x94d049bb133111eb)
        z = z ^ (z >> np.uint64(31))
        return z

    with np.errstate(over="ignore"):
        x = np.full(len(rows), 0x1234567, np.uint64)
        y = np.full(len(rows), 0x89abcdef, np.uint64)
        for c in range(rows.shape[1] if rows.ndim == 2 else 0):
            v = rows[:, c].astype(np.int64).astype(np.uint64) & np.uint64(0xFFFFFFFF)
            x = mix(x ^ v)
            y = mix(y ^ v)
        a = int(np.sum(x, dtype=np.uint64)) if len(rows) else 0
        b = int(np.sum(y, dtype=np.uint64)) if len(rows) else 0
    del M
    return (len(rows), a, b)
