"""Seeded synthetic RDF workloads: power-law triple sets and random-walk BGPs.

This package only produces inputs.  It holds no part of the join: the CPU
oracle (``oracle/``) and the GPU library both consume the arrays it returns,
and neither side shares any other code through it.

Graph recipe (stand-in for the paper's WatDiv/YAGO/DBpedia data, which are not
available): integer vertex ids in [0, V), predicates in [0, P) drawn from
Zipf(s); out-degrees follow a discrete power law with exponent 2.2 capped per
configuration; objects are drawn in proportion to a power-law in-weight that is
rank-correlated with the out-degree draw, so that hubs exist while the large
majority of vertices keep a small total degree; the triple set is exactly T
distinct triples in pseudo-random order.

Query recipe: each BGP is a random walk (chain, subject star, object star,
snowflake) over the generated graph in which every walk position is a fresh
variable, so the walk itself is a witness and no query is empty.  Optionally
one leaf is replaced by its witness value (a constant).  Queries are accepted
or rejected by their exact result size, computed by a tree counting program
that is independent of the join.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import math
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libworkload.so")
_SRC = os.path.join(_HERE, "gen.c")

# Pattern encoding shared with the ABI: an endpoint >= 0 is a vertex constant,
# an endpoint < 0 is variable number -(x+1).


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        i64, i32, u64, dbl, vp = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.c_double, ctypes.c_void_p)
        L.wl_gen_graph.restype = i64
        L.wl_gen_graph.argtypes = [i64, i32, i64, dbl, dbl, i64, dbl, i64, dbl, u64, vp, vp, vp]
        L.wl_index_new.restype = vp
        L.wl_index_new.argtypes = [vp, vp, vp, i64, i64, i32]
        L.wl_index_free.argtypes = [vp]
        L.wl_count_tree.restype = i64
        L.wl_count_tree.argtypes = [vp, vp, i32, i32]
        L.wl_count_many.restype = None
        L.wl_count_many.argtypes = [vp, vp, vp, vp, vp, i32, vp]
        L.wl_walk_query.restype = i32
        L.wl_walk_query.argtypes = [vp, i32, i32, i32, i32, dbl, u64, u64, vp, vp]
        L.wl_out_degree.restype = i64
        L.wl_out_degree.argtypes = [vp, i32]
        L.wl_in_degree.restype = i64
        L.wl_in_degree.argtypes = [vp, i32]
        L.wl_vertices_with_degree.restype = i64
        L.wl_vertices_with_degree.argtypes = [vp, i64, vp, i64]
        L.wl_count_degree_le.restype = i64
        L.wl_count_degree_le.argtypes = [vp, i64]
        L.wl_max_degree.restype = i64
        L.wl_max_degree.argtypes = [vp, i32]
        L.wl_mix64.restype = u64
        L.wl_mix64.argtypes = [u64]
        L.wl_unmix64.restype = u64
        L.wl_unmix64.argtypes = [u64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class GraphSpec:
    name: str
    V: int
    P: int
    T: int
    zipf_s: float
    out_cap: int
    in_cap: int
    out_exp: float = 2.2
    in_alpha: float = 0.3
    rho: float = -1.0
    seed: int = 0x18070769


@dataclass
class QuerySpec:
    n_queries: int
    min_tp: int
    max_tp: int
    count_cap: int
    # explicit list of (kind, n_tp, const_mode) for small fixed mixes
    fixed: list = field(default_factory=list)
    const_frac: float = 0.0
    hub_frac: float = 0.0
    seed_offset: int = 1


KIND_CHAIN, KIND_SSTAR, KIND_OSTAR, KIND_SNOW = 0, 1, 2, 3
KIND_NAMES = {0: "chain", 1: "subject-star", 2: "object-star", 3: "snowflake"}

# Configurations: each workload's graph and query specification.
CONFIGS = {
    "tiny": (GraphSpec("tiny", V=10_000, P=16, T=100_000, zipf_s=1.1, out_cap=2000,
                       in_cap=2000, seed=0x18070769 ^ 1),
             QuerySpec(8, 2, 4, 10**7, fixed=[(0, 2, 0), (0, 3, 0), (1, 2, 0), (1, 3, 0),
                                                (1, 4, 0), (3, 4, 0), (3, 4, 0), (0, 2, 1)])),
    "medium": (GraphSpec("medium", V=2_000_000, P=64, T=20_000_000, zipf_s=1.1, out_cap=2000,
                         in_cap=20_000, seed=0x18070769 ^ 2),
               QuerySpec(64, 2, 6, 10**7, const_frac=0.25)),
    "large": (GraphSpec("large", V=40_000_000, P=1024, T=200_000_000, zipf_s=1.2,
                        out_cap=100_000, in_cap=1_000_000, seed=0x18070769 ^ 3),
              QuerySpec(128, 2, 8, 10**9, const_frac=0.25, hub_frac=0.125)),
}


def gen_graph(spec: GraphSpec):
    """Return (s, p, o) int32 arrays with exactly spec.T distinct triples."""
    L = lib()
    s = np.empty(spec.T, np.int32)
    p = np.empty(spec.T, np.int32)
    o = np.empty(spec.T, np.int32)
    n = L.wl_gen_graph(spec.V, spec.P, spec.T, spec.zipf_s, spec.out_exp, spec.out_cap,
                       spec.in_alpha, spec.in_cap, spec.rho, spec.seed & (2**64 - 1),
                       _ptr(s), _ptr(p), _ptr(o))
    if n != spec.T:
        raise RuntimeError(f"graph generation failed: code {n}")
    return s, p, o


class GraphIndex:
    """Generator-private adjacency used to draw walks and count tree queries."""

    def __init__(self, s, p, o, V, P):
        self._keep = (np.ascontiguousarray(s, np.int32), np.ascontiguousarray(p, np.int32),
                      np.ascontiguousarray(o, np.int32))
        self.V, self.P = V, P
        self.h = lib().wl_index_new(_ptr(self._keep[0]), _ptr(self._keep[1]),
                                    _ptr(self._keep[2]), len(s), V, P)

    def close(self):
        if self.h:
            lib().wl_index_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def count(self, tps: np.ndarray, n_vars: int) -> int:
        """Exact result size of a tree-shaped BGP; -1 if not a tree."""
        t = np.ascontiguousarray(tps, np.int32).reshape(-1, 3)
        return int(lib().wl_count_tree(self.h, _ptr(t), len(t), n_vars))

    def count_many(self, queries):
        """Exact counts of several (tps, n_vars) queries, computed concurrently."""
        if not queries:
            return []
        tps = np.ascontiguousarray(np.concatenate([np.asarray(t, np.int32).reshape(-1, 3)
                                                   for t, _ in queries]), np.int32)
        ntp = np.array([len(np.asarray(t).reshape(-1, 3)) for t, _ in queries], np.int32)
        nv = np.array([v for _, v in queries], np.int32)
        off = np.concatenate([[0], np.cumsum(ntp)[:-1]]).astype(np.int64)
        out = np.empty(len(queries), np.int64)
        lib().wl_count_many(self.h, _ptr(tps), _ptr(ntp), _ptr(nv), _ptr(off), len(queries),
                            _ptr(out))
        return out.tolist()

    def degree_le_fraction(self, d: int) -> float:
        return lib().wl_count_degree_le(self.h, d) / self.V

    def max_degree(self, which: int = 0) -> int:
        return int(lib().wl_max_degree(self.h, which))

    def hubs(self, top_frac: float) -> np.ndarray:
        """Vertices in the top `top_frac` of total degree (at least one)."""
        L = lib()
        # find the degree threshold by scanning decreasing powers of two
        want = max(1, int(self.V * top_frac))
        thr = self.max_degree(0)
        while thr > 1 and L.wl_vertices_with_degree(self.h, thr, None, 0) < want:
            thr = thr * 3 // 4
        n = L.wl_vertices_with_degree(self.h, thr, None, 0)
        out = np.empty(n, np.int32)
        L.wl_vertices_with_degree(self.h, thr, _ptr(out), n)
        return out

    def walk(self, kind, n, const_mode, start, seed, ctr, bias=0.0):
        tp = np.empty((n, 3), np.int32)
        wit = np.empty(n + 1, np.int32)
        nv = lib().wl_walk_query(self.h, kind, n, const_mode, start, bias, seed & (2**64 - 1),
                                 ctr, _ptr(tp), _ptr(wit))
        if nv <= 0:
            return None
        return tp, wit[:nv].copy(), nv


@dataclass
class Query:
    tps: np.ndarray  # (n, 3) int32
    n_vars: int
    witness: np.ndarray
    count: int
    kind: int
    const_mode: int


def _rng_u64(seed, i):
    return int(lib().wl_mix64((seed ^ lib().wl_mix64(i * 0x9E3779B97F4A7C15 & (2**64 - 1)))
                              & (2**64 - 1)))


# predicate-choice bias per shape: stars and snowflakes favour rarer predicates
SHAPE_BIAS = {KIND_CHAIN: 0.0, KIND_SSTAR: 2.0, KIND_OSTAR: 2.0, KIND_SNOW: 1.0}


def gen_queries(gi: GraphIndex, spec: GraphSpec, qs: QuerySpec, escalate_every=400,
                max_attempts=20_000):
    """Draw the configured BGP mix; every query is a tree with a known count.

    A candidate whose exact count exceeds the cap is rejected.  After every
    `escalate_every` rejections of one query slot, one more leaf of the walk is
    bound to its witness value (free-leaf stars on power-law graphs are
    otherwise far above any cap), never all variables.
    """
    seed = (spec.seed + qs.seed_offset) & (2**64 - 1)
    plan = []
    if qs.fixed:
        plan = list(qs.fixed)
    else:
        kinds = [KIND_CHAIN, KIND_SSTAR, KIND_OSTAR, KIND_SNOW]
        for i in range(qs.n_queries):
            r = _rng_u64(seed, 10 * i + 1)
            kind = kinds[i % 4]
            lo = 4 if kind == KIND_SNOW else qs.min_tp
            n = lo + (r % (qs.max_tp - lo + 1))
            cm = 1 if (_rng_u64(seed, 10 * i + 2) % 1000) < qs.const_frac * 1000 else 0
            plan.append((kind, n, cm))
    hubs = None
    if qs.hub_frac > 0:
        hubs = gi.hubs(1e-4)
    out = []
    ctr = 0
    for qi, (kind, n, cm) in enumerate(plan):
        use_hub = (hubs is not None and len(hubs) > 0 and kind in (KIND_SSTAR, KIND_OSTAR)
                   and (_rng_u64(seed, 10 * qi + 3) % 1000) < qs.hub_frac * 1000 * 2)
        got = None
        for att in range(max_attempts):
            ctr += 1
            k = cm + att // escalate_every
            if k >= n + 1:
                break
            start = -1
            if use_hub:
                start = int(hubs[_rng_u64(seed, 7_000_000 + ctr) % len(hubs)])
            w = gi.walk(kind, n, k, start, seed, ctr, SHAPE_BIAS[kind])
            if w is None:
                continue
            tp, wit, nv = w
            c = gi.count(tp, nv)
            if c < 1 or c > qs.count_cap:
                continue
            got = Query(tp, nv, wit, c, kind, k)
            break
        if got is None:
            raise RuntimeError(f"could not draw query {qi} kind={kind} n={n}")
        out.append(got)
    return out


# Batched workload: the large graph with many small-to-medium BGPs whose result
# sizes spread log-uniformly over [1, 1e6] (one decade per query slot, cycling).
BATCH = QuerySpec(4096, 1, 6, 10**6, seed_offset=7)


def gen_batch_queries(gi: GraphIndex, spec: GraphSpec, qs: QuerySpec = BATCH, n_queries=None,
                      round_size=512, max_rounds=200):
    """n_queries BGPs whose exact counts fill the six decades [10^d, 10^(d+1))
    of [1, count_cap] equally (the last decade includes count_cap), in a
    seeded order.  Candidates are drawn in rounds of `round_size`; each is
    steered at the open decade with the most places left (more bound leaves
    for smaller decades), counted exactly, and accepted in candidate order if
    its decade still has room.  The outcome depends only on the seed."""
    seed = (spec.seed + qs.seed_offset) & (2**64 - 1)
    nq = qs.n_queries if n_queries is None else n_queries
    kinds = [KIND_CHAIN, KIND_SSTAR, KIND_OSTAR, KIND_SNOW]
    cum = np.cumsum([25, 30, 30, 15])
    room = [nq // 6 + (1 if d < nq % 6 else 0) for d in range(6)]
    bins = [[] for _ in range(6)]
    steer = [0] * 6          # per decade: +1 after a candidate above it, -1 below

    def decade(c):
        return 5 if c >= 10**5 else int(math.floor(math.log10(c)))

    def candidate(j, d):
        ctr = j + 1
        r = _rng_u64(seed, 3 * ctr)
        kind = kinds[int(np.searchsorted(cum, int(r % int(cum[-1])), side="right"))]
        r2 = _rng_u64(seed, 3 * ctr + 1)
        n = int((4 + r2 % 3) if kind == KIND_SNOW else (1 + r2 % 6))
        if n == 1:
            kind = KIND_CHAIN
        # bound leaves: many for the small decades, none for the largest,
        # moved by that decade's previous misses, plus a jitter of -1..1
        cmax = min(n, 3) if n > 1 else 1
        jit = int(_rng_u64(seed, 3 * ctr + 2) % 3) - 1
        cm = min(cmax, max(0, round(cmax * (5 - d) / 5) + steer[d] + jit))
        w = gi.walk(kind, n, cm, -1, seed, ctr, SHAPE_BIAS[kind])
        if w is None or w[2] < 1:
            return None
        return kind, cm, w

    j = 0
    for _ in range(max_rounds):
        if not any(room):
            break
        # target decades for this round, in proportion to the places left
        left = sum(room)
        plan = []
        for d in range(6):
            plan += [d] * max(1 if room[d] else 0, round(round_size * room[d] / left))
        pend = []
        for d in plan:
            c = candidate(j, d)
            j += 1
            if c is not None:
                pend.append((d, c))
        counts = gi.count_many([(c[2][0], c[2][2]) for _, c in pend])
        for (d, (kind, cm, (tp, wit, nv))), cnt in zip(pend, counts):
            if cnt < 1:
                continue
            if cnt > qs.count_cap:
                steer[d] = min(3, steer[d] + 1)
                continue
            e = decade(cnt)
            if e != d:
                steer[d] = max(-3, min(3, steer[d] + (1 if e > d else -1)))
            if room[e]:
                bins[e].append(Query(tp, nv, wit, int(cnt), kind, cm))
                room[e] -= 1
    if any(room):
        raise RuntimeError("could not draw the batch workload")
    # interleave the decades in a seeded order
    out = [q for b in bins for q in b]
    perm = np.argsort([_rng_u64(seed ^ 0x5bd1e995, i) for i in range(len(out))], kind="stable")
    return [out[i] for i in perm]


def gen_heavy_queries(gi: GraphIndex, spec: GraphSpec, n_queries=16, lo=5 * 10**7,
                      hi=2 * 10**8, seed_offset=11, round_size=64, max_rounds=100):
    """n_queries BGPs with exact counts in [lo, hi] (the heavy share of a
    served mix): constant-free walks of 2-4 patterns, counted exactly and
    accepted in candidate order."""
    seed = (spec.seed + seed_offset) & (2**64 - 1)
    kinds = [KIND_CHAIN, KIND_SSTAR, KIND_OSTAR, KIND_SNOW]
    out = []
    j = 0
    for _ in range(max_rounds):
        if len(out) >= n_queries:
            break
        pend = []
        for _ in range(round_size):
            ctr = j + 1
            j += 1
            kind = kinds[int(_rng_u64(seed, 2 * ctr) % 4)]
            nt = int(4 if kind == KIND_SNOW else 2 + _rng_u64(seed, 2 * ctr + 1) % 3)
            w = gi.walk(kind, nt, 0, -1, seed, ctr, SHAPE_BIAS[kind])
            if w is not None:
                pend.append((kind, w))
        counts = gi.count_many([(w[0], w[2]) for _, w in pend])
        for (kind, (tp, wit, nv)), cnt in zip(pend, counts):
            if lo <= cnt <= hi and len(out) < n_queries:
                out.append(Query(tp, nv, wit, int(cnt), kind, 0))
    if len(out) < n_queries:
        raise RuntimeError("could not draw the heavy queries")
    return out


def make_workload(name: str):
    spec, qs = CONFIGS[name]
    s, p, o = gen_graph(spec)
    gi = GraphIndex(s, p, o, spec.V, spec.P)
    qs_list = gen_queries(gi, spec, qs)
    return spec, (s, p, o), gi, qs_list
