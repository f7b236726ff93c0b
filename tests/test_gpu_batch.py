"""Batched join parity: every query of a batch yields exactly the rows (in the
same order) and per-step row counts it yields alone through gsmat_join, and
the oracle's row multiset.  Batches mix shapes, sizes, plan modes, repeated
queries, empty results and the cases the batch hands to the single-query
executor (Cartesian steps, (?x p ?x) patterns, budget overflow)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _sorted(a):
    a = np.asarray(a)
    if a.ndim != 2 or len(a) == 0 or a.shape[1] == 0:
        return a
    return a[np.lexsort(a.T[::-1])]


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1807_07691_amd as G
    return G


@pytest.fixture(scope="module")
def O():
    import oracle
    return oracle


def _store(G, s, p, o, V, P, **kw):
    st = G.gsmat_load_triples(s, p, o, V, P)
    G.gsmat_build_index(st, **kw)
    return st


def _single(G, st, tps, mode, budget=0, max_rows=-1):
    pl = G.gsmat_plan(st, tps, mode)
    try:
        r = G.gsmat_join(st, pl, budget, max_rows)
        try:
            return G.gsmat_fetch_bindings(r), G.gsmat_result_info(r)
        finally:
            r.close()
    finally:
        pl.close()


def _check_batch(G, st, queries, mode, budget=0, oracle_rows=None):
    """Batch vs alone (exact order and step counts) and vs the oracle."""
    plans, stat = G.gsmat_plan_batch(st, queries, mode)
    assert stat == [0] * len(queries)
    try:
        for tps, pl in zip(queries, plans):
            one = G.gsmat_plan(st, tps, mode)
            assert G.gsmat_plan_info(pl) == G.gsmat_plan_info(one)
            one.close()
        results, stat = G.gsmat_join_batch(st, plans, budget)
        assert stat == [0] * len(queries)
        try:
            for i, (tps, r) in enumerate(zip(queries, results)):
                got = G.gsmat_fetch_bindings(r)
                info = G.gsmat_result_info(r)
                alone, info1 = _single(G, st, tps, mode, budget)
                assert np.array_equal(got, alone), (i, tps)
                assert info == info1, (i, tps)
                if oracle_rows is not None:
                    want = oracle_rows[i]
                    assert np.array_equal(_sorted(got), want), (i, tps)
        finally:
            for r in results:
                r.close()
    finally:
        for pl in plans:
            pl.close()


# ------------------------------------------------------------------ tiny workload
@pytest.fixture(scope="module")
def tiny(G, O):
    import workload as W
    spec, (s, p, o), gi, qs = W.make_workload("tiny")
    st = _store(G, s, p, o, spec.V, spec.P)
    want = [O.join(s, p, o, q.tps, q.n_vars) for q in qs]
    return spec, s, p, o, qs, st, want


# sparse expansions: off, default, and forced on every expansion with an
# empty row (theta 1, any size)
SPARSE = [(0.0, 4096), (0.5, 4096), (1.0, 1)]


@pytest.mark.parametrize("engine", [1, 0])
@pytest.mark.parametrize("sparse", SPARSE)
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_tiny_workload(G, tiny, mode, sparse, engine):
    spec, s, p, o, qs, st, want = tiny
    print(f"[gpu] batch tiny mode={mode} sparse={sparse} engine={engine}", flush=True)
    G.gsmat_set_sparse_expand(st, *sparse)
    G.gsmat_set_batch_engine(st, engine)
    try:
        queries = [q.tps for q in qs] * 8  # each query 8 times in one batch
        _check_batch(G, st, queries, mode, oracle_rows=want * 8)
    finally:
        G.gsmat_set_sparse_expand(st, 0.5, 4096)
        G.gsmat_set_batch_engine(st, 1)


# starting output slab and scratch region of the device-driven rounds: the
# defaults, and sizes far below one round's needs (tasks wait for space, the
# host adds larger regions between groups of rounds)
REGIONS = [(0, 0), (64 << 10, 8 << 10), (8 << 10, 256 << 10), (1 << 20, 4 << 10)]


@pytest.mark.parametrize("regions", REGIONS)
@pytest.mark.parametrize("mode", [0, 2])
def test_batch_device_regions(G, tiny, mode, regions):
    spec, s, p, o, qs, st, want = tiny
    print(f"[gpu] batch tiny regions={regions} mode={mode}", flush=True)
    G.gsmat_set_sparse_expand(st, 1.0, 1)
    try:
        for rep in range(2):  # the second batch starts from the first one's sizes
            if rep == 0:
                G.gsmat_set_batch_regions(st, *regions)
            queries = [q.tps for q in qs] * 4
            _check_batch(G, st, queries, mode, oracle_rows=want * 4)
    finally:
        G.gsmat_set_sparse_expand(st, 0.5, 4096)
        G.gsmat_set_batch_regions(st, 0, 0)


def _join_all(G, st, plans, budget=0, engine=1):
    G.gsmat_set_batch_engine(st, engine)
    try:
        results, stat = G.gsmat_join_batch(st, plans, budget)
    finally:
        G.gsmat_set_batch_engine(st, 1)
    out = [(G.gsmat_fetch_bindings(r), G.gsmat_result_info(r)) for r in results]
    for r in results:
        r.close()
    return out, stat


def test_batch_autotune(G, tiny):
    """The tuner keeps one candidate of each setting; results do not depend on it."""
    spec, s, p, o, qs, st, want = tiny
    G.gsmat_set_sparse_expand(st, 0.5, 1)
    try:
        queries = [q.tps for q in qs] * 8
        plans, _ = G.gsmat_plan_batch(st, queries, G.PLAN_ADAPTIVE, as_set=True)
        rep = G.gsmat_autotune_batch(st, plans)
        print(f"[gpu] autotune: {rep}", flush=True)
        assert rep["sparse_theta"] in G.SPARSE_CANDIDATES
        assert rep["count_items"] in G.ITEMS_CANDIDATES
        assert rep["intersect"] in G.ISECT_NAMES
        ms = rep["candidate_ms"]
        assert len(ms["sparse_theta"]) == 5 and all(v > 0 for v in ms["sparse_theta"].values())
        assert len(ms["count_items"]) == 3 and all(v > 0 for v in ms["count_items"].values())
        assert len(ms["intersect"]) == 3 and all(v > 0 for v in ms["intersect"].values())
        got = G.gsmat_get_batch_tuning(st)
        assert got["count_items"] == rep["count_items"] and got["intersect"] == rep["intersect"]
        _check_batch(G, st, queries, G.PLAN_ADAPTIVE, oracle_rows=want * 8)
        plans.close()
        # with the host-driven rounds only theta is tuned
        G.gsmat_set_batch_engine(st, 0)
        plans, _ = G.gsmat_plan_batch(st, [q.tps for q in qs], G.PLAN_ADAPTIVE, as_set=True)
        rep = G.gsmat_autotune_batch(st, plans)
        assert all(v == -1 for v in rep["candidate_ms"]["intersect"].values())
        plans.close()
    finally:
        G.gsmat_set_sparse_expand(st, 0.5, 4096)
        G.gsmat_set_batch_engine(st, 1)
        G.gsmat_set_batch_tuning(st, 8, G.ISECT_SEARCH)


# count-phase rows per thread and sorted-list intersection strategy of the
# device-driven rounds
TUNING = [(items, isect) for items in (4, 8, 16) for isect in (0, 1, 2)]


@pytest.mark.parametrize("tuning", TUNING)
def test_batch_tuning_tiny(G, tiny, tuning):
    spec, s, p, o, qs, st, want = tiny
    print(f"[gpu] batch tiny tuning={tuning}", flush=True)
    G.gsmat_set_batch_tuning(st, *tuning)
    G.gsmat_set_sparse_expand(st, 1.0, 1)
    try:
        queries = [q.tps for q in qs] * 2
        for mode in (1, 2):  # the modes that plan star intersections
            _check_batch(G, st, queries, mode, oracle_rows=want * 2)
    finally:
        G.gsmat_set_batch_tuning(st, 8, G.ISECT_SEARCH)
        G.gsmat_set_sparse_expand(st, 0.5, 4096)


def _star_graph():
    """Rows of constant objects made for the intersection strategies: a
    dense run, sparse ids over the whole range, a run overlapping the first,
    half of all ids, every id, and a predicate with variable objects (a list
    of row keys).  Driver tiles then meet windows shorter and longer than the
    2048 ids a workgroup stages."""
    rng = np.random.default_rng(11)
    V = 60_000
    def take(ids, pred, obj):
        return ids.astype(np.int32), np.full(len(ids), pred, np.int32), np.full(len(ids), obj, np.int32)
    parts = [
        take(np.flatnonzero(rng.random(6000) < 0.9), 0, 1),
        take(np.flatnonzero(rng.random(V) < 0.05), 1, 2),
        take(np.arange(3000, 9000), 2, 3),
        take(rng.choice(V, V // 2, replace=False), 3, 4),
        take(np.arange(V), 4, 5),
    ]
    ks = rng.choice(V, 20_000, replace=False)
    parts.append((ks.astype(np.int32), np.full(len(ks), 5, np.int32),
                  rng.integers(0, V, len(ks)).astype(np.int32)))
    s = np.concatenate([a for a, _, _ in parts])
    p = np.concatenate([b for _, b, _ in parts])
    o = np.concatenate([c for _, _, c in parts])
    return s, p, o, V


STARS = [
    [[-1, 0, 1], [-1, 2, 3]],                   # dense run against an overlapping run
    [[-1, 0, 1], [-1, 3, 4], [-1, 4, 5]],       # dense driver, half and all ids
    [[-1, 1, 2], [-1, 4, 5]],                   # sparse driver: windows past 2048 ids
    [[-1, 1, 2], [-1, 3, 4], [-1, 5, -2]],      # sparse driver, half, row keys
    [[-1, 2, 3], [-1, 3, 4], [-1, 4, 5], [-1, 0, 1]],
    [[-1, 3, 4], [-1, 4, 5]],                   # a long driver (many tiles)
    [[-1, 3, 4], [-1, 5, -2], [-2, 4, 5]],      # intersection, then an expansion
    [[-1, 0, 1], [-1, 1, 2], [-1, 2, 3]],       # few common ids
]


@pytest.mark.parametrize("tuning", TUNING)
def test_batch_tuning_star_intersections(G, O, tuning):
    """Star-centre intersections of long sorted lists under every strategy
    and tile shape: identical to the single-query join (which searches) and
    to the oracle."""
    s, p, o, V = _star_graph()
    st = _store(G, s, p, o, V, 6)
    want = [O.join(s, p, o, q, int(-np.min(np.asarray(q)))) for q in STARS]
    assert min(len(w) for w in want) > 0 and max(len(w) for w in want) > 5000
    print(f"[gpu] batch star intersections tuning={tuning} rows={[len(w) for w in want]}",
          flush=True)
    G.gsmat_set_batch_tuning(st, *tuning)
    for mode in (1, 2):  # the planner's star intersections
        _check_batch(G, st, STARS * 2, mode, oracle_rows=want * 2)
    st.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_batch_tiny_budget_fallback(G, tiny, mode):
    """A budget below some steps' outputs: those queries finish alone."""
    spec, s, p, o, qs, st, want = tiny
    print(f"[gpu] batch tiny budget mode={mode}", flush=True)
    for budget in (4 * 4 * 997, 4 * 4 * 50_000):
        _check_batch(G, st, [q.tps for q in qs], mode, budget=budget, oracle_rows=want)


def test_batch_max_rows_fails_only_that_query(G, tiny):
    spec, s, p, o, qs, st, want = tiny
    big = max(range(len(qs)), key=lambda i: qs[i].count)
    plans, _ = G.gsmat_plan_batch(st, [q.tps for q in qs], G.PLAN_ADAPTIVE)
    limit = qs[big].count - 1
    results, stat = G.gsmat_join_batch(st, plans, max_rows=limit, raise_on_error=False)
    for i, q in enumerate(qs):
        if q.count > limit:
            assert stat[i] == G.GSMAT_ETOOBIG and results[i] is None
        else:
            assert stat[i] == 0
            assert np.array_equal(_sorted(G.gsmat_fetch_bindings(results[i])), want[i])
            results[i].close()
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_join_batch(st, plans, max_rows=limit)
    assert e.value.status == G.GSMAT_ETOOBIG
    for pl in plans:
        pl.close()


def test_batch_empty_and_errors(G, tiny):
    spec, s, p, o, qs, st, want = tiny
    assert G.gsmat_join_batch(st, []) == ([], [])
    plans, stat = G.gsmat_plan_batch(st, [[[-1, 0, -2]], [[-1, -1, -2]], [[-1, 0, -3]]],
                                     raise_on_error=False)
    assert stat == [0, G.GSMAT_EUNSUPPORTED, G.GSMAT_EINVAL]
    assert plans[0] is not None and plans[1] is None and plans[2] is None
    plans[0].close()


# ------------------------------------------------------------------ shapes and random graphs
SHAPES = [
    ([[-1, 0, -2], [-2, 1, -3], [-3, 0, -1]], 3),      # triangle
    ([[-1, 0, -1], [-1, 1, -2]], 2),                   # self loop + expansion
    ([[-1, 2, -1]], 1),                                # self loop only (runs alone)
    ([[-1, 0, -2], [-1, 0, -2], [-2, 1, -3]], 3),      # repeated pattern
    ([[-1, 0, -2], [-3, 1, -4]], 4),                   # disconnected (runs alone)
    ([[1, 0, 2]], 0),                                  # all constant
    ([[1, 0, 2], [5, 1, 5]], 0),                       # all constant, false
    ([[1, 0, -1], [-1, 1, -2]], 2),                    # constant subject chain
    ([[-1, 0, 2], [-1, 1, -2], [-1, 2, -3]], 3),       # star with a constant object
    ([[-1, 0, -2], [-2, 0, -1]], 2),                   # two-cycle
    ([[-2, 0, -1], [-3, 1, -1], [-4, 2, -1]], 4),      # object star
    ([[-1, 0, -2], [-2, 1, -3], [-1, 2, -3]], 3),      # filter with both ends bound
    ([[-1, 0, 99], [-1, 1, -2]], 2),                   # absent constant
    ([[-1, 7, -2]], 2),                                # absent predicate
    ([[-1, 1, -2]], 2),                                # one pattern
    ([[1, 0, -1], [-1, 1, 2]], 1),                     # constants at both ends of a chain
]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_shapes(G, O, mode):
    rng = np.random.default_rng(7)
    V, P = 12, 3
    s, p, o = (rng.integers(0, V, 150).astype(np.int32), rng.integers(0, P, 150).astype(np.int32),
               rng.integers(0, V, 150).astype(np.int32))
    s = np.concatenate([s, [1, 2, 3, 4]]).astype(np.int32)
    p = np.concatenate([p, [0, 0, 0, 2]]).astype(np.int32)
    o = np.concatenate([o, [2, 2, 3, 4]]).astype(np.int32)
    st = _store(G, s, p, o, 100, 8)
    print(f"[gpu] batch shapes mode={mode}", flush=True)
    want = [O.join(s, p, o, t, nv) for t, nv in SHAPES]
    _check_batch(G, st, [t for t, _ in SHAPES], mode, oracle_rows=want)


@pytest.mark.parametrize("regions", [(0, 0), (64 << 10, 8 << 10)])
def test_batch_past_register_kernels(G, O, regions):
    """More than 4096 queries in one batch (the shapes, a few rows each): the
    single-workgroup kernels that hold four queries per thread in registers
    give way to their looping versions, also with tasks deferred for want of
    space."""
    rng = np.random.default_rng(7)
    s, p, o = (rng.integers(0, 12, 150).astype(np.int32), rng.integers(0, 3, 150).astype(np.int32),
               rng.integers(0, 12, 150).astype(np.int32))
    st = _store(G, s, p, o, 100, 8)
    want = [O.join(s, p, o, t, nv) for t, nv in SHAPES]
    reps = 4200 // len(SHAPES) + 1
    queries = [t for t, _ in SHAPES] * reps
    assert len(queries) > 4096 and sum(len(w) for w in want) * reps < 10**6
    print(f"[gpu] batch of {len(queries)} queries, regions={regions}", flush=True)
    G.gsmat_set_batch_regions(st, *regions)
    _check_batch(G, st, queries, G.PLAN_ADAPTIVE, oracle_rows=want * reps)
    st.close()


@pytest.mark.parametrize("seed", range(8))
def test_batch_random_graphs(G, O, seed):
    rng = np.random.default_rng(900 + seed)
    V = int(rng.integers(5, 3000))
    P = int(rng.integers(1, 6))
    n = int(rng.integers(10, 40000))
    s, p, o = (rng.integers(0, V, n).astype(np.int32), rng.integers(0, P, n).astype(np.int32),
               rng.integers(0, V, n).astype(np.int32))
    st = G.gsmat_load_triples(s, p, o, V, P)
    if seed % 2:  # bitmaps for the rows of at least 1-7 members
        G.gsmat_set_hub_options(st, int(rng.integers(1, 8)), 1 << 26)
    G.gsmat_build_index(st, dense_div=int(rng.choice([1, 32, 10**6])))
    G.gsmat_set_sparse_expand(st, *SPARSE[seed % 3])
    G.gsmat_set_batch_tuning(st, *TUNING[(seed * 4) % len(TUNING)])
    queries, want = [], []
    while len(queries) < 70:
        ntp = int(rng.integers(1, 5))
        nvars = int(rng.integers(1, 5))
        tps = []
        for _ in range(ntp):
            def term():
                return int(rng.integers(0, V)) if rng.random() < 0.25 else -int(rng.integers(0, nvars)) - 1
            tps.append([term(), int(rng.integers(0, P)), term()])
        used = sorted({-t - 1 for tp in tps for t in (tp[0], tp[2]) if t < 0})
        remap = {x: i for i, x in enumerate(used)}
        tps = [[(-remap[-a - 1] - 1) if a < 0 else a, b, (-remap[-c - 1] - 1) if c < 0 else c]
               for a, b, c in tps]
        try:
            w = O.join(s, p, o, tps, len(used), cap_rows=3_000_000)
        except ValueError:
            continue  # too large for this test
        queries.append(np.array(tps, np.int32))
        want.append(w)
    print(f"[gpu] batch random seed={seed} V={V} P={P} n={n}", flush=True)
    for mode in (0, 1, 2):
        _check_batch(G, st, queries, mode, oracle_rows=want)
    # the host-driven and device-driven rounds give the same rows, in the
    # same order, and the same step counts
    plans, _ = G.gsmat_plan_batch(st, queries, 2)
    a, sa = _join_all(G, st, plans, engine=0)
    b, sb = _join_all(G, st, plans, engine=1)
    assert sa == sb == [0] * len(queries)
    for i, ((ra, ia), (rb, ib)) in enumerate(zip(a, b)):
        assert np.array_equal(ra, rb) and ia == ib, i
    for pl in plans:
        pl.close()


# ------------------------------------------------------------------ medium graph
@pytest.mark.timeout(600)
def test_batch_medium_workload(G, O):
    """The medium graph's 64 BGPs (up to 1e7 rows) in one batch: identical to
    the single-query join; the oracle's rows or row fingerprint."""
    import workload as W
    spec, (s, p, o), gi, qs = W.make_workload("medium")
    gi.close()
    st = _store(G, s, p, o, spec.V, spec.P)
    G.gsmat_set_sparse_expand(st, 1.0, 1)  # every expansion with an empty row compacted
    ds = O.Dataset(s, p, o)
    queries = [q.tps for q in qs]
    plans, _ = G.gsmat_plan_batch(st, queries, G.PLAN_ADAPTIVE)
    results, _ = G.gsmat_join_batch(st, plans, 64 * 2**30)
    checked = 0
    for i, (q, r) in enumerate(zip(qs, results)):
        print(f"[gpu] batch medium q{i} rows={q.count}", flush=True)
        got = G.gsmat_fetch_bindings(r)
        assert len(got) == q.count
        alone, _ = _single(G, st, q.tps, G.PLAN_ADAPTIVE, 64 * 2**30)
        assert np.array_equal(got, alone), i
        try:
            if q.count <= 2 * 10**6:
                assert np.array_equal(_sorted(got), ds.join(q.tps, q.n_vars, cap_rows=5 * 10**7))
            else:
                want = ds.join(q.tps, q.n_vars, cap_rows=5 * 10**7, fingerprint=True)
                assert O.fingerprint_rows(got) == want
            checked += 1
        except ValueError:
            pass  # the oracle's intermediate exceeded its cap; the count pins it
        r.close()
    for pl in plans:
        pl.close()
    assert checked >= 50


# ------------------------------------------------------------------ wide tables
def _wide_graph(seed, V=300):
    """Two predicates giving most vertices one successor (a few two, some
    none), so long chains keep tens to hundreds of rows and expansions have
    input rows without output."""
    rng = np.random.default_rng(seed)
    s, p, o = [], [], []
    for pred in (0, 1):
        src = rng.choice(V, int(V * 0.9), replace=False)
        dst = rng.integers(0, V, len(src))
        extra = rng.choice(V, V // 5, replace=False)
        s += [src, extra]
        o += [dst, rng.integers(0, V, len(extra))]
        p += [np.full(len(src) + len(extra), pred)]
    return (np.concatenate(s).astype(np.int32), np.concatenate(p).astype(np.int32),
            np.concatenate(o).astype(np.int32), V)


def _chain(n, preds, const_start=None):
    tps = []
    for i in range(n):
        a = -(i + 1) if (i > 0 or const_start is None) else const_start
        tps.append([a, preds[i % len(preds)], -(i + 2)])
    if const_start is not None:  # renumber: variables from 0
        tps = [[x if x >= 0 else x + 1, q, y + 1] for x, q, y in tps]
    return tps


@pytest.mark.parametrize("sparse", [(0.0, 4096), (1.0, 1)])
def test_batch_wide_tables(G, O, sparse):
    """Chains of 7 to 14 patterns: every column count of the batched write and
    compaction (8 to 15 columns, past the specialised ones), against the
    plain join and the oracle, with the sparse write off and forced on."""
    s, p, o, V = _wide_graph(21)
    st = _store(G, s, p, o, V, 2)
    queries = []
    for n in range(7, 15):
        queries.append(_chain(n, [0, 1]))
        queries.append(_chain(n, [1, 1, 0], const_start=int(n * 7 % V)))
    # a snowflake closing a cycle: a filter over a wide table
    queries.append(_chain(11, [0]) + [[-12, 1, -1]])
    nv = [int(-np.min(np.asarray(q))) for q in queries]
    want = [O.join(s, p, o, q, k) for q, k in zip(queries, nv)]
    assert max(len(w) for w in want) > 50
    print(f"[gpu] batch wide tables sparse={sparse} rows={[len(w) for w in want]}", flush=True)
    G.gsmat_set_sparse_expand(st, *sparse)
    for mode in (0, 2):
        _check_batch(G, st, queries, mode, oracle_rows=want)
    st.close()


# ------------------------------------------------------------------ fused plan + join
def _check_fused(G, st, queries, mode, budget=0, oracle_rows=None):
    """gsmat_join_batch_bgp against gsmat_plan_batch + gsmat_join_batch (the
    device-driven rounds): the same rows in the same order and the same
    per-step counters; the oracle's sorted rows where given."""
    G.gsmat_set_batch_engine(st, 1)
    plans, _ = G.gsmat_plan_batch(st, queries, mode)
    want, _ = G.gsmat_join_batch(st, plans, budget)
    got, stat = G.gsmat_join_batch_bgp(st, queries, mode, budget)
    assert stat == [0] * len(queries)
    for i, (a, b) in enumerate(zip(got, want)):
        ra, rb = G.gsmat_fetch_bindings(a), G.gsmat_fetch_bindings(b)
        assert np.array_equal(ra, rb), (i, queries[i])
        assert G.gsmat_result_info(a) == G.gsmat_result_info(b), i
        if oracle_rows is not None:
            assert np.array_equal(_sorted(ra), oracle_rows[i]), i
        a.close()
        b.close()
    for pl in plans:
        pl.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_fused_tiny_and_shapes(G, O, tiny, mode):
    spec, s, p, o, qs, st, want = tiny
    print(f"[gpu] fused plan + join, tiny and shapes, mode={mode}", flush=True)
    _check_fused(G, st, [q.tps for q in qs] * 2, mode, oracle_rows=want * 2)
    rng = np.random.default_rng(7)
    s2, p2, o2 = (rng.integers(0, 12, 150).astype(np.int32),
                  rng.integers(0, 3, 150).astype(np.int32),
                  rng.integers(0, 12, 150).astype(np.int32))
    st2 = _store(G, s2, p2, o2, 100, 8)
    w2 = [O.join(s2, p2, o2, t, nv) for t, nv in SHAPES]
    _check_fused(G, st2, [t for t, _ in SHAPES], mode, oracle_rows=w2)
    st2.close()


def test_fused_errors_budget_and_large_batch(G, tiny):
    """Invalid queries fail alone with their planning status; a small budget
    sends queries to the chunked single path with their plans built on the
    way; a batch above 4096 queries."""
    spec, s, p, o, qs, st, want = tiny
    queries = [qs[0].tps, [[-1, 0, -3]], qs[1].tps, [[-1, -1, -2]]]
    res, stat = G.gsmat_join_batch_bgp(st, queries, G.PLAN_ADAPTIVE, raise_on_error=False)
    assert stat == [0, G.GSMAT_EINVAL, 0, G.GSMAT_EUNSUPPORTED]
    assert res[1] is None and res[3] is None
    for i, w in ((0, want[0]), (2, want[1])):
        assert np.array_equal(_sorted(G.gsmat_fetch_bindings(res[i])), w)
        res[i].close()
    with pytest.raises(G.GsmatError):
        G.gsmat_join_batch_bgp(st, queries, G.PLAN_ADAPTIVE)
    _check_fused(G, st, [q.tps for q in qs], G.PLAN_ADAPTIVE, budget=4 * 4 * 50_000,
                 oracle_rows=want)
    small = [q.tps for q in qs if q.count <= 5000] or [qs[0].tps]
    reps = 4200 // len(small) + 1
    print(f"[gpu] fused batch of {len(small) * reps} queries", flush=True)
    _check_fused(G, st, small * reps, G.PLAN_ADAPTIVE)
