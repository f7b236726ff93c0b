"""GPU parity: the C-ABI library against the CPU oracle, bit-exact.

Every comparison is on sorted row multisets (row order of the library is
unspecified; the sorted set is unique because D is a set and every variable
is projected).
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


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


# ------------------------------------------------------------------ worked example
@pytest.fixture(scope="module")
def example(G):
    with open(os.path.join(GOLD, "worked_example.json")) as f:
        g = json.load(f)
    spo = np.array(g["cube_spo"], np.int32)
    st = _store(G, spo[:, 0], spo[:, 1], spo[:, 2], g["n_vertices"], g["n_predicates"])
    return g, spo, st


@pytest.mark.parametrize("mode", [0, 1])
def test_worked_example_answer(G, example, mode):
    g, spo, st = example
    print(f"[gpu] worked example mode={mode}", flush=True)
    rows = _sorted(G.evaluate(st, g["query_tps"], mode))
    assert rows.tolist() == g["answer_xyzw"]


def test_worked_example_index(G, O, example):
    g, spo, st = example
    assert G.gsmat_store_stats(st)["n_triples"] == 9
    for h, pairs in g["matrices"].items():
        for orient in (0, 1):
            want = O.csr(spo[:, 0], spo[:, 1], spo[:, 2], int(h), orient)
            got = G.gsmat_export_matrix(st, int(h), orient)
            for a, b in zip(got, want):
                assert np.array_equal(a, b), (h, orient)
    keys, ptr, nbr = G.gsmat_export_matrix(st, 1, 0)
    assert keys.tolist() == g["aux_A_X"]["Row"]
    assert np.diff(ptr).tolist() == g["aux_A_X"]["Num"]


def test_worked_example_plan_and_steps(G, example):
    g, spo, st = example
    pl = G.gsmat_plan(st, g["query_tps"], G.PLAN_PAPER)
    nv, steps = G.gsmat_plan_info(pl)
    assert [s["tp"] for s in steps] == g["paper_plan_order"]
    r = G.gsmat_join(st, pl)
    info = G.gsmat_result_info(r)
    # C = (x likes w) join (z likes w) has 5 rows; final answer 1 row
    assert info["step_rows_out"][0] == 3 and info["step_rows_out"][1] == 5
    assert info["rows"] == 1


# ------------------------------------------------------------------ tiny power-law workload
@pytest.fixture(scope="module")
def tiny(G):
    import workload as W
    spec, (s, p, o), gi, qs = W.make_workload("tiny")
    st = _store(G, s, p, o, spec.V, spec.P)
    st_dense = _store(G, s, p, o, spec.V, spec.P, dense_div=100000)  # all predicates dense
    return spec, s, p, o, qs, st, st_dense


def test_tiny_index_matches_oracle(G, O, tiny):
    spec, s, p, o, qs, st, st_dense = tiny
    assert G.gsmat_store_stats(st)["n_triples"] == len(O.dedupe(s, p, o)[0])
    for pred in range(spec.P):
        for orient in (0, 1):
            want = O.csr(s, p, o, pred, orient)
            got = G.gsmat_export_matrix(st, pred, orient)
            assert all(np.array_equal(a, b) for a, b in zip(got, want)), (pred, orient)


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("qi", range(8))
def test_tiny_queries(G, O, tiny, mode, qi):
    spec, s, p, o, qs, st, st_dense = tiny
    q = qs[qi]
    print(f"[gpu] tiny query {qi} mode={mode} tps={q.tps.tolist()}", flush=True)
    want = O.join(s, p, o, q.tps, q.n_vars)
    assert len(want) == q.count
    for store in (st, st_dense):
        got = _sorted(G.evaluate(store, q.tps, mode))
        assert got.shape == want.shape
        assert np.array_equal(got, want)


@pytest.fixture(scope="module")
def tiny_hub(G, tiny):
    """The tiny graph with a bitmap for every row of at least 2 members."""
    spec, s, p, o, qs, st, st_dense = tiny
    h = G.gsmat_load_triples(s, p, o, spec.V, spec.P)
    G.gsmat_set_hub_options(h, 2, 1 << 30)
    G.gsmat_build_index(h)
    assert G.gsmat_store_stats(h)["device_bytes"] > G.gsmat_store_stats(st)["device_bytes"]
    return h


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_tiny_queries_with_hub_bitmaps(G, O, tiny, tiny_hub, mode):
    """Filters and constant-row intersections answered by bitmaps give the
    same rows, in the same order, as searching the rows."""
    spec, s, p, o, qs, st, st_dense = tiny
    print(f"[gpu] tiny queries with hub bitmaps mode={mode}", flush=True)
    for q in qs:
        want = O.join(s, p, o, q.tps, q.n_vars)
        got = G.evaluate(tiny_hub, q.tps, mode)
        assert np.array_equal(_sorted(got), want)
        assert np.array_equal(got, G.evaluate(st, q.tps, mode))
    # stars through constants and filters with both ends bound
    for tps, nv in [([[-1, 0, int(o[0])], [-1, 1, -2], [-1, 2, int(o[5])]], 2),
                    ([[int(s[3]), 0, -1], [-1, 1, -2], [int(s[3]), 2, -2]], 2),
                    ([[-1, 0, -2], [-2, 1, -3], [-1, 2, -3]], 3)]:
        want = O.join(s, p, o, tps, nv)
        assert np.array_equal(_sorted(G.evaluate(tiny_hub, tps, mode)), want)


@pytest.mark.parametrize("qi", [1, 4, 5])
def test_tiny_chunked(G, O, tiny, qi):
    """A tiny byte budget forces every expansion to be cut into output ranges."""
    spec, s, p, o, qs, st, st_dense = tiny
    q = qs[qi]
    print(f"[gpu] tiny chunked query {qi}", flush=True)
    want = O.join(s, p, o, q.tps, q.n_vars)
    for budget in (4 * (q.n_vars + 1) * 997, 4 * (q.n_vars + 1) * 50_000):
        for mode in (1, 2):
            got = _sorted(G.evaluate(st, q.tps, mode, budget_bytes=budget))
            assert np.array_equal(got, want), (budget, mode)


def test_tiny_plan_permutation_invariance(G, O, tiny):
    spec, s, p, o, qs, st, st_dense = tiny
    rng = np.random.default_rng(0)
    for q in qs[:6]:
        want = O.join(s, p, o, q.tps, q.n_vars)
        for _ in range(3):
            perm = rng.permutation(len(q.tps))
            got = _sorted(G.evaluate(st, q.tps[perm], 2))
            assert np.array_equal(got, want)


def test_tiny_step_counts_consistent(G, O, tiny):
    """Per-step output rows equal the oracle's row count of the same prefix join."""
    spec, s, p, o, qs, st, st_dense = tiny
    q = qs[1]
    pl = G.gsmat_plan(st, q.tps, G.PLAN_PAPER)
    nv, steps = G.gsmat_plan_info(pl)
    r = G.gsmat_join(st, pl)
    info = G.gsmat_result_info(r)
    order = [stp["tp"] for stp in steps]
    for j in range(len(order)):
        sub = q.tps[order[: j + 1]]
        used = sorted({-t - 1 for t in sub[:, [0, 2]].ravel() if t < 0})
        remap = {v: i for i, v in enumerate(used)}
        sub2 = np.array([[(-remap[-a - 1] - 1) if a < 0 else a, b, (-remap[-c - 1] - 1) if c < 0 else c]
                         for a, b, c in sub.tolist()], np.int32)
        n = O.join(s, p, o, sub2, len(used), fingerprint=True)[0]
        assert info["step_rows_out"][j] == n, j


# ------------------------------------------------------------------ random toys and shapes
def _rand_graph(rng, V, P, n):
    return (rng.integers(0, V, n).astype(np.int32), rng.integers(0, P, n).astype(np.int32),
            rng.integers(0, V, n).astype(np.int32))


SHAPES = {
    "triangle": ([[-1, 0, -2], [-2, 1, -3], [-3, 0, -1]], 3),
    "self_loop": ([[-1, 0, -1], [-1, 1, -2]], 2),
    "self_loop_only": ([[-1, 2, -1]], 1),
    "repeated_tp": ([[-1, 0, -2], [-1, 0, -2], [-2, 1, -3]], 3),
    "disconnected": ([[-1, 0, -2], [-3, 1, -4]], 4),
    "all_constant": ([[1, 0, 2]], 0),
    "all_constant_false": ([[1, 0, 2], [5, 1, 5]], 0),
    "const_subject": ([[1, 0, -1], [-1, 1, -2]], 2),
    "const_object_star": ([[-1, 0, 2], [-1, 1, -2], [-1, 2, -3]], 3),
    "two_cycle": ([[-1, 0, -2], [-2, 0, -1]], 2),
    "object_star": ([[-2, 0, -1], [-3, 1, -1], [-4, 2, -1]], 4),
    "filter_both_bound": ([[-1, 0, -2], [-2, 1, -3], [-1, 2, -3]], 3),
    "absent_constant": ([[-1, 0, 99], [-1, 1, -2]], 2),
    "absent_predicate": ([[-1, 7, -2]], 2),
    "single_tp": ([[-1, 1, -2]], 2),
    "const_both_in_chain": ([[1, 0, -1], [-1, 1, 2]], 1),
}


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_shapes(G, O, shape, mode):
    tps, nv = SHAPES[shape]
    rng = np.random.default_rng(7)
    V, P = 12, 3
    s, p, o = _rand_graph(rng, V, P, 150)
    s = np.concatenate([s, [1, 2, 3, 4]]).astype(np.int32)
    p = np.concatenate([p, [0, 0, 0, 2]]).astype(np.int32)
    o = np.concatenate([o, [2, 2, 3, 4]]).astype(np.int32)
    print(f"[gpu] shape {shape} mode={mode}", flush=True)
    st = _store(G, s, p, o, 100, 8)
    want = O.join(s, p, o, tps, nv)
    got = _sorted(G.evaluate(st, tps, mode))
    assert got.shape == want.shape and np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(24))
def test_random_bgps(G, O, seed):
    rng = np.random.default_rng(500 + seed)
    V = int(rng.integers(5, 60))
    P = int(rng.integers(1, 5))
    s, p, o = _rand_graph(rng, V, P, int(rng.integers(10, 600)))
    s = np.concatenate([s, s[:20]])  # duplicates: the store keeps the set
    p = np.concatenate([p, p[:20]])
    o = np.concatenate([o, o[:20]])
    st = G.gsmat_load_triples(s, p, o, V, P)
    if rng.random() < 0.5:  # bitmaps for the rows of at least 1-7 members
        G.gsmat_set_hub_options(st, int(rng.integers(1, 8)), 1 << 26)
    G.gsmat_build_index(st, dense_div=int(rng.choice([1, 32, 10**6])))
    for trial in range(4):
        ntp = int(rng.integers(1, 6))
        nvars = int(rng.integers(1, 5))
        tps = []
        for _ in range(ntp):
            def term():
                return int(rng.integers(0, V)) if rng.random() < 0.2 else -int(rng.integers(0, nvars)) - 1
            tps.append([term(), int(rng.integers(0, P)), term()])
        used = sorted({-t - 1 for tp in tps for t in (tp[0], tp[2]) if t < 0})
        remap = {x: i for i, x in enumerate(used)}
        tps = [[(-remap[-a - 1] - 1) if a < 0 else a, b, (-remap[-c - 1] - 1) if c < 0 else c]
               for a, b, c in tps]
        want = O.join(s, p, o, tps, len(used), cap_rows=2_000_000)
        for mode in (0, 1, 2):
            got = _sorted(G.evaluate(st, tps, mode))
            assert got.shape == want.shape and np.array_equal(got, want), (tps, mode)


def test_empty_store_and_errors(G):
    st = _store(G, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32), 10, 2)
    assert G.gsmat_store_stats(st)["n_triples"] == 0
    assert G.evaluate(st, [[-1, 0, -2]]).shape == (0, 2)
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_plan(st, [[-1, -1, -2]])
    assert e.value.status == G.GSMAT_EUNSUPPORTED
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_plan(st, [[-1, 0, -3]])  # variable 1 missing
    assert e.value.status == G.GSMAT_EINVAL


def test_max_rows_and_budget_errors(G, O, tiny):
    spec, s, p, o, qs, st, st_dense = tiny
    q = qs[1]
    pl = G.gsmat_plan(st, q.tps)
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_join(st, pl, max_rows=q.count - 1)
    assert e.value.status == G.GSMAT_ETOOBIG
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_join(st, pl, budget_bytes=3)
    assert e.value.status == G.GSMAT_ENOMEM
    r = G.gsmat_join(st, pl, max_rows=q.count)
    assert G.gsmat_result_info(r)["rows"] == q.count
    # paging through fetch gives the same multiset
    want = O.join(s, p, o, q.tps, q.n_vars)
    parts = [G.gsmat_fetch_bindings(r, off, 1000) for off in range(0, q.count, 1000)]
    assert np.array_equal(_sorted(np.concatenate(parts)), want)
