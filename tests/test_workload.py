"""Seeded workload generator: determinism, set size, degree shape, query validity."""
import numpy as np
import pytest

import workload as W


def test_mix_bijection_inverse():
    L = W.lib()
    rng = np.random.default_rng(0)
    for x in rng.integers(0, 2**63, 200, dtype=np.int64).tolist() + [0, 1, 2**64 - 1]:
        assert L.wl_unmix64(L.wl_mix64(x)) == x


@pytest.fixture(scope="module")
def tiny():
    spec, qs = W.CONFIGS["tiny"]
    s, p, o = W.gen_graph(spec)
    return spec, qs, s, p, o


def test_graph_deterministic(tiny):
    spec, qs, s, p, o = tiny
    s2, p2, o2 = W.gen_graph(spec)
    assert np.array_equal(s, s2) and np.array_equal(p, p2) and np.array_equal(o, o2)


def test_graph_is_a_set_of_exact_size(tiny):
    spec, qs, s, p, o = tiny
    assert len(s) == spec.T
    assert len(set(zip(s.tolist(), p.tolist(), o.tolist()))) == spec.T
    assert s.min() >= 0 and s.max() < spec.V and o.min() >= 0 and o.max() < spec.V
    assert p.min() >= 0 and p.max() < spec.P
    # every predicate is used, frequencies fall with the Zipf rank
    cnt = np.bincount(p, minlength=spec.P)
    assert (cnt > 0).all()
    assert cnt[0] > cnt[spec.P // 2] > 0


def test_degree_shape(tiny):
    spec, qs, s, p, o = tiny
    gi = W.GraphIndex(s, p, o, spec.V, spec.P)
    assert gi.degree_le_fraction(40) >= 0.95
    assert gi.max_degree(1) <= spec.out_cap
    assert gi.max_degree(0) > 200  # hubs exist


def test_queries_nonempty_and_counted(tiny):
    spec, qs, s, p, o = tiny
    gi = W.GraphIndex(s, p, o, spec.V, spec.P)
    ql = W.gen_queries(gi, spec, qs)
    assert len(ql) == 8
    kinds = [q.kind for q in ql]
    assert kinds.count(W.KIND_CHAIN) == 3 and kinds.count(W.KIND_SSTAR) == 3
    assert kinds.count(W.KIND_SNOW) == 2
    assert any(q.const_mode > 0 and q.kind == W.KIND_CHAIN for q in ql)
    D = set(zip(s.tolist(), p.tolist(), o.tolist()))
    for q in ql:
        assert 1 <= q.count <= qs.count_cap
        for a, b, c in q.tps.tolist():  # the witness satisfies every pattern
            sa = a if a >= 0 else int(q.witness[-a - 1])
            oc = c if c >= 0 else int(q.witness[-c - 1])
            assert (sa, b, oc) in D
    ql2 = W.gen_queries(gi, spec, qs)
    assert all(np.array_equal(a.tps, b.tps) for a, b in zip(ql, ql2))


def test_tree_count_small_brute_force():
    import oracle as O  # the count program is checked against enumeration
    rng = np.random.default_rng(11)
    V, P = 6, 2
    s = rng.integers(0, V, 40).astype(np.int32)
    p = rng.integers(0, P, 40).astype(np.int32)
    o = rng.integers(0, V, 40).astype(np.int32)
    s, p, o = O.dedupe(s, p, o)
    gi = W.GraphIndex(s, p, o, V, P)
    for tps, nv in [([[-1, 0, -2], [-2, 1, -3]], 3), ([[-1, 0, -2], [-1, 1, -3], [-4, 0, -1]], 4),
                    ([[-1, 1, 3], [-1, 0, -2]], 2), ([[-1, 0, -2], [-3, 1, -4]], 4)]:
        assert gi.count(np.array(tps), nv) == len(O.brute_force(s, p, o, tps, nv, V))
    assert gi.count(np.array([[-1, 0, -2], [-2, 1, -1]]), 2) == -1  # cycle: not a tree


def test_tree_count_push_and_pull_paths_match_oracle():
    """Random tree BGPs with constant leaves (small child supports take the
    generator's push path, free leaves the pull path) against the oracle."""
    import oracle as O
    spec, qs = W.CONFIGS["tiny"]
    s, p, o = W.gen_graph(spec)
    gi = W.GraphIndex(s, p, o, spec.V, spec.P)
    seed = 12345
    checked = 0
    for ctr in range(1, 400):
        kind = ctr % 4
        n = 2 + ctr % 3 if kind != W.KIND_SNOW else 4
        w = gi.walk(kind, n, ctr % 3, -1, seed, ctr, W.SHAPE_BIAS[kind])
        if w is None:
            continue
        tp, wit, nv = w
        c = gi.count(tp, nv)
        if c > 200_000:
            continue
        assert c == len(O.join(s, p, o, tp, nv)), tp.tolist()
        checked += 1
        if checked >= 40:
            break
    assert checked >= 30
