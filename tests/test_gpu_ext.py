"""OPTIONAL / UNION / FILTER on the GPU (gsmat_join_ext) against the oracle
(oracle/algebra.py, pinned on the CPU by brute force): row multisets equal,
unbound variables as -1.  Random graphs with random well-designed queries,
tables of several tiles with a ragged tail, chunked steps, and the edge
cases: empty required results, OPTIONALs that never or always match, no
required BGP, filter-only branches, variables no branch binds, max_rows."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1807_07691_amd as G
    return G


@pytest.fixture(scope="module")
def A():
    from oracle import algebra
    return algebra


def _sorted(a):
    a = np.asarray(a)
    if a.ndim != 2 or len(a) == 0 or a.shape[1] == 0:
        return a
    return a[np.lexsort(a.T[::-1])]


def _run(G, st, pats, filters, n_vars, **kw):
    r = G.gsmat_join_ext(st, pats, filters, n_vars, **kw)
    try:
        return G.gsmat_fetch_bindings(r)
    finally:
        r.close()


def _check(G, A, st, spo, pats, filters, n_vars, **kw):
    s, p, o = spo
    want = A.join_ext(s, p, o, pats, filters, n_vars)
    got = _run(G, st, pats, filters, n_vars, **kw)
    assert got.shape == (len(want), n_vars), (got.shape, want.shape)
    assert np.array_equal(_sorted(got), want), (np.asarray(pats).tolist(), np.asarray(filters).tolist())
    return len(want)


def _random_query(rng, V, P, spo):
    """A well-designed query: per branch a connected required BGP of 1-3
    patterns grown from a vertex with edges, OPTIONAL groups hanging off
    required variables (new variables private to the group, sometimes a
    constant or a second pattern), and FILTERs over any variable."""
    s, p, o = spo
    n_vars = 0
    pats, filters = [], []
    for br in range(int(rng.integers(1, 3))):
        req_vars = []
        def new_var():
            nonlocal n_vars
            n_vars += 1
            return -n_vars
        if rng.random() < 0.08:
            x = new_var()
        else:
            e = int(rng.integers(0, len(s)))
            x = new_var()
            req_vars.append(x)
            y = new_var() if rng.random() < 0.8 else int(o[e])
            pats.append([x, int(p[e]), y, br, 0])
            if y < 0:
                req_vars.append(y)
            for _ in range(int(rng.integers(0, 3))):
                a = int(rng.choice(req_vars))
                z = new_var()
                if rng.random() < 0.5:
                    pats.append([a, int(rng.integers(0, P)), z, br, 0])
                else:
                    pats.append([z, int(rng.integers(0, P)), a, br, 0])
                req_vars.append(z)
        # without a required BGP one OPTIONAL group at most (a second one
        # would be a Cartesian product with the first)
        for g in range(1, int(rng.integers(1, 4 if req_vars else 3))):
            anchor = int(rng.choice(req_vars)) if req_vars else new_var()
            w = new_var()
            pr = int(rng.integers(0, P))
            if rng.random() < 0.5:
                pats.append([anchor, pr, w, br, g])
            else:
                pats.append([w, pr, anchor, br, g])
            if rng.random() < 0.3:  # a second pattern: a filter or another expansion
                other = w if rng.random() < 0.5 else anchor
                pats.append([other, int(rng.integers(0, P)),
                             int(rng.integers(0, V)) if rng.random() < 0.5 else new_var(), br, g])
        for _ in range(int(rng.integers(0, 3))):
            op = int(rng.integers(0, 8))
            a = -int(rng.integers(1, n_vars + 1))
            b = int(rng.integers(0, V)) if rng.random() < 0.3 else -int(rng.integers(1, n_vars + 1))
            filters.append([op, a, b, br])
    return (np.array(pats, np.int32).reshape(-1, 5), np.array(filters, np.int32).reshape(-1, 4),
            n_vars)


@pytest.mark.parametrize("seed", range(6))
def test_ext_random_graphs(G, A, seed):
    rng = np.random.default_rng(7100 + seed)
    V = int(rng.integers(5, 3000))
    P = int(rng.integers(1, 5))
    n = int(rng.integers(10, 30000))
    s, p, o = (rng.integers(0, V, n).astype(np.int32), rng.integers(0, P, n).astype(np.int32),
               rng.integers(0, V, n).astype(np.int32))
    st = G.gsmat_load_triples(s, p, o, V, P)
    G.gsmat_build_index(st, dense_div=int(rng.choice([1, 32, 10**6])))
    done, rows = 0, 0
    while done < 20:
        pats, filters, nv = _random_query(rng, V, P, (s, p, o))
        if nv > 31 or len(pats) + len(filters) == 0:
            continue  # too wide, or an empty query (EINVAL)
        try:
            want_n = len(A.join_ext(s, p, o, pats, filters, nv, cap_rows=100_000))
        except ValueError:
            continue
        if want_n > 100_000:
            continue
        rows += _check(G, A, st, (s, p, o), pats, filters, nv)
        done += 1
    print(f"[gpu] ext random seed={seed} V={V} P={P} n={n}: 20 queries, {rows} rows", flush=True)
    st.close()


def _chain_graph(V=120_000, seed=3):
    """p0: most vertices one successor; p1: about half two or three objects;
    p2: a tenth one object.  Tables of tens of thousands of rows: many
    tiles, a ragged tail, OPTIONAL groups that match some rows."""
    rng = np.random.default_rng(seed)
    s, p, o = [], [], []
    src = rng.choice(V, int(V * 0.9), replace=False)
    s.append(src); p.append(np.zeros(len(src), np.int32)); o.append(rng.integers(0, V, len(src)))
    half = rng.choice(V, V // 2, replace=False)
    reps = rng.integers(2, 4, len(half))
    s.append(np.repeat(half, reps)); p.append(np.ones(int(reps.sum()), np.int32))
    o.append(rng.integers(0, V, int(reps.sum())))
    tenth = rng.choice(V, V // 10, replace=False)
    s.append(tenth); p.append(np.full(len(tenth), 2, np.int32)); o.append(rng.integers(0, 50, len(tenth)))
    return (np.concatenate(s).astype(np.int32), np.concatenate(p).astype(np.int32),
            np.concatenate(o).astype(np.int32), V)


@pytest.fixture(scope="module")
def chain(G):
    s, p, o, V = _chain_graph()
    st = G.gsmat_load_triples(s, p, o, V, 3)
    G.gsmat_build_index(st)
    yield st, (s, p, o)
    st.close()


CHAIN_QUERIES = [
    # ?x p0 ?y OPTIONAL { ?y p1 ?z }
    ([[-1, 0, -2, 0, 0], [-2, 1, -3, 0, 1]], []),
    # ... OPTIONAL { ?y p2 ?w } OPTIONAL { ?x p1 ?z }: two groups, both partial
    ([[-1, 0, -2, 0, 0], [-2, 2, -4, 0, 1], [-1, 1, -3, 0, 2]], []),
    # an OPTIONAL of two patterns (a path), then FILTER(BOUND(?w))
    ([[-1, 0, -2, 0, 0], [-2, 1, -3, 0, 1], [-3, 2, -4, 0, 1]], [[6, -4, 0, 0]]),
    # FILTER(!BOUND(?z)): the rows with no partner
    ([[-1, 0, -2, 0, 0], [-2, 1, -3, 0, 1]], [[7, -3, 0, 0]]),
    # FILTER(?x < ?y) and FILTER(?z != 17) over an OPTIONAL
    ([[-1, 0, -2, 0, 0], [-2, 1, -3, 0, 1]], [[2, -1, -2, 0], [1, -3, 17, 0]]),
    # UNION of the two directions, a constant in an OPTIONAL
    ([[-1, 0, -2, 0, 0], [-2, 2, 7, 0, 1], [-2, 1, -1, 1, 0], [-1, 2, -3, 1, 1]], []),
    # an OPTIONAL that always matches (the required pattern again): the inner join
    ([[-1, 1, -2, 0, 0], [-1, 1, -2, 0, 1]], []),
    # an OPTIONAL over a constant object that matches a few rows
    ([[-1, 2, -2, 0, 0], [-1, 0, -3, 0, 1], [-3, 2, 3, 0, 1]], [[4, -1, 100, 0]]),
]


@pytest.mark.parametrize("qi", range(len(CHAIN_QUERIES)))
def test_ext_many_tiles(G, A, chain, qi):
    st, spo = chain
    pats, filters = CHAIN_QUERIES[qi]
    nv = int(-min(np.min(np.asarray(pats)[:, [0, 2]]), 0))
    n = _check(G, A, st, spo, pats, filters, nv)
    print(f"[gpu] ext many tiles q{qi}: {n} rows", flush=True)
    assert n > 2048 or qi == 7
    # chunked steps (a budget of 3000 rows of the widest table) give the same rows
    _check(G, A, st, spo, pats, filters, nv, budget_bytes=4 * 5 * 3000)


def test_ext_edge_cases(G, A, chain):
    st, spo = chain
    s, p, o = spo
    # empty required result: nothing, whatever the OPTIONAL
    assert _check(G, A, st, spo, [[-1, 0, 5_000_000, 0, 0], [-1, 1, -2, 0, 1]], [], 2) == 0
    # an OPTIONAL over an absent predicate keeps every row, unbound
    got = _run(G, st, [[-1, 2, -2, 0, 0], [-1, 9, -3, 0, 1]], [], 3)
    assert len(got) == int((p == 2).sum()) and (got[:, 2] == -1).all()
    # no required BGP: the OPTIONAL's own rows (or one unbound row when it has none)
    _check(G, A, st, spo, [[-1, 2, 3, 0, 1]], [], 1)
    assert _run(G, st, [[-1, 2, 5_000_000, 0, 1]], [], 1).tolist() == [[-1]]
    # a filter-only branch: one unbound row if the filter holds
    assert _run(G, st, [], [[7, -1, 0, 0]], 1).tolist() == [[-1]]
    assert _run(G, st, [], [[6, -1, 0, 0]], 1).shape == (0, 1)
    # a variable that no branch binds comes back unbound
    got = _run(G, st, [[-1, 2, -2, 0, 0]], [], 3)
    assert (got[:, 2] == -1).all()
    # n_vars 0: yes/no queries
    for tp, want in (([int(s[0]), int(p[0]), int(o[0])], 1), ([int(s[0]), 2, 99], 0)):
        if want == 0:
            assert not ((s == tp[0]) & (p == 2) & (o == 99)).any()
        r = G.gsmat_join_ext(st, [tp + [0, 0]], [], 0)
        assert G.gsmat_result_info(r)["rows"] == want
        r.close()
    # branches come in branch order
    got = _run(G, st, [[-1, 2, -2, 1, 0], [-3, 2, -4, 0, 0]], [], 4)
    k = int((p == 2).sum())
    assert (got[:k, :2] == -1).all() and (got[k:, 2:] == -1).all()
    # max_rows bounds the result
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_join_ext(st, [[-1, 0, -2, 0, 0], [-2, 1, -3, 0, 1]], [], 3, max_rows=1000)
    assert e.value.status == G.GSMAT_ETOOBIG
    # not well designed
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_join_ext(st, [[-1, 0, -2, 0, 0], [-2, 1, -3, 0, 1], [-3, 1, -1, 0, 2]], [], 3)
    assert e.value.status == G.GSMAT_EUNSUPPORTED
