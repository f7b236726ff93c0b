"""Pins of the OPTIONAL / UNION / FILTER oracle (oracle/algebra.py) against
the definitions written out a second way: solution mappings as Python dicts
over their own domains, every BGP solved by enumerating all assignments of
its variables, LeftJoin, Union and Filter taken from the SPARQL algebra's
definitions (a comparison with an unbound operand is an error, and a FILTER
drops the row).  Tiny graphs only.  Also special cases with a known answer:
an OPTIONAL that always matches is the inner join, one that never matches
keeps its left side, a union of a query with itself doubles every row."""
import itertools

import numpy as np
import pytest

import oracle as O
from oracle import algebra as A


def _triples(rng, V, P, n):
    return (rng.integers(0, V, n).astype(np.int32), rng.integers(0, P, n).astype(np.int32),
            rng.integers(0, V, n).astype(np.int32))


# ---------------------------------------------------------------- the second way
def _bf_bgp(D, tps, V):
    """Every mapping of the BGP's variables (and only those) that puts each
    pattern's triple in D."""
    vs = sorted({t for tp in tps for t in (tp[0], tp[2]) if t < 0})
    out = []
    for vals in itertools.product(range(V), repeat=len(vs)):
        mu = dict(zip(vs, vals))
        val = lambda t: mu[t] if t < 0 else t
        if all((val(a), b, val(c)) in D for a, b, c in tps):
            out.append(mu)
    return out


def _compatible(m1, m2):
    return all(m1[k] == m2[k] for k in m1.keys() & m2.keys())


def _bf_left_join(L, R):
    out = []
    for m1 in L:
        ext = [{**m1, **m2} for m2 in R if _compatible(m1, m2)]
        out += ext if ext else [m1]
    return out


def _bf_filter(L, conds):
    def ev(mu, op, a, b):
        def val(t):
            if t >= 0:
                return t
            if t not in mu:
                raise LookupError  # unbound: an error
            return mu[t]
        if op == A.F_BOUND:
            return a in mu
        if op == A.F_NOT_BOUND:
            return a not in mu
        try:
            x, y = val(a), val(b)
        except LookupError:
            return False
        return {A.F_EQ: x == y, A.F_NE: x != y, A.F_LT: x < y, A.F_LE: x <= y,
                A.F_GT: x > y, A.F_GE: x >= y}[op]
    return [mu for mu in L if all(ev(mu, *c) for c in conds)]


def _bf_query(s, p, o, pats, filters, n_vars, V):
    D = set(zip(s.tolist(), p.tolist(), o.tolist()))
    branches = sorted({int(x[3]) for x in pats} | {int(f[3]) for f in filters})
    rows = []
    for br in branches:
        mine = [list(map(int, x)) for x in pats if x[3] == br]
        req = [x[:3] for x in mine if x[4] == 0]
        L = _bf_bgp(D, req, V) if req else [{}]
        for g in sorted({x[4] for x in mine} - {0}):
            L = _bf_left_join(L, _bf_bgp(D, [x[:3] for x in mine if x[4] == g], V))
        L = _bf_filter(L, [tuple(map(int, f[:3])) for f in filters if f[3] == br])
        for mu in L:
            rows.append([mu.get(-(v + 1), -1) for v in range(n_vars)])
    out = np.array(rows, np.int32).reshape(len(rows), n_vars)
    return out[np.lexsort(out.T[::-1])] if len(out) and n_vars else out


# ---------------------------------------------------------------- random queries
def _random_query(rng, V, P, n_vars, well_designed):
    n_br = int(rng.integers(1, 3))
    pats, filters = [], []
    for br in range(n_br):
        n_groups = int(rng.integers(1, 4))
        req_vars = set()
        for g in range(n_groups):
            if g == 0 and rng.random() < 0.1:
                continue  # no required BGP: the unit bag
            for _ in range(int(rng.integers(1, 3))):
                def term():
                    if rng.random() < 0.25:
                        return int(rng.integers(0, V))
                    v = int(rng.integers(0, n_vars))
                    if well_designed and g > 0 and rng.random() < 0.5 and req_vars:
                        v = int(rng.choice(sorted(req_vars)))
                    return -(v + 1)
                a, c = term(), term()
                pats.append([a, int(rng.integers(0, P)), c, br, g])
                if g == 0:
                    req_vars |= {-t - 1 for t in (a, c) if t < 0}
        for _ in range(int(rng.integers(0, 3))):
            op = int(rng.integers(0, 8))
            a = -(int(rng.integers(0, n_vars)) + 1)
            b = int(rng.integers(0, V)) if rng.random() < 0.4 else -(int(rng.integers(0, n_vars)) + 1)
            filters.append([op, a, b, br])
    return np.array(pats, np.int32).reshape(-1, 5), np.array(filters, np.int32).reshape(-1, 4)


@pytest.mark.parametrize("seed", range(300))
def test_ext_oracle_matches_mapping_definitions(seed):
    rng = np.random.default_rng(4000 + seed)
    V, P = int(rng.integers(2, 6)), int(rng.integers(1, 3))
    s, p, o = _triples(rng, V, P, int(rng.integers(3, 20)))
    n_vars = int(rng.integers(1, 4))
    pats, filters = _random_query(rng, V, P, n_vars, well_designed=bool(seed % 2))
    got = A.join_ext(s, p, o, pats, filters, n_vars)
    want = _bf_query(s, p, o, pats, filters, n_vars, V)
    assert np.array_equal(got, want), (pats.tolist(), filters.tolist())


def test_optional_special_cases():
    rng = np.random.default_rng(5)
    s, p, o = _triples(rng, 8, 2, 40)
    # an OPTIONAL whose group is implied by the required one is the inner join
    req = [[-1, 0, -2, 0, 0]]
    same = A.join_ext(s, p, o, req + [[-1, 0, -2, 0, 1]], [], 2)
    assert np.array_equal(same, O.join(s, p, o, [[-1, 0, -2]], 2))
    # an OPTIONAL over an absent predicate keeps the left side, unbound
    kept = A.join_ext(s, p, o, req + [[-2, 5, -3, 0, 1]], [], 3)
    base = O.join(s, p, o, [[-1, 0, -2]], 2)
    assert np.array_equal(kept[:, :2], base) and (kept[:, 2] == -1).all()
    # the inner join rows plus the rows with no partner: the two counts add up
    inner = O.join(s, p, o, [[-1, 0, -2], [-2, 1, -3]], 3)
    opt = A.join_ext(s, p, o, req + [[-2, 1, -3, 0, 1]], [], 3)
    lonely = {tuple(r) for r in base} - {tuple(r[:2]) for r in inner}
    assert len(opt) == len(inner) + len(lonely)
    # a union of a query with itself doubles every row
    two = A.join_ext(s, p, o, req + [[-1, 0, -2, 1, 0]], [], 2)
    assert np.array_equal(two, np.repeat(base, 2, axis=0))
    # FILTER(?x != ?x) removes everything; FILTER(?x = ?x) nothing;
    # FILTER(BOUND) of an unbound variable removes everything
    assert len(A.join_ext(s, p, o, req, [[A.F_NE, -1, -1, 0]], 2)) == 0
    assert np.array_equal(A.join_ext(s, p, o, req, [[A.F_EQ, -1, -1, 0]], 2), base)
    assert len(A.join_ext(s, p, o, req, [[A.F_BOUND, -3, 0, 0]], 3)) == 0
    # no required BGP: the unit bag, one row with nothing bound
    unit = A.join_ext(s, p, o, np.zeros((0, 5), np.int32), [[A.F_NOT_BOUND, -1, 0, 0]], 1)
    assert unit.tolist() == [[-1]]


def test_filter_comparisons_by_hand():
    row = np.array([3, -1, 7], np.int32)
    assert A.filter_ok(row, [(A.F_LT, -1, -3)]) and not A.filter_ok(row, [(A.F_GT, -1, -3)])
    assert A.filter_ok(row, [(A.F_LE, -1, 3), (A.F_GE, -1, 3), (A.F_EQ, -1, 3)])
    assert not A.filter_ok(row, [(A.F_NE, -1, 3)])
    # an unbound operand fails every comparison, != included
    for op in (A.F_EQ, A.F_NE, A.F_LT, A.F_LE, A.F_GT, A.F_GE):
        assert not A.filter_ok(row, [(op, -2, 5)])
    assert A.filter_ok(row, [(A.F_NOT_BOUND, -2, 0), (A.F_BOUND, -3, 0)])


@pytest.mark.parametrize("seed", range(150))
def test_inner_join_form_equals_left_join(seed):
    """join_ext_wd (inner joins of required + each OPTIONAL group, grouped by
    the required values) gives join_ext's answer on well-designed queries."""
    rng = np.random.default_rng(9000 + seed)
    V, P = int(rng.integers(2, 7)), int(rng.integers(1, 3))
    s, p, o = _triples(rng, V, P, int(rng.integers(3, 25)))
    n_vars = int(rng.integers(1, 5))
    while True:
        pats, filters = _random_query(rng, V, P, n_vars, well_designed=True)
        ok = True
        for br in set(pats[:, 3].tolist()):
            mine = pats[pats[:, 3] == br]
            req = set(A._vars_of(mine[mine[:, 4] == 0][:, :3]))
            groups = sorted(set(mine[:, 4].tolist()) - {0})
            for g in groups:
                mv = set(A._vars_of(mine[mine[:, 4] == g][:, :3]))
                rest = req.union(*[A._vars_of(mine[mine[:, 4] == h][:, :3]) for h in groups if h != g])
                ok &= not (mv & rest - req)
        if ok:
            break
    bgp = lambda t, nv, cap: O.join(s, p, o, t, nv, cap_rows=cap)  # noqa: E731
    assert np.array_equal(A.join_ext_wd(bgp, pats, filters, n_vars),
                          A.join_ext(s, p, o, pats, filters, n_vars)), (pats.tolist(), filters.tolist())
