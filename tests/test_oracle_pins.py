"""Pins for the CPU oracle: values the paper prints, closed forms, brute force.

None of these compare the oracle with itself: every expected value is either
printed in the paper (fixtures under tests/golden/, each citing its source),
derived by enumeration of all assignments, or a textbook closed form computed
with scipy's sparse integer products.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def ex():
    g = _load("worked_example.json")
    spo = np.array(g["cube_spo"], np.int32)
    g["s"], g["p"], g["o"] = spo[:, 0], spo[:, 1], spo[:, 2]
    return g


def sorted_rows(a):
    a = np.asarray(a, np.int64)
    if a.size == 0:
        return a.reshape(0, a.shape[1] if a.ndim == 2 else 0)
    return a[np.lexsort(a.T[::-1])]


# ---------------------------------------------------------------- worked example
def test_worked_example_answer(ex):
    # Sec. 6.3: the single answer (1,3,6,4) in plan schema (X,W,Z,Y), i.e.
    # (x,y,z,w) = (1,4,6,3), decoded to (A, l2, C, B).
    got = O.join(ex["s"], ex["p"], ex["o"], ex["query_tps"], 4)
    assert got.tolist() == ex["answer_xyzw"]
    perm = [ex["query_vars"].index(v) for v in ex["answer_paper_schema"]]
    assert got[0, perm].tolist() == ex["answer_paper_row"]
    names = {v: k for k, v in ex["vertices"].items()}
    assert [names[v] for v in got[0, perm].tolist()] == ex["answer_decoded"]


def test_worked_example_brute_force(ex):
    bf = O.brute_force(ex["s"], ex["p"], ex["o"], ex["query_tps"], 4, ex["n_vertices"])
    assert bf.tolist() == ex["answer_xyzw"]


def test_worked_example_intermediate(ex):
    # C = (?X likes ?W) join (?Z likes ?W) in schema (X, W, Z); the paper prints
    # the row (1,2,1); enumeration gives all rows.
    tps = [[-1, 1, -2], [-3, 1, -2]]  # x=0, w=1, z=2
    got = O.join(ex["s"], ex["p"], ex["o"], tps, 3)
    bf = O.brute_force(ex["s"], ex["p"], ex["o"], tps, 3, ex["n_vertices"])
    assert got.tolist() == bf.tolist()
    assert ex["intermediate_C_printed_row"] in got.tolist()
    assert len(got) == 5


def test_worked_example_matrices(ex):
    for h, pairs in ex["matrices"].items():
        keys, ptr, nbr = O.csr(ex["s"], ex["p"], ex["o"], int(h), 0)
        got = [[int(keys[r]), int(nbr[j])] for r in range(len(keys)) for j in range(ptr[r], ptr[r + 1])]
        assert got == pairs, h
    total = sum(len(v) for v in ex["matrices"].values())
    assert 2 * total == ex["storage_units"]
    assert 7 * 7 * 3 == ex["adjacency_units"]


def test_worked_example_aux_arrays(ex):
    keys, ptr, nbr = O.csr(ex["s"], ex["p"], ex["o"], ex["predicates"]["likes"], 0)
    assert keys.tolist() == ex["aux_A_X"]["Row"]
    assert np.diff(ptr).tolist() == ex["aux_A_X"]["Num"]
    assert (ptr[:-1] + 1).tolist() == ex["aux_A_X"]["Rpos_1based"]
    keys, ptr, nbr = O.csr(ex["s"], ex["p"], ex["o"], ex["predicates"]["likes"], 1)
    first = ex["aux_B_W_first"]
    assert (int(keys[0]), int(ptr[1] - ptr[0]), int(ptr[0] + 1)) == (
        first["Row"], first["Num"], first["Rpos_1based"])


def test_worked_example_column_compressed(ex):
    # Sec. 6.3 prints the first entry of B(W), the likes matrix keyed by its
    # object; the fixture holds both entries and the column-compressed
    # M_1..M_3 derived by transposing the printed matrices
    for h, want in ex["csc"].items():
        keys, ptr, nbr = O.csr(ex["s"], ex["p"], ex["o"], int(h), 1)
        assert keys.tolist() == want["col_ids"], h
        assert ptr.tolist() == want["ptr"], h
        assert nbr.tolist() == want["rows"], h
    keys, ptr, nbr = O.csr(ex["s"], ex["p"], ex["o"], ex["predicates"]["likes"], 1)
    bw = ex["aux_B_W"]
    assert keys.tolist() == bw["Row"]
    assert np.diff(ptr).tolist() == bw["Num"]
    assert (ptr[:-1] + 1).tolist() == bw["Rpos_1based"]
    assert (bw["Row"][0], bw["Num"][0], bw["Rpos_1based"][0]) == (
        ex["aux_B_W_first"]["Row"], ex["aux_B_W_first"]["Num"], ex["aux_B_W_first"]["Rpos_1based"])
    # the two orientations hold the same pairs
    for h, pairs in ex["matrices"].items():
        keys, ptr, nbr = O.csr(ex["s"], ex["p"], ex["o"], int(h), 1)
        t = sorted([int(nbr[j]), int(keys[r])] for r in range(len(keys))
                   for j in range(ptr[r], ptr[r + 1]))
        assert t == sorted(pairs), h


def test_worked_example_plan(ex):
    nnz = {int(h): len(v) for h, v in ex["matrices"].items()}
    stat = [nnz[t[1]] for t in ex["query_tps"]]
    assert O.plan_order(ex["query_tps"], stat) == ex["paper_plan_order"]


# ---------------------------------------------------------------- SpGEMM example
def test_spgemm_example_join_and_product():
    g = _load("spgemm_example.json")
    ids = g["ids"]
    pa, pb = 0, 1
    s = [ids[a] for a, _ in g["A"]] + [ids[a] for a, _ in g["B"]]
    o = [ids[b] for _, b in g["A"]] + [ids[b] for _, b in g["B"]]
    p = [pa] * len(g["A"]) + [pb] * len(g["B"])
    got = O.join(s, p, o, [[-1, pa, -2], [-2, pb, -3]], 3)
    want = sorted_rows([[ids[a], ids[b], ids[c]] for a, b, c in g["join_rows"]])
    assert got.tolist() == want.tolist()
    n = len(ids)
    A = sp.csr_matrix((np.ones(len(g["A"]), np.int64), ([ids[a] for a, _ in g["A"]], [ids[b] for _, b in g["A"]])), shape=(n, n))
    B = sp.csr_matrix((np.ones(len(g["B"]), np.int64), ([ids[a] for a, _ in g["B"]], [ids[b] for _, b in g["B"]])), shape=(n, n))
    C = (A @ B).tocoo()
    prod = sorted((int(r), int(c), int(v)) for r, c, v in zip(C.row, C.col, C.data))
    assert prod == sorted((ids[a], ids[b], v) for a, b, v in g["C_product"])
    # the join keeps the join column: its size is the sum of the product entries
    assert len(got) == int(C.data.sum())


# ---------------------------------------------------------------- brute force on random toys
def _random_graph(rng, V, P, n):
    s = rng.integers(0, V, n).astype(np.int32)
    p = rng.integers(0, P, n).astype(np.int32)
    o = rng.integers(0, V, n).astype(np.int32)
    return s, p, o


def _random_bgp(rng, V, P, nv, ntp, const_prob=0.2):
    tps = []
    for _ in range(ntp):
        def term():
            if rng.random() < const_prob:
                return int(rng.integers(0, V + 1))  # V: a constant absent from D
            return -int(rng.integers(0, nv)) - 1
        tps.append([term(), int(rng.integers(0, P)), term()])
    used = sorted({-t - 1 for tp in tps for t in (tp[0], tp[2]) if t < 0})
    remap = {x: i for i, x in enumerate(used)}
    tps = [[(-remap[-a - 1] - 1) if a < 0 else a, b, (-remap[-c - 1] - 1) if c < 0 else c]
           for a, b, c in tps]
    return tps, len(used)


@pytest.mark.parametrize("seed", range(40))
def test_oracle_matches_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    V = int(rng.integers(3, 8))
    P = int(rng.integers(1, 4))
    s, p, o = _random_graph(rng, V, P, int(rng.integers(5, 40)))
    ntp = int(rng.integers(1, 5))
    tps, nv = _random_bgp(rng, V, P, int(rng.integers(1, 5)), ntp)
    got = O.join(s, p, o, tps, nv)
    bf = O.brute_force(s, p, o, tps, nv, V + 1)
    assert got.tolist() == bf.tolist(), (tps, nv)


SHAPES = {
    "triangle": ([[-1, 0, -2], [-2, 1, -3], [-3, 0, -1]], 3),
    "self_loop": ([[-1, 0, -1], [-1, 1, -2]], 2),
    "repeated_tp": ([[-1, 0, -2], [-1, 0, -2], [-2, 1, -3]], 3),
    "disconnected": ([[-1, 0, -2], [-3, 1, -4]], 4),
    "all_constant_true": ([[1, 0, 2]], 0),
    "const_subject": ([[1, 0, -1], [-1, 1, -2]], 2),
    "two_cycle": ([[-1, 0, -2], [-2, 0, -1]], 2),
    "object_star": ([[-2, 0, -1], [-3, 1, -1], [-4, 2, -1]], 4),
    "filter_both_bound": ([[-1, 0, -2], [-2, 1, -3], [-1, 2, -3]], 3),
}


@pytest.mark.parametrize("shape", sorted(SHAPES))
def test_oracle_shapes_brute_force(shape):
    tps, nv = SHAPES[shape]
    rng = np.random.default_rng(7)
    V = 6
    s, p, o = _random_graph(rng, V, 3, 60)
    s = np.concatenate([s, [1, 2, 3]]).astype(np.int32)
    p = np.concatenate([p, [0, 0, 0]]).astype(np.int32)
    o = np.concatenate([o, [2, 2, 3]]).astype(np.int32)
    got = O.join(s, p, o, tps, nv)
    bf = O.brute_force(s, p, o, tps, nv, V)
    assert got.tolist() == bf.tolist()
    if shape == "all_constant_true":
        assert got.shape == (1, 0)


@pytest.mark.parametrize("seed", range(12))
def test_multicore_oracle_equals_single_thread(seed):
    """The OpenMP evaluation (the CPU baseline's multi-core form) gives the
    single-threaded oracle's rows, on brute-force-sized toys and on larger
    random graphs, every shape, and any thread count; an intermediate above
    the row cap is refused by both."""
    rng = np.random.default_rng(3000 + seed)
    if seed < 6:
        V, P, n = int(rng.integers(3, 8)), int(rng.integers(1, 4)), int(rng.integers(5, 40))
    else:
        V, P, n = int(rng.integers(50, 400)), int(rng.integers(1, 5)), int(rng.integers(500, 8000))
    s, p, o = _random_graph(rng, V, P, n)
    ds = O.Dataset(s, p, o)
    cases = [_random_bgp(rng, V, P, int(rng.integers(1, 5)), int(rng.integers(1, 5)))
             for _ in range(6)] + list(SHAPES.values())
    for tps, nv in cases:
        try:
            want = ds.join(tps, nv, cap_rows=200_000)
        except ValueError:
            want = None
        for threads in (1, 2, 7):
            if want is None:
                with pytest.raises(ValueError):
                    ds.join_omp(tps, nv, threads, cap_rows=200_000)
            else:
                got = ds.join_omp(tps, nv, threads, cap_rows=200_000)
                assert got.tolist() == want.tolist(), (tps, nv, threads)
    ds.close()


def test_set_semantics_duplicates_removed():
    rng = np.random.default_rng(3)
    s, p, o = _random_graph(rng, 5, 2, 30)
    tps = [[-1, 0, -2], [-2, 1, -3]]
    a = O.join(s, p, o, tps, 3)
    b = O.join(np.tile(s, 3), np.tile(p, 3), np.tile(o, 3), tps, 3)
    assert a.tolist() == b.tolist()
    d = O.dedupe(np.tile(s, 2), np.tile(p, 2), np.tile(o, 2))
    assert len(d[0]) == len(set(zip(s.tolist(), p.tolist(), o.tolist())))


def test_permutation_invariance():
    rng = np.random.default_rng(5)
    s, p, o = _random_graph(rng, 30, 3, 400)
    tps = [[-1, 0, -2], [-2, 1, -3], [-1, 2, -4], [-3, 0, -4]]
    base = O.join(s, p, o, tps, 4)
    for perm in ([3, 2, 1, 0], [1, 3, 0, 2], [2, 0, 3, 1]):
        assert O.join(s, p, o, [tps[i] for i in perm], 4).tolist() == base.tolist()


def test_fingerprint_matches_rows():
    rng = np.random.default_rng(9)
    s, p, o = _random_graph(rng, 40, 2, 800)
    tps = [[-1, 0, -2], [-2, 1, -3]]
    rows = O.join(s, p, o, tps, 3)
    assert O.join(s, p, o, tps, 3, fingerprint=True) == O.fingerprint_rows(rows)
    # fingerprint is order independent
    assert O.fingerprint_rows(rows[::-1]) == O.fingerprint_rows(rows)


def test_fingerprint_finaliser_is_splitmix64():
    # the row hashes chain the SplitMix64 finaliser: its outputs over the
    # generator's state sequence are the published ones
    g = _load("splitmix64.json")
    gamma = int(g["gamma"], 16)
    M = (1 << 64) - 1
    for seed, want in ((0, [int(x, 16) for x in g["seed_0_hex"]]), (1234567, g["seed_1234567"])):
        st = seed
        got = []
        for _ in want:
            st = (st + gamma) & M
            got.append(O.mix64(st))
        assert got == want, seed


def test_fingerprint_discriminates_row_multisets():
    # the fingerprint must change under every plausible parity mistake: a
    # changed value, two values swapped inside a row, a duplicated row, a
    # dropped row, a row replaced by another answer (same count)
    rng = np.random.default_rng(11)
    s, p, o = _random_graph(rng, 60, 2, 1500)
    rows = O.join(s, p, o, [[-1, 0, -2], [-2, 1, -3]], 3)
    assert len(rows) > 100
    base = O.fingerprint_rows_c(rows)
    assert base == O.fingerprint_rows(rows) == O.join(s, p, o, [[-1, 0, -2], [-2, 1, -3]], 3,
                                                       fingerprint=True)
    variants = {}
    r = rows.copy(); r[17, 1] += 1; variants["value"] = r
    i = int(np.flatnonzero(rows[:, 0] != rows[:, 2])[0])
    r = rows.copy(); r[i, [0, 2]] = r[i, [2, 0]]; variants["swap"] = r
    variants["duplicate"] = np.concatenate([rows, rows[5:6]])
    variants["drop"] = rows[1:]
    r = rows.copy(); r[3] = r[4]; variants["replace"] = r
    for name, v in variants.items():
        assert O.fingerprint_rows_c(v) != base, name
        assert O.fingerprint_rows(v) != base, name
    # and must not change with the row order
    perm = rng.permutation(len(rows))
    assert O.fingerprint_rows_c(rows[perm]) == base


def test_hash_partition_covers_rows_once():
    # the 1/64 partition compare: the partitions over all residues are
    # disjoint, cover every row, and the Python selection of GPU rows picks
    # the rows the C oracle returns for the same residue
    rng = np.random.default_rng(13)
    s, p, o = _random_graph(rng, 80, 2, 3000)
    tps = [[-1, 0, -2], [-2, 1, -3]]
    rows = O.join(s, p, o, tps, 3)
    parts = []
    for res in range(64):
        fp, part = O.join(s, p, o, tps, 3, partition=(64, res))
        assert fp == O.fingerprint_rows_c(rows)
        assert np.array_equal(part, O.partition_rows(rows[::-1], 64, res)), res
        parts.append(part)
    allp = np.concatenate(parts)
    assert len(allp) == len(rows)
    assert np.array_equal(allp[np.lexsort(allp.T[::-1])], rows)


# ---------------------------------------------------------------- closed forms on a power-law graph
@pytest.fixture(scope="module")
def tiny():
    import workload as W
    spec, (s, p, o), gi, qs = W.make_workload("tiny")
    return spec, s, p, o, gi, qs


def _adj(s, p, o, pred, V):
    m = p == pred
    return sp.csr_matrix((np.ones(int(m.sum()), np.int64), (s[m], o[m])), shape=(V, V))


def test_closed_form_two_chain(tiny):
    spec, s, p, o, gi, qs = tiny
    V = spec.V
    for p1, p2 in [(0, 1), (3, 3), (1, 7), (15, 0)]:
        A1, A2 = _adj(s, p, o, p1, V), _adj(s, p, o, p2, V)
        want = int((A1 @ A2).sum())  # 1^T A1 A2 1 = sum_b indeg_p1(b) outdeg_p2(b)
        got = O.join(s, p, o, [[-1, p1, -2], [-2, p2, -3]], 3, fingerprint=True)[0]
        assert got == want


def test_closed_form_subject_star(tiny):
    spec, s, p, o, gi, qs = tiny
    V = spec.V
    for preds in [(2, 5), (4, 6, 9), (11, 12, 13, 14)]:
        deg = [np.bincount(s[p == q], minlength=V).astype(object) for q in preds]
        want = int(np.sum(np.prod(np.stack(deg), axis=0)))
        tps = [[-1, q, -(i + 2)] for i, q in enumerate(preds)]
        got = O.join(s, p, o, tps, len(preds) + 1, fingerprint=True)[0]
        assert got == want


def test_closed_form_constant_object(tiny):
    spec, s, p, o, gi, qs = tiny
    V = spec.V
    c = int(o[0])
    p1, p2 = 0, int(p[0])
    indeg = np.bincount(o[p == p1], minlength=V)
    member = np.zeros(V, bool)
    member[s[(p == p2) & (o == c)]] = True
    want = int(indeg[member].sum())
    got = O.join(s, p, o, [[-1, p1, -2], [-2, p2, c]], 2, fingerprint=True)[0]
    assert got == want


def test_tree_counts_match_generator(tiny):
    # the generator's tree counting program is independent of the oracle
    spec, s, p, o, gi, qs = tiny
    for q in qs:
        rows = O.join(s, p, o, q.tps, q.n_vars)
        assert len(rows) == q.count
        # the walk's witness is an answer (soundness of the generated query)
        assert q.witness.tolist() in rows.tolist()


def test_soundness_every_row_satisfies_every_pattern(tiny):
    spec, s, p, o, gi, qs = tiny
    D = set(zip(s.tolist(), p.tolist(), o.tolist()))
    for q in qs[:6]:
        rows = O.join(s, p, o, q.tps, q.n_vars)
        take = rows[:: max(1, len(rows) // 2000)]
        for r in take.tolist():
            for a, b, c in q.tps.tolist():
                sa = a if a >= 0 else r[-a - 1]
                oc = c if c >= 0 else r[-c - 1]
                assert (sa, b, oc) in D
