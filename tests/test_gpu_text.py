"""Text end to end on the GPU: text triples -> dictionary codes -> device
store; query text -> patterns -> join -> decoded rows, against the paper's
worked example and against the oracle on random text data."""
import numpy as np
import pytest

from test_dict import D_G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1807_07691_amd as G
    return G


def _sorted(a):
    a = np.asarray(a)
    if a.ndim != 2 or len(a) == 0 or a.shape[1] == 0:
        return a
    return a[np.lexsort(a.T[::-1])]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_worked_example_from_text(G, mode):
    d = G.gsmat_dict_new()
    s, p, o = G.gsmat_dict_load_text(d, D_G)
    nv, npred = G.gsmat_dict_sizes(d)
    st = G.gsmat_load_triples(s, p, o, nv, npred)
    G.gsmat_build_index(st)
    tps, names = G.gsmat_parse_bgp(
        d, "SELECT * WHERE { ?x :follows ?y . ?y :follows ?z . ?x :likes ?w . ?z :likes ?w }")
    rows = G.evaluate(st, tps, mode)
    decoded = [[G.gsmat_dict_term(d, c) for c in r] for r in rows.tolist()]
    assert names == ["x", "y", "z", "w"]
    assert decoded == [["A", "B", "C", "l2"]]


@pytest.mark.parametrize("seed", range(3))
def test_random_text_against_oracle(G, seed):
    import oracle as O
    rng = np.random.default_rng(2100 + seed)
    ents = [f"<http://e/{i}>" for i in range(400)] + [f'"v{i}"@en' for i in range(50)]
    preds = [f"<http://p/{i}>" for i in range(6)]
    lines = [f"{ents[int(rng.integers(0, 400))]} {preds[int(rng.integers(0, 6))]} "
             f"{ents[int(rng.integers(0, 450))]} ." for _ in range(5000)]
    d = G.gsmat_dict_new()
    s, p, o = G.gsmat_dict_load_text(d, "\n".join(lines))
    nv, npred = G.gsmat_dict_sizes(d)
    st = G.gsmat_load_triples(s, p, o, nv, npred)
    G.gsmat_build_index(st)
    queries = [
        f"?a {preds[0]} ?b . ?b {preds[1]} ?c",
        f"?a {preds[2]} ?b . ?a {preds[3]} ?c . ?a {preds[4]} ?d",
        f"SELECT ?x WHERE {{ ?x {preds[5]} {ents[7]} . ?x {preds[0]} ?y }}",
        f"?a {preds[1]} ?b . ?b {preds[1]} ?a",
        f"?a <http://p/none> ?b",
    ]
    for q in queries:
        tps, names = G.gsmat_parse_bgp(d, q)
        want = O.join(s, p, o, tps, len(names))
        got = _sorted(G.evaluate(st, tps, G.PLAN_ADAPTIVE))
        assert np.array_equal(got, want), q
        for r in got[:20].tolist():  # decoding is the inverse of the coding
            assert [G.gsmat_dict_lookup(d, G.gsmat_dict_term(d, c)) for c in r] == r
