"""Text boundary (no GPU): dictionary encoding by order of occurrence, the
BGP parser and decoding, pinned to the paper's worked example (Sec. 5.2
h_p/h_so figure and Table 1; the query of Sec. 3.2; the decoded answer of
Sec. 6.3) and checked on syntax and round trips."""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")

# D_G as text, in the order of the paper's Table 1 (predicates with the
# paper's ':' prefix; l1/l2 are the table's I1/I2, reading 4)
D_G = """A :likes l1 .
A :likes l2 .
A :follows B .
B :related h .
B :follows C .
B :follows D .
C :likes l2 .
C :follows D .
D :related h .
"""


@pytest.fixture(scope="module")
def G():
    import paper_1807_07691_amd as G
    return G


@pytest.fixture(scope="module")
def gold():
    with open(os.path.join(GOLD, "worked_example.json")) as f:
        return json.load(f)


def test_codes_follow_order_of_occurrence(G, gold):
    d = G.gsmat_dict_new()
    s, p, o = G.gsmat_dict_load_text(d, D_G)
    # the paper's codes are 1-based; the dictionary's 0-based
    for name, code in gold["vertices"].items():
        assert G.gsmat_dict_lookup(d, name) == code - 1, name
    for name, code in gold["predicates"].items():
        assert G.gsmat_dict_lookup(d, ":" + name, True) == code - 1, name
    cube = np.stack([s, p, o], 1)
    assert cube.tolist() == (np.array(gold["cube_spo"]) - 1).tolist()
    assert G.gsmat_dict_sizes(d) == (7, 3)


def test_query_text_and_decoded_answer(G, gold):
    d = G.gsmat_dict_new()
    s, p, o = G.gsmat_dict_load_text(d, D_G)
    text = gold["query_text"].replace("follows", ":follows").replace("likes", ":likes")
    tps, names = G.gsmat_parse_bgp(d, text)
    want = np.array(gold["query_tps"])
    want[:, 1] -= 1
    assert tps.tolist() == want.tolist()
    assert names == gold["query_vars"]
    rows = O.join(s, p, o, tps, len(names))
    assert rows.tolist() == (np.array(gold["answer_xyzw"]) - 1).tolist()
    # the paper prints (1,3,6,4) in its plan's schema (x, w, z, y) and decodes
    # it to (A, I2, C, B)
    paper_row = [c - 1 for c in gold["answer_paper_row"]]
    assert [G.gsmat_dict_term(d, c) for c in paper_row] == gold["answer_decoded"]


def test_select_form_constants_and_unknown_terms(G):
    d = G.gsmat_dict_new()
    G.gsmat_dict_load_text(d, D_G)
    tps, names = G.gsmat_parse_bgp(
        d, "SELECT ?a WHERE {\n ?a :follows $b . # comment\n $b :related h }")
    assert names == ["a", "b"]
    assert tps.tolist() == [[-1, 1, -2], [-2, 2, 4]]
    tps, names = G.gsmat_parse_bgp(d, "?a :knows Zed .")
    assert tps.tolist() == [[-1, 3, 7]]  # unseen: one past the last code, matches nothing
    assert G.gsmat_dict_sizes(d) == (7, 3)  # parsing adds no terms
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_parse_bgp(d, "?a ?p ?b")
    assert e.value.status == G.GSMAT_EUNSUPPORTED
    for bad in ("?a :likes", "SELECT ?a WHERE ?a :likes ?b", "?a :likes . ?b"):
        with pytest.raises(G.GsmatError) as e:
            G.gsmat_parse_bgp(d, bad)
        assert e.value.status == G.GSMAT_EINVAL, bad


def test_term_syntax(G):
    d = G.gsmat_dict_new()
    text = ('<http://x/a> <http://x/p> "a literal with \\"quotes\\" . inside"@en .\n'
            '_:b1 <http://x/p> "42"^^<http://www.w3.org/2001/XMLSchema#integer> .\n'
            '# a comment line\n'
            '\n'
            '<http://x/a> <http://x/q> _:b1\n'
            'ex:c ex:r <http://x/a> . # trailing comment\n')
    s, p, o = G.gsmat_dict_load_text(d, text)
    assert len(s) == 4
    terms = [G.gsmat_dict_term(d, c) for c in range(G.gsmat_dict_sizes(d)[0])]
    assert terms == ['<http://x/a>', '"a literal with \\"quotes\\" . inside"@en', '_:b1',
                     '"42"^^<http://www.w3.org/2001/XMLSchema#integer>', 'ex:c']
    assert [G.gsmat_dict_term(d, c, True) for c in range(3)] == [
        '<http://x/p>', '<http://x/q>', 'ex:r']
    assert np.stack([s, p, o], 1).tolist() == [[0, 0, 1], [2, 0, 3], [0, 1, 2], [4, 2, 0]]


def test_syntax_errors_leave_the_dictionary_unchanged(G):
    d = G.gsmat_dict_new()
    G.gsmat_dict_load_text(d, D_G)
    for bad, line in (("A :likes\n", 1), ("A :likes l1 l2 .\n", 1), ('A :p "open\n', 1),
                      ("A :p <open\n", 1), ("A :p B .\nC :q\n", 2), ("?x :p B .\n", 1)):
        with pytest.raises(G.GsmatError) as e:
            G.gsmat_dict_load_text(d, bad)
        assert e.value.status == G.GSMAT_EINVAL
        assert f"line {line}" in str(e.value), (bad, str(e.value))
    assert G.gsmat_dict_sizes(d) == (7, 3)
    with pytest.raises(G.GsmatError):
        G.gsmat_dict_term(d, 7)


@pytest.mark.parametrize("seed", range(5))
def test_codes_are_first_occurrence_bijections(G, seed):
    """Against a plain Python first-occurrence numbering, over two loads (codes
    continue), with repeated terms and a predicate also used as a subject."""
    rng = np.random.default_rng(seed)
    pool = [f"<http://e/{i}>" for i in range(60)] + [f'"lit {i}"' for i in range(20)]
    preds = [f"<http://p/{i}>" for i in range(7)] + ["<http://e/3>"]
    d = G.gsmat_dict_new()
    so, pc = {}, {}
    for part in range(2):
        lines = []
        want = []
        for _ in range(int(rng.integers(1, 200))):
            a, b, c = (pool[int(rng.integers(0, 60))], preds[int(rng.integers(0, 8))],
                       pool[int(rng.integers(0, 80))])
            lines.append(f"{a} {b} {c} .")
            want.append((so.setdefault(a, len(so)), pc.setdefault(b, len(pc)),
                         so.setdefault(c, len(so))))
        s, p, o = G.gsmat_dict_load_text(d, "\n".join(lines))
        assert list(zip(s.tolist(), p.tolist(), o.tolist())) == want
    assert G.gsmat_dict_sizes(d) == (len(so), len(pc))
    for t, c in so.items():
        assert G.gsmat_dict_term(d, c) == t and G.gsmat_dict_lookup(d, t) == c
    for t, c in pc.items():
        assert G.gsmat_dict_term(d, c, True) == t and G.gsmat_dict_lookup(d, t, True) == c
