"""The allocation-free join (gsmat_join_noalloc) against gsmat_join: the same
rows in the same order, on two calls in a row (the second with a smaller
result, so stale contents of the shared device array would show), its error
paths (a result above out_cap, intermediates above the 64 MiB array) and a
correct call after each error."""
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
def tiny(G):
    import workload as W
    spec, (s, p, o), gi, qs = W.make_workload("tiny")
    gi.close()
    st = G.gsmat_load_triples(s, p, o, spec.V, spec.P)
    G.gsmat_build_index(st)
    yield qs, st
    st.close()


def _plain(G, st, pl):
    r = G.gsmat_join(st, pl)
    try:
        return G.gsmat_fetch_bindings(r)
    finally:
        r.close()


def _noalloc(G, st, pl, n_vars, cap):
    import torch
    out = torch.full((max(n_vars, 1), cap), -7, dtype=torch.int32, device="cuda")
    n = G.gsmat_join_noalloc(st, pl, out.data_ptr(), cap, cap)
    torch.cuda.synchronize()
    cols = out[:n_vars, :n].cpu().numpy()
    # rows past the result were not written
    assert n == cap or bool((out[:n_vars, n:] == -7).all())
    return n, cols.T.copy() if n_vars else np.zeros((n, 0), np.int32)


def test_noalloc_two_calls_match_join(G, tiny):
    qs, st = tiny
    order = sorted(range(len(qs)), key=lambda i: qs[i].count)
    fits = [i for i in order if 10 <= qs[i].count <= 300_000]
    assert len(fits) >= 2
    big, small = fits[-1], fits[0]
    for rep in range(2):
        for i in (big, small):  # the second call has the smaller result
            q = qs[i]
            pl = G.gsmat_plan(st, q.tps, G.PLAN_ADAPTIVE)
            want = _plain(G, st, pl)
            n, got = _noalloc(G, st, pl, q.n_vars, q.count + 5)
            pl.close()
            print(f"[gpu] noalloc q{i} rows={n}", flush=True)
            assert n == q.count == len(want)
            assert np.array_equal(got, want), i


def test_noalloc_errors_then_correct(G, tiny):
    import torch
    qs, st = tiny
    order = sorted(range(len(qs)), key=lambda i: qs[i].count)
    out = torch.empty((8, 4), dtype=torch.int32, device="cuda")
    # a result above out_cap: ETOOBIG with the row count
    q = qs[order[-2]]
    pl = G.gsmat_plan(st, q.tps, G.PLAN_ADAPTIVE)
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_join_noalloc(st, pl, out.data_ptr(), 4, 4)
    assert e.value.status == G.GSMAT_ETOOBIG and e.value.n_rows == q.count
    # out_stride below out_cap: EINVAL before any device work
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_join_noalloc(st, pl, out.data_ptr(), 4, 8)
    assert e.value.status == G.GSMAT_EINVAL
    pl.close()
    # intermediates above the 64 MiB array: ENOMEM naming the limit
    big = qs[order[-1]]
    assert big.count * 4 * big.n_vars > 64 << 20
    pl = G.gsmat_plan(st, big.tps, G.PLAN_ADAPTIVE)
    with pytest.raises(G.GsmatError) as e:
        G.gsmat_join_noalloc(st, pl, out.data_ptr(), 4, 4)
    assert e.value.status == G.GSMAT_ENOMEM and "64 MiB" in str(e.value)
    pl.close()
    # the next call is correct
    q = qs[order[len(order) // 2]]
    pl = G.gsmat_plan(st, q.tps, G.PLAN_ADAPTIVE)
    want = _plain(G, st, pl)
    n, got = _noalloc(G, st, pl, q.n_vars, q.count)
    pl.close()
    print(f"[gpu] noalloc after errors: rows={n}", flush=True)
    assert n == q.count and np.array_equal(got, want)
