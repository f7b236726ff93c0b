"""Serving parity: queries submitted to the continuous-batching server at
different rounds (joining queries already running) yield exactly the rows, in
the same order, and the per-step counts they yield alone through gsmat_join,
and the oracle's rows; under tight admission (one slot, a memory budget that
admits one query at a time, rounds that must defer steps) and with failing
and run-alone queries in the mix."""
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


def _alone(G, st, tps, mode, budget=0, max_rows=-1):
    pl = G.gsmat_plan(st, tps, mode)
    try:
        r = G.gsmat_join(st, pl, budget, max_rows)
    except G.GsmatError as e:
        pl.close()
        return None, None, e.status
    try:
        return G.gsmat_fetch_bindings(r), G.gsmat_result_info(r), 0
    finally:
        r.close()
        pl.close()


def _serve(G, st, queries, mode, waves, mem=0, step=0, max_rows=-1, slots=4096):
    """Submits the queries in waves (a list of counts), one server step after
    each wave, then steps until all are polled.  Returns {tag: (rows, info,
    status)} and the largest active count seen."""
    import time
    sv = G.gsmat_server_new(st, mem, step, max_rows, slots)
    got = {}
    seen_active = 0
    nxt = 0
    steps = 0
    t0 = time.perf_counter()
    try:
        for w in list(waves) + [0] * 10_000:
            for _ in range(w):
                if nxt < len(queries):
                    G.gsmat_server_submit(sv, G.gsmat_plan(st, queries[nxt], mode), nxt)
                    nxt += 1
            a, wt, d = G.gsmat_server_step(sv)
            steps += 1
            seen_active = max(seen_active, a)
            assert a <= slots
            for tag, r, status in G.gsmat_server_poll(sv):
                if r is None:
                    got[tag] = (None, None, status)
                else:
                    got[tag] = (G.gsmat_fetch_bindings(r), G.gsmat_result_info(r), status)
                    r.close()
            if nxt == len(queries) and len(got) == len(queries):
                break
        assert len(got) == len(queries)
    finally:
        sv.close()
    print(f"[gpu]   served {len(queries)} queries in {steps} steps, "
          f"{time.perf_counter() - t0:.3f}s", flush=True)
    return got, seen_active


def _check(G, st, queries, mode, got, want=None, budget=0, max_rows=-1):
    import time
    t0 = time.perf_counter()
    _check_rows(G, st, queries, mode, got, want, budget, max_rows)
    print(f"[gpu]   checked {len(queries)} queries in {time.perf_counter() - t0:.3f}s", flush=True)


def _check_rows(G, st, queries, mode, got, want, budget, max_rows):
    for i, tps in enumerate(queries):
        rows, info, status = got[i]
        alone, info1, status1 = _alone(G, st, tps, mode, budget, max_rows)
        assert status == status1, (i, tps)
        if status:
            continue
        assert np.array_equal(rows, alone), (i, tps)
        assert info == info1, (i, tps)
        if want is not None:
            assert np.array_equal(_sorted(rows), want[i]), (i, tps)


@pytest.fixture(scope="module")
def tiny(G, O):
    import workload as W
    spec, (s, p, o), gi, qs = W.make_workload("tiny")
    st = _store(G, s, p, o, spec.V, spec.P)
    # disconnected (a small Cartesian product, runs alone), self loop (runs
    # alone), all constant
    j = len(s) // 2
    extra = [
        np.array([[int(s[0]), int(p[0]), -1], [-2, int(p[j]), int(o[j])]], np.int32),
        np.array([[-1, 2, -1]], np.int32),
        np.array([[int(s[0]), int(p[0]), int(o[0])]], np.int32),
    ]
    queries = [q.tps for q in qs] + extra
    nv = [q.n_vars for q in qs] + [2, 1, 0]
    want = [O.join(s, p, o, t, n) for t, n in zip(queries, nv)]
    return st, queries, want


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_serve_staggered_arrivals(G, tiny, mode):
    st, queries, want = tiny
    print(f"[gpu] serve tiny staggered mode={mode}", flush=True)
    got, _ = _serve(G, st, queries, mode, waves=[3, 0, 2, 1, 1, 0, 4])
    _check(G, st, queries, mode, got, want)


def test_serve_one_slot(G, tiny):
    st, queries, want = tiny
    print("[gpu] serve tiny one slot", flush=True)
    got, seen = _serve(G, st, queries, 2, waves=[len(queries)], slots=1)
    assert seen == 1
    _check(G, st, queries, 2, got, want)


def test_serve_memory_admission_and_deferral(G, tiny):
    """A 1-byte budget admits one query at a time; a 64 KiB budget admits
    several whose rounds overflow it, so later steps wait a round."""
    st, queries, want = tiny
    print("[gpu] serve tiny memory budgets", flush=True)
    got, seen = _serve(G, st, queries, 2, waves=[len(queries)], mem=1)
    assert seen == 1
    _check(G, st, queries, 2, got, want)
    got, _ = _serve(G, st, queries, 2, waves=[len(queries)], mem=64 * 1024)
    _check(G, st, queries, 2, got, want)


def test_serve_step_budget_and_max_rows(G, tiny):
    st, queries, want = tiny
    print("[gpu] serve tiny step budget and max_rows", flush=True)
    step = 4 * 4 * 997  # some steps are chunked alone
    got, _ = _serve(G, st, queries, 2, waves=[2, 2, 2, 2, 2, 2], step=step)
    _check(G, st, queries, 2, got, want, budget=step)
    counts = sorted(len(w) for w in want)
    limit = counts[len(counts) // 2]
    got, _ = _serve(G, st, queries, 2, waves=[len(queries)], max_rows=limit)
    for i, w in enumerate(want):
        assert got[i][2] == (G.GSMAT_ETOOBIG if len(w) > limit else 0), i
    _check(G, st, queries, 2, got, want, max_rows=limit)


@pytest.mark.parametrize("seed", range(4))
def test_serve_random_graphs(G, O, seed):
    rng = np.random.default_rng(1300 + seed)
    V = int(rng.integers(5, 3000))
    P = int(rng.integers(1, 6))
    n = int(rng.integers(10, 40000))
    s, p, o = (rng.integers(0, V, n).astype(np.int32), rng.integers(0, P, n).astype(np.int32),
               rng.integers(0, V, n).astype(np.int32))
    st = _store(G, s, p, o, V, P)
    queries, want = [], []
    while len(queries) < 30:
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
            continue
        queries.append(np.array(tps, np.int32))
        want.append(w)
    waves = [int(x) for x in rng.integers(0, 6, 40)]
    print(f"[gpu] serve random seed={seed} V={V} P={P} n={n}", flush=True)
    for mode in (0, 1, 2):
        got, _ = _serve(G, st, queries, mode, waves=waves)
        _check(G, st, queries, mode, got, want)
