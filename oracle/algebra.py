"""Oracle for queries beyond a single BGP: OPTIONAL, UNION and FILTER.

TEST INFRASTRUCTURE, like the rest of this package: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU baseline leg of ``bench.py`` may use it.

The paper names these three operators as future work (Sec. 9) without
defining them; their meaning here is the SPARQL algebra's over bags of
solution mappings (a mapping is a row over all query variables, -1 where the
variable is unbound):

  * a query is a bag union of branches, taken in ascending branch id;
  * a branch is its required BGP (group 0; absent: the bag holding one empty
    mapping), left-joined with each OPTIONAL BGP (groups 1, 2, ...) in
    ascending group id, then restricted by the conjunction of its FILTERs;
  * LeftJoin(A, B) holds every merge of a row of A with a compatible row of B
    (equal on every variable bound in both) and every row of A that has no
    compatible row in B, alone;
  * a FILTER comparison (=, !=, <, <=, >, >= over term ids) with an unbound
    operand is an error, which a FILTER treats as false; BOUND(?v) and
    !BOUND(?v) test whether ?v is bound.

Each BGP is evaluated by this package's BGP oracle (``join``) after its
variables are renumbered densely; the algebra around it is written out with
plain Python loops and dictionaries (test sizes only).

Encodings (the same as the library's ``gsmat_join_ext``):
  pats    (n, 5) int32: s, p, o, branch, group (terms: id >= 0, variable v as
          -(v + 1));
  filters (m, 4) int32: op, a, b, branch (op one of the F_* codes; a, b terms;
          b unused by BOUND / NOT_BOUND).
"""
from __future__ import annotations

import numpy as np

from . import join

UNBOUND = -1
F_EQ, F_NE, F_LT, F_LE, F_GT, F_GE, F_BOUND, F_NOT_BOUND = range(8)


def _vars_of(tps):
    return sorted({-t - 1 for tp in tps for t in (tp[0], tp[2]) if t < 0})


def bgp_rows(s, p, o, tps, n_vars, cap_rows=-1, bgp=None):
    """Solutions of one BGP as rows over all n_vars variables (-1 where the
    BGP has no such variable); no pattern: one row with every variable
    unbound.  bgp(local_tps, n_local, cap_rows) replaces the oracle join over
    (s, p, o) when given (for instance a prebuilt Dataset's join)."""
    tps = [list(map(int, t)) for t in tps]
    if not tps:
        return np.full((1, n_vars), UNBOUND, np.int32)
    used = _vars_of(tps)
    loc = {v: i for i, v in enumerate(used)}

    def rn(t):
        return -loc[-t - 1] - 1 if t < 0 else t

    local = np.array([[rn(a), b, rn(c)] for a, b, c in tps], np.int32)
    if bgp is not None:
        r = bgp(local, len(used), cap_rows)
    else:
        r = join(s, p, o, local, len(used), cap_rows=cap_rows)
    out = np.full((len(r), n_vars), UNBOUND, np.int32)
    for v, i in loc.items():
        out[:, v] = r[:, i]
    return out


def left_join(A, B, b_vars, cap_rows=-1):
    """SPARQL LeftJoin of the row bags A and B; every row of B binds exactly
    b_vars.  Rows of B are indexed by their values on the variables of
    b_vars that a row of A binds (one index per such subset).  ValueError
    once the result holds more than cap_rows rows (cap_rows >= 0)."""
    n_vars = A.shape[1]
    index = {}

    def matches(mask, key):
        if mask not in index:
            d = {}
            for b in B:
                d.setdefault(tuple(int(b[v]) for v in mask), []).append(b)
            index[mask] = d
        return index[mask].get(key, [])

    out = []
    for a in A:
        mask = tuple(v for v in b_vars if a[v] != UNBOUND)
        found = matches(mask, tuple(int(a[v]) for v in mask))
        if found:
            for b in found:
                out.append(np.where(a != UNBOUND, a, b))
        else:
            out.append(a)
        if 0 <= cap_rows < len(out):
            raise ValueError("left join result exceeds cap_rows")
    return np.array(out, np.int32).reshape(len(out), n_vars)


def _term(row, t):
    return int(t) if t >= 0 else int(row[-t - 1])


def filter_ok(row, conds):
    """The conjunction of the FILTER conditions on one row."""
    for op, a, b in conds:
        va = _term(row, a)
        if op == F_BOUND:
            ok = va != UNBOUND
        elif op == F_NOT_BOUND:
            ok = va == UNBOUND
        else:
            vb = _term(row, b)
            if va == UNBOUND or vb == UNBOUND:
                ok = False  # an error: the row is dropped
            elif op == F_EQ:
                ok = va == vb
            elif op == F_NE:
                ok = va != vb
            elif op == F_LT:
                ok = va < vb
            elif op == F_LE:
                ok = va <= vb
            elif op == F_GT:
                ok = va > vb
            elif op == F_GE:
                ok = va >= vb
            else:
                raise ValueError(f"unknown filter op {op}")
        if not ok:
            return False
    return True


def join_ext(s, p, o, pats, filters, n_vars, cap_rows=-1, sort=True):
    """Rows (rows x n_vars int32, -1 unbound) of the query; sorted unless
    sort=False (then in branch order).  ValueError when a BGP's intermediate
    or a left join's result exceeds cap_rows (cap_rows >= 0)."""
    pats = np.asarray(pats, np.int32).reshape(-1, 5)
    filters = np.asarray(filters, np.int32).reshape(-1, 4)
    branches = sorted(set(pats[:, 3].tolist()) | set(filters[:, 3].tolist()))
    parts = []
    for br in branches:
        mine = pats[pats[:, 3] == br]
        groups = sorted(set(mine[:, 4].tolist()) - {0})
        omega = bgp_rows(s, p, o, mine[mine[:, 4] == 0][:, :3], n_vars, cap_rows)
        for g in groups:
            tps = mine[mine[:, 4] == g][:, :3]
            omega = left_join(omega, bgp_rows(s, p, o, tps, n_vars, cap_rows), _vars_of(tps),
                              cap_rows)
        conds = [tuple(map(int, f[:3])) for f in filters if f[3] == br]
        if conds:
            keep = [i for i, row in enumerate(omega) if filter_ok(row, conds)]
            omega = omega[keep]
        parts.append(omega)
    out = (np.concatenate(parts) if parts else np.zeros((0, n_vars), np.int32)).astype(np.int32)
    if sort and len(out) and n_vars:
        out = out[np.lexsort(out.T[::-1])]
    return out


def join_ext_wd(bgp, pats, filters, n_vars, cap_rows=-1):
    """The answer of join_ext for well-designed queries (every variable an
    OPTIONAL group shares with the rest of its branch occurs in the required
    BGP), computed from inner joins: for each OPTIONAL group g, the BGP
    required + g is joined by bgp(local_tps, n_local, cap_rows) and its rows
    are grouped by their required values; a required row r then takes, group
    after group, every merge with its extensions, or stays as it is when it
    has none (what LeftJoin keeps when the shared variables are all bound).
    Suited to large triple sets, where a group's own relation is too big for
    the left join's index."""
    pats = np.asarray(pats, np.int32).reshape(-1, 5)
    filters = np.asarray(filters, np.int32).reshape(-1, 4)
    branches = sorted(set(pats[:, 3].tolist()) | set(filters[:, 3].tolist()))
    parts = []
    for br in branches:
        mine = pats[pats[:, 3] == br]
        req = [list(map(int, t)) for t in mine[mine[:, 4] == 0][:, :3]]
        req_vars = _vars_of(req)
        base = bgp_rows(None, None, None, req, n_vars, cap_rows, bgp=bgp)
        ext = []
        for g in sorted(set(mine[:, 4].tolist()) - {0}):
            both = req + [list(map(int, t)) for t in mine[mine[:, 4] == g][:, :3]]
            index = {}
            for row in bgp_rows(None, None, None, both, n_vars, cap_rows, bgp=bgp):
                index.setdefault(tuple(int(row[v]) for v in req_vars), []).append(row)
            ext.append(index)
        conds = [tuple(map(int, f[:3])) for f in filters if f[3] == br]
        out = []
        for r in base:
            key = tuple(int(r[v]) for v in req_vars)
            rows = [r]
            for index in ext:
                e = index.get(key)
                if e:
                    rows = [np.where(a != UNBOUND, a, b) for a in rows for b in e]
                if 0 <= cap_rows < len(out) + len(rows):
                    raise ValueError("result exceeds cap_rows")
            out += [x for x in rows if not conds or filter_ok(x, conds)]
        parts.append(np.array(out, np.int32).reshape(len(out), n_vars))
    out = np.concatenate(parts) if parts else np.zeros((0, n_vars), np.int32)
    if len(out) and n_vars:
        out = out[np.lexsort(out.T[::-1])]
    return out
