// Query planner (host only): orders the triple patterns of a BGP and decides
// how each step is evaluated.
//
// Ordering follows the paper's "connected minimal upper bound" (Sec. 6.2.1,
// Algorithm "Query Plan Generated"): sort the edges by their statistic, start
// with the smallest, then repeatedly take the first edge in sorted order that
// shares a variable with the already bound ones.  The plan's cost estimate is
// the upper bound of Theorem 1: the running product of the relation sizes.
//
// Readings of the text (the printed listing and the prose disagree):
//   * ties in the sort keep the original pattern order;
//   * "a node of e_i in N" means a shared variable; constants do not connect;
//   * with no connected edge left, the first remaining edge is taken
//     (Cartesian step).
// GSMAT_PLAN_DEFAULT adds, without changing the result: constant-only
// patterns first; the start variable of a star is bound by intersecting the
// row (column) id lists of its patterns; among connected patterns, those whose
// endpoints are all bound (filters) go before expansions.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "plan.hpp"

namespace gsmat {

namespace {

inline bool is_var(int32_t t) { return t < 0; }
inline int var_of(int32_t t) { return -t - 1; }

int64_t sat_mul(int64_t a, int64_t b) {
  if (a <= 0 || b <= 0) return 0;
  if (a > INT64_MAX / b) return INT64_MAX;
  return a * b;
}

}  // namespace

gsmat_status validate_patterns(const gsmat_pattern* pats, int32_t n, int32_t* n_vars,
                               std::string* err) {
  if (!pats || n <= 0) {
    *err = "BGP needs at least one pattern";
    return GSMAT_EINVAL;
  }
  if (n > kMaxPats) {
    *err = "BGP has more than 32 patterns";
    return GSMAT_EUNSUPPORTED;
  }
  uint64_t seen = 0;
  int maxv = -1;
  for (int i = 0; i < n; ++i) {
    if (pats[i].p < 0) {
      *err = "variable predicate in pattern " + std::to_string(i) + " is not supported";
      return GSMAT_EUNSUPPORTED;
    }
    for (int32_t t : {pats[i].s, pats[i].o}) {
      if (is_var(t)) {
        int v = var_of(t);
        if (v >= kMaxCols) {
          *err = "variable number " + std::to_string(v) + " exceeds the limit of 32 variables";
          return GSMAT_EUNSUPPORTED;
        }
        seen |= 1ull << v;
        maxv = std::max(maxv, v);
      }
    }
  }
  const int nv = maxv + 1;
  if (nv > 0 && seen != ((nv == 64) ? ~0ull : ((1ull << nv) - 1))) {
    *err = "variables must be numbered densely from 0";
    return GSMAT_EINVAL;
  }
  *n_vars = nv;
  return GSMAT_OK;
}

gsmat_status build_plan(const gsmat_pattern* pats, int32_t n, int32_t mode, const TpStat* st,
                        gsmat_query_plan* out, std::string* err) {
  int32_t nv = 0;
  gsmat_status rc = validate_patterns(pats, n, &nv, err);
  if (rc != GSMAT_OK) return rc;
  if (mode != GSMAT_PLAN_PAPER && mode != GSMAT_PLAN_DEFAULT && mode != GSMAT_PLAN_ADAPTIVE) {
    *err = "unknown plan mode";
    return GSMAT_EINVAL;
  }
  out->pats.assign(pats, pats + n);
  out->n_vars = nv;
  out->mode = mode;
  out->steps.clear();
  out->steps.reserve(n + 1);  // at most one step per pattern, plus an intersection
  if (mode == GSMAT_PLAN_ADAPTIVE) mode = GSMAT_PLAN_DEFAULT;  // same static order

  // stable insertion sort by the statistic (n <= kMaxPats)
  int order[kMaxPats];
  for (int i = 0; i < n; ++i) {
    int j = i;
    for (; j > 0 && st[i].stat < st[order[j - 1]].stat; --j) order[j] = order[j - 1];
    order[j] = i;
  }
  int rem_buf[kMaxPats];  // remaining, in sorted order
  int n_rem = n;
  std::copy(order, order + n, rem_buf);
  const int* const rem = rem_buf;
  uint64_t bound = 0;
  int64_t est = 1;

  auto all_const = [&](int t) { return !is_var(pats[t].s) && !is_var(pats[t].o); };
  auto has_bound_var = [&](int t) {
    return (is_var(pats[t].s) && (bound >> var_of(pats[t].s) & 1)) ||
           (is_var(pats[t].o) && (bound >> var_of(pats[t].o) & 1));
  };
  auto all_bound = [&](int t) {
    return (!is_var(pats[t].s) || (bound >> var_of(pats[t].s) & 1)) &&
           (!is_var(pats[t].o) || (bound >> var_of(pats[t].o) & 1));
  };
  auto bind = [&](int t) {
    if (is_var(pats[t].s)) bound |= 1ull << var_of(pats[t].s);
    if (is_var(pats[t].o)) bound |= 1ull << var_of(pats[t].o);
  };
  auto erase = [&](int t) {
    int i = 0;
    while (rem_buf[i] != t) ++i;
    std::copy(rem_buf + i + 1, rem_buf + n_rem, rem_buf + i);
    --n_rem;
  };
  auto push = [&](int kind, int tp, int orient, int var, uint32_t members) {
    gsmat_step_info s;
    std::memset(&s, 0, sizeof(s));
    s.kind = kind;
    s.tp = tp;
    s.orient = orient;
    s.var = var;
    s.members = members;
    s.est_rows = est;
    out->steps.push_back(s);
  };

  if (mode == GSMAT_PLAN_DEFAULT) {
    // constant-only patterns are a yes/no test; do them first
    for (int i = 0; i < n; ++i) {
      const int t = order[i];
      if (!all_const(t)) continue;
      est = std::min<int64_t>(est, st[t].stat);
      push(GSMAT_STEP_FILTER, t, -1, -1, 0);
      erase(t);
    }
  }

  bool first = true;
  while (n_rem > 0) {
    if (first) {
      first = false;
      const int e1 = rem[0];
      if (mode == GSMAT_PLAN_DEFAULT && !all_const(e1)) {
        // star centre intersection on a variable endpoint of e1
        int best_v = -1;
        int64_t best_est = INT64_MAX;
        uint32_t best_mem = 0;
        for (int32_t term : {pats[e1].s, pats[e1].o}) {
          if (!is_var(term)) continue;
          const int v = var_of(term);
          uint32_t mem = 0;
          int cnt = 0;
          int64_t e = INT64_MAX;
          for (int i = 0; i < n_rem; ++i) {
            const int t = rem[i];
            if (cnt >= kMaxLists) break;
            const bool vs = pats[t].s == term, vo = pats[t].o == term;
            if (vs == vo) continue;  // not incident, or a self loop on v
            mem |= 1u << t;
            ++cnt;
            e = std::min(e, vs ? st[t].rows_s : st[t].rows_o);
          }
          if (cnt >= 2 && e < best_est) {
            best_est = e;
            best_v = v;
            best_mem = mem;
          }
        }
        if (best_v >= 0) {
          est = std::min(sat_mul(est, best_est), best_est);
          int first_member = -1;
          for (int i = 0; i < n; ++i)
            if (best_mem >> order[i] & 1) {
              first_member = order[i];
              break;
            }
          push(GSMAT_STEP_INTERSECT, first_member, -1, best_v, best_mem);
          bound |= 1ull << best_v;
          for (int t = 0; t < n; ++t)
            if ((best_mem >> t & 1) && all_bound(t)) erase(t);  // satisfied exactly
          continue;
        }
      }
      est = sat_mul(est, st[e1].stat);
      int v = is_var(pats[e1].s) ? var_of(pats[e1].s) : (is_var(pats[e1].o) ? var_of(pats[e1].o) : -1);
      push(all_const(e1) ? GSMAT_STEP_FILTER : GSMAT_STEP_SCAN, e1, -1, v, 0);
      bind(e1);
      erase(e1);
      continue;
    }
    int pick = -1;
    if (mode == GSMAT_PLAN_DEFAULT) {
      for (int i = 0; i < n_rem; ++i)
        if (has_bound_var(rem[i]) && all_bound(rem[i])) {
          pick = rem[i];
          break;
        }
    }
    if (pick < 0)
      for (int i = 0; i < n_rem; ++i)
        if (has_bound_var(rem[i])) {
          pick = rem[i];
          break;
        }
    if (pick < 0) {
      pick = rem[0];
      if (all_const(pick)) {
        est = std::min<int64_t>(est, st[pick].stat);
        push(GSMAT_STEP_FILTER, pick, -1, -1, 0);
      } else {
        est = sat_mul(est, st[pick].stat);
        int v = is_var(pats[pick].s) ? var_of(pats[pick].s) : var_of(pats[pick].o);
        push(GSMAT_STEP_CARTESIAN, pick, -1, v, 0);
        bind(pick);
      }
      erase(pick);
      continue;
    }
    if (all_bound(pick)) {
      push(GSMAT_STEP_FILTER, pick, -1, -1, 0);
    } else {
      const bool s_bound = is_var(pats[pick].s) && (bound >> var_of(pats[pick].s) & 1);
      const int orient = s_bound ? 0 : 1;
      const int newv = s_bound ? var_of(pats[pick].o) : var_of(pats[pick].s);
      est = sat_mul(est, st[pick].stat);
      push(GSMAT_STEP_EXPAND, pick, orient, newv, 0);
    }
    bind(pick);
    erase(pick);
  }
  return GSMAT_OK;
}

}  // namespace gsmat
