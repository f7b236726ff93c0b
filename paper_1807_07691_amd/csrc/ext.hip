// OPTIONAL, UNION and FILTER around the BGP join.
//
// The paper leaves these operators to future work (Sec. 9); their meaning
// here is the SPARQL algebra's over bags of solution mappings, and every BGP
// inside a query runs on the sparse-matrix join of Sec. 6-7:
//   * a branch's required BGP runs from the unit table, as gsmat_join does;
//   * LeftJoin(T, B) gives every row of T a row id and runs B's patterns
//     from T itself (the adaptive executor picks expansions and filters off
//     T's bound columns, as for any later step of a BGP), so the rows that
//     match come out already merged with their T row; a kernel marks the ids
//     that survived, and the rows of T never marked are compacted out and
//     kept with B's variables unbound;
//   * FILTER evaluates its conditions per row and compacts; conditions on the
//     required variables and constants alone run before the left joins;
//   * UNION is the concatenation of the branches' tables.
// A query's result is a list of column tables ("parts"), each binding a
// subset of the variables; a variable a part lacks is unbound (fetched as -1).
//
// The left joins are restricted to well-designed patterns: a variable an
// OPTIONAL group shares with the rest of its branch must occur in the
// branch's required BGP.  Every such variable is then bound in every row of
// T, so the match is an equi-join on bound columns.

#include <algorithm>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "device.hpp"
#include "exec.hpp"

namespace gsmat {
namespace {

constexpr int kMaxConds = 16;  // FILTER conditions per branch

struct XCond {
  int32_t op, a, b;
};
struct XConds {
  XCond c[kMaxConds];
  int32_t n;
};

__global__ void k_x_iota(int32_t* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)i;
}

// hit[rid[i]] = 1 for every row of a matched table (several rows may carry
// the same id: they all store the same byte).
__global__ void k_x_mark(const int32_t* __restrict__ rid, int64_t n, uint8_t* __restrict__ hit) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    hit[rid[i]] = 1;
}

// In place, per tile of kTile rows: f[i] = 1 for the rows never marked, and
// the tile's count of them.
__global__ __launch_bounds__(kBlock) void k_x_unmatched(uint8_t* __restrict__ f, int64_t n,
                                                        int64_t* __restrict__ ts) {
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
  int64_t loc = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = tile0 + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) {
      const uint8_t v = f[i] ? 0 : 1;
      f[i] = v;
      loc += v;
    }
  }
  const int64_t tot = dev::block_sum(loc);
  if (threadIdx.x == 0) ts[blockIdx.x] = tot;
}

// A term's value in row i: a constant id, the variable's column, or -1 when
// the part does not bind the variable.
__device__ inline int32_t x_term(const ColSet& cols, int32_t t, int64_t i) {
  if (t >= 0) return t;
  const int32_t* c = cols.c[-t - 1];
  return c ? c[i] : -1;
}

__device__ inline bool x_holds(const XCond& q, const ColSet& cols, int64_t i) {
  const int32_t a = x_term(cols, q.a, i);
  if (q.op == GSMAT_F_BOUND) return a >= 0;
  if (q.op == GSMAT_F_NOT_BOUND) return a < 0;
  const int32_t b = x_term(cols, q.b, i);
  if (a < 0 || b < 0) return false;  // an unbound operand is an error: the row goes
  switch (q.op) {
    case GSMAT_F_EQ: return a == b;
    case GSMAT_F_NE: return a != b;
    case GSMAT_F_LT: return a < b;
    case GSMAT_F_LE: return a <= b;
    case GSMAT_F_GT: return a > b;
    default: return a >= b;
  }
}

// FILTER flags of one tile (the conjunction of the branch's conditions;
// cols indexed by variable) and the tile's count of kept rows.
__global__ __launch_bounds__(kBlock) void k_x_filter(ColSet cols, XConds fc, int64_t n,
                                                     uint8_t* __restrict__ flags,
                                                     int64_t* __restrict__ ts) {
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
  int64_t loc = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = tile0 + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) {
      bool ok = true;
      for (int c = 0; c < fc.n && ok; ++c) ok = x_holds(fc.c[c], cols, i);
      flags[i] = ok ? 1 : 0;
      loc += ok ? 1 : 0;
    }
  }
  const int64_t tot = dev::block_sum(loc);
  if (threadIdx.x == 0) ts[blockIdx.x] = tot;
}

unsigned rows_grid(int64_t n) {
  return (unsigned)std::min<int64_t>(std::max<int64_t>(ceil_div(n, kBlock), 1), 65536);
}

// ---------------------------------------------------------------- host side

struct XPart {
  int64_t n = 0;
  int k = 0;
  const int32_t* col[kMaxCols] = {};
  int var[kMaxCols] = {};                    // query variables
  std::vector<std::shared_ptr<Arena>> keep;  // what the columns live in
  int col_of(int v) const {
    for (int c = 0; c < k; ++c)
      if (var[c] == v) return c;
    return -1;
  }
};

struct XBranch {
  std::vector<gsmat_pattern> req;
  std::vector<std::vector<gsmat_pattern>> opt;  // ascending group id
  std::vector<XCond> conds;
};

uint64_t vars_of(const std::vector<gsmat_pattern>& ps) {
  uint64_t m = 0;
  for (const gsmat_pattern& q : ps)
    for (int32_t t : {q.s, q.o})
      if (is_var(t)) m |= 1ull << var_of(t);
  return m;
}

// Checks the query and groups it by branch (ascending id) and group.
void parse_query(const gsmat_ext_pattern* pats, int32_t n_pats, const gsmat_filter* filters,
                 int32_t n_filters, int32_t n_vars, std::vector<XBranch>* out) {
  if (n_pats < 0 || n_filters < 0) throw StatusFail{GSMAT_EINVAL, "negative count"};
  if ((n_pats > 0 && !pats) || (n_filters > 0 && !filters))
    throw StatusFail{GSMAT_EINVAL, "pattern or filter array is NULL"};
  if (n_pats + n_filters == 0) throw StatusFail{GSMAT_EINVAL, "empty query"};
  if (n_vars < 0 || n_vars >= kMaxCols)
    throw StatusFail{GSMAT_EUNSUPPORTED, "n_vars must be in [0, 31]"};
  auto check_term = [&](int32_t t, const std::string& where) {
    if (is_var(t) && var_of(t) >= n_vars)
      throw StatusFail{GSMAT_EINVAL, where + ": variable beyond n_vars"};
  };
  std::vector<int32_t> ids;
  for (int32_t i = 0; i < n_pats; ++i) {
    const gsmat_ext_pattern& q = pats[i];
    const std::string w = "pattern " + std::to_string(i);
    if (q.p < 0) throw StatusFail{GSMAT_EUNSUPPORTED, w + ": variable predicate"};
    if (q.branch < 0 || q.group < 0) throw StatusFail{GSMAT_EINVAL, w + ": negative branch or group"};
    check_term(q.s, w);
    check_term(q.o, w);
    ids.push_back(q.branch);
  }
  for (int32_t i = 0; i < n_filters; ++i) {
    const gsmat_filter& f = filters[i];
    const std::string w = "filter " + std::to_string(i);
    if (f.op < GSMAT_F_EQ || f.op > GSMAT_F_NOT_BOUND) throw StatusFail{GSMAT_EINVAL, w + ": unknown op"};
    if (f.branch < 0) throw StatusFail{GSMAT_EINVAL, w + ": negative branch"};
    check_term(f.a, w);
    if (f.op == GSMAT_F_BOUND || f.op == GSMAT_F_NOT_BOUND) {
      if (!is_var(f.a)) throw StatusFail{GSMAT_EINVAL, w + ": BOUND needs a variable"};
    } else {
      check_term(f.b, w);
    }
    ids.push_back(f.branch);
  }
  std::sort(ids.begin(), ids.end());
  ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
  out->assign(ids.size(), XBranch{});
  for (size_t b = 0; b < ids.size(); ++b) {
    XBranch& br = (*out)[b];
    std::vector<int32_t> groups;
    for (int32_t i = 0; i < n_pats; ++i)
      if (pats[i].branch == ids[b] && pats[i].group > 0) groups.push_back(pats[i].group);
    std::sort(groups.begin(), groups.end());
    groups.erase(std::unique(groups.begin(), groups.end()), groups.end());
    br.opt.assign(groups.size(), {});
    for (int32_t i = 0; i < n_pats; ++i) {
      const gsmat_ext_pattern& q = pats[i];
      if (q.branch != ids[b]) continue;
      const gsmat_pattern tp{q.s, q.p, q.o};
      if (q.group == 0) {
        br.req.push_back(tp);
      } else {
        const size_t g = std::lower_bound(groups.begin(), groups.end(), q.group) - groups.begin();
        br.opt[g].push_back(tp);
      }
    }
    if (br.req.size() > (size_t)kMaxPats)
      throw StatusFail{GSMAT_EUNSUPPORTED, "a BGP has more than 32 patterns"};
    for (const auto& g : br.opt)
      if (g.size() > (size_t)kMaxPats)
        throw StatusFail{GSMAT_EUNSUPPORTED, "a BGP has more than 32 patterns"};
    // well-designed: what an OPTIONAL group shares with the rest of the
    // branch is bound by the required BGP
    const uint64_t req = vars_of(br.req);
    for (size_t g = 0; g < br.opt.size(); ++g) {
      uint64_t rest = req;
      for (size_t h = 0; h < br.opt.size(); ++h)
        if (h != g) rest |= vars_of(br.opt[h]);
      if (vars_of(br.opt[g]) & rest & ~req)
        throw StatusFail{GSMAT_EUNSUPPORTED,
                         "an OPTIONAL group shares a variable that the required BGP does not bind"};
    }
    for (int32_t i = 0; i < n_filters; ++i)
      if (filters[i].branch == ids[b]) br.conds.push_back(XCond{filters[i].op, filters[i].a, filters[i].b});
    if (br.conds.size() > (size_t)kMaxConds)
      throw StatusFail{GSMAT_EUNSUPPORTED, "more than 16 FILTER conditions in a branch"};
  }
}

struct XRun {
  gsmat_store* st;
  hipStream_t s;
  int64_t budget;

  DeviceMem* mem() { return st->mem.get(); }

  std::shared_ptr<Arena> arena(size_t bytes) {
    return std::make_shared<Arena>(mem(), std::max<size_t>(bytes, 4), s);
  }

  // The BGP's patterns with variables renumbered densely from 0 (first
  // occurrence order); loc[v] = local id of query variable v, or -1.
  std::unique_ptr<gsmat_query_plan, void (*)(gsmat_query_plan*)> plan(
      const std::vector<gsmat_pattern>& ps, int* loc, int* glob, int* L) {
    std::fill(loc, loc + kMaxCols, -1);
    int n = 0;
    std::vector<gsmat_pattern> q = ps;
    for (gsmat_pattern& t : q)
      for (int32_t* e : {&t.s, &t.o})
        if (is_var(*e)) {
          const int v = var_of(*e);
          if (loc[v] < 0) {
            glob[n] = v;
            loc[v] = n++;
          }
          *e = -(loc[v] + 1);
        }
    *L = n;
    gsmat_query_plan* pl = nullptr;
    const gsmat_status rc = gsmat_plan(st, q.data(), (int32_t)q.size(), GSMAT_PLAN_ADAPTIVE, s, &pl);
    if (rc != GSMAT_OK) throw StatusFail{rc, gsmat_last_error()};
    return {pl, gsmat_plan_free};
  }

  // A collected table as a part: owned memory adopted; map[c] = the query
  // variable of column c (-1: drop the column); columns that are views into
  // the arenas of `from` keep those arenas.
  XPart adopt(const Table& t, const int* map, const std::vector<std::shared_ptr<Arena>>& from) {
    XPart p;
    p.n = t.n;
    if (t.owned) p.keep.push_back(std::make_shared<Arena>(mem(), t.owned, t.owned_bytes, s));
    for (int c = 0; c < t.k; ++c) {
      if (map[c] < 0) continue;
      p.col[p.k] = t.col[c];
      p.var[p.k] = map[c];
      ++p.k;
      const uintptr_t a = (uintptr_t)t.col[c];
      for (const auto& h : from) {
        const uintptr_t lo = (uintptr_t)h->p;
        if (a >= lo && a < lo + h->bytes &&
            std::find(p.keep.begin(), p.keep.end(), h) == p.keep.end())
          p.keep.push_back(h);
      }
    }
    return p;
  }

  // Scans the tile sums ts[0, nt) in place; the total.
  int64_t total(int64_t* ts, int64_t nt) {
    launch_scan_tile_sums(ts, nt, ts + nt, s, nullptr);
    int64_t m = 0;
    GS_HIP(hipMemcpyAsync(&m, ts + nt, sizeof(m), hipMemcpyDeviceToHost, s));
    host_sync(s);
    return m;
  }

  // The rows of p with a non-zero flag (ts: scanned tile sums), m of them.
  XPart compact(const XPart& p, const uint8_t* flags, const int64_t* ts, int64_t m) {
    XPart o;
    o.n = m;
    o.k = p.k;
    std::copy(p.var, p.var + p.k, o.var);
    if (p.k == 0) return o;
    const int64_t stride = col_stride(m);
    auto a = arena(sizeof(int32_t) * (size_t)stride * (size_t)p.k);
    ColSet in{};
    OutSet out{};
    for (int c = 0; c < p.k; ++c) {
      in.c[c] = p.col[c];
      out.c[c] = (int32_t*)a->p + (size_t)c * (size_t)stride;
      o.col[c] = out.c[c];
    }
    launch_compact_cols(in, p.k, flags, p.n, ts, out, s);
    o.keep.push_back(a);
    return o;
  }

  std::vector<XPart> bgp(const std::vector<gsmat_pattern>& ps) {
    std::vector<XPart> out;
    if (ps.empty()) {  // the unit bag: one row, nothing bound
      XPart u;
      u.n = 1;
      out.push_back(u);
      return out;
    }
    int loc[kMaxCols], glob[kMaxCols], L = 0;
    auto pl = plan(ps, loc, glob, &L);
    std::vector<Table> tabs;
    run_collect(st, pl.get(), nullptr, budget, s, &tabs);
    for (const Table& t : tabs) {
      int map[kMaxCols];
      for (int c = 0; c < t.k; ++c) map[c] = glob[t.var[c]];
      out.push_back(adopt(t, map, {}));
    }
    return out;
  }

  // Every part of `left` left-joined with the BGP ps.
  std::vector<XPart> left_join(std::vector<XPart> left, const std::vector<gsmat_pattern>& ps) {
    int loc[kMaxCols], glob[kMaxCols], L = 0;
    auto pl = plan(ps, loc, glob, &L);
    std::vector<XPart> out;
    for (XPart& P : left) {
      if (P.n == 0) continue;
      if (P.n >= ((int64_t)1 << 31))
        throw StatusFail{GSMAT_EUNSUPPORTED, "an OPTIONAL's left side has 2^31 rows or more"};
      // the starting table: P's columns (shared variables under their local
      // ids, the others after them) and the row ids
      auto rid = arena(sizeof(int32_t) * (size_t)P.n);
      hipLaunchKernelGGL(k_x_iota, dim3(rows_grid(P.n)), dim3(kBlock), 0, s, (int32_t*)rid->p, P.n);
      GS_HIP(hipGetLastError());
      Table t0;
      t0.n = P.n;
      t0.k = P.k + 1;
      int back[64];  // starting-table id -> query variable (-1: row id)
      int next = L;
      for (int c = 0; c < P.k; ++c) {
        const int v = P.var[c];
        const int id = loc[v] >= 0 ? loc[v] : next++;
        t0.col[c] = P.col[c];
        t0.var[c] = id;
        back[id] = v;
      }
      const int rid_id = next;
      t0.col[P.k] = (const int32_t*)rid->p;
      t0.var[P.k] = rid_id;
      back[rid_id] = -1;
      for (int i = 0; i < L; ++i) back[i] = glob[i];
      std::vector<Table> tabs;
      run_collect(st, pl.get(), &t0, budget, s, &tabs);
      // the left rows some match kept
      auto hit = arena((size_t)P.n);
      GS_HIP(hipMemsetAsync(hit->p, 0, (size_t)P.n, s));
      std::vector<std::shared_ptr<Arena>> from = P.keep;
      from.push_back(rid);
      std::vector<XPart> matched;
      for (const Table& t : tabs) {
        const int rc = t.col_of(rid_id);
        if (rc < 0) throw StatusFail{GSMAT_EHIP, "internal: row ids lost in an OPTIONAL join"};
        if (t.n > 0) {
          hipLaunchKernelGGL(k_x_mark, dim3(rows_grid(t.n)), dim3(kBlock), 0, s, t.col[rc], t.n,
                             (uint8_t*)hit->p);
          GS_HIP(hipGetLastError());
        }
        int map[kMaxCols];
        for (int c = 0; c < t.k; ++c) map[c] = back[t.var[c]];
        matched.push_back(adopt(t, map, from));
      }
      const int64_t nt = ceil_div(P.n, kTile);
      auto ts = arena(sizeof(int64_t) * (size_t)(nt + 1));
      hipLaunchKernelGGL(k_x_unmatched, dim3((unsigned)nt), dim3(kBlock), 0, s, (uint8_t*)hit->p,
                         P.n, (int64_t*)ts->p);
      GS_HIP(hipGetLastError());
      const int64_t m = total((int64_t*)ts->p, nt);
      for (XPart& q : matched)
        if (q.n > 0) out.push_back(std::move(q));
      if (m == P.n) {
        out.push_back(std::move(P));
      } else if (m > 0) {
        out.push_back(compact(P, (const uint8_t*)hit->p, (const int64_t*)ts->p, m));
      }
    }
    return out;
  }

  std::vector<XPart> filter(std::vector<XPart> parts, const std::vector<XCond>& conds) {
    XConds fc{};
    fc.n = (int32_t)conds.size();
    std::copy(conds.begin(), conds.end(), fc.c);
    std::vector<XPart> out;
    for (XPart& P : parts) {
      if (P.n == 0) continue;
      ColSet cols{};
      for (int c = 0; c < P.k; ++c) cols.c[P.var[c]] = P.col[c];
      const int64_t nt = ceil_div(P.n, kTile);
      auto flags = arena((size_t)P.n);
      auto ts = arena(sizeof(int64_t) * (size_t)(nt + 1));
      hipLaunchKernelGGL(k_x_filter, dim3((unsigned)nt), dim3(kBlock), 0, s, cols, fc, P.n,
                         (uint8_t*)flags->p, (int64_t*)ts->p);
      GS_HIP(hipGetLastError());
      const int64_t m = total((int64_t*)ts->p, nt);
      if (m == P.n) {
        out.push_back(std::move(P));
      } else if (m > 0) {
        out.push_back(compact(P, (const uint8_t*)flags->p, (const int64_t*)ts->p, m));
      }
    }
    return out;
  }
};

}  // namespace
}  // namespace gsmat

using namespace gsmat;

extern "C" gsmat_status gsmat_join_ext(gsmat_store* st, const gsmat_ext_pattern* pats,
                                       int32_t n_pats, const gsmat_filter* filters,
                                       int32_t n_filters, int32_t n_vars, int64_t budget_bytes,
                                       int64_t max_rows, void* stream, gsmat_result** out) {
  return guarded([&]() -> gsmat_status {
    if (!out) throw StatusFail{GSMAT_EINVAL, "out is NULL"};
    *out = nullptr;
    std::vector<XBranch> branches;
    parse_query(pats, n_pats, filters, n_filters, n_vars, &branches);
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<gsmat_result> res(new gsmat_result);
    res->st = st;
    res->stream = s;
    res->n_vars = n_vars;
    res->reset_steps(0);
    XRun x{st, s, budget_bytes};
    for (const XBranch& br : branches) {
      // conditions on required variables and constants only hold or fail the
      // same before the left joins (those variables are bound in every row and
      // a left join never changes them): applied first, on the smaller table
      const uint64_t req = vars_of(br.req);
      std::vector<XCond> early, late;
      for (const XCond& c : br.conds) {
        const bool cmp = c.op != GSMAT_F_BOUND && c.op != GSMAT_F_NOT_BOUND;
        bool on_req = !is_var(c.a) || (req >> var_of(c.a) & 1);
        if (cmp) on_req = on_req && (!is_var(c.b) || (req >> var_of(c.b) & 1));
        (on_req ? early : late).push_back(c);
      }
      std::vector<XPart> parts = x.bgp(br.req);
      if (!early.empty()) parts = x.filter(std::move(parts), early);
      for (const auto& g : br.opt) parts = x.left_join(std::move(parts), g);
      if (!late.empty()) parts = x.filter(std::move(parts), late);
      for (XPart& p : parts) {
        if (p.n == 0) continue;
        Segment seg;
        seg.rows = p.n;
        for (int v = 0; v < n_vars; ++v) {
          const int c = p.col_of(v);
          seg.col[v] = c >= 0 ? p.col[c] : nullptr;
        }
        seg.hold = std::make_shared<std::vector<std::shared_ptr<Arena>>>(std::move(p.keep));
        res->rows += seg.rows;
        res->segs.push_back(std::move(seg));
        if (max_rows >= 0 && res->rows > max_rows)
          throw StatusFail{GSMAT_ETOOBIG,
                           "result exceeds max_rows (" + std::to_string(max_rows) + ")"};
      }
    }
    GS_HIP(hipStreamSynchronize(s));
    *out = res.release();
    return GSMAT_OK;
  });
}
