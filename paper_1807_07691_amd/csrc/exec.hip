// Query execution (paper Sec. 6.3 and Sec. 7.2): runs a plan's steps over
// device-resident binding tables.
//
// A binding table is columnar int32 (one array per bound variable).  Each
// step follows the preallocation scheme of Algorithm "Pre-allocating result
// matrix space": per input row, count the output rows (N_i); exclusive prefix
// sum (P_i, int64); allocate exactly P_n rows; write every input row's
// outputs at its offset.  Expansions write through a merge path over
// (row ends, output indices) so hub rows are split across workgroups; filters
// and star-centre intersections write through a stable ballot compaction.
// When a step's output exceeds the byte budget it is cut into output ranges,
// each carried through the remaining steps before the next one is produced
// (chunked expansion); the final table may therefore consist of segments.
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "exec.hpp"

using namespace gsmat;

namespace {

template <class T>
struct Tmp {
  DeviceMem* mem;
  hipStream_t s;
  T* p = nullptr;
  size_t bytes = 0;
  Tmp(DeviceMem* m, int64_t n, hipStream_t st) : mem(m), s(st) {
    bytes = sizeof(T) * (size_t)std::max<int64_t>(n, 1);
    p = (T*)mem->alloc(bytes, s);
    if (!p) throw OomFail{bytes};
  }
  ~Tmp() {
    if (p) mem->free(p, bytes, s);
  }
  Tmp(const Tmp&) = delete;
  Tmp& operator=(const Tmp&) = delete;
};

// Per-thread pinned host area that kernels write small results into (sizes
// of the next step, lookups, fan-out samples); read after the stream syncs.
struct PinnedArea {
  int64_t total[8];
  LookupRes res[kMaxLookups];
  int64_t part[kMaxPats * kSampleBlocks];
};

static_assert(sizeof(PinnedArea) <= kStageBytes, "staged results must fit the staging area");

PinnedArea* pinned() {
  thread_local PinnedArea* a = nullptr;
  if (!a) GS_HIP(hipHostMalloc((void**)&a, sizeof(PinnedArea), hipHostMallocDefault));
  return a;
}

struct Exec {
  gsmat_store* st;
  const gsmat_query_plan* pl;
  hipStream_t s;
  int64_t budget;
  int64_t max_rows;
  gsmat_result* res;
  bool adaptive;

  void sync_stream() { host_sync(s); }

  // table allocations not yet released or handed to the result
  std::vector<std::pair<void*, size_t>> live;

  // Device memory of the tables and step scratch (null: the store's), and
  // where kernels leave small results for the host: null means pinned host
  // memory; otherwise this device area, copied to the host after the stream
  // synchronises (the allocation-free entry point uses both).
  DeviceMem* dm = nullptr;
  PinnedArea* dev_area = nullptr;
  // set: final tables are appended here rather than added to res
  std::vector<Table>* collect = nullptr;

  DeviceMem* mem() { return dm ? dm : st->mem.get(); }

  // Copies `bytes` of the device area at `p` to host memory at `h` (staged
  // small results) and waits for the stream.
  void stage_back(void* h, const void* p, size_t bytes) {
    GS_HIP(hipMemcpyAsync(h, p, bytes, hipMemcpyDeviceToHost, s));
    host_sync(s);
  }

  // Scans the tile sums in place and returns the grand total.
  int64_t scan_total(int64_t* ts, int64_t nt, hipStream_t st_) {
    if (dev_area) {
      launch_scan_tile_sums(ts, nt, ts + nt, st_, nullptr);
      int64_t v = 0;
      stage_back(&v, ts + nt, sizeof(v));
      return v;
    }
    PinnedArea* h = pinned();
    launch_scan_tile_sums(ts, nt, ts + nt, st_, &h->total[0]);
    host_sync(st_);
    return h->total[0];
  }

  void forget(void* p) {
    for (size_t i = 0; i < live.size(); ++i)
      if (live[i].first == p) {
        live[i] = live.back();
        live.pop_back();
        return;
      }
  }

  void release(Table& t) {
    if (t.owned) {
      forget(t.owned);
      mem()->free(t.owned, t.owned_bytes, s);
    }
    t.owned = nullptr;
  }

  // frees every table still alive (error paths)
  void release_all() {
    for (auto& a : live) mem()->free(a.first, a.second, s);
    live.clear();
  }

  // Allocates a table of n rows for the given variables (columns in order).
  // Columns start on 256-byte boundaries (stride rounded up to 64 values) so
  // that a wave's 64 stores of one column cover whole cache lines.
  Table alloc_table(int64_t n, const int* vars, int k) {
    Table t;
    t.n = n;
    t.k = k;
    const int64_t stride = col_stride(n);
    const size_t bytes = sizeof(int32_t) * (size_t)stride * (size_t)std::max(k, 1);
    if (k > 0) {
      t.owned = mem()->alloc(bytes, s);
      if (!t.owned) throw OomFail{bytes};
      t.owned_bytes = bytes;
      live.push_back({t.owned, bytes});
    }
    for (int c = 0; c < k; ++c) {
      t.var[c] = vars[c];
      t.col[c] = (int32_t*)t.owned + (size_t)c * (size_t)stride;
    }
    return t;
  }

  // Lookup of pattern tp's constant endpoint(s): the plan's, when it was
  // planned on this store, else one device lookup.
  LookupRes lookup_tp(int tp, int orient, int32_t p, int32_t v, int32_t member) {
    if (pl->lk_store == st->uid && tp < (int)pl->lk.size() && pl->lk[tp].valid) {
      const gsmat_pat_lookup& l = pl->lk[tp];
      return LookupRes{l.start, l.len, l.found, 0};
    }
    return lookup(orient, p, v, member);
  }

  LookupRes lookup(int orient, int32_t p, int32_t v, int32_t member) {
    LookupBatch b{};
    b.req[0] = LookupReq{orient, p, v, member};
    b.n = 1;
    if (dev_area) {
      launch_lookup(b, st->out.d_desc, st->in.d_desc, st->out.ptrs(), st->in.ptrs(),
                    dev_area->res, s);
      LookupRes r;
      stage_back(&r, dev_area->res, sizeof(r));
      return r;
    }
    PinnedArea* h = pinned();
    launch_lookup(b, st->out.d_desc, st->in.d_desc, st->out.ptrs(), st->in.ptrs(), h->res, s);
    host_sync(s);
    return h->res[0];
  }

  void emit(Table& t) {
    if (collect) {
      if (t.owned) forget(t.owned);
      collect->push_back(t);
      t.owned = nullptr;
      return;
    }
    const int nv = pl->n_vars;
    Segment seg;
    seg.rows = t.n;
    for (int v = 0; v < nv; ++v) {
      const int c = t.col_of(v);
      if (c < 0) throw StatusFail{GSMAT_EHIP, "internal: unbound variable at the end of the plan"};
      seg.col[v] = t.col[c];
    }
    seg.owned = t.owned;
    seg.owned_bytes = t.owned_bytes;
    if (t.owned) forget(t.owned);
    t.owned = nullptr;
    res->rows += seg.rows;
    res->segs.push_back(seg);
    if (max_rows >= 0 && res->rows > max_rows)
      throw StatusFail{GSMAT_ETOOBIG, "result exceeds max_rows (" + std::to_string(max_rows) + ")"};
  }

  int64_t chunk_rows(int width) {
    if (budget <= 0) return INT64_MAX;
    const int64_t r = budget / (4 * (int64_t)std::max(width, 1));
    if (r < 1) throw StatusFail{GSMAT_ENOMEM, "budget_bytes cannot hold one output row"};
    return r;
  }

  // The relation of one TP on its own (views into the store where possible).
  Table tp_relation(int tp) {
    const gsmat_pattern& q = pl->pats[tp];
    const int32_t p = q.p;
    Table t;
    if (is_var(q.s) && is_var(q.o)) {
      const PredView pv = st->out.view(p);
      if (q.s != q.o) {
        t.n = pv.nnz;
        t.k = 2;
        t.col[0] = pv.src;
        t.var[0] = var_of(q.s);
        t.col[1] = pv.nbr;
        t.var[1] = var_of(q.o);
        return t;
      }
      // (?x p ?x): the diagonal
      const int64_t n = pv.nnz;
      const int64_t nt = ceil_div(std::max<int64_t>(n, 1), kTile);
      Tmp<uint8_t> flags(mem(), n, s);
      Tmp<int64_t> ts(mem(), nt + 1, s);
      if (n > 0) launch_flag_diag(pv.src, pv.nbr, n, flags.p, ts.p, s);
      const int64_t m = n > 0 ? scan_total(ts.p, nt, s) : 0;
      int v = var_of(q.s);
      Table o = alloc_table(m, &v, 1);
      if (m > 0) {
        ColSet in{};
        in.c[0] = pv.src;
        OutSet out{};
        out.c[0] = const_cast<int32_t*>(o.col[0]);
        launch_compact_cols(in, 1, flags.p, n, ts.p, out, s);
      }
      return o;
    }
    if (!is_var(q.s) && is_var(q.o)) {
      const LookupRes r = lookup_tp(tp, 0, p, q.s, -1);
      const PredView pv = st->out.view(p);
      t.n = r.len;
      t.k = 1;
      t.col[0] = pv.nbr + r.start;
      t.var[0] = var_of(q.o);
      return t;
    }
    if (is_var(q.s) && !is_var(q.o)) {
      const LookupRes r = lookup_tp(tp, 1, p, q.o, -1);
      const PredView pv = st->in.view(p);
      t.n = r.len;
      t.k = 1;
      t.col[0] = pv.nbr + r.start;
      t.var[0] = var_of(q.s);
      return t;
    }
    const LookupRes r = lookup_tp(tp, 0, p, q.s, q.o);
    t.n = r.found ? 1 : 0;
    t.k = 0;
    return t;
  }

  uint32_t completes(const gsmat_step_info& sp) const { return step_completes(pl, sp); }

  // Adaptive choice of the next step on the bound table t (fan-out samples
  // of the candidate expansions are taken on the device).
  gsmat_step_info choose(const Table& t, uint32_t rem) {
    StepChoice c;
    step_candidates(st, pl, t, rem, c);
    if (c.has_filter) return c.filter;
    if (c.nc == 0) return c.cartesian;
    if (c.nc == 1) return step_pick(pl, c, nullptr);
    SampleSet ss{};
    for (int i = 0; i < c.nc; ++i) candidate_view(st, pl, t, c, i, &ss.col[i], &ss.pv[i]);
    ss.n = t.n;
    ss.ncand = c.nc;
    int64_t part[kMaxPats * kSampleBlocks];
    if (dev_area) {
      launch_sample_fanout(ss, dev_area->part, s);
      stage_back(part, dev_area->part, sizeof(int64_t) * c.nc * kSampleBlocks);
    } else {
      PinnedArea* h = pinned();
      launch_sample_fanout(ss, h->part, s);
      sync_stream();
      std::copy(h->part, h->part + c.nc * kSampleBlocks, part);
    }
    int64_t sum[kMaxPats];
    for (int i = 0; i < c.nc; ++i) {
      sum[i] = 0;
      for (int b = 0; b < kSampleBlocks; ++b) sum[i] += part[i * kSampleBlocks + b];
    }
    return step_pick(pl, c, sum);
  }

  void run(int si, Table& t, uint32_t rem) {
    if (t.n == 0) {
      release(t);
      return;
    }
    if (rem == 0) {
      emit(t);
      return;
    }
    const gsmat_step_info sp =
        (adaptive && !t.unit()) ? choose(t, rem) : pl->steps[std::min<size_t>(si, pl->steps.size() - 1)];
    const uint32_t next = rem & ~completes(sp);
    if (si < res->n_steps) res->step_in[si] += t.n;
    switch (sp.kind) {
      case GSMAT_STEP_SCAN:
      case GSMAT_STEP_CARTESIAN: {
        Table r = tp_relation(sp.tp);
        combine(si, t, r, next);
        break;
      }
      case GSMAT_STEP_INTERSECT: {
        Table r = intersect(sp);
        combine(si, t, r, next);
        break;
      }
      case GSMAT_STEP_FILTER:
        filter(si, sp, t, next);
        break;
      case GSMAT_STEP_EXPAND:
        expand(si, sp, t, next);
        break;
      default:
        throw StatusFail{GSMAT_EINVAL, "unknown step kind"};
    }
  }

  void add_out(int si, int64_t m) {
    if (si < res->n_steps) res->step_out[si] += m;
  }

  // t x r: r alone when t is the unit table, else the Cartesian product.
  void combine(int si, Table& t, Table& r, uint32_t next) {
    if (t.unit()) {
      add_out(si, r.n);
      release(t);
      run(si + 1, r, next);
      return;
    }
    if (r.n == 0) {
      release(t);
      release(r);
      return;
    }
    if (t.k + r.k > kMaxCols) throw StatusFail{GSMAT_EUNSUPPORTED, "too many columns"};
    if (r.n > 0 && t.n > INT64_MAX / r.n) throw StatusFail{GSMAT_ETOOBIG, "Cartesian product overflows"};
    const int64_t m = t.n * r.n;
    add_out(si, m);
    int vars[kMaxCols];
    for (int c = 0; c < t.k; ++c) vars[c] = t.var[c];
    for (int c = 0; c < r.k; ++c) vars[t.k + c] = r.var[c];
    const int k = t.k + r.k;
    const int64_t rpc = chunk_rows(k);
    ColSet a{}, b{};
    for (int c = 0; c < t.k; ++c) a.c[c] = t.col[c];
    for (int c = 0; c < r.k; ++c) b.c[c] = r.col[c];
    for (int64_t J0 = 0; J0 < m; J0 += rpc) {
      const int64_t J1 = std::min(m, J0 + rpc);
      Table o = alloc_table(J1 - J0, vars, k);
      OutSet out{};
      for (int c = 0; c < k; ++c) out.c[c] = const_cast<int32_t*>(o.col[c]);
      if (k > 0) launch_cartesian(a, t.k, t.n, b, r.k, r.n, J0, J1, out, s);
      run(si + 1, o, next);
    }
    release(t);
    release(r);
  }

  Table intersect(const gsmat_step_info& sp) {
    const int32_t cterm = -(sp.var + 1);
    struct L {
      ListRef ref;
      const int32_t* ids;  // the list as an array (row ids or segment)
    };
    std::vector<L> lists;
    for (int tp = 0; tp < (int)pl->pats.size(); ++tp) {
      if (!(sp.members >> tp & 1)) continue;
      const gsmat_pattern& q = pl->pats[tp];
      L l{};
      if (q.s == cterm && is_var(q.o)) {
        l.ref.pv = st->out.view(q.p);
        l.ref.is_keys = 1;
        l.ref.len = l.ref.pv.nr;
        l.ids = l.ref.pv.keys;
      } else if (q.o == cterm && is_var(q.s)) {
        l.ref.pv = st->in.view(q.p);
        l.ref.is_keys = 1;
        l.ref.len = l.ref.pv.nr;
        l.ids = l.ref.pv.keys;
      } else if (q.s == cterm) {  // (v p c): v among the subjects of object c
        const LookupRes r = lookup_tp(tp, 1, q.p, q.o, -1);
        l.ref.seg = st->in.view(q.p).nbr + r.start;
        l.ref.bm = st->in.row_bitmap(q.p, q.o);
        l.ref.len = r.len;
        l.ids = l.ref.seg;
      } else {  // (c p v): v among the objects of subject c
        const LookupRes r = lookup_tp(tp, 0, q.p, q.s, -1);
        l.ref.seg = st->out.view(q.p).nbr + r.start;
        l.ref.bm = st->out.row_bitmap(q.p, q.s);
        l.ref.len = r.len;
        l.ids = l.ref.seg;
      }
      lists.push_back(l);
    }
    Table t;
    t.k = 1;
    t.var[0] = sp.var;
    size_t d = 0;
    for (size_t i = 1; i < lists.size(); ++i)
      if (lists[i].ref.len < lists[d].ref.len) d = i;
    const int64_t n = lists[d].ref.len;
    if (n == 0) {
      t.n = 0;
      return t;
    }
    ListSet ls{};
    for (size_t i = 0; i < lists.size(); ++i)
      if (i != d) ls.l[ls.n++] = lists[i].ref;
    const int64_t nt = ceil_div(n, kTile);
    Tmp<uint8_t> flags(mem(), n, s);
    Tmp<int64_t> ts(mem(), nt + 1, s);
    launch_flag_intersect(lists[d].ids, n, ls, flags.p, ts.p, s);
    const int64_t m = scan_total(ts.p, nt, s);
    if (m == n) {  // every driver id survives: the driver list itself
      t.n = n;
      t.col[0] = lists[d].ids;
      return t;
    }
    int v = sp.var;
    Table o = alloc_table(m, &v, 1);
    if (m > 0) {
      ColSet in{};
      in.c[0] = lists[d].ids;
      OutSet out{};
      out.c[0] = const_cast<int32_t*>(o.col[0]);
      launch_compact_cols(in, 1, flags.p, n, ts.p, out, s);
    }
    return o;
  }

  void filter(int si, const gsmat_step_info& sp, Table& t, uint32_t next) {
    const gsmat_pattern& q = pl->pats[sp.tp];
    if (!is_var(q.s) && !is_var(q.o)) {
      const LookupRes r = lookup_tp(sp.tp, 0, q.p, q.s, q.o);
      if (r.found) {
        add_out(si, t.n);
        run(si + 1, t, next);
      } else {
        release(t);
      }
      return;
    }
    ProbeArgs pa{};
    if (is_var(q.s)) pa.s_col = t.col[t.col_of(var_of(q.s))];
    else pa.s_const = q.s;
    if (is_var(q.o)) pa.o_col = t.col[t.col_of(var_of(q.o))];
    else pa.o_const = q.o;
    const PredView pv = st->out.view(q.p);
    const int64_t n = t.n;
    const int64_t nt = ceil_div(n, kTile);
    Tmp<uint8_t> flags(mem(), n, s);
    Tmp<int64_t> ts(mem(), nt + 1, s);
    launch_flag_filter(pa, n, pv, flags.p, ts.p, s);
    const int64_t m = scan_total(ts.p, nt, s);
    add_out(si, m);
    if (m == n) {  // nothing removed: pass the table on unchanged
      run(si + 1, t, next);
      return;
    }
    if (m == 0) {
      release(t);
      return;
    }
    Table o = alloc_table(m, t.var, t.k);
    ColSet in{};
    OutSet out{};
    for (int c = 0; c < t.k; ++c) {
      in.c[c] = t.col[c];
      out.c[c] = const_cast<int32_t*>(o.col[c]);
    }
    launch_compact_cols(in, t.k, flags.p, n, ts.p, out, s);
    release(t);
    run(si + 1, o, next);
  }

  void expand(int si, const gsmat_step_info& sp, Table& t, uint32_t next) {
    const gsmat_pattern& q = pl->pats[sp.tp];
    const int bound_var = sp.orient == 0 ? var_of(q.s) : var_of(q.o);
    const int new_var = sp.orient == 0 ? var_of(q.o) : var_of(q.s);
    const int bc = t.col_of(bound_var);
    if (bc < 0) throw StatusFail{GSMAT_EHIP, "internal: expansion from an unbound variable"};
    if (t.k + 1 > kMaxCols) throw StatusFail{GSMAT_EUNSUPPORTED, "too many columns"};
    const PredView pv = sp.orient == 0 ? st->out.view(q.p) : st->in.view(q.p);
    const int64_t n = t.n;
    const int64_t nt = ceil_div(n, kTile);
    Tmp<int32_t> N(mem(), n, s), start(mem(), n, s);
    Tmp<int64_t> ts(mem(), nt + 1, s), P(mem(), n + 1, s);
    launch_count_expand(t.col[bc], n, pv, N.p, start.p, ts.p, s);
    const int64_t m = scan_total(ts.p, nt, s);
    add_out(si, m);
    if (m == 0) {
      release(t);
      return;
    }
    launch_scan_add_i32(N.p, n, ts.p, P.p, s);
    int vars[kMaxCols];
    for (int c = 0; c < t.k; ++c) vars[c] = t.var[c];
    vars[t.k] = new_var;
    const int k = t.k;
    const int64_t rpc = chunk_rows(k + 1);
    ColSet in{};
    for (int c = 0; c < k; ++c) in.c[c] = t.col[c];
    for (int64_t J0 = 0; J0 < m; J0 += rpc) {
      const int64_t J1 = std::min(m, J0 + rpc);
      const int64_t ntiles = ceil_div(n + (J1 - J0), kTile);
      Tmp<int64_t> split(mem(), ntiles + 1, s);
      launch_mp_partition(P.p, n, J0, J1, split.p, ntiles, s);
      Table o = alloc_table(J1 - J0, vars, k + 1);
      OutSet out{};
      for (int c = 0; c <= k; ++c) out.c[c] = const_cast<int32_t*>(o.col[c]);
      const double parents = (double)n * (double)(J1 - J0) / (double)m;
      const double bytes = 4.0 * (double)(J1 - J0) * (k + 2) + parents * (4.0 * k + 12.0);
      launch_write_expand(in, k, P.p, start.p, n, pv.nbr, J0, J1, split.p, ntiles, out, bytes, s);
      run(si + 1, o, next);
    }
    release(t);
  }
};

}  // namespace

namespace gsmat {

Arena::Arena(DeviceMem* m, size_t b, hipStream_t st) : mem(m), bytes(b), s(st) {
  p = mem->alloc(bytes, s);
  if (!p) throw OomFail{bytes};
}
Arena::~Arena() {
  if (p) mem->free(p, bytes, s);
}

uint32_t step_completes(const gsmat_query_plan* pl, const gsmat_step_info& sp) {
  if (sp.kind != GSMAT_STEP_INTERSECT) return 1u << sp.tp;
  uint32_t m = 0;
  const int32_t cterm = -(sp.var + 1);
  for (int tp = 0; tp < (int)pl->pats.size(); ++tp) {
    if (!(sp.members >> tp & 1)) continue;
    const gsmat_pattern& q = pl->pats[tp];
    const int32_t other = q.s == cterm ? q.o : q.s;
    if (!is_var(other)) m |= 1u << tp;
  }
  return m;
}

void step_candidates(const gsmat_store* st, const gsmat_query_plan* pl, const Table& t,
                     uint32_t rem, StepChoice& ch) {
  uint64_t bound = 0;
  for (int c = 0; c < t.k; ++c) bound |= 1ull << t.var[c];
  auto is_bound = [&](int32_t term) { return !is_var(term) || (bound >> var_of(term) & 1); };
  ch.has_filter = false;
  ch.nc = 0;
  const int np = (int)pl->pats.size();
  for (int tp = 0; tp < np; ++tp) {
    if (!(rem >> tp & 1)) continue;
    const gsmat_pattern& q = pl->pats[tp];
    const bool connected = (is_var(q.s) && (bound >> var_of(q.s) & 1)) ||
                           (is_var(q.o) && (bound >> var_of(q.o) & 1));
    const bool all_const = !is_var(q.s) && !is_var(q.o);
    if ((connected || all_const) && is_bound(q.s) && is_bound(q.o)) {
      std::memset(&ch.filter, 0, sizeof(ch.filter));
      ch.filter.kind = GSMAT_STEP_FILTER;
      ch.filter.tp = tp;
      ch.filter.orient = -1;
      ch.filter.var = -1;
      ch.has_filter = true;
      return;
    }
  }
  for (int tp = 0; tp < np; ++tp) {
    if (!(rem >> tp & 1)) continue;
    const gsmat_pattern& q = pl->pats[tp];
    const bool sb = is_var(q.s) && (bound >> var_of(q.s) & 1);
    const bool ob = is_var(q.o) && (bound >> var_of(q.o) & 1);
    if (sb == ob) continue;  // not connected (both bound were handled above)
    const int32_t free_term = sb ? q.o : q.s;
    if (!is_var(free_term)) continue;
    ch.cand_tp[ch.nc] = (int8_t)tp;
    ch.cand_or[ch.nc] = sb ? 0 : 1;
    ++ch.nc;
  }
  int pick = -1;
  int64_t best_nnz = INT64_MAX;
  for (int tp = 0; tp < np; ++tp) {
    if (!(rem >> tp & 1)) continue;
    const int64_t z = st->out.desc[pl->pats[tp].p].nnz;
    if (z < best_nnz) {
      best_nnz = z;
      pick = tp;
    }
  }
  std::memset(&ch.cartesian, 0, sizeof(ch.cartesian));
  ch.cartesian.kind = GSMAT_STEP_CARTESIAN;
  ch.cartesian.tp = pick;
  ch.cartesian.orient = -1;
  ch.cartesian.var = -1;
}

void candidate_view(const gsmat_store* st, const gsmat_query_plan* pl, const Table& t,
                    const StepChoice& c, int i, const int32_t** col, PredView* pv) {
  const gsmat_pattern& q = pl->pats[c.cand_tp[i]];
  const bool from_s = c.cand_or[i] == 0;
  *col = t.col[t.col_of(var_of(from_s ? q.s : q.o))];
  *pv = from_s ? st->out.view(q.p) : st->in.view(q.p);
}

gsmat_step_info step_pick(const gsmat_query_plan* pl, const StepChoice& c, const int64_t* sums) {
  int best = 0;
  if (sums)
    for (int i = 1; i < c.nc; ++i)
      if (sums[i] < sums[best]) best = i;
  const gsmat_pattern& q = pl->pats[c.cand_tp[best]];
  gsmat_step_info sp;
  std::memset(&sp, 0, sizeof(sp));
  sp.kind = GSMAT_STEP_EXPAND;
  sp.tp = c.cand_tp[best];
  sp.orient = c.cand_or[best];
  sp.var = c.cand_or[best] == 0 ? var_of(q.o) : var_of(q.s);
  return sp;
}

void run_query(gsmat_store* st, const gsmat_query_plan* pl, int64_t budget_bytes,
               int64_t max_rows, hipStream_t s, gsmat_result* res, DeviceMem* mem,
               void* dev_area) {
  // a pattern over an absent predicate or vertex matches nothing
  for (const gsmat_pattern& q : pl->pats) {
    if (q.p >= st->P) return;
    if (!is_var(q.s) && q.s >= st->V) return;
    if (!is_var(q.o) && q.o >= st->V) return;
  }
  Exec ex{st, pl, s, budget_bytes, max_rows, res, pl->mode == GSMAT_PLAN_ADAPTIVE, {},
          mem, (PinnedArea*)dev_area};
  Table unit;
  unit.n = 1;
  unit.k = 0;
  const uint32_t all = pl->pats.size() >= 32 ? 0xFFFFFFFFu : ((1u << pl->pats.size()) - 1);
  try {
    ex.run(0, unit, all);
  } catch (...) {
    ex.release_all();
    throw;
  }
}

void run_collect(gsmat_store* st, const gsmat_query_plan* pl, const Table* t0,
                 int64_t budget_bytes, hipStream_t s, std::vector<Table>* out) {
  for (const gsmat_pattern& q : pl->pats) {
    if (q.p >= st->P) return;
    if (!is_var(q.s) && q.s >= st->V) return;
    if (!is_var(q.o) && q.o >= st->V) return;
  }
  gsmat_result counters;  // step counters only (no steps kept)
  counters.st = st;
  counters.stream = s;
  Exec ex{st, pl, s, budget_bytes, -1, &counters, true, {}, nullptr, nullptr, out};
  Table t;
  if (t0) {
    if (t0->owned) throw StatusFail{GSMAT_EHIP, "internal: a starting table must not own memory"};
    t = *t0;
  } else {
    t.n = 1;
    t.k = 0;
  }
  const size_t first = out->size();
  const uint32_t all = pl->pats.size() >= 32 ? 0xFFFFFFFFu : ((1u << pl->pats.size()) - 1);
  try {
    ex.run(0, t, all);
  } catch (...) {
    ex.release_all();
    for (size_t i = first; i < out->size(); ++i)
      if ((*out)[i].owned) st->mem->free((*out)[i].owned, (*out)[i].owned_bytes, s);
    out->resize(first);
    throw;
  }
}

// Statistics of each pattern for the planner.
std::vector<TpStat> pattern_stats(const gsmat_store* st, const gsmat_pattern* pats, int n,
                                  int mode, hipStream_t s, std::vector<gsmat_pat_lookup>* lk) {
  std::vector<TpStat> out(n);
  if (lk) lk->assign(n, gsmat_pat_lookup{});
  std::vector<LookupReq> reqs;
  std::vector<int> req_of(n, -1);
  for (int i = 0; i < n; ++i) {
    const gsmat_pattern& q = pats[i];
    TpStat& t = out[i];
    if (q.p < 0 || q.p >= st->P) continue;  // absent predicate: empty relation
    const PredDesc& dout = st->out.desc[q.p];
    const PredDesc& din = st->in.desc[q.p];
    t.stat = dout.nnz;
    t.rows_s = dout.nr;
    t.rows_o = din.nr;
    if (mode == GSMAT_PLAN_PAPER) continue;
    const bool sc = !is_var(q.s), oc = !is_var(q.o);
    if ((sc && q.s >= st->V) || (oc && q.o >= st->V)) {
      t.stat = t.rows_s = t.rows_o = 0;
      continue;
    }
    if (sc && oc) {
      req_of[i] = (int)reqs.size();
      reqs.push_back({0, q.p, q.s, q.o});
    } else if (sc) {
      req_of[i] = (int)reqs.size();
      reqs.push_back({0, q.p, q.s, -1});
    } else if (oc) {
      req_of[i] = (int)reqs.size();
      reqs.push_back({1, q.p, q.o, -1});
    }
  }
  if (!reqs.empty()) {
    LookupBatch b{};
    for (size_t i = 0; i < reqs.size(); ++i) b.req[i] = reqs[i];
    b.n = (int32_t)reqs.size();
    PinnedArea* h = pinned();
    launch_lookup(b, st->out.d_desc, st->in.d_desc, st->out.ptrs(), st->in.ptrs(), h->res, s);
    host_sync(s);
    std::vector<LookupRes> res(h->res, h->res + reqs.size());
    for (int i = 0; i < n; ++i) {
      if (req_of[i] < 0) continue;
      const LookupRes& r = res[req_of[i]];
      if (lk) (*lk)[i] = gsmat_pat_lookup{r.start, r.len, r.found, 1};
      const gsmat_pattern& q = pats[i];
      const bool sc = !is_var(q.s), oc = !is_var(q.o);
      const int64_t v = (sc && oc) ? r.found : r.len;
      out[i].stat = v;
      out[i].rows_s = v;
      out[i].rows_o = v;
    }
  }
  return out;
}

}  // namespace gsmat

extern "C" gsmat_status gsmat_plan(const gsmat_store* st, const gsmat_pattern* pats,
                                   int32_t n_pats, int32_t mode, void* stream, gsmat_query_plan** out) {
  return guarded([&]() -> gsmat_status {
    if (!out) throw StatusFail{GSMAT_EINVAL, "out is NULL"};
    *out = nullptr;
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    std::string err;
    int32_t nv = 0;
    gsmat_status rc = validate_patterns(pats, n_pats, &nv, &err);
    if (rc != GSMAT_OK) throw StatusFail{rc, err};
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    std::vector<gsmat_pat_lookup> lk;
    std::vector<TpStat> ts = pattern_stats(st, pats, n_pats, mode, (hipStream_t)stream, &lk);
    std::unique_ptr<gsmat_query_plan> pl(new gsmat_query_plan);
    rc = build_plan(pats, n_pats, mode, ts.data(), pl.get(), &err);
    if (rc != GSMAT_OK) throw StatusFail{rc, err};
    if (mode != GSMAT_PLAN_PAPER) {
      pl->lk = std::move(lk);
      pl->lk_store = st->uid;
    }
    *out = pl.release();
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_join(gsmat_store* st, const gsmat_query_plan* pl, int64_t budget_bytes,
                                   int64_t max_rows, void* stream, gsmat_result** out) {
  return guarded([&]() -> gsmat_status {
    if (!out) throw StatusFail{GSMAT_EINVAL, "out is NULL"};
    *out = nullptr;
    if (!st || !pl) throw StatusFail{GSMAT_EINVAL, "store or plan is NULL"};
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<gsmat_result> res(new gsmat_result);
    res->st = st;
    res->stream = s;
    res->n_vars = pl->n_vars;
    res->reset_steps(pl->steps.size());
    run_query(st, pl, budget_bytes, max_rows, s, res.get());
    GS_HIP(hipStreamSynchronize(s));
    *out = res.release();
    return GSMAT_OK;
  });
}

// ---------------------------------------------------------- allocation-free join
//
// gsmat_join_noalloc keeps every intermediate table and every step's scratch
// in one file-scope device array of kNoAllocBytes (each GPU the library runs
// on has its own copy, held until the process ends).  Host code never uses
// the array's name as a device address: the address comes from
// hipGetSymbolAddress, taken once per device with that device current.

namespace {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

struct NoAllocDevice {
  std::mutex mu;          // serialises the calls on this device
  char* base = nullptr;   // the array's device address
};

NoAllocDevice* noalloc_device(int dev) {
  static std::mutex mu;
  static std::map<int, NoAllocDevice*> devs;
  std::lock_guard<std::mutex> g(mu);
  NoAllocDevice*& d = devs[dev];
  if (!d) {
    std::unique_ptr<NoAllocDevice> nd(new NoAllocDevice);
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw StatusFail{GSMAT_EHIP, std::string("no-alloc scratch: hipGetSymbolAddress failed: ") +
                                       hipGetErrorString(e)};
    nd->base = (char*)p;
    d = nd.release();
  }
  return d;
}

// Stack allocator over the array: blocks come off the top; a free marks its
// block, and the top drops past every freed block at the top (the executor
// frees in nearly reverse order).  The first kStageBytes hold the staged
// small results.
struct ScratchStack {
  char* base = nullptr;
  size_t top = kStageBytes;
  size_t want = 0;  // largest request that did not fit
  std::vector<size_t> off, len;
  std::vector<char> freed;

  void* alloc(size_t bytes) {
    const size_t b = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    if (b > kNoAllocBytes - top) {
      want = std::max(want, b);
      return nullptr;
    }
    off.push_back(top);
    len.push_back(b);
    freed.push_back(0);
    void* p = base + top;
    top += b;
    return p;
  }
  void free(void* p) {
    const size_t o = (size_t)((char*)p - base);
    for (size_t i = off.size(); i-- > 0;)
      if (off[i] == o && !freed[i]) {
        freed[i] = 1;
        break;
      }
    while (!off.empty() && freed.back()) {
      top = off.back();
      off.pop_back();
      len.pop_back();
      freed.pop_back();
    }
  }
  static void* alloc_cb(size_t bytes, void* stream, void* ctx) {
    (void)stream;
    return ((ScratchStack*)ctx)->alloc(bytes);
  }
  static void free_cb(void* p, size_t bytes, void* stream, void* ctx) {
    (void)bytes;
    (void)stream;
    ((ScratchStack*)ctx)->free(p);
  }
};

}  // namespace

extern "C" gsmat_status gsmat_join_noalloc(gsmat_store* st, const gsmat_query_plan* pl,
                                           int32_t* out, int64_t out_stride, int64_t out_cap,
                                           int64_t* n_rows, void* stream) {
  return guarded([&]() -> gsmat_status {
    if (!st || !pl || !n_rows) throw StatusFail{GSMAT_EINVAL, "store, plan or n_rows is NULL"};
    *n_rows = 0;
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    if (out_cap < 0 || out_stride < out_cap)
      throw StatusFail{GSMAT_EINVAL, "out_cap must be >= 0 and out_stride >= out_cap"};
    if (!out && out_cap > 0 && pl->n_vars > 0) throw StatusFail{GSMAT_EINVAL, "out is NULL"};
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    GS_HIP(hipGetDevice(&dev));
    NoAllocDevice* nd = noalloc_device(dev);
    std::lock_guard<std::mutex> lock(nd->mu);
    ScratchStack stack;
    stack.base = nd->base;
    const gsmat_allocator a{&ScratchStack::alloc_cb, &ScratchStack::free_cb, &stack};
    DeviceMem mem(&a);
    gsmat_result res;
    res.st = st;
    res.stream = s;
    res.n_vars = pl->n_vars;
    res.reset_steps(pl->steps.size());
    struct Drop {  // the segments live in the array: nothing to free
      gsmat_result& r;
      ~Drop() {
        for (Segment& g : r.segs) g.owned = nullptr;
      }
    } drop{res};
    try {
      run_query(st, pl, 0, -1, s, &res, &mem, nd->base);
    } catch (const OomFail&) {
      (void)hipStreamSynchronize(s);  // nothing may still use the array
      throw StatusFail{GSMAT_ENOMEM,
                       "the join needs more than the " + std::to_string(kNoAllocBytes >> 20) +
                           " MiB of the allocation-free scratch (a block of " +
                           std::to_string(stack.want) + " bytes did not fit)"};
    } catch (...) {
      (void)hipStreamSynchronize(s);
      throw;
    }
    *n_rows = res.rows;
    if (res.rows > out_cap) {
      host_sync(s);
      throw StatusFail{GSMAT_ETOOBIG, "result has " + std::to_string(res.rows) +
                                          " rows, more than out_cap (" + std::to_string(out_cap) +
                                          ")"};
    }
    int64_t at = 0;
    for (const Segment& g : res.segs) {
      for (int v = 0; v < pl->n_vars && g.rows > 0; ++v)
        GS_HIP(hipMemcpyAsync(out + (int64_t)v * out_stride + at, g.col[v],
                              sizeof(int32_t) * (size_t)g.rows, hipMemcpyDeviceToDevice, s));
      at += g.rows;
    }
    // the array is reused by the next call: its work ends before this returns
    host_sync(s);
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_result_info(const gsmat_result* r, int64_t* n_rows, int32_t* n_vars,
                                          int32_t* n_steps, int64_t* step_rows_in,
                                          int64_t* step_rows_out) {
  return guarded([&]() -> gsmat_status {
    if (!r) throw StatusFail{GSMAT_EINVAL, "result is NULL"};
    if (n_rows) *n_rows = r->rows;
    if (n_vars) *n_vars = r->n_vars;
    if (n_steps) *n_steps = r->n_steps;
    if (step_rows_in) std::copy(r->step_in, r->step_in + r->n_steps, step_rows_in);
    if (step_rows_out) std::copy(r->step_out, r->step_out + r->n_steps, step_rows_out);
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_fetch_bindings(const gsmat_result* r, int64_t row_offset,
                                             int64_t max_rows, int32_t* host_rows,
                                             int64_t* n_written, void* stream) {
  return guarded([&]() -> gsmat_status {
    if (!r) throw StatusFail{GSMAT_EINVAL, "result is NULL"};
    if (row_offset < 0 || max_rows < 0) throw StatusFail{GSMAT_EINVAL, "negative offset or count"};
    const int64_t lo = std::min(row_offset, r->rows);
    const int64_t hi = std::min(r->rows, lo + max_rows);
    if (n_written) *n_written = hi - lo;
    const int nv = r->n_vars;
    if (hi <= lo || nv == 0) return GSMAT_OK;
    if (!host_rows) throw StatusFail{GSMAT_EINVAL, "host_rows is NULL"};
    hipStream_t s = (hipStream_t)stream;
    DeviceMem* mem = r->st->mem.get();
    const int64_t stage_rows = std::min<int64_t>(hi - lo, (int64_t)1 << 24);
    Tmp<int32_t> stage(mem, stage_rows * nv, s);
    int64_t seg_lo = 0;
    int64_t written = 0;
    for (const Segment& seg : r->segs) {
      const int64_t seg_hi = seg_lo + seg.rows;
      int64_t a = std::max(lo, seg_lo), b = std::min(hi, seg_hi);
      while (a < b) {
        const int64_t c = std::min(b - a, stage_rows);
        ColSet cs{};
        for (int v = 0; v < nv; ++v) cs.c[v] = seg.col[v];
        launch_pack_rows(cs, nv, a - seg_lo, c, stage.p, s);
        GS_HIP(hipMemcpyAsync(host_rows + written * nv, stage.p, sizeof(int32_t) * c * nv,
                              hipMemcpyDeviceToHost, s));
        GS_HIP(hipStreamSynchronize(s));
        written += c;
        a += c;
      }
      seg_lo = seg_hi;
    }
    return GSMAT_OK;
  });
}

extern "C" void gsmat_result_free(gsmat_result* r) { delete r; }
