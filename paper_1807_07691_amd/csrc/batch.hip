// Batched join: many BGP plans evaluated together, one step of every query
// per round (paper Sec. 7.2 evaluates one plan step as count, prefix sum,
// exact allocation and write; here each of those phases is one launch for the
// whole batch).
//
// A round takes the next step of every unfinished query: expansions, filters
// and star-centre intersections become tasks of one count/flag launch whose
// tiles are the concatenation of every task's tiles; one scan of all tile
// sums and one per-task reduction give every task's output size, read back
// with a single wait.  The host then allocates one arena for all outputs of
// the round and issues one prefix-sum launch, one merge-path partition
// launch, and one write (expansions) or compaction (filters, intersections)
// launch per column count.  Expansions in which few input rows have output
// first compact those rows (their offsets come from the same prefix sum) and
// are written by a variant that walks only them; the fill threshold is the
// store's, set directly or by the autotuner at the end of this file.  Steps
// needing no kernel (pattern scans, which are views into the store) are
// applied on the host.  The adaptive step choice samples every query's
// candidate expansions in one launch per round.  A query whose next step
// would be a Cartesian product, a (?x p ?x) scan, or an output above the byte
// budget leaves the batch and is run on its own by the single-query
// executor, which handles those cases.  The serving loop (gsmat_server_*)
// keeps a batch alive across calls and admits new queries between rounds.
//
// Each query takes exactly the steps it takes alone (same plan, same choice
// rule on the same tables), so its result rows come out in the same order.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <memory>

#include "batch.hpp"
#include "exec.hpp"
#include "host_pool.hpp"

using namespace gsmat;

namespace {

// ---------------------------------------------------------------- host side

// Growable pinned host buffer (per thread and purpose).  A buffer is only
// rewritten after the stream has synchronised past the copy that read it.
struct Pinned {
  void* p = nullptr;
  size_t bytes = 0;
  void* get(size_t want) {
    if (want <= bytes) return p;
    if (p) GS_HIP(hipHostFree(p));
    p = nullptr;
    bytes = 0;
    size_t b = 1 << 16;
    while (b < want) b <<= 1;
    GS_HIP(hipHostMalloc(&p, b, hipHostMallocDefault));
    bytes = b;
    return p;
  }
};
enum { kPinCount = 0, kPinWrite, kPinSample, kPinTotals, kPinParts, kPinLookup, kPinCount_ };
// Per slot (a batch may use its own set).
Pinned* pins(int slot = 0) {
  thread_local Pinned p[2][kPinCount_];
  return p[slot];
}

// An event owned by one batch (created on first use).
struct Event {
  hipEvent_t e = nullptr;
  Event() = default;
  Event(const Event&) = delete;
  Event& operator=(const Event&) = delete;
  ~Event() {
    if (e) (void)hipEventDestroy(e);
  }
  hipEvent_t get() {
    if (!e) GS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return e;
  }
};

// Byte layout of several device slices inside one arena (256-byte aligned).
struct Layout {
  size_t bytes = 0;
  size_t add(size_t b) {
    const size_t at = bytes;
    bytes += (b + 255) / 256 * 256;
    return at;
  }
};

// Batched lookups: one launch and one synchronisation for all requests.
std::vector<LookupRes> lookup_many(const gsmat_store* st, const std::vector<LookupReq>& req,
                                   hipStream_t s) {
  std::vector<LookupRes> out(req.size());
  if (req.empty()) return out;
  const size_t n = req.size();
  if (n <= (size_t)kMaxLookups) {  // few requests: passed by value, no upload
    LookupBatch b{};
    for (size_t i = 0; i < n; ++i) b.req[i] = req[i];
    b.n = (int32_t)n;
    LookupRes* hres = (LookupRes*)pins()[kPinTotals].get(sizeof(LookupRes) * n);
    launch_lookup(b, st->out.d_desc, st->in.d_desc, st->out.ptrs(), st->in.ptrs(), hres, s);
    host_sync(s);
    std::memcpy(out.data(), hres, sizeof(LookupRes) * n);
    return out;
  }
  Layout L;
  const size_t o_req = L.add(sizeof(LookupReq) * n);
  Arena a(st->mem.get(), L.bytes, s);
  char* dev = (char*)a.p;
  LookupReq* hreq = (LookupReq*)pins()[kPinLookup].get(sizeof(LookupReq) * n);
  LookupRes* hres = (LookupRes*)pins()[kPinTotals].get(sizeof(LookupRes) * n);
  std::memcpy(hreq, req.data(), sizeof(LookupReq) * n);
  GS_HIP(hipMemcpyAsync(dev + o_req, hreq, sizeof(LookupReq) * n, hipMemcpyHostToDevice, s));
  launch_lookup_many((const LookupReq*)(dev + o_req), (int32_t)n, st->out.d_desc, st->in.d_desc,
                     st->out.ptrs(), st->in.ptrs(), hres, s);
  host_sync(s);
  std::memcpy(out.data(), hres, sizeof(LookupRes) * n);
  return out;
}

enum QState { kActive, kDone, kFallback, kFailed };


struct BQ {
  const gsmat_query_plan* pl = nullptr;
  std::unique_ptr<gsmat_result> res;
  Table t;
  uint32_t rem = 0;
  int si = 0;
  QState state = kActive;
  gsmat_status status = GSMAT_OK;
  std::string err;
  gsmat_step_info sp{};
  uint32_t next = 0;
  LookupRes lk[kMaxPats];  // row lookup of each pattern with a constant
  int64_t tag = 0;         // caller's id (server)
  int64_t est_bytes = 0;   // admission estimate (server)
  int cand0 = -1;       // first sampled candidate this round
  StepChoice choice;
  // pending task output (intersection result before it is combined)
  int new_var = -1;
};

struct Batch {
  gsmat_store* st;
  hipStream_t s;
  int64_t budget;
  int64_t max_rows;
  std::vector<BQ> q;
  int64_t round_budget = 0;    // outputs of one round (<= 0: none)
  bool defer = false;          // over the round budget: wait a round (else run alone)
  int slot = 0;                // pinned buffer set
  Event ev;                    // end of the last phase's launches

  // state of the round in progress, carried from one phase to the next
  struct Round {
    bool sampled = false;
    int64_t* hp = nullptr;  // fan-out sample partials (pinned)
    int nt = 0;             // tasks of the count launch
    int64_t ntiles = 0;
    std::vector<CTask> tasks;
    std::vector<int> owner;  // query of each task
    std::vector<GItem> items;
    std::vector<size_t> o_P;
    std::shared_ptr<Arena> A;  // count-phase scratch
    int64_t* ts = nullptr;
    int64_t* tsn = nullptr;  // rows with output per count tile (expansions)
    int64_t* htot = nullptr;
  } R;
  // expansions of at least sparse_min_rows input rows of which fewer than
  // this fraction have output walk only those rows (0: never)
  double sparse_theta = 0.0;
  int64_t sparse_min_rows = 4096;

  DeviceMem* mem() { return st->mem.get(); }

  void add_in(BQ& b, int64_t n) {
    if (b.si < b.res->n_steps) b.res->step_in[b.si] += n;
  }
  void add_out(BQ& b, int64_t m) {
    if (b.si < b.res->n_steps) b.res->step_out[b.si] += m;
  }

  void fail(BQ& b, gsmat_status st_, const std::string& msg) {
    b.state = kFailed;
    b.status = st_;
    b.err = msg;
    b.t = Table();
    b.res.reset();
  }

  // Emits the finished table as the query's result.
  void emit(BQ& b) {
    const Table& t = b.t;
    const int nv = b.pl->n_vars;
    Segment seg;
    seg.rows = t.n;
    for (int v = 0; v < nv; ++v) {
      const int c = t.col_of(v);
      if (c < 0) throw StatusFail{GSMAT_EHIP, "internal: unbound variable at the end of the plan"};
      seg.col[v] = t.col[c];
    }
    seg.keep = t.keep;
    b.res->rows += seg.rows;
    b.res->segs.push_back(seg);
    b.state = kDone;
    b.t = Table();
    if (max_rows >= 0 && b.res->rows > max_rows)
      fail(b, GSMAT_ETOOBIG, "result exceeds max_rows (" + std::to_string(max_rows) + ")");
  }

  // The query moves on with table t: the next step index, the patterns left.
  void advance(BQ& b, Table t) {
    b.t = std::move(t);
    b.rem = b.next;
    b.si += 1;
    if (b.t.n == 0) {
      b.state = kDone;
      b.t = Table();
    } else if (b.rem == 0) {
      emit(b);
    }
  }

  // Relation of one pattern as a view into the store (a scan step on the unit
  // table); false when it is not a plain view (the (?x p ?x) diagonal).
  bool scan_view(BQ& b, int tp, Table& t) {
    const gsmat_pattern& p = b.pl->pats[tp];
    if (is_var(p.s) && is_var(p.o)) {
      if (p.s == p.o) return false;
      const PredView pv = st->out.view(p.p);
      t.n = pv.nnz;
      t.k = 2;
      t.col[0] = pv.src;
      t.var[0] = var_of(p.s);
      t.col[1] = pv.nbr;
      t.var[1] = var_of(p.o);
      return true;
    }
    const LookupRes& r = b.lk[tp];
    if (!is_var(p.s) && is_var(p.o)) {
      t.n = r.len;
      t.k = 1;
      t.col[0] = st->out.view(p.p).nbr + r.start;
      t.var[0] = var_of(p.o);
    } else if (is_var(p.s) && !is_var(p.o)) {
      t.n = r.len;
      t.k = 1;
      t.col[0] = st->in.view(p.p).nbr + r.start;
      t.var[0] = var_of(p.s);
    } else {
      t.n = r.found ? 1 : 0;
      t.k = 0;
    }
    return true;
  }

  void admit(size_t first);
  void run();
  // One round in three phases, each ending with launches and an event the
  // next phase waits for.  (Interleaving the phases of two half batches on one
  // stream was measured slower: half-size launches cost more than the overlap
  // of host work saves.)
  bool phase_sample();  // false when no query is active
  void phase_count();
  void phase_write();
  void round() {
    if (phase_sample()) {
      phase_count();
      phase_write();
    }
  }
};

// Constant lookups of queries [first, q.size()): the plan's where it made
// them on this store, the rest in one launch.
void Batch::admit(size_t first) {
  std::vector<LookupReq> req;
  std::vector<LookupRes*> req_at;
  for (size_t i = first; i < q.size(); ++i) {
    BQ& b = q[i];
    if (b.state != kActive) continue;
    const gsmat_query_plan* pl = b.pl;
    const bool have = pl->lk_store == st->uid && pl->lk.size() == pl->pats.size();
    for (int tp = 0; tp < (int)pl->pats.size(); ++tp) {
      const gsmat_pattern& p = pl->pats[tp];
      const bool sc = !is_var(p.s), oc = !is_var(p.o);
      if (!sc && !oc) continue;
      if (have && pl->lk[tp].valid) {
        const gsmat_pat_lookup& l = pl->lk[tp];
        b.lk[tp] = LookupRes{l.start, l.len, l.found, 0};
        continue;
      }
      req_at.push_back(&b.lk[tp]);
      if (sc && oc) req.push_back({0, p.p, p.s, p.o});
      else if (sc) req.push_back({0, p.p, p.s, -1});
      else req.push_back({1, p.p, p.o, -1});
    }
  }
  if (req.empty()) return;
  const std::vector<LookupRes> r = lookup_many(st, req, s);
  for (size_t j = 0; j < r.size(); ++j) *req_at[j] = r[j];
}

void Batch::run() {
  admit(0);
  for (;;) {
    bool any = false;
    for (const BQ& b : q) any |= b.state == kActive;
    if (!any) break;
    round();
  }
}

bool Batch::phase_sample() {
  // ---- step choice (adaptive queries sample their candidate expansions)
  R = Round();
  bool any = false;
  std::vector<SCand> cands;
  for (BQ& b : q) {
    if (b.state != kActive) continue;
    any = true;
    b.cand0 = -1;
    const gsmat_query_plan* pl = b.pl;
    if (pl->mode == GSMAT_PLAN_ADAPTIVE && !b.t.unit()) {
      step_candidates(st, pl, b.t, b.rem, b.choice);
      const StepChoice& c = b.choice;
      if (c.has_filter) b.sp = c.filter;
      else if (c.nc == 0) b.sp = c.cartesian;
      else if (c.nc == 1) b.sp = step_pick(pl, c, nullptr);
      else {
        b.cand0 = (int)cands.size();
        for (int i = 0; i < c.nc; ++i) {
          SCand sc;
          candidate_view(st, pl, b.t, c, i, &sc.col, &sc.pv);
          sc.n = b.t.n;
          cands.push_back(sc);
        }
      }
    } else {
      b.sp = pl->steps[std::min<size_t>(b.si, pl->steps.size() - 1)];
    }
  }
  if (!cands.empty()) {
    const size_t nc = cands.size();
    Layout L;
    const size_t o_c = L.add(sizeof(SCand) * nc);
    Arena a(mem(), L.bytes, s);  // freed in stream order after the launch
    SCand* hc = (SCand*)pins(slot)[kPinSample].get(sizeof(SCand) * nc);
    R.hp = (int64_t*)pins(slot)[kPinParts].get(sizeof(int64_t) * nc * kSampleBlocks);
    std::memcpy(hc, cands.data(), sizeof(SCand) * nc);
    GS_HIP(hipMemcpyAsync((char*)a.p + o_c, hc, sizeof(SCand) * nc, hipMemcpyHostToDevice, s));
    launch_b_sample((const SCand*)((char*)a.p + o_c), (int64_t)nc, R.hp, s);
    GS_HIP(hipEventRecord(ev.get(), s));
    R.sampled = true;
  }
  return any;
}

void Batch::phase_count() {
  const int nq = (int)q.size();
  if (R.sampled) {
    host_event_sync(ev.get());
    const int64_t* hp = R.hp;
    for (BQ& b : q) {
      if (b.state != kActive || b.cand0 < 0) continue;
      int64_t sum[kMaxPats];
      for (int i = 0; i < b.choice.nc; ++i) {
        sum[i] = 0;
        for (int j = 0; j < kSampleBlocks; ++j) sum[i] += hp[(size_t)(b.cand0 + i) * kSampleBlocks + j];
      }
      b.sp = step_pick(b.pl, b.choice, sum);
    }
  }

  // ---- count phase: tasks
  std::vector<CTask>& tasks = R.tasks;
  std::vector<int>& owner = R.owner;
  std::vector<ListRef> lists;
  for (int qi = 0; qi < nq; ++qi) {
    BQ& b = q[qi];
    if (b.state != kActive) continue;
    const gsmat_query_plan* pl = b.pl;
    const gsmat_step_info& sp = b.sp;
    b.next = b.rem & ~step_completes(pl, sp);
    add_in(b, b.t.n);
    const gsmat_pattern& p = pl->pats[sp.tp];
    switch (sp.kind) {
      case GSMAT_STEP_SCAN:
      case GSMAT_STEP_CARTESIAN: {
        Table r;
        if (!b.t.unit() || !scan_view(b, sp.tp, r)) {
          b.state = kFallback;
          break;
        }
        add_out(b, r.n);
        advance(b, r);
        break;
      }
      case GSMAT_STEP_INTERSECT: {
        if (!b.t.unit()) {
          b.state = kFallback;
          break;
        }
        const int32_t cterm = -(sp.var + 1);
        ListRef ls[kMaxLists];
        const int32_t* ids[kMaxLists];
        int nl = 0;
        for (int tp = 0; tp < (int)pl->pats.size(); ++tp) {
          if (!(sp.members >> tp & 1)) continue;
          const gsmat_pattern& m = pl->pats[tp];
          ListRef l{};
          if (m.s == cterm && is_var(m.o)) {
            l.pv = st->out.view(m.p);
            l.is_keys = 1;
            l.len = l.pv.nr;
            ids[nl] = l.pv.keys;
          } else if (m.o == cterm && is_var(m.s)) {
            l.pv = st->in.view(m.p);
            l.is_keys = 1;
            l.len = l.pv.nr;
            ids[nl] = l.pv.keys;
          } else if (m.s == cterm) {
            const LookupRes& r = b.lk[tp];
            l.seg = st->in.view(m.p).nbr + r.start;
            l.bm = st->in.row_bitmap(m.p, m.o);
            l.len = r.len;
            ids[nl] = l.seg;
          } else {
            const LookupRes& r = b.lk[tp];
            l.seg = st->out.view(m.p).nbr + r.start;
            l.bm = st->out.row_bitmap(m.p, m.s);
            l.len = r.len;
            ids[nl] = l.seg;
          }
          ls[nl++] = l;
        }
        int d = 0;
        for (int i = 1; i < nl; ++i)
          if (ls[i].len < ls[d].len) d = i;
        if (ls[d].len == 0) {
          add_out(b, 0);
          b.state = kDone;
          b.t = Table();
          break;
        }
        CTask c{};
        c.kind = kTaskIntersect;
        c.n = ls[d].len;
        c.col = ids[d];
        c.l0 = (int32_t)lists.size();
        for (int i = 0; i < nl; ++i)
          if (i != d) lists.push_back(ls[i]);
        c.nl = (int32_t)lists.size() - c.l0;
        b.new_var = sp.var;
        tasks.push_back(c);
        owner.push_back(qi);
        break;
      }
      case GSMAT_STEP_FILTER: {
        if (!is_var(p.s) && !is_var(p.o)) {
          if (b.lk[sp.tp].found) {
            add_out(b, b.t.n);
            advance(b, b.t);
          } else {
            b.state = kDone;
            b.t = Table();
          }
          break;
        }
        CTask c{};
        c.kind = kTaskFilter;
        c.n = b.t.n;
        if (is_var(p.s)) c.pa.s_col = b.t.col[b.t.col_of(var_of(p.s))];
        else c.pa.s_const = p.s;
        if (is_var(p.o)) c.pa.o_col = b.t.col[b.t.col_of(var_of(p.o))];
        else c.pa.o_const = p.o;
        c.pv = st->out.view(p.p);
        tasks.push_back(c);
        owner.push_back(qi);
        break;
      }
      case GSMAT_STEP_EXPAND: {
        const int bound_var = sp.orient == 0 ? var_of(p.s) : var_of(p.o);
        const int bc = b.t.col_of(bound_var);
        if (bc < 0 || b.t.k + 1 > kMaxCols) {
          b.state = kFallback;  // the single-query executor reports it
          break;
        }
        CTask c{};
        c.kind = kTaskExpand;
        c.n = b.t.n;
        c.col = b.t.col[bc];
        c.pv = sp.orient == 0 ? st->out.view(p.p) : st->in.view(p.p);
        b.new_var = sp.orient == 0 ? var_of(p.o) : var_of(p.s);
        tasks.push_back(c);
        owner.push_back(qi);
        break;
      }
      default:
        b.state = kFallback;
    }
  }
  const int nt = (int)tasks.size();
  R.nt = nt;
  if (nt == 0) return;

  // scratch of the count phase
  int64_t ntiles = 0;
  std::vector<GItem>& items = R.items;
  items.resize(nt);
  Layout LA;
  std::vector<size_t>& o_P = R.o_P;
  o_P.resize(nt);
  std::vector<size_t> o_N(nt), o_start(nt), o_flags(nt);
  for (int i = 0; i < nt; ++i) {
    items[i] = GItem{ntiles, i, 0};
    ntiles += ceil_div(tasks[i].n, kTile);
    const int64_t n = tasks[i].n;
    if (tasks[i].kind == kTaskExpand) {
      o_N[i] = LA.add(sizeof(int32_t) * n);
      o_start[i] = LA.add(sizeof(int32_t) * n);
      o_P[i] = LA.add(sizeof(int64_t) * (n + 1));
    } else {
      o_flags[i] = LA.add((size_t)n);
    }
  }
  const size_t o_ts = LA.add(sizeof(int64_t) * (ntiles + 1));
  const size_t o_tsn = LA.add(sizeof(int64_t) * (ntiles + 1));
  // uploaded together: tasks, items, lists, then the zeroed non-empty counters
  const size_t o_tasks = LA.add(sizeof(CTask) * nt);
  const size_t o_items = LA.add(sizeof(GItem) * nt);
  const size_t o_lists = LA.add(sizeof(ListRef) * std::max<size_t>(lists.size(), 1));
  const size_t o_ne = LA.add(sizeof(int64_t) * nt);
  R.A = std::make_shared<Arena>(mem(), LA.bytes, s);
  char* da = (char*)R.A->p;
  int64_t* dne = (int64_t*)(da + o_ne);
  for (int i = 0; i < nt; ++i) {
    if (tasks[i].kind == kTaskExpand) {
      tasks[i].N = (int32_t*)(da + o_N[i]);
      tasks[i].start = (int32_t*)(da + o_start[i]);
      tasks[i].nonempty = dne + i;
    } else {
      tasks[i].flags = (uint8_t*)(da + o_flags[i]);
    }
  }
  int64_t* ts = (int64_t*)(da + o_ts);
  int64_t* tsn = (int64_t*)(da + o_tsn);
  {
    const size_t up = o_ne + sizeof(int64_t) * nt - o_tasks;
    char* h = (char*)pins(slot)[kPinCount].get(up);
    std::memcpy(h, tasks.data(), sizeof(CTask) * nt);
    std::memcpy(h + (o_items - o_tasks), items.data(), sizeof(GItem) * nt);
    if (!lists.empty()) std::memcpy(h + (o_lists - o_tasks), lists.data(), sizeof(ListRef) * lists.size());
    std::memset(h + (o_ne - o_tasks), 0, sizeof(int64_t) * nt);
    GS_HIP(hipMemcpyAsync(da + o_tasks, h, up, hipMemcpyHostToDevice, s));
  }
  int64_t* htot = (int64_t*)pins(slot)[kPinTotals].get(2 * sizeof(int64_t) * nt);
  const CTask* dtasks = (const CTask*)(da + o_tasks);
  const GItem* ditems = (const GItem*)(da + o_items);
  launch_b_count(dtasks, ditems, nt, (const ListRef*)(da + o_lists), ts, tsn, ntiles,
                 20.0 * ntiles * kTile, s);
  launch_scan_tile_sums2(ts, tsn, ntiles, s);
  launch_b_totals(ditems, nt, ts, ntiles, dne, htot, s);
  GS_HIP(hipEventRecord(ev.get(), s));
  R.ntiles = ntiles;
  R.ts = ts;
  R.tsn = tsn;
  R.htot = htot;
}

void Batch::phase_write() {
  const int nt = R.nt;
  if (nt == 0) return;
  host_event_sync(ev.get());
  const std::vector<CTask>& tasks = R.tasks;
  const std::vector<int>& owner = R.owner;
  const std::vector<GItem>& items = R.items;
  const std::vector<size_t>& o_P = R.o_P;
  char* da = (char*)R.A->p;
  int64_t* ts = R.ts;
  const int64_t* htot = R.htot;
  std::vector<int64_t> tot(htot, htot + nt), nonempty(htot + nt, htot + 2 * nt);

  // ---- write phase: outputs
  std::vector<WTask> w(nt);
  std::vector<int> has_out(nt, 0);
  Layout LB;  // output tables (kept by the next tables / results)
  std::vector<size_t> o_out(nt);
  int64_t round_bytes = 0;
  for (int i = 0; i < nt; ++i) {
    BQ& b = q[owner[i]];
    const CTask& c = tasks[i];
    const int64_t m = tot[i];
    WTask& wt = w[i];
    wt.n = c.n;
    wt.m = m;
    wt.t0 = items[i].w0;
    int kout = 0;
    if (c.kind == kTaskExpand) {
      if (m == 0) {
        add_out(b, 0);
        b.state = kDone;
        b.t = Table();
        continue;
      }
      kout = b.t.k + 1;
    } else if (c.kind == kTaskFilter) {
      if (m == c.n) {  // nothing removed: the table goes on unchanged
        add_out(b, m);
        advance(b, b.t);
        continue;
      }
      if (m == 0) {
        add_out(b, 0);
        b.state = kDone;
        b.t = Table();
        continue;
      }
      kout = b.t.k;
    } else {
      if (m == c.n) {  // every driver id survives: the driver list itself
        Table r;
        r.n = m;
        r.k = 1;
        r.col[0] = c.col;
        r.var[0] = b.new_var;
        add_out(b, r.n);
        advance(b, r);
        continue;
      }
      if (m == 0) {
        add_out(b, 0);
        b.state = kDone;
        b.t = Table();
        continue;
      }
      kout = 1;
    }
    const size_t bytes = sizeof(int32_t) * (size_t)col_stride(m) * (size_t)kout;
    if (budget > 0 && m > budget / (4 * (int64_t)std::max(kout, 1))) {
      // above the step budget: chunked by the single-query executor
      b.state = kFallback;
      b.t = Table();
      continue;
    }
    if (round_budget > 0 && round_bytes > 0 && round_bytes + (int64_t)bytes > round_budget) {
      if (defer) {
        // the round is full: this query repeats the step next round
        if (b.si < b.res->n_steps) b.res->step_in[b.si] -= b.t.n;
        continue;
      }
      b.state = kFallback;
      b.t = Table();
      continue;
    }
    if (c.kind != kTaskIntersect) add_out(b, m);
    round_bytes += (int64_t)bytes;
    o_out[i] = LB.add(bytes);
    has_out[i] = 1;
  }
  std::shared_ptr<Arena> B;
  if (LB.bytes > 0) B = std::make_shared<Arena>(mem(), LB.bytes, s);

  // expansion scratch (splits, compacted rows) and launch groups
  Layout LC;
  std::vector<size_t> o_split(nt), o_ridx(nt), o_cstart(nt), o_cP(nt);
  std::vector<char> sparse(nt, 0);
  std::vector<GItem> g_scan, g_crow, g_part, g_write[kMaxK + 2], g_wi[kMaxK + 2],
      g_comp[kMaxK + 2];
  int64_t n_scan = 0, n_crow = 0, n_part = 0, n_write[kMaxK + 2] = {}, n_wi[kMaxK + 2] = {},
          n_comp[kMaxK + 2] = {};
  double bytes_write[kMaxK + 2] = {}, bytes_wi[kMaxK + 2] = {}, bytes_comp[kMaxK + 2] = {};
  double bytes_crow = 0;
  for (int i = 0; i < nt; ++i) {
    if (!has_out[i]) continue;
    BQ& b = q[owner[i]];
    const CTask& c = tasks[i];
    WTask& wt = w[i];
    wt.out0 = (int32_t*)((char*)B->p + o_out[i]);
    wt.ostride = col_stride(wt.m);
    const int64_t cnt_tiles = ceil_div(c.n, kTile);
    if (c.kind == kTaskExpand) {
      wt.k = b.t.k;
      for (int cc = 0; cc < b.t.k; ++cc) wt.in.c[cc] = b.t.col[cc];
      wt.nbr = c.pv.nbr;
      wt.N = c.N;
      const int gk = wt.k <= kMaxK ? wt.k : kMaxK + 1;
      // sparse: few input rows have output; the write walks only those
      sparse[i] = sparse_expand(sparse_theta, sparse_min_rows, c.n, nonempty[i]);
      if (sparse[i]) {
        const int64_t ne = nonempty[i];
        wt.n_in = c.n;
        wt.n = ne;
        wt.start_in = c.start;
        o_ridx[i] = LC.add(sizeof(int32_t) * ne);
        o_cstart[i] = LC.add(sizeof(int32_t) * ne);
        o_cP[i] = LC.add(sizeof(int64_t) * (ne + 1));
        g_crow.push_back(GItem{n_crow, i, 0});
        n_crow += cnt_tiles;
        // N of every input row; index, start and offset of every compacted row
        bytes_crow += 4.0 * c.n + 20.0 * ne;
      } else {
        wt.start = c.start;
        wt.P = (int64_t*)(da + o_P[i]);
        g_scan.push_back(GItem{n_scan, i, 0});
        n_scan += cnt_tiles;
      }
      const int64_t pt = ceil_div(wt.n + wt.m, kTile);
      o_split[i] = LC.add(sizeof(int64_t) * (pt + 1));
      g_part.push_back(GItem{n_part, i, 0});
      n_part += pt + 1;
      // outputs written (k + 1 columns), one member id read per output, the
      // offsets and starts of every row walked (and its index when
      // compacted), the k values of rows with output
      if (sparse[i]) {
        g_wi[gk].push_back(GItem{n_wi[gk], i, 0});
        n_wi[gk] += pt;
        bytes_wi[gk] += 4.0 * wt.m * (wt.k + 2) + 16.0 * wt.n + 4.0 * wt.k * wt.n;
      } else {
        g_write[gk].push_back(GItem{n_write[gk], i, 0});
        n_write[gk] += pt;
        bytes_write[gk] += 4.0 * wt.m * (wt.k + 2) + 12.0 * wt.n + 4.0 * wt.k * nonempty[i];
      }
    } else {
      const bool inter = c.kind == kTaskIntersect;
      wt.k = inter ? 1 : b.t.k;
      if (inter) wt.in.c[0] = c.col;
      else
        for (int cc = 0; cc < b.t.k; ++cc) wt.in.c[cc] = b.t.col[cc];
      wt.flags = c.flags;
      const int gk = wt.k <= kMaxK ? wt.k : kMaxK + 1;
      g_comp[gk].push_back(GItem{n_comp[gk], i, 0});
      n_comp[gk] += cnt_tiles;
      bytes_comp[gk] += (1.0 + 4.0 * wt.k) * wt.n + 4.0 * wt.k * wt.m;
    }
  }
  // the dense expansion writes go in one launch, grouped by column count
  std::vector<GItem> g_wall;
  int64_t n_wall = 0;
  double bytes_wall = 0;
  for (int k = 0; k < kMaxK + 2; ++k) {
    for (const GItem& g : g_write[k]) g_wall.push_back(GItem{n_wall + g.w0, g.task, 0});
    n_wall += n_write[k];
    bytes_wall += bytes_write[k];
  }
  // one upload: tasks, then every group's items
  const size_t o_w = LC.add(sizeof(WTask) * nt);
  auto put_group = [&](std::vector<GItem>& g) { return LC.add(sizeof(GItem) * std::max<size_t>(g.size(), 1)); };
  const size_t o_gscan = put_group(g_scan), o_gcrow = put_group(g_crow), o_gpart = put_group(g_part);
  const size_t o_gwall = put_group(g_wall);
  size_t o_gwi[kMaxK + 2], o_gc[kMaxK + 2];
  for (int k = 0; k < kMaxK + 2; ++k) {
    o_gwi[k] = put_group(g_wi[k]);
    o_gc[k] = put_group(g_comp[k]);
  }
  auto C = std::make_shared<Arena>(mem(), LC.bytes, s);
  char* dc = (char*)C->p;
  for (int i = 0; i < nt; ++i) {
    if (!has_out[i] || tasks[i].kind != kTaskExpand) continue;
    w[i].split = (int64_t*)(dc + o_split[i]);
    if (sparse[i]) {
      w[i].ridx = (int32_t*)(dc + o_ridx[i]);
      w[i].cstart = (int32_t*)(dc + o_cstart[i]);
      w[i].start = w[i].cstart;
      w[i].P = (int64_t*)(dc + o_cP[i]);
    }
  }
  {
    const size_t up = LC.bytes - o_w;
    char* h = (char*)pins(slot)[kPinWrite].get(up);
    std::memcpy(h, w.data(), sizeof(WTask) * nt);
    auto copy_group = [&](std::vector<GItem>& g, size_t off) {
      if (!g.empty()) std::memcpy(h + (off - o_w), g.data(), sizeof(GItem) * g.size());
    };
    copy_group(g_scan, o_gscan);
    copy_group(g_crow, o_gcrow);
    copy_group(g_part, o_gpart);
    copy_group(g_wall, o_gwall);
    for (int k = 0; k < kMaxK + 2; ++k) {
      copy_group(g_wi[k], o_gwi[k]);
      copy_group(g_comp[k], o_gc[k]);
    }
    GS_HIP(hipMemcpyAsync(dc + o_w, h, up, hipMemcpyHostToDevice, s));
  }
  const WTask* dw = (const WTask*)(dc + o_w);
  if (!g_scan.empty())
    launch_b_scan_add(dw, (const GItem*)(dc + o_gscan), (int)g_scan.size(), ts, n_scan,
                      12.0 * n_scan * kTile, s);
  if (!g_crow.empty()) {
    const int64_t* tsn = R.tsn;
    launch_b_compact_rows(dw, (const GItem*)(dc + o_gcrow), (int)g_crow.size(), ts, tsn, n_crow,
                          bytes_crow, s);
  }
  if (!g_part.empty())
    launch_b_partition(dw, (const GItem*)(dc + o_gpart), (int)g_part.size(), n_part, s);
  if (!g_wall.empty())
    launch_b_write(dw, (const GItem*)(dc + o_gwall), (int)g_wall.size(), n_wall, bytes_wall, s);
  for (int k = 0; k < kMaxK + 2; ++k) {
    if (!g_wi[k].empty())
      launch_b_write_idx(k, dw, (const GItem*)(dc + o_gwi[k]), (int)g_wi[k].size(), n_wi[k],
                         bytes_wi[k], s);
    if (!g_comp[k].empty())
      launch_b_compact(k, dw, (const GItem*)(dc + o_gc[k]), (int)g_comp[k].size(), ts,
                n_comp[k], bytes_comp[k], s);
  }

  // ---- the queries move on with their new tables
  for (int i = 0; i < nt; ++i) {
    if (!has_out[i]) continue;
    BQ& b = q[owner[i]];
    const CTask& c = tasks[i];
    const WTask& wt = w[i];
    Table r;
    r.n = wt.m;
    r.keep = B;
    if (c.kind == kTaskExpand) {
      r.k = b.t.k + 1;
      for (int cc = 0; cc < b.t.k; ++cc) r.var[cc] = b.t.var[cc];
      r.var[b.t.k] = b.new_var;
    } else if (c.kind == kTaskFilter) {
      r.k = b.t.k;
      for (int cc = 0; cc < b.t.k; ++cc) r.var[cc] = b.t.var[cc];
    } else {
      r.k = 1;
      r.var[0] = b.new_var;
      add_out(b, r.n);
    }
    for (int cc = 0; cc < r.k; ++cc) r.col[cc] = wt.out0 + (int64_t)cc * wt.ostride;
    advance(b, r);
  }
  R = Round();  // the scratch arenas go back in stream order, after these launches
}

}  // namespace

// Candidate fill thresholds the autotuner times; a candidate replaces the
// current threshold only when it is faster by more than 3 %.
constexpr int kTuneCandidates = 5;
constexpr double kTuneMargin = 0.97;

// ---------------------------------------------------------------- serving

namespace {

// Admission estimate of a plan's largest table in bytes: the first step's
// relation exactly (from the planning lookups where there are any), each
// later expansion multiplying the rows by the mean row length of its
// predicate in the expanded direction, filters and intersections adding
// none; capped by the plan's Theorem 1 bound.
int64_t estimate_bytes(const gsmat_store* st, const gsmat_query_plan* pl) {
  const bool have = pl->lk_store == st->uid && pl->lk.size() == pl->pats.size();
  auto rel_rows = [&](int tp) -> double {
    const gsmat_pattern& p = pl->pats[tp];
    if (p.p < 0 || p.p >= st->P) return 0.0;
    const PredDesc& o = st->out.desc[p.p];
    const PredDesc& i = st->in.desc[p.p];
    const bool sc = !is_var(p.s), oc = !is_var(p.o);
    if (!sc && !oc) return (double)o.nnz;
    if (have && pl->lk[tp].valid) return sc && oc ? pl->lk[tp].found : pl->lk[tp].len;
    if (sc && oc) return 1.0;
    const PredDesc& d = sc ? o : i;
    return d.nr ? (double)d.nnz / (double)d.nr : 0.0;
  };
  double rows = 1.0, peak = 0.0;
  int k = 0;
  uint64_t bound = 0;
  auto bind = [&](int tp) {
    const gsmat_pattern& p = pl->pats[tp];
    for (int32_t t : {p.s, p.o})
      if (is_var(t) && !(bound >> var_of(t) & 1)) {
        bound |= 1ull << var_of(t);
        ++k;
      }
  };
  for (const gsmat_step_info& sp : pl->steps) {
    const gsmat_pattern& p = pl->pats[sp.tp];
    switch (sp.kind) {
      case GSMAT_STEP_SCAN:
      case GSMAT_STEP_CARTESIAN:
        rows *= rel_rows(sp.tp);
        bind(sp.tp);
        break;
      case GSMAT_STEP_INTERSECT: {
        double m = -1.0;
        for (int tp = 0; tp < (int)pl->pats.size(); ++tp) {
          if (!(sp.members >> tp & 1)) continue;
          const gsmat_pattern& q = pl->pats[tp];
          const bool centre_s = q.s == -(sp.var + 1);
          const bool other_const = !is_var(centre_s ? q.o : q.s);
          const double len = other_const ? rel_rows(tp)
                                         : (double)(centre_s ? st->out.desc[q.p].nr
                                                             : st->in.desc[q.p].nr);
          m = m < 0 ? len : std::min(m, len);
        }
        rows *= std::max(m, 0.0);
        if (!(bound >> sp.var & 1)) {
          bound |= 1ull << sp.var;
          ++k;
        }
        break;
      }
      case GSMAT_STEP_EXPAND: {
        const PredDesc& d = sp.orient == 0 ? st->out.desc[p.p] : st->in.desc[p.p];
        rows *= d.nr ? (double)d.nnz / (double)d.nr : 0.0;
        bind(sp.tp);
        break;
      }
      default:
        break;
    }
    rows = std::min(rows, (double)sp.est_rows);
    peak = std::max(peak, rows * 4.0 * std::max(k, 1));
  }
  return (int64_t)std::min(peak, 9.0e18);
}

struct Pending {
  const gsmat_query_plan* pl;
  int64_t tag;
  int64_t est;
};

struct Finished {
  int64_t tag;
  gsmat_result* res;
  gsmat_status status;
};

}  // namespace

// A request loop over one resident store: submitted plans wait in arrival
// order until admission (estimated bytes within the memory budget, a free
// slot); every step admits what fits and then runs one round of the batched
// executor over all admitted queries, so queries that arrive while others
// run join them at the next round.
struct gsmat_server {
  gsmat_store* st;
  hipStream_t s;
  int64_t mem_budget;
  int32_t max_active;
  Batch bt;
  std::deque<Pending> waiting;
  std::deque<Finished> done;

  gsmat_server(gsmat_store* st_, int64_t mem, int64_t step, int64_t max_rows, int32_t slots,
               hipStream_t s_)
      : st(st_), s(s_), mem_budget(mem), max_active(slots),
        bt{st_, s_, step, max_rows, {}, mem, true} {}

  ~gsmat_server() {
    for (Finished& f : done) delete f.res;
  }

  // Bytes the admitted queries hold or are expected to need, and those of
  // finished results not yet polled.
  int64_t committed() const {
    int64_t c = 0;
    for (const BQ& b : bt.q) {
      const int64_t held = b.t.keep ? 4 * col_stride(b.t.n) * (int64_t)b.t.k : 0;
      c += std::max(held, b.est_bytes);
    }
    for (const Finished& f : done)
      if (f.res) c += 4 * col_stride(f.res->rows) * (int64_t)std::max(f.res->n_vars, 1);
    return c;
  }

  void admit() {
    if (waiting.empty()) return;
    int64_t c = committed();
    const size_t first = bt.q.size();
    while (!waiting.empty() && (int32_t)bt.q.size() < max_active) {
      const Pending& w = waiting.front();
      if (!bt.q.empty() && mem_budget > 0 && c + w.est > mem_budget) break;
      bt.q.emplace_back();
      BQ& b = bt.q.back();
      b.pl = w.pl;
      b.tag = w.tag;
      b.est_bytes = w.est;
      b.res.reset(new gsmat_result);
      b.res->st = st;
      b.res->stream = s;
      b.res->n_vars = w.pl->n_vars;
      b.res->reset_steps(w.pl->steps.size());
      b.t.n = 1;
      b.t.k = 0;
      b.rem = w.pl->pats.size() >= 32 ? 0xFFFFFFFFu : ((1u << w.pl->pats.size()) - 1);
      for (const gsmat_pattern& p : w.pl->pats)
        if (p.p >= st->P || (!is_var(p.s) && p.s >= st->V) || (!is_var(p.o) && p.o >= st->V)) {
          b.state = kDone;
          b.t = Table();
        }
      c += w.est;
      waiting.pop_front();
    }
    bt.admit(first);
  }

  // Moves finished queries to the done list (queries that left the batch
  // are run alone first).
  void collect() {
    size_t keep = 0;
    for (size_t i = 0; i < bt.q.size(); ++i) {
      BQ& b = bt.q[i];
      if (b.state == kActive) {
        if (keep != i) bt.q[keep] = std::move(b);
        ++keep;
        continue;
      }
      if (b.state == kFallback) {
        b.res.reset(new gsmat_result);
        b.res->st = st;
        b.res->stream = s;
        b.res->n_vars = b.pl->n_vars;
        b.res->reset_steps(b.pl->steps.size());
        gsmat_result* r = b.res.get();
        const gsmat_status rc = guarded([&]() -> gsmat_status {
          run_query(st, b.pl, bt.budget, bt.max_rows, s, r);
          return GSMAT_OK;
        });
        b.state = rc == GSMAT_OK ? kDone : kFailed;
        b.status = rc;
        if (rc != GSMAT_OK) b.res.reset();
      }
      done.push_back(Finished{b.tag, b.state == kDone ? b.res.release() : nullptr,
                              b.state == kDone ? GSMAT_OK : b.status});
    }
    bt.q.resize(keep);
  }
};

extern "C" gsmat_status gsmat_server_new(gsmat_store* st, int64_t mem_budget_bytes,
                                         int64_t step_budget_bytes, int64_t max_rows,
                                         int32_t max_active, void* stream, gsmat_server** out) {
  return guarded([&]() -> gsmat_status {
    if (!out) throw StatusFail{GSMAT_EINVAL, "out is NULL"};
    *out = nullptr;
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    if (max_active < 1) throw StatusFail{GSMAT_EINVAL, "max_active must be at least 1"};
    *out = new gsmat_server(st, mem_budget_bytes, step_budget_bytes, max_rows, max_active,
                            (hipStream_t)stream);
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_server_submit(gsmat_server* sv, const gsmat_query_plan* pl,
                                            int64_t tag) {
  return guarded([&]() -> gsmat_status {
    if (!sv || !pl) throw StatusFail{GSMAT_EINVAL, "server or plan is NULL"};
    sv->waiting.push_back(Pending{pl, tag, estimate_bytes(sv->st, pl)});
    return GSMAT_OK;
  });
}

// Queries the server runs one after another instead of batching them (see
// gsmat_server_step).
constexpr int kAloneMax = 2;

extern "C" gsmat_status gsmat_server_step(gsmat_server* sv, int32_t* n_active, int32_t* n_waiting,
                                          int32_t* n_done) {
  return guarded([&]() -> gsmat_status {
    if (!sv) throw StatusFail{GSMAT_EINVAL, "server is NULL"};
    sv->admit();
    sv->bt.sparse_theta = sv->st->sparse_theta;
    sv->bt.sparse_min_rows = sv->st->sparse_min_rows;
    int active = 0, fresh = 0;
    for (BQ& b : sv->bt.q)
      if (b.state == kActive) {
        ++active;
        fresh += b.si == 0 && b.t.unit();
      }
    // At most kAloneMax queries in the server, none started and none waiting:
    // the oldest runs to completion with the single-query executor and the
    // step returns, so its result can be polled before the next one runs.
    // For so few queries the batch's rounds cost more than running them one
    // after another (each round adds its host bookkeeping and a second wait
    // per step).  Queries arriving meanwhile are admitted at the next step.
    if (active > 0 && active <= kAloneMax && fresh == active && sv->waiting.empty()) {
      for (BQ& b : sv->bt.q)
        if (b.state == kActive) {
          b.state = kFallback;
          b.t = Table();
          break;
        }
      active = 0;
    }
    const bool any = active > 0;
    if (any) {
      // a round that fails part-way (device allocation, HIP error) has
      // already counted rows of its steps: the queries it carried fail with
      // its status instead of repeating the step in the next round
      const gsmat_status rc = guarded([&]() -> gsmat_status {
        sv->bt.round();
        return GSMAT_OK;
      });
      if (rc != GSMAT_OK) {
        const std::string msg = gsmat_last_error();
        for (BQ& b : sv->bt.q)
          if (b.state == kActive) sv->bt.fail(b, rc, msg);
        sv->bt.R = Batch::Round();
        sv->collect();
        throw StatusFail{rc, msg};
      }
    }
    sv->collect();
    if (n_active) *n_active = (int32_t)sv->bt.q.size();
    if (n_waiting) *n_waiting = (int32_t)sv->waiting.size();
    if (n_done) *n_done = (int32_t)sv->done.size();
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_server_poll(gsmat_server* sv, int32_t cap, int64_t* tags,
                                          gsmat_result** results, gsmat_status* status,
                                          int32_t* n_out) {
  return guarded([&]() -> gsmat_status {
    if (!sv || !n_out) throw StatusFail{GSMAT_EINVAL, "server or n_out is NULL"};
    if (cap < 0) throw StatusFail{GSMAT_EINVAL, "negative capacity"};
    if (cap > 0 && (!tags || !results || !status))
      throw StatusFail{GSMAT_EINVAL, "tags, results or status is NULL"};
    int32_t n = 0;
    if (cap > 0 && !sv->done.empty()) GS_HIP(hipStreamSynchronize(sv->s));
    while (n < cap && !sv->done.empty()) {
      const Finished& f = sv->done.front();
      tags[n] = f.tag;
      results[n] = f.res;
      status[n] = f.status;
      ++n;
      sv->done.pop_front();
    }
    *n_out = n;
    return GSMAT_OK;
  });
}

extern "C" void gsmat_server_free(gsmat_server* sv) { delete sv; }

namespace {

// gsmat_join_batch with device-driven rounds: the queries that leave the
// batch run alone afterwards, from the start.
gsmat_status join_batch_device(gsmat_store* st, const gsmat_query_plan* const* plans,
                               int32_t n_plans, int64_t budget_bytes, int64_t max_rows,
                               hipStream_t s, gsmat_result** out, gsmat_status* status) {
  std::vector<DevQueryOut> dq;
  run_batch_device(st, plans, n_plans, budget_bytes, max_rows, s, dq);
  bool alone = false;
  gsmat_status first = GSMAT_OK;
  std::string first_err;
  for (int i = 0; i < n_plans; ++i) {
    gsmat_status rc = dq[i].status;
    std::string err;
    if (dq[i].state == kDevFallback) {
      alone = true;
      std::unique_ptr<gsmat_result> r(new gsmat_result);
      r->st = st;
      r->stream = s;
      r->n_vars = plans[i]->n_vars;
      r->reset_steps(plans[i]->steps.size());
      rc = guarded([&]() -> gsmat_status {
        run_query(st, plans[i], budget_bytes, max_rows, s, r.get());
        return GSMAT_OK;
      });
      if (rc == GSMAT_OK) out[i] = r.release();
      else err = gsmat_last_error();
    } else if (dq[i].state == kDevDone) {
      out[i] = dq[i].res;
    } else if (rc == GSMAT_ETOOBIG) {
      err = "result exceeds max_rows (" + std::to_string(max_rows) + ")";
    } else {
      err = "query failed";
    }
    if (status) status[i] = rc;
    if (rc != GSMAT_OK && first == GSMAT_OK) {
      first = rc;
      first_err = "query " + std::to_string(i) + ": " + err;
    }
  }
  // the batch's own work was waited for; what ran alone is waited for here
  if (alone) host_sync(s);
  if (first != GSMAT_OK) throw StatusFail{first, first_err};
  return GSMAT_OK;
}

}  // namespace

extern "C" gsmat_status gsmat_join_batch_bgp(gsmat_store* st, const gsmat_pattern* pats,
                                             const int32_t* n_pats, int32_t n_queries,
                                             int32_t mode, int64_t budget_bytes, int64_t max_rows,
                                             void* stream, gsmat_result** out,
                                             gsmat_status* status) {
  return guarded([&]() -> gsmat_status {
    if (n_queries < 0) throw StatusFail{GSMAT_EINVAL, "negative query count"};
    if (n_queries > 0 && (!out || !n_pats || !pats))
      throw StatusFail{GSMAT_EINVAL, "pats, n_pats or out is NULL"};
    for (int i = 0; i < n_queries; ++i) out[i] = nullptr;
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    if (mode != GSMAT_PLAN_PAPER && mode != GSMAT_PLAN_DEFAULT && mode != GSMAT_PLAN_ADAPTIVE)
      throw StatusFail{GSMAT_EINVAL, "unknown plan mode " + std::to_string(mode)};
    hipStream_t s = (hipStream_t)stream;
    std::vector<DevQueryOut> dq;
    std::vector<gsmat_status> prc;
    std::vector<std::string> pmsg;
    std::vector<std::unique_ptr<gsmat_query_plan>> fb;
    run_batch_device_bgp(st, pats, n_pats, n_queries, mode, budget_bytes, max_rows, s, dq, prc,
                         pmsg, fb);
    bool alone = false;
    gsmat_status first = GSMAT_OK;
    std::string first_err;
    for (int i = 0; i < n_queries; ++i) {
      gsmat_status rc = prc[i];
      std::string err = rc != GSMAT_OK ? pmsg[i] : std::string();
      if (rc == GSMAT_OK) {
        rc = dq[i].status;
        if (dq[i].state == kDevFallback) {
          alone = true;
          std::unique_ptr<gsmat_result> r(new gsmat_result);
          r->st = st;
          r->stream = s;
          r->n_vars = fb[i]->n_vars;
          r->reset_steps(fb[i]->steps.size());
          rc = guarded([&]() -> gsmat_status {
            run_query(st, fb[i].get(), budget_bytes, max_rows, s, r.get());
            return GSMAT_OK;
          });
          if (rc == GSMAT_OK) out[i] = r.release();
          else err = gsmat_last_error();
        } else if (dq[i].state == kDevDone) {
          out[i] = dq[i].res;
        } else if (rc == GSMAT_ETOOBIG) {
          err = "result exceeds max_rows (" + std::to_string(max_rows) + ")";
        } else {
          err = "query failed";
        }
      }
      if (status) status[i] = rc;
      if (rc != GSMAT_OK && first == GSMAT_OK) {
        first = rc;
        first_err = "query " + std::to_string(i) + ": " + err;
      }
    }
    if (alone) host_sync(s);
    if (first != GSMAT_OK) throw StatusFail{first, first_err};
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_join_batch(gsmat_store* st, const gsmat_query_plan* const* plans,
                                         int32_t n_plans, int64_t budget_bytes, int64_t max_rows,
                                         void* stream, gsmat_result** out, gsmat_status* status) {
  return guarded([&]() -> gsmat_status {
    if (n_plans < 0) throw StatusFail{GSMAT_EINVAL, "negative query count"};
    if (n_plans > 0 && (!out || !plans)) throw StatusFail{GSMAT_EINVAL, "plans or out is NULL"};
    for (int i = 0; i < n_plans; ++i) out[i] = nullptr;
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    for (int i = 0; i < n_plans; ++i)
      if (!plans[i]) throw StatusFail{GSMAT_EINVAL, "plan " + std::to_string(i) + " is NULL"};
    hipStream_t s = (hipStream_t)stream;
    if (st->batch_engine == 1) return join_batch_device(st, plans, n_plans, budget_bytes, max_rows,
                                                        s, out, status);
    Batch bt{st, s, budget_bytes, max_rows, {}, budget_bytes, false};
    bt.sparse_theta = st->sparse_theta;
    bt.sparse_min_rows = st->sparse_min_rows;
    bt.q.resize(n_plans);
    for (int i = 0; i < n_plans; ++i) {
      BQ& b = bt.q[i];
      b.pl = plans[i];
      b.res.reset(new gsmat_result);
      b.res->st = st;
      b.res->stream = s;
      b.res->n_vars = b.pl->n_vars;
      b.res->reset_steps(b.pl->steps.size());
      b.t.n = 1;
      b.t.k = 0;
      b.rem = b.pl->pats.size() >= 32 ? 0xFFFFFFFFu : ((1u << b.pl->pats.size()) - 1);
      // a pattern over an absent predicate or vertex matches nothing
      for (const gsmat_pattern& p : b.pl->pats)
        if (p.p >= st->P || (!is_var(p.s) && p.s >= st->V) || (!is_var(p.o) && p.o >= st->V)) {
          b.state = kDone;
          b.t = Table();
        }
    }
    bt.run();
    // queries that left the batch run alone, from the start
    for (int i = 0; i < n_plans; ++i) {
      BQ& b = bt.q[i];
      if (b.state != kFallback) continue;
      b.res.reset(new gsmat_result);
      b.res->st = st;
      b.res->stream = s;
      b.res->n_vars = b.pl->n_vars;
      b.res->reset_steps(b.pl->steps.size());
      gsmat_result* r = b.res.get();
      const gsmat_status rc = guarded([&]() -> gsmat_status {
        run_query(st, b.pl, budget_bytes, max_rows, s, r);
        return GSMAT_OK;
      });
      if (rc != GSMAT_OK) {
        b.state = kFailed;
        b.status = rc;
        b.err = gsmat_last_error();
        b.res.reset();
      } else {
        b.state = kDone;
      }
    }
    host_sync(s);
    gsmat_status first = GSMAT_OK;
    std::string first_err;
    for (int i = 0; i < n_plans; ++i) {
      BQ& b = bt.q[i];
      if (status) status[i] = b.state == kFailed ? b.status : GSMAT_OK;
      if (b.state == kFailed) {
        if (first == GSMAT_OK) {
          first = b.status;
          first_err = "query " + std::to_string(i) + ": " + b.err;
        }
        continue;
      }
      out[i] = b.res.release();
    }
    if (first != GSMAT_OK) throw StatusFail{first, first_err};
    return GSMAT_OK;
  });
}

namespace gsmat {

void plan_prepare(const gsmat_store* st, const gsmat_pattern* pats, const int32_t* n_pats,
                  int32_t nq, int32_t mode, hipStream_t s, PlanPrep* pp) {
  PlanPrep& P = *pp;
  // off: first pattern of each query; so: its first statistics slot (a query
  // over the pattern limit fails validation and takes none)
  P.off.assign(nq + 1, 0);
  P.so.assign(nq + 1, 0);
  for (int i = 0; i < nq; ++i) {
    if (n_pats[i] < 0) throw StatusFail{GSMAT_EINVAL, "negative pattern count"};
    P.off[i + 1] = P.off[i] + n_pats[i];
    P.so[i + 1] = P.so[i] + (n_pats[i] <= kMaxPats ? n_pats[i] : 0);
  }
  P.rc.assign(nq, GSMAT_OK);
  P.msg.assign(nq, std::string());
  P.nv.assign(nq, 0);
  P.stats.assign(P.so[nq], TpStat{});
  P.req_of.assign(P.so[nq], -1);
  std::vector<LookupReq> req;
  req.reserve(P.so[nq]);
  for (int i = 0; i < nq; ++i) {
    const gsmat_pattern* pq = pats + P.off[i];
    const int n = n_pats[i];
    P.rc[i] = validate_patterns(pq, n, &P.nv[i], &P.msg[i]);
    if (P.rc[i] != GSMAT_OK) continue;
    // the statistics pattern_stats gathers, with the lookups pooled
    TpStat* ts = P.stats.data() + P.so[i];
    int* ro = P.req_of.data() + P.so[i];
    for (int j = 0; j < n; ++j) {
      const gsmat_pattern& p = pq[j];
      TpStat& t = ts[j];
      if (p.p < 0 || p.p >= st->P) continue;
      t.stat = st->out.desc[p.p].nnz;
      t.rows_s = st->out.desc[p.p].nr;
      t.rows_o = st->in.desc[p.p].nr;
      if (mode == GSMAT_PLAN_PAPER) continue;
      const bool sc = !is_var(p.s), oc = !is_var(p.o);
      if ((sc && p.s >= st->V) || (oc && p.o >= st->V)) {
        t.stat = t.rows_s = t.rows_o = 0;
        continue;
      }
      if (!sc && !oc) continue;
      ro[j] = (int)req.size();
      if (sc && oc) req.push_back({0, p.p, p.s, p.o});
      else if (sc) req.push_back({0, p.p, p.s, -1});
      else req.push_back({1, p.p, p.o, -1});
    }
  }
  P.res = lookup_many(st, req, s);
}

gsmat_status plan_build(const gsmat_store* st, const gsmat_pattern* pats, const int32_t* n_pats,
                        int32_t mode, PlanPrep& P, int64_t i, gsmat_query_plan* pl) {
  const gsmat_pattern* pq = pats + P.off[i];
  TpStat* ts = P.stats.data() + P.so[i];
  const int* ro = P.req_of.data() + P.so[i];
  for (int j = 0; j < n_pats[i]; ++j) {
    const int r = ro[j];
    if (r < 0) continue;
    const bool both = !is_var(pq[j].s) && !is_var(pq[j].o);
    const int64_t v = both ? P.res[r].found : P.res[r].len;
    ts[j].stat = ts[j].rows_s = ts[j].rows_o = v;
  }
  const gsmat_status rc = build_plan(pq, n_pats[i], mode, ts, pl, &P.msg[i]);
  if (rc == GSMAT_OK && mode != GSMAT_PLAN_PAPER) {
    pl->lk.assign(n_pats[i], gsmat_pat_lookup{});
    for (int j = 0; j < n_pats[i]; ++j) {
      const int r = ro[j];
      if (r >= 0) pl->lk[j] = gsmat_pat_lookup{P.res[r].start, P.res[r].len, P.res[r].found, 1};
    }
    pl->lk_store = st->uid;
  } else {
    pl->lk.clear();
    pl->lk_store = 0;
  }
  return rc;
}

}  // namespace gsmat

extern "C" gsmat_status gsmat_plan_batch(const gsmat_store* st, const gsmat_pattern* pats,
                                         const int32_t* n_pats, int32_t n_queries, int32_t mode,
                                         void* stream, gsmat_query_plan** out,
                                         gsmat_status* status) {
  return guarded([&]() -> gsmat_status {
    if (n_queries < 0) throw StatusFail{GSMAT_EINVAL, "negative query count"};
    if (n_queries > 0 && (!out || !n_pats || !pats))
      throw StatusFail{GSMAT_EINVAL, "pats, n_pats or out is NULL"};
    for (int i = 0; i < n_queries; ++i) out[i] = nullptr;
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    if (mode != GSMAT_PLAN_PAPER && mode != GSMAT_PLAN_DEFAULT && mode != GSMAT_PLAN_ADAPTIVE)
      throw StatusFail{GSMAT_EINVAL, "unknown plan mode " + std::to_string(mode)};
    PlanPrep P;
    plan_prepare(st, pats, n_pats, n_queries, mode, (hipStream_t)stream, &P);
    // the plans are independent: built on the host pool's threads
    host_parallel_for(n_queries, 256, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i) {
        if (P.rc[i] != GSMAT_OK) continue;
        try {
          std::unique_ptr<gsmat_query_plan> pl(new gsmat_query_plan);
          P.rc[i] = plan_build(st, pats, n_pats, mode, P, i, pl.get());
          if (P.rc[i] == GSMAT_OK) out[i] = pl.release();
        } catch (...) {
          P.rc[i] = GSMAT_ENOMEM;
          P.msg[i] = "host memory exhausted while planning";
        }
      }
    });
    gsmat_status first = GSMAT_OK;
    std::string first_err;
    for (int i = 0; i < n_queries; ++i) {
      if (status) status[i] = P.rc[i];
      if (P.rc[i] != GSMAT_OK && first == GSMAT_OK) {
        first = P.rc[i];
        first_err = "query " + std::to_string(i) + ": " + P.msg[i];
      }
    }
    if (first != GSMAT_OK) throw StatusFail{first, first_err};
    return GSMAT_OK;
  });
}

extern "C" void gsmat_plan_free_many(gsmat_query_plan** plans, int32_t n) {
  if (!plans) return;
  for (int32_t i = 0; i < n; ++i) {
    delete plans[i];
    plans[i] = nullptr;
  }
}

extern "C" void gsmat_result_free_many(gsmat_result** results, int32_t n) {
  if (!results) return;
  for (int32_t i = 0; i < n; ++i) {
    delete results[i];
    results[i] = nullptr;
  }
}

extern "C" gsmat_status gsmat_result_rows_many(const gsmat_result* const* results, int32_t n,
                                               int64_t* rows) {
  return guarded([&]() -> gsmat_status {
    if (n < 0) throw StatusFail{GSMAT_EINVAL, "negative count"};
    if (n > 0 && (!results || !rows)) throw StatusFail{GSMAT_EINVAL, "results or rows is NULL"};
    for (int32_t i = 0; i < n; ++i) rows[i] = results[i] ? results[i]->rows : -1;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_set_sparse_expand(gsmat_store* st, double theta, int64_t min_rows) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (!(theta >= 0.0 && theta <= 1.0)) throw StatusFail{GSMAT_EINVAL, "theta must be in [0, 1]"};
    if (min_rows < 1) throw StatusFail{GSMAT_EINVAL, "min_rows must be at least 1"};
    st->sparse_theta = theta;
    st->sparse_min_rows = min_rows;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_set_batch_engine(gsmat_store* st, int32_t engine) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (engine != 0 && engine != 1) throw StatusFail{GSMAT_EINVAL, "engine must be 0 or 1"};
    st->batch_engine = engine;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_set_batch_tuning(gsmat_store* st, int32_t count_items,
                                              int32_t intersect) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (count_items != 4 && count_items != 8 && count_items != 16)
      throw StatusFail{GSMAT_EINVAL, "count_items must be 4, 8 or 16"};
    if (intersect < GSMAT_ISECT_SEARCH || intersect > GSMAT_ISECT_MERGE)
      throw StatusFail{GSMAT_EINVAL, "intersect must be 0, 1 or 2"};
    st->count_items = count_items;
    st->intersect = intersect;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_get_batch_tuning(const gsmat_store* st, double* theta,
                                              int64_t* min_rows, int32_t* count_items,
                                              int32_t* intersect) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (theta) *theta = st->sparse_theta;
    if (min_rows) *min_rows = st->sparse_min_rows;
    if (count_items) *count_items = st->count_items;
    if (intersect) *intersect = st->intersect;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_set_batch_regions(gsmat_store* st, int64_t out_bytes,
                                               int64_t scratch_bytes) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (out_bytes < 0 || scratch_bytes < 0) throw StatusFail{GSMAT_EINVAL, "negative size"};
    st->dbatch_out_hint = out_bytes;
    st->dbatch_scr_hint = scratch_bytes;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_batch_round_stats(const gsmat_store* st, int64_t* out,
                                               int32_t cap, int32_t* n_rounds) {
  return guarded([&]() -> gsmat_status {
    if (!st || !n_rounds) throw StatusFail{GSMAT_EINVAL, "store or n_rounds is NULL"};
    if (cap < 0 || (cap > 0 && !out)) throw StatusFail{GSMAT_EINVAL, "bad output array"};
    const int32_t n = (int32_t)(st->dbatch_stats.size() / kStatFields);
    *n_rounds = n;
    for (int32_t i = 0; i < std::min(n, cap); ++i)
      for (int f = 0; f < kStatFields; ++f)
        out[(size_t)i * kStatFields + f] = st->dbatch_stats[(size_t)i * kStatFields + f];
    return GSMAT_OK;
  });
}

extern "C" int32_t gsmat_expand_strategy(double theta, int64_t min_rows, int64_t n_in,
                                         int64_t n_nonempty) {
  return sparse_expand(theta, min_rows, n_in, n_nonempty) ? 1 : 0;
}

extern "C" gsmat_status gsmat_autotune_batch(gsmat_store* st,
                                             const gsmat_query_plan* const* plans,
                                             int32_t n_plans, int64_t budget_bytes, void* stream,
                                             gsmat_tune_report* rep) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (n_plans < 0 || (n_plans > 0 && !plans)) throw StatusFail{GSMAT_EINVAL, "bad plan array"};
    hipStream_t s = (hipStream_t)stream;
    std::vector<gsmat_result*> res(std::max(n_plans, 1));
    // the fastest of three runs (one untimed run first when warm is set)
    auto time_batch = [&](bool warm) {
      double t_min = 0;
      for (int rep_i = warm ? -1 : 0; rep_i < 3; ++rep_i) {
        GS_HIP(hipStreamSynchronize(s));
        const auto t0 = std::chrono::steady_clock::now();
        const gsmat_status rc =
            gsmat_join_batch(st, plans, n_plans, budget_bytes, -1, stream, res.data(), nullptr);
        GS_HIP(hipStreamSynchronize(s));
        const double t = std::chrono::duration<double, std::milli>(
                             std::chrono::steady_clock::now() - t0).count();
        for (int i = 0; i < n_plans; ++i) gsmat_result_free(res[i]);
        if (rc != GSMAT_OK) throw StatusFail{rc, gsmat_last_error()};
        if (rep_i >= 0) t_min = rep_i == 0 ? t : std::min(t_min, t);
      }
      return t_min;
    };
    // one setting: every candidate timed, the current value kept unless
    // another is faster by a clear margin
    auto tune = [&](auto set, auto get, const auto* cand, int nc, double* ms) {
      const auto current = get();
      double current_ms = -1.0, best_ms = 0;
      int best = -1;
      for (int c = 0; c < nc; ++c) {
        set(cand[c]);
        const double t = time_batch(false);
        if (ms) ms[c] = t;
        if (cand[c] == current) current_ms = t;
        if (best < 0 || t < best_ms) {
          best = c;
          best_ms = t;
        }
      }
      set((current_ms > 0 && best_ms > kTuneMargin * current_ms) ? current : cand[best]);
    };
    gsmat_tune_report r{};
    std::fill(r.theta_ms, r.theta_ms + 5, -1.0);
    std::fill(r.items_ms, r.items_ms + 3, -1.0);
    std::fill(r.intersect_ms, r.intersect_ms + 3, -1.0);
    static const double kTheta[kTuneCandidates] = {0.0, 0.25, 0.5, 0.75, 1.0};
    static const int32_t kItemsCand[3] = {4, 8, 16};
    static const int32_t kIsectCand[3] = {GSMAT_ISECT_SEARCH, GSMAT_ISECT_WINDOW,
                                          GSMAT_ISECT_MERGE};
    time_batch(true);  // allocator, caches and round hints warm
    tune([&](double v) { st->sparse_theta = v; }, [&] { return st->sparse_theta; }, kTheta,
         kTuneCandidates, r.theta_ms);
    if (st->batch_engine == 1) {
      tune([&](int32_t v) { st->count_items = v; }, [&] { return st->count_items; }, kItemsCand, 3,
           r.items_ms);
      tune([&](int32_t v) { st->intersect = v; }, [&] { return st->intersect; }, kIsectCand, 3,
           r.intersect_ms);
    }
    r.theta = st->sparse_theta;
    r.count_items = st->count_items;
    r.intersect = st->intersect;
    if (rep) *rep = r;
    return GSMAT_OK;
  });
}
