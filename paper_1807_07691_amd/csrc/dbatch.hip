// Device-driven batched join.  Every query's state (its binding table, the
// patterns left, its step) lives in device memory, and a round of the
// batched join (paper Sec. 7.2: count, prefix sum, exact allocation and
// write, for the next step of every query) is a fixed sequence of launches
// whose sizes are read on the device:
//
//   choose    one thread per query: applies the previous round's outcome,
//             then picks the next step (the plan's, or the adaptive rule's
//             filter / candidate expansions)
//   sample    fan-out samples of every query's candidate expansions
//   task      one thread per query: the sampled choice, then the step either
//             finishes at once (a view into the store, an all-constant
//             filter, an empty intersection) or becomes a count-phase task
//   layout    one workgroup: tiles and count-phase scratch of every task,
//             bump-allocated from the round's scratch region
//   count     count / flag tiles of every task (Algorithm "Pre-allocating
//             result matrix space", first loop)
//   scan      one workgroup: tile sums scanned (second loop)
//   outcome   one thread per query: the task's output size and outcome
//   alloc     one workgroup: output tables bump-allocated from the current
//             output slab, write scratch from the round's scratch region
//   describe  one thread per query: write descriptors
//   post      row offsets (dense expansions), rows with output (sparse
//             expansions) and compactions (filters, intersections)
//   partition merge-path splits of every expansion
//   write     merge-path expansion writes
//
// The tile kernels run as many workgroups as the device holds at once, each
// striding over the round's tiles (their count is read on the device), so
// the host enqueues rounds without waiting for them.  (Taking tiles from a
// shared counter instead was measured slower: one atomic per tile on one
// address costs more than the uneven tiles it balances.)  The
// single-workgroup kernels only scan per-query arrays laid out one value per
// query.  The host waits
// once per group of rounds (as many rounds as the longest plan can take) and
// then only reads a small summary.  Allocation never waits for the host: a
// task whose scratch or output does not fit the current regions is deferred
// (it repeats its step in a later round), and at the wait the host adds a
// larger output slab or scratch region and runs the remaining rounds.  Each
// query takes exactly the steps it takes under the single-query executor
// (same plan, same choice rule, same sampled fan-outs) and writes its rows in
// the same order.  A query whose next step is a Cartesian product, a
// (?x p ?x) scan or an output above the step budget leaves the batch and is
// finished by the single-query executor.
#include <algorithm>
#include <cstring>
#include <functional>
#include <memory>
#include <vector>

#include "batch.hpp"
#include "batch_tiles.hpp"
#include "device.hpp"
#include "exec.hpp"
#include "host_pool.hpp"

namespace gsmat {

namespace {

using namespace dev;

constexpr int kQBlock = 256;  // threads per workgroup of the per-query kernels
constexpr int kPartGrid = 1024;  // workgroups of the split kernel (one thread per split)

enum : int32_t { kQActive = 0, kQDone = 1, kQFallback = 2, kQFailed = 3 };
// outcome of a query's step in the current round
enum : int32_t {
  kONone = 0,   // nothing pending
  kOTask,       // counted this round (decided by `decide`)
  kODefer,      // did not fit the memory regions: repeat the step
  kODone,       // empty output: the query is finished with no rows
  kOPass,       // filter that removed nothing: the table goes on
  kODriver,     // intersection whose driver ids all survive
  kOWrite,      // output table written
  kOFallback    // leaves the batch
};

struct DPat {
  int32_t s, p, o;
};
struct DStep {
  int8_t kind, tp, orient, var;
  uint32_t members;
};
struct DPlanQ {
  int32_t np, nsteps, nv, mode, absent, pad;
};
struct DLk {  // a planning lookup (valid = 0: look up on the device)
  int32_t start, len, found, valid;
};

// A binding table: column c holds variable var[c]; slab = output slab
// holding the columns (-1: store memory).
struct DTab {
  int64_t n;
  int32_t k, slab;
  const int32_t* col[kMaxCols];
  int8_t var[kMaxCols];
};

struct DQ {
  DTab t;
  int32_t state, status;
  int32_t si, new_var;
  uint32_t rem, next;
  int32_t cand0, nc;
  int8_t cand_tp[kMaxPats], cand_or[kMaxPats];
  DStep sp;
  int32_t kind;      // task kind of the current step
  int32_t kout, sparse, pad;
  int64_t n_in;      // rows entering the step
  int64_t m, ne;     // task output rows, expansion rows with output
  int64_t rows;      // result rows once emitted
};

// Shared control block: the memory regions, this round's sizes, the summary
// the host reads at its wait, and the algorithmic bytes of the pass.
struct DCtl {
  char* out_base;
  int64_t out_cap, out_used;
  char* scr_base;
  int64_t scr_cap, scr_used, scr_peak;
  int64_t* ts;
  int64_t* tsn;
  int64_t ntiles, n_post, n_part, n_write;
  int64_t want_out, want_scr;
  int64_t bytes_count, bytes_post, bytes_write;
  int64_t scr_need;  // largest scratch a round asked for (deferred tasks included)
  // per round: tasks counted, count tiles, post tiles, write tiles, tables
  // written, output bytes, candidates sampled, deferred tasks
  int64_t stats[kStatRounds][kStatFields];
  int32_t out_slab, ncand, active, deferred, error, round;
};

struct DRes {
  int32_t state, status, slab, pad;
  int64_t rows;
};

struct DArgs {
  int32_t nq, mp, ms, mv;
  int64_t budget, round_budget, max_rows;
  double theta;
  int64_t min_rows;
  const PredDesc* dout;
  const PredDesc* din;
  OriPtrs out, in;
  const int32_t* out_src;
  const DPlanQ* pq;
  const DPat* pats;
  const DStep* steps;
  const DLk* lkin;
  LookupRes* lk;
  DQ* q;
  int64_t* sin;
  int64_t* sout;
  SCand* cands;
  int64_t* part;
  CTask* ct;
  ListRef* lists;
  WTask* wt;
  int64_t* ne;
  int64_t* w_cnt;  // [nq + 1] first count tile of each query's task
  int64_t* w_post;
  int64_t* w_part;
  int64_t* w_write;
  // per query, one value each: this round's outcome (kO*), the task's
  // count-phase cost, tiles, scratch and algorithmic bytes, its scratch
  // offset; the write-phase sizes; the output and write scratch offsets
  int32_t* oc;
  int64_t *tk_cost, *tk_tiles, *tk_cb, *tk_alg, *cnt_off;
  int64_t *wz_ob, *wz_sb, *wz_post, *wz_part, *wz_write, *wz_alg_post, *wz_alg_write;
  int64_t *out_off, *scr_off;
  DCtl* ctl;
  DRes* res;
  const int32_t** res_col;  // [nq * mv]
};

__device__ inline bool d_isvar(int32_t t) { return t < 0; }
__device__ inline int d_var(int32_t t) { return -t - 1; }
__device__ inline int64_t d_a256(int64_t b) { return (b + 255) & ~(int64_t)255; }
__device__ inline int64_t d_stride(int64_t n) { return ((n > 1 ? n : 1) + 63) / 64 * 64; }
__device__ inline int64_t d_tiles(int64_t n) { return (n + kTile - 1) / kTile; }

__device__ inline int tab_col(const DTab& t, int v) {
  for (int c = 0; c < t.k; ++c)
    if (t.var[c] == v) return c;
  return -1;
}

__device__ inline PredView d_view(const DArgs& A, int orient, int32_t p) {
  if (orient == 0) {
    PredView pv = view_of(A.dout[p], A.out);
    pv.src = A.out_src + A.dout[p].nbr_base;
    return pv;
  }
  return view_of(A.din[p], A.in);
}

// Bitmap of row v of predicate p in one orientation, or null.
__device__ inline const uint32_t* d_row_bitmap(const DArgs& A, int orient, int32_t p, int32_t v) {
  const PredDesc& d = orient == 0 ? A.dout[p] : A.din[p];
  const OriPtrs& o = orient == 0 ? A.out : A.in;
  if (!d.hub_n) return nullptr;
  const int32_t* a = o.hub_keys + d.hub_base;
  const int32_t r = lower_bound_i32(a, d.hub_n, v);
  if (r >= d.hub_n || a[r] != v) return nullptr;
  return o.hub_bm + (d.hub_base + r) * o.hub_words;
}

__device__ inline void d_error(const DArgs& A, int qi, DQ& Q) {
  atomicAdd(&A.ctl->error, 1);
  Q.state = kQFallback;
  A.oc[qi] = kONone;
}

// The patterns a step completes (its own; an intersection: the members whose
// other endpoint is a constant).
__device__ inline uint32_t d_completes(const DPat* pats, int np, const DStep& sp) {
  if (sp.kind != GSMAT_STEP_INTERSECT) return 1u << sp.tp;
  uint32_t m = 0;
  const int32_t cterm = -(sp.var + 1);
  for (int tp = 0; tp < np; ++tp) {
    if (!(sp.members >> tp & 1)) continue;
    const DPat q = pats[tp];
    const int32_t other = q.s == cterm ? q.o : q.s;
    if (!d_isvar(other)) m |= 1u << tp;
  }
  return m;
}

// Adaptive choice on a bound table: true with sp = a filter when a remaining
// connected pattern has both endpoints bound; else Q.nc candidate
// expansions, and sp = the Cartesian step over the smallest remaining
// pattern for when there are none.
__device__ inline bool d_candidates(const DArgs& A, const DPat* pats, int np, DQ& Q, DStep& sp) {
  uint64_t bound = 0;
  for (int c = 0; c < Q.t.k; ++c) bound |= 1ull << Q.t.var[c];
  auto vb = [&](int32_t x) { return d_isvar(x) && ((bound >> d_var(x)) & 1); };
  auto is_bound = [&](int32_t x) { return !d_isvar(x) || ((bound >> d_var(x)) & 1); };
  for (int tp = 0; tp < np; ++tp) {
    if (!(Q.rem >> tp & 1)) continue;
    const DPat q = pats[tp];
    const bool connected = vb(q.s) || vb(q.o);
    const bool all_const = !d_isvar(q.s) && !d_isvar(q.o);
    if ((connected || all_const) && is_bound(q.s) && is_bound(q.o)) {
      sp = DStep{(int8_t)GSMAT_STEP_FILTER, (int8_t)tp, -1, -1, 0u};
      return true;
    }
  }
  int nc = 0;
  for (int tp = 0; tp < np; ++tp) {
    if (!(Q.rem >> tp & 1)) continue;
    const DPat q = pats[tp];
    const bool sb = vb(q.s), ob = vb(q.o);
    if (sb == ob) continue;
    const int32_t free_term = sb ? q.o : q.s;
    if (!d_isvar(free_term)) continue;
    Q.cand_tp[nc] = (int8_t)tp;
    Q.cand_or[nc] = sb ? 0 : 1;
    ++nc;
  }
  Q.nc = nc;
  int pick = -1;
  int64_t best = INT64_MAX;
  for (int tp = 0; tp < np; ++tp) {
    if (!(Q.rem >> tp & 1)) continue;
    const int64_t z = A.dout[pats[tp].p].nnz;
    if (z < best) {
      best = z;
      pick = tp;
    }
  }
  sp = DStep{(int8_t)GSMAT_STEP_CARTESIAN, (int8_t)(pick < 0 ? 0 : pick), -1, -1, 0u};
  return false;
}

// Expansion step of candidate `best`.
__device__ inline DStep d_pick(const DPat* pats, const DQ& Q, int best) {
  const DPat q = pats[Q.cand_tp[best]];
  const int o = Q.cand_or[best];
  return DStep{(int8_t)GSMAT_STEP_EXPAND, Q.cand_tp[best], (int8_t)o,
               (int8_t)(o == 0 ? d_var(q.o) : d_var(q.s)), 0u};
}

// The step is done and Q.t already holds the query's new table (tables are
// updated in place: a copy of the column pointers would go through
// private memory): counters, then the query moves on.
__device__ inline void d_step_done(const DArgs& A, int qi, DQ& Q, int64_t m) {
  const DPlanQ& pl = A.pq[qi];
  if (Q.si < pl.nsteps) {
    A.sin[(int64_t)qi * A.ms + Q.si] += Q.n_in;
    A.sout[(int64_t)qi * A.ms + Q.si] += m;
  }
  Q.rem = Q.next;
  Q.si += 1;
  A.oc[qi] = kONone;
  if (Q.t.n == 0) {
    Q.state = kQDone;
    Q.rows = 0;
  } else if (Q.rem == 0) {
    Q.rows = Q.t.n;
    if (A.max_rows >= 0 && Q.t.n > A.max_rows) {
      Q.state = kQFailed;
      Q.status = GSMAT_ETOOBIG;
    } else {
      Q.state = kQDone;
    }
  }
}

__device__ inline void d_done_empty(const DArgs& A, int qi, DQ& Q) {
  Q.t.n = 0;
  Q.t.k = 0;
  Q.t.slab = -1;
  d_step_done(A, qi, Q, 0);
}

// Relation of pattern tp as a view into the store, written over the query's
// unit table (a scan step); false, with the table untouched, for the
// (?x p ?x) diagonal.
__device__ inline bool d_scan_view(const DArgs& A, int qi, int tp, DTab& r) {
  const DPat p = A.pats[(int64_t)qi * A.mp + tp];
  const LookupRes& lk = A.lk[(int64_t)qi * A.mp + tp];
  if (d_isvar(p.s) && d_isvar(p.o)) {
    if (p.s == p.o) return false;
    const PredDesc& d = A.dout[p.p];
    r.n = d.nnz;
    r.k = 2;
    r.col[0] = A.out_src + d.nbr_base;
    r.var[0] = (int8_t)d_var(p.s);
    r.col[1] = A.out.nbr + d.nbr_base;
    r.var[1] = (int8_t)d_var(p.o);
  } else if (!d_isvar(p.s) && d_isvar(p.o)) {
    r.n = lk.len;
    r.k = 1;
    r.col[0] = A.out.nbr + A.dout[p.p].nbr_base + lk.start;
    r.var[0] = (int8_t)d_var(p.o);
  } else if (d_isvar(p.s) && !d_isvar(p.o)) {
    r.n = lk.len;
    r.k = 1;
    r.col[0] = A.in.nbr + A.din[p.p].nbr_base + lk.start;
    r.var[0] = (int8_t)d_var(p.s);
  } else {
    r.n = lk.found ? 1 : 0;
    r.k = 0;
  }
  r.slab = -1;
  return true;
}

// Applies the outcome decided for the query's task in the last round.
__device__ inline void d_apply(const DArgs& A, int qi, DQ& Q) {
  if (Q.state != kQActive) return;
  switch (A.oc[qi]) {
    case kONone:
      return;
    case kODefer:
      A.oc[qi] = kONone;
      return;
    case kOFallback:
      Q.state = kQFallback;
      A.oc[qi] = kONone;
      return;
    case kODone:
      d_done_empty(A, qi, Q);
      return;
    case kOPass:
      d_step_done(A, qi, Q, Q.m);
      return;
    case kODriver:
      Q.t.n = Q.m;
      Q.t.k = 1;
      Q.t.slab = -1;
      Q.t.col[0] = A.ct[qi].col;
      Q.t.var[0] = (int8_t)Q.new_var;
      d_step_done(A, qi, Q, Q.m);
      return;
    case kOWrite: {
      const WTask& w = A.wt[qi];
      if (Q.kind == kTaskExpand) {
        Q.t.var[Q.t.k] = (int8_t)Q.new_var;
        Q.t.k += 1;
      } else if (Q.kind == kTaskIntersect) {
        Q.t.k = 1;
        Q.t.var[0] = (int8_t)Q.new_var;
      }
      Q.t.n = Q.m;
      Q.t.slab = A.ctl->out_slab;  // the host changes it only between groups of rounds
      for (int c = 0; c < Q.t.k; ++c) Q.t.col[c] = w.out0 + (int64_t)c * w.ostride;
      d_step_done(A, qi, Q, Q.m);
      return;
    }
    default:
      d_error(A, qi, Q);
  }
}

// ------------------------------------------------------------------ kernels

__global__ void k_d_init(DArgs A) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= A.nq) return;
  DQ& Q = A.q[qi];
  const DPlanQ& pl = A.pq[qi];
  Q.t.n = 1;
  Q.t.k = 0;
  Q.t.slab = -1;
  Q.state = kQActive;
  Q.status = 0;
  Q.si = 0;
  Q.new_var = -1;
  Q.rem = pl.np >= 32 ? 0xFFFFFFFFu : ((1u << pl.np) - 1);
  Q.next = Q.rem;
  Q.cand0 = -1;
  Q.nc = 0;
  Q.n_in = 0;
  Q.rows = 0;
  A.oc[qi] = kONone;
  for (int i = 0; i < A.ms; ++i) {
    A.sin[(int64_t)qi * A.ms + i] = 0;
    A.sout[(int64_t)qi * A.ms + i] = 0;
  }
  if (pl.absent) {  // a pattern over an absent predicate or vertex matches nothing
    Q.state = kQDone;
    return;
  }
  for (int tp = 0; tp < pl.np; ++tp) {
    const DPat p = A.pats[(int64_t)qi * A.mp + tp];
    const DLk& l = A.lkin[(int64_t)qi * A.mp + tp];
    LookupRes& r = A.lk[(int64_t)qi * A.mp + tp];
    r = LookupRes{0, 0, 0, 0};
    const bool sc = !d_isvar(p.s), oc = !d_isvar(p.o);
    if (!sc && !oc) continue;
    if (l.valid) {
      r = LookupRes{l.start, l.len, l.found, 0};
      continue;
    }
    LookupReq q;
    if (sc && oc) q = LookupReq{0, p.p, p.s, p.o};
    else if (sc) q = LookupReq{0, p.p, p.s, -1};
    else q = LookupReq{1, p.p, p.o, -1};
    r = lookup_one(q, A.dout, A.din, A.out, A.in);
  }
}

// Applies the last round's outcomes; with `choose`, picks every active
// query's next step (adaptive candidates go to the round's list), else
// writes the per-query summary the host reads at its wait.
__global__ void k_d_choose(DArgs A, int choose) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= A.nq) return;
  DQ& Q = A.q[qi];
  d_apply(A, qi, Q);
  if (Q.state == kQActive) atomicAdd(&A.ctl->active, 1);
  if (!choose) {
    const DPlanQ& pl = A.pq[qi];
    DRes& r = A.res[qi];
    const bool rows = Q.state == kQDone && Q.rows > 0;
    r.state = Q.state;
    r.status = Q.status;
    r.slab = rows ? Q.t.slab : -1;
    r.pad = 0;
    r.rows = Q.state == kQDone ? Q.rows : 0;
    for (int v = 0; v < pl.nv; ++v) {
      const int c = rows ? tab_col(Q.t, v) : -1;
      if (rows && c < 0) atomicAdd(&A.ctl->error, 1);
      A.res_col[(int64_t)qi * A.mv + v] = c >= 0 ? Q.t.col[c] : nullptr;
    }
    return;
  }
  if (Q.state != kQActive) return;
  Q.cand0 = -1;
  Q.nc = 0;
  const DPlanQ& pl = A.pq[qi];
  const DPat* pats = A.pats + (int64_t)qi * A.mp;
  const bool unit = Q.t.n == 1 && Q.t.k == 0;
  if (pl.mode == GSMAT_PLAN_ADAPTIVE && !unit) {
    DStep sp;
    if (d_candidates(A, pats, pl.np, Q, sp) || Q.nc == 0) {
      Q.nc = 0;
      Q.sp = sp;
    } else if (Q.nc == 1) {
      Q.sp = d_pick(pats, Q, 0);
    } else {
      const int c0 = atomicAdd(&A.ctl->ncand, Q.nc);
      if (c0 + Q.nc > A.nq * A.mp) {
        d_error(A, qi, Q);
        return;
      }
      Q.cand0 = c0;
      for (int i = 0; i < Q.nc; ++i) {
        const DPat q = pats[Q.cand_tp[i]];
        const bool from_s = Q.cand_or[i] == 0;
        const int c = tab_col(Q.t, d_var(from_s ? q.s : q.o));
        if (c < 0) {
          d_error(A, qi, Q);
          return;
        }
        SCand& sc = A.cands[c0 + i];
        sc.col = Q.t.col[c];
        sc.pv = d_view(A, from_s ? 0 : 1, q.p);
        sc.n = Q.t.n;
      }
    }
  } else {
    if (pl.nsteps < 1) {
      d_error(A, qi, Q);
      return;
    }
    const int i = Q.si < pl.nsteps ? Q.si : pl.nsteps - 1;
    Q.sp = A.steps[(int64_t)qi * A.ms + i];
  }
}

// Fan-out sample slices of every candidate (kSampleBlocks per candidate).
// The tile kernels take their arrays as separate read-only, non-aliased
// parameters, so that the descriptors are fetched with scalar loads.
__global__ __launch_bounds__(kBlock) void k_d_sample(const SCand* __restrict__ cands,
                                                     int64_t* __restrict__ part,
                                                     const DCtl* __restrict__ ctl) {
  const int64_t total = (int64_t)ctl->ncand * kSampleBlocks;
  for (int64_t j = blockIdx.x; j < total; j += gridDim.x) {
    const SCand& sc = cands[j / kSampleBlocks];
    const int64_t t = sample_fanout_slice((int)(j % kSampleBlocks), sc.col, sc.n, sc.pv);
    if (threadIdx.x == 0) part[j] = t;
    __syncthreads();
  }
}

// Count-phase scratch of a task: N, start and offsets P of an expansion, or
// the keep flags of a filter or intersection.
__device__ inline int64_t d_cnt_bytes(int kind, int64_t n) {
  if (kind == kTaskExpand) return 2 * d_a256(4 * n) + d_a256(8 * (n + 1));
  return d_a256(n);
}

// Algorithmic bytes of a count task: a lookup of every input row's bound
// value (4 read + 8 row extent) and its count and start written (expansion);
// two values, one probe word and a flag (filter); the driver id, one probe
// per other list and a flag (intersection).
__device__ inline int64_t d_count_alg(const CTask& c) {
  if (c.kind == kTaskExpand) return 20 * c.n;
  if (c.kind == kTaskFilter) return 13 * c.n;
  return (5 + 4 * (int64_t)c.nl) * c.n;
}

// The step of every active query: finished at once, or a count-phase task.
__global__ void k_d_task(DArgs A) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= A.nq) return;
  DQ& Q = A.q[qi];
  if (Q.state != kQActive) return;
  const DPlanQ& pl = A.pq[qi];
  const DPat* pats = A.pats + (int64_t)qi * A.mp;
  if (Q.cand0 >= 0) {
    // the candidate with the smallest sampled fan-out (the first on ties)
    int best = 0;
    int64_t best_sum = 0;
    for (int i = 0; i < Q.nc; ++i) {
      int64_t sum = 0;
      for (int j = 0; j < kSampleBlocks; ++j)
        sum += A.part[(int64_t)(Q.cand0 + i) * kSampleBlocks + j];
      if (i == 0 || sum < best_sum) {
        best = i;
        best_sum = sum;
      }
    }
    Q.sp = d_pick(pats, Q, best);
  }
  const DStep sp = Q.sp;
  Q.next = Q.rem & ~d_completes(pats, pl.np, sp);
  Q.n_in = Q.t.n;
  A.oc[qi] = kONone;
  const DPat p = pats[sp.tp];
  const bool unit = Q.t.n == 1 && Q.t.k == 0;
  CTask c{};
  switch (sp.kind) {
    case GSMAT_STEP_SCAN:
    case GSMAT_STEP_CARTESIAN: {
      if (!unit || !d_scan_view(A, qi, sp.tp, Q.t)) {
        Q.state = kQFallback;
        return;
      }
      d_step_done(A, qi, Q, Q.t.n);
      return;
    }
    case GSMAT_STEP_INTERSECT: {
      if (!unit) {
        Q.state = kQFallback;
        return;
      }
      const int32_t cterm = -(sp.var + 1);
      ListRef* out = A.lists + (int64_t)qi * kMaxLists;
      // the shortest list (the first on ties) drives; the others follow it
      int nl = 0, d = -1;
      const int32_t* dids = nullptr;
      int64_t dlen = 0;
      for (int pass = 0; pass < 2; ++pass) {
        int j = 0, w = 0;
        for (int tp = 0; tp < pl.np; ++tp) {
          if (!(sp.members >> tp & 1)) continue;
          if (j >= kMaxLists) {
            d_error(A, qi, Q);
            return;
          }
          const DPat m = pats[tp];
          ListRef l{};
          const int32_t* ids;
          if (m.s == cterm && d_isvar(m.o)) {
            l.pv = d_view(A, 0, m.p);
            l.is_keys = 1;
            l.len = l.pv.nr;
            ids = l.pv.keys;
          } else if (m.o == cterm && d_isvar(m.s)) {
            l.pv = d_view(A, 1, m.p);
            l.is_keys = 1;
            l.len = l.pv.nr;
            ids = l.pv.keys;
          } else if (m.s == cterm) {
            const LookupRes& r = A.lk[(int64_t)qi * A.mp + tp];
            l.seg = A.in.nbr + A.din[m.p].nbr_base + r.start;
            l.bm = d_row_bitmap(A, 1, m.p, m.o);
            l.len = r.len;
            ids = l.seg;
          } else {
            const LookupRes& r = A.lk[(int64_t)qi * A.mp + tp];
            l.seg = A.out.nbr + A.dout[m.p].nbr_base + r.start;
            l.bm = d_row_bitmap(A, 0, m.p, m.s);
            l.len = r.len;
            ids = l.seg;
          }
          if (pass == 0) {
            if (d < 0 || l.len < dlen) {
              d = j;
              dlen = l.len;
              dids = ids;
            }
          } else if (j != d) {
            out[w++] = l;
          }
          ++j;
        }
        nl = w;
      }
      if (d < 0 || dlen == 0) {
        d_done_empty(A, qi, Q);
        return;
      }
      c.kind = kTaskIntersect;
      c.n = dlen;
      c.col = dids;
      c.l0 = qi * kMaxLists;
      c.nl = nl;
      Q.new_var = sp.var;
      break;
    }
    case GSMAT_STEP_FILTER: {
      if (!d_isvar(p.s) && !d_isvar(p.o)) {
        if (A.lk[(int64_t)qi * A.mp + sp.tp].found) {
          d_step_done(A, qi, Q, Q.t.n);
        } else {
          d_done_empty(A, qi, Q);
        }
        return;
      }
      c.kind = kTaskFilter;
      c.n = Q.t.n;
      if (d_isvar(p.s)) {
        const int cs = tab_col(Q.t, d_var(p.s));
        if (cs < 0) {
          Q.state = kQFallback;
          return;
        }
        c.pa.s_col = Q.t.col[cs];
      } else {
        c.pa.s_const = p.s;
      }
      if (d_isvar(p.o)) {
        const int co = tab_col(Q.t, d_var(p.o));
        if (co < 0) {
          Q.state = kQFallback;
          return;
        }
        c.pa.o_col = Q.t.col[co];
      } else {
        c.pa.o_const = p.o;
      }
      c.pv = d_view(A, 0, p.p);
      break;
    }
    case GSMAT_STEP_EXPAND: {
      const int bound_var = sp.orient == 0 ? d_var(p.s) : d_var(p.o);
      const int bc = tab_col(Q.t, bound_var);
      if (bc < 0 || Q.t.k + 1 > kMaxCols) {
        Q.state = kQFallback;  // the single-query executor reports it
        return;
      }
      c.kind = kTaskExpand;
      c.n = Q.t.n;
      c.col = Q.t.col[bc];
      c.pv = d_view(A, sp.orient == 0 ? 0 : 1, p.p);
      Q.new_var = sp.orient == 0 ? d_var(p.o) : d_var(p.s);
      break;
    }
    default:
      Q.state = kQFallback;
      return;
  }
  Q.kind = c.kind;
  A.ct[qi] = c;
  const int64_t cb = d_cnt_bytes(c.kind, c.n), tiles = d_tiles(c.n);
  A.tk_cb[qi] = cb;
  A.tk_tiles[qi] = tiles;
  A.tk_cost[qi] = cb + 16 * tiles;  // with its share of the two tile-sum arrays
  A.tk_alg[qi] = d_count_alg(c);
  A.oc[qi] = kOTask;
}

// Queries per thread that the single-workgroup kernels hold in registers
// (batches of up to kAllocRegs * kScanBlock queries).
constexpr int kAllocRegs = 4;

// The end of k_d_layout: deferrals, the round's tile-sum arrays, and its
// statistics (t1: total scratch asked; t2: totals of tiles, scratch bytes
// and algorithmic bytes; tasks: tasks counted this round).
__device__ inline void d_layout_finish(DArgs& A, DCtl& C, const int64_t (&t1)[1],
                                       const int64_t (&t2)[3], int64_t tasks, int defer,
                                       int64_t want) {
  __shared__ int s_defer;
  __shared__ unsigned long long s_want;
  if (threadIdx.x == 0) {
    s_defer = 0;
    s_want = 0;
  }
  __syncthreads();
  if (defer) {
    atomicAdd(&s_defer, defer);
    atomicMax(&s_want, (unsigned long long)want);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t nt = t2[0];
    char* base = C.scr_base;
    C.scr_need = max(C.scr_need, t1[0] + 1024);
    if (C.round < kStatRounds) {
      int64_t* st = C.stats[C.round];
      st[0] = tasks;
      st[1] = nt;
      st[6] = C.ncand;
      st[7] = s_defer;
    }
    A.w_cnt[A.nq] = nt;
    C.ntiles = nt;
    C.ts = (int64_t*)(base + t2[1]);
    C.tsn = (int64_t*)(base + t2[1] + d_a256(8 * (nt + 1)));
    C.scr_used = t2[1] + 2 * d_a256(8 * (nt + 1));
    C.bytes_count += t2[2];
    C.ncand = 0;
    C.active = 0;
    C.deferred += s_defer;
    C.want_scr = max(C.want_scr, (int64_t)s_want);
  }
}

// Tiles and count-phase scratch of every task (one workgroup of kScanBlock
// threads; thread t takes a contiguous range of queries).  A task whose
// scratch (with its share of the tile-sum arrays) does not fit the scratch
// region is deferred; fitting is a prefix property, so the tasks that run
// are the first ones in query order.
__global__ __launch_bounds__(kScanBlock) void k_d_layout_loop(DArgs A) {
  DCtl& C = *A.ctl;
  const int per = (A.nq + kScanBlock - 1) / kScanBlock;
  const int q0 = min(A.nq, (int)threadIdx.x * per), q1 = min(A.nq, q0 + per);
  const int64_t cap = C.scr_cap;
  int64_t v1[1] = {0}, e1[1], t1[1];
  for (int q = q0; q < q1; ++q)
    if (A.oc[q] == kOTask) v1[0] += A.tk_cost[q];
  block_excl_scan_n<1>(v1, e1, t1);
  int64_t v2[3] = {0, 0, 0}, e2[3], t2[3];  // tiles, scratch bytes, algorithmic bytes
  int64_t run = e1[0];
  int defer = 0;
  int64_t want = 0;
  for (int q = q0; q < q1; ++q) {
    if (A.oc[q] != kOTask) continue;
    const int64_t cost = A.tk_cost[q];
    run += cost;
    if (run + 1024 > cap) {
      A.oc[q] = kODefer;
      ++defer;
      want = max(want, cost + 1024);
      continue;
    }
    v2[0] += A.tk_tiles[q];
    v2[1] += A.tk_cb[q];
    v2[2] += A.tk_alg[q];
  }
  block_excl_scan_n<3>(v2, e2, t2);
  int64_t w = e2[0], off = e2[1];
  for (int q = q0; q < q1; ++q) {
    A.w_cnt[q] = w;
    if (A.oc[q] != kOTask) continue;
    A.cnt_off[q] = off;
    A.ne[q] = 0;
    w += A.tk_tiles[q];
    off += A.tk_cb[q];
  }
  // tasks counted this round
  int64_t vt[1] = {0}, et[1], tt[1];
  for (int q = q0; q < q1; ++q) vt[0] += A.oc[q] == kOTask;
  block_excl_scan_n<1>(vt, et, tt);
  d_layout_finish(A, C, t1, t2, tt[0], defer, want);
}

// The same with thread t's queries [t * kAP, (t + 1) * kAP) held in
// registers (every field read once, all loads in flight together); up to
// kAP * kScanBlock queries.
template <int kAP>
__global__ __launch_bounds__(kScanBlock) void k_d_layout(DArgs A) {
  DCtl& C = *A.ctl;
  const int q0 = (int)threadIdx.x * kAP;
  const int64_t cap = C.scr_cap;
  int32_t oc[kAP];
  int64_t cost[kAP], tiles[kAP], cb[kAP], alg[kAP];
#pragma unroll
  for (int j = 0; j < kAP; ++j) {
    const int q = q0 + j;
    const bool in = q < A.nq;
    oc[j] = in ? A.oc[q] : kONone;
    cost[j] = in ? A.tk_cost[q] : 0;
    tiles[j] = in ? A.tk_tiles[q] : 0;
    cb[j] = in ? A.tk_cb[q] : 0;
    alg[j] = in ? A.tk_alg[q] : 0;
  }
  int64_t v1[1] = {0}, e1[1], t1[1];
#pragma unroll
  for (int j = 0; j < kAP; ++j)
    if (oc[j] == kOTask) v1[0] += cost[j];
  block_excl_scan_n<1>(v1, e1, t1);
  int64_t v2[4] = {0, 0, 0, 0}, e2[4], t2x[4];  // tiles, scratch, algorithmic bytes, tasks
  int64_t run = e1[0];
  int defer = 0;
  int64_t want = 0;
#pragma unroll
  for (int j = 0; j < kAP; ++j) {
    if (oc[j] != kOTask) continue;
    run += cost[j];
    if (run + 1024 > cap) {
      oc[j] = kODefer;
      A.oc[q0 + j] = kODefer;
      ++defer;
      want = max(want, cost[j] + 1024);
      continue;
    }
    v2[0] += tiles[j];
    v2[1] += cb[j];
    v2[2] += alg[j];
    v2[3] += 1;
  }
  block_excl_scan_n<4>(v2, e2, t2x);
  int64_t w = e2[0], off = e2[1];
#pragma unroll
  for (int j = 0; j < kAP; ++j) {
    const int q = q0 + j;
    if (q >= A.nq) break;
    A.w_cnt[q] = w;
    if (oc[j] != kOTask) continue;
    A.cnt_off[q] = off;
    A.ne[q] = 0;
    w += tiles[j];
    off += cb[j];
  }
  const int64_t t2[3] = {t2x[0], t2x[1], t2x[2]};
  d_layout_finish(A, C, t1, t2, t2x[3], defer, want);
}

template <int kT, int kS>
__global__ __launch_bounds__(kT) void k_d_count(const CTask* __restrict__ ct,
                                                    const ListRef* __restrict__ lists,
                                                    const int64_t* __restrict__ w_cnt,
                                                    const int64_t* __restrict__ cnt_off,
                                                    int64_t* __restrict__ ne, int nq,
                                                    const DCtl* __restrict__ ctl) {
  const int64_t nt = ctl->ntiles;
  int64_t* ts = ctl->ts;
  int64_t* tsn = ctl->tsn;
  char* base = ctl->scr_base;
  for (int64_t b = blockIdx.x; b < nt; b += gridDim.x) {
    const int qi = find_first_tile(w_cnt, nq, b);
    const CTask& T = ct[qi];
    char* cb = base + cnt_off[qi];
    int64_t k;
    const int64_t sum =
        b_count_tile<kT, kS>(T, b - w_cnt[qi], lists, (int32_t*)cb, (int32_t*)(cb + d_a256(4 * T.n)),
                     (uint8_t*)cb, ne + qi, &k);
    if (threadIdx.x == 0) {
      ts[b] = sum;
      tsn[b] = k;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanBlock) void k_d_scan(DArgs A) {
  const DCtl& C = *A.ctl;
  scan_tile_sums2_block(C.ts, C.tsn, C.ntiles);
}

// Output bytes of a task's table.
__device__ inline int64_t d_out_bytes(int64_t m, int kout) {
  return 4 * d_stride(m) * (int64_t)(kout > 1 ? kout : 1);
}

// Every counted task's output size and outcome; for a table to write, its
// output bytes, write scratch, tiles of the post launch, split entries,
// write tiles and algorithmic bytes.
__global__ void k_d_outcome(DArgs A) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= A.nq || A.oc[qi] != kOTask) return;
  DQ& Q = A.q[qi];
  const DCtl& C = *A.ctl;
  const CTask& c = A.ct[qi];
  const int64_t m = C.ts[A.w_cnt[qi + 1]] - C.ts[A.w_cnt[qi]];
  const int64_t n = c.n;
  const int64_t ne = Q.kind == kTaskExpand ? A.ne[qi] : 0;
  Q.m = m;
  Q.ne = ne;
  int o;
  if (Q.kind == kTaskExpand) {
    o = m == 0 ? kODone : kOWrite;
    Q.kout = Q.t.k + 1;
  } else if (Q.kind == kTaskFilter) {
    o = m == n ? kOPass : (m == 0 ? kODone : kOWrite);
    Q.kout = Q.t.k;
  } else {
    o = m == n ? kODriver : (m == 0 ? kODone : kOWrite);
    Q.kout = 1;
  }
  if (o == kOWrite && A.budget > 0 && m > A.budget / (4 * (int64_t)max(Q.kout, 1)))
    o = kOFallback;  // above the step budget: chunked by the single-query executor
  A.oc[qi] = o;
  if (o != kOWrite) return;
  const int64_t k = Q.t.k;
  int64_t sb = 0, post = d_tiles(n), part = 0, write = 0, alg_post, alg_write = 0;
  Q.sparse = Q.kind == kTaskExpand && sparse_expand(A.theta, A.min_rows, n, ne);
  if (Q.kind == kTaskExpand) {
    const int64_t pt = d_tiles((Q.sparse ? ne : n) + m);
    part = pt + 1;
    write = pt;
    sb = d_a256(8 * (pt + 1));
    if (Q.sparse) {
      sb += 2 * d_a256(4 * ne) + d_a256(8 * (ne + 1));
      alg_post = 4 * n + 20 * ne;
      alg_write = 4 * m * (k + 2) + 16 * ne + 4 * k * ne;
    } else {
      alg_post = 12 * n;
      alg_write = 4 * m * (k + 2) + 12 * n + 4 * k * ne;
    }
  } else {
    const int64_t kk = Q.kind == kTaskIntersect ? 1 : k;
    alg_post = (1 + 4 * kk) * n + 4 * kk * m;
  }
  A.wz_ob[qi] = d_out_bytes(m, Q.kout);
  A.wz_sb[qi] = sb;
  A.wz_post[qi] = post;
  A.wz_part[qi] = part;
  A.wz_write[qi] = write;
  A.wz_alg_post[qi] = alg_post;
  A.wz_alg_write[qi] = alg_write;
}

// k_d_alloc: output tables and write scratch of the tables to write,
// bump-allocated; the launch groups' first tiles.  One workgroup of
// kScanBlock threads.  The round's outputs above the round budget send the
// later queries to the single-query executor; a table or scratch that does
// not fit the current regions waits for a later round.  Both rules keep a
// prefix of the tasks in query order.
//
// Its end: the round's totals, deferrals and statistics (tc: totals of the
// seven per-table sums; tb: of the two table sizes).
__device__ inline void d_alloc_finish(DArgs& A, DCtl& C, const int64_t (&tc)[7],
                                      const int64_t (&tb)[2], int defer, int64_t want_o,
                                      int64_t want_s, int64_t out_used, int64_t scr_used) {
  __shared__ int s_defer;
  __shared__ unsigned long long s_wo, s_ws;
  if (threadIdx.x == 0) {
    s_defer = 0;
    s_wo = s_ws = 0;
  }
  __syncthreads();
  if (defer) {
    atomicAdd(&s_defer, defer);
    atomicMax(&s_wo, (unsigned long long)want_o);
    atomicMax(&s_ws, (unsigned long long)want_s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    A.w_post[A.nq] = tc[0];
    A.w_part[A.nq] = tc[1];
    A.w_write[A.nq] = tc[2];
    C.n_post = tc[0];
    C.n_part = tc[1];
    C.n_write = tc[2];
    C.out_used = out_used + tc[3];
    C.scr_used = scr_used + tc[4];
    C.scr_peak = max(C.scr_peak, C.scr_used);
    C.scr_need = max(C.scr_need, scr_used + tb[1]);
    if (C.round < kStatRounds) {
      int64_t* st = C.stats[C.round];
      st[2] = tc[0];
      st[3] = tc[2];
      st[4] = tc[1];  // split entries: tables written + path tiles
      st[5] = tc[3];
      st[7] += s_defer;
    }
    C.round += 1;
    C.bytes_post += tc[5];
    C.bytes_write += tc[6];
    C.deferred += s_defer;
    C.want_out = max(C.want_out, (int64_t)s_wo);
    C.want_scr = max(C.want_scr, (int64_t)s_ws);
  }
}

// Any number of queries: thread t takes queries [t * per, (t + 1) * per).
__global__ __launch_bounds__(kScanBlock) void k_d_alloc_loop(DArgs A) {
  DCtl& C = *A.ctl;
  const int per = (A.nq + kScanBlock - 1) / kScanBlock;
  const int q0 = min(A.nq, (int)threadIdx.x * per), q1 = min(A.nq, q0 + per);
  int64_t va[1] = {0}, ea[1], ta[1];
  for (int q = q0; q < q1; ++q)
    if (A.oc[q] == kOWrite) va[0] += A.wz_ob[q];
  block_excl_scan_n<1>(va, ea, ta);
  int64_t vb[2] = {0, 0}, eb[2], tb[2];
  int64_t run = ea[0];
  for (int q = q0; q < q1; ++q) {
    if (A.oc[q] != kOWrite) continue;
    const int64_t ob = A.wz_ob[q];
    const bool over = A.round_budget > 0 && run > 0 && run + ob > A.round_budget;
    run += ob;
    if (over) {
      A.oc[q] = kOFallback;
      continue;
    }
    vb[0] += ob;
    vb[1] += A.wz_sb[q];
  }
  block_excl_scan_n<2>(vb, eb, tb);
  int64_t vc[7] = {0, 0, 0, 0, 0, 0, 0}, ec[7], tc[7];
  int64_t ro = eb[0], rs = eb[1];
  const int64_t out_used = C.out_used, scr_used = C.scr_used;
  const int64_t out_cap = C.out_cap, scr_cap = C.scr_cap;
  int defer = 0;
  int64_t want_o = 0, want_s = 0;
  for (int q = q0; q < q1; ++q) {
    if (A.oc[q] != kOWrite) continue;
    const int64_t ob = A.wz_ob[q], sb = A.wz_sb[q];
    if (out_used + ro + ob <= out_cap && scr_used + rs + sb <= scr_cap) {
      A.out_off[q] = out_used + ro;
      A.scr_off[q] = scr_used + rs;
      vc[0] += A.wz_post[q];
      vc[1] += A.wz_part[q];
      vc[2] += A.wz_write[q];
      vc[3] += ob;
      vc[4] += sb;
      vc[5] += A.wz_alg_post[q];
      vc[6] += A.wz_alg_write[q];
    } else {
      A.oc[q] = kODefer;
      ++defer;
      want_o = max(want_o, ob);
      want_s = max(want_s, A.tk_cost[q] + sb + 1024);
    }
    ro += ob;
    rs += sb;
  }
  block_excl_scan_n<7>(vc, ec, tc);
  int64_t wp = ec[0], wq = ec[1], ww = ec[2];
  for (int q = q0; q < q1; ++q) {
    A.w_post[q] = wp;
    A.w_part[q] = wq;
    A.w_write[q] = ww;
    if (A.oc[q] != kOWrite) continue;
    wp += A.wz_post[q];
    wq += A.wz_part[q];
    ww += A.wz_write[q];
  }
  d_alloc_finish(A, C, tc, tb, defer, want_o, want_s, out_used, scr_used);
}

// Up to kAP * kScanBlock queries: thread t holds queries [t * kAP, (t + 1) *
// kAP) in registers, every field read once with all loads in flight together
// (the loop above waits for each query's loads in turn).  Same rules, same
// results.
template <int kAP>
__global__ __launch_bounds__(kScanBlock) void k_d_alloc(DArgs A) {
  DCtl& C = *A.ctl;
  const int q0 = (int)threadIdx.x * kAP;
  int32_t oc[kAP];
  int64_t ob[kAP], sb[kAP], zp[kAP], zq[kAP], zw[kAP], ap[kAP], aw[kAP], cost[kAP];
#pragma unroll
  for (int j = 0; j < kAP; ++j) {
    const int q = q0 + j;
    const bool in = q < A.nq;
    oc[j] = in ? A.oc[q] : kONone;
    ob[j] = in ? A.wz_ob[q] : 0;
    sb[j] = in ? A.wz_sb[q] : 0;
    zp[j] = in ? A.wz_post[q] : 0;
    zq[j] = in ? A.wz_part[q] : 0;
    zw[j] = in ? A.wz_write[q] : 0;
    ap[j] = in ? A.wz_alg_post[q] : 0;
    aw[j] = in ? A.wz_alg_write[q] : 0;
    cost[j] = in ? A.tk_cost[q] : 0;
  }
  int64_t va[1] = {0}, ea[1], ta[1];
#pragma unroll
  for (int j = 0; j < kAP; ++j)
    if (oc[j] == kOWrite) va[0] += ob[j];
  block_excl_scan_n<1>(va, ea, ta);
  int64_t vb[2] = {0, 0}, eb[2], tb[2];
  int64_t run = ea[0];
  bool changed[kAP];
#pragma unroll
  for (int j = 0; j < kAP; ++j) {
    changed[j] = false;
    if (oc[j] != kOWrite) continue;
    const bool over = A.round_budget > 0 && run > 0 && run + ob[j] > A.round_budget;
    run += ob[j];
    if (over) {
      oc[j] = kOFallback;
      changed[j] = true;
      continue;
    }
    vb[0] += ob[j];
    vb[1] += sb[j];
  }
  block_excl_scan_n<2>(vb, eb, tb);
  int64_t vc[7] = {0, 0, 0, 0, 0, 0, 0}, ec[7], tc[7];
  int64_t ro = eb[0], rs = eb[1];
  const int64_t out_used = C.out_used, scr_used = C.scr_used;
  const int64_t out_cap = C.out_cap, scr_cap = C.scr_cap;
  int defer = 0;
  int64_t want_o = 0, want_s = 0;
#pragma unroll
  for (int j = 0; j < kAP; ++j) {
    if (oc[j] != kOWrite) continue;
    if (out_used + ro + ob[j] <= out_cap && scr_used + rs + sb[j] <= scr_cap) {
      A.out_off[q0 + j] = out_used + ro;
      A.scr_off[q0 + j] = scr_used + rs;
      vc[0] += zp[j];
      vc[1] += zq[j];
      vc[2] += zw[j];
      vc[3] += ob[j];
      vc[4] += sb[j];
      vc[5] += ap[j];
      vc[6] += aw[j];
    } else {
      oc[j] = kODefer;
      changed[j] = true;
      ++defer;
      want_o = max(want_o, ob[j]);
      want_s = max(want_s, cost[j] + sb[j] + 1024);
    }
    ro += ob[j];
    rs += sb[j];
  }
  block_excl_scan_n<7>(vc, ec, tc);
  int64_t wp = ec[0], wq = ec[1], ww = ec[2];
#pragma unroll
  for (int j = 0; j < kAP; ++j) {
    const int q = q0 + j;
    if (q >= A.nq) break;
    A.w_post[q] = wp;
    A.w_part[q] = wq;
    A.w_write[q] = ww;
    if (changed[j]) A.oc[q] = oc[j];
    if (oc[j] != kOWrite) continue;
    wp += zp[j];
    wq += zq[j];
    ww += zw[j];
  }
  d_alloc_finish(A, C, tc, tb, defer, want_o, want_s, out_used, scr_used);
}

// Write descriptors of the tables to write.
__global__ void k_d_describe(DArgs A) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= A.nq || A.oc[qi] != kOWrite) return;
  const DQ& Q = A.q[qi];
  const DCtl& C = *A.ctl;
  const CTask& c = A.ct[qi];
  // fields written one by one (a local descriptor would go through private memory)
  WTask& w = A.wt[qi];
  const int64_t m = Q.m;
  w.nbr = nullptr;
  w.N = nullptr;
  w.start = nullptr;
  w.P = nullptr;
  w.split = nullptr;
  w.flags = nullptr;
  w.ridx = nullptr;
  w.cstart = nullptr;
  w.start_in = nullptr;
  w.n_in = 0;
  w.n = c.n;
  w.m = m;
  w.t0 = A.w_cnt[qi];
  w.out0 = (int32_t*)(C.out_base + A.out_off[qi]);
  w.ostride = d_stride(m);
  char* sb = C.scr_base + A.scr_off[qi];
  char* cb = C.scr_base + A.cnt_off[qi];
  if (Q.kind == kTaskExpand) {
    w.k = Q.t.k;
    for (int cc = 0; cc < Q.t.k; ++cc) w.in.c[cc] = Q.t.col[cc];
    w.nbr = c.pv.nbr;
    w.N = (const int32_t*)cb;
    const int32_t* start = (const int32_t*)(cb + d_a256(4 * c.n));
    if (Q.sparse) {
      const int64_t ne = Q.ne;
      w.n_in = c.n;
      w.n = ne;
      w.start_in = start;
      w.ridx = (int32_t*)sb;
      w.cstart = (int32_t*)(sb + d_a256(4 * ne));
      w.P = (int64_t*)(sb + 2 * d_a256(4 * ne));
      w.start = w.cstart;
      w.split = (int64_t*)(sb + 2 * d_a256(4 * ne) + d_a256(8 * (ne + 1)));
    } else {
      w.start = start;
      w.P = (int64_t*)(cb + 2 * d_a256(4 * c.n));
      w.split = (int64_t*)sb;
    }
  } else {
    if (Q.kind == kTaskFilter) {
      w.k = Q.t.k;
      for (int cc = 0; cc < Q.t.k; ++cc) w.in.c[cc] = Q.t.col[cc];
    } else {
      w.k = 1;
      w.in.c[0] = c.col;
    }
    w.flags = (const uint8_t*)cb;
  }
}

// Row offsets of the dense expansions, rows with output of the sparse ones,
// compactions of the filters and intersections.
__global__ __launch_bounds__(kBlock) void k_d_post(const WTask* __restrict__ wt,
                                                   const int64_t* __restrict__ w_post, int nq,
                                                   const DCtl* __restrict__ ctl) {
  const int64_t nt = ctl->n_post;
  const int64_t* ts = ctl->ts;
  const int64_t* tsn = ctl->tsn;
  for (int64_t b = blockIdx.x; b < nt; b += gridDim.x) {
    const int qi = find_first_tile(w_post, nq, b);
    const WTask& T = wt[qi];
    const int64_t tile = b - w_post[qi];
    if (T.flags) b_compact_tile_any(T, tile, ts);
    else if (T.ridx) b_compact_rows_tile(T, tile, ts, tsn);
    else b_scan_add_tile(T, tile, ts);
    __syncthreads();  // the next tile reuses the LDS
  }
}

__global__ __launch_bounds__(kBlock) void k_d_partition(const WTask* __restrict__ wt,
                                                        const int64_t* __restrict__ w_part,
                                                        int nq, const DCtl* __restrict__ ctl) {
  const int64_t total = ctl->n_part;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int qi = find_first_tile(w_part, nq, g);
    const WTask& T = wt[qi];
    T.split[g - w_part[qi]] = mp_split(T.P, T.n, 0, T.m, g - w_part[qi]);
  }
}

// Every expansion write of the round, dense and compacted, any column count.
__global__ __launch_bounds__(kBlock) void k_d_write(const WTask* __restrict__ wt,
                                                    const int64_t* __restrict__ w_write, int nq,
                                                    const DCtl* __restrict__ ctl) {
  __shared__ int32_t sE[kTile + 1];
  __shared__ int32_t sRb[kTile + 1];
  __shared__ uint16_t sRow[kTile];
  const TileLds L{sE, sRb, sRow, nullptr};
  const int64_t nt = ctl->n_write;
  for (int64_t b = blockIdx.x; b < nt; b += gridDim.x) {
    const int qi = find_first_tile(w_write, nq, b);
    const WTask& T = wt[qi];
    const int64_t t = b - w_write[qi];
    if (T.ridx) b_write_tile_any<true>(T, t, L);
    else b_write_tile_any<false>(T, t, L);
    __syncthreads();  // the next tile reuses the LDS
  }
}

// ------------------------------------------------------------------ host

// Growable pinned host buffer.
struct PinnedBuf {
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
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
};
PinnedBuf& pin_in() {
  thread_local PinnedBuf b;
  return b;
}
PinnedBuf& pin_out() {
  thread_local PinnedBuf b;
  return b;
}
PinnedBuf& pin_ctl() {
  thread_local PinnedBuf b;
  return b;
}

struct Lay {
  size_t bytes = 0;
  size_t add(size_t b) {
    const size_t at = bytes;
    bytes += (b + 255) / 256 * 256;
    return at;
  }
};

int64_t round_up(int64_t b, int64_t g) { return (b + g - 1) / g * g; }

// Workgroups of each tile kernel: as many as the device holds at once (the
// kernels take tiles from a counter, so more would only wait for a slot).
struct Grids {
  unsigned sample, post, write;  // the count launch's: count_resident()
};
const Grids& resident_grids() {
  static Grids g = [] {
    int dev = 0, cus = 0;
    GS_HIP(hipGetDevice(&dev));
    GS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    auto res = [&](const void* k) {
      int per = 0;
      GS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, kBlock, 0));
      return (unsigned)std::max(1, per * std::max(cus, 1));
    };
    return Grids{res((const void*)k_d_sample), res((const void*)k_d_post),
                 res((const void*)k_d_write)};
  }();
  return g;
}

#define GS_DLAUNCH(cls, kern, grid, block, ...)                               \
  do {                                                                       \
    const bool _prof = prof_on(cls);                                         \
    if (_prof) prof_begin(s, cls);                                           \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, __VA_ARGS__);    \
    GS_HIP(hipGetLastError());                                               \
    if (_prof) prof_end(s, cls, 0.0);                                        \
  } while (0)

// The count launch for the store's tile shape (threads per workgroup) and
// intersection strategy; every variant takes the same tiles, so the round's
// scratch layout does not depend on the choice.
template <int kT, int kS>
unsigned count_resident() {
  static const unsigned r = [] {
    int dev = 0, cus = 0, per = 0;
    GS_HIP(hipGetDevice(&dev));
    GS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    GS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_d_count<kT, kS>, kT,
                                                        0));
    return (unsigned)std::max(1, per * std::max(cus, 1));
  }();
  return r;
}
template <int kT, int kS>
void launch_count_as(hipStream_t s, const DArgs& A, int nq, const std::function<unsigned(unsigned)>& grid) {
  auto k = k_d_count<kT, kS>;
  GS_DLAUNCH(GSMAT_K_COUNT, k, grid(count_resident<kT, kS>()), kT, A.ct, A.lists, A.w_cnt,
             A.cnt_off, A.ne, nq, A.ctl);
}
template <int kS>
void launch_count_s(int items, hipStream_t s, const DArgs& A, int nq,
                    const std::function<unsigned(unsigned)>& grid) {
  if (items == 4) return launch_count_as<kTile / 4, kS>(s, A, nq, grid);
  if (items == 16) return launch_count_as<kTile / 16, kS>(s, A, nq, grid);
  return launch_count_as<kTile / 8, kS>(s, A, nq, grid);
}
void launch_count(int items, int strategy, hipStream_t s, const DArgs& A, int nq,
                  const std::function<unsigned(unsigned)>& grid) {
  if (strategy == kIsWindow) return launch_count_s<kIsWindow>(items, s, A, nq, grid);
  if (strategy == kIsMerge) return launch_count_s<kIsMerge>(items, s, A, nq, grid);
  return launch_count_s<kIsSearch>(items, s, A, nq, grid);
}

}  // namespace

// The host side of a device-driven batch: the upload's row widths, each
// query's variables and steps, and the filler of its upload rows (queries
// [lo, hi): pq[i], pats and lookups [i * mp, (i + 1) * mp), steps
// [i * ms, (i + 1) * ms)).  n_vars and n_steps are read after fill.
struct PackedBatch {
  int32_t nq = 0;
  int mp = 1, ms = 1, mv = 1;
  std::vector<int32_t> n_vars, n_steps;
  std::function<void(DPlanQ*, DPat*, DStep*, DLk*)> fill;
};

void run_batch_packed(gsmat_store* st, PackedBatch& pb, int64_t budget, int64_t max_rows,
                      hipStream_t s, std::vector<DevQueryOut>& out) {
  const int32_t nq = pb.nq;
  out.assign(nq, DevQueryOut{nullptr, kDevDone, GSMAT_OK});
  if (nq == 0) return;
  DeviceMem* mem = st->mem.get();
  const int mp = pb.mp, ms = pb.ms, mv = pb.mv;
  const size_t n = (size_t)nq;
  // ---- device layout: uploaded inputs first, then the state
  Lay L;
  const size_t o_pq = L.add(sizeof(DPlanQ) * n), o_pats = L.add(sizeof(DPat) * n * mp),
               o_steps = L.add(sizeof(DStep) * n * ms), o_lkin = L.add(sizeof(DLk) * n * mp),
               o_ctl = L.add(sizeof(DCtl));
  const size_t up_bytes = L.bytes;
  const size_t o_lk = L.add(sizeof(LookupRes) * n * mp), o_q = L.add(sizeof(DQ) * n),
               o_cands = L.add(sizeof(SCand) * n * mp),
               o_part = L.add(sizeof(int64_t) * n * mp * kSampleBlocks),
               o_ct = L.add(sizeof(CTask) * n), o_lists = L.add(sizeof(ListRef) * n * kMaxLists),
               o_wt = L.add(sizeof(WTask) * n), o_ne = L.add(sizeof(int64_t) * n),
               o_wc = L.add(sizeof(int64_t) * (n + 1)), o_wpo = L.add(sizeof(int64_t) * (n + 1)),
               o_wpa = L.add(sizeof(int64_t) * (n + 1)), o_ww = L.add(sizeof(int64_t) * (n + 1)),
               o_oc = L.add(sizeof(int32_t) * n);
  constexpr int kSoa = 14;  // per-query int64 arrays
  size_t o_soa[kSoa];
  for (int i = 0; i < kSoa; ++i) o_soa[i] = L.add(sizeof(int64_t) * n);
  // read back at the end, contiguous: results, their columns, step counters
  const size_t o_res = L.add(sizeof(DRes) * n), o_rcol = L.add(sizeof(int32_t*) * n * mv),
               o_sin = L.add(sizeof(int64_t) * n * ms), o_sout = L.add(sizeof(int64_t) * n * ms);
  const size_t back_bytes = L.bytes - o_res;
  Arena state(mem, L.bytes, s);
  char* dv = (char*)state.p;

  // ---- memory regions: the output slab and the round scratch
  const int64_t g = (int64_t)1 << 20;  // sizes are kept in whole MiB
  int64_t out_cap = st->dbatch_out_hint > 0 ? st->dbatch_out_hint : (int64_t)256 << 20;
  int64_t scr_cap = st->dbatch_scr_hint > 0 ? st->dbatch_scr_hint : (int64_t)128 << 20;
  scr_cap = std::max<int64_t>(scr_cap, 4096);  // the tile-sum arrays of an empty round
  std::vector<std::shared_ptr<Arena>> slabs;
  slabs.push_back(std::make_shared<Arena>(mem, (size_t)out_cap, s));
  std::unique_ptr<Arena> scr(new Arena(mem, (size_t)scr_cap, s));

  // ---- the upload: every query's plan rows, then the control block
  char* h = (char*)pin_in().get(up_bytes);
  DPlanQ* hpq = (DPlanQ*)(h + o_pq);
  DPat* hpats = (DPat*)(h + o_pats);
  DStep* hsteps = (DStep*)(h + o_steps);
  DLk* hlk = (DLk*)(h + o_lkin);
  pb.fill(hpq, hpats, hsteps, hlk);
  DCtl* hctl = (DCtl*)(h + o_ctl);
  std::memset(hctl, 0, sizeof(DCtl));
  hctl->out_base = (char*)slabs[0]->p;
  hctl->out_cap = out_cap;
  hctl->scr_base = (char*)scr->p;
  hctl->scr_cap = scr_cap;
  GS_HIP(hipMemcpyAsync(dv, h, up_bytes, hipMemcpyHostToDevice, s));

  DArgs A{};
  A.nq = nq;
  A.mp = mp;
  A.ms = ms;
  A.mv = mv;
  A.budget = budget;
  A.round_budget = budget;
  A.max_rows = max_rows;
  A.theta = st->sparse_theta;
  A.min_rows = st->sparse_min_rows;
  A.dout = st->out.d_desc;
  A.din = st->in.d_desc;
  A.out = st->out.ptrs();
  A.in = st->in.ptrs();
  A.out_src = st->out.src;
  A.pq = (const DPlanQ*)(dv + o_pq);
  A.pats = (const DPat*)(dv + o_pats);
  A.steps = (const DStep*)(dv + o_steps);
  A.lkin = (const DLk*)(dv + o_lkin);
  A.lk = (LookupRes*)(dv + o_lk);
  A.q = (DQ*)(dv + o_q);
  A.sin = (int64_t*)(dv + o_sin);
  A.sout = (int64_t*)(dv + o_sout);
  A.cands = (SCand*)(dv + o_cands);
  A.part = (int64_t*)(dv + o_part);
  A.ct = (CTask*)(dv + o_ct);
  A.lists = (ListRef*)(dv + o_lists);
  A.wt = (WTask*)(dv + o_wt);
  A.ne = (int64_t*)(dv + o_ne);
  A.w_cnt = (int64_t*)(dv + o_wc);
  A.w_post = (int64_t*)(dv + o_wpo);
  A.w_part = (int64_t*)(dv + o_wpa);
  A.w_write = (int64_t*)(dv + o_ww);
  A.oc = (int32_t*)(dv + o_oc);
  int64_t** soa[kSoa] = {&A.tk_cost, &A.tk_tiles, &A.tk_cb, &A.tk_alg, &A.cnt_off,
                         &A.wz_ob, &A.wz_sb, &A.wz_post, &A.wz_part, &A.wz_write,
                         &A.wz_alg_post, &A.wz_alg_write, &A.out_off, &A.scr_off};
  for (int i = 0; i < kSoa; ++i) *soa[i] = (int64_t*)(dv + o_soa[i]);
  A.ctl = (DCtl*)(dv + o_ctl);
  A.res = (DRes*)(dv + o_res);
  A.res_col = (const int32_t**)(dv + o_rcol);

  const unsigned qgrid = (unsigned)ceil_div(nq, kQBlock);
  const Grids& grids = resident_grids();
  GS_DLAUNCH(GSMAT_K_OTHER, k_d_init, qgrid, kQBlock, A);
  DCtl* hc = (DCtl*)pin_ctl().get(sizeof(DCtl));
  char* hb = (char*)pin_out().get(back_bytes);
  // every round completes at least one pattern of each query that is not
  // deferred (an intersection first step: none), so mp + 1 rounds finish
  // every query unless memory ran short
  const int rounds = mp + 1;
  // Launch sizes: a tile kernel whose round had T tiles in the store's last
  // batch gets a grid of T (plus an eighth) workgroups, one tile each when
  // the round repeats; otherwise, or when there are more tiles, the
  // workgroups stride over the tiles, and never fewer than the device holds.
  const std::vector<int64_t> prev = st->dbatch_stats;
  auto hinted = [&](int gr, int f, unsigned floor_) -> unsigned {
    if ((size_t)(gr + 1) * kStatFields > prev.size()) return floor_;
    const int64_t t = prev[(size_t)gr * kStatFields + f];
    return (unsigned)std::min<int64_t>(std::max<int64_t>(t + t / 8, floor_), 1 << 22);
  };
  int64_t out_total = 0;
  std::vector<std::unique_ptr<gsmat_result>> made;
  int gr = 0;  // rounds launched so far
  for (int iter = 0;; ++iter) {
    for (int r = 0; r < rounds; ++r, ++gr) {
      GS_DLAUNCH(GSMAT_K_OTHER, k_d_choose, qgrid, kQBlock, A, 1);
      GS_DLAUNCH(GSMAT_K_OTHER, k_d_sample, grids.sample, kBlock, A.cands, A.part, A.ctl);
      GS_DLAUNCH(GSMAT_K_OTHER, k_d_task, qgrid, kQBlock, A);
      if (nq <= kAllocRegs * kScanBlock) {
        GS_DLAUNCH(GSMAT_K_SCAN, k_d_layout<kAllocRegs>, 1, kScanBlock, A);
      } else {
        GS_DLAUNCH(GSMAT_K_SCAN, k_d_layout_loop, 1, kScanBlock, A);
      }
      launch_count(st->count_items, st->intersect, s, A, nq,
                   [&](unsigned floor_) { return hinted(gr, 1, floor_); });
      GS_DLAUNCH(GSMAT_K_SCAN, k_d_scan, 1, kScanBlock, A);
      GS_DLAUNCH(GSMAT_K_OTHER, k_d_outcome, qgrid, kQBlock, A);
      if (nq <= kAllocRegs * kScanBlock) {
        GS_DLAUNCH(GSMAT_K_SCAN, k_d_alloc<kAllocRegs>, 1, kScanBlock, A);
      } else {
        GS_DLAUNCH(GSMAT_K_SCAN, k_d_alloc_loop, 1, kScanBlock, A);
      }
      GS_DLAUNCH(GSMAT_K_OTHER, k_d_describe, qgrid, kQBlock, A);
      GS_DLAUNCH(GSMAT_K_COMPACT, k_d_post, hinted(gr, 2, grids.post), kBlock, A.wt, A.w_post,
                 nq, A.ctl);
      GS_DLAUNCH(GSMAT_K_OTHER, k_d_partition, kPartGrid, kBlock, A.wt, A.w_part, nq, A.ctl);
      GS_DLAUNCH(GSMAT_K_WRITE, k_d_write, hinted(gr, 3, grids.write), kBlock, A.wt, A.w_write,
                 nq, A.ctl);
    }
    GS_DLAUNCH(GSMAT_K_OTHER, k_d_choose, qgrid, kQBlock, A, 0);
    // the summary, and the results in case every query has finished
    GS_HIP(hipMemcpyAsync(hc, A.ctl, sizeof(DCtl), hipMemcpyDeviceToHost, s));
    GS_HIP(hipMemcpyAsync(hb, dv + o_res, back_bytes, hipMemcpyDeviceToHost, s));
    if (iter == 0) {
      // while the device runs: the result objects, filled after the wait
      made.resize(nq);
      for (int i = 0; i < nq; ++i) {
        gsmat_result* r = new gsmat_result;
        made[i].reset(r);
        r->st = st;
        r->stream = s;
        r->n_vars = pb.n_vars[i];
        r->reset_steps(pb.n_steps[i]);
        r->segs.reserve(1);
      }
    }
    host_sync(s);
    if (hc->error) throw StatusFail{GSMAT_EHIP, "internal: batched join state inconsistent"};
    if (hc->active == 0 || iter >= 16) break;
    if (hc->deferred == 0)  // cannot happen: a query needs more rounds only after a deferral
      throw StatusFail{GSMAT_EHIP, "internal: batched join made no progress"};
    // the regions were too small: a larger output slab and scratch region
    if (hc->want_out > 0) {
      out_total += hc->out_used;
      const int64_t cap = round_up(std::max(2 * hc->out_cap, 2 * hc->want_out), g);
      slabs.push_back(std::make_shared<Arena>(mem, (size_t)cap, s));
      hc->out_base = (char*)slabs.back()->p;
      hc->out_cap = cap;
      hc->out_used = 0;
      hc->out_slab = (int32_t)slabs.size() - 1;
    }
    if (hc->want_scr > 0) {
      const int64_t cap = round_up(std::max(2 * hc->scr_cap, hc->want_scr), g);
      scr.reset(new Arena(mem, (size_t)cap, s));
      hc->scr_base = (char*)scr->p;
      hc->scr_cap = cap;
    }
    hc->deferred = 0;
    hc->want_out = hc->want_scr = 0;
    GS_HIP(hipMemcpyAsync(A.ctl, hc, sizeof(DCtl), hipMemcpyHostToDevice, s));
  }
  out_total += hc->out_used;
  // the pass's sizes are the next pass's starting regions
  st->dbatch_out_hint = std::max<int64_t>(round_up(out_total + out_total / 8, g), g);
  st->dbatch_scr_hint = std::max<int64_t>(round_up(hc->scr_need + hc->scr_need / 8, g), g);
  st->dbatch_stats.assign(&hc->stats[0][0],
                          &hc->stats[0][0] + (size_t)std::min(hc->round, kStatRounds) * kStatFields);
  prof_add_bytes(GSMAT_K_COUNT, (double)hc->bytes_count);
  prof_add_bytes(GSMAT_K_COMPACT, (double)hc->bytes_post);
  prof_add_bytes(GSMAT_K_WRITE, (double)hc->bytes_write);

  // ---- results (read back with the last summary)
  const DRes* hr = (const DRes*)hb;
  const int32_t* const* hcol = (const int32_t* const*)(hb + (o_rcol - o_res));
  const int64_t* hsin = (const int64_t*)(hb + (o_sin - o_res));
  const int64_t* hsout = (const int64_t*)(hb + (o_sout - o_res));
  for (int i = 0; i < nq; ++i) {
    const DRes& r = hr[i];
    DevQueryOut& o = out[i];
    if (r.state == kQFailed) {
      o.state = kDevFailed;
      o.status = r.status;
      continue;
    }
    if (r.state != kQDone) {  // left the batch (or unfinished): run alone
      o.state = kDevFallback;
      continue;
    }
    std::unique_ptr<gsmat_result>& res = made[i];
    for (int j = 0; j < pb.n_steps[i]; ++j) {
      res->step_in[j] = hsin[(size_t)i * ms + j];
      res->step_out[j] = hsout[(size_t)i * ms + j];
    }
    if (r.rows > 0) {
      Segment seg;
      seg.rows = r.rows;
      for (int v = 0; v < pb.n_vars[i]; ++v) seg.col[v] = hcol[(size_t)i * mv + v];
      if (r.slab >= 0) {
        if (r.slab >= (int)slabs.size())
          throw StatusFail{GSMAT_EHIP, "internal: result in an unknown slab"};
        seg.keep = slabs[r.slab];
      }
      res->rows = r.rows;
      res->segs.push_back(seg);
    }
    o.res = res.release();
    o.state = kDevDone;
  }
}


// One query's upload rows from its plan.
void pack_plan(const gsmat_store* st, const gsmat_query_plan* pl, int mp, int ms, DPlanQ& q,
               DPat* pats, DStep* steps, DLk* lk) {
  const int np = (int)pl->pats.size();
  const bool have = pl->lk_store == st->uid && pl->lk.size() == pl->pats.size();
  q.np = np;
  q.nsteps = (int)pl->steps.size();
  q.nv = pl->n_vars;
  q.mode = pl->mode;
  q.absent = 0;
  q.pad = 0;
  for (int j = 0; j < mp; ++j) {
    DPat& d = pats[j];
    DLk& l = lk[j];
    if (j < np) {
      const gsmat_pattern& p = pl->pats[j];
      d = DPat{p.s, p.p, p.o};
      if (p.p >= st->P || (p.s >= 0 && p.s >= st->V) || (p.o >= 0 && p.o >= st->V))
        q.absent = 1;
      l = have && pl->lk[j].valid ? DLk{pl->lk[j].start, pl->lk[j].len, pl->lk[j].found, 1}
                                  : DLk{0, 0, 0, 0};
    } else {
      d = DPat{0, 0, 0};
      l = DLk{0, 0, 0, 0};
    }
  }
  for (int j = 0; j < ms; ++j) {
    DStep& d = steps[j];
    if (j < q.nsteps) {
      const gsmat_step_info& sp = pl->steps[j];
      d = DStep{(int8_t)sp.kind, (int8_t)sp.tp, (int8_t)sp.orient, (int8_t)sp.var, sp.members};
    } else {
      d = DStep{0, 0, 0, 0, 0u};
    }
  }
}

void run_batch_device(gsmat_store* st, const gsmat_query_plan* const* plans, int32_t nq,
                      int64_t budget, int64_t max_rows, hipStream_t s,
                      std::vector<DevQueryOut>& out) {
  PackedBatch pb;
  pb.nq = nq;
  pb.n_vars.resize(nq);
  pb.n_steps.resize(nq);
  for (int i = 0; i < nq; ++i) {
    pb.mp = std::max(pb.mp, (int)plans[i]->pats.size());
    pb.ms = std::max(pb.ms, (int)plans[i]->steps.size());
    pb.mv = std::max(pb.mv, (int)plans[i]->n_vars);
    pb.n_vars[i] = plans[i]->n_vars;
    pb.n_steps[i] = (int32_t)plans[i]->steps.size();
  }
  pb.fill = [&](DPlanQ* pq, DPat* pats, DStep* steps, DLk* lk) {
    for (int i = 0; i < nq; ++i)
      pack_plan(st, plans[i], pb.mp, pb.ms, pq[i], pats + (size_t)i * pb.mp,
                steps + (size_t)i * pb.ms, lk + (size_t)i * pb.mp);
  };
  run_batch_packed(st, pb, budget, max_rows, s, out);
}

void run_batch_device_bgp(gsmat_store* st, const gsmat_pattern* pats, const int32_t* n_pats,
                          int32_t nq, int32_t mode, int64_t budget, int64_t max_rows,
                          hipStream_t s, std::vector<DevQueryOut>& out,
                          std::vector<gsmat_status>& status, std::vector<std::string>& msg,
                          std::vector<std::unique_ptr<gsmat_query_plan>>& fallback) {
  PlanPrep P;
  plan_prepare(st, pats, n_pats, nq, mode, s, &P);
  // the valid queries form the batch, in order
  std::vector<int32_t> vi;
  vi.reserve(nq);
  PackedBatch pb;
  for (int i = 0; i < nq; ++i) {
    if (P.rc[i] != GSMAT_OK) continue;
    vi.push_back(i);
    pb.mp = std::max(pb.mp, n_pats[i]);
    pb.mv = std::max(pb.mv, P.nv[i]);
  }
  pb.nq = (int32_t)vi.size();
  pb.ms = pb.mp + 1;  // at most one step per pattern, plus an intersection
  pb.n_vars.assign(pb.nq, 0);
  pb.n_steps.assign(pb.nq, 0);
  // each plan is built in a per-thread scratch plan and packed at once
  pb.fill = [&](DPlanQ* pq, DPat* up, DStep* us, DLk* ul) {
    host_parallel_for(pb.nq, 256, [&](int64_t lo, int64_t hi) {
      gsmat_query_plan pl;
      for (int64_t k = lo; k < hi; ++k) {
        const int i = vi[k];
        try {
          P.rc[i] = plan_build(st, pats, n_pats, mode, P, i, &pl);
        } catch (...) {
          P.rc[i] = GSMAT_ENOMEM;
          P.msg[i] = "host memory exhausted while planning";
        }
        if (P.rc[i] != GSMAT_OK) {  // cannot happen after validation: an empty query
          pl = gsmat_query_plan();
          pl.n_vars = P.nv[i];
        }
        pack_plan(st, &pl, pb.mp, pb.ms, pq[k], up + (size_t)k * pb.mp,
                  us + (size_t)k * pb.ms, ul + (size_t)k * pb.mp);
        if (P.rc[i] != GSMAT_OK) pq[k].absent = 1;
        pb.n_vars[k] = pl.n_vars;
        pb.n_steps[k] = (int32_t)pl.steps.size();
      }
    });
  };
  std::vector<DevQueryOut> dq;
  run_batch_packed(st, pb, budget, max_rows, s, dq);
  out.assign(nq, DevQueryOut{nullptr, kDevFailed, GSMAT_OK});
  fallback.clear();
  fallback.resize(nq);
  for (int32_t k = 0; k < pb.nq; ++k) {
    const int i = vi[k];
    out[i] = dq[k];
    if (P.rc[i] != GSMAT_OK) {  // planning failed after all: drop any result
      if (out[i].res) gsmat_result_free(out[i].res);
      out[i] = DevQueryOut{nullptr, kDevFailed, P.rc[i]};
      continue;
    }
    if (dq[k].state == kDevFallback) {  // runs alone: it needs its plan object
      fallback[i].reset(new gsmat_query_plan);
      const gsmat_status rc = plan_build(st, pats, n_pats, mode, P, i, fallback[i].get());
      if (rc != GSMAT_OK) throw StatusFail{rc, P.msg[i]};
    }
  }
  status = P.rc;
  msg = P.msg;
}

}  // namespace gsmat
