// Host-side executor types shared by the single-query and the batched join:
// binding tables, result segments, and the adaptive step selection.
#pragma once

#include <algorithm>
#include <memory>

#include "store.hpp"

namespace gsmat {

inline bool is_var(int32_t t) { return t < 0; }
inline int var_of(int32_t t) { return -t - 1; }

// A block of device memory shared by several tables or results (the batched
// join allocates one per round); freed, stream-ordered, with its last user.
struct Arena {
  DeviceMem* mem = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  Arena(DeviceMem* m, size_t b, hipStream_t st);
  // takes over an allocation of b bytes at p made from m
  Arena(DeviceMem* m, void* p_, size_t b, hipStream_t st) : mem(m), p(p_), bytes(b), s(st) {}
  ~Arena();
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
};

struct Segment {
  int64_t rows = 0;
  const int32_t* col[kMaxCols] = {};  // variable order
  void* owned = nullptr;
  size_t owned_bytes = 0;
  std::shared_ptr<Arena> keep;        // arena holding the columns, if any
  std::shared_ptr<void> hold;         // anything else the columns live in
};

// Columnar int32 binding table: column c holds variable var[c].  The columns
// are views (into the store or an arena) or one owned allocation.
struct Table {
  int64_t n = 0;
  int k = 0;
  const int32_t* col[kMaxCols] = {};
  int var[kMaxCols] = {};
  void* owned = nullptr;
  size_t owned_bytes = 0;
  std::shared_ptr<Arena> keep;
  bool unit() const { return n == 1 && k == 0; }
  int col_of(int v) const {
    for (int c = 0; c < k; ++c)
      if (var[c] == v) return c;
    return -1;
  }
};

// Column stride (in values) of an n-row table: columns start on 256-byte
// boundaries so that a wave's 64 stores of one column cover whole lines.
inline int64_t col_stride(int64_t n) { return (std::max<int64_t>(n, 1) + 63) / 64 * 64; }

// The patterns a step completes: its own, or for a star-centre intersection
// the members whose other endpoint is a constant (their membership is exact).
uint32_t step_completes(const gsmat_query_plan* pl, const gsmat_step_info& sp);

// Adaptive choice on a bound table, first half: a filter when a remaining
// connected pattern has both endpoints bound (filters never add rows), else
// the connected expansions whose fan-out is to be sampled (nc of them:
// pattern cand_tp[i] from its bound side, cand_or[i] = 0 subject, 1 object).
// With nothing connected, `cartesian` names the smallest remaining pattern.
struct StepChoice {
  bool has_filter = false;
  gsmat_step_info filter{};
  int nc = 0;
  int8_t cand_tp[kMaxPats];
  int8_t cand_or[kMaxPats];
  gsmat_step_info cartesian{};
};
void step_candidates(const gsmat_store* st, const gsmat_query_plan* pl, const Table& t,
                     uint32_t rem, StepChoice& out);
// Bound column and predicate view that candidate i's fan-out sample reads.
void candidate_view(const gsmat_store* st, const gsmat_query_plan* pl, const Table& t,
                    const StepChoice& c, int i, const int32_t** col, PredView* pv);
// Second half: the expansion with the smallest sampled fan-out (the first
// on ties); sums may be null when nc == 1.
gsmat_step_info step_pick(const gsmat_query_plan* pl, const StepChoice& c, const int64_t* sums);

// Runs one plan with the single-query executor, adding to res.  mem (null:
// the store's allocator) provides the tables and step scratch; dev_area
// (null: pinned host memory) is a device area of at least kStageBytes where
// kernels leave the small results the host reads.
constexpr size_t kStageBytes = 4096;
void run_query(gsmat_store* st, const gsmat_query_plan* pl, int64_t budget_bytes,
               int64_t max_rows, hipStream_t s, gsmat_result* res, DeviceMem* mem = nullptr,
               void* dev_area = nullptr);

// Runs plan pl (adaptive step choice) from table t0, or from the unit table
// when t0 is null, and appends the final tables to out instead of adding them
// to a result: each table's owned allocation (if any) passes to the caller,
// and its columns may also be views into t0 or the store.  t0's columns stay
// the caller's (t0.owned must be null).
void run_collect(gsmat_store* st, const gsmat_query_plan* pl, const Table* t0,
                 int64_t budget_bytes, hipStream_t s, std::vector<Table>* out);

// Per-pattern statistics for the planner; lookups of constant endpoints go
// to the device in one batch.
std::vector<TpStat> pattern_stats(const gsmat_store* st, const gsmat_pattern* pats, int n,
                                  int mode, hipStream_t s,
                                  std::vector<gsmat_pat_lookup>* lk = nullptr);

}  // namespace gsmat

struct gsmat_result {
  gsmat_store* st = nullptr;
  hipStream_t stream = nullptr;
  int32_t n_vars = 0;
  int64_t rows = 0;
  std::vector<gsmat::Segment> segs;
  // rows into and out of each plan step (summed over chunks), kept inline: a
  // plan has at most one step per pattern
  static constexpr int kMaxSteps = gsmat::kMaxPats + 1;
  int32_t n_steps = 0;
  int64_t step_in[kMaxSteps], step_out[kMaxSteps];
  // n counters, zeroed
  void reset_steps(size_t n) {
    if (n > (size_t)kMaxSteps) throw gsmat::StatusFail{GSMAT_EHIP, "internal: plan has too many steps"};
    n_steps = (int32_t)n;
    std::fill(step_in, step_in + n, 0);
    std::fill(step_out, step_out + n, 0);
  }
  ~gsmat_result() {
    for (auto& s : segs)
      if (s.owned) st->mem->free(s.owned, s.owned_bytes, stream);
  }
};
