// Batched join: task descriptors shared by the host executor (batch.hip)
// and the batched kernels (kernels_batch.hip), and the launchers.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "plan.hpp"

namespace gsmat {

enum : int32_t { kTaskExpand = 0, kTaskFilter = 1, kTaskIntersect = 2 };

// Count-phase task: one step of one query.
struct CTask {
  int64_t n;           // input rows (intersection: driver list length)
  int32_t kind;
  int32_t l0, nl;      // intersection: lists[l0, l0 + nl)
  int32_t pad;
  PredView pv;         // expansion: view of the bound orientation; filter: by subject
  ProbeArgs pa;        // filter
  const int32_t* col;  // expansion: bound column; intersection: driver list
  int32_t* N;          // expansion: output count per row
  int32_t* start;      // expansion: row offset per row
  uint8_t* flags;      // filter, intersection: keep flags
  int64_t* nonempty;   // expansion: rows with output (starts at 0)
};

// Write-phase task.
struct WTask {
  int64_t n, m;        // input rows, output rows
  int64_t t0;          // first tile of the task in the count launch
  ColSet in;           // input columns
  int32_t* out0;       // output column c at out0 + c * ostride
  int64_t ostride;
  int32_t k;           // input columns
  int32_t pad;
  const int32_t* nbr;  // expansion: members of the predicate view
  const int32_t* N;    // expansion: output count per input row
  const int32_t* start;  // expansion: row offset per row of the write
  int64_t* P;          // expansion: output offsets per row of the write (+ 1)
  int64_t* split;      // expansion: merge-path splits (path tiles + 1)
  const uint8_t* flags;
  // sparse expansion: the write covers only the n input rows with output,
  // compacted from n_in rows; ridx[i] is row i's input row
  int32_t* ridx;
  int32_t* cstart;     // start of each compacted row (start points here)
  const int32_t* start_in;
  int64_t n_in;
};

// One task inside a launch: its tiles start at w0 of the launch's tiles.
struct GItem {
  int64_t w0;
  int32_t task;
  int32_t pad;
};

// Candidate expansion whose fan-out is sampled.
struct SCand {
  const int32_t* col;
  PredView pv;
  int64_t n;
};

// Column counts with their own write / compaction instantiation.
constexpr int kMaxK = 11;

// Write strategy of a batched expansion of n input rows of which ne have
// output: true = compact the rows with output and walk only those (the
// compacted row list holds int32 input row indices, so n must stay below
// 2^31); false = the merge path over every input row.
__host__ __device__ inline bool sparse_expand(double theta, int64_t min_rows, int64_t n,
                                              int64_t ne) {
  return theta > 0 && n >= min_rows && n <= (int64_t)INT32_MAX &&
         (double)ne < theta * (double)n;
}

// Device-driven batched join (dbatch.hip): every plan evaluated with its
// state on the device.  out[i]: state kDevDone with res set (owned by the
// caller), kDevFallback (the query left the batch: run it alone), or
// kDevFailed with status.
enum : int32_t { kDevDone = 0, kDevFallback = 1, kDevFailed = 2 };
constexpr int kStatRounds = 64;  // rounds recorded per device-driven batch
constexpr int kStatFields = 8;
struct DevQueryOut {
  gsmat_result* res;
  int32_t state;
  gsmat_status status;
};
void run_batch_device(gsmat_store* st, const gsmat_query_plan* const* plans, int32_t n,
                      int64_t budget, int64_t max_rows, hipStream_t s,
                      std::vector<DevQueryOut>& out);

// Planning of a batch of BGPs, shared by gsmat_plan_batch and the fused
// gsmat_join_batch_bgp: prepare validates every query, takes each pattern's
// statistics and does every constant's row lookup in one device launch;
// build then plans query i (rc[i] == GSMAT_OK) into pl, as gsmat_plan would.
struct PlanPrep {
  std::vector<int64_t> off, so;     // first pattern / first statistics slot per query
  std::vector<gsmat_status> rc;
  std::vector<std::string> msg;
  std::vector<int32_t> nv;          // variables per valid query
  std::vector<TpStat> stats;        // per pattern, flat over the batch
  std::vector<int> req_of;          // lookup of each pattern (-1: none)
  std::vector<LookupRes> res;
};
void plan_prepare(const gsmat_store* st, const gsmat_pattern* pats, const int32_t* n_pats,
                  int32_t nq, int32_t mode, hipStream_t s, PlanPrep* pp);
gsmat_status plan_build(const gsmat_store* st, const gsmat_pattern* pats, const int32_t* n_pats,
                        int32_t mode, PlanPrep& pp, int64_t i, gsmat_query_plan* pl);

// The fused batch (plans built on the host straight into the device upload,
// no plan objects): out[i] as above for the valid queries; status[i] is the
// planning status (out[i] untouched where it is not GSMAT_OK); fallback[i]
// holds a plan for each query that left the batch.
void run_batch_device_bgp(gsmat_store* st, const gsmat_pattern* pats, const int32_t* n_pats,
                          int32_t nq, int32_t mode, int64_t budget, int64_t max_rows,
                          hipStream_t s, std::vector<DevQueryOut>& out,
                          std::vector<gsmat_status>& status, std::vector<std::string>& msg,
                          std::vector<std::unique_ptr<gsmat_query_plan>>& fallback);

void launch_lookup_many(const LookupReq* req, int32_t n, const PredDesc* dout, const PredDesc* din,
                        OriPtrs out, OriPtrs in, LookupRes* res, hipStream_t s);
// fan-out samples: kSampleBlocks partial sums per candidate to part[c * kSampleBlocks + b]
void launch_b_sample(const SCand* cands, int64_t nc, int64_t* part, hipStream_t s);
// count / flag tiles of every task (items in task order) -> tile sums ts[ntiles]
// and, per tile, the expansion rows with output tsn[ntiles]
void launch_b_count(const CTask* tasks, const GItem* items, int nitems, const ListRef* lists,
                    int64_t* ts, int64_t* tsn, int64_t ntiles, double bytes, hipStream_t s);
// sparse expansions: the rows with output of every count tile, compacted in
// order, with their output offsets (ts, tsn scanned)
void launch_b_compact_rows(const WTask* tasks, const GItem* items, int nitems, const int64_t* ts,
                           const int64_t* tsn, int64_t tiles, double bytes, hipStream_t s);
// out[task] = output rows, out[nitems + task] = non-empty rows (expansions)
void launch_b_totals(const GItem* items, int nitems, const int64_t* ts, int64_t ntiles,
                     const int64_t* ne, int64_t* out, hipStream_t s);
void launch_b_scan_add(const WTask* tasks, const GItem* items, int nitems, const int64_t* ts,
                       int64_t tiles, double bytes, hipStream_t s);
void launch_b_partition(const WTask* tasks, const GItem* items, int nitems, int64_t total,
                        hipStream_t s);
// every expansion write of a round (any column counts) in one launch
void launch_b_write(const WTask* tasks, const GItem* items, int nitems, int64_t tiles,
                    double bytes, hipStream_t s);
// writes over compacted rows (sparse expansions), one launch per column
// count; k > kMaxK selects the generic instantiation
void launch_b_write_idx(int k, const WTask* tasks, const GItem* items, int nitems, int64_t tiles,
                        double bytes, hipStream_t s);
void launch_b_compact(int k, const WTask* tasks, const GItem* items, int nitems,
                      const int64_t* ts, int64_t tiles, double bytes, hipStream_t s);

}  // namespace gsmat
