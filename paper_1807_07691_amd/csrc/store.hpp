// Device-resident sparse-matrix store (one boolean matrix per predicate, kept
// row-compressed by subject and column-compressed by object).
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"

namespace gsmat {

// One orientation of every predicate matrix, in global arrays ordered by
// (predicate, row, member).
struct Orientation {
  int32_t* nbr = nullptr;    // [T] members
  int32_t* src = nullptr;    // [T] row id of each member (by-subject orientation only)
  int32_t* keys = nullptr;   // [R] non-empty row ids per predicate
  int32_t* ptr = nullptr;    // [R + P] row offsets per predicate, one sentinel each
  int32_t* dense = nullptr;  // dense row pointers of heavy predicates
  int32_t* dir = nullptr;    // bucket directories of the other predicates
  int32_t* hub_keys = nullptr;  // row ids of the rows with a bitmap, per predicate
  uint32_t* hub_bm = nullptr;   // their bitmaps, hub_words words each
  int64_t hub_words = 0;
  int32_t hub_min = 0;          // rows shorter than this have no bitmap
  std::vector<int32_t> hub_keys_host;
  int64_t R = 0;
  int64_t dense_len = 0;
  int64_t dir_len = 0;
  std::vector<PredDesc> desc;   // [P]
  PredDesc* d_desc = nullptr;   // device copy
  PredView view(int32_t p) const;
  OriPtrs ptrs() const { return OriPtrs{keys, ptr, nbr, dense, dir, hub_keys, hub_bm, hub_words, hub_min}; }
  // bitmap of predicate p's row v, or null
  const uint32_t* row_bitmap(int32_t p, int32_t v) const;
};

struct Alloc {
  void* p;
  size_t bytes;
};

}  // namespace gsmat

struct gsmat_store {
  std::unique_ptr<gsmat::DeviceMem> mem;
  int32_t V = 0, P = 0;
  int vb = 1, pb = 1;
  int64_t n_in = 0;
  int32_t* d_s = nullptr;  // raw triples until the index is built
  int32_t* d_p = nullptr;
  int32_t* d_o = nullptr;
  bool built = false;
  double sparse_theta = 0.5;       // batched expansions: compact rows below this fill ...
  int64_t sparse_min_rows = 4096;  // ... in expansions of at least this many rows
  int32_t batch_engine = 1;       // gsmat_join_batch: 1 device-driven rounds, 0 host-driven
  int32_t count_items = 8;        // device-driven count tiles: rows per thread (4, 8 or 16)
  int32_t intersect = 0;          // ... sorted-list intersections: 0 search, 1 window, 2 merge
  int64_t dbatch_out_hint = 0;    // device-driven rounds: output slab and scratch sizes of
  int64_t dbatch_scr_hint = 0;    // the last batch (the next one starts with them)
  std::vector<int64_t> dbatch_stats;  // the last device-driven batch's rounds
  int64_t hub_min_len = 1 << 14;  // rows this long get a bitmap ...
  int64_t hub_max_bytes = 0;      // ... within this many bytes per orientation (0: none)
  uint64_t uid = 0;        // distinct for every index build in the process
  int64_t T = 0;           // distinct triples
  gsmat::Orientation out;  // by subject: rows = subjects, members = objects
  gsmat::Orientation in;   // by object: rows = objects, members = subjects
  std::vector<gsmat::Alloc> index_allocs;
  int64_t device_bytes = 0;

  void* dalloc(size_t bytes, hipStream_t s, bool index);
  void dfree_index(hipStream_t s);
};
