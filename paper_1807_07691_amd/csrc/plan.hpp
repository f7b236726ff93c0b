// Host-side planner types (no device code).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "gsmat.h"

namespace gsmat {

constexpr int kMaxPats = 32;   // patterns per BGP (step member masks are 32-bit)
constexpr int kMaxCols = 32;   // variables per BGP = columns of a binding table
constexpr int kMaxLists = 8;   // patterns in one star-centre intersection

// Per-pattern statistics used for ordering and estimates.
struct TpStat {
  int64_t stat = 0;    // the sort key (paper: pair count of the predicate)
  int64_t rows_s = 0;  // size of the id list the pattern gives its subject
  int64_t rows_o = 0;  // size of the id list the pattern gives its object
};

gsmat_status validate_patterns(const gsmat_pattern* pats, int32_t n, int32_t* n_vars,
                               std::string* err);

}  // namespace gsmat

// Row lookup of a pattern's constant endpoint(s), as taken while planning:
// the row's offset and length in the orientation keyed by the constant, and
// for an all-constant pattern whether the pair exists.
struct gsmat_pat_lookup {
  int32_t start = 0, len = 0, found = 0, valid = 0;
};

struct gsmat_query_plan {
  std::vector<gsmat_pattern> pats;
  int32_t n_vars = 0;
  int32_t mode = 0;
  std::vector<gsmat_step_info> steps;
  // lookups of every pattern with a constant, valid for the index build
  // with uid `lk_store` (empty when planning made none)
  std::vector<gsmat_pat_lookup> lk;
  uint64_t lk_store = 0;
};

namespace gsmat {
// `st` holds one entry per pattern.
gsmat_status build_plan(const gsmat_pattern* pats, int32_t n, int32_t mode, const TpStat* st,
                        gsmat_query_plan* out, std::string* err);
}  // namespace gsmat
