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

struct gsmat_query_plan {
  std::vector<gsmat_pattern> pats;
  int32_t n_vars = 0;
  int32_t mode = 0;
  std::vector<gsmat_step_info> steps;
};

namespace gsmat {
gsmat_status build_plan(const gsmat_pattern* pats, int32_t n, int32_t mode,
                        const std::vector<TpStat>& st, gsmat_query_plan* out, std::string* err);
}  // namespace gsmat
