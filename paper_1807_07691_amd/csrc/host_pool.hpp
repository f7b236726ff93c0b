// A small persistent pool of host threads for loops over independent items
// (building the plans of a batch): the items are cut into contiguous chunks
// that the pool's threads and the calling thread take in turn.
#pragma once

#include <cstdint>
#include <functional>

namespace gsmat {

// Calls fn(lo, hi) on disjoint ranges covering [0, n), on up to the pool's
// threads plus the caller, and returns when every range is done.  Loops of
// fewer than min_per_thread items per thread, and calls made while another
// caller holds the pool, run on the calling thread alone.  fn must not throw.
// The pool has GSMAT_HOST_THREADS threads (environment; default the smaller
// of 7 and the number of hardware threads less one; 0 disables it).
void host_parallel_for(int64_t n, int64_t min_per_thread,
                       const std::function<void(int64_t, int64_t)>& fn);

}  // namespace gsmat
