// Batched join kernels: every launch covers the tasks of many queries, whose
// tiles are concatenated; a workgroup finds its task by a binary search over
// the tasks' first tiles and then runs the same per-tile body as the
// single-query kernels (device.hpp).
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "batch_tiles.hpp"
#include "device.hpp"

namespace gsmat {

namespace {

using namespace dev;

__global__ void k_lookup_many(const LookupReq* __restrict__ req, int32_t n, const PredDesc* dout,
                              const PredDesc* din, OriPtrs out, OriPtrs in, LookupRes* res) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  res[i] = lookup_one(req[i], dout, din, out, in);
}

__global__ __launch_bounds__(kBlock) void k_b_sample(const SCand* __restrict__ c,
                                                     int64_t* __restrict__ part) {
  const int cand = blockIdx.x / kSampleBlocks;
  const int slice = blockIdx.x % kSampleBlocks;
  const SCand& sc = c[cand];
  const int64_t t = sample_fanout_slice(slice, sc.col, sc.n, sc.pv);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Count / flag tiles of every task; tile sums to ts.
__global__ __launch_bounds__(kBlock) void k_b_count(const CTask* __restrict__ tasks,
                                                    const GItem* __restrict__ items, int nitems,
                                                    const ListRef* __restrict__ lists,
                                                    int64_t* __restrict__ ts,
                                                    int64_t* __restrict__ tsn) {
  const GItem& it = items[find_item(items, nitems, blockIdx.x)];
  const CTask& T = tasks[it.task];
  const int64_t tile = (int64_t)blockIdx.x - it.w0;
  int64_t ne;
  const int64_t sum = b_count_tile(T, tile, lists, T.N, T.start, T.flags, T.nonempty, &ne);
  if (threadIdx.x == 0) {
    ts[blockIdx.x] = sum;
    tsn[blockIdx.x] = ne;
  }
}

// Sparse expansions: the rows with output of every count tile, compacted.
__global__ __launch_bounds__(kBlock) void k_b_compact_rows(const WTask* __restrict__ tasks,
                                                           const GItem* __restrict__ items,
                                                           int nitems,
                                                           const int64_t* __restrict__ ts,
                                                           const int64_t* __restrict__ tsn) {
  const GItem& it = items[find_item(items, nitems, blockIdx.x)];
  b_compact_rows_tile(tasks[it.task], (int64_t)blockIdx.x - it.w0, ts, tsn);
}

// Output size of every task from the scanned tile sums (exclusive, with the
// grand total at ts[ntiles]); written to pinned host memory.
// Also copies each task's non-empty row count (ne[task], tasks in item order)
// to out[nitems + task].
__global__ void k_b_totals(const GItem* __restrict__ items, int nitems, const int64_t* ts,
                           int64_t ntiles, const int64_t* __restrict__ ne,
                           int64_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  const int64_t a = items[i].w0;
  const int64_t b = i + 1 < nitems ? items[i + 1].w0 : ntiles;
  out[items[i].task] = ts[b] - ts[a];
  out[nitems + items[i].task] = ne[items[i].task];
}

// Expansion row offsets P (relative to the task) from the tile offsets.
__global__ __launch_bounds__(kBlock) void k_b_scan_add(const WTask* __restrict__ tasks,
                                                       const GItem* __restrict__ items,
                                                       int nitems, const int64_t* __restrict__ ts) {
  const GItem& it = items[find_item(items, nitems, blockIdx.x)];
  b_scan_add_tile(tasks[it.task], (int64_t)blockIdx.x - it.w0, ts);
}

// Merge-path splits of every expansion: one thread per split entry.
__global__ void k_b_partition(const WTask* __restrict__ tasks, const GItem* __restrict__ items,
                              int nitems, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const GItem& it = items[find_item(items, nitems, g)];
  const WTask& T = tasks[it.task];
  const int64_t t = g - it.w0;
  T.split[t] = mp_split(T.P, T.n, 0, T.m, t);
}

// The expansion writes of a round, every column count in one launch: a
// workgroup runs the variant of its task's count (uniform per workgroup).
// The variants share one LDS staging area, so the launch has the
// occupancy of a single variant and no launch waits for another's tail.
__global__ __launch_bounds__(kBlock) void k_b_write(const WTask* __restrict__ tasks,
                                                    const GItem* __restrict__ items, int nitems) {
  __shared__ int32_t sE[kTile + 1];
  __shared__ int32_t sRb[kTile + 1];
  __shared__ uint16_t sRow[kTile];
  const TileLds L{sE, sRb, sRow, nullptr};
  const GItem& it = items[find_item(items, nitems, blockIdx.x)];
  const WTask& T = tasks[it.task];
  const int64_t t = (int64_t)blockIdx.x - it.w0;
  b_write_tile_any<false>(T, t, L);
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_b_write_idx(const WTask* __restrict__ tasks,
                                                        const GItem* __restrict__ items,
                                                        int nitems) {
  const GItem& it = items[find_item(items, nitems, blockIdx.x)];
  const WTask& T = tasks[it.task];
  const int64_t t = (int64_t)blockIdx.x - it.w0;
  __shared__ int32_t sE[kTile + 1];
  __shared__ int32_t sRb[kTile + 1];
  __shared__ uint16_t sRow[kTile];
  b_write_tile<K, true>(T, t, TileLds{sE, sRb, sRow, nullptr});
}

// Stable compaction of one tile of a filter or intersection task (K
// columns; K < 0: any count).
template <int K>
__global__ __launch_bounds__(kBlock) void k_b_compact(const WTask* __restrict__ tasks,
                                                      const GItem* __restrict__ items, int nitems,
                                                      const int64_t* __restrict__ ts) {
  const GItem& it = items[find_item(items, nitems, blockIdx.x)];
  b_compact_tile<K>(tasks[it.task], (int64_t)blockIdx.x - it.w0, ts);
}


#define GS_BLAUNCH(cls, bytes, ...)             \
  do {                                          \
    const bool _prof = prof_on(cls);            \
    if (_prof) prof_begin(s, cls);              \
    __VA_ARGS__;                                \
    GS_HIP(hipGetLastError());                  \
    if (_prof) prof_end(s, cls, bytes);         \
  } while (0)

template <int K>
void b_write_idx(const WTask* t, const GItem* g, int ng, int64_t tiles, double bytes,
                 hipStream_t s) {
  GS_BLAUNCH(GSMAT_K_WRITE, bytes,
             hipLaunchKernelGGL(k_b_write_idx<K>, dim3((unsigned)tiles), dim3(kBlock), 0, s, t, g,
                                ng));
}
template <int K>
void b_compact(const WTask* t, const GItem* g, int ng, const int64_t* ts, int64_t tiles,
               double bytes, hipStream_t s) {
  GS_BLAUNCH(GSMAT_K_COMPACT, bytes,
             hipLaunchKernelGGL(k_b_compact<K>, dim3((unsigned)tiles), dim3(kBlock), 0, s, t, g,
                                ng, ts));
}

}  // namespace

void launch_lookup_many(const LookupReq* req, int32_t n, const PredDesc* dout, const PredDesc* din,
                        OriPtrs out, OriPtrs in, LookupRes* res, hipStream_t s) {
  if (n <= 0) return;
  GS_BLAUNCH(GSMAT_K_OTHER, 32.0 * n,
             hipLaunchKernelGGL(k_lookup_many, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock),
                                0, s, req, n, dout, din, out, in, res));
}

void launch_b_sample(const SCand* cands, int64_t nc, int64_t* part, hipStream_t s) {
  if (nc <= 0) return;
  GS_BLAUNCH(GSMAT_K_OTHER, 0.0,
             hipLaunchKernelGGL(k_b_sample, dim3((unsigned)(nc * kSampleBlocks)), dim3(kBlock), 0,
                                s, cands, part));
}

void launch_b_count(const CTask* tasks, const GItem* items, int nitems, const ListRef* lists,
                    int64_t* ts, int64_t* tsn, int64_t ntiles, double bytes, hipStream_t s) {
  GS_BLAUNCH(GSMAT_K_COUNT, bytes,
             hipLaunchKernelGGL(k_b_count, dim3((unsigned)ntiles), dim3(kBlock), 0, s, tasks,
                                items, nitems, lists, ts, tsn));
}

void launch_b_compact_rows(const WTask* tasks, const GItem* items, int nitems, const int64_t* ts,
                           const int64_t* tsn, int64_t tiles, double bytes, hipStream_t s) {
  GS_BLAUNCH(GSMAT_K_SCAN, bytes,
             hipLaunchKernelGGL(k_b_compact_rows, dim3((unsigned)tiles), dim3(kBlock), 0, s, tasks,
                                items, nitems, ts, tsn));
}

void launch_b_totals(const GItem* items, int nitems, const int64_t* ts, int64_t ntiles,
                     const int64_t* ne, int64_t* out, hipStream_t s) {
  GS_BLAUNCH(GSMAT_K_SCAN, 16.0 * nitems,
             hipLaunchKernelGGL(k_b_totals, dim3((unsigned)ceil_div(nitems, kBlock)), dim3(kBlock),
                                0, s, items, nitems, ts, ntiles, ne, out));
}

void launch_b_scan_add(const WTask* tasks, const GItem* items, int nitems, const int64_t* ts,
                       int64_t tiles, double bytes, hipStream_t s) {
  GS_BLAUNCH(GSMAT_K_SCAN, bytes,
             hipLaunchKernelGGL(k_b_scan_add, dim3((unsigned)tiles), dim3(kBlock), 0, s, tasks,
                                items, nitems, ts));
}

void launch_b_partition(const WTask* tasks, const GItem* items, int nitems, int64_t total,
                        hipStream_t s) {
  GS_BLAUNCH(GSMAT_K_OTHER, 8.0 * total,
             hipLaunchKernelGGL(k_b_partition, dim3((unsigned)ceil_div(total, kBlock)),
                                dim3(kBlock), 0, s, tasks, items, nitems, total));
}

void launch_b_write(const WTask* t, const GItem* g, int ng, int64_t tiles, double bytes,
                    hipStream_t s) {
  GS_BLAUNCH(GSMAT_K_WRITE, bytes,
             hipLaunchKernelGGL(k_b_write, dim3((unsigned)tiles), dim3(kBlock), 0, s, t, g, ng));
}

void launch_b_write_idx(int k, const WTask* t, const GItem* g, int ng, int64_t tiles, double bytes,
                        hipStream_t s) {
  switch (k) {
    case 0: return b_write_idx<0>(t, g, ng, tiles, bytes, s);
    case 1: return b_write_idx<1>(t, g, ng, tiles, bytes, s);
    case 2: return b_write_idx<2>(t, g, ng, tiles, bytes, s);
    case 3: return b_write_idx<3>(t, g, ng, tiles, bytes, s);
    case 4: return b_write_idx<4>(t, g, ng, tiles, bytes, s);
    case 5: return b_write_idx<5>(t, g, ng, tiles, bytes, s);
    case 6: return b_write_idx<6>(t, g, ng, tiles, bytes, s);
    case 7: return b_write_idx<7>(t, g, ng, tiles, bytes, s);
    case 8: return b_write_idx<8>(t, g, ng, tiles, bytes, s);
    default: return b_write_idx<-1>(t, g, ng, tiles, bytes, s);
  }
}

void launch_b_compact(int k, const WTask* t, const GItem* g, int ng, const int64_t* ts,
                      int64_t tiles, double bytes, hipStream_t s) {
  switch (k) {
    case 1: return b_compact<1>(t, g, ng, ts, tiles, bytes, s);
    case 2: return b_compact<2>(t, g, ng, ts, tiles, bytes, s);
    case 3: return b_compact<3>(t, g, ng, ts, tiles, bytes, s);
    case 4: return b_compact<4>(t, g, ng, ts, tiles, bytes, s);
    case 5: return b_compact<5>(t, g, ng, ts, tiles, bytes, s);
    case 6: return b_compact<6>(t, g, ng, ts, tiles, bytes, s);
    case 7: return b_compact<7>(t, g, ng, ts, tiles, bytes, s);
    case 8: return b_compact<8>(t, g, ng, ts, tiles, bytes, s);
    default: return b_compact<-1>(t, g, ng, ts, tiles, bytes, s);
  }
}

}  // namespace gsmat
