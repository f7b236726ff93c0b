// Batched join kernels: every launch covers the tasks of many queries, whose
// tiles are concatenated; a workgroup finds its task by a binary search over
// the tasks' first tiles and then runs the same per-tile body as the
// single-query kernels (device.hpp).
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "device.hpp"

namespace gsmat {

namespace {

using namespace dev;

// Index of the item owning tile b: the last item with w0 <= b.
__device__ inline int find_item(const GItem* __restrict__ g, int n, int64_t b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g[mid].w0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

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
  int64_t sum, ne = 0;
  if (T.kind == kTaskExpand) {
    const PredView pv = T.pv;
    const int64_t packed = count_expand_tile<true>(tile, T.col, T.n, pv, T.N, T.start);
    sum = packed & (((int64_t)1 << kNonEmptyShift) - 1);
    ne = packed >> kNonEmptyShift;
    if (threadIdx.x == 0 && ne > 0) atomicAdd((unsigned long long*)T.nonempty, (unsigned long long)ne);
  } else if (T.kind == kTaskFilter) {
    const PredView pv = T.pv;
    const ProbeArgs pa = T.pa;
    sum = flag_filter_tile(tile, pa, T.n, pv, T.flags);
  } else {
    sum = flag_intersect_tile(tile, T.col, T.n, lists + T.l0, T.nl, T.flags);
  }
  if (threadIdx.x == 0) {
    ts[blockIdx.x] = sum;
    tsn[blockIdx.x] = ne;
  }
}

// Sparse expansion, one count tile: the rows with output, compacted in
// order, with their index, start and output offset (exclusive prefix of N
// from the tile's base).  Thread t takes the tile's rows 8t..8t+7, so one
// block scan of (outputs, rows with output) gives every kept row its offset
// and place; the pair is packed into one int64, the row count in the low 12
// bits (a tile has 2048 rows) and the outputs above it (at most 2048 rows of
// fewer than 2^31 each: 2^42).
__global__ __launch_bounds__(kBlock) void k_b_compact_rows(const WTask* __restrict__ tasks,
                                                           const GItem* __restrict__ items,
                                                           int nitems,
                                                           const int64_t* __restrict__ ts,
                                                           const int64_t* __restrict__ tsn) {
  static_assert(kTile < (1 << 12), "row count must fit the low 12 bits");
  const GItem& it = items[find_item(items, nitems, blockIdx.x)];
  const WTask& T = tasks[it.task];
  const int64_t tile = (int64_t)blockIdx.x - it.w0;
  const int64_t n = T.n_in;
  const int64_t i0 = tile * kTile + (int64_t)threadIdx.x * kItems;
  const int32_t* __restrict__ N = T.N;
  int32_t v[kItems];
  if (i0 + kItems <= n && ((uintptr_t)(N + i0) & 15) == 0) {
    const int4 a = *reinterpret_cast<const int4*>(N + i0);
    const int4 b = *reinterpret_cast<const int4*>(N + i0 + 4);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
    v[4] = b.x;
    v[5] = b.y;
    v[6] = b.z;
    v[7] = b.w;
  } else {
#pragma unroll
    for (int j = 0; j < kItems; ++j) v[j] = i0 + j < n ? N[i0 + j] : 0;
  }
  int64_t sum = 0;
  int64_t cnt = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    sum += v[j];
    cnt += v[j] > 0;
  }
  int64_t tot;
  const int64_t ex = block_excl_scan(sum << 12 | cnt, &tot);
  int64_t off = ts[T.t0 + tile] - ts[T.t0] + (ex >> 12);
  int64_t pos = tsn[T.t0 + tile] - tsn[T.t0] + (ex & 0xFFF);
  int32_t* __restrict__ ridx = T.ridx;
  int32_t* __restrict__ cstart = T.cstart;
  int64_t* __restrict__ P = T.P;
  const int32_t* __restrict__ st = T.start_in;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    if (v[j] > 0) {
      ridx[pos] = (int32_t)(i0 + j);
      cstart[pos] = st[i0 + j];
      P[pos] = off;
      ++pos;
    }
    off += v[j];
  }
  if (threadIdx.x == 0 && (tile + 1) * kTile >= n) P[T.n] = T.m;
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
  const WTask& T = tasks[it.task];
  const int64_t tile = (int64_t)blockIdx.x - it.w0;
  const int64_t base = ts[T.t0 + tile] - ts[T.t0];
  const int64_t tot = scan_add_tile<int32_t, int64_t>(tile, T.N, T.n, base, T.P);
  if (threadIdx.x == 0 && (tile + 1) * kTile >= T.n) T.P[T.n] = base + tot;
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

// One tile of an expansion task with K parent columns (K < 0: T.k columns).
template <int K>
__device__ inline void b_write_tile(const WTask& T, int64_t t, const TileLds& L) {
  const OutStrided out{T.out0, T.ostride};
  if constexpr (K >= 0) {
    ColSet in;
#pragma unroll
    for (int c = 0; c < K; ++c) in.c[c] = T.in.c[c];
    write_expand_tile_in<K>(L, t, in, K, T.P, T.start, T.n, T.nbr, 0, T.m, T.split, out);
  } else {
    write_expand_tile_in<K>(L, t, T.in, T.k, T.P, T.start, T.n, T.nbr, 0, T.m, T.split, out);
  }
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
  static_assert(kMaxK == 11, "one case per specialised column count");
  switch (T.k) {
    case 0: return b_write_tile<0>(T, t, L);
    case 1: return b_write_tile<1>(T, t, L);
    case 2: return b_write_tile<2>(T, t, L);
    case 3: return b_write_tile<3>(T, t, L);
    case 4: return b_write_tile<4>(T, t, L);
    case 5: return b_write_tile<5>(T, t, L);
    case 6: return b_write_tile<6>(T, t, L);
    case 7: return b_write_tile<7>(T, t, L);
    case 8: return b_write_tile<8>(T, t, L);
    case 9: return b_write_tile<9>(T, t, L);
    case 10: return b_write_tile<10>(T, t, L);
    case 11: return b_write_tile<11>(T, t, L);
    default: return b_write_tile<-1>(T, t, L);
  }
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_b_write_idx(const WTask* __restrict__ tasks,
                                                        const GItem* __restrict__ items,
                                                        int nitems) {
  const GItem& it = items[find_item(items, nitems, blockIdx.x)];
  const WTask& T = tasks[it.task];
  const int64_t t = (int64_t)blockIdx.x - it.w0;
  const OutStrided out{T.out0, T.ostride};
  if constexpr (K >= 0) {
    ColSet in;
#pragma unroll
    for (int c = 0; c < K; ++c) in.c[c] = T.in.c[c];
    write_expand_tile<K, OutStrided, true>(t, in, K, T.P, T.start, T.n, T.nbr, 0, T.m, T.split,
                                           out, T.ridx);
  } else {
    write_expand_tile<K, OutStrided, true>(t, T.in, T.k, T.P, T.start, T.n, T.nbr, 0, T.m,
                                           T.split, out, T.ridx);
  }
}

// Stable compaction of one tile of a filter or intersection task (rows
// with a non-zero flag, K columns; K < 0: T.k columns).  Thread t takes the
// tile's rows 8t..8t+7: one block scan of its kept-row count gives its first
// output place, then a thread with kept rows reads its 8 values of each
// column and writes the kept ones in row order.
template <int K>
__global__ __launch_bounds__(kBlock) void k_b_compact(const WTask* __restrict__ tasks,
                                                      const GItem* __restrict__ items, int nitems,
                                                      const int64_t* __restrict__ ts) {
  const GItem& it = items[find_item(items, nitems, blockIdx.x)];
  const WTask& T = tasks[it.task];
  const int64_t tile = (int64_t)blockIdx.x - it.w0;
  const int64_t n = T.n;
  const int64_t i0 = tile * kTile + (int64_t)threadIdx.x * kItems;
  const bool full = i0 + kItems <= n;
  const uint8_t* __restrict__ flags = T.flags;
  uint32_t keep = 0;  // bit j: row i0 + j is kept
  if (full && ((uintptr_t)(flags + i0) & 7) == 0) {
    const uint64_t f = *reinterpret_cast<const uint64_t*>(flags + i0);
#pragma unroll
    for (int j = 0; j < kItems; ++j) keep |= ((f >> (8 * j)) & 0xFF) ? 1u << j : 0u;
  } else {
#pragma unroll
    for (int j = 0; j < kItems; ++j) keep |= (i0 + j < n && flags[i0 + j] != 0) ? 1u << j : 0u;
  }
  int64_t tot;
  const int64_t pos = ts[T.t0 + tile] - ts[T.t0] + block_excl_scan(__popc(keep), &tot);
  if (keep == 0) return;  // no barrier follows
  auto column = [&](const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
    int32_t x[kItems];
    if (full && ((uintptr_t)(src + i0) & 15) == 0) {
      const int4 a = *reinterpret_cast<const int4*>(src + i0);
      const int4 b = *reinterpret_cast<const int4*>(src + i0 + 4);
      x[0] = a.x;
      x[1] = a.y;
      x[2] = a.z;
      x[3] = a.w;
      x[4] = b.x;
      x[5] = b.y;
      x[6] = b.z;
      x[7] = b.w;
    } else {
#pragma unroll
      for (int j = 0; j < kItems; ++j) x[j] = (keep >> j & 1) ? src[i0 + j] : 0;
    }
    int64_t p = pos;
#pragma unroll
    for (int j = 0; j < kItems; ++j)
      if (keep >> j & 1) dst[p++] = x[j];
  };
  if constexpr (K >= 0) {
#pragma unroll
    for (int c = 0; c < K; ++c) column(T.in.c[c], T.out0 + (int64_t)c * T.ostride);
  } else {
    for (int c = 0; c < T.k; ++c) column(T.in.c[c], T.out0 + (int64_t)c * T.ostride);
  }
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
