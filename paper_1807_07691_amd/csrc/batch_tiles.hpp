// Per-tile bodies of the batched join steps, shared by the host-driven
// rounds (kernels_batch.hip) and the device-driven rounds (dbatch.hip).  A
// tile body receives its task descriptor and the tile's index within the
// task; every body with a barrier must be called by the whole workgroup.
#pragma once

#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "device.hpp"

namespace gsmat {
namespace dev {

// Index of the entry owning tile b in an array of first tiles: the last
// entry with w0 <= b.  Entries without tiles share their successor's first
// tile and are skipped by this rule.
__device__ inline int find_item(const GItem* __restrict__ g, int n, int64_t b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g[mid].w0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
__device__ inline int find_first_tile(const int64_t* __restrict__ w0, int n, int64_t b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (w0[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Count / flag tile of one count-phase task, writing to N/start
// (expansions) or flags; the tile sum is returned, and for expansions the
// rows with output go to ne and are added to *nonempty (one atomic per
// workgroup).  kT threads per workgroup; kS: the intersection strategy.
template <int kT = kBlock, int kS = kIsSearch>
__device__ inline int64_t b_count_tile(const CTask& T, int64_t tile, const ListRef* lists,
                                       int32_t* N, int32_t* start, uint8_t* flags,
                                       int64_t* nonempty, int64_t* ne) {
  if (T.kind == kTaskExpand) {
    const PredView pv = T.pv;
    const int64_t packed = count_expand_tile<true, kT>(tile, T.col, T.n, pv, N, start);
    const int64_t k = packed >> kNonEmptyShift;
    if (threadIdx.x == 0 && k > 0) atomicAdd((unsigned long long*)nonempty, (unsigned long long)k);
    *ne = k;
    return packed & (((int64_t)1 << kNonEmptyShift) - 1);
  }
  *ne = 0;
  if (T.kind == kTaskFilter) {
    const PredView pv = T.pv;
    const ProbeArgs pa = T.pa;
    return flag_filter_tile<kT>(tile, pa, T.n, pv, flags);
  }
  return flag_intersect_tile<kT, kS>(tile, T.col, T.n, lists + T.l0, T.nl, flags);
}

// Sparse expansion, one count tile: the rows with output, compacted in
// order, with their index, start and output offset (exclusive prefix of N
// from the task's base; ts/tsn are the scanned tile sums of outputs and of
// rows with output).  Thread t takes the tile's rows 8t..8t+7, so one block
// scan of (outputs, rows with output) gives every kept row its offset and
// place; the pair is packed into one int64, the row count in the low 12 bits
// (a tile has 2048 rows) and the outputs above it (at most 2048 rows of fewer
// than 2^31 each: 2^42).
__device__ inline void b_compact_rows_tile(const WTask& T, int64_t tile,
                                           const int64_t* __restrict__ ts,
                                           const int64_t* __restrict__ tsn) {
  static_assert(kTile < (1 << 12), "row count must fit the low 12 bits");
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

// Dense expansion, one count tile: row offsets P relative to the task.
__device__ inline void b_scan_add_tile(const WTask& T, int64_t tile,
                                       const int64_t* __restrict__ ts) {
  const int64_t base = ts[T.t0 + tile] - ts[T.t0];
  const int64_t tot = scan_add_tile<int32_t, int64_t>(tile, T.N, T.n, base, T.P);
  if (threadIdx.x == 0 && (tile + 1) * kTile >= T.n) T.P[T.n] = base + tot;
}

// One path tile of an expansion task with K parent columns (K < 0: T.k
// columns), staged in L; kIdx: the task walks its compacted rows.
template <int K, bool kIdx>
__device__ inline void b_write_tile(const WTask& T, int64_t t, const TileLds& L) {
  const OutStrided out{T.out0, T.ostride};
  if constexpr (K >= 0) {
    ColSet in;
#pragma unroll
    for (int c = 0; c < K; ++c) in.c[c] = T.in.c[c];
    write_expand_tile_in<K, OutStrided, kIdx>(L, t, in, K, T.P, T.start, T.n, T.nbr, 0, T.m,
                                              T.split, out, kIdx ? T.ridx : nullptr);
  } else {
    write_expand_tile_in<K, OutStrided, kIdx>(L, t, T.in, T.k, T.P, T.start, T.n, T.nbr, 0, T.m,
                                              T.split, out, kIdx ? T.ridx : nullptr);
  }
}

// The variant of a task's column count (uniform per workgroup).
template <bool kIdx>
__device__ inline void b_write_tile_any(const WTask& T, int64_t t, const TileLds& L) {
  static_assert(kMaxK == 11, "one case per specialised column count");
  switch (T.k) {
    case 0: return b_write_tile<0, kIdx>(T, t, L);
    case 1: return b_write_tile<1, kIdx>(T, t, L);
    case 2: return b_write_tile<2, kIdx>(T, t, L);
    case 3: return b_write_tile<3, kIdx>(T, t, L);
    case 4: return b_write_tile<4, kIdx>(T, t, L);
    case 5: return b_write_tile<5, kIdx>(T, t, L);
    case 6: return b_write_tile<6, kIdx>(T, t, L);
    case 7: return b_write_tile<7, kIdx>(T, t, L);
    case 8: return b_write_tile<8, kIdx>(T, t, L);
    case 9: return b_write_tile<9, kIdx>(T, t, L);
    case 10: return b_write_tile<10, kIdx>(T, t, L);
    case 11: return b_write_tile<11, kIdx>(T, t, L);
    default: return b_write_tile<-1, kIdx>(T, t, L);
  }
}

// Stable compaction of one tile of a filter or intersection task (rows
// with a non-zero flag, K columns; K < 0: T.k columns).  Thread t takes the
// tile's rows 8t..8t+7: one block scan of its kept-row count gives its first
// output place, then a thread with kept rows reads its 8 values of each
// column and writes the kept ones in row order.
template <int K>
__device__ inline void b_compact_tile(const WTask& T, int64_t tile, const int64_t* __restrict__ ts) {
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

__device__ inline void b_compact_tile_any(const WTask& T, int64_t tile, const int64_t* ts) {
  switch (T.k) {
    case 1: return b_compact_tile<1>(T, tile, ts);
    case 2: return b_compact_tile<2>(T, tile, ts);
    case 3: return b_compact_tile<3>(T, tile, ts);
    case 4: return b_compact_tile<4>(T, tile, ts);
    case 5: return b_compact_tile<5>(T, tile, ts);
    case 6: return b_compact_tile<6>(T, tile, ts);
    case 7: return b_compact_tile<7>(T, tile, ts);
    case 8: return b_compact_tile<8>(T, tile, ts);
    default: return b_compact_tile<-1>(T, tile, ts);
  }
}

}  // namespace dev
}  // namespace gsmat
