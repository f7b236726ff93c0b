// Device-side building blocks shared by the single-query and the batched
// kernels: wave/workgroup scans, row lookup in a compressed predicate
// matrix, stable tile compaction and the per-tile bodies of the join steps.
// Every function that contains a barrier must be called by all threads of
// the workgroup.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace gsmat {
namespace dev {

__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline int wave_id() { return threadIdx.x >> 6; }
constexpr int kWaves = kBlock / 64;

__device__ inline uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline int64_t wave_incl_scan(int64_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ inline int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Exclusive scan of one value per thread over the workgroup.  Contains
// barriers: every thread of the block must call it.
__device__ inline int64_t block_excl_scan(int64_t v, int64_t* total) {
  __shared__ int64_t ws[kWaves];
  const int64_t inc = wave_incl_scan(v);
  if (lane_id() == 63) ws[wave_id()] = inc;
  __syncthreads();
  int64_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    if (i < wave_id()) off += ws[i];
    tot += ws[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// Exclusive scans of F values per thread over the whole workgroup (any
// multiple of 64 threads up to 1024); tot receives the workgroup totals.
// Contains barriers: every thread of the block must call it.
template <int F>
__device__ inline void block_excl_scan_n(const int64_t (&v)[F], int64_t (&ex)[F],
                                         int64_t (&tot)[F]) {
  __shared__ int64_t ws[F][16];
  const int nw = (int)(blockDim.x >> 6);
  int64_t inc[F];
#pragma unroll
  for (int f = 0; f < F; ++f) inc[f] = wave_incl_scan(v[f]);
  if (lane_id() == 63) {
#pragma unroll
    for (int f = 0; f < F; ++f) ws[f][wave_id()] = inc[f];
  }
  __syncthreads();
#pragma unroll
  for (int f = 0; f < F; ++f) {
    int64_t off = 0, t = 0;
    for (int q = 0; q < nw; ++q) {
      const int64_t a = ws[f][q];
      if (q < wave_id()) off += a;
      t += a;
    }
    ex[f] = off + inc[f] - v[f];
    tot[f] = t;
  }
  __syncthreads();
}

// Sum over a workgroup of kT threads.
template <int kT = kBlock>
__device__ inline int64_t block_sum(int64_t v) {
  constexpr int kW = kT / 64;
  __shared__ int64_t ws[kW];
  v = wave_sum(v);
  if (lane_id() == 0) ws[wave_id()] = v;
  __syncthreads();
  int64_t tot = 0;
#pragma unroll
  for (int i = 0; i < kW; ++i) tot += ws[i];
  __syncthreads();
  return tot;
}

// Two tile-sum arrays (neither null) scanned in one pass by one workgroup of kScanBlock
// threads: exclusive prefix
// sums in place, the totals at [nt].  One workgroup of 1024 threads walks the
// arrays in chunks of kScanBlock * kPer sums (kPer consecutive per thread); both scans share
// each chunk's pair of barriers.
constexpr int kScanBlock = 1024;
template <int kPer = kItems>
__device__ inline void scan_tile_sums2_block(int64_t* ts, int64_t* ts2, int64_t nt) {
  constexpr int W = kScanBlock / 64;
  __shared__ int64_t ws[2][W];
  const int lane = lane_id();
  const int wid = wave_id();
  int64_t carry = 0, carry2 = 0;
  for (int64_t c0 = 0; c0 < nt; c0 += (int64_t)kScanBlock * kPer) {
    int64_t v[kPer], w[kPer];
    int64_t loc = 0, loc2 = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t i = c0 + (int64_t)threadIdx.x * kPer + j;
      v[j] = i < nt ? ts[i] : 0;
      w[j] = i < nt ? ts2[i] : 0;
      loc += v[j];
      loc2 += w[j];
    }
    const int64_t inc = wave_incl_scan(loc);
    const int64_t inc2 = wave_incl_scan(loc2);
    if (lane == 63) {
      ws[0][wid] = inc;
      ws[1][wid] = inc2;
    }
    __syncthreads();
    int64_t off = 0, off2 = 0, tot = 0, tot2 = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const int64_t a = ws[0][q], b = ws[1][q];
      if (q < wid) {
        off += a;
        off2 += b;
      }
      tot += a;
      tot2 += b;
    }
    __syncthreads();
    int64_t ex = carry + off + inc - loc;
    int64_t ex2 = carry2 + off2 + inc2 - loc2;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t i = c0 + (int64_t)threadIdx.x * kPer + j;
      if (i < nt) {
        ts[i] = ex;
        ts2[i] = ex2;
      }
      ex += v[j];
      ex2 += w[j];
    }
    carry += tot;
    carry2 += tot2;
  }
  if (threadIdx.x == 0) {
    ts[nt] = carry;
    ts2[nt] = carry2;
  }
}

__device__ inline int32_t lower_bound_i32(const int32_t* __restrict__ a, int32_t n, int32_t v) {
  int32_t lo = 0, len = n;
  while (len > 0) {
    int32_t half = len >> 1;
    if (a[lo + half] < v) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo;
}

// Row of vertex v in one predicate's compressed matrix: (start, len), len 0
// when v has no entry.
__device__ inline void row_lookup(const PredView& pv, int32_t v, int32_t& start, int32_t& len) {
  if (pv.dense) {
    start = pv.dense[v];
    len = pv.dense[v + 1] - start;
    return;
  }
  // the bucket directory narrows the search to a few neighbouring keys
  int32_t lo = 0, n = pv.nr;
  if (pv.dir) {
    const int32_t b = v >> pv.dir_shift;
    lo = pv.dir[b];
    n = pv.dir[b + 1] - lo;
  }
  const int32_t r = lo + lower_bound_i32(pv.keys + lo, n, v);
  if (r < pv.nr && pv.keys[r] == v) {
    start = pv.ptr[r];
    len = pv.ptr[r + 1] - start;
  } else {
    start = 0;
    len = 0;
  }
}

// Lower bounds of N values, v[j] in a[lo[j], lo[j] + n[j]): the searches
// advance in lockstep, one round of N independent loads per halving; on
// return lo[j] is the position of the first element >= v[j].
template <int N>
__device__ inline void lower_bound_n(const int32_t* __restrict__ a, const int32_t (&v)[N],
                                     int32_t (&lo)[N], int32_t (&n)[N]) {
  for (;;) {
    int32_t kv[N];
    bool any = false;
#pragma unroll
    for (int j = 0; j < N; ++j) kv[j] = n[j] > 0 ? a[lo[j] + (n[j] >> 1)] : 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if (n[j] > 0) {
        const int32_t h = n[j] >> 1;
        if (kv[j] < v[j]) {
          lo[j] += h + 1;
          n[j] -= h + 1;
        } else {
          n[j] = h;
        }
      }
      any |= n[j] > 0;
    }
    if (!any) break;
  }
}

__device__ inline bool bit_set(const uint32_t* __restrict__ bm, int32_t u) {
  return (bm[u >> 5] >> (u & 31)) & 1u;
}

// Row lookups of N values at once: the N searches advance in lockstep, so
// each round of their loads is issued together instead of one search after
// another.  ok[j] false: start = len = 0.
template <int N>
__device__ inline void row_lookup_n(const PredView& pv, const int32_t (&v)[N], const bool (&ok)[N],
                                    int32_t (&start)[N], int32_t (&len)[N]) {
  if (pv.dense) {
    int32_t a[N], b[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      a[j] = ok[j] ? pv.dense[v[j]] : 0;
      b[j] = ok[j] ? pv.dense[v[j] + 1] : 0;
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
      start[j] = a[j];
      len[j] = b[j] - a[j];
    }
    return;
  }
  int32_t lo[N], n[N];
  if (pv.dir) {
    int32_t a[N], b[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int32_t bk = v[j] >> pv.dir_shift;
      a[j] = ok[j] ? pv.dir[bk] : 0;
      b[j] = ok[j] ? pv.dir[bk + 1] : 0;
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
      lo[j] = a[j];
      n[j] = b[j] - a[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      lo[j] = 0;
      n[j] = ok[j] ? pv.nr : 0;
    }
  }
  lower_bound_n<N>(pv.keys, v, lo, n);
  int32_t k[N];
#pragma unroll
  for (int j = 0; j < N; ++j) k[j] = (ok[j] && lo[j] < pv.nr) ? pv.keys[lo[j]] : -1;
  int32_t a[N], b[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const bool hit = ok[j] && k[j] == v[j];
    a[j] = hit ? pv.ptr[lo[j]] : 0;
    b[j] = hit ? pv.ptr[lo[j] + 1] : 0;
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    start[j] = a[j];
    len[j] = b[j] - a[j];
  }
}

__device__ inline bool seg_contains(const int32_t* __restrict__ a, int32_t n, int32_t v) {
  const int32_t r = lower_bound_i32(a, n, v);
  return r < n && a[r] == v;
}

// Stable compaction of tile `tile` of n items: emit(i, pos) for each kept
// item i, pos counted from base.  Barriers inside: all threads must call.
template <class Keep, class Emit>
__device__ inline void compact_tile(int64_t tile, int64_t n, int64_t base, Keep keep, Emit emit) {
  __shared__ uint32_t wtot[kWaves];
  const int64_t tile0 = tile * kTile;
  int64_t running = base;
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = tile0 + (int64_t)j * kBlock + threadIdx.x;
    const bool f = (i < n) && keep(i);
    const uint64_t m = __ballot(f);
    const uint32_t rank = mbcnt(m);
    if (lane_id() == 0) wtot[wave_id()] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t wp = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      const uint32_t c = wtot[q];
      if (q < wave_id()) wp += c;
      tot += c;
    }
    if (f) emit(i, running + wp + rank);
    running += tot;
    __syncthreads();
  }
}

__device__ inline PredView view_of(const PredDesc& d, const OriPtrs& o) {
  const int32_t* keys = o.keys;
  const int32_t* ptr = o.ptr;
  const int32_t* nbr = o.nbr;
  const int32_t* dense = o.dense;
  const int32_t* dir = o.dir;
  PredView pv;
  pv.keys = keys + d.row_base;
  pv.ptr = ptr + d.ptr_base;
  pv.nbr = nbr + d.nbr_base;
  pv.src = nullptr;
  pv.dense = d.dense_base >= 0 ? dense + d.dense_base : nullptr;
  pv.dir = d.dir_base >= 0 ? dir + d.dir_base : nullptr;
  pv.hub_keys = d.hub_n ? o.hub_keys + d.hub_base : nullptr;
  pv.hub_bm = d.hub_n ? o.hub_bm + d.hub_base * o.hub_words : nullptr;
  pv.hub_words = o.hub_words;
  pv.nr = (int32_t)d.nr;
  pv.nnz = (int32_t)d.nnz;
  pv.dir_shift = d.dir_shift;
  pv.hub_n = d.hub_n;
  pv.hub_min = o.hub_min;
  pv.pad = 0;
  return pv;
}

// Output column accessors: out(c) is column c's base pointer.
struct OutCols {  // an explicit pointer per column
  const OutSet* s;
  __device__ int32_t* operator()(int c) const { return s->c[c]; }
};
struct OutStrided {  // columns at a fixed stride from one base
  int32_t* base;
  int64_t stride;
  __device__ int32_t* operator()(int c) const { return base + (int64_t)c * stride; }
};

// One lookup request against the two orientations' descriptor tables.
__device__ inline LookupRes lookup_one(const LookupReq& q, const PredDesc* dout,
                                       const PredDesc* din, const OriPtrs& out,
                                       const OriPtrs& in) {
  const PredView pv = q.orient == 0 ? view_of(dout[q.pred], out) : view_of(din[q.pred], in);
  LookupRes r;
  row_lookup(pv, q.v, r.start, r.len);
  r.found = (q.member >= 0 && r.len > 0) ? (seg_contains(pv.nbr + r.start, r.len, q.member) ? 1 : 0)
                                         : 0;
  r.pad = 0;
  return r;
}

constexpr int64_t kSampleRows = 16384;

// Fan-out sample of an expansion candidate: the sum of row lengths over a
// strided sample of at most kSampleRows values of the bound column; slice
// `slice` (of kSampleBlocks) of it per workgroup.
__device__ inline int64_t sample_fanout_slice(int slice, const int32_t* __restrict__ col,
                                              int64_t n, const PredView& pv) {
  const int64_t S = n < kSampleRows ? n : kSampleRows;
  const int64_t stride = S > 0 ? n / S : 1;
  int64_t loc = 0;
  for (int64_t j = (int64_t)slice * kBlock + threadIdx.x; j < S;
       j += (int64_t)kSampleBlocks * kBlock) {
    int32_t st, len;
    row_lookup(pv, col[j * stride], st, len);
    loc += len;
  }
  return block_sum(loc);
}

// ---------------------------------------------------------------- step tiles
// Each returns the workgroup's sum of its per-item results (for the tile
// sums that feed the offsets' prefix sum).

// Expansion count: N_i = length of row col[i], start_i its offset.  With
// kNonEmpty the result also carries, above bit kNonEmptyShift, the number of
// rows with N_i > 0 (a tile's length sum stays below 2^kNonEmptyShift).
constexpr int kNonEmptyShift = 48;
// The count-phase tiles take a tile of kTile rows with a workgroup of kT
// threads (kT in {128, 256, 512}: 16, 8 or 4 rows per thread); row
// tile0 + j * kT + t goes to thread t.
template <bool kNonEmpty = false, int kT = kBlock>
__device__ inline int64_t count_expand_tile(int64_t tile, const int32_t* __restrict__ col,
                                            int64_t n, const PredView& pv,
                                            int32_t* __restrict__ N,
                                            int32_t* __restrict__ start) {
  constexpr int kI = kTile / kT;
  const int64_t tile0 = tile * kTile;
  int32_t v[kI], st[kI], len[kI];
  bool ok[kI];
#pragma unroll
  for (int j = 0; j < kI; ++j) {
    const int64_t i = tile0 + (int64_t)j * kT + threadIdx.x;
    ok[j] = i < n;
    v[j] = ok[j] ? col[i] : 0;
  }
  row_lookup_n<kI>(pv, v, ok, st, len);
  int64_t loc = 0;
#pragma unroll
  for (int j = 0; j < kI; ++j) {
    const int64_t i = tile0 + (int64_t)j * kT + threadIdx.x;
    if (ok[j]) {
      N[i] = len[j];
      start[i] = st[j];
      loc += len[j];
      if (kNonEmpty && len[j] > 0) loc += (int64_t)1 << kNonEmptyShift;
    }
  }
  return block_sum<kT>(loc);
}

// Filter: keep row i when (s_i, o_i) is a pair of the predicate.
template <int kT = kBlock>
__device__ inline int64_t flag_filter_tile(int64_t tile, const ProbeArgs& pa, int64_t n,
                                           const PredView& pv, uint8_t* __restrict__ flags) {
  constexpr int kI = kTile / kT;
  const int64_t tile0 = tile * kTile;
  int32_t sv[kI], ov[kI], st[kI], len[kI];
  bool ok[kI];
#pragma unroll
  for (int j = 0; j < kI; ++j) {
    const int64_t i = tile0 + (int64_t)j * kT + threadIdx.x;
    ok[j] = i < n;
    sv[j] = ok[j] ? (pa.s_col ? pa.s_col[i] : pa.s_const) : 0;
    ov[j] = ok[j] ? (pa.o_col ? pa.o_col[i] : pa.o_const) : 0;
  }
  row_lookup_n<kI>(pv, sv, ok, st, len);
  // rows with a bitmap answer with one bit; the others are searched
  int32_t hub[kI];
#pragma unroll
  for (int j = 0; j < kI; ++j) hub[j] = -1;
  if (pv.hub_n > 0) {
    int32_t hl[kI], hn[kI], hk[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      hl[j] = 0;
      hn[j] = len[j] >= pv.hub_min ? pv.hub_n : 0;
    }
    lower_bound_n<kI>(pv.hub_keys, sv, hl, hn);
#pragma unroll
    for (int j = 0; j < kI; ++j) hk[j] = (len[j] >= pv.hub_min && hl[j] < pv.hub_n) ? pv.hub_keys[hl[j]] : -1;
#pragma unroll
    for (int j = 0; j < kI; ++j) hub[j] = (len[j] > 0 && hk[j] == sv[j]) ? hl[j] : -1;
  }
  // o_i among the members of row s_i
  int32_t lo[kI], cnt[kI], k[kI];
#pragma unroll
  for (int j = 0; j < kI; ++j) {
    lo[j] = st[j];
    cnt[j] = hub[j] >= 0 ? 0 : len[j];
  }
  lower_bound_n<kI>(pv.nbr, ov, lo, cnt);
#pragma unroll
  for (int j = 0; j < kI; ++j) {
    if (hub[j] >= 0)
      k[j] = bit_set(pv.hub_bm + (int64_t)hub[j] * pv.hub_words, ov[j]) ? ov[j] : -1;
    else
      k[j] = (len[j] > 0 && lo[j] < st[j] + len[j]) ? pv.nbr[lo[j]] : -1;
  }
  int64_t loc = 0;
#pragma unroll
  for (int j = 0; j < kI; ++j) {
    const int64_t i = tile0 + (int64_t)j * kT + threadIdx.x;
    if (ok[j]) {
      const uint8_t f = (len[j] > 0 && k[j] == ov[j]) ? 1 : 0;
      flags[i] = f;
      loc += f;
    }
  }
  return block_sum<kT>(loc);
}

// Star-centre intersection: keep driver id x when it is in every list.
// Lists of keys are answered by row lookups and lists with a row bitmap by
// one bit; a sorted list (a row of a compressed matrix) by one of three
// strategies, uniform over a launch:
//   kIsSearch  every driver id binary-searches the whole list in memory;
//   kIsWindow  the tile's driver ids are sorted, so the ids they can meet
//              form one window of the list, found by two searches; a window
//              of at most kWinCap ids is staged in LDS and searched there,
//              a longer one is searched in memory within its bounds;
//   kIsMerge   the window staged as above is merged with the tile's driver
//              ids along the merge path (each thread walks an equal share
//              of the two sorted sequences); a window longer than kWinCap
//              is searched in memory as with kIsWindow.
// kIsWindow and kIsMerge need the driver sorted ascending and distinct, as
// every intersection driver is (a row of a compressed matrix, or a
// predicate's sorted row keys).
constexpr int kIsSearch = 0;
constexpr int kIsWindow = 1;
constexpr int kIsMerge = 2;
constexpr int kWinCap = 2048;

// First index in a[0, n) whose value exceeds v.
__device__ inline int32_t upper_bound_i32(const int32_t* __restrict__ a, int32_t n, int32_t v) {
  int32_t lo = 0, len = n;
  while (len > 0) {
    const int32_t half = len >> 1;
    if (a[lo + half] <= v) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo;
}

// Membership of the driver ids x (tile rows, kT threads) in the sorted list
// seg[0, len) under strategy kS (kIsWindow or kIsMerge); d points at the
// tile's nd driver ids.  Called by the whole workgroup.
template <int kT, int kS>
__device__ inline void window_members(const int32_t* __restrict__ seg, int32_t len,
                                      const int32_t* __restrict__ d, int nd,
                                      const int32_t (&x)[kTile / kT], bool (&keep)[kTile / kT]) {
  constexpr int kI = kTile / kT;
  __shared__ int32_t sWin[2];
  __shared__ int32_t sW[kWinCap];
  if (threadIdx.x == 0) sWin[0] = lower_bound_i32(seg, len, d[0]);
  if (threadIdx.x == 1) sWin[1] = upper_bound_i32(seg, len, d[nd - 1]);
  __syncthreads();
  const int32_t w0 = sWin[0];
  const int32_t nw = sWin[1] - w0;
  if (nw > kWinCap) {
    // the window does not fit: search it in memory
    int32_t lo[kI], cnt[kI], k[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      lo[j] = w0;
      cnt[j] = keep[j] ? nw : 0;
    }
    lower_bound_n<kI>(seg, x, lo, cnt);
#pragma unroll
    for (int j = 0; j < kI; ++j) k[j] = (keep[j] && lo[j] < w0 + nw) ? seg[lo[j]] : -1;
#pragma unroll
    for (int j = 0; j < kI; ++j) keep[j] = keep[j] && k[j] == x[j];
    __syncthreads();  // sWin is rewritten by the next list
    return;
  }
  for (int i = threadIdx.x; i < nw; i += kT) sW[i] = seg[w0 + i];
  if constexpr (kS == kIsWindow) {
    __syncthreads();
    int32_t lo[kI], cnt[kI], k[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      lo[j] = 0;
      cnt[j] = keep[j] ? nw : 0;
    }
    lower_bound_n<kI>(sW, x, lo, cnt);
#pragma unroll
    for (int j = 0; j < kI; ++j) k[j] = (keep[j] && lo[j] < nw) ? sW[lo[j]] : -1;
#pragma unroll
    for (int j = 0; j < kI; ++j) keep[j] = keep[j] && k[j] == x[j];
  } else {
    __shared__ int32_t sD[kTile];
    __shared__ uint8_t sF[kTile];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      const int i = j * kT + threadIdx.x;
      if (i < nd) sD[i] = x[j];
    }
    __syncthreads();
    // thread t merges outputs [t * per, (t + 1) * per) of the merged
    // sequence, a driver id taken before an equal list id; its first driver
    // index is the merge-path split of its first diagonal
    const int total = nd + nw;
    const int per = (total + kT - 1) / kT;
    const int g0 = min(total, (int)threadIdx.x * per);
    const int g1 = min(total, g0 + per);
    int lo = max(0, g0 - nw), hi = min(g0, nd);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sD[mid] <= sW[g0 - mid - 1]) lo = mid + 1;
      else hi = mid;
    }
    int a = lo, b = g0 - lo;
    for (int g = g0; g < g1; ++g) {
      if (a < nd && (b >= nw || sD[a] <= sW[b])) {
        sF[a] = (b < nw && sD[a] == sW[b]) ? 1 : 0;
        ++a;
      } else {
        ++b;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kI; ++j) keep[j] = keep[j] && sF[j * kT + threadIdx.x] != 0;
  }
  __syncthreads();  // sWin, sW (and sD, sF) are rewritten by the next list
}

template <int kT = kBlock, int kS = kIsSearch>
__device__ inline int64_t flag_intersect_tile(int64_t tile, const int32_t* __restrict__ driver,
                                              int64_t n, const ListRef* lists, int nl,
                                              uint8_t* __restrict__ flags) {
  constexpr int kI = kTile / kT;
  const int64_t tile0 = tile * kTile;
  int32_t x[kI];
  bool keep[kI];
#pragma unroll
  for (int j = 0; j < kI; ++j) {
    const int64_t i = tile0 + (int64_t)j * kT + threadIdx.x;
    keep[j] = i < n;
    x[j] = keep[j] ? driver[i] : 0;
  }
  for (int l = 0; l < nl; ++l) {
    const ListRef& L = lists[l];
    if (L.is_keys) {
      int32_t st[kI], len[kI];
      row_lookup_n<kI>(L.pv, x, keep, st, len);
#pragma unroll
      for (int j = 0; j < kI; ++j) keep[j] = keep[j] && len[j] > 0;
    } else if (L.bm) {
#pragma unroll
      for (int j = 0; j < kI; ++j) keep[j] = keep[j] && bit_set(L.bm, x[j]);
    } else if constexpr (kS != kIsSearch) {
      const int nd = (int)(n - tile0 < kTile ? n - tile0 : kTile);
      window_members<kT, kS>(L.seg, (int32_t)L.len, driver + tile0, nd, x, keep);
    } else {
      int32_t lo[kI], cnt[kI], k[kI];
#pragma unroll
      for (int j = 0; j < kI; ++j) {
        lo[j] = 0;
        cnt[j] = keep[j] ? (int32_t)L.len : 0;
      }
      lower_bound_n<kI>(L.seg, x, lo, cnt);
#pragma unroll
      for (int j = 0; j < kI; ++j) k[j] = (keep[j] && lo[j] < (int32_t)L.len) ? L.seg[lo[j]] : -1;
#pragma unroll
      for (int j = 0; j < kI; ++j) keep[j] = keep[j] && k[j] == x[j];
    }
  }
  int64_t loc = 0;
#pragma unroll
  for (int j = 0; j < kI; ++j) {
    const int64_t i = tile0 + (int64_t)j * kT + threadIdx.x;
    if (i < n) {
      flags[i] = keep[j] ? 1 : 0;
      loc += keep[j] ? 1 : 0;
    }
  }
  return block_sum<kT>(loc);
}

// Exclusive prefix sum of one tile of x, offset by base: out[i] for the
// tile's items; returns the tile's total.
template <class Tin, class Tout>
__device__ inline int64_t scan_add_tile(int64_t tile, const Tin* __restrict__ x, int64_t n,
                                        int64_t base, Tout* __restrict__ out) {
  __shared__ int64_t s[kTile];
  const int64_t tile0 = tile * kTile;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = tile0 + (int64_t)j * kBlock + threadIdx.x;
    s[j * kBlock + threadIdx.x] = i < n ? (int64_t)x[i] : 0;
  }
  __syncthreads();
  int64_t loc = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) loc += s[threadIdx.x * kItems + j];
  int64_t tot;
  int64_t ex = block_excl_scan(loc, &tot) + base;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t v = s[threadIdx.x * kItems + j];
    s[threadIdx.x * kItems + j] = ex;
    ex += v;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = tile0 + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) out[i] = (Tout)s[j * kBlock + threadIdx.x];
  }
  return tot;
}

// Stable compaction of the K columns of one tile (K < 0: kdyn columns).
template <int K, class Out>
__device__ inline void compact_cols_tile(int64_t tile, const ColSet& in, int kdyn,
                                         const uint8_t* __restrict__ flags, int64_t n,
                                         int64_t base, const Out& out) {
  compact_tile(
      tile, n, base, [&](int64_t i) { return flags[i] != 0; },
      [&](int64_t i, int64_t pos) {
        if (K >= 0) {
          int32_t x[K > 0 ? K : 1];
#pragma unroll
          for (int c = 0; c < K; ++c) x[c] = in.c[c][i];
#pragma unroll
          for (int c = 0; c < K; ++c) out(c)[pos] = x[c];
        } else {
          for (int c = 0; c < kdyn; ++c) out(c)[pos] = in.c[c][i];
        }
      });
}

// Merge-path split of path position t*kTile over A = row ends P[i+1]
// (i < n) and B = output indices J0..J1-1, rows before outputs on ties:
// the number of rows consumed before that position.
__device__ inline int64_t mp_split(const int64_t* __restrict__ P, int64_t n, int64_t J0,
                                   int64_t J1, int64_t t) {
  const int64_t nb = J1 - J0;
  const int64_t d = min(t * (int64_t)kTile, n + nb);
  int64_t lo = max((int64_t)0, d - nb), hi = min(d, n);
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (P[mid + 1] <= J0 + (d - 1 - mid)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Expansion write: output j in [P_i, P_{i+1}) copies the parent row i and
// appends the (j - P_i)-th member of row i's segment (start_i) in nbr.
//
// A tile is kTile consecutive items of the merge path over (row ends, output
// indices); split[t] gives the rows consumed before it, so the tile covers
// rows a0..a1 and outputs jb + [0, nbt).  Per row the tile keeps in LDS the
// row end relative to jb (clamped to [-1, kTile + 1], which preserves every
// comparison the walk makes) and rb = start_i + (jb - P_i), so that output o of
// row r reads nbr[rb[r] + o]; both fit int32.  Each thread walks kItems path
// items to label outputs with their row; then the tile's outputs are written
// column by column with unit stride.
//
// The write loop is laid out for the memory system: output columns start on
// 256-byte boundaries and the loop is shifted by the tile's offset modulo 64,
// so every wave store covers whole 128-byte lines (unaligned tile starts
// halved the store bandwidth); each thread handles U outputs per iteration
// (four for up to three parent columns, else two) and issues all their loads
// (neighbour ids, K parent values) before any store.  K is a compile-time
// column count (-1: any count, in groups of 4).
template <int K, class Out>
__device__ inline void write_outputs(const ColSet& in, int kdyn, const int32_t* __restrict__ nbr,
                                     const uint16_t* sRow, const int32_t* sRb,
                                     const int32_t* sIdx, int64_t a0, int64_t ob, int nbt,
                                     const Out& out) {
  constexpr int U = (K >= 0 && K <= 3) ? 4 : 2;
  const int k = K >= 0 ? K : kdyn;
  const int al = (int)(ob & 63);
  const int span = nbt + al;
  for (int q = threadIdx.x; q < span; q += U * kBlock) {
    int o[U];
    bool ok[U];
    int r[U];
    int32_t v[U];
    int64_t row[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      o[u] = q + u * kBlock - al;
      ok[u] = o[u] >= 0 && o[u] < nbt;
      r[u] = ok[u] ? sRow[o[u]] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = ok[u] ? nbr[sRb[r[u]] + o[u]] : 0;
      // parent rows: consecutive, or (compacted rows) their original indices
      row[u] = sIdx ? (int64_t)sIdx[r[u]] : a0 + r[u];
    }
    if (K >= 0) {
      int32_t x[U][K > 0 ? K : 1];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < K; ++c) x[u][c] = ok[u] ? in.c[c][row[u]] : 0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) {
#pragma unroll
          for (int c = 0; c < K; ++c) __builtin_nontemporal_store(x[u][c], &out(c)[ob + o[u]]);
        }
    } else {
      for (int c0 = 0; c0 < k; c0 += 4) {
        int32_t x[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) x[u][c] = (ok[u] && c0 + c < k) ? in.c[c0 + c][row[u]] : 0;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (ok[u] && c0 + c < k) __builtin_nontemporal_store(x[u][c], &out(c0 + c)[ob + o[u]]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) __builtin_nontemporal_store(v[u], &out(k)[ob + o[u]]);
  }
}

// LDS staging of one path tile: each row's end offset and neighbour base
// relative to the tile, the row of each output, and (compacted rows) each
// row's input index.
struct TileLds {
  int32_t* sE;     // [kTile + 1]
  int32_t* sRb;    // [kTile + 1]
  uint16_t* sRow;  // [kTile]
  int32_t* sIdx;   // [kTile + 1] with compacted rows (null: staged in sE after the walk)
};

// One path tile t of an expansion (all threads of the workgroup call it),
// staged in L.  With ridx (kIdx), the rows are a compacted list: row i of
// P/start is the input row ridx[i].
template <int K, class Out, bool kIdx = false>
__device__ inline void write_expand_tile_in(const TileLds& L, int64_t t, const ColSet& in,
                                            int kdyn, const int64_t* __restrict__ P,
                                            const int32_t* __restrict__ start, int64_t n,
                                            const int32_t* __restrict__ nbr, int64_t J0,
                                            int64_t J1, const int64_t* __restrict__ split,
                                            const Out& out,
                                            const int32_t* __restrict__ ridx = nullptr) {
  int32_t* const sE = L.sE;
  int32_t* const sRb = L.sRb;
  uint16_t* const sRow = L.sRow;
  int32_t* const sIdx = L.sIdx;
  const int64_t nb = J1 - J0;
  const int64_t total = n + nb;
  const int64_t d0 = t * (int64_t)kTile;
  const int64_t d1 = min(d0 + (int64_t)kTile, total);
  const int64_t a0 = split[t], a1 = split[t + 1];
  const int64_t b0 = d0 - a0, b1 = d1 - a1;
  const int nat = (int)(a1 - a0), nbt = (int)(b1 - b0);
  if (nbt <= 0) return;  // block-uniform
  const int64_t jb = J0 + b0;
  const int64_t rl = min(a1, n - 1);
  const int nr = (int)(rl - a0 + 1);
  for (int i = threadIdx.x; i < nr; i += kBlock) {
    const int64_t pb = P[a0 + i], pe = P[a0 + i + 1];
    const int64_t er = pe - jb;
    sE[i] = er > (int64_t)kTile + 1 ? kTile + 1 : (er < -1 ? -1 : (int32_t)er);
    sRb[i] = (int32_t)((int64_t)start[a0 + i] + (jb - pb));
    if (kIdx && sIdx) sIdx[i] = ridx[a0 + i];
  }
  __syncthreads();
  const int dl = min((int)threadIdx.x * kItems, nat + nbt);
  const int de = min((int)threadIdx.x * kItems + kItems, nat + nbt);
  int lo = max(0, dl - nbt), hi = min(dl, nat);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sE[mid] <= dl - 1 - mid) lo = mid + 1;
    else hi = mid;
  }
  int a = lo, b = dl - lo;
  for (int step = dl; step < de; ++step) {
    const bool takeA = (a < nat) && (b >= nbt || sE[a] <= b);
    if (takeA) {
      ++a;
    } else {
      sRow[b] = (uint16_t)a;
      ++b;
    }
  }
  __syncthreads();
  if (kIdx && !sIdx) {
    // without an area of its own the row indices take the place of the row
    // ends, which the walk no longer needs
    for (int i = threadIdx.x; i < nr; i += kBlock) sE[i] = ridx[a0 + i];
    __syncthreads();
  }
  write_outputs<K, Out>(in, kdyn, nbr, sRow, sRb, kIdx ? (sIdx ? sIdx : sE) : nullptr, a0,
                        jb - J0, nbt, out);
}

// write_expand_tile_in with the workgroup's own staging.
template <int K, class Out, bool kIdx = false>
__device__ inline void write_expand_tile(int64_t t, const ColSet& in, int kdyn,
                                         const int64_t* __restrict__ P,
                                         const int32_t* __restrict__ start, int64_t n,
                                         const int32_t* __restrict__ nbr, int64_t J0, int64_t J1,
                                         const int64_t* __restrict__ split, const Out& out,
                                         const int32_t* __restrict__ ridx = nullptr) {
  __shared__ int32_t sE[kTile + 1];
  __shared__ int32_t sRb[kTile + 1];
  __shared__ uint16_t sRow[kTile];
  __shared__ int32_t sIdx[kIdx ? kTile + 1 : 1];
  write_expand_tile_in<K, Out, kIdx>(TileLds{sE, sRb, sRow, sIdx}, t, in, kdyn, P, start, n, nbr,
                                     J0, J1, split, out, ridx);
}

}  // namespace dev
}  // namespace gsmat
