// Device kernels of the gsmat library (CDNA4 / gfx950, wave64).
//
// All per-row work uses the same tiling: a workgroup of kBlock threads owns a
// tile of kTile consecutive items and thread t touches items t, t+kBlock, ...,
// so every global access of a tile is coalesced.  Kernels that feed a prefix
// sum also write one partial sum per tile; the offsets are then produced by a
// small single-workgroup scan over the tile sums and an add pass.  Ordered
// (stable) compaction ranks the kept items of a tile with wave ballots and
// mbcnt, so output order equals input order.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "device.hpp"

namespace gsmat {

namespace {

using namespace dev;

// ---------------------------------------------------------------- prefix sums
__global__ __launch_bounds__(kBlock) void k_scan_tile_sums(int64_t* ts, int64_t nt,
                                                           int64_t* total, int64_t* host_total) {
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nt; c0 += kTile) {
    int64_t v[kItems];
    int64_t loc = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t i = c0 + (int64_t)threadIdx.x * kItems + j;
      v[j] = i < nt ? ts[i] : 0;
      loc += v[j];
    }
    int64_t tot;
    int64_t ex = block_excl_scan(loc, &tot) + carry;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t i = c0 + (int64_t)threadIdx.x * kItems + j;
      if (i < nt) ts[i] = ex;
      ex += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    total[0] = carry;
    if (host_total) host_total[0] = carry;  // pinned host memory: read after the stream syncs
  }
}

// Two tile-sum arrays (neither null) scanned in one pass (device.hpp).
__global__ __launch_bounds__(kScanBlock) void k_scan_tile_sums2(int64_t* ts, int64_t* ts2,
                                                                int64_t nt) {
  scan_tile_sums2_block(ts, ts2, nt);
}

template <class Tin, class Tout>
__global__ __launch_bounds__(kBlock) void k_scan_add(const Tin* __restrict__ x, int64_t n,
                                                     const int64_t* __restrict__ tile_off,
                                                     Tout* __restrict__ out, int write_total) {
  const int64_t tot = scan_add_tile<Tin, Tout>(blockIdx.x, x, n, tile_off[blockIdx.x], out);
  if (write_total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1)
    out[n] = (Tout)(tile_off[blockIdx.x] + tot);
}

__global__ __launch_bounds__(kBlock) void k_tile_reduce_u32(const uint32_t* __restrict__ x,
                                                            int64_t n, int64_t* ts) {
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
  int64_t loc = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = tile0 + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) loc += x[i];
  }
  const int64_t t = block_sum(loc);
  if (threadIdx.x == 0) ts[blockIdx.x] = t;
}

// ---------------------------------------------------------------- radix sort
__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                    int shift, uint32_t* __restrict__ hist,
                                                    int64_t nb) {
  __shared__ uint32_t h[kWaves][256];
  for (int i = threadIdx.x; i < kWaves * 256; i += kBlock) (&h[0][0])[i] = 0;
  __syncthreads();
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = tile0 + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[wave_id()][(keys[i] >> shift) & 255], 1u);
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) c += h[w][threadIdx.x];
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = c;
}

__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint64_t* __restrict__ in,
                                                       uint64_t* __restrict__ out, int64_t n,
                                                       int shift,
                                                       const uint32_t* __restrict__ offs,
                                                       int64_t nb) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kWaves][256];
  base[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
  const uint64_t lt = __lanemask_lt();
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = tile0 + (int64_t)j * kBlock + threadIdx.x;
    const bool valid = i < n;
    const uint64_t k = valid ? in[i] : 0;
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && (peers & lt) == 0) wcnt[wave_id()][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + rank;
      for (int w = 0; w < wave_id(); ++w) pos += wcnt[w][d];
      out[pos] = k;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      add += wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = 0;
    }
    base[threadIdx.x] += add;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- index build
__global__ void k_pack_keys(const int32_t* __restrict__ s, const int32_t* __restrict__ p,
                            const int32_t* __restrict__ o, int64_t n, int vb,
                            uint64_t* __restrict__ ks, uint64_t* __restrict__ ko) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t pp = (uint64_t)(uint32_t)p[i] << (2 * vb);
    const uint64_t ss = (uint32_t)s[i], oo = (uint32_t)o[i];
    ks[i] = pp | (ss << vb) | oo;
    ko[i] = pp | (oo << vb) | ss;
  }
}

__global__ __launch_bounds__(kBlock) void k_flag_adjacent(const uint64_t* __restrict__ k,
                                                          int64_t n, int sh,
                                                          uint8_t* __restrict__ flags,
                                                          int64_t* __restrict__ ts) {
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
  int64_t loc = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = tile0 + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) {
      const uint8_t f = (i == 0 || (k[i] >> sh) != (k[i - 1] >> sh)) ? 1 : 0;
      flags[i] = f;
      loc += f;
    }
  }
  const int64_t t = block_sum(loc);
  if (threadIdx.x == 0) ts[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_compact_u64(const uint64_t* __restrict__ in,
                                                        const uint8_t* __restrict__ flags,
                                                        int64_t n,
                                                        const int64_t* __restrict__ tile_off,
                                                        uint64_t* __restrict__ out) {
  compact_tile(
      blockIdx.x, n, tile_off[blockIdx.x], [&](int64_t i) { return flags[i] != 0; },
      [&](int64_t i, int64_t pos) { out[pos] = in[i]; });
}

__global__ __launch_bounds__(kBlock) void k_compact_index(const uint8_t* __restrict__ flags,
                                                          int64_t n,
                                                          const int64_t* __restrict__ tile_off,
                                                          int64_t* __restrict__ out) {
  compact_tile(
      blockIdx.x, n, tile_off[blockIdx.x], [&](int64_t i) { return flags[i] != 0; },
      [&](int64_t i, int64_t pos) { out[pos] = i; });
}

__global__ void k_split_members(const uint64_t* __restrict__ k, int64_t n, int vb,
                                int32_t* __restrict__ nbr, int32_t* __restrict__ src) {
  const uint64_t vmask = (vb >= 64) ? ~0ull : ((1ull << vb) - 1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t x = k[i];
    nbr[i] = (int32_t)(x & vmask);
    if (src) src[i] = (int32_t)((x >> vb) & vmask);
  }
}

__global__ void k_pred_heads(const uint64_t* __restrict__ k, const int64_t* __restrict__ row_pos,
                             int64_t R, int vb, int64_t* __restrict__ pfe,
                             int64_t* __restrict__ pfr) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = row_pos[r];
    const uint64_t p = k[i] >> (2 * vb);
    if (r == 0 || p != (k[row_pos[r - 1]] >> (2 * vb))) {
      pfe[p] = i;
      pfr[p] = r;
    }
  }
}

__global__ void k_fill_rows(const uint64_t* __restrict__ k, const int64_t* __restrict__ row_pos,
                            int64_t R, int vb, const int64_t* __restrict__ pfe,
                            int32_t* __restrict__ keys, int32_t* __restrict__ ptr) {
  const uint64_t vmask = (1ull << vb) - 1;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = row_pos[r];
    const uint64_t x = k[i];
    const int64_t p = (int64_t)(x >> (2 * vb));
    keys[r] = (int32_t)((x >> vb) & vmask);
    ptr[r + p] = (int32_t)(i - pfe[p]);
  }
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_dense_ptr(PredView pv, int64_t V, int32_t* __restrict__ dense) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= V;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = (v >= (int64_t)INT32_MAX) ? pv.nr : lower_bound_i32(pv.keys, pv.nr, (int32_t)v);
    dense[v] = pv.ptr[r];
  }
}

__global__ void k_row_dir(PredView pv, int32_t shift, int64_t nb, int32_t* __restrict__ dir) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = b << shift;
    dir[b] = v >= (int64_t)INT32_MAX ? pv.nr : lower_bound_i32(pv.keys, pv.nr, (int32_t)v);
  }
}

__global__ void k_long_rows(PredView pv, int32_t min_len, int32_t* __restrict__ out,
                            int32_t* __restrict__ count, int32_t cap) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < pv.nr;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t len = pv.ptr[r + 1] - pv.ptr[r];
    if (len >= min_len) {
      const int32_t i = atomicAdd(count, 1);
      if (i < cap) {
        out[2 * i] = pv.keys[r];
        out[2 * i + 1] = len;
      }
    }
  }
}

__global__ void k_row_bitmap(PredView pv, int32_t v, uint32_t* __restrict__ bm) {
  int32_t st, len;
  row_lookup(pv, v, st, len);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = pv.nbr[st + i];
    atomicOr(&bm[u >> 5], 1u << (u & 31));
  }
}

__global__ void k_ptr_sentinels(const PredDesc* __restrict__ d, int32_t P, int32_t* __restrict__ ptr) {
  const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) ptr[d[p].ptr_base + d[p].nr] = (int32_t)d[p].nnz;
}

__global__ void k_lookup(LookupBatch b, const PredDesc* dout, const PredDesc* din, OriPtrs out,
                         OriPtrs in, LookupRes* res) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  res[i] = lookup_one(b.req[i], dout, din, out, in);
}

// ---------------------------------------------------------------- join steps
__global__ __launch_bounds__(kBlock) void k_count_expand(const int32_t* __restrict__ col,
                                                         int64_t n, PredView pv,
                                                         int32_t* __restrict__ N,
                                                         int32_t* __restrict__ start,
                                                         int64_t* __restrict__ ts) {
  const int64_t t = count_expand_tile(blockIdx.x, col, n, pv, N, start);
  if (threadIdx.x == 0) ts[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_flag_filter(ProbeArgs pa, int64_t n, PredView pv,
                                                        uint8_t* __restrict__ flags,
                                                        int64_t* __restrict__ ts) {
  const int64_t t = flag_filter_tile(blockIdx.x, pa, n, pv, flags);
  if (threadIdx.x == 0) ts[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_flag_diag(const int32_t* __restrict__ a,
                                                      const int32_t* __restrict__ b, int64_t n,
                                                      uint8_t* __restrict__ flags,
                                                      int64_t* __restrict__ ts) {
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
  int64_t loc = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = tile0 + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) {
      const uint8_t f = a[i] == b[i] ? 1 : 0;
      flags[i] = f;
      loc += f;
    }
  }
  const int64_t t = block_sum(loc);
  if (threadIdx.x == 0) ts[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_flag_intersect(const int32_t* __restrict__ driver,
                                                           int64_t n, ListSet ls,
                                                           uint8_t* __restrict__ flags,
                                                           int64_t* __restrict__ ts) {
  const int64_t t = flag_intersect_tile(blockIdx.x, driver, n, ls.l, ls.n, flags);
  if (threadIdx.x == 0) ts[blockIdx.x] = t;
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_compact_cols(ColSet in, int kdyn,
                                                         const uint8_t* __restrict__ flags,
                                                         int64_t n,
                                                         const int64_t* __restrict__ tile_off,
                                                         OutSet out) {
  compact_cols_tile<K>(blockIdx.x, in, kdyn, flags, n, tile_off[blockIdx.x], OutCols{&out});
}

// Merge path over A = row ends E[i] = P[i+1] (i < n) and B = output indices
// J0..J1-1, rows before outputs on ties.  split[t] = rows consumed before path
// position t*kTile.
__global__ void k_mp_partition(const int64_t* __restrict__ P, int64_t n, int64_t J0, int64_t J1,
                               int64_t* __restrict__ split, int64_t ntiles) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  split[t] = mp_split(P, n, J0, J1, t);
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_write_expand(ColSet in, int kdyn,
                                                         const int64_t* __restrict__ P,
                                                         const int32_t* __restrict__ start,
                                                         int64_t n,
                                                         const int32_t* __restrict__ nbr,
                                                         int64_t J0, int64_t J1,
                                                         const int64_t* __restrict__ split,
                                                         OutSet out) {
  write_expand_tile<K>(blockIdx.x, in, kdyn, P, start, n, nbr, J0, J1, split, OutCols{&out});
}

__global__ void k_cartesian(ColSet a, int ka, ColSet b, int kb, int64_t nb, int64_t J0,
                            int64_t J1, OutSet out) {
  for (int64_t j = J0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < J1;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ia = j / nb, ib = j - ia * nb;
    const int64_t oj = j - J0;
    for (int c = 0; c < ka; ++c) out.c[c][oj] = a.c[c][ia];
    for (int c = 0; c < kb; ++c) out.c[ka + c][oj] = b.c[c][ib];
  }
}

// Sum of row lengths over a strided sample of the bound column; blockIdx.y
// selects the candidate, blockIdx.x one of kSampleBlocks slices of the sample.
__global__ __launch_bounds__(kBlock) void k_sample_fanout(SampleSet ss, int64_t* __restrict__ part) {
  const int cand = blockIdx.y;
  const int64_t t = sample_fanout_slice(blockIdx.x, ss.col[cand], ss.n, ss.pv[cand]);
  if (threadIdx.x == 0) part[cand * kSampleBlocks + blockIdx.x] = t;
}

__global__ void k_pack_rows(ColSet cols, int k, int64_t row0, int64_t rows,
                            int32_t* __restrict__ out) {
  const int64_t total = rows * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / k;
    const int c = (int)(e - r * k);
    const int32_t* col = cols.c[c];
    out[e] = col ? col[row0 + r] : -1;  // no column: the variable is unbound
  }
}

inline unsigned grid_for(int64_t n, int block = kBlock, int64_t cap = 65536) {
  int64_t g = ceil_div(n > 0 ? n : 1, block);
  if (g > cap) g = cap;
  return (unsigned)g;
}
inline unsigned tiles_for(int64_t n) { return (unsigned)ceil_div(n > 0 ? n : 1, kTile); }

}  // namespace

// ---------------------------------------------------------------- launchers
#define GS_LAUNCH(cls, bytes, ...)              \
  do {                                          \
    const bool _prof = prof_on(cls);            \
    if (_prof) prof_begin(s, cls);              \
    __VA_ARGS__;                                \
    GS_HIP(hipGetLastError());                  \
    if (_prof) prof_end(s, cls, bytes);         \
  } while (0)

void launch_scan_tile_sums(int64_t* tile_sum, int64_t nt, int64_t* total, hipStream_t s,
                           int64_t* host_total) {
  GS_LAUNCH(GSMAT_K_SCAN, 16.0 * nt,
            hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(kBlock), 0, s, tile_sum, nt, total,
                               host_total));
}

void launch_scan_tile_sums2(int64_t* ts, int64_t* ts2, int64_t nt, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_SCAN, 32.0 * nt,
            hipLaunchKernelGGL(k_scan_tile_sums2, dim3(1), dim3(kScanBlock), 0, s, ts, ts2, nt));
}

void launch_scan_add_i32(const int32_t* N, int64_t n, const int64_t* tile_off, int64_t* P,
                         hipStream_t s) {
  GS_LAUNCH(GSMAT_K_SCAN, 12.0 * n,
            hipLaunchKernelGGL((k_scan_add<int32_t, int64_t>), dim3(tiles_for(n)), dim3(kBlock),
                               0, s, N, n, tile_off, P, 1));
}

void launch_tile_reduce_u32(const uint32_t* x, int64_t n, int64_t* tile_sum, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 4.0 * n,
            hipLaunchKernelGGL(k_tile_reduce_u32, dim3(tiles_for(n)), dim3(kBlock), 0, s, x, n,
                               tile_sum));
}

void launch_scan_add_u32(const uint32_t* x, int64_t n, const int64_t* tile_off, uint32_t* out,
                         hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 8.0 * n,
            hipLaunchKernelGGL((k_scan_add<uint32_t, uint32_t>), dim3(tiles_for(n)),
                               dim3(kBlock), 0, s, x, n, tile_off, out, 0));
}

void radix_sort_u64(uint64_t* keys, uint64_t* tmp, int64_t n, int nbits, DeviceMem& mem,
                    hipStream_t s) {
  if (n <= 1) return;
  const int64_t nb = ceil_div(n, kTile);
  const int64_t hn = 256 * nb;
  const int64_t ht = ceil_div(hn, kTile);
  uint32_t* hist = (uint32_t*)mem.alloc(sizeof(uint32_t) * hn, s);
  uint32_t* offs = (uint32_t*)mem.alloc(sizeof(uint32_t) * hn, s);
  int64_t* ts = (int64_t*)mem.alloc(sizeof(int64_t) * (ht + 1), s);
  if (!hist || !offs || !ts) {
    if (hist) mem.free(hist, sizeof(uint32_t) * hn, s);
    if (offs) mem.free(offs, sizeof(uint32_t) * hn, s);
    if (ts) mem.free(ts, sizeof(int64_t) * (ht + 1), s);
    throw OomFail{sizeof(uint32_t) * (size_t)hn};
  }
  uint64_t* src = keys;
  uint64_t* dst = tmp;
  const int passes = (nbits + 7) / 8;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 8 * pass;
    GS_LAUNCH(GSMAT_K_OTHER, 8.0 * n,
              hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(kBlock), 0, s, src, n, shift,
                                 hist, nb));
    launch_tile_reduce_u32(hist, hn, ts, s);
    launch_scan_tile_sums(ts, ht, ts + ht, s, nullptr);
    launch_scan_add_u32(hist, hn, ts, offs, s);
    GS_LAUNCH(GSMAT_K_OTHER, 16.0 * n,
              hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(kBlock), 0, s, src, dst,
                                 n, shift, offs, nb));
    std::swap(src, dst);
  }
  if (src != keys) GS_HIP(hipMemcpyAsync(keys, src, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
  mem.free(hist, sizeof(uint32_t) * hn, s);
  mem.free(offs, sizeof(uint32_t) * hn, s);
  mem.free(ts, sizeof(int64_t) * (ht + 1), s);
}

void launch_pack_keys(const int32_t* sv, const int32_t* p, const int32_t* o, int64_t n, int vb,
                      uint64_t* k_by_s, uint64_t* k_by_o, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 28.0 * n,
            hipLaunchKernelGGL(k_pack_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, sv, p, o, n,
                               vb, k_by_s, k_by_o));
}

void launch_flag_unique(const uint64_t* k, int64_t n, uint8_t* flags, int64_t* tile_sum,
                        hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 9.0 * n,
            hipLaunchKernelGGL(k_flag_adjacent, dim3(tiles_for(n)), dim3(kBlock), 0, s, k, n, 0,
                               flags, tile_sum));
}

void launch_flag_row_heads(const uint64_t* k, int64_t n, int vb, uint8_t* flags,
                           int64_t* tile_sum, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 9.0 * n,
            hipLaunchKernelGGL(k_flag_adjacent, dim3(tiles_for(n)), dim3(kBlock), 0, s, k, n, vb,
                               flags, tile_sum));
}

void launch_compact_u64(const uint64_t* in, const uint8_t* flags, int64_t n,
                        const int64_t* tile_off, uint64_t* out, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_COMPACT, 17.0 * n,
            hipLaunchKernelGGL(k_compact_u64, dim3(tiles_for(n)), dim3(kBlock), 0, s, in, flags,
                               n, tile_off, out));
}

void launch_compact_index(const uint8_t* flags, int64_t n, const int64_t* tile_off,
                          int64_t* out_idx, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_COMPACT, 9.0 * n,
            hipLaunchKernelGGL(k_compact_index, dim3(tiles_for(n)), dim3(kBlock), 0, s, flags, n,
                               tile_off, out_idx));
}

void launch_split_members(const uint64_t* k, int64_t n, int vb, int32_t* nbr, int32_t* src,
                          hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 16.0 * n,
            hipLaunchKernelGGL(k_split_members, dim3(grid_for(n)), dim3(kBlock), 0, s, k, n, vb,
                               nbr, src));
}

void launch_pred_heads(const uint64_t* k, const int64_t* row_pos, int64_t R, int vb,
                       int64_t* pfe, int64_t* pfr, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 24.0 * R,
            hipLaunchKernelGGL(k_pred_heads, dim3(grid_for(R)), dim3(kBlock), 0, s, k, row_pos,
                               R, vb, pfe, pfr));
}

void launch_fill_rows(const uint64_t* k, const int64_t* row_pos, int64_t R, int vb,
                      const int64_t* pfe, int32_t* keys, int32_t* ptr, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 24.0 * R,
            hipLaunchKernelGGL(k_fill_rows, dim3(grid_for(R)), dim3(kBlock), 0, s, k, row_pos, R,
                               vb, pfe, keys, ptr));
}

void launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) {
  if (n <= 0) return;
  GS_LAUNCH(GSMAT_K_OTHER, 8.0 * n,
            hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v));
}

void launch_dense_ptr(PredView pv, int64_t V, int32_t* dense, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 4.0 * (V + 1),
            hipLaunchKernelGGL(k_dense_ptr, dim3(grid_for(V + 1)), dim3(kBlock), 0, s, pv, V,
                               dense));
}

void launch_row_dir(PredView pv, int32_t shift, int64_t nb, int32_t* dir, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 4.0 * (nb + 1),
            hipLaunchKernelGGL(k_row_dir, dim3(grid_for(nb + 1)), dim3(kBlock), 0, s, pv, shift, nb,
                               dir));
}

void launch_long_rows(PredView pv, int32_t min_len, int32_t* out, int32_t* count, int32_t cap,
                      hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 8.0 * pv.nr,
            hipLaunchKernelGGL(k_long_rows, dim3(grid_for(pv.nr)), dim3(kBlock), 0, s, pv, min_len,
                               out, count, cap));
}

void launch_row_bitmap(PredView pv, int32_t v, int64_t len, uint32_t* bm, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 8.0 * len,
            hipLaunchKernelGGL(k_row_bitmap, dim3(grid_for(len)), dim3(kBlock), 0, s, pv, v, bm));
}

void launch_ptr_sentinels(const PredDesc* d, int32_t P, int32_t* ptr, hipStream_t s) {
  if (P <= 0) return;
  GS_LAUNCH(GSMAT_K_OTHER, 0.0,
            hipLaunchKernelGGL(k_ptr_sentinels, dim3((unsigned)ceil_div(P, kBlock)), dim3(kBlock), 0,
                               s, d, P, ptr));
}

void launch_lookup(const LookupBatch& b, const PredDesc* desc_out, const PredDesc* desc_in,
                   OriPtrs out, OriPtrs in, LookupRes* res, hipStream_t s) {
  if (b.n <= 0) return;
  GS_LAUNCH(GSMAT_K_OTHER, 32.0 * b.n,
            hipLaunchKernelGGL(k_lookup, dim3(1), dim3(64), 0, s, b, desc_out, desc_in, out, in,
                               res));
}

void launch_count_expand(const int32_t* col, int64_t n, PredView pv, int32_t* N, int32_t* start,
                         int64_t* tile_sum, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_COUNT, 20.0 * n,
            hipLaunchKernelGGL(k_count_expand, dim3(tiles_for(n)), dim3(kBlock), 0, s, col, n, pv,
                               N, start, tile_sum));
}

void launch_flag_filter(ProbeArgs pa, int64_t n, PredView pv, uint8_t* flags, int64_t* tile_sum,
                        hipStream_t s) {
  GS_LAUNCH(GSMAT_K_COUNT, 21.0 * n,
            hipLaunchKernelGGL(k_flag_filter, dim3(tiles_for(n)), dim3(kBlock), 0, s, pa, n, pv,
                               flags, tile_sum));
}

void launch_flag_diag(const int32_t* a, const int32_t* b, int64_t n, uint8_t* flags,
                      int64_t* tile_sum, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_COUNT, 9.0 * n,
            hipLaunchKernelGGL(k_flag_diag, dim3(tiles_for(n)), dim3(kBlock), 0, s, a, b, n, flags,
                               tile_sum));
}

void launch_flag_intersect(const int32_t* driver, int64_t n, ListSet ls, uint8_t* flags,
                           int64_t* tile_sum, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_COUNT, (4.0 + 4.0 * ls.n + 1.0) * n,
            hipLaunchKernelGGL(k_flag_intersect, dim3(tiles_for(n)), dim3(kBlock), 0, s, driver, n,
                               ls, flags, tile_sum));
}

void launch_compact_cols(ColSet in, int k, const uint8_t* flags, int64_t n,
                         const int64_t* tile_off, OutSet out, hipStream_t s) {
#define GS_COMPACT_CASE(KK)                                                                    \
  case KK:                                                                                   \
    hipLaunchKernelGGL(k_compact_cols<KK>, dim3(tiles_for(n)), dim3(kBlock), 0, s, in, k, flags, \
                       n, tile_off, out);                                                    \
    break;
  GS_LAUNCH(GSMAT_K_COMPACT, (1.0 + 4.0 * k) * n, switch (k) {
    GS_COMPACT_CASE(1)
    GS_COMPACT_CASE(2)
    GS_COMPACT_CASE(3)
    GS_COMPACT_CASE(4)
    GS_COMPACT_CASE(5)
    GS_COMPACT_CASE(6)
    GS_COMPACT_CASE(7)
    GS_COMPACT_CASE(8)
    default:
      hipLaunchKernelGGL(k_compact_cols<-1>, dim3(tiles_for(n)), dim3(kBlock), 0, s, in, k, flags, n,
                         tile_off, out);
  });
#undef GS_COMPACT_CASE
}

void launch_mp_partition(const int64_t* P, int64_t n, int64_t J0, int64_t J1, int64_t* split,
                         int64_t ntiles, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 8.0 * (ntiles + 1),
            hipLaunchKernelGGL(k_mp_partition, dim3((unsigned)ceil_div(ntiles + 1, kBlock)),
                               dim3(kBlock), 0, s, P, n, J0, J1, split, ntiles));
}

void launch_write_expand(ColSet in, int k, const int64_t* P, const int32_t* start, int64_t n,
                         const int32_t* nbr, int64_t J0, int64_t J1, const int64_t* split,
                         int64_t ntiles, OutSet out, double alg_bytes, hipStream_t s) {
#define GS_WRITE_CASE(KK)                                                                        \
  case KK:                                                                                     \
    hipLaunchKernelGGL(k_write_expand<KK>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, in, k, P, \
                       start, n, nbr, J0, J1, split, out);                                      \
    break;
  GS_LAUNCH(GSMAT_K_WRITE, alg_bytes, switch (k) {
    GS_WRITE_CASE(0)
    GS_WRITE_CASE(1)
    GS_WRITE_CASE(2)
    GS_WRITE_CASE(3)
    GS_WRITE_CASE(4)
    GS_WRITE_CASE(5)
    GS_WRITE_CASE(6)
    GS_WRITE_CASE(7)
    GS_WRITE_CASE(8)
    GS_WRITE_CASE(9)
    GS_WRITE_CASE(10)
    GS_WRITE_CASE(11)
    default:
      hipLaunchKernelGGL(k_write_expand<-1>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, in, k, P,
                         start, n, nbr, J0, J1, split, out);
  });
#undef GS_WRITE_CASE
}

void launch_cartesian(ColSet a, int ka, int64_t na, ColSet b, int kb, int64_t nb, int64_t J0,
                      int64_t J1, OutSet out, hipStream_t s) {
  (void)na;
  GS_LAUNCH(GSMAT_K_OTHER, 4.0 * (ka + kb) * 2.0 * (J1 - J0),
            hipLaunchKernelGGL(k_cartesian, dim3(grid_for(J1 - J0)), dim3(kBlock), 0, s, a, ka, b,
                               kb, nb, J0, J1, out));
}

void launch_sample_fanout(const SampleSet& ss, int64_t* part, hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 0.0,
            hipLaunchKernelGGL(k_sample_fanout, dim3(kSampleBlocks, (unsigned)ss.ncand),
                               dim3(kBlock), 0, s, ss, part));
}

void launch_pack_rows(ColSet cols, int k, int64_t row0, int64_t rows, int32_t* out,
                      hipStream_t s) {
  GS_LAUNCH(GSMAT_K_OTHER, 8.0 * k * rows,
            hipLaunchKernelGGL(k_pack_rows, dim3(grid_for(rows * k)), dim3(kBlock), 0, s, cols, k,
                               row0, rows, out));
}

}  // namespace gsmat
