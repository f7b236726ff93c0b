// Storage (paper Sec. 5): loading the triple set and building, on the device,
// one boolean sparse matrix per predicate in two compressed orientations.
//
// Build pipeline per orientation (all on the device, one stream):
//   pack (p, row, member) into one 64-bit key -> LSD radix sort -> drop
//   adjacent duplicates (D is a set, Sec. 3.1) -> flag the first entry of every
//   (p, row) -> compact their positions -> per-predicate first entry/row ->
//   row ids + row offsets (the Row / Rpos auxiliary arrays of Sec. 6.3) and
//   member lists -> optional dense row pointers for heavy predicates.
#include <algorithm>
#include <atomic>
#include <cstring>

#include "store.hpp"

namespace gsmat {

namespace {

int bits_for(int64_t maxval) {
  int b = 1;
  while (b < 62 && ((int64_t)1 << b) <= maxval) ++b;
  return b;
}

// Temporary device buffer returned to the pool when it goes out of scope.
template <class T>
struct Tmp {
  DeviceMem* mem;
  hipStream_t s;
  T* p = nullptr;
  size_t bytes = 0;
  Tmp(DeviceMem* m, int64_t n, hipStream_t st) : mem(m), s(st) {
    bytes = sizeof(T) * (size_t)std::max<int64_t>(n, 1);
    p = (T*)mem->alloc(bytes, s);
    if (!p) throw OomFail{bytes};
  }
  ~Tmp() { release(); }
  void release() {
    if (p) mem->free(p, bytes, s);
    p = nullptr;
  }
  Tmp(const Tmp&) = delete;
  Tmp& operator=(const Tmp&) = delete;
};

int64_t read_i64(const int64_t* d, hipStream_t s) {
  int64_t v = 0;
  GS_HIP(hipMemcpyAsync(&v, d, sizeof(v), hipMemcpyDeviceToHost, s));
  GS_HIP(hipStreamSynchronize(s));
  return v;
}

}  // namespace

PredView Orientation::view(int32_t p) const {
  const PredDesc& d = desc[p];
  PredView v;
  v.keys = keys + d.row_base;
  v.ptr = ptr + d.ptr_base;
  v.nbr = nbr + d.nbr_base;
  v.src = src ? src + d.nbr_base : nullptr;
  v.dense = d.dense_base >= 0 ? dense + d.dense_base : nullptr;
  v.dir = d.dir_base >= 0 ? dir + d.dir_base : nullptr;
  v.hub_keys = d.hub_n ? hub_keys + d.hub_base : nullptr;
  v.hub_bm = d.hub_n ? hub_bm + d.hub_base * hub_words : nullptr;
  v.hub_words = hub_words;
  v.nr = (int32_t)d.nr;
  v.nnz = (int32_t)d.nnz;
  v.dir_shift = d.dir_shift;
  v.hub_n = d.hub_n;
  v.hub_min = hub_min;
  v.pad = 0;
  return v;
}

const uint32_t* Orientation::row_bitmap(int32_t p, int32_t v) const {
  const PredDesc& d = desc[p];
  if (!d.hub_n) return nullptr;
  const int32_t* a = hub_keys_host.data() + d.hub_base;
  const int32_t* it = std::lower_bound(a, a + d.hub_n, v);
  if (it == a + d.hub_n || *it != v) return nullptr;
  return hub_bm + (d.hub_base + (it - a)) * hub_words;
}

}  // namespace gsmat

using namespace gsmat;

void* gsmat_store::dalloc(size_t bytes, hipStream_t s, bool index) {
  bytes = std::max<size_t>(bytes, 4);
  void* p = mem->alloc(bytes, s);
  if (!p) throw OomFail{bytes};
  if (index) {
    index_allocs.push_back({p, bytes});
    device_bytes += (int64_t)bytes;
  }
  return p;
}

void gsmat_store::dfree_index(hipStream_t s) {
  for (auto& a : index_allocs) mem->free(a.p, a.bytes, s);
  index_allocs.clear();
  device_bytes = 0;
}

namespace {

void build_hubs(gsmat_store* st, Orientation& ori, hipStream_t s);

// Builds one orientation from sorted distinct keys (p << 2vb | row << vb | member).
void build_orientation(gsmat_store* st, const uint64_t* keys, int64_t U, Orientation& ori,
                       bool with_src, int dense_div, hipStream_t s) {
  DeviceMem* mem = st->mem.get();
  const int32_t P = st->P;
  const int64_t nt = ceil_div(std::max<int64_t>(U, 1), kTile);
  // rows: first entry of every (p, row)
  int64_t R = 0;
  Tmp<int64_t> row_pos(mem, U, s);
  {
    Tmp<uint8_t> flags(mem, U, s);
    Tmp<int64_t> ts(mem, nt + 1, s);
    if (U > 0) {
      launch_flag_row_heads(keys, U, st->vb, flags.p, ts.p, s);
      launch_scan_tile_sums(ts.p, nt, ts.p + nt, s, nullptr);
      R = read_i64(ts.p + nt, s);
      launch_compact_index(flags.p, U, ts.p, row_pos.p, s);
    }
  }
  // first entry and first row of every predicate
  std::vector<int64_t> pfe(P), pfr(P);
  {
    Tmp<int64_t> d_pfe(mem, P, s), d_pfr(mem, P, s);
    launch_fill_i64(d_pfe.p, P, -1, s);
    launch_fill_i64(d_pfr.p, P, -1, s);
    if (R > 0) launch_pred_heads(keys, row_pos.p, R, st->vb, d_pfe.p, d_pfr.p, s);
    GS_HIP(hipMemcpyAsync(pfe.data(), d_pfe.p, sizeof(int64_t) * P, hipMemcpyDeviceToHost, s));
    GS_HIP(hipMemcpyAsync(pfr.data(), d_pfr.p, sizeof(int64_t) * P, hipMemcpyDeviceToHost, s));
    GS_HIP(hipStreamSynchronize(s));
  }
  ori.desc.assign(P, PredDesc{});
  ori.R = R;
  {
    // walk predicates in order; the next present predicate bounds this one
    int64_t next_e = U, next_r = R;
    for (int32_t p = P - 1; p >= 0; --p) {
      PredDesc& d = ori.desc[p];
      if (pfe[p] >= 0) {
        d.nbr_base = pfe[p];
        d.row_base = pfr[p];
        d.nnz = next_e - pfe[p];
        d.nr = next_r - pfr[p];
        next_e = pfe[p];
        next_r = pfr[p];
      } else {
        d.nbr_base = next_e;
        d.row_base = next_r;
        d.nnz = 0;
        d.nr = 0;
      }
      d.ptr_base = d.row_base + p;
      if (d.nnz >= INT32_MAX)
        throw StatusFail{GSMAT_EUNSUPPORTED, "a predicate has 2^31 or more pairs"};
    }
  }
  // dense row pointers for predicates with many non-empty rows; the others
  // get a bucket directory over the id range with about kDirKeys rows per
  // bucket, so a lookup searches a few adjacent keys instead of all of them
  int64_t dense_len = 0, dir_len = 0;
  const int64_t V = st->V;
  for (int32_t p = 0; p < P; ++p) {
    PredDesc& d = ori.desc[p];
    if (d.nr > 0 && d.nr * (int64_t)dense_div >= V) {
      d.dense_base = dense_len;
      dense_len += V + 1;
    } else if (d.nr > kDirKeys && V > 1) {
      // largest bucket width 2^s with V / 2^s >= nr / kDirKeys buckets
      int s = 0;
      while (s < 30 && ((V - 1) >> (s + 1)) + 1 >= d.nr / kDirKeys) ++s;
      d.dir_shift = s;
      d.dir_base = dir_len;
      dir_len += ((V - 1) >> s) + 2;
    }
  }
  ori.nbr = (int32_t*)st->dalloc(sizeof(int32_t) * (size_t)U, s, true);
  ori.src = with_src ? (int32_t*)st->dalloc(sizeof(int32_t) * (size_t)U, s, true) : nullptr;
  ori.keys = (int32_t*)st->dalloc(sizeof(int32_t) * (size_t)R, s, true);
  ori.ptr = (int32_t*)st->dalloc(sizeof(int32_t) * (size_t)(R + P), s, true);
  ori.dense = dense_len ? (int32_t*)st->dalloc(sizeof(int32_t) * (size_t)dense_len, s, true) : nullptr;
  ori.dense_len = dense_len;
  ori.dir = dir_len ? (int32_t*)st->dalloc(sizeof(int32_t) * (size_t)dir_len, s, true) : nullptr;
  ori.dir_len = dir_len;
  ori.d_desc = (PredDesc*)st->dalloc(sizeof(PredDesc) * (size_t)P, s, true);
  GS_HIP(hipMemcpyAsync(ori.d_desc, ori.desc.data(), sizeof(PredDesc) * P, hipMemcpyHostToDevice, s));
  if (U > 0) {
    Tmp<int64_t> d_pfe(mem, P, s);
    GS_HIP(hipMemcpyAsync(d_pfe.p, pfe.data(), sizeof(int64_t) * P, hipMemcpyHostToDevice, s));
    launch_fill_rows(keys, row_pos.p, R, st->vb, d_pfe.p, ori.keys, ori.ptr, s);
    launch_split_members(keys, U, st->vb, ori.nbr, ori.src, s);
    GS_HIP(hipStreamSynchronize(s));  // d_pfe is a host-copied source
  }
  launch_ptr_sentinels(ori.d_desc, P, ori.ptr, s);
  for (int32_t p = 0; p < P; ++p) {
    const PredDesc& d = ori.desc[p];
    if (d.dense_base >= 0) launch_dense_ptr(ori.view(p), st->V, ori.dense + d.dense_base, s);
    if (d.dir_base >= 0) {
      // the view without its directory: the directory is built from the keys
      PredView pv = ori.view(p);
      pv.dir = nullptr;
      launch_row_dir(pv, d.dir_shift, ((V - 1) >> d.dir_shift) + 1, ori.dir + d.dir_base, s);
    }
  }
  GS_HIP(hipStreamSynchronize(s));
  build_hubs(st, ori, s);
}

// Bitmaps of the longest rows (at least hub_min_len members), longest first
// while they fit in hub_max_bytes: a membership test on such a row reads one
// bit instead of searching the row.
void build_hubs(gsmat_store* st, Orientation& ori, hipStream_t s) {
  const int32_t P = st->P;
  const int64_t V = st->V;
  if (st->hub_min_len <= 0 || st->hub_max_bytes <= 0 || V <= 0) return;
  const int64_t words = (V + 31) / 32;
  const int64_t bm_bytes = 4 * words;
  const int64_t max_hubs = st->hub_max_bytes / bm_bytes;
  if (max_hubs <= 0) return;
  const int32_t min_len = (int32_t)std::min<int64_t>(st->hub_min_len, INT32_MAX);
  struct Cand {
    int32_t p, row, len;
  };
  std::vector<Cand> cand;
  DeviceMem* mem = st->mem.get();
  for (int32_t p = 0; p < P; ++p) {
    const PredDesc& d = ori.desc[p];
    if (d.nnz < min_len) continue;
    const int32_t cap = (int32_t)std::min<int64_t>(d.nnz / min_len + 1, d.nr);
    Tmp<int32_t> out(mem, 2 * (int64_t)cap + 1, s);
    GS_HIP(hipMemsetAsync(out.p + 2 * cap, 0, sizeof(int32_t), s));
    launch_long_rows(ori.view(p), min_len, out.p, out.p + 2 * cap, cap, s);
    std::vector<int32_t> h(2 * (size_t)cap + 1);
    GS_HIP(hipMemcpyAsync(h.data(), out.p, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, s));
    GS_HIP(hipStreamSynchronize(s));
    const int32_t n = std::min(h[2 * cap], cap);
    for (int32_t i = 0; i < n; ++i) cand.push_back(Cand{p, h[2 * i], h[2 * i + 1]});
  }
  if (cand.empty()) return;
  std::sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
    return a.len != b.len ? a.len > b.len : (a.p != b.p ? a.p < b.p : a.row < b.row);
  });
  if ((int64_t)cand.size() > max_hubs) cand.resize((size_t)max_hubs);
  std::sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
    return a.p != b.p ? a.p < b.p : a.row < b.row;
  });
  const int64_t H = (int64_t)cand.size();
  ori.hub_words = words;
  ori.hub_min = min_len;
  ori.hub_keys_host.resize(H);
  for (int64_t i = 0; i < H; ++i) {
    ori.hub_keys_host[i] = cand[i].row;
    PredDesc& d = ori.desc[cand[i].p];
    if (d.hub_n == 0) d.hub_base = i;
    ++d.hub_n;
  }
  ori.hub_keys = (int32_t*)st->dalloc(sizeof(int32_t) * H, s, true);
  ori.hub_bm = (uint32_t*)st->dalloc(sizeof(uint32_t) * H * words, s, true);
  GS_HIP(hipMemcpyAsync(ori.hub_keys, ori.hub_keys_host.data(), sizeof(int32_t) * H,
                        hipMemcpyHostToDevice, s));
  GS_HIP(hipMemsetAsync(ori.hub_bm, 0, sizeof(uint32_t) * H * words, s));
  // each bitmap from its row's members (found by a device lookup of the row)
  for (int64_t i = 0; i < H; ++i) {
    const PredView pv = ori.view(cand[i].p);
    launch_row_bitmap(pv, cand[i].row, cand[i].len, ori.hub_bm + i * words, s);
  }
  GS_HIP(hipMemcpyAsync(ori.d_desc, ori.desc.data(), sizeof(PredDesc) * P, hipMemcpyHostToDevice, s));
  GS_HIP(hipStreamSynchronize(s));
}

// Sort + deduplicate one key array in place; returns the distinct count.
int64_t sort_unique(gsmat_store* st, uint64_t* keys, int64_t n, uint64_t* tmp, hipStream_t s) {
  DeviceMem* mem = st->mem.get();
  const int nbits = st->pb + 2 * st->vb;
  radix_sort_u64(keys, tmp, n, nbits, *mem, s);
  const int64_t nt = ceil_div(std::max<int64_t>(n, 1), kTile);
  Tmp<uint8_t> flags(mem, n, s);
  Tmp<int64_t> ts(mem, nt + 1, s);
  launch_flag_unique(keys, n, flags.p, ts.p, s);
  launch_scan_tile_sums(ts.p, nt, ts.p + nt, s, nullptr);
  const int64_t U = read_i64(ts.p + nt, s);
  launch_compact_u64(keys, flags.p, n, ts.p, tmp, s);
  GS_HIP(hipMemcpyAsync(keys, tmp, sizeof(uint64_t) * (size_t)U, hipMemcpyDeviceToDevice, s));
  GS_HIP(hipStreamSynchronize(s));
  return U;
}

}  // namespace

extern "C" gsmat_status gsmat_load_triples(const int32_t* s, const int32_t* p, const int32_t* o,
                                           int64_t n, int32_t n_vertices, int32_t n_predicates,
                                           const gsmat_allocator* alloc, void* stream,
                                           gsmat_store** out) {
  return guarded([&]() -> gsmat_status {
    if (!out) throw StatusFail{GSMAT_EINVAL, "out is NULL"};
    *out = nullptr;
    if (n < 0) throw StatusFail{GSMAT_EINVAL, "n < 0"};
    // the device radix sort ranks keys with 32-bit bucket positions
    if (n >= ((int64_t)1 << 32))
      throw StatusFail{GSMAT_EUNSUPPORTED, "2^32 or more input triples"};
    if (n > 0 && (!s || !p || !o)) throw StatusFail{GSMAT_EINVAL, "NULL triple array"};
    if (n_vertices < 1 || n_predicates < 1)
      throw StatusFail{GSMAT_EINVAL, "n_vertices and n_predicates must be >= 1"};
    if (alloc && (!alloc->alloc || !alloc->free))
      throw StatusFail{GSMAT_EINVAL, "allocator needs alloc and free"};
    const int vb = bits_for((int64_t)n_vertices - 1), pb = bits_for((int64_t)n_predicates - 1);
    if (pb + 2 * vb > 64)
      throw StatusFail{GSMAT_EUNSUPPORTED, "vertex and predicate ids do not pack into 64 bits"};
    for (int64_t i = 0; i < n; ++i) {
      if ((uint32_t)s[i] >= (uint32_t)n_vertices || (uint32_t)o[i] >= (uint32_t)n_vertices)
        throw StatusFail{GSMAT_EINVAL, "vertex id out of range at triple " + std::to_string(i)};
      if ((uint32_t)p[i] >= (uint32_t)n_predicates)
        throw StatusFail{GSMAT_EINVAL, "predicate id out of range at triple " + std::to_string(i)};
    }
    std::unique_ptr<gsmat_store> st(new gsmat_store);
    st->mem.reset(new DeviceMem(alloc));
    st->V = n_vertices;
    st->P = n_predicates;
    st->vb = vb;
    st->pb = pb;
    st->n_in = n;
    hipStream_t hs = (hipStream_t)stream;
    const size_t bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1);
    st->d_s = (int32_t*)st->mem->alloc(bytes, hs);
    st->d_p = st->d_s ? (int32_t*)st->mem->alloc(bytes, hs) : nullptr;
    st->d_o = st->d_p ? (int32_t*)st->mem->alloc(bytes, hs) : nullptr;
    if (!st->d_o) {
      if (st->d_p) st->mem->free(st->d_p, bytes, hs);
      if (st->d_s) st->mem->free(st->d_s, bytes, hs);
      st->d_s = st->d_p = nullptr;
      throw OomFail{bytes};
    }
    if (n > 0) {
      GS_HIP(hipMemcpyAsync(st->d_s, s, sizeof(int32_t) * n, hipMemcpyHostToDevice, hs));
      GS_HIP(hipMemcpyAsync(st->d_p, p, sizeof(int32_t) * n, hipMemcpyHostToDevice, hs));
      GS_HIP(hipMemcpyAsync(st->d_o, o, sizeof(int32_t) * n, hipMemcpyHostToDevice, hs));
    }
    GS_HIP(hipStreamSynchronize(hs));
    *out = st.release();
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_set_hub_options(gsmat_store* st, int64_t min_len,
                                              int64_t max_bytes) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (st->built) throw StatusFail{GSMAT_ESTATE, "index already built"};
    st->hub_min_len = min_len;
    st->hub_max_bytes = max_bytes;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_build_index(gsmat_store* st, int32_t dense_div, void* stream) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (st->built) return GSMAT_OK;
    if (dense_div <= 0) dense_div = 32;
    hipStream_t s = (hipStream_t)stream;
    DeviceMem* mem = st->mem.get();
    const int64_t n = st->n_in;
    const size_t raw = sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1);
    {
      Tmp<uint64_t> ks(mem, n, s), ko(mem, n, s);
      if (n > 0) launch_pack_keys(st->d_s, st->d_p, st->d_o, n, st->vb, ks.p, ko.p, s);
      Tmp<uint64_t> tmp(mem, n, s);
      const int64_t U = n > 0 ? sort_unique(st, ks.p, n, tmp.p, s) : 0;
      build_orientation(st, ks.p, U, st->out, true, dense_div, s);
      ks.release();
      const int64_t U2 = n > 0 ? sort_unique(st, ko.p, n, tmp.p, s) : 0;
      if (U2 != U) throw StatusFail{GSMAT_EHIP, "orientations disagree on the distinct count"};
      build_orientation(st, ko.p, U2, st->in, false, dense_div, s);
      st->T = U;
    }
    mem->free(st->d_s, raw, s);
    mem->free(st->d_p, raw, s);
    mem->free(st->d_o, raw, s);
    st->d_s = st->d_p = st->d_o = nullptr;
    GS_HIP(hipStreamSynchronize(s));
    static std::atomic<uint64_t> next_uid{1};
    st->uid = next_uid.fetch_add(1);
    st->built = true;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_store_stats(const gsmat_store* st, int64_t* n_triples,
                                          int32_t* n_predicates, int64_t* device_bytes) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    if (n_triples) *n_triples = st->T;
    if (n_predicates) *n_predicates = st->P;
    if (device_bytes) *device_bytes = st->device_bytes;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_pred_stats(const gsmat_store* st, int32_t pred, int64_t* nnz,
                                         int64_t* n_rows, int64_t* n_cols) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    if (pred < 0 || pred >= st->P) throw StatusFail{GSMAT_EINVAL, "predicate out of range"};
    if (nnz) *nnz = st->out.desc[pred].nnz;
    if (n_rows) *n_rows = st->out.desc[pred].nr;
    if (n_cols) *n_cols = st->in.desc[pred].nr;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_export_matrix(const gsmat_store* st, int32_t pred, int32_t orient,
                                            int32_t* keys, int32_t* ptr, int32_t* nbr,
                                            void* stream) {
  return guarded([&]() -> gsmat_status {
    if (!st) throw StatusFail{GSMAT_EINVAL, "store is NULL"};
    if (!st->built) throw StatusFail{GSMAT_ESTATE, "index not built"};
    if (pred < 0 || pred >= st->P) throw StatusFail{GSMAT_EINVAL, "predicate out of range"};
    if (orient != 0 && orient != 1) throw StatusFail{GSMAT_EINVAL, "orient must be 0 or 1"};
    if (!keys || !ptr || !nbr) throw StatusFail{GSMAT_EINVAL, "NULL output buffer"};
    const Orientation& ori = orient == 0 ? st->out : st->in;
    const PredDesc& d = ori.desc[pred];
    hipStream_t s = (hipStream_t)stream;
    if (d.nr > 0)
      GS_HIP(hipMemcpyAsync(keys, ori.keys + d.row_base, sizeof(int32_t) * d.nr, hipMemcpyDeviceToHost, s));
    GS_HIP(hipMemcpyAsync(ptr, ori.ptr + d.ptr_base, sizeof(int32_t) * (d.nr + 1), hipMemcpyDeviceToHost, s));
    if (d.nnz > 0)
      GS_HIP(hipMemcpyAsync(nbr, ori.nbr + d.nbr_base, sizeof(int32_t) * d.nnz, hipMemcpyDeviceToHost, s));
    GS_HIP(hipStreamSynchronize(s));
    return GSMAT_OK;
  });
}

extern "C" void gsmat_store_free(gsmat_store* st) {
  if (!st) return;
  try {
    hipStream_t s = nullptr;
    (void)hipDeviceSynchronize();
    st->dfree_index(s);
    const size_t raw = sizeof(int32_t) * (size_t)std::max<int64_t>(st->n_in, 1);
    if (st->d_s) st->mem->free(st->d_s, raw, s);
    if (st->d_p) st->mem->free(st->d_p, raw, s);
    if (st->d_o) st->mem->free(st->d_o, raw, s);
    (void)hipDeviceSynchronize();
  } catch (...) {
  }
  delete st;
}
