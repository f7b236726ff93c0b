// Internal declarations shared by the host-side modules and the kernels of the
// gsmat library (sparse-matrix BGP join, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "gsmat.h"
#include "plan.hpp"

namespace gsmat {

constexpr int kBlock = 256;              // threads per workgroup (4 wave64)
constexpr int kItems = 8;                // items per thread in tiled kernels
constexpr int kTile = kBlock * kItems;   // items per workgroup tile

// Column pointers of a binding table (columnar int32, one array per column).
struct ColSet {
  const int32_t* c[kMaxCols];
};
struct OutSet {
  int32_t* c[kMaxCols];
};

// One predicate's compressed matrix in one orientation, as device pointers
// already offset to the predicate's range.
//   keys[nr]      non-empty row ids, ascending
//   ptr[nr + 1]   row offsets into nbr (local to the predicate)
//   nbr[nnz]      members, ascending within a row
//   src[nnz]      row id of each member (row-compressed orientation only)
//   dense[V + 1]  optional: ptr value of the first row >= v, for every vertex v
//   dir[nb + 1]   optional (predicates without dense): index of the first row
//                 whose id is >= b << dir_shift, for every bucket b of ids
//   hub_keys[hub_n]  optional: ids of the rows (of at least hub_min members)
//                    that also have a bitmap, ascending; row hub_keys[h] has
//                    bit u of hub_bm[h * hub_words ...] set iff u is a member
struct PredView {
  const int32_t* keys;
  const int32_t* ptr;
  const int32_t* nbr;
  const int32_t* src;
  const int32_t* dense;
  const int32_t* dir;
  const int32_t* hub_keys;
  const uint32_t* hub_bm;
  int64_t hub_words;
  int32_t nr;
  int32_t nnz;
  int32_t dir_shift;
  int32_t hub_n;
  int32_t hub_min;
  int32_t pad;
};

// Global arrays of one orientation (the per-predicate views are offsets into
// them, given by the orientation's PredDesc table).
struct OriPtrs {
  const int32_t* keys;
  const int32_t* ptr;
  const int32_t* nbr;
  const int32_t* dense;
  const int32_t* dir;
  const int32_t* hub_keys;
  const uint32_t* hub_bm;
  int64_t hub_words;
  int32_t hub_min;
};

// Host record of one predicate in one orientation (offsets into the global
// orientation arrays).
struct PredDesc {
  int64_t nbr_base = 0;    // first member
  int64_t row_base = 0;    // first row id in keys
  int64_t ptr_base = 0;    // first row offset in ptr (= row_base + predicate index)
  int64_t dense_base = -1; // first entry in dense, -1 if none
  int64_t nnz = 0;
  int64_t nr = 0;
  int64_t dir_base = -1;   // first entry in dir, -1 if none
  int32_t dir_shift = 0;   // bucket b holds ids [b << dir_shift, (b + 1) << dir_shift)
  int32_t hub_n = 0;       // rows with a bitmap
  int64_t hub_base = 0;    // first of them in the hub key list and the bitmap pool
};

// A list taking part in a star-centre intersection: either a predicate's
// non-empty row ids (membership by row lookup) or an explicit sorted segment.
struct ListRef {
  PredView pv;         // used when is_keys
  const int32_t* seg;  // used when !is_keys
  const uint32_t* bm;  // !is_keys: the segment's row bitmap, if it has one
  int64_t len;
  int32_t is_keys;
  int32_t pad;
};
struct ListSet {
  ListRef l[kMaxLists];
  int32_t n;
};

// A membership probe description for the filter step: subject value from a
// column (s_col) or constant (s_const), likewise for the object.
struct ProbeArgs {
  const int32_t* s_col;
  const int32_t* o_col;
  int32_t s_const;
  int32_t o_const;
};

// Candidate expansions whose fan-out is estimated on a strided sample of the
// bound column (one workgroup per candidate).
struct SampleSet {
  const int32_t* col[kMaxPats];
  PredView pv[kMaxPats];
  int64_t n;
  int32_t ncand;
};

struct LookupReq {
  int32_t orient;  // 0 by subject, 1 by object
  int32_t pred;
  int32_t v;       // the row (vertex) to look up
  int32_t member;  // >= 0: also test membership of this value in the row
};
constexpr int kMaxLookups = 32;
struct LookupBatch {
  LookupReq req[kMaxLookups];
  int32_t n;
};
struct LookupRes {
  int32_t start;   // local offset of the row (0 if absent)
  int32_t len;     // row length (0 if absent)
  int32_t found;   // membership result (0/1) when requested
  int32_t pad;
};

constexpr int kSampleBlocks = 8;  // workgroups per fan-out sample of one candidate
constexpr int64_t kDirKeys = 4;   // target rows per bucket of a row directory

// -------------------------------------------------------------------------
// device memory
// -------------------------------------------------------------------------
class DeviceMem {
 public:
  explicit DeviceMem(const gsmat_allocator* a);
  ~DeviceMem();
  void* alloc(size_t bytes, hipStream_t s);  // nullptr on failure
  void free(void* p, size_t bytes, hipStream_t s);
  int device() const { return dev_; }

 private:
  gsmat_allocator user_{};
  bool has_user_ = false;
  void* cache_ = nullptr;  // the device's block cache
  int dev_ = 0;
};

// -------------------------------------------------------------------------
// errors
// -------------------------------------------------------------------------
void set_error(const std::string& msg);
struct HipFail {
  hipError_t e;
  std::string where;
};
#define GS_HIP(expr)                                                                      \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess) throw ::gsmat::HipFail{_e, std::string(#expr) + " @" + __FILE__ + \
                                                        ":" + std::to_string(__LINE__)};   \
  } while (0)
struct OomFail {
  size_t bytes;
};
struct StatusFail {
  gsmat_status st;
  std::string msg;
};

// Runs f (returning gsmat_status) and maps every failure to a status code.
template <class F>
gsmat_status guarded(F&& f) {
  try {
    return f();
  } catch (const HipFail& e) {
    set_error(std::string("HIP error: ") + hipGetErrorString(e.e) + " in " + e.where);
    return GSMAT_EHIP;
  } catch (const OomFail& e) {
    set_error("device allocation of " + std::to_string(e.bytes) + " bytes failed");
    return GSMAT_ENOMEM;
  } catch (const StatusFail& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GSMAT_ENOMEM;
  } catch (...) {
    set_error("unexpected internal error");
    return GSMAT_EHIP;
  }
}

// -------------------------------------------------------------------------
// profiling of kernel classes
// -------------------------------------------------------------------------
void prof_begin(hipStream_t s, int cls);
void host_sync(hipStream_t s);  // hipStreamSynchronize, timed for instrumentation
void host_event_sync(hipEvent_t e);  // hipEventSynchronize, timed likewise
void prof_end(hipStream_t s, int cls, double bytes);
bool prof_on(int cls);
// adds algorithmic bytes to a class whose launches were sized on the device
// (their byte counts are known only after the stream has synchronised)
void prof_add_bytes(int cls, double bytes);

// -------------------------------------------------------------------------
// kernel launchers (kernels.hip)
// -------------------------------------------------------------------------
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// prefix sums
// scan of tile sums in place; the grand total goes to total[0] and, if given,
// to host_total[0] (pinned host memory, valid after the stream synchronizes)
void launch_scan_tile_sums(int64_t* tile_sum, int64_t nt, int64_t* total, hipStream_t s,
                           int64_t* host_total);
// two tile-sum arrays [nt + 1] scanned together (totals at [nt])
void launch_scan_tile_sums2(int64_t* ts, int64_t* ts2, int64_t nt, hipStream_t s);
void launch_scan_add_i32(const int32_t* N, int64_t n, const int64_t* tile_off, int64_t* P,
                         hipStream_t s);
void launch_tile_reduce_u32(const uint32_t* x, int64_t n, int64_t* tile_sum, hipStream_t s);
void launch_scan_add_u32(const uint32_t* x, int64_t n, const int64_t* tile_off, uint32_t* out,
                         hipStream_t s);

// radix sort of 64-bit keys on their low nbits (LSD, 8-bit digits); result in keys
void radix_sort_u64(uint64_t* keys, uint64_t* tmp, int64_t n, int nbits, DeviceMem& mem,
                    hipStream_t s);

// build
void launch_pack_keys(const int32_t* s, const int32_t* p, const int32_t* o, int64_t n, int vb,
                      uint64_t* k_by_s, uint64_t* k_by_o, hipStream_t st);
void launch_flag_unique(const uint64_t* k, int64_t n, uint8_t* flags, int64_t* tile_sum,
                        hipStream_t s);
void launch_flag_row_heads(const uint64_t* k, int64_t n, int vb, uint8_t* flags,
                           int64_t* tile_sum, hipStream_t s);
void launch_compact_u64(const uint64_t* in, const uint8_t* flags, int64_t n,
                        const int64_t* tile_off, uint64_t* out, hipStream_t s);
void launch_compact_index(const uint8_t* flags, int64_t n, const int64_t* tile_off,
                          int64_t* out_idx, hipStream_t s);
void launch_split_members(const uint64_t* k, int64_t n, int vb, int32_t* nbr, int32_t* src,
                          hipStream_t s);
void launch_pred_heads(const uint64_t* k, const int64_t* row_pos, int64_t R, int vb,
                       int64_t* pred_first_entry, int64_t* pred_first_row, hipStream_t s);
void launch_fill_rows(const uint64_t* k, const int64_t* row_pos, int64_t R, int vb,
                      const int64_t* pred_first_entry, int32_t* keys, int32_t* ptr,
                      hipStream_t s);
void launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s);
void launch_dense_ptr(PredView pv, int64_t V, int32_t* dense, hipStream_t s);
// dir[b] = first row index with id >= b << shift, for b in [0, nb]
void launch_row_dir(PredView pv, int32_t shift, int64_t nb, int32_t* dir, hipStream_t s);
// appends (row id, length) of every row with at least min_len members to
// out[2 * i], out[2 * i + 1] for i < *count (count must start at 0)
void launch_long_rows(PredView pv, int32_t min_len, int32_t* out, int32_t* count, int32_t cap,
                      hipStream_t s);
// sets the bits of the members of row v in the bitmap bm (zeroed before)
void launch_row_bitmap(PredView pv, int32_t v, int64_t len, uint32_t* bm, hipStream_t s);
void launch_ptr_sentinels(const PredDesc* d, int32_t P, int32_t* ptr, hipStream_t s);

// lookups (planner statistics, constant scans)
void launch_lookup(const LookupBatch& b, const PredDesc* desc_out, const PredDesc* desc_in,
                   OriPtrs out, OriPtrs in, LookupRes* res, hipStream_t s);

// join steps
void launch_count_expand(const int32_t* col, int64_t n, PredView pv, int32_t* N, int32_t* start,
                         int64_t* tile_sum, hipStream_t s);
void launch_flag_filter(ProbeArgs pa, int64_t n, PredView pv, uint8_t* flags, int64_t* tile_sum,
                        hipStream_t s);
void launch_flag_diag(const int32_t* a, const int32_t* b, int64_t n, uint8_t* flags,
                      int64_t* tile_sum, hipStream_t s);
void launch_flag_intersect(const int32_t* driver, int64_t n, ListSet ls, uint8_t* flags,
                           int64_t* tile_sum, hipStream_t s);
void launch_compact_cols(ColSet in, int k, const uint8_t* flags, int64_t n,
                         const int64_t* tile_off, OutSet out, hipStream_t s);
void launch_mp_partition(const int64_t* P, int64_t n, int64_t J0, int64_t J1, int64_t* split,
                         int64_t ntiles, hipStream_t s);
void launch_write_expand(ColSet in, int k, const int64_t* P, const int32_t* start, int64_t n,
                         const int32_t* nbr, int64_t J0, int64_t J1, const int64_t* split,
                         int64_t ntiles, OutSet out, double alg_bytes, hipStream_t s);
void launch_cartesian(ColSet a, int ka, int64_t na, ColSet b, int kb, int64_t nb, int64_t J0,
                      int64_t J1, OutSet out, hipStream_t s);
// writes kSampleBlocks partial sums per candidate to part[cand * kSampleBlocks + b]
void launch_sample_fanout(const SampleSet& ss, int64_t* part, hipStream_t s);
void launch_pack_rows(ColSet cols, int k, int64_t row0, int64_t rows, int32_t* out,
                      hipStream_t s);

}  // namespace gsmat
