// C-ABI glue: errors, device memory pool, host-only planning entry points and
// kernel-class profiling.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace gsmat {

namespace {
thread_local std::string g_err;
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;
}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

DeviceMem::DeviceMem(const gsmat_allocator* a) {
  if (a) {
    user_ = *a;
    has_user_ = true;
  }
}

DeviceMem::~DeviceMem() = default;

void* DeviceMem::alloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 4;
  if (has_user_) return user_.alloc(bytes, (void*)s, user_.ctx);
  if (!pool_) {
    GS_HIP(hipGetDevice(&dev_));
    std::lock_guard<std::mutex> g(g_pool_mu);
    auto it = g_pools.find(dev_);
    if (it != g_pools.end()) {
      pool_ = it->second;
    } else {
      hipMemPoolProps props;
      std::memset(&props, 0, sizeof(props));
      props.allocType = hipMemAllocationTypePinned;
      props.handleTypes = hipMemHandleTypeNone;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = dev_;
      GS_HIP(hipMemPoolCreate(&pool_, &props));
      uint64_t thr = UINT64_MAX;
      GS_HIP(hipMemPoolSetAttribute(pool_, hipMemPoolAttrReleaseThreshold, &thr));
      g_pools[dev_] = pool_;
    }
  }
  void* p = nullptr;
  if (hipMallocFromPoolAsync(&p, bytes, pool_, s) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void DeviceMem::free(void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  if (has_user_) {
    user_.free(p, bytes, (void*)s, user_.ctx);
    return;
  }
  (void)hipFreeAsync(p, s);
}

// ---------------------------------------------------------------- profiling
namespace {
struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_open;  // begin events awaiting their end, per call order
int64_t g_launch[GSMAT_K_NCLASS];
double g_ms[GSMAT_K_NCLASS];
double g_bytes[GSMAT_K_NCLASS];

void prof_drain_locked() {
  for (ProfRec& r : g_prof_pending) {
    float ms = 0;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g_launch[r.cls] += 1;
      g_ms[r.cls] += ms;
      g_bytes[r.cls] += r.bytes;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof_pending.clear();
}
}  // namespace

bool prof_on() { return g_prof_on; }

void prof_begin(hipStream_t s, int cls) {
  (void)cls;
  hipEvent_t e;
  GS_HIP(hipEventCreate(&e));
  GS_HIP(hipEventRecord(e, s));
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_open.push_back(e);
}

void prof_end(hipStream_t s, int cls, double bytes) {
  hipEvent_t e;
  GS_HIP(hipEventCreate(&e));
  GS_HIP(hipEventRecord(e, s));
  std::lock_guard<std::mutex> g(g_prof_mu);
  hipEvent_t a = g_prof_open.back();
  g_prof_open.pop_back();
  g_prof_pending.push_back({cls, a, e, bytes});
  if (g_prof_pending.size() > 4096) prof_drain_locked();
}

}  // namespace gsmat

using namespace gsmat;

extern "C" const char* gsmat_last_error(void) { return g_err.c_str(); }

extern "C" gsmat_status gsmat_release_pools(void) {
  return guarded([&]() -> gsmat_status {
    std::lock_guard<std::mutex> g(g_pool_mu);
    if (g_pools.empty()) return GSMAT_OK;
    GS_HIP(hipDeviceSynchronize());
    for (auto& kv : g_pools) {
      (void)hipMemPoolTrimTo(kv.second, 0);
    }
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_plan_from_stats(const gsmat_pattern* pats, int32_t n_pats,
                                              int32_t mode, const int64_t* stat,
                                              gsmat_query_plan** out) {
  return guarded([&]() -> gsmat_status {
    if (!out) throw StatusFail{GSMAT_EINVAL, "out is NULL"};
    *out = nullptr;
    std::string err;
    int32_t nv = 0;
    gsmat_status rc = validate_patterns(pats, n_pats, &nv, &err);
    if (rc != GSMAT_OK) throw StatusFail{rc, err};
    if (!stat) throw StatusFail{GSMAT_EINVAL, "stat is NULL"};
    std::vector<TpStat> ts(n_pats);
    for (int i = 0; i < n_pats; ++i) {
      if (stat[i] < 0) throw StatusFail{GSMAT_EINVAL, "negative statistic"};
      ts[i].stat = ts[i].rows_s = ts[i].rows_o = stat[i];
    }
    std::unique_ptr<gsmat_query_plan> pl(new gsmat_query_plan);
    rc = build_plan(pats, n_pats, mode, ts, pl.get(), &err);
    if (rc != GSMAT_OK) throw StatusFail{rc, err};
    *out = pl.release();
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_plan_info(const gsmat_query_plan* pl, int32_t* n_steps, int32_t* n_vars,
                                        gsmat_step_info* steps, int32_t cap) {
  return guarded([&]() -> gsmat_status {
    if (!pl) throw StatusFail{GSMAT_EINVAL, "plan is NULL"};
    if (n_steps) *n_steps = (int32_t)pl->steps.size();
    if (n_vars) *n_vars = pl->n_vars;
    if (steps)
      for (int32_t i = 0; i < cap && i < (int32_t)pl->steps.size(); ++i) steps[i] = pl->steps[i];
    return GSMAT_OK;
  });
}

extern "C" void gsmat_plan_free(gsmat_query_plan* pl) { delete pl; }

extern "C" void gsmat_prof_enable(int32_t on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  prof_drain_locked();
  for (int i = 0; i < GSMAT_K_NCLASS; ++i) {
    g_launch[i] = 0;
    g_ms[i] = 0;
    g_bytes[i] = 0;
  }
  g_prof_on = on != 0;
}

extern "C" gsmat_status gsmat_prof_read(int64_t* launches, double* ms, double* bytes) {
  return guarded([&]() -> gsmat_status {
    std::lock_guard<std::mutex> g(g_prof_mu);
    prof_drain_locked();
    for (int i = 0; i < GSMAT_K_NCLASS; ++i) {
      if (launches) launches[i] = g_launch[i];
      if (ms) ms[i] = g_ms[i];
      if (bytes) bytes[i] = g_bytes[i];
    }
    return GSMAT_OK;
  });
}
