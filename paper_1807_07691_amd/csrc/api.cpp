// C-ABI glue: errors, device memory pool, host-only planning entry points and
// kernel-class profiling.
#include <hip/hip_runtime.h>

#include <chrono>
#include <algorithm>
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
}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

namespace {
// host-side instrumentation: time spent in device allocation calls and in
// waits for the stream (the join's per-step size read-backs)
std::mutex g_host_mu;
double g_alloc_ms = 0, g_free_ms = 0, g_sync_ms = 0;
int64_t g_allocs = 0, g_syncs = 0;
inline double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
struct HostTimer {
  double* acc;
  int64_t* cnt;
  double t0 = now_ms();
  HostTimer(double* a, int64_t* c) : acc(a), cnt(c) {}
  ~HostTimer() {
    const double dt = now_ms() - t0;
    std::lock_guard<std::mutex> g(g_host_mu);
    *acc += dt;
    if (cnt) ++*cnt;
  }
};
}  // namespace

void host_sync(hipStream_t s) {
  HostTimer t(&g_sync_ms, &g_syncs);
  GS_HIP(hipStreamSynchronize(s));
}

void host_event_sync(hipEvent_t e) {
  HostTimer t(&g_sync_ms, &g_syncs);
  GS_HIP(hipEventSynchronize(e));
}

// Device memory: a caching block allocator per device.  Blocks come from
// hipMalloc and are never returned to the driver while the process runs
// (unless an allocation fails, or gsmat_release_pools is called): a freed
// block is kept with the stream it was last used on and an event recorded on
// that stream, and a later request of a similar size reuses it -- at once on
// the same stream (stream order makes it safe), after a device-side wait on
// the event otherwise.  Requests up to 1 MiB round to a power of two; larger
// ones to 2 MiB and reuse a block at most 1/8 (or 64 MiB) larger.
namespace {
struct Cached {
  void* p;
  size_t size;
  hipStream_t stream;
  hipEvent_t ev;
};

class BlockCache {
 public:
  explicit BlockCache(int dev) : dev_(dev) {}

  static size_t round(size_t b) {
    if (b <= (1u << 20)) {
      size_t r = 512;
      while (r < b) r <<= 1;
      return r;
    }
    const size_t g = (size_t)2 << 20;
    return (b + g - 1) / g * g;
  }

  void* alloc(size_t bytes, hipStream_t s) {
    const size_t want = round(bytes);
    const size_t slack = want <= (1u << 20) ? 0 : std::max<size_t>(want / 8, (size_t)64 << 20);
    {
      std::lock_guard<std::mutex> g(mu_);
      auto it = free_.lower_bound(want);
      // prefer a block last used on this stream among the first few fits
      auto pick = free_.end();
      int seen = 0;
      for (auto j = it; j != free_.end() && j->first <= want + slack && seen < 8; ++j, ++seen) {
        if (j->second.stream == s) {
          pick = j;
          break;
        }
        if (pick == free_.end()) pick = j;
      }
      if (pick != free_.end()) {
        Cached c = pick->second;
        free_.erase(pick);
        cached_ -= c.size;
        if (c.stream != s && c.ev) GS_HIP(hipStreamWaitEvent(s, c.ev, 0));
        if (c.ev) events_.push_back(c.ev);
        live_[c.p] = c.size;
        return c.p;
      }
    }
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      trim();
      if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    std::lock_guard<std::mutex> g(mu_);
    live_[p] = want;
    return p;
  }

  void free(void* p, hipStream_t s) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    const size_t size = it->second;
    live_.erase(it);
    hipEvent_t ev = nullptr;
    if (!events_.empty()) {
      ev = events_.back();
      events_.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      ev = nullptr;
    }
    if (ev && hipEventRecord(ev, s) != hipSuccess) {
      (void)hipEventDestroy(ev);
      ev = nullptr;
    }
    free_.insert({size, Cached{p, size, s, ev}});
    cached_ += size;
  }

  // Waits for the device and returns every cached block to the driver.
  void trim() {
    std::lock_guard<std::mutex> g(mu_);
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(dev_);
    (void)hipDeviceSynchronize();
    for (auto& kv : free_) {
      (void)hipFree(kv.second.p);
      if (kv.second.ev) events_.push_back(kv.second.ev);
    }
    free_.clear();
    cached_ = 0;
    (void)hipSetDevice(cur);
  }

 private:
  int dev_;
  std::mutex mu_;
  std::multimap<size_t, Cached> free_;
  std::map<void*, size_t> live_;
  std::vector<hipEvent_t> events_;
  size_t cached_ = 0;
};

std::map<int, BlockCache*> g_caches;  // one per device, kept until process end

BlockCache* cache_for(int dev) {
  std::lock_guard<std::mutex> g(g_pool_mu);
  auto it = g_caches.find(dev);
  if (it != g_caches.end()) return it->second;
  BlockCache* c = new BlockCache(dev);
  g_caches[dev] = c;
  return c;
}
}  // namespace

DeviceMem::DeviceMem(const gsmat_allocator* a) {
  if (a) {
    user_ = *a;
    has_user_ = true;
  }
}

DeviceMem::~DeviceMem() = default;

void* DeviceMem::alloc(size_t bytes, hipStream_t s) {
  HostTimer timer(&g_alloc_ms, &g_allocs);
  if (bytes == 0) bytes = 4;
  if (has_user_) return user_.alloc(bytes, (void*)s, user_.ctx);
  if (!cache_) {
    GS_HIP(hipGetDevice(&dev_));
    cache_ = cache_for(dev_);
  }
  return static_cast<BlockCache*>(cache_)->alloc(bytes, s);
}

void DeviceMem::free(void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  HostTimer timer(&g_free_ms, nullptr);
  if (has_user_) {
    user_.free(p, bytes, (void*)s, user_.ctx);
    return;
  }
  static_cast<BlockCache*>(cache_)->free(p, s);
}

// ---------------------------------------------------------------- profiling
namespace {
struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double bytes;
};
std::mutex g_prof_mu;
int32_t g_prof_mask = 0;
std::vector<hipEvent_t> g_free_events;
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
    g_free_events.push_back(r.a);
    g_free_events.push_back(r.b);
  }
  g_prof_pending.clear();
}
}  // namespace

bool prof_on(int cls) { return (g_prof_mask >> cls) & 1; }

namespace {
hipEvent_t take_event_locked() {
  if (!g_free_events.empty()) {
    hipEvent_t e = g_free_events.back();
    g_free_events.pop_back();
    return e;
  }
  hipEvent_t e;
  GS_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

void prof_begin(hipStream_t s, int cls) {
  (void)cls;
  std::lock_guard<std::mutex> g(g_prof_mu);
  hipEvent_t e = take_event_locked();
  GS_HIP(hipEventRecord(e, s));
  g_prof_open.push_back(e);
}

void prof_end(hipStream_t s, int cls, double bytes) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  hipEvent_t e = take_event_locked();
  GS_HIP(hipEventRecord(e, s));
  hipEvent_t a = g_prof_open.back();
  g_prof_open.pop_back();
  g_prof_pending.push_back({cls, a, e, bytes});
  if (g_prof_pending.size() > 4096) prof_drain_locked();
}

void prof_add_bytes(int cls, double bytes) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if ((g_prof_mask >> cls) & 1) g_bytes[cls] += bytes;
}

}  // namespace gsmat

using namespace gsmat;

extern "C" const char* gsmat_last_error(void) { return g_err.c_str(); }

extern "C" gsmat_status gsmat_release_pools(void) {
  return guarded([&]() -> gsmat_status {
    std::vector<BlockCache*> cs;
    {
      std::lock_guard<std::mutex> g(g_pool_mu);
      for (auto& kv : g_caches) cs.push_back(kv.second);
    }
    for (BlockCache* c : cs) c->trim();
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
    rc = build_plan(pats, n_pats, mode, ts.data(), pl.get(), &err);
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

extern "C" void gsmat_prof_enable(int32_t class_mask) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  prof_drain_locked();
  for (int i = 0; i < GSMAT_K_NCLASS; ++i) {
    g_launch[i] = 0;
    g_ms[i] = 0;
    g_bytes[i] = 0;
  }
  g_prof_mask = class_mask;
  std::lock_guard<std::mutex> h(g_host_mu);
  g_alloc_ms = g_free_ms = g_sync_ms = 0;
  g_allocs = g_syncs = 0;
}

extern "C" gsmat_status gsmat_prof_host(double* out5) {
  return guarded([&]() -> gsmat_status {
    if (!out5) throw StatusFail{GSMAT_EINVAL, "out is NULL"};
    std::lock_guard<std::mutex> h(g_host_mu);
    out5[0] = g_alloc_ms;
    out5[1] = (double)g_allocs;
    out5[2] = g_free_ms;
    out5[3] = g_sync_ms;
    out5[4] = (double)g_syncs;
    return GSMAT_OK;
  });
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
