#include "host_pool.hpp"

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

namespace gsmat {
namespace {

class Pool {
 public:
  explicit Pool(int n) {
    for (int i = 0; i < n; ++i) workers_.emplace_back([this] { loop(); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (std::thread& t : workers_) t.join();
  }
  int size() const { return (int)workers_.size(); }
  std::mutex& owner() { return owner_; }

  // Runs chunks [0, nchunks) of fn over the workers and the caller.
  void run(int64_t n, int64_t nchunks, const std::function<void(int64_t, int64_t)>* fn) {
    {
      std::lock_guard<std::mutex> g(mu_);
      fn_ = fn;
      n_ = n;
      nchunks_ = nchunks;
      next_.store(0);
      done_ = 0;
      ++gen_;
    }
    cv_.notify_all();
    work();
    // every chunk done and no worker still inside work(), so none can take
    // a chunk of the next call
    std::unique_lock<std::mutex> g(mu_);
    done_cv_.wait(g, [&] { return done_ == nchunks_ && busy_ == 0; });
    fn_ = nullptr;
  }

 private:
  void work() {
    for (;;) {
      const int64_t c = next_.fetch_add(1);
      if (c >= nchunks_) return;
      const int64_t lo = n_ * c / nchunks_, hi = n_ * (c + 1) / nchunks_;
      (*fn_)(lo, hi);
      std::lock_guard<std::mutex> g(mu_);
      if (++done_ == nchunks_) done_cv_.notify_one();
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [&] { return stop_ || (gen_ != seen && fn_ != nullptr); });
        if (stop_) return;
        seen = gen_;
        ++busy_;
      }
      work();
      std::lock_guard<std::mutex> g(mu_);
      if (--busy_ == 0) done_cv_.notify_one();
    }
  }

  std::vector<std::thread> workers_;
  std::mutex mu_, owner_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int64_t, int64_t)>* fn_ = nullptr;
  int64_t n_ = 0, nchunks_ = 0, done_ = 0;
  int busy_ = 0;  // workers inside work()
  std::atomic<int64_t> next_{0};
  uint64_t gen_ = 0;
  bool stop_ = false;
};

int pool_threads() {
  if (const char* e = std::getenv("GSMAT_HOST_THREADS")) return std::max(0, std::atoi(e));
  const int hw = (int)std::thread::hardware_concurrency();
  return std::max(0, std::min(7, hw - 1));
}

Pool* pool() {
  static Pool* p = [] {
    const int n = pool_threads();
    return n > 0 ? new Pool(n) : nullptr;  // lives until the process ends
  }();
  return p;
}

}  // namespace

void host_parallel_for(int64_t n, int64_t min_per_thread,
                       const std::function<void(int64_t, int64_t)>& fn) {
  if (n <= 0) return;
  Pool* p = pool();
  const int64_t parts =
      p ? std::min<int64_t>(p->size() + 1, n / std::max<int64_t>(min_per_thread, 1)) : 1;
  if (parts <= 1) {
    fn(0, n);
    return;
  }
  std::unique_lock<std::mutex> own(p->owner(), std::try_to_lock);
  if (!own.owns_lock()) {  // another caller holds the pool
    fn(0, n);
    return;
  }
  p->run(n, parts * 4, &fn);
}

}  // namespace gsmat
