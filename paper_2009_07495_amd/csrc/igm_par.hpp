// Host-side parallel loops of the setup (plain std::thread, no pool).
//
// The setup passes are elementwise or row-wise, so they are split into
// contiguous ranges, one per thread; each range does exactly the operations
// the serial loop would do for its rows, so results are bit-identical for any
// thread count. Setups that run concurrently (batched and served solvers
// prepare several systems at once) share the cores: each gets the core count
// divided by the number of setups in progress.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

namespace igm {

// Threads for one setup now (at least 1). IGM_SETUP_THREADS overrides the
// core count (at most 64).
int setup_thread_count();

// Marks a setup in progress for the lifetime of the object.
struct SetupRegion {
  SetupRegion();
  ~SetupRegion();
};

// f(chunk, lo, hi) over [0, n) in nt contiguous chunks (serially when nt <= 1
// or n is below `serial_below` items). Chunk c covers rows before those of
// chunk c + 1. Callers whose items are large (slices of many rows) pass a
// smaller threshold.
template <class F>
void par_ranges(int nt, int64_t n, F &&f, int64_t serial_below = 32768) {
  if (nt <= 1 || n < serial_below) {
    f(0, (int64_t)0, n);
    return;
  }
  const int64_t per = (n + nt - 1) / nt;
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) {
    const int64_t lo = t * per, hi = std::min(n, lo + per);
    if (lo < hi) th.emplace_back([&f, t, lo, hi] { f(t, lo, hi); });
  }
  f(0, (int64_t)0, std::min(n, per));
  for (auto &x : th) x.join();
}

// dst = src[0 .. count) (converted element by element to dst's type), resized
// and copied in parallel chunks.
template <class V, class T>
void par_assign(V &dst, const T *src, int64_t count) {
  dst.resize(count);
  auto *d = dst.data();
  par_ranges(setup_thread_count(), count,
             [&](int, int64_t lo, int64_t hi) { std::copy(src + lo, src + hi, d + lo); });
}

// Spinning barrier for a fixed set of threads (the level loop of ILU(0)).
class SpinBarrier {
 public:
  explicit SpinBarrier(int n) : n_(n) {}
  void wait() {
    const int g = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
      count_.store(0, std::memory_order_relaxed);
      gen_.store(g + 1, std::memory_order_release);
    } else {
      while (gen_.load(std::memory_order_acquire) == g) std::this_thread::yield();
    }
  }

 private:
  const int n_;
  std::atomic<int> count_{0};
  std::atomic<int> gen_{0};
};

}  // namespace igm
