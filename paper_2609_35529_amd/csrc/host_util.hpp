// Host-side utilities of the 2-D and 3-D libraries: a worker pool kept for the
// life of the process, shared by every context (hierarchy changes run many
// short parallel sections, per level and per band of rows, and creating
// threads for each costs more than the work on a virtual machine), and a
// phase timer for hierarchy changes.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace vlbm_host {

class Pool {
 public:
  // The process-wide pool: min(15, hardware threads - 1) workers, created on
  // first use and never destroyed (the threads end with the process).
  static Pool &get() {
    static Pool *p = new Pool(std::min(15, std::max(1, (int)std::thread::hardware_concurrency() - 1)));
    return *p;
  }

  // Calls f(i) for every i in [0, n) on the workers and the calling thread,
  // and returns when all have returned. The caller takes items of its own
  // call until none is left, so a call made from inside f (nested) always
  // progresses, whatever the workers are doing. If items throw, every item
  // still runs and the first exception caught is rethrown to the caller.
  void run(int n, const std::function<void(int)> &f) {
    if (n <= 0) return;
    if (n == 1) {
      f(0);
      return;
    }
    Batch b;
    b.f = &f;
    b.n = n;
    {
      std::lock_guard<std::mutex> g(m_);
      q_.push_back(&b);
      queued_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    for (int i; (i = b.next.fetch_add(1)) < n;) b.item(i);
    {  // no worker can claim an item of b once it has left the queue
      std::lock_guard<std::mutex> g(m_);
      auto it = std::find(q_.begin(), q_.end(), &b);
      if (it != q_.end()) {
        q_.erase(it);
        queued_.fetch_sub(1, std::memory_order_relaxed);
      }
    }
    while (b.done.load(std::memory_order_acquire) < n) std::this_thread::yield();
    if (b.err) std::rethrow_exception(b.err);
  }

 private:
  struct Batch {
    const std::function<void(int)> *f = nullptr;
    int n = 0;
    std::atomic<int> next{0}, done{0};
    std::mutex em;
    std::exception_ptr err;  // the first exception an item threw
    void item(int i) {
      try {
        (*f)(i);
      } catch (...) {
        std::lock_guard<std::mutex> g(em);
        if (!err) err = std::current_exception();
      }
      done.fetch_add(1, std::memory_order_release);  // the batch may end right after this
    }
  };

  explicit Pool(int nworkers) {
    for (int i = 0; i < nworkers; ++i) std::thread([this] { loop(); }).detach();
  }

  // One claimed item (batch, index) or none, under the lock: a batch whose
  // items are all claimed leaves the queue.
  bool claim(Batch *&b, int &i) {
    while (!q_.empty()) {
      b = q_.front();
      i = b->next.fetch_add(1);
      if (i < b->n) return true;
      q_.pop_front();
      queued_.fetch_sub(1, std::memory_order_relaxed);
    }
    return false;
  }

  void loop() {
    using clock = std::chrono::steady_clock;
    for (;;) {
      Batch *b = nullptr;
      int i = 0;
      {
        std::unique_lock<std::mutex> l(m_);
        if (!claim(b, i)) {
          // sections of a hierarchy change follow each other closely: look
          // for work for a short while before sleeping
          l.unlock();
          const auto until = clock::now() + std::chrono::microseconds(200);
          while (queued_.load(std::memory_order_acquire) == 0 && clock::now() < until) std::this_thread::yield();
          l.lock();
          cv_.wait(l, [&] { return claim(b, i); });
        }
      }
      b->item(i);
    }
  }

  std::mutex m_;
  std::condition_variable cv_;
  std::deque<Batch *> q_;
  std::atomic<int> queued_{0};
};

// VLBM_TIMING=1 prints host-side phase timings of hierarchy changes to stderr.
struct PhaseTimer {
  bool on;
  std::chrono::steady_clock::time_point t;
  const char *what;
  explicit PhaseTimer(const char *w)
      : on(getenv("VLBM_TIMING") != nullptr), t(std::chrono::steady_clock::now()), what(w) {}
  void mark(const char *phase) {
    if (!on) return;
    auto now = std::chrono::steady_clock::now();
    fprintf(stderr, "[vlbm] %s %s %.3f ms\n", what, phase, std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

}  // namespace vlbm_host
