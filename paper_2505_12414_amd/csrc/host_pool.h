// A small pool of host threads for the server's per-fit arithmetic (plain
// C++, no device code: the CPU tests build it on its own).
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace uml {

// A few host threads that share a batch's per-fit arithmetic (the start
// metric at admission, the covariance at retirement) with the worker.  Each
// call of run() is a job of its own with its own counters: a helper that
// wakes late finds the job's items taken and does nothing, and run()
// returns once every item has been done, so the function is never called
// after run() returns.
class HostPool {
 public:
  explicit HostPool(int helpers) {
    for (int t = 0; t < helpers; ++t) th_.emplace_back([this] { loop(); });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  // f(0) .. f(n - 1) on the helpers and the calling thread.
  void run(int n, const std::function<void(int)>& f) {
    if (th_.empty() || n < 8) {
      for (int i = 0; i < n; ++i) f(i);
      return;
    }
    auto job = std::make_shared<Task>();
    job->f = &f;
    job->n = n;
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = job;
      ++gen_;
    }
    cv_.notify_all();
    job->work();
    while (job->done.load(std::memory_order_acquire) < n) std::this_thread::yield();
  }

 private:
  struct Task {
    const std::function<void(int)>* f = nullptr;
    int n = 0;
    std::atomic<int> next{0}, done{0};
    void work() {
      for (int i; (i = next.fetch_add(1, std::memory_order_relaxed)) < n;) {
        (*f)(i);
        done.fetch_add(1, std::memory_order_release);
      }
    }
  };
  void loop() {
    uint64_t seen = 0;
    while (true) {
      std::shared_ptr<Task> job;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        job = job_;
      }
      job->work();
    }
  }
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::shared_ptr<Task> job_;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

}  // namespace uml
