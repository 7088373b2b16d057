// Persistent host worker pool of the calling thread (internal header).
#pragma once

#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace sm {

// Workers that persist between the calls of one calling thread; joined when that thread
// exits. run() is not reentrant; workers may use their own pools.
class WorkerPool {
 public:
  ~WorkerPool() {
    {
      std::lock_guard<std::mutex> g(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
  }

  // Runs fn(k) on workers k = 0..n-1 and waits for all of them.
  void run(int n, const std::function<void(int)>& fn) {
    while ((int)threads_.size() < n) {
      const int k = (int)threads_.size();
      threads_.emplace_back([this, k] { loop(k); });
    }
    std::unique_lock<std::mutex> g(m_);
    job_ = &fn;
    active_ = n;
    pending_ = n;
    ++gen_;
    cv_.notify_all();
    done_.wait(g, [&] { return pending_ == 0; });
    job_ = nullptr;
  }

 private:
  void loop(int k) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int)>* job;
      {
        std::unique_lock<std::mutex> g(m_);
        cv_.wait(g, [&] { return stop_ || (gen_ != seen && k < active_); });
        if (stop_) return;
        seen = gen_;
        job = job_;
      }
      (*job)(k);
      {
        std::lock_guard<std::mutex> g(m_);
        if (--pending_ == 0) done_.notify_one();
      }
    }
  }

  std::vector<std::thread> threads_;
  std::mutex m_;
  std::condition_variable cv_, done_;
  const std::function<void(int)>* job_ = nullptr;
  int active_ = 0, pending_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

inline WorkerPool& thread_pool() {
  static thread_local WorkerPool p;
  return p;
}

}  // namespace sm
