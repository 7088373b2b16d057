// sm_solve_batch: many independent frames solved concurrently by a pool of host
// workers, each with its own stream and workspace (contract in stereomesh.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sm_common.hpp"
#include "stereomesh.h"

namespace sm {
namespace {

// Workers that persist between the batch calls of one calling thread; joined when that
// thread exits. Each worker keeps its own per-thread solver state (staging, mesh).
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

WorkerPool& pool() {
  static thread_local WorkerPool p;
  return p;
}

}  // namespace
}  // namespace sm

using namespace sm;

extern "C" sm_status sm_solve_batch(sm_frame* frames, int32_t n, void* const* streams, void* const* ws,
                                    const size_t* ws_bytes, int32_t n_workers, sm_stats* st) {
  last_error().clear();
  if (n < 0 || (n > 0 && !frames)) return fail(SM_ERR_ARG, "bad frame array / count");
  if (n_workers < 1 || n_workers > 256 || !streams || !ws || !ws_bytes)
    return fail(SM_ERR_ARG, "need 1..256 workers with streams and workspaces");
  size_t ws_min = ws_bytes[0];
  for (int32_t k = 0; k < n_workers; ++k) {
    if (!ws[k] || ((uintptr_t)ws[k] & 255u)) return fail(SM_ERR_ARG, "workspace %d missing or not 256-byte aligned", k);
    ws_min = std::min(ws_min, ws_bytes[k]);
  }
  for (int32_t i = 0; i < n; ++i) {
    const sm_frame& f = frames[i];
    if (!dims_ok(f.W, f.H)) return fail(SM_ERR_ARG, "frame %d: size %dx%d outside [3, 8192]^2", i, f.W, f.H);
    if (f.stride < f.W) return fail(SM_ERR_ARG, "frame %d: stride < W", i);
    if (!f.L || !f.R || !f.D_f || !f.C_f || !f.mask) return fail(SM_ERR_ARG, "frame %d: NULL buffer", i);
    const sm_status ps = check_params(&f.p);
    if (ps != SM_OK) return fail(ps, "frame %d: %s", i, last_error().c_str());
    const size_t need = sm_solve_workspace_bytes(f.W, f.H, &f.p);
    if (need > ws_min) return fail(SM_ERR_CAPACITY, "frame %d needs %zu workspace bytes, a worker has %zu", i, need, ws_min);
  }
  const int32_t workers = std::max(1, std::min(n_workers, n));
  std::atomic<int32_t> next(0);
  std::vector<sm_stats> wst((size_t)workers);
  for (auto& s : wst) {
    std::memset(&s, 0, sizeof(s));
    s.timing = st ? st->timing : 0;
  }
  std::mutex err_m;
  int32_t first_bad = -1;
  std::string first_msg;
  auto body = [&](int k) {
    sm_stats acc;
    std::memset(&acc, 0, sizeof(acc));
    for (;;) {
      const int32_t i = next.fetch_add(1);
      if (i >= n) break;
      sm_frame& f = frames[i];
      const auto t0 = std::chrono::steady_clock::now();
      sm_stats one;
      std::memset(&one, 0, sizeof(one));
      one.timing = wst[k].timing;
      f.status = sm_solve(f.L, f.R, f.W, f.H, f.stride, &f.p, ws[k], ws_bytes[k], f.D_f, f.C_f, f.mask,
                          st ? &one : nullptr, streams[k]);
      f.worker = k;
      f.latency_us = std::chrono::duration<float, std::micro>(std::chrono::steady_clock::now() - t0).count();
      if (f.status != SM_OK) {
        std::lock_guard<std::mutex> g(err_m);
        if (first_bad < 0 || i < first_bad) {
          first_bad = i;
          first_msg = sm_last_error();
        }
      } else if (st) {
        for (int s = 0; s < 8; ++s) {
          acc.n_support[s] += one.n_support[s];
          acc.n_tris[s] += one.n_tris[s];
        }
        acc.n_valid += one.n_valid;
        for (int s = 0; s < SM_STAGES; ++s) {
          acc.stage_us[s] += one.stage_us[s];
          acc.stage_launches[s] += one.stage_launches[s];
        }
      }
    }
    wst[k] = acc;
  };
  try {
    pool().run(workers, body);
  } catch (...) {
    return fail(SM_ERR_INTERNAL, "could not start batch workers");
  }
  if (st) {
    const int32_t keep = st->timing;
    std::memset(st, 0, sizeof(*st));
    st->timing = keep;
    for (const auto& a : wst) {
      for (int s = 0; s < 8; ++s) {
        st->n_support[s] += a.n_support[s];
        st->n_tris[s] += a.n_tris[s];
      }
      st->n_valid += a.n_valid;
      for (int s = 0; s < SM_STAGES; ++s) {
        st->stage_us[s] += a.stage_us[s];
        st->stage_launches[s] += a.stage_launches[s];
      }
    }
  }
  if (first_bad >= 0) return fail(frames[first_bad].status, "frame %d: %s", first_bad, first_msg.c_str());
  return SM_OK;
}
