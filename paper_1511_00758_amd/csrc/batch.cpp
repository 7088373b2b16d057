// sm_solve_batch: many independent frames solved concurrently by a pool of host
// workers, each with its own stream and workspace (contract in stereomesh.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "delaunay.hpp"
#include "kernels.hpp"
#include "star.hpp"
#include "pool.hpp"
#include "sm_common.hpp"
#include "stereomesh.h"

namespace sm {
namespace {
inline WorkerPool& pool() { return thread_pool(); }
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

// =====================================================================================
// sm_solve_many: stage-batched solve. Every stage of Alg. 1 is one launch over all
// frames (mixed sizes and parameters); the host triangulations of the frames run on a
// worker pool between the stages that need them.
// =====================================================================================
namespace sm {
namespace {

struct ManyPlan {
  std::vector<Layout> lay;
  std::vector<size_t> base;      // workspace offset of each frame
  std::vector<int32_t> pack_off;  // staging slot offset of each frame (header + capacity)
  std::vector<int32_t> pack_cap;
  std::vector<int32_t> groups;   // distinct (rx << 8 | ry) census windows
  // device-mesh frames: their triangles (tdev_off, in triangles)
  std::vector<int32_t> tdev_off;
  size_t desc_off = 0, off_off = 0, job_off = 0, soff_off = 0, tri_off = 0, pack_dev = 0, tdev = 0, mstat = 0,
         nvalid = 0, total = 0;
  int32_t pack_slots = 0, tri_cap = 0, n_off_arrays = 0, tdev_cap = 0;
};

constexpr int kOffArrays = 5;  // match, raster, validate, rematch, + one per census group

sm_status plan_many(const sm_frame* frames, int32_t n, ManyPlan& P) {
  P = ManyPlan{};
  size_t o = 0;
  std::map<int32_t, int> grp;
  for (int32_t f = 0; f < n; ++f) {
    const sm_frame& fr = frames[f];
    if (!dims_ok(fr.W, fr.H)) return fail(SM_ERR_ARG, "frame %d: size %dx%d outside [3, 8192]^2", f, fr.W, fr.H);
    if (fr.stride < fr.W) return fail(SM_ERR_ARG, "frame %d: stride < W", f);
    if (!fr.L || !fr.R || !fr.D_f || !fr.C_f || !fr.mask) return fail(SM_ERR_ARG, "frame %d: NULL buffer", f);
    const sm_status ps = check_params(&fr.p);
    if (ps != SM_OK) return fail(ps, "frame %d: %s", f, last_error().c_str());
    if (fr.p.support_mode != 0)
      return fail(SM_ERR_ARG, "frame %d: sm_solve_many takes grid supports only (support_mode 0)", f);
    const Layout L = layout_of(fr.W, fr.H, fr.p);
    P.lay.push_back(L);
    P.base.push_back(o);
    o = align256(o + L.total);
    int32_t cap = L.n_grid;
    for (int it = 1; it < fr.p.n_iters; ++it) cap = std::max(cap, 2 * cells_of(fr.W, fr.H, occ_size(fr.p, it)));
    P.pack_off.push_back(P.pack_slots);
    P.pack_cap.push_back(cap);
    P.pack_slots += cap + 1;
    P.tri_cap += L.T_cap;
    P.tdev_off.push_back(P.tdev_cap);
    if (L.mesh_on) P.tdev_cap += L.T_cap;
    const int32_t key = ((fr.p.census_w - 1) / 2) << 8 | ((fr.p.census_h - 1) / 2);
    if (!grp.count(key)) {
      grp[key] = (int)P.groups.size();
      P.groups.push_back(key);
    }
  }
  P.n_off_arrays = kOffArrays - 1 + (int)P.groups.size();
  P.desc_off = o;
  o += (size_t)n * sizeof(BatchFrame);
  P.off_off = o;
  o += (size_t)P.n_off_arrays * (n + 1) * sizeof(int32_t);
  P.job_off = align256(o);
  o = P.job_off + (size_t)n * sizeof(StarJob);
  P.soff_off = o;  // prefix sums of the star jobs' workgroups
  o += (size_t)(n + 1) * sizeof(int32_t);
  P.tri_off = align256(o);  // desc + offsets + mesh jobs + triangles go up in one copy
  o = P.tri_off + (size_t)P.tri_cap * sizeof(sm_tri);
  P.pack_dev = align256(o);
  o = P.pack_dev + (size_t)P.pack_slots * sizeof(sm_support);
  P.tdev = align256(o);
  o = P.tdev + (size_t)P.tdev_cap * sizeof(sm_tri);
  P.mstat = align256(o);  // every frame's mesh status words (a copy the mesh kernels keep)
  o = P.mstat + (size_t)n * kMeshStatusWords * sizeof(int32_t);
  P.nvalid = align256(o);  // every frame's valid-pixel count, side by side for one read-back
  o = P.nvalid + (size_t)n * sizeof(unsigned long long);
  P.total = align256(o);
  return SM_OK;
}

struct ManyCtx {
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  std::vector<Delaunay> dl;
  std::vector<std::vector<sm_tri>> tris;
  std::vector<std::vector<int32_t>> bu, bv, bext;
  std::vector<hipEvent_t> ev;
};

ManyCtx& many_ctx() {
  static thread_local ManyCtx* c = new ManyCtx();
  return *c;
}

// A capture of the device work of one batch (sm_solve_many_capture): its own pinned
// staging, which the graph's copies read on every replay.
struct GraphBuild {
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // what a replay's read-back needs
  ManyPlan P;
  uint8_t* base = nullptr;
  int32_t* hmstat = nullptr;
  unsigned long long* hnv = nullptr;
  std::vector<int32_t> iters;
};

// Ends a stream capture left open by an early return.
struct CaptureGuard {
  hipStream_t s;
  bool active = false;
  explicit CaptureGuard(hipStream_t ss) : s(ss) {}
  ~CaptureGuard() {
    if (!active) return;
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
  }
};

// End of a batch whose meshes all live on the device: one read-back of every frame's
// status words and valid-pixel count, then each frame whose device mesh failed is solved
// again alone with host meshes (in its own part of the workspace); st gets the counts.
sm_status finish_device_batch(const sm_frame* frames, int32_t n, const ManyPlan& P, uint8_t* base, int32_t* hmstat,
                              unsigned long long* hnv, const std::vector<int32_t>& iters, sm_stats* st,
                              hipStream_t s, float& us_xfer) {
  const int32_t* dmstat = (const int32_t*)(base + P.mstat);
  const unsigned long long* dnv = (const unsigned long long*)(base + P.nvalid);
  auto t1 = std::chrono::steady_clock::now();
  SM_HIP(hipMemcpyAsync(hmstat, dmstat, (size_t)n * kMeshStatusWords * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SM_HIP(hipMemcpyAsync(hnv, dnv, (size_t)n * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  SM_HIP(hipStreamSynchronize(s));
  us_xfer += std::chrono::duration<float, std::micro>(std::chrono::steady_clock::now() - t1).count();
  for (int32_t f = 0; f < n; ++f) {
    const int32_t* w = hmstat + (size_t)kMeshStatusWords * f;
    if (w[kMeshErr] != 0) {  // this frame again, alone, every tessellation on the host
      sm_params q = frames[f].p;
      q.host_mesh = 1;
      sm_stats one;
      std::memset(&one, 0, sizeof(one));
      const sm_frame& fr = frames[f];
      const sm_status r = sm_solve(fr.L, fr.R, fr.W, fr.H, fr.stride, &q, base + P.base[f], P.lay[f].total, fr.D_f,
                                   fr.C_f, fr.mask, &one, s);
      if (r != SM_OK) return fail(r, "frame %d: %s", f, last_error().c_str());
      if (st) {
        ++st->mesh_fallback;
        st->n_valid += one.n_valid;
        for (int k = 0; k < iters[f] && k < 8; ++k) {
          st->n_support[k] += one.n_support[k];
          st->n_tris[k] += one.n_tris[k];
        }
      }
      continue;
    }
    if (st) {
      st->n_valid += (int64_t)hnv[f];
      st->mesh_device += iters[f];
      for (int k = 0; k < iters[f] && k < 8; ++k) {
        st->n_support[k] += w[kMeshLog + 2 * k];
        st->n_tris[k] += star_log_tris(w, k, iters[f]);
      }
    }
  }
  return SM_OK;
}

sm_status many_impl(sm_frame* frames, int32_t n, void* ws, size_t ws_bytes, int32_t n_threads, sm_stats* st,
                    void* stream, GraphBuild* gb);

}  // namespace
}  // namespace sm

extern "C" size_t sm_solve_many_workspace_bytes(const sm_frame* frames, int32_t n) {
  if (n <= 0 || !frames) return 0;
  ManyPlan P;
  if (plan_many(frames, n, P) != SM_OK) return 0;
  return P.total;
}

extern "C" sm_status sm_solve_many(sm_frame* frames, int32_t n, void* ws, size_t ws_bytes, int32_t n_threads,
                                   sm_stats* st, void* stream) {
  last_error().clear();
  return sm::many_impl(frames, n, ws, ws_bytes, n_threads, st, stream, nullptr);
}

namespace sm {
namespace {

sm_status many_impl(sm_frame* frames, int32_t n, void* ws, size_t ws_bytes, int32_t n_threads, sm_stats* st,
                    void* stream, GraphBuild* gb) {
  if (n < 0 || (n > 0 && !frames)) return fail(SM_ERR_ARG, "bad frame array / count");
  if (n == 0) return gb ? fail(SM_ERR_ARG, "nothing to capture") : SM_OK;
  if (n_threads < 1 || n_threads > 256) return fail(SM_ERR_ARG, "n_threads must be in [1, 256]");
  ManyPlan P;
  SM_TRY(plan_many(frames, n, P));
  if (!ws || ((uintptr_t)ws & 255u)) return fail(SM_ERR_ARG, "workspace missing or not 256-byte aligned");
  if (ws_bytes < P.total) return fail(SM_ERR_CAPACITY, "workspace %zu < %zu bytes", ws_bytes, P.total);
  if (gb)
    for (int32_t f = 0; f < n; ++f)
      if (!P.lay[f].mesh_on) return fail(SM_ERR_ARG, "frame %d: a captured batch keeps its meshes on the device", f);
  const hipStream_t s = (hipStream_t)stream;
  const int32_t timing = st && !gb ? st->timing : 0;  // no timing events inside a capture
  const uint32_t timed = (timing & SM_TIME_SELECTED) ? (uint32_t)timing & 0xffffu : 0xffffu;
  if (st) {
    const int32_t keep = st->timing;
    std::memset(st, 0, sizeof(*st));
    st->timing = keep;
  }
  const auto t_start = std::chrono::steady_clock::now();
  ManyCtx& c = many_ctx();
  // pinned staging: [desc | offsets | mesh jobs | triangles] (uploaded together), then
  // [packed supports], [mesh status words], [valid-pixel counts], and for batches whose
  // meshes all live on the device one [desc | offsets | mesh jobs] per iteration
  const size_t up_bytes = P.pack_dev - P.desc_off;
  const size_t pack_bytes = align256((size_t)P.pack_slots * sizeof(sm_support));
  const size_t stat_bytes = align256((size_t)n * kMeshStatusWords * sizeof(int32_t));
  const size_t nv_bytes = align256((size_t)n * sizeof(unsigned long long));
  const size_t desc_bytes = align256(P.tri_off - P.desc_off);
  const size_t pin_need = up_bytes + pack_bytes + stat_bytes + nv_bytes + 8 * desc_bytes;
  void*& pinned = gb ? gb->pinned : c.pinned;  // a capture owns its staging
  size_t& pinned_bytes = gb ? gb->pinned_bytes : c.pinned_bytes;
  if (pinned_bytes < pin_need) {
    if (pinned) SM_HIP(hipHostFree(pinned));
    pinned = nullptr;
    pinned_bytes = 0;
    SM_HIP(hipHostMalloc(&pinned, pin_need, hipHostMallocDefault));
    pinned_bytes = pin_need;
  }
  if ((int32_t)c.dl.size() < n) {
    c.dl.resize(n);
    c.tris.resize(n);
    c.bu.resize(n);
    c.bv.resize(n);
    c.bext.resize(n);
  }
  uint8_t* base = (uint8_t*)ws;
  uint8_t* hp = (uint8_t*)pinned;
  BatchFrame* hF = (BatchFrame*)hp;
  int32_t* hoff = (int32_t*)(hp + (P.off_off - P.desc_off));
  sm_tri* hT = (sm_tri*)(hp + (P.tri_off - P.desc_off));
  sm_support* hpack = (sm_support*)(hp + up_bytes);
  int32_t* hmstat = (int32_t*)(hp + up_bytes + pack_bytes);
  unsigned long long* hnv = (unsigned long long*)(hp + up_bytes + pack_bytes + stat_bytes);
  uint8_t* hstage = hp + up_bytes + pack_bytes + stat_bytes + nv_bytes;
  unsigned long long* dnv = (unsigned long long*)(base + P.nvalid);
  StarJob* hjobs = (StarJob*)(hp + (P.job_off - P.desc_off));
  int32_t* hsoff = (int32_t*)(hp + (P.soff_off - P.desc_off));
  const StarJob* djobs = (const StarJob*)(base + P.job_off);
  const int32_t* dsoff = (const int32_t*)(base + P.soff_off);
  // the workgroup offsets of jobs [0, n_jobs) (in the staged copy at h); returns their total
  auto star_offsets = [](const StarJob* J, int32_t* o, int32_t n_jobs) {
    o[0] = 0;
    for (int32_t j = 0; j < n_jobs; ++j) o[j + 1] = o[j] + J[j].blocks;
    return o[n_jobs];
  };
  sm_tri* dTdev = (sm_tri*)(base + P.tdev);
  int32_t* dmstat = (int32_t*)(base + P.mstat);
  const BatchFrame* dF = (const BatchFrame*)(base + P.desc_off);
  const int32_t* doff = (const int32_t*)(base + P.off_off);
  sm_tri* dT = (sm_tri*)(base + P.tri_off);
  sm_support* dpack = (sm_support*)(base + P.pack_dev);
  auto off_arr = [&](int k) { return hoff + (size_t)k * (n + 1); };
  auto doff_arr = [&](int k) { return doff + (size_t)k * (n + 1); };
  enum { kMatch = 0, kRaster = 1, kValidate = 2, kRematch = 3, kCensus0 = 4 };

  // stage timing: an armed event pair per launch, summed after the final synchronisation
  std::vector<std::pair<int, int>> marks;
  int used = 0;
  auto arm = [&](int stage) -> sm_status {
    if (!timing || !(timed >> stage & 1u)) return SM_OK;
    while ((int)c.ev.size() < used + 2) {
      hipEvent_t e;
      SM_HIP(hipEventCreate(&e));
      c.ev.push_back(e);
    }
    set_launch_events(c.ev[used], c.ev[used + 1]);
    marks.push_back({stage, used});
    used += 2;
    return SM_OK;
  };
  float us_host = 0.f, us_xfer = 0.f;
  auto since = [](std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<float, std::micro>(std::chrono::steady_clock::now() - t).count();
  };

  // static frame descriptors
  for (int32_t f = 0; f < n; ++f) {
    const sm_frame& fr = frames[f];
    const Layout& L = P.lay[f];
    uint8_t* b = base + P.base[f];
    BatchFrame& d = hF[f];
    std::memset(&d, 0, sizeof(d));
    d.L = fr.L;
    d.R = fr.R;
    d.W = fr.W;
    d.H = fr.H;
    d.stride = fr.stride;
    d.p = fr.p;
    d.cL = (uint64_t*)(b + L.cL);
    d.cR = (uint64_t*)(b + L.cR);
    d.omega = b + L.omega;
    d.occ = b + L.occ;
    d.D_it = (float*)(b + L.D_it);
    d.cell_g = (uint64_t*)(b + L.cell_g);
    d.cell_b = (uint64_t*)(b + L.cell_b);
    d.S = (sm_support*)(b + L.S);
    d.counters = (int32_t*)(b + L.counters);
    d.n_valid = dnv + f;
    d.D_f = fr.D_f;
    d.C_f = fr.C_f;
    d.mask = fr.mask;
    d.n_grid = L.n_grid;
    d.match_lanes = match_lanes_for(fr.W, fr.H, fr.p);
    d.census_rows = census_rows_for(fr.W, fr.H, fr.p.census_w, fr.p.census_h, true);
    d.gw = L.n_grid > 0 ? (fr.W - 1 - fr.p.support_step / 2) / fr.p.support_step + 1 : 0;
    d.sz = occ_size(fr.p, 1);
    d.pack = L.mesh_on ? nullptr : dpack + P.pack_off[f];  // device-mesh frames keep their supports
    d.pack_cap = L.n_grid;
  }
  // census (one launch per census window) + grid matching offsets
  for (size_t g = 0; g < P.groups.size(); ++g) {
    int32_t* o = off_arr(kCensus0 + (int)g);
    o[0] = 0;
    for (int32_t f = 0; f < n; ++f) {
      const int32_t key = ((frames[f].p.census_w - 1) / 2) << 8 | ((frames[f].p.census_h - 1) / 2);
      o[f + 1] = o[f] + (key == P.groups[g] ? 2 * census_tiles(frames[f].W, frames[f].H, hF[f].census_rows) : 0);
    }
  }
  {
    int32_t* o = off_arr(kMatch);
    o[0] = 0;
    for (int32_t f = 0; f < n; ++f) o[f + 1] = o[f] + match_units(P.lay[f].n_grid, hF[f].match_lanes);
  }
  // frames whose meshes live on the device (grid supports, host_mesh = 0): the first mesh is
  // built by one launch over them right after compaction; job j's status words come back
  // in one copy
  int64_t mesh_candidates = 0;  // star kernel layout of the batch (star_grouped)
  for (int32_t f = 0; f < n; ++f)
    if (P.lay[f].mesh_on) mesh_candidates += P.lay[f].n_grid;
  const bool grouped = star_grouped(mesh_candidates);
  // every frame's meshes on the device: the star kernel's workgroups rasterise the triangles
  // they find, and the batch has no raster stage
  bool all_dev = true;
  for (int32_t f = 0; f < n; ++f) all_dev &= P.lay[f].mesh_on;
  const bool star_raster = all_dev;
  std::vector<uint8_t> mesh_dev(n, 0), job_start;
  std::vector<int32_t> host_upto(n, 0), nT_dev(n, 0), job_frame;
  auto add_job = [&](int32_t f, int32_t start, const int32_t* n_new) {
    const Layout& L = P.lay[f];
    uint8_t* b = base + P.base[f];
    StarJob& jb = hjobs[job_frame.size()];
    jb.S = hF[f].S;
    jb.first = start;
    jb.compact_n = 0;  // the batched stages compact the supports
    jb.occ = nullptr;
    jb.compact_count = nullptr;
    jb.n_new = n_new;
    jb.status = (int32_t*)(b + L.mstatus);
    jb.status_copy = dmstat + (size_t)kMeshStatusWords * f;
    jb.T = dTdev + P.tdev_off[f];
    jb.T_cap = L.T_cap;
    jb.W = hF[f].W;
    jb.H = hF[f].H;
    jb.blocks = star_blocks_many(L.S_cap, grouped);
    jb.D = star_raster ? hF[f].D_it : nullptr;
    jb.w = star_work_at(b + L.mwork, hF[f].W, hF[f].H, L.S_cap);
    job_frame.push_back(f);
    job_start.push_back((uint8_t)start);
  };
  for (int32_t f = 0; f < n; ++f)
    if (P.lay[f].mesh_on) {
      mesh_dev[f] = 1;
      add_job(f, 1, (const int32_t*)(hF[f].S + hF[f].n_grid));
    }
  const int32_t first_blocks = star_offsets(hjobs, hsoff, (int32_t)job_frame.size());
  bool all_lds = true;  // every frame's star preparation fits in LDS
  for (int32_t f = 0; f < n; ++f) all_lds &= prep_in_lds(frames[f].W, frames[f].H);
  CaptureGuard cap(s);
  if (gb) {  // everything enqueued from here to the last mesh launch goes into the graph
    SM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    cap.active = true;
  }
  auto t0 = std::chrono::steady_clock::now();
  SM_HIP(hipMemcpyAsync(base + P.desc_off, hp, P.tri_off - P.desc_off, hipMemcpyHostToDevice, s));
  SM_HIP(launch_zero(dnv, (size_t)n * sizeof(unsigned long long), s));
  us_xfer += since(t0);
  for (size_t g = 0; g < P.groups.size(); ++g) {
    SM_TRY(arm(SM_ST_CENSUS));
    SM_HIP(launch_batch_census(dF, doff_arr(kCensus0 + (int)g), n, off_arr(kCensus0 + (int)g)[n], P.groups[g] >> 8,
                               P.groups[g] & 255, s));
  }
  SM_TRY(arm(SM_ST_MATCH));
  SM_HIP(launch_batch_match(dF, doff_arr(kMatch), n, off_arr(kMatch)[n], s));
  SM_TRY(arm(SM_ST_COMPACT));
  SM_HIP(launch_batch_compact(dF, n, 0, s));
  SM_TRY(arm(SM_ST_COMPACT));
  SM_HIP(launch_batch_pack(dF, n, 0, s));
  if (!job_frame.empty()) {
    SM_TRY(arm(SM_ST_MESH));
    SM_HIP(launch_star_many(djobs, dsoff, (int32_t)job_frame.size(), first_blocks, all_lds, grouped, s));
  }

  std::vector<int32_t> n_S(n, 0), iters(n);
  int max_iters = 0;
  for (int32_t f = 0; f < n; ++f) max_iters = std::max(max_iters, iters[f] = frames[f].p.n_iters);

  // Every frame's meshes on the device: the counts stay there too (each frame's mesh status,
  // read by the raster, resampling and mesh kernels; each mesh kernel first compacts its new
  // supports), so the batch runs without a synchronisation until its end. Every iteration's
  // descriptors are staged in a host buffer of their own, since earlier uploads may still be
  // pending. A frame whose device mesh failed is then solved again alone, with host meshes.
  if (all_dev) {
    constexpr int32_t kRasterUnits = 1024;  // waves per frame, striding over its triangles
    for (int it = 1; it <= max_iters; ++it) {
      uint8_t* h = hstage + (size_t)(it - 1) * desc_bytes;
      std::memcpy(h, hp, P.tri_off - P.desc_off);  // static descriptors and offsets
      BatchFrame* F = (BatchFrame*)h;
      int32_t* ho = (int32_t*)(h + (P.off_off - P.desc_off));
      StarJob* J = (StarJob*)(h + (P.job_off - P.desc_off));
      int32_t* J_off = (int32_t*)(h + (P.soff_off - P.desc_off));
      int32_t* o_r = ho + (size_t)kRaster * (n + 1);
      int32_t* o_v = ho + (size_t)kValidate * (n + 1);
      int32_t* o_m = ho + (size_t)kRematch * (n + 1);
      o_r[0] = o_v[0] = o_m[0] = 0;
      std::vector<uint8_t> active(n, 0);
      int32_t n_jobs = 0;
      bool resample = false;
      for (int32_t f = 0; f < n; ++f) {
        BatchFrame& d = F[f];
        const Layout& L = P.lay[f];
        uint8_t* b = base + P.base[f];
        const bool act = it <= iters[f];
        active[f] = act;
        d.sz = occ_size(frames[f].p, std::min(it, iters[f]));
        d.last = act && it == iters[f];
        d.counts = (const int32_t*)(b + L.mstatus);
        d.S_cap = L.S_cap;
        d.T_cap = L.T_cap;
        d.T = dTdev + P.tdev_off[f];
        d.n_T = d.n_S = 0;
        const bool rs = act && it < iters[f];
        d.region_n = rs ? 2 * cells_of(d.W, d.H, d.sz) : 0;
        d.region = nullptr;
        d.pack = nullptr;
        d.pack_cap = 0;
        o_r[f + 1] = o_r[f] + (act ? kRasterUnits : 0);
        o_m[f + 1] = o_m[f] + d.region_n / 2;
        if (rs) {  // this iteration's resampled supports, compacted and inserted by the mesh kernel
          StarJob& jb = J[n_jobs++];
          jb = StarJob{};
          jb.S = d.S;
          jb.first = 0;  // the new supports start at the frame's support count on the device
          jb.compact_n = d.region_n;
          jb.occ = d.occ;
          jb.compact_count = d.counters + 1;
          jb.n_new = nullptr;
          jb.status = (int32_t*)(b + L.mstatus);
          jb.status_copy = dmstat + (size_t)kMeshStatusWords * f;
          jb.T = dTdev + P.tdev_off[f];
          jb.T_cap = L.T_cap;
          jb.W = d.W;
          jb.H = d.H;
          jb.blocks = star_blocks_many(L.S_cap, grouped);
          jb.w = star_work_at(b + L.mwork, d.W, d.H, L.S_cap);
          jb.D = star_raster ? d.D_it : nullptr;
        }
        resample |= rs;
      }
      struct VCtx {
        const BatchFrame* F;
        const uint8_t* act;
        int32_t n;
      } vc{F, active.data(), n};
      const int nw = validate_pick_nw(
          [](int w, void* x) {
            const VCtx& q = *(const VCtx*)x;
            int64_t tot = 0;
            for (int32_t f = 0; f < q.n; ++f)
              if (q.act[f]) tot += (int64_t)validate_blocks(q.F[f].W, q.F[f].H, q.F[f].sz, w) * w;
            return tot;
          },
          &vc);
      for (int32_t f = 0; f < n; ++f)
        o_v[f + 1] = o_v[f] + (active[f] ? validate_blocks(F[f].W, F[f].H, F[f].sz, nw) : 0);
      const int32_t it_blocks = star_offsets(J, J_off, n_jobs);
      SM_HIP(hipMemcpyAsync(base + P.desc_off, h, P.tri_off - P.desc_off, hipMemcpyHostToDevice, s));
      if (!star_raster) {
        SM_TRY(arm(SM_ST_RASTER));
        SM_HIP(launch_batch_raster(dF, doff_arr(kRaster), n, o_r[n], s));
      }
      SM_TRY(arm(SM_ST_VALIDATE));
      SM_HIP(launch_batch_validate(dF, doff_arr(kValidate), n, o_v[n], nw, s));
      if (!resample) break;
      SM_TRY(arm(SM_ST_REMATCH));
      SM_HIP(launch_batch_rematch(dF, doff_arr(kRematch), n, o_m[n], s));
      SM_TRY(arm(SM_ST_MESH));
      SM_HIP(launch_star_many(djobs, dsoff, n_jobs, it_blocks, all_lds, grouped, s));
    }
    if (gb) {  // the graph of the batch, then its first run
      cap.active = false;
      SM_HIP(hipStreamEndCapture(s, &gb->graph));
      SM_HIP(hipGraphInstantiate(&gb->exec, gb->graph, nullptr, nullptr, 0));
      SM_HIP(hipGraphLaunch(gb->exec, s));
      gb->P = P;
      gb->base = base;
      gb->hmstat = hmstat;
      gb->hnv = hnv;
      gb->iters = iters;
    }
    SM_TRY(finish_device_batch(frames, n, P, base, hmstat, hnv, iters, st, s, us_xfer));
    if (st) {
      for (const auto& mk : marks) {
        float ms = 0.f;
        SM_HIP(hipEventElapsedTime(&ms, c.ev[mk.second], c.ev[mk.second + 1]));
        st->stage_us[mk.first] += ms * 1e3f;
        st->stage_launches[mk.first] += 1;
      }
    }
    if (st) {
      st->stage_us[SM_ST_HOST_TRI] = us_host;
      st->stage_us[SM_ST_HOST_COPY] = us_xfer;
    }
    for (int32_t f = 0; f < n; ++f) {
      frames[f].status = SM_OK;
      frames[f].worker = 0;
    }
    const float total_us = since(t_start);
    for (int32_t f = 0; f < n; ++f) frames[f].latency_us = total_us;
    if (st) st->stage_us[SM_ST_TOTAL] = total_us;
    return SM_OK;
  }
  std::atomic<int32_t> next(0);
  std::atomic<int32_t> bad(-1);
  // new supports (staged by k_batch_pack) into frame f's mesh; from == 0 starts the mesh
  auto triangulate = [&](int32_t f, bool first) {
    const sm_support* src = hpack + P.pack_off[f];
    int32_t cnt;
    std::memcpy(&cnt, src, sizeof(cnt));
    if (cnt < 0 || cnt > P.pack_cap[f]) {
      bad = f;
      return;
    }
    try {
      if (first) c.dl[f].reset();
      c.bu[f].resize(cnt);
      c.bv[f].resize(cnt);
      c.bext[f].resize(cnt);
      for (int32_t k = 0; k < cnt; ++k) {
        c.bu[f][k] = src[1 + k].u;
        c.bv[f][k] = src[1 + k].v;
        c.bext[f][k] = n_S[f] + k;
      }
      if (!c.dl[f].insert_many(c.bu[f].data(), c.bv[f].data(), c.bext[f].data(), cnt)) bad = f;
      c.tris[f].clear();
      c.dl[f].emit_banded(c.tris[f], 3);
    } catch (...) {
      bad = f;
    }
    n_S[f] += cnt;
  };
  std::vector<int32_t> todo;
  // the frame's supports S[host_upto, upto) into its host mesh (after a device error)
  auto host_catch_up = [&](int32_t f, int32_t upto) -> sm_status {
    const int32_t m = upto - host_upto[f];
    std::vector<sm_support> tmp((size_t)std::max(m, 0));
    auto t1 = std::chrono::steady_clock::now();
    if (m > 0)
      SM_HIP(hipMemcpy(tmp.data(), hF[f].S + host_upto[f], (size_t)m * sizeof(sm_support), hipMemcpyDeviceToHost));
    us_xfer += since(t1);
    auto th = std::chrono::steady_clock::now();
    try {
      if (host_upto[f] == 0) c.dl[f].reset();
      std::vector<int32_t> u(m), v(m), e(m);
      for (int32_t k = 0; k < m; ++k) {
        u[k] = tmp[k].u;
        v[k] = tmp[k].v;
        e[k] = host_upto[f] + k;
      }
      if (!c.dl[f].insert_many(u.data(), v.data(), e.data(), m))
        return fail(SM_ERR_INTERNAL, "frame %d: triangulation input out of range", f);
      c.tris[f].clear();
      c.dl[f].emit_banded(c.tris[f], 3);
    } catch (...) {
      return fail(SM_ERR_INTERNAL, "frame %d: host triangulation failed", f);
    }
    us_host += since(th);
    host_upto[f] = upto;
    return SM_OK;
  };
  auto run_host = [&](bool first) -> sm_status {
    auto t1 = std::chrono::steady_clock::now();
    if (!todo.empty())
      SM_HIP(hipMemcpyAsync(hpack, dpack, (size_t)P.pack_slots * sizeof(sm_support), hipMemcpyDeviceToHost, s));
    if (!job_frame.empty())
      SM_HIP(hipMemcpyAsync(hmstat, dmstat, (size_t)n * kMeshStatusWords * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SM_HIP(hipStreamSynchronize(s));
    us_xfer += since(t1);
    for (size_t j = 0; j < job_frame.size(); ++j) {
      const int32_t f = job_frame[j];
      const int32_t* w = hmstat + (size_t)kMeshStatusWords * f;
      const int32_t n_new = w[kMeshNew];
      const int32_t n_max = job_start[j] ? hF[f].n_grid : hF[f].region_n;
      if (n_new < 0 || n_new > n_max) return fail(SM_ERR_INTERNAL, "frame %d: support count %d", f, n_new);
      if (w[kMeshErr] == 0) {
        if (w[kMeshTris] < 0 || w[kMeshTris] > P.lay[f].T_cap)
          return fail(SM_ERR_INTERNAL, "frame %d: device triangle count %d", f, w[kMeshTris]);
        nT_dev[f] = w[kMeshTris];
        n_S[f] += n_new;
        if (st) ++st->mesh_device;
        continue;
      }
      // the device could not finish this frame: its host mesh takes every support so far, and
      // the frame stays on the host
      mesh_dev[f] = 0;
      if (st) ++st->mesh_fallback;
      SM_TRY(host_catch_up(f, n_S[f] + n_new));
      n_S[f] += n_new;
    }
    job_frame.clear();
    job_start.clear();
    if (todo.empty()) return SM_OK;
    auto th = std::chrono::steady_clock::now();
    next = 0;
    const int32_t m = (int32_t)todo.size();
    auto body = [&](int) {
      for (;;) {
        const int32_t i = next.fetch_add(1);
        if (i >= m) break;
        triangulate(todo[i], first);
      }
    };
    try {
      pool().run(std::max(1, std::min(n_threads, m)), body);
    } catch (...) {
      return fail(SM_ERR_INTERNAL, "could not start triangulation workers");
    }
    us_host += since(th);
    if (bad >= 0) return fail(SM_ERR_INTERNAL, "frame %d: triangulation input out of range", (int)bad);
    return SM_OK;
  };
  todo.clear();
  for (int32_t f = 0; f < n; ++f)
    if (!mesh_dev[f]) todo.push_back(f);
  SM_TRY(run_host(true));
  for (int it = 1; it <= max_iters; ++it) {
    // iteration state, offsets and the triangles of every active frame
    int32_t toff = 0;
    int32_t* o_r = off_arr(kRaster);
    int32_t* o_v = off_arr(kValidate);
    int32_t* o_m = off_arr(kRematch);
    o_r[0] = o_v[0] = o_m[0] = 0;
    std::vector<uint8_t> active(n, 0);
    bool resample = false;
    for (int32_t f = 0; f < n; ++f) {
      BatchFrame& d = hF[f];
      const bool act = it <= iters[f];
      active[f] = act;
      d.n_S = n_S[f];
      d.sz = occ_size(frames[f].p, std::min(it, iters[f]));
      d.last = act && it == iters[f];
      if (mesh_dev[f]) {  // triangles written by the device
        d.n_T = act ? nT_dev[f] : 0;
        d.T = dTdev + P.tdev_off[f];
      } else {
        d.n_T = act ? (int32_t)c.tris[f].size() : 0;
        if (d.n_T > P.lay[f].T_cap) return fail(SM_ERR_INTERNAL, "frame %d: triangle capacity exceeded", f);
        d.T = dT + toff;
        if (d.n_T) std::memcpy(hT + toff, c.tris[f].data(), (size_t)d.n_T * sizeof(sm_tri));
        toff += d.n_T;
      }
      const bool rs = act && it < iters[f];
      d.region_n = rs ? 2 * cells_of(d.W, d.H, d.sz) : 0;
      if (rs && n_S[f] + d.region_n + 1 > P.lay[f].S_cap)
        return fail(SM_ERR_INTERNAL, "frame %d: support capacity exceeded", f);
      d.region = rs ? d.S + n_S[f] : nullptr;
      d.pack_cap = d.region_n;
      d.pack = mesh_dev[f] ? nullptr : dpack + P.pack_off[f];
      if (rs && mesh_dev[f])  // this iteration's resampled supports join the device mesh
        add_job(f, 0, (const int32_t*)(d.region + d.region_n));
      resample |= rs;
      if (st && act && it <= 8) {
        st->n_support[it - 1] += n_S[f];
        st->n_tris[it - 1] += d.n_T;
      }
      o_r[f + 1] = o_r[f] + d.n_T;
      o_m[f + 1] = o_m[f] + (rs ? d.region_n / 2 : 0);
    }
    struct VCtx {
      const BatchFrame* F;
      const uint8_t* act;
      int32_t n;
    } vc{hF, active.data(), n};
    const int nw = validate_pick_nw(
        [](int w, void* x) {
          const VCtx& q = *(const VCtx*)x;
          int64_t tot = 0;
          for (int32_t f = 0; f < q.n; ++f)
            if (q.act[f]) tot += (int64_t)validate_blocks(q.F[f].W, q.F[f].H, q.F[f].sz, w) * w;
          return tot;
        },
        &vc);
    for (int32_t f = 0; f < n; ++f)
      o_v[f + 1] = o_v[f] + (active[f] ? validate_blocks(hF[f].W, hF[f].H, hF[f].sz, nw) : 0);
    const int32_t mix_blocks = star_offsets(hjobs, hsoff, (int32_t)job_frame.size());
    t0 = std::chrono::steady_clock::now();
    SM_HIP(hipMemcpyAsync(base + P.desc_off, hp, (P.tri_off - P.desc_off) + (size_t)toff * sizeof(sm_tri),
                          hipMemcpyHostToDevice, s));
    us_xfer += since(t0);
    SM_TRY(arm(SM_ST_RASTER));
    SM_HIP(launch_batch_raster(dF, doff_arr(kRaster), n, o_r[n], s));
    SM_TRY(arm(SM_ST_VALIDATE));
    SM_HIP(launch_batch_validate(dF, doff_arr(kValidate), n, o_v[n], nw, s));
    if (!resample) break;
    SM_TRY(arm(SM_ST_REMATCH));
    SM_HIP(launch_batch_rematch(dF, doff_arr(kRematch), n, o_m[n], s));
    SM_TRY(arm(SM_ST_COMPACT));
    SM_HIP(launch_batch_compact(dF, n, 1, s));
    SM_TRY(arm(SM_ST_COMPACT));
    SM_HIP(launch_batch_pack(dF, n, 1, s));
    if (!job_frame.empty()) {
      SM_TRY(arm(SM_ST_MESH));
      SM_HIP(launch_star_many(djobs, dsoff, (int32_t)job_frame.size(), mix_blocks, all_lds, grouped, s));
    }
    todo.clear();
    for (int32_t f = 0; f < n; ++f)
      if (hF[f].region_n > 0 && !mesh_dev[f]) todo.push_back(f);
    SM_TRY(run_host(false));
  }
  if (st) {
    // validated-pixel counts: every frame's counter, gathered on the host
    t0 = std::chrono::steady_clock::now();
    SM_HIP(hipMemcpyAsync(hnv, dnv, (size_t)n * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    SM_HIP(hipStreamSynchronize(s));
    us_xfer += since(t0);
    for (int32_t f = 0; f < n; ++f) st->n_valid += (int64_t)hnv[f];
    for (const auto& mk : marks) {
      float ms = 0.f;
      SM_HIP(hipEventElapsedTime(&ms, c.ev[mk.second], c.ev[mk.second + 1]));
      st->stage_us[mk.first] += ms * 1e3f;
      st->stage_launches[mk.first] += 1;
    }
    st->stage_us[SM_ST_HOST_TRI] = us_host;
    st->stage_us[SM_ST_HOST_COPY] = us_xfer;
  } else {
    SM_HIP(hipStreamSynchronize(s));
  }
  for (int32_t f = 0; f < n; ++f) {
    frames[f].status = SM_OK;
    frames[f].worker = 0;
  }
  const float total_us = since(t_start);
  for (int32_t f = 0; f < n; ++f) frames[f].latency_us = total_us;
  if (st) st->stage_us[SM_ST_TOTAL] = total_us;
  return SM_OK;
}

}  // namespace
}  // namespace sm

struct sm_many_graph {
  sm::GraphBuild gb;
  std::vector<sm_frame> frames;
  ~sm_many_graph() {
    if (gb.exec) (void)hipGraphExecDestroy(gb.exec);
    if (gb.graph) (void)hipGraphDestroy(gb.graph);
    if (gb.pinned) (void)hipHostFree(gb.pinned);
  }
};

extern "C" sm_status sm_solve_many_capture(sm_frame* frames, int32_t n, void* ws, size_t ws_bytes, sm_stats* st,
                                           void* stream, sm_many_graph** out) {
  using namespace sm;
  last_error().clear();
  if (!out) return fail(SM_ERR_ARG, "out is NULL");
  *out = nullptr;
  sm_many_graph* g = nullptr;
  try {
    g = new sm_many_graph();
    g->frames.assign(frames, frames + (n > 0 && frames ? n : 0));
  } catch (...) {
    delete g;
    return fail(SM_ERR_INTERNAL, "out of host memory");
  }
  const sm_status r = many_impl(frames, n, ws, ws_bytes, 1, st, stream, &g->gb);
  if (r != SM_OK) {
    delete g;
    return r;
  }
  *out = g;
  return SM_OK;
}

extern "C" sm_status sm_many_graph_run(sm_many_graph* g, sm_stats* st, void* stream) {
  using namespace sm;
  last_error().clear();
  if (!g || !g->gb.exec) return fail(SM_ERR_ARG, "no captured batch");
  if (st) {
    const int32_t keep = st->timing;
    std::memset(st, 0, sizeof(*st));
    st->timing = keep;
  }
  const auto t_start = std::chrono::steady_clock::now();
  const hipStream_t s = (hipStream_t)stream;
  SM_HIP(hipGraphLaunch(g->gb.exec, s));
  float us_xfer = 0.f;
  SM_TRY(finish_device_batch(g->frames.data(), (int32_t)g->frames.size(), g->gb.P, g->gb.base, g->gb.hmstat,
                             g->gb.hnv, g->gb.iters, st, s, us_xfer));
  if (st) {
    st->stage_us[SM_ST_HOST_COPY] = us_xfer;
    st->stage_us[SM_ST_TOTAL] =
        std::chrono::duration<float, std::micro>(std::chrono::steady_clock::now() - t_start).count();
  }
  return SM_OK;
}

extern "C" void sm_many_graph_destroy(sm_many_graph* g) { delete g; }
