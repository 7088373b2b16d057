// C ABI of the stereomesh library (declarations and contracts in stereomesh.h):
// argument checking, launch sequencing, host triangulation and the Alg. 1 loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <initializer_list>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "delaunay.hpp"
#include "kernels.hpp"
#include "star.hpp"
#include "sm_common.hpp"
#include "stereomesh.h"

namespace sm {

std::string& last_error() {
  static thread_local std::string msg;
  return msg;
}

sm_status fail(sm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  last_error() = buf;
  return st;
}

sm_status check_params(const sm_params* p) {
  if (!p) return fail(SM_ERR_ARG, "params is NULL");
  if (p->d_min < 0 || p->d_max < p->d_min || p->d_max > 255)
    return fail(SM_ERR_ARG, "need 0 <= d_min <= d_max <= 255 (got %d, %d)", p->d_min, p->d_max);
  if (!census_ok(p->census_w, p->census_h))
    return fail(SM_ERR_ARG, "census window %dx%d: odd sides in [3, 9], at most 64 bits", p->census_w,
                p->census_h);
  if (p->support_step < 1) return fail(SM_ERR_ARG, "support_step must be >= 1");
  if (p->n_iters < 1 || p->n_iters > 8) return fail(SM_ERR_ARG, "n_iters must be in [1, 8]");
  if (p->t_hi < 0 || p->t_hi > 64 || p->t_lo < 0 || p->t_lo > p->t_hi)
    return fail(SM_ERR_ARG, "need 0 <= t_lo <= t_hi <= 64 (got %d, %d)", p->t_lo, p->t_hi);
  if (p->grad_thr < 0) return fail(SM_ERR_ARG, "grad_thr must be >= 0");
  if (p->lr_tol < 0) return fail(SM_ERR_ARG, "lr_tol must be >= 0");
  if (p->uniqueness < 0 || p->uniqueness > 64) return fail(SM_ERR_ARG, "uniqueness must be in [0, 64]");
  if (p->sz_occ0 < 1 || p->sz_occ0 > 1024) return fail(SM_ERR_ARG, "sz_occ0 must be in [1, 1024]");
  if (p->support_mode != 0 && p->support_mode != 1) return fail(SM_ERR_ARG, "support_mode must be 0 or 1");
  if (p->levels != 1 && p->levels != 3 && p->levels != 5) return fail(SM_ERR_ARG, "levels must be 1, 3 or 5");
  if (p->host_mesh != 0 && p->host_mesh != 1) return fail(SM_ERR_ARG, "host_mesh must be 0 or 1");
  if (p->support_mode == 1) SM_TRY(check_fast_params(p));
  return SM_OK;
}

sm_status check_fast_params(const sm_params* p) {
  if (p->fast_threshold < 0 || p->fast_threshold > 254) return fail(SM_ERR_ARG, "fast_threshold must be in [0, 254]");
  if (p->fast_bins_x < 1 || p->fast_bins_x > 1024 || p->fast_bins_y < 1 || p->fast_bins_y > 1024)
    return fail(SM_ERR_ARG, "fast_bins_x, fast_bins_y must be in [1, 1024]");
  if (p->fast_per_bin < 1 || p->fast_per_bin > 4096) return fail(SM_ERR_ARG, "fast_per_bin must be in [1, 4096]");
  if (fast_slots(*p) > (1 << 22)) return fail(SM_ERR_ARG, "fast_bins_x * fast_bins_y * fast_per_bin exceeds 2^22");
  return SM_OK;
}

namespace {

// ---------------------------------------------------------------------------------
// Per-thread host state of sm_solve: pinned staging, triangulation, timing events.
// Never freed (lives as long as the thread); no HIP call happens at teardown.
// ---------------------------------------------------------------------------------
struct StageTimer {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, int>> marks;  // (stage, event index of the begin event)
  int used = 0;
};

struct ThreadCtx {
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t copy_done = nullptr;  // last host-to-device copy out of `pinned`
  bool copy_pending = false;
  Delaunay dl;
  std::vector<sm_tri> tris;
  std::vector<int32_t> bu, bv, bext;
  StageTimer timer;
};

ThreadCtx& ctx() {
  static thread_local ThreadCtx* c = new ThreadCtx();
  return *c;
}

sm_status ensure_pinned(ThreadCtx& c, size_t bytes) {
  // a previous solve of this thread (possibly on another stream) may still be reading
  // the staging buffer
  if (c.copy_pending) {
    SM_HIP(hipEventSynchronize(c.copy_done));
    c.copy_pending = false;
  }
  if (!c.copy_done) SM_HIP(hipEventCreateWithFlags(&c.copy_done, hipEventDisableTiming));
  if (c.pinned_bytes >= bytes) return SM_OK;
  if (c.pinned) SM_HIP(hipHostFree(c.pinned));
  c.pinned = nullptr;
  c.pinned_bytes = 0;
  size_t want = std::max<size_t>(bytes, 1 << 16);
  SM_HIP(hipHostMalloc(&c.pinned, want, hipHostMallocDefault));
  c.pinned_bytes = want;
  return SM_OK;
}

struct Timer {
  StageTimer& t;
  hipStream_t s;
  bool on;
  uint32_t stages;  // bit k: time the kernels of stage k
  Timer(StageTimer& tt, hipStream_t ss, int32_t timing) : t(tt), s(ss), on(timing != 0) {
    stages = (timing & SM_TIME_SELECTED) ? (uint32_t)timing & 0xffffu : 0xffffu;
    t.used = 0;
    t.marks.clear();
  }
  sm_status event(hipEvent_t* out) {
    if ((size_t)t.used == t.pool.size()) {
      hipEvent_t e;
      SM_HIP(hipEventCreate(&e));
      t.pool.push_back(e);
    }
    *out = t.pool[t.used++];
    return SM_OK;
  }
  // arms an event pair that the next launch records around its kernel
  sm_status begin(int stage) {
    if (!on || !(stages >> stage & 1u)) return SM_OK;
    hipEvent_t e0, e1;
    SM_TRY(event(&e0));
    SM_TRY(event(&e1));
    t.marks.emplace_back(stage, t.used - 2);
    set_launch_events(e0, e1);
    return SM_OK;
  }
  sm_status end() {
    if (!on) return SM_OK;
    if (launch_events_pending()) {  // nothing was launched (or not timed): forget the mark
      set_launch_events(nullptr, nullptr);
      t.marks.pop_back();
      t.used -= 2;
    }
    return SM_OK;
  }
  // after the stream has been synchronised
  sm_status collect(sm_stats* st) {
    if (!on || !st) return SM_OK;
    for (auto& m : t.marks) {
      float ms = 0.f;
      SM_HIP(hipEventElapsedTime(&ms, t.pool[m.second], t.pool[m.second + 1]));
      st->stage_us[m.first] += ms * 1000.f;
      st->stage_launches[m.first] += 1;
    }
    return SM_OK;
  }
};

using clk = std::chrono::steady_clock;
inline float us_since(clk::time_point t0) {
  return std::chrono::duration<float, std::micro>(clk::now() - t0).count();
}

// Workspace layout of sm_solve (256-byte aligned sub-buffers).
sm_status check_image_args(int32_t W, int32_t H) {
  if (!dims_ok(W, H)) return fail(SM_ERR_ARG, "image size %dx%d outside [3, 8192]^2", W, H);
  return SM_OK;
}

}  // namespace


Layout layout_of(int32_t W, int32_t H, const sm_params& p) {
  Layout L{};
  const size_t npx = (size_t)W * H;
  L.n_grid = p.support_mode == 1 ? (int32_t)fast_slots(p) : grid_count(W, H, p.support_step);
  L.cells_max = cells_of(W, H, occ_size(p, p.n_iters));
  // each slot region is followed by one header slot that receives its count
  int64_t scap = L.n_grid + 1;
  for (int it = 1; it < p.n_iters; ++it) scap += 2 * (int64_t)cells_of(W, H, occ_size(p, it)) + 1;
  L.S_cap = (int32_t)std::max<int64_t>(scap, 1);
  L.T_cap = std::max<int32_t>(2 * L.S_cap, 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.cL = take(npx * 8);
  L.cR = take(npx * 8);
  L.omega = take(npx);
  L.occ = take(npx);
  L.D_it = take(npx * 4);
  L.cell_g = take((size_t)L.cells_max * 8);
  L.cell_b = take((size_t)L.cells_max * 8);
  L.S = take((size_t)L.S_cap * sizeof(sm_support));
  L.T = take((size_t)L.T_cap * sizeof(sm_tri));
  L.counters = take(64);
  // device meshes of the frame's tessellations; their status words follow the counters, so
  // that one copy brings both back
  L.mesh_on = p.host_mesh == 0;
  if (L.mesh_on) L.mstatus = take(kMeshStatusWords * sizeof(int32_t));
  L.score = p.support_mode == 1 ? take(npx) : 0;  // FAST scores
  if (L.mesh_on) L.mwork = take(star_work_bytes(W, H, L.S_cap));
  L.total = o;
  return L;
}

namespace {

// Device buffers of one frame inside an sm_solve workspace.
struct FrameBufs {
  uint64_t *cL, *cR;
  uint8_t *omega, *occ;
  float* D_it;
  uint64_t *cell_g, *cell_b;
  sm_support* S;
  sm_tri* T;
  int32_t* counters;
  unsigned long long* n_valid;  // 32 bytes into the counters
  int32_t* mstatus;             // device mesh status words (nullptr without a device mesh)
  StarWork mw;
};

FrameBufs frame_bufs(uint8_t* base, int32_t W, int32_t H, const Layout& Lo) {
  FrameBufs b;
  b.cL = (uint64_t*)(base + Lo.cL);
  b.cR = (uint64_t*)(base + Lo.cR);
  b.omega = base + Lo.omega;
  b.occ = base + Lo.occ;
  b.D_it = (float*)(base + Lo.D_it);
  b.cell_g = (uint64_t*)(base + Lo.cell_g);
  b.cell_b = (uint64_t*)(base + Lo.cell_b);
  b.S = (sm_support*)(base + Lo.S);
  b.T = (sm_tri*)(base + Lo.T);
  b.counters = (int32_t*)(base + Lo.counters);
  b.n_valid = (unsigned long long*)(base + Lo.counters + 32);
  b.mstatus = Lo.mesh_on ? (int32_t*)(base + Lo.mstatus) : nullptr;
  b.mw = Lo.mesh_on ? star_work_at(base + Lo.mwork, W, H, Lo.S_cap) : StarWork{};
  return b;
}

// Census of both images fused with the per-frame initialisation (D_f = 0, C_f = t_hi as
// Alg. 1 starts, occupancy cleared, D_it = NaN -- coverage only grows over the
// iterations, S_it being a subset of S_it+1, so one fill per frame suffices -- the
// support-grid candidate slots and the counters), the FAST candidates when asked, and
// S_1 = SparseStereo over the candidates; the match count lands in the slot after the
// candidates, so that one copy brings both back. `compact` also compacts the matches
// (the device-mesh path compacts them inside its first mesh kernel instead).
sm_status enqueue_census_match(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t stride,
                               const sm_params& p, const Layout& Lo, uint8_t* base, const FrameBufs& b,
                               float* D_f, uint8_t* C_f, bool compact, Timer& tm, hipStream_t s) {
  CensusJob jobs[2] = {{L, stride, b.cL, b.omega}, {R, stride, b.cR, nullptr}};
  const bool fast = p.support_mode == 1;
  CensusExtras ex;
  ex.D_nan = b.D_it;
  ex.grid_slots = fast ? nullptr : b.S;
  ex.step = p.support_step;
  ex.gw = Lo.n_grid > 0 ? (W - 1 - p.support_step / 2) / p.support_step + 1 : 0;
  ex.zero = b.counters;
  ex.n_zero = 16;
  SM_TRY(tm.begin(SM_ST_CENSUS));
  SM_HIP(launch_census(jobs, 2, W, H, p.census_w, p.census_h, p.grad_thr, D_f, C_f, p.t_hi, b.occ, &ex, s));
  SM_TRY(tm.end());
  if (fast) {  // FAST keypoints from spatial bins as the candidates (Sec. III-A)
    SM_TRY(tm.begin(SM_ST_FAST));
    SM_HIP(launch_fast_score(L, stride, W, H, base + Lo.score, s));
    SM_TRY(tm.end());
    SM_TRY(tm.begin(SM_ST_FAST));
    SM_HIP(launch_fast_select(base + Lo.score, W, H, p, b.S, nullptr, s));
    SM_TRY(tm.end());
  }
  SM_TRY(tm.begin(SM_ST_MATCH));
  SM_HIP(launch_match(b.cL, b.cR, W, H, p, b.S, Lo.n_grid, s));
  SM_TRY(tm.end());
  if (compact) {
    SM_TRY(tm.begin(SM_ST_COMPACT));
    SM_HIP(launch_compact(b.S, Lo.n_grid, &b.counters[0], b.occ, W, (int32_t*)(b.S + Lo.n_grid), s));
    SM_TRY(tm.end());
  }
  return SM_OK;
}

// The rest of a frame whose every tessellation runs on the device: each tessellation of
// S_it is built from scratch by the per-point star kernels (star.hpp), after its new
// supports are compacted (the matched candidates, then each iteration's resampled ones),
// and every star rasterises its own triangles into D_it as soon as it has them (the
// interpolation of Alg. 1 needs no launch of its own). The counts stay on the device (read
// by the resampling and mesh kernels), so nothing here waits for the device; the caller
// reads the counters and status words back.
sm_status enqueue_device_meshes(const sm_params& p, int32_t W, int32_t H, const Layout& Lo, const FrameBufs& b,
                                float* D_f, uint8_t* C_f, uint8_t* mask, Timer& tm, hipStream_t s) {
  auto star_job = [&](int32_t first, int32_t compact_n, int32_t* compact_count) {
    StarJob job;
    job.S = b.S;
    job.first = first;
    job.compact_n = compact_n;
    job.occ = b.occ;
    job.compact_count = compact_count;
    job.n_new = nullptr;
    job.status = b.mstatus;
    job.status_copy = nullptr;
    job.T = b.T;
    job.T_cap = Lo.T_cap;
    job.W = W;
    job.H = H;
    job.blocks = star_blocks(Lo.S_cap);
    job.w = b.mw;
    job.D = b.D_it;  // each star rasterises its triangles: no raster launch
    return job;
  };
  const int32_t* counts = b.mstatus;
  SM_TRY(tm.begin(SM_ST_MESH));
  SM_HIP(launch_star(star_job(1, Lo.n_grid, &b.counters[0]), s));  // S_1: the matched candidates
  SM_TRY(tm.end());
  for (int it = 1; it <= p.n_iters; ++it) {
    const int32_t sz = occ_size(p, it);
    const bool last = it == p.n_iters;
    SM_TRY(tm.begin(SM_ST_VALIDATE));
    SM_HIP(launch_validate_only(b.cL, b.cR, b.omega, b.D_it, W, H, p, sz, nullptr, D_f, C_f, b.cell_g, b.cell_b,
                                last ? mask : nullptr, last ? b.n_valid : nullptr, s));
    SM_TRY(tm.end());
    if (last) break;
    const int32_t cells = cells_of(W, H, sz);
    SM_TRY(tm.begin(SM_ST_REMATCH));
    SM_HIP(launch_resample(b.cL, b.cR, b.cell_g, b.cell_b, b.D_it, W, H, sz, p, b.S, b.occ, s, counts + kMeshSupports,
                           Lo.S_cap));
    SM_TRY(tm.end());
    SM_TRY(tm.begin(SM_ST_MESH));  // S_it+1 = S_it and the resampled supports
    SM_HIP(launch_star(star_job(0, 2 * cells, &b.counters[1]), s));
    SM_TRY(tm.end());
  }
  return SM_OK;
}

// Bytes from the counters to the end of the mesh status words: one copy brings back the
// valid-pixel count and the frame's mesh record.
inline size_t status_span(const Layout& Lo) { return Lo.mstatus - Lo.counters + kMeshStatusWords * sizeof(int32_t); }

// Per-frame counts of a device-mesh frame from its read-back span.
void device_frame_stats(const sm_params& p, const uint8_t* span, const Layout& Lo, sm_stats* st) {
  const int32_t* ms = (const int32_t*)(span + (Lo.mstatus - Lo.counters));
  for (int k = 0; k < p.n_iters && k < 8; ++k) {
    st->n_support[k] = ms[kMeshLog + 2 * k];
    st->n_tris[k] = star_log_tris(ms, k, p.n_iters);
  }
  st->mesh_device = p.n_iters;
  unsigned long long nv = 0;
  std::memcpy(&nv, span + 32, sizeof(nv));  // n_valid sits 32 bytes into the counters
  st->n_valid = (int64_t)nv;
}

}  // namespace

// Workspace of sm_solve_noalloc: one per GPU, held until the process ends. In host code
// `scratch` names a host-side stand-in, never the device memory: its device address comes
// from hipGetSymbolAddress, once per device (noalloc_workspace below).
static __device__ __align__(256) uint8_t scratch[SM_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's `scratch` (looked up on the first call made with
// that device current).
sm_status noalloc_workspace(void** out) {
  int dev = -1;
  SM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SM_ERR_ARG, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SM_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SM_OK;
}

}  // namespace
}  // namespace sm

using namespace sm;

extern "C" {

const char* sm_last_error(void) { return last_error().c_str(); }

const char* sm_version(void) { return "stereomesh 0.1 gfx950"; }

int32_t sm_grid_candidates(int32_t W, int32_t H, int32_t support_step) {
  if (W <= 0 || H <= 0 || support_step < 1) return 0;
  return grid_count(W, H, support_step);
}

int32_t sm_cells(int32_t W, int32_t H, int32_t sz_occ) {
  if (W <= 0 || H <= 0 || sz_occ < 1) return 0;
  return cells_of(W, H, sz_occ);
}

sm_status sm_census(const uint8_t* img, int32_t W, int32_t H, int32_t stride, int32_t census_w,
                    int32_t census_h, int32_t grad_thr, uint64_t* census, uint8_t* omega,
                    void* stream) {
  last_error().clear();
  SM_TRY(check_image_args(W, H));
  if (!img || !census) return fail(SM_ERR_ARG, "img and census must be non-NULL");
  if (stride < W) return fail(SM_ERR_ARG, "stride %d < W %d", stride, W);
  if (!census_ok(census_w, census_h)) return fail(SM_ERR_ARG, "bad census window %dx%d", census_w, census_h);
  if (grad_thr < 0) return fail(SM_ERR_ARG, "grad_thr must be >= 0");
  CensusJob j{img, stride, census, omega};
  SM_HIP(launch_census(&j, 1, W, H, census_w, census_h, grad_thr, nullptr, nullptr, 0, nullptr,
                       nullptr, (hipStream_t)stream));
  return SM_OK;
}

sm_status sm_match_support(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega, int32_t W,
                           int32_t H, const int16_t* cand_uv, int32_t n_cand, const sm_params* p,
                           sm_support* out, int32_t cap, int32_t* n_out, void* stream) {
  last_error().clear();
  SM_TRY(check_image_args(W, H));
  SM_TRY(check_params(p));
  if (!cL || !cR || !out || !n_out) return fail(SM_ERR_ARG, "cL, cR, out and n_out must be non-NULL");
  int32_t n;
  if (cand_uv) {
    if (n_cand < 0) return fail(SM_ERR_ARG, "n_cand must be >= 0");
    n = n_cand;
  } else {
    if (!omega) return fail(SM_ERR_ARG, "omega is required for grid candidates");
    n = grid_count(W, H, p->support_step);
  }
  if (cap < n) return fail(SM_ERR_CAPACITY, "cap %d < %d candidates", cap, n);
  hipStream_t s = (hipStream_t)stream;
  if (cand_uv) SM_HIP(launch_list_slots(cand_uv, n, out, s));
  else SM_HIP(launch_grid_slots(omega, W, H, p->support_step, out, n, s));
  SM_HIP(launch_match(cL, cR, W, H, *p, out, n, s));
  SM_HIP(launch_compact(out, n, n_out, nullptr, W, nullptr, s));
  return SM_OK;
}

sm_status sm_triangulate(const sm_support* S, int32_t n, sm_tri* tris, int32_t cap, int32_t* n_tris) {
  last_error().clear();
  if (n < 0 || (n > 0 && !S) || !n_tris) return fail(SM_ERR_ARG, "bad support array / count");
  try {
    for (int32_t i = 0; i < n; ++i)
      if (S[i].u < 0 || S[i].v < 0 || S[i].u > 8191 || S[i].v > 8191)
        return fail(SM_ERR_ARG, "support %d at (%d, %d) outside [0, 8191]^2", i, S[i].u, S[i].v);
    // keep the first occurrence of every pixel (the insertion order is randomised below)
    std::vector<uint64_t> key(n);
    for (int32_t i = 0; i < n; ++i)
      key[i] = ((uint64_t)(uint16_t)S[i].v << 48) | ((uint64_t)(uint16_t)S[i].u << 32) | (uint32_t)i;
    std::sort(key.begin(), key.end());
    std::vector<int32_t> u, v, ext;
    u.reserve(n);
    v.reserve(n);
    ext.reserve(n);
    for (int32_t k = 0; k < n; ++k) {
      if (k > 0 && (key[k] >> 32) == (key[k - 1] >> 32)) continue;
      const int32_t i = (int32_t)(key[k] & 0xffffffffu);
      u.push_back(S[i].u);
      v.push_back(S[i].v);
      ext.push_back(i);
    }
    Delaunay dl;
    dl.insert_many(u.data(), v.data(), ext.data(), (int32_t)u.size());
    std::vector<sm_tri> out;
    dl.emit(out, true);
    *n_tris = (int32_t)out.size();
    if ((int32_t)out.size() > cap) return fail(SM_ERR_CAPACITY, "need %zu triangles, cap %d", out.size(), cap);
    if (!out.empty()) std::memcpy(tris, out.data(), out.size() * sizeof(sm_tri));
  } catch (const std::bad_alloc&) {
    return fail(SM_ERR_INTERNAL, "out of host memory");
  } catch (...) {
    return fail(SM_ERR_INTERNAL, "unexpected exception in triangulation");
  }
  return SM_OK;
}

sm_status sm_fast_candidates(const uint8_t* img, int32_t W, int32_t H, int32_t stride, const sm_params* p,
                             uint8_t* score, int16_t* cand_uv, int32_t cap, int32_t* n_out, void* stream) {
  last_error().clear();
  SM_TRY(check_image_args(W, H));
  if (stride < W) return fail(SM_ERR_ARG, "stride %d < W %d", stride, W);
  if (!img || !score || !cand_uv || !n_out) return fail(SM_ERR_ARG, "NULL buffer");
  if (!p) return fail(SM_ERR_ARG, "params is NULL");
  SM_TRY(check_fast_params(p));
  const int64_t slots = fast_slots(*p);
  if (cap < slots) return fail(SM_ERR_CAPACITY, "cap %d < %lld candidate slots", cap, (long long)slots);
  const hipStream_t s = (hipStream_t)stream;
  SM_HIP(launch_fast_score(img, stride, W, H, score, s));
  SM_HIP(launch_fast_select(score, W, H, *p, nullptr, cand_uv, s));
  SM_HIP(launch_compact_uv(cand_uv, (int32_t)slots, n_out, s));
  return SM_OK;
}

sm_status sm_interpolate(const sm_support* S, int32_t n_support, const sm_tri* T, int32_t n_tris,
                         int32_t W, int32_t H, float* D_it, void* stream) {
  last_error().clear();
  SM_TRY(check_image_args(W, H));
  if (!D_it) return fail(SM_ERR_ARG, "D_it must be non-NULL");
  if (n_tris < 0 || n_support < 0) return fail(SM_ERR_ARG, "negative count");
  if (n_tris > 0 && (!S || !T)) return fail(SM_ERR_ARG, "S and T must be non-NULL");
  SM_HIP(launch_interpolate(S, n_support, T, n_tris, W, H, D_it, (hipStream_t)stream));
  return SM_OK;
}

sm_status sm_validate(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega, const float* D_it,
                      int32_t W, int32_t H, const sm_params* p, int32_t sz_occ, uint8_t* C_it,
                      float* D_f, uint8_t* C_f, uint64_t* cell_g, uint64_t* cell_b, void* stream) {
  last_error().clear();
  SM_TRY(check_image_args(W, H));
  SM_TRY(check_params(p));
  if (!cL || !cR || !omega || !D_it || !D_f || !C_f || !cell_g || !cell_b)
    return fail(SM_ERR_ARG, "only C_it may be NULL");
  if (sz_occ < 1 || sz_occ > 8192) return fail(SM_ERR_ARG, "sz_occ must be in [1, 8192]");
  SM_HIP(launch_validate(cL, cR, omega, D_it, W, H, *p, sz_occ, C_it, D_f, C_f, cell_g, cell_b, nullptr,
                         nullptr, (hipStream_t)stream));
  return SM_OK;
}

sm_status sm_resample(const uint64_t* cL, const uint64_t* cR, const float* D_it, const uint64_t* cell_g,
                      const uint64_t* cell_b, int32_t W, int32_t H, int32_t sz_occ, const sm_params* p,
                      const sm_support* S, int32_t n_S, uint8_t* occ, sm_support* out, int32_t cap,
                      int32_t* n_out, void* stream) {
  last_error().clear();
  SM_TRY(check_image_args(W, H));
  SM_TRY(check_params(p));
  if (!cL || !cR || !D_it || !cell_g || !cell_b || !occ || !out || !n_out)
    return fail(SM_ERR_ARG, "only S may be NULL (when n_S == 0)");
  if (n_S < 0 || (n_S > 0 && !S)) return fail(SM_ERR_ARG, "bad support array / count");
  if (sz_occ < 1 || sz_occ > 8192) return fail(SM_ERR_ARG, "sz_occ must be in [1, 8192]");
  const int32_t cells = cells_of(W, H, sz_occ);
  if (cap < 2 * cells) return fail(SM_ERR_CAPACITY, "cap %d < 2 * %d cells", cap, cells);
  hipStream_t s = (hipStream_t)stream;
  SM_HIP(launch_mark(S, n_S, occ, W, H, s));
  SM_HIP(launch_resample(cL, cR, cell_g, cell_b, D_it, W, H, sz_occ, *p, out, occ, s));
  SM_HIP(launch_compact(out, 2 * cells, n_out, occ, W, nullptr, s));
  return SM_OK;
}

size_t sm_solve_workspace_bytes(int32_t W, int32_t H, const sm_params* p) {
  if (!dims_ok(W, H) || check_params(p) != SM_OK) return 0;
  return layout_of(W, H, *p).total;
}

sm_status sm_solve(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t stride,
                   const sm_params* p, void* ws, size_t ws_bytes, float* D_f, uint8_t* C_f,
                   uint8_t* mask, sm_stats* st, void* stream) {
  last_error().clear();
  SM_TRY(check_image_args(W, H));
  SM_TRY(check_params(p));
  if (!L || !R || !ws || !D_f || !C_f || !mask) return fail(SM_ERR_ARG, "only st may be NULL");
  if (stride < W) return fail(SM_ERR_ARG, "stride %d < W %d", stride, W);
  if (((uintptr_t)ws & 255u) != 0) return fail(SM_ERR_ARG, "workspace must be 256-byte aligned");
  const Layout Lo = layout_of(W, H, *p);
  if (ws_bytes < Lo.total) return fail(SM_ERR_CAPACITY, "workspace %zu < %zu bytes", ws_bytes, Lo.total);
  const auto t_start = clk::now();
  hipStream_t s = (hipStream_t)stream;
  ThreadCtx& c = ctx();
  const int32_t timing = st ? st->timing : 0;
  if (st) {
    const int32_t keep = st->timing;
    std::memset(st, 0, sizeof(*st));
    st->timing = keep;
  }
  uint8_t* base = (uint8_t*)ws;
  const FrameBufs b = frame_bufs(base, W, H, Lo);
  uint64_t* cL = b.cL;
  uint64_t* cR = b.cR;
  uint8_t* omega = b.omega;
  uint8_t* occ = b.occ;
  float* D_it = b.D_it;
  uint64_t* cell_g = b.cell_g;
  uint64_t* cell_b = b.cell_b;
  sm_support* Sd = b.S;
  sm_tri* Td = b.T;
  int32_t* counters = b.counters;
  unsigned long long* n_valid = b.n_valid;
  // pinned staging: [counts | supports or triangles | mesh status]
  // (a device-mesh frame also reads its counters and status words back through this region)
  const size_t st_span = Lo.mesh_on ? status_span(Lo) : 0;
  const size_t st_main =
      align256(std::max({(size_t)Lo.S_cap * sizeof(sm_support), (size_t)Lo.T_cap * sizeof(sm_tri), st_span}));
  SM_TRY(ensure_pinned(c, 256 + st_main + kMeshStatusWords * sizeof(int32_t)));
  int32_t* h_count = (int32_t*)c.pinned;
  sm_support* h_S = (sm_support*)((uint8_t*)c.pinned + 256);
  sm_tri* h_T = (sm_tri*)((uint8_t*)c.pinned + 256);
  int32_t* h_mstatus = (int32_t*)((uint8_t*)c.pinned + 256 + st_main);
  Timer tm(c.timer, s, timing);
  float us_host = 0.f, us_xfer = 0.f;

  const bool device_path = Lo.mesh_on;  // every tessellation on the device
  SM_TRY(enqueue_census_match(L, R, W, H, stride, *p, Lo, base, b, D_f, C_f, !device_path, tm, s));

  // Device meshes: the frame needs one synchronisation, at its end. A frame whose device
  // mesh fails is solved again with host meshes.
  if (device_path) {
    SM_TRY(enqueue_device_meshes(*p, W, H, Lo, b, D_f, C_f, mask, tm, s));
    // counters (the valid-pixel count) and status words in one copy
    auto t1 = clk::now();
    const size_t span = status_span(Lo);
    uint8_t* h_span = (uint8_t*)h_S;  // free in this path
    SM_HIP(hipMemcpyAsync(h_span, base + Lo.counters, span, hipMemcpyDeviceToHost, s));
    SM_HIP(hipStreamSynchronize(s));
    us_xfer += us_since(t1);
    std::memcpy(h_mstatus, h_span + (Lo.mstatus - Lo.counters), kMeshStatusWords * sizeof(int32_t));
    if (h_mstatus[kMeshErr] != 0) {  // the frame again, every tessellation on the host
      sm_params q = *p;
      q.host_mesh = 1;
      const sm_status r = sm_solve(L, R, W, H, stride, &q, ws, ws_bytes, D_f, C_f, mask, st, stream);
      if (st) ++st->mesh_fallback;
      return r;
    }
    if (st) {
      device_frame_stats(*p, h_span, Lo, st);
      SM_TRY(tm.collect(st));
      st->stage_us[SM_ST_HOST_TRI] = us_host;
      st->stage_us[SM_ST_HOST_COPY] = us_xfer;
      st->stage_us[SM_ST_TOTAL] = us_since(t_start);
    }
    return SM_OK;
  }

  // Host meshes (host_mesh = 1): the supports come to the host for every tessellation
  auto t0 = clk::now();
  int32_t n_S = -1, n_T = 0;
  SM_HIP(hipMemcpyAsync(h_S, Sd, (size_t)(Lo.n_grid + 1) * sizeof(sm_support), hipMemcpyDeviceToHost, s));
  SM_HIP(hipStreamSynchronize(s));
  us_xfer += us_since(t0);
  std::memcpy(&n_S, &h_S[Lo.n_grid], sizeof(int32_t));
  if (n_S < 0 || n_S > Lo.n_grid) return fail(SM_ERR_INTERNAL, "support count %d out of range", n_S);

  auto triangulate_and_upload = [&](int32_t from, int32_t to) -> sm_status {
    auto th = clk::now();
    try {
      if (from == 0) c.dl.reset();
      const int32_t m = to - from;
      c.bu.resize(m);
      c.bv.resize(m);
      c.bext.resize(m);
      for (int32_t k = 0; k < m; ++k) {
        c.bu[k] = h_S[k].u;
        c.bv[k] = h_S[k].v;
        c.bext[k] = from + k;
      }
      if (!c.dl.insert_many(c.bu.data(), c.bv.data(), c.bext.data(), m))
        return fail(SM_ERR_INTERNAL, "support outside range");
      c.tris.clear();
      c.dl.emit_banded(c.tris, 3);
    } catch (...) {
      return fail(SM_ERR_INTERNAL, "host triangulation failed");
    }
    n_T = (int32_t)c.tris.size();
    if (n_T > Lo.T_cap) return fail(SM_ERR_INTERNAL, "triangle capacity exceeded");
    us_host += us_since(th);
    auto tx = clk::now();
    // the staging buffer is free again: the supports it held were consumed above
    if (n_T > 0) {
      std::memcpy(h_T, c.tris.data(), (size_t)n_T * sizeof(sm_tri));
      SM_HIP(hipMemcpyAsync(Td, h_T, (size_t)n_T * sizeof(sm_tri), hipMemcpyHostToDevice, s));
      SM_HIP(hipEventRecord(c.copy_done, s));
      c.copy_pending = true;
    }
    us_xfer += us_since(tx);
    return SM_OK;
  };
  SM_TRY(triangulate_and_upload(0, n_S));

  for (int it = 1; it <= p->n_iters; ++it) {
    const int32_t sz = occ_size(*p, it);
    const bool last = it == p->n_iters;
    if (st) {
      st->n_support[it - 1] = n_S;
      st->n_tris[it - 1] = n_T;
    }
    if (n_T > 0) {
      SM_TRY(tm.begin(SM_ST_RASTER));
      SM_HIP(launch_raster(Sd, n_S, Td, n_T, W, H, D_it, s));
      SM_TRY(tm.end());
    }
    SM_TRY(tm.begin(SM_ST_VALIDATE));
    SM_HIP(launch_validate_only(cL, cR, omega, D_it, W, H, *p, sz, nullptr, D_f, C_f, cell_g, cell_b,
                                last ? mask : nullptr, last ? n_valid : nullptr, s));
    SM_TRY(tm.end());
    if (last) break;
    // S_it+1 = SupportResampling(C_g, C_b, S_it), appended in place after S_it
    const int32_t cells = cells_of(W, H, sz);
    if (n_S + 2 * cells + 1 > Lo.S_cap) return fail(SM_ERR_INTERNAL, "support capacity exceeded");
    sm_support* region = Sd + n_S;
    SM_TRY(tm.begin(SM_ST_REMATCH));
    SM_HIP(launch_resample(cL, cR, cell_g, cell_b, D_it, W, H, sz, *p, region, occ, s));
    SM_TRY(tm.end());
    SM_TRY(tm.begin(SM_ST_COMPACT));
    SM_HIP(launch_compact(region, 2 * cells, &counters[1], occ, W, (int32_t*)(region + 2 * cells), s));
    SM_TRY(tm.end());
    t0 = clk::now();
    SM_HIP(hipMemcpyAsync(h_S, region, (size_t)(2 * cells + 1) * sizeof(sm_support), hipMemcpyDeviceToHost, s));
    SM_HIP(hipStreamSynchronize(s));
    us_xfer += us_since(t0);
    int32_t n_new;
    std::memcpy(&n_new, &h_S[2 * cells], sizeof(int32_t));
    if (n_new < 0 || n_new > 2 * cells) return fail(SM_ERR_INTERNAL, "resample count %d out of range", n_new);
    SM_TRY(triangulate_and_upload(n_S, n_S + n_new));
    n_S += n_new;
  }
  if (st) {
    t0 = clk::now();
    unsigned long long nv = 0;
    SM_HIP(hipMemcpyAsync(h_count, n_valid, sizeof(nv), hipMemcpyDeviceToHost, s));
    SM_HIP(hipStreamSynchronize(s));
    std::memcpy(&nv, h_count, sizeof(nv));
    us_xfer += us_since(t0);
    st->n_valid = (int64_t)nv;
    SM_TRY(tm.collect(st));
    st->stage_us[SM_ST_HOST_TRI] = us_host;
    st->stage_us[SM_ST_HOST_COPY] = us_xfer;
    st->stage_us[SM_ST_TOTAL] = us_since(t_start);
  }
  return SM_OK;
}


// sm_solve on the library's per-device workspace, allocating nothing: the launch sequence
// of a device-mesh frame, then one read-back of the counters and mesh status words into
// thread-local host memory.
sm_status sm_solve_noalloc(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t stride,
                           const sm_params* p, float* D_f, uint8_t* C_f, uint8_t* mask, sm_stats* st,
                           void* stream) {
  last_error().clear();
  SM_TRY(check_image_args(W, H));
  SM_TRY(check_params(p));
  if (!L || !R || !D_f || !C_f || !mask) return fail(SM_ERR_ARG, "only st may be NULL");
  if (stride < W) return fail(SM_ERR_ARG, "stride %d < W %d", stride, W);
  if (p->host_mesh != 0) return fail(SM_ERR_ARG, "sm_solve_noalloc needs device meshes (host_mesh 0)");
  const Layout Lo = layout_of(W, H, *p);
  if (!Lo.mesh_on) return fail(SM_ERR_INTERNAL, "no device mesh in the layout");
  if (Lo.total > SM_NOALLOC_MAX_BYTES)
    return fail(SM_ERR_CAPACITY, "a %dx%d frame needs a %zu-byte workspace, above the %zu bytes of "
                "sm_solve_noalloc; use sm_solve", W, H, Lo.total, (size_t)SM_NOALLOC_MAX_BYTES);
  static thread_local uint8_t h_span[512];  // counters + mesh status words, read back
  const size_t span = status_span(Lo);
  if (span > sizeof(h_span)) return fail(SM_ERR_INTERNAL, "status span %zu too large", span);
  void* ws = nullptr;
  SM_TRY(noalloc_workspace(&ws));
  const hipStream_t s = (hipStream_t)stream;
  if (st) {
    std::memset(st, 0, sizeof(*st));  // counts only: no timing events are created here
  }
  uint8_t* base = (uint8_t*)ws;
  const FrameBufs b = frame_bufs(base, W, H, Lo);
  StageTimer no_events;
  Timer tm(no_events, s, 0);
  SM_TRY(enqueue_census_match(L, R, W, H, stride, *p, Lo, base, b, D_f, C_f, false, tm, s));
  SM_TRY(enqueue_device_meshes(*p, W, H, Lo, b, D_f, C_f, mask, tm, s));
  SM_HIP(hipMemcpyAsync(h_span, base + Lo.counters, span, hipMemcpyDeviceToHost, s));
  SM_HIP(hipStreamSynchronize(s));
  const int32_t err = ((const int32_t*)(h_span + (Lo.mstatus - Lo.counters)))[kMeshErr];
  if (err != 0)
    return fail(SM_ERR_INTERNAL, "the device mesh could not finish this frame (code %d); sm_solve solves "
                "it with host meshes", err);
  if (st) device_frame_stats(*p, h_span, Lo, st);
  return SM_OK;
}

sm_status sm_set_launch_shape(int32_t kind, int32_t W, int32_t H, int32_t key, int32_t value) {
  last_error().clear();
  SM_TRY(check_image_args(W, H));
  auto one_of = [&](std::initializer_list<int32_t> ok) {
    if (value == 0) return true;
    for (int32_t v : ok)
      if (v == value) return true;
    return false;
  };
  bool ok = false;
  switch (kind) {
    case kTuneValidateWaves: ok = key >= 1 && one_of({1, 2, 4, 8, 16}); break;
    case kTuneRasterBlocks: ok = key == 0 && one_of({512, 1024, 2048, 4096, 8192}); break;
    case kTuneMatchLanes: ok = key >= 1 && key <= 256 && one_of({16, 32, 64}); break;
    case kTuneCensusRows: ok = key >= 0 && one_of({8, 16, 32}); break;
    default: break;
  }
  if (!ok) return fail(SM_ERR_ARG, "launch shape kind %d, key %d, value %d not accepted", kind, key, value);
  set_tuned_choice(kind, W, H, key, value);
  return SM_OK;
}

// Measured launch shapes for one frame size and parameter set (the autotuner of the
// batched and per-frame solves). Each tunable launch's candidates are timed inside whole
// solves of the frame -- every kernel then sees its inputs and the caches as the solve
// leaves them (timed alone, back to back, a kernel finds its inputs in its own L2 and the
// order of the candidates can differ) -- by the device time of the launches they shape
// (events on that stage only: a solve's wall time varies by more than the few microseconds
// between candidates), one launch after another, the others at their current best; the
// fastest is recorded for (W, H[, key]) and later solves of that size use it. The last
// solve leaves the frame's results in D_f, C_f and mask.
sm_status sm_autotune(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t stride,
                      const sm_params* p, void* ws, size_t ws_bytes, float* D_f, uint8_t* C_f, uint8_t* mask,
                      int32_t* choices, void* stream) {
  last_error().clear();
  SM_TRY(check_image_args(W, H));
  SM_TRY(check_params(p));
  if (!choices) return fail(SM_ERR_ARG, "choices is NULL");
  for (int k = 0; k < 11; ++k) choices[k] = 0;
  const Layout Lo = layout_of(W, H, *p);
  struct Knob {
    int kind;
    int32_t key;
    std::vector<int> values;
    int slot;   // in choices
    int stage;  // the sm_stage of the launches it shapes
  };
  std::vector<Knob> knobs;
  knobs.push_back({kTuneCensusRows, ((p->census_w - 1) / 2) << 8 | ((p->census_h - 1) / 2), {8, 16, 32}, 10,
                   SM_ST_CENSUS});
  if (p->support_mode == 0 && Lo.n_grid > 0)
    knobs.push_back({kTuneMatchLanes, p->d_max - p->d_min + 1, {64, 32, 16}, 9, SM_ST_MATCH});
  for (int it = 1; it <= p->n_iters && it <= 8; ++it)
    knobs.push_back({kTuneValidateWaves, occ_size(*p, it), {1, 2, 4, 8, 16}, it - 1, SM_ST_VALIDATE});
  for (const Knob& k : knobs) set_tuned_choice(k.kind, W, H, k.key, 0);  // the built-in rules to start
  SM_TRY(sm_solve(L, R, W, H, stride, p, ws, ws_bytes, D_f, C_f, mask, nullptr, stream));
  // device time of a stage's launches in one solve, from events on those launches only (the
  // rest of the solve runs as usual): the best of 4 runs of 4 solves
  auto time_stage = [&](int stage, double* t) -> sm_status {
    *t = -1.0;
    for (int run = 0; run < 4; ++run) {
      double sum = 0.0;
      for (int r = 0; r < 4; ++r) {
        sm_stats st{};
        st.timing = SM_TIME_SELECTED | (1 << stage);
        SM_TRY(sm_solve(L, R, W, H, stride, p, ws, ws_bytes, D_f, C_f, mask, &st, stream));
        sum += st.stage_us[stage];
      }
      if (*t < 0.0 || sum < *t) *t = sum;
    }
    return SM_OK;
  };
  for (const Knob& k : knobs) {
    int best = 0;
    double best_t = 0.0;
    for (int v : k.values) {
      set_tuned_choice(k.kind, W, H, k.key, v);
      double t = 0.0;
      SM_TRY(time_stage(k.stage, &t));
      if (best == 0 || t < best_t) best = v, best_t = t;
    }
    set_tuned_choice(k.kind, W, H, k.key, best);
    choices[k.slot] = best;
  }
  // the frame's results with the chosen shapes
  return sm_solve(L, R, W, H, stride, p, ws, ws_bytes, D_f, C_f, mask, nullptr, stream);
}

}  // extern "C"
