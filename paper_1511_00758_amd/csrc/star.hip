// Device Delaunay triangulation by per-point stars (Sec. III-A; the steps and why they are
// exact are in mesh_star.hpp): the preparation kernel builds the frame's bucket grid, the
// star kernel runs one star per wavefront (one frame: latency) or per 16-lane group (the
// stage-batched solve: four stars per wavefront, fewer instructions per star) over the
// whole chip.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "mesh_star.hpp"
#include "raster.hpp"
#include "star.hpp"

namespace sm {

namespace {

using geom::P2;
using star::Grid;
using star::Region;

constexpr int kPrepThreads = 1024;
constexpr int kStarWaves = 4;      // wavefronts (supports) per star workgroup
constexpr int kStageCap = 256;     // candidates a wavefront stages in LDS
constexpr int32_t kNoRow = 1 << 30;

__device__ __forceinline__ int32_t pack_uv(int32_t u, int32_t v) { return u | (v << 16); }

// A value the caller knows to be equal on every lane of the wavefront, as a wave-uniform
// (scalar) value: control flow that depends on it compiles to scalar branches.
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  return ((uint64_t)(uint32_t)uniform((int32_t)(v >> 32)) << 32) | (uint32_t)uniform((int32_t)v);
}

// Wavefront-wide scans and reductions on DPP: shifts by 1, 2, 4 and 8 lanes within each
// row of 16, then the broadcasts of lanes 15 and 31 into the following rows; every step is
// one VALU operation with no LDS round trip. All 64 lanes must be active.
template <int Ctrl, int RowMask>
__device__ __forceinline__ int32_t dpp(int32_t old, int32_t v) {
  return __builtin_amdgcn_update_dpp(old, v, Ctrl, RowMask, 0xf, false);
}
// inclusive prefix sum over the lanes
__device__ __forceinline__ int32_t wave_scan(int32_t v) {
  v += dpp<0x111, 0xf>(0, v);  // row_shr:1
  v += dpp<0x112, 0xf>(0, v);  // row_shr:2
  v += dpp<0x114, 0xf>(0, v);  // row_shr:4
  v += dpp<0x118, 0xf>(0, v);  // row_shr:8
  v += dpp<0x142, 0xa>(0, v);  // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xc>(0, v);  // row_bcast:31 into rows 2 and 3
  return v;
}
// minimum over the lanes, as a wave-uniform value (lane 63 ends with it)
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  int32_t v = (int32_t)x;
  auto mn = [](int32_t a, int32_t b) { return (uint32_t)a < (uint32_t)b ? a : b; };
  v = mn(v, dpp<0x111, 0xf>(-1, v));
  v = mn(v, dpp<0x112, 0xf>(-1, v));
  v = mn(v, dpp<0x114, 0xf>(-1, v));
  v = mn(v, dpp<0x118, 0xf>(-1, v));
  v = mn(v, dpp<0x142, 0xa>(-1, v));
  v = mn(v, dpp<0x143, 0xc>(-1, v));
  return (uint32_t)__builtin_amdgcn_readlane(v, 63);
}
// float keys as unsigned integers in the same order (non-negative floats above negative
// ones; NaN does not occur)
__device__ __forceinline__ uint32_t float_key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Writes the status words 0..7 and log entry k to the status and its copy (thread 0).
__device__ void put_status(const StarJob& a, const int32_t (&w)[8], int k, int32_t log_s, int32_t log_t) {
  for (int i = 0; i < 8; ++i) {
    a.status[i] = w[i];
    if (a.status_copy) a.status_copy[i] = w[i];
  }
  if (k >= 0 && k < 8) {
    a.status[kMeshLog + 2 * k] = log_s;
    a.status[kMeshLog + 2 * k + 1] = log_t;
    if (a.status_copy) {
      a.status_copy[kMeshLog + 2 * k] = log_s;
      a.status_copy[kMeshLog + 2 * k + 1] = log_t;
    }
  }
}

// The preparation's loops give thread t the items base + j * kPrepThreads + t, j < kPrepPer,
// of each pass, and issue every load of a pass before the first is used: one memory latency
// per pass instead of one per kPrepThreads items.
constexpr int kPrepPer = 16;
constexpr int32_t kPrepPass = kPrepPer * kPrepThreads;
constexpr int kPrepWaves = kPrepThreads / 64;

// Exclusive prefix sum of cnt[0, n) (LDS or global) into out[0, n] and into cnt itself (the
// fill cursors) by one 1024-thread workgroup: thread t sums its run of consecutive counts,
// a DPP scan and the wave totals place the runs.
__device__ void block_scan(int32_t* cnt, int32_t* out, int32_t n) {
  __shared__ int32_t wsum[kPrepWaves];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int32_t per = (n + kPrepThreads - 1) / kPrepThreads, c0 = tid * per, c1 = min(c0 + per, n);
  int32_t sum = 0;
  for (int32_t c = c0; c < c1; ++c) sum += cnt[c];
  const int32_t inc = wave_scan(sum);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int32_t run = inc - sum;
  for (int k = 0; k < w; ++k) run += wsum[k];
  for (int32_t c = c0; c < c1; ++c) {
    const int32_t v = cnt[c];
    out[c] = run;
    cnt[c] = run;
    run += v;
  }
  if (tid == kPrepThreads - 1) out[n] = run;
}

// The preparation's per-support steps. A support's (u, v) is the first word of its record,
// u in the low half; a support inside the frame has it equal to its packed coordinates.
__device__ __forceinline__ int32_t support_word(const sm_support* S, int32_t i) {
  return reinterpret_cast<const int32_t*>(S)[2 * i];
}
__device__ __forceinline__ bool word_inside(int32_t q, int32_t W, int32_t H) {
  const int32_t u = (int16_t)(q & 0xffff), v = q >> 16;
  return u >= 0 && v >= 0 && u < W && v < H;
}
// Row extremes of the lanes' supports (q >= 0: packed coordinates) by LDS atomics: the lanes
// on the first such lane's row (most of them, for supports in raster order) are reduced over
// the wavefront first and take one atomic each way. All 64 lanes must be active.
__device__ __forceinline__ void row_extremes(int32_t q, int32_t* rmin, int32_t* rmax) {
  const bool ok = q >= 0;
  const uint64_t vm = __ballot(ok);
  if (!vm) return;
  const int32_t qv = q >> 16, qu = q & 0xffff;
  const int32_t rv = __builtin_amdgcn_readlane(qv, __ffsll((long long)vm) - 1);
  const bool same = ok && qv == rv;
  const uint32_t lo = wave_min_u32(same ? (uint32_t)qu : 0xffffffffu);
  const uint32_t hi = ~wave_min_u32(same ? ~(uint32_t)qu : 0xffffffffu);
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&rmin[rv], (int32_t)lo);
    atomicMax(&rmax[rv], (int32_t)hi);
  }
  if (ok && !same) {
    atomicMin(&rmin[qv], qu);
    atomicMax(&rmax[qv], qu);
  }
}
__device__ __forceinline__ void count_cell(const StarWork& w, int32_t q, int32_t* cnt) {
  atomicAdd(&cnt[((q >> 16) / star::kStarCell) * w.gw + (q & 0xffff) / star::kStarCell], 1);
}

// Order-preserving compaction of the slots S[p0, p0 + compact_n) in place, as compact_block
// (slots that hold a match move to the front in order), a pass of kPrepPass slots at a time
// with all their loads in flight together; each kept support is then counted into the
// bucket grid and the row extremes, its packed coordinates written and its pixel marked in
// occ. A slot's place is the count of kept slots before it: earlier passes, then, in its
// pass, earlier rounds j, earlier wavefronts of round j and earlier lanes. Slots whose pixel
// is already a support were emptied by their producer (the re-match reads the occupancy).
// Returns the count (every thread); `bad` is set for a support outside the frame.
__device__ int32_t prep_compact(const StarJob& a, int32_t p0, int32_t* cnt, int32_t* rmin, int32_t* rmax,
                                bool& bad) {
  __shared__ int32_t s_off[kPrepPer * kPrepWaves];  // kept per (round, wavefront), then their offsets
  __shared__ int32_t s_total;
  sm_support* slots = a.S + p0;
  const int32_t n = a.compact_n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  int32_t base = 0;
  for (int32_t start = 0; start < n; start += kPrepPass) {
    sm_support s[kPrepPer];
#pragma unroll
    for (int j = 0; j < kPrepPer; ++j) {
      const int32_t i = start + j * kPrepThreads + tid;
      s[j] = i < n ? slots[i] : sm_support{0, 0, kRejected};
    }
    uint32_t keep = 0;
#pragma unroll
    for (int j = 0; j < kPrepPer; ++j) {
      const bool k = s[j].d != kPending && s[j].d != kRejected;
      keep |= (uint32_t)k << j;
      const uint64_t m = __ballot(k);
      if (lane == 0) s_off[j * kPrepWaves + w] = __popcll(m);
    }
    __syncthreads();
    if (w == 0) {  // exclusive prefix of the (round, wavefront) counts in that order
      constexpr int kPer = kPrepPer * kPrepWaves / 64;
      int32_t v[kPer], sum = 0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) v[k] = s_off[lane * kPer + k], sum += v[k];
      const int32_t inc = wave_scan(sum);
      int32_t run = inc - sum;
#pragma unroll
      for (int k = 0; k < kPer; ++k) s_off[lane * kPer + k] = run, run += v[k];
      if (lane == 63) s_total = inc;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPrepPer; ++j) {
      const bool k = (keep >> j) & 1u;
      const uint64_t m = __ballot(k);
      int32_t q = -1;
      if (k) {
        const int32_t pos = base + s_off[j * kPrepWaves + w] + __popcll(m & below);
        slots[pos] = s[j];
        const int32_t word = (int32_t)(uint16_t)s[j].u | ((int32_t)s[j].v << 16);
        if (word_inside(word, a.W, a.H)) {
          q = word;
          a.w.uv[p0 + pos] = q;
          if (a.occ) a.occ[(size_t)s[j].v * a.W + s[j].u] = 1;
          count_cell(a.w, q, cnt);
        } else {
          bad = true;
        }
      }
      row_extremes(q, rmin, rmax);
    }
    base += s_total;
    __syncthreads();  // (s_off and s_total are rewritten by the next pass)
  }
  return base;
}

// One workgroup per frame: the new supports' compaction, then the frame's bucket grid and
// row extents over all its supports, and its status words for the star kernel. The cell
// counts and row extents are gathered with LDS atomics when they fit (kLds), else in the
// frame's global arrays. The loads of the supports before the new ones are issued first and
// are in flight during the compaction.
constexpr int32_t kLdsCells = 12288;  // cells (48 KiB)
constexpr int32_t kLdsRows = 4096;    // pixel rows (2 x 16 KiB)

template <bool kLds>
__device__ void star_prep(const StarJob& a) {
  const int tid = threadIdx.x;
  const StarWork& w = a.w;
  __shared__ int32_t s_p0, s_err, s_tess, s_n;
  __shared__ int32_t s_cnt[kLds ? kLdsCells : 1];
  __shared__ int32_t s_rmin[kLds ? kLdsRows : 1], s_rmax[kLds ? kLdsRows : 1];
  if (tid == 0) {
    s_p0 = a.first ? 0 : a.status[kMeshSupports];
    s_err = a.first ? 0 : a.status[kMeshErr];
    s_tess = a.first ? 0 : a.status[kMeshTess];
    if (s_err == 0 && (s_p0 < 0 || s_p0 > w.S_cap || (int64_t)s_p0 + a.compact_n + 1 > w.S_cap))
      s_err = star::kStarErrCapacity;
    // without slots to compact the new supports are in place already, counted on the device
    // (no count: none, e.g. a frame too small for any grid candidate)
    int32_t n_new = 0;
    if (s_err == 0 && a.compact_n == 0) {
      n_new = a.n_new ? *a.n_new : 0;
      if (n_new < 0 || (int64_t)s_p0 + n_new > w.S_cap) s_err = star::kStarErrCapacity, n_new = 0;
    }
    s_n = s_p0 + n_new;  // (with slots: completed after the compaction)
  }
  __syncthreads();
  // (a frame whose earlier tessellation failed is redone on the host: uniform from here)
  if (s_err == 0) {
    const int32_t p0 = s_p0;
    const int32_t n_cells = w.gw * w.gh;
    int32_t* cnt = kLds ? s_cnt : w.cell_cur;
    int32_t* rmin = kLds ? s_rmin : w.row_min;
    int32_t* rmax = kLds ? s_rmax : w.row_max;
    const int32_t n_read = a.compact_n > 0 ? p0 : s_n;  // the supports the counting loop reads
    int32_t q[kPrepPer];
#pragma unroll
    for (int j = 0; j < kPrepPer; ++j) {  // its first pass, in flight from here
      const int32_t i = j * kPrepThreads + tid;
      q[j] = i < n_read ? support_word(a.S, i) : 0;
    }
    for (int32_t c = tid; c < n_cells; c += kPrepThreads) cnt[c] = 0;
    for (int32_t v = tid; v < a.H; v += kPrepThreads) rmin[v] = kNoRow, rmax[v] = -1;
    __syncthreads();
    bool bad = false;
    if (a.compact_n > 0) {
      const int32_t kept = prep_compact(a, p0, cnt, rmin, rmax, bad);
      if (tid == 0) {
        *a.compact_count = kept;
        *(int32_t*)(a.S + p0 + a.compact_n) = kept;
        s_n = p0 + kept;
      }
    }
    for (int32_t start = 0; start < n_read; start += kPrepPass) {
      if (start > 0) {
#pragma unroll
        for (int j = 0; j < kPrepPer; ++j) {
          const int32_t i = start + j * kPrepThreads + tid;
          q[j] = i < n_read ? support_word(a.S, i) : 0;
        }
      }
#pragma unroll
      for (int j = 0; j < kPrepPer; ++j) {
        const int32_t i = start + j * kPrepThreads + tid;
        int32_t qj = -1;
        if (i < n_read) {
          if (word_inside(q[j], a.W, a.H)) {
            qj = q[j];
            w.uv[i] = qj;
            count_cell(w, qj, cnt);
          } else {
            bad = true;
          }
        }
        row_extremes(qj, rmin, rmax);
      }
    }
    if (bad) atomicCAS(&s_err, 0, star::kStarErrSupport);
    __syncthreads();
    const int32_t n = s_n;
    if (s_err == 0) {  // (uniform: every thread reads s_err after the barrier)
      block_scan(cnt, w.cell_start, n_cells);
      for (int32_t v = tid; v < a.H; v += kPrepThreads) w.rows[v].lo = rmin[v], w.rows[v].hi = rmax[v];
      __syncthreads();
      for (int32_t start = 0; start < n; start += kPrepPass) {
#pragma unroll
        for (int j = 0; j < kPrepPer; ++j) {
          const int32_t i = start + j * kPrepThreads + tid;
          q[j] = i < n ? w.uv[i] : -1;
        }
#pragma unroll
        for (int j = 0; j < kPrepPer; ++j) {
          const int32_t i = start + j * kPrepThreads + tid;
          if (q[j] < 0) continue;
          const int32_t qu = q[j] & 0xffff, qv = q[j] >> 16;
          const int32_t e = atomicAdd(&cnt[(qv / star::kStarCell) * w.gw + qu / star::kStarCell], 1);
          w.cell_e[e] = star::CellEntry{i, q[j]};
          // the ids of the row's extreme points (one support per pixel: one writer each)
          if (qu == rmin[qv]) w.rows[qv].lo_id = i;
          if (qu == rmax[qv]) w.rows[qv].hi_id = i;
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    // the previous tessellation's triangle count is final now (kernel order): into its log
    if (!a.first && s_tess >= 1 && s_tess <= 8) {
      const int32_t prev = a.status[kMeshTris];
      a.status[kMeshLog + 2 * (s_tess - 1) + 1] = prev;
      if (a.status_copy) a.status_copy[kMeshLog + 2 * (s_tess - 1) + 1] = prev;
    }
    const int32_t words[8] = {0, 0, s_err, 0, s_n - s_p0, s_n, s_tess + 1, 0};
    put_status(a, words, s_tess, s_n, 0);
  }
}

template <bool kLds>
__global__ __launch_bounds__(kPrepThreads) void k_star_prep(StarJob a) {
  star_prep<kLds>(a);
}

template <bool kLds>
__global__ __launch_bounds__(kPrepThreads) void k_star_prep_many(const StarJob* __restrict__ jobs) {
  star_prep<kLds>(jobs[blockIdx.x]);
}

// A wavefront as the group of the star steps; the candidates of the current region are
// staged in LDS when they fit.
struct DevWave {
  static constexpr int kN = 64;
  int lane_;
  int32_t* s_id;
  int32_t* s_uv;
  int32_t* s_mark;        // [kN * kInFlight] run starts of a gather chunk
  int32_t n_staged = -1;  // -1: nothing staged
  int32_t rx0 = 0, rx1 = -1, ry0 = 0, ry1 = -1;

  __device__ int lane() const { return lane_; }
  __device__ bool any(bool b) const { return __ballot(b) != 0; }
  __device__ uint64_t min_u64(uint64_t x) const {
    const uint32_t hi = wave_min_u32((uint32_t)(x >> 32));
    const uint32_t lo = wave_min_u32((uint32_t)(x >> 32) == hi ? (uint32_t)x : 0xffffffffu);
    return ((uint64_t)hi << 32) | lo;
  }
  __device__ int32_t pick(bool mine, int32_t v) const {
    const uint64_t m = __ballot(mine);
    return __builtin_amdgcn_readlane(v, m ? __ffsll((long long)m) - 1 : 0);
  }
  // The group's best of the lanes' bests (every lane ends with it, wave-uniform): the
  // smallest single-precision quotient by a DPP minimum; the other candidates within 2^-19
  // of it (the only ones whose exact quotient can be as small, the rounding being below
  // 5 * 2^-24 of each) are then compared exactly, one after another (usually there are none).
  __device__ void reduce_best(P2 X, P2 Y, int32_t* b, P2* B, float* t) const {
    const uint32_t kmin = wave_min_u32(*b >= 0 ? float_key(*t) : 0xffffffffu);
    if (kmin == 0xffffffffu) {  // no lane has a candidate
      *b = -1;
      return;
    }
    const float tmin = __uint_as_float((kmin & 0x80000000u) ? (kmin & 0x7fffffffu) : ~kmin);
    const bool close = *b >= 0 && *t <= tmin + 0x1p-19f * fabsf(tmin);
    const int w = __ffsll((long long)__ballot(close)) - 1;
    int32_t wb = __builtin_amdgcn_readlane(*b, w);
    P2 WB{__builtin_amdgcn_readlane(B->x, w), __builtin_amdgcn_readlane(B->y, w)};
    float wt = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(*t), w));
    // other candidates as close (many lanes can hold the same one, e.g. a scan's start)
    uint64_t near = __ballot(close && *b != wb);
    while (near) {
      const int c = __ffsll((long long)near) - 1;
      const int32_t cb = __builtin_amdgcn_readlane(*b, c);
      near &= ~__ballot(*b == cb);  // (every lane that holds it)
      const P2 CB{__builtin_amdgcn_readlane(B->x, c), __builtin_amdgcn_readlane(B->y, c)};
      const float ct = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(*t), c));
      if (star::beats(X, Y, wb, WB, wt, cb, CB, ct)) wb = cb, WB = CB, wt = ct;
    }
    *b = wb;
    *B = WB;
    *t = wt;
  }
  // Visits the entries of n cell runs (row(i) gives run i), 64 runs at a time: lane i sets
  // up run i (its two cell_start reads, all lanes at once), a prefix sum over the lanes
  // places the runs end to end, and every lane then takes entries j = lane, lane + 64, ...
  // of the chunk. A lane finds the run of its entry from the chunk's run starts, marked in
  // LDS: the last start at or before it (or the run carried over from the previous 64).
  // The loads of kInFlight such rounds are issued before the first is used (one memory
  // latency per 64 * kInFlight entries). fn2(j, id, uv) gets the entry's position in the
  // chunk, its point id and its packed coordinates. Control flow stays uniform.
  static constexpr int kInFlight = 2;
  static constexpr int32_t kNoMark = INT32_MIN;
  __device__ static void wave_sync() {  // a wavefront's LDS writes before its lanes read them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  template <class RowFn, class Fn2>
  __device__ int32_t gather(const Grid& g, int32_t n, RowFn&& row, Fn2&& fn2) const {
    int32_t all = 0;
    for (int32_t base = 0; base < n; base += kN) {
      const int32_t i = base + lane_;
      int32_t e0 = 0, len = 0;
      if (i < n) {
        const star::CellRow c = row(i);
        if (c.x0 <= c.x1) {
          e0 = g.cell_start[c.cy * g.gw + c.x0];
          len = g.cell_start[c.cy * g.gw + c.x1 + 1] - e0;
        }
      }
      const int32_t inc = wave_scan(len);
      const int32_t exc = inc - len;
      const int32_t total = __builtin_amdgcn_readlane(inc, kN - 1);
      const int32_t delta = e0 - exc;  // entry j of this lane's run is cell entry j + delta
      int32_t carry = 0;               // delta of the run that covers a chunk's first entry
      for (int32_t j0 = 0; j0 < total; j0 += kN * kInFlight) {
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) s_mark[u * kN + lane_] = kNoMark;
        wave_sync();
        if (len > 0 && exc >= j0 && exc < j0 + kN * kInFlight) s_mark[exc - j0] = delta;
        wave_sync();
        int32_t id[kInFlight], uv[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
          id[u] = -1, uv[u] = 0;
          if (j0 + u * kN >= total) continue;  // (uniform)
          const int32_t d = s_mark[u * kN + lane_];
          const uint64_t has = __ballot(d != kNoMark);
          const uint64_t upto = has & (lane_ == kN - 1 ? ~0ull : ((2ull << lane_) - 1));
          const int32_t src = upto ? 63 - __clzll((long long)upto) : 0;
          const int32_t from = __shfl(d, src);
          const int32_t dj = upto ? from : carry;
          if (has) carry = __builtin_amdgcn_readlane(d, 63 - __clzll((long long)has));
          const int32_t j = j0 + u * kN + lane_;
          if (j < total) {
            const star::CellEntry ce = g.cell_e[j + dj];
            id[u] = ce.id, uv[u] = ce.uv;
          }
        }
        // one call site of fn2: the rounds move down the registers
#pragma unroll 1
        for (int u = 0; u < kInFlight && j0 + u * kN < total; ++u) {
          const int32_t j = j0 + u * kN + lane_;
          if (j < total) fn2(all + j, id[0], uv[0]);
#pragma unroll
          for (int k = 0; k + 1 < kInFlight; ++k) id[k] = id[k + 1], uv[k] = uv[k + 1];
        }
        wave_sync();  // (the marks are rewritten by the next chunk)
      }
      all += total;
    }
    return all;
  }
  template <class RowFn, class Fn>
  __device__ void for_rows(const Grid& g, int32_t n, RowFn&& row, Fn&& fn) {
    gather(g, n, row, [&](int32_t, int32_t id, int32_t uv) { fn(id, star::unpack(uv)); });
  }
  // the walk's square: its points into LDS when they fit
  __device__ void set_base(const Grid& g, const Region& r) {
    if (n_staged >= 0 && r.x0 == rx0 && r.x1 == rx1 && r.y0 == ry0 && r.y1 == ry1) return;
    rx0 = r.x0, rx1 = r.x1, ry0 = r.y0, ry1 = r.y1;
    int32_t* sid = s_id;
    int32_t* suv = s_uv;
    n_staged = gather(g, r.y1 - r.y0 + 1, star::RegionRows{r}, [&](int32_t j, int32_t id, int32_t uv) {
      if (j < kStageCap) sid[j] = id, suv[j] = uv;
    });
    wave_sync();  // the staged entries before any lane reads another lane's
  }
  template <class Fn>
  __device__ void for_candidates(const Grid& g, const Region& r, Fn&& fn) {
    if (n_staged >= 0 && n_staged <= kStageCap && r.x0 == rx0 && r.x1 == rx1 && r.y0 == ry0 && r.y1 == ry1) {
      for (int32_t j = lane_; j < n_staged; j += kN) fn(s_id[j], star::unpack(s_uv[j]));
    } else {
      for_rows(g, r.y1 - r.y0 + 1, star::RegionRows{r}, fn);
    }
  }
};

// DPP all-reduce within each row of 16 lanes (every lane of the row ends with the result):
// adjacent pairs, quads, the mirrored half-rows, the mirrored rows.
__device__ __forceinline__ uint32_t row_min_u32(uint32_t x) {
  int32_t v = (int32_t)x;
  auto mn = [](int32_t a, int32_t b) { return (uint32_t)a < (uint32_t)b ? a : b; };
  v = mn(v, dpp<0xb1, 0xf>(-1, v));   // quad_perm [1, 0, 3, 2]
  v = mn(v, dpp<0x4e, 0xf>(-1, v));   // quad_perm [2, 3, 0, 1]
  v = mn(v, dpp<0x141, 0xf>(-1, v));  // row_half_mirror
  v = mn(v, dpp<0x140, 0xf>(-1, v));  // row_mirror
  return (uint32_t)v;
}
// inclusive prefix sum within each row of 16 lanes
__device__ __forceinline__ int32_t row_scan(int32_t v) {
  v += dpp<0x111, 0xf>(0, v);  // row_shr:1
  v += dpp<0x112, 0xf>(0, v);  // row_shr:2
  v += dpp<0x114, 0xf>(0, v);  // row_shr:4
  v += dpp<0x118, 0xf>(0, v);  // row_shr:8
  return v;
}

// A group of 16 lanes -- one DPP row -- as the group of the star steps: four stars per
// wavefront, for throughput (the stage-batched solve). Control flow is uniform per group,
// not per wavefront, so nothing here is made wave-uniform; values move between lanes of a
// group by DPP within the row or by ds_bpermute.
struct DevGroup16 {
  static constexpr int kN = 16;
  static constexpr int kInFlight = 2;
  static constexpr int kCap = 128;  // candidates a group stages in LDS
  int lane_;                        // 0..15
  int gbase;                        // first lane of the group in the wavefront
  int32_t* s_id;
  int32_t* s_uv;
  int32_t* s_mark;                  // [kN * kInFlight]
  int32_t n_staged = -1;
  int32_t rx0 = 0, rx1 = -1, ry0 = 0, ry1 = -1;

  __device__ int lane() const { return lane_; }
  __device__ uint32_t mask(bool b) const { return (uint32_t)((__ballot(b) >> gbase) & 0xffffu); }
  __device__ bool any(bool b) const { return mask(b) != 0u; }
  __device__ uint64_t min_u64(uint64_t x) const {
    const uint32_t hi = row_min_u32((uint32_t)(x >> 32));
    const uint32_t lo = row_min_u32((uint32_t)(x >> 32) == hi ? (uint32_t)x : 0xffffffffu);
    return ((uint64_t)hi << 32) | lo;
  }
  __device__ int32_t pick(bool mine, int32_t v) const {
    const uint32_t m = mask(mine);
    return __shfl(v, gbase + (m ? __ffs(m) - 1 : 0));
  }
  // as DevWave::reduce_best, within the group
  __device__ void reduce_best(P2 X, P2 Y, int32_t* b, P2* B, float* t) const {
    const uint32_t kmin = row_min_u32(*b >= 0 ? float_key(*t) : 0xffffffffu);
    if (kmin == 0xffffffffu) {
      *b = -1;
      return;
    }
    const float tmin = __uint_as_float((kmin & 0x80000000u) ? (kmin & 0x7fffffffu) : ~kmin);
    const bool close = *b >= 0 && *t <= tmin + 0x1p-19f * fabsf(tmin);
    const int w = gbase + __ffs(mask(close)) - 1;
    int32_t wb = __shfl(*b, w);
    P2 WB{__shfl(B->x, w), __shfl(B->y, w)};
    float wt = __shfl(*t, w);
    uint32_t near = mask(close && *b != wb);
    while (near) {
      const int c = gbase + __ffs(near) - 1;
      const int32_t cb = __shfl(*b, c);
      const P2 CB{__shfl(B->x, c), __shfl(B->y, c)};
      const float ct = __shfl(*t, c);
      near &= ~mask(*b == cb);
      if (star::beats(X, Y, wb, WB, wt, cb, CB, ct)) wb = cb, WB = CB, wt = ct;
    }
    *b = wb;
    *B = WB;
    *t = wt;
  }
  // as DevWave::gather, 16 runs and 16 entries per round
  template <class RowFn, class Fn2>
  __device__ int32_t gather(const Grid& g, int32_t n, RowFn&& row, Fn2&& fn2) const {
    int32_t all = 0;
    for (int32_t base = 0; base < n; base += kN) {
      const int32_t i = base + lane_;
      int32_t e0 = 0, len = 0;
      if (i < n) {
        const star::CellRow c = row(i);
        if (c.x0 <= c.x1) {
          e0 = g.cell_start[c.cy * g.gw + c.x0];
          len = g.cell_start[c.cy * g.gw + c.x1 + 1] - e0;
        }
      }
      const int32_t inc = row_scan(len);
      const int32_t exc = inc - len;
      const int32_t total = __shfl(inc, gbase + kN - 1);
      const int32_t delta = e0 - exc;
      int32_t carry = 0;
      for (int32_t j0 = 0; j0 < total; j0 += kN * kInFlight) {
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) s_mark[u * kN + lane_] = kNoMark16;
        DevWave::wave_sync();
        if (len > 0 && exc >= j0 && exc < j0 + kN * kInFlight) s_mark[exc - j0] = delta;
        DevWave::wave_sync();
        int32_t id[kInFlight], uv[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
          id[u] = -1, uv[u] = 0;
          if (j0 + u * kN >= total) continue;  // (uniform in the group)
          const int32_t d = s_mark[u * kN + lane_];
          const uint32_t has = mask(d != kNoMark16);
          const uint32_t upto = has & (lane_ == kN - 1 ? 0xffffu : ((2u << lane_) - 1));
          const int32_t from = __shfl(d, gbase + (upto ? 31 - __clz(upto) : 0));
          const int32_t last = __shfl(d, gbase + (has ? 31 - __clz(has) : 0));
          const int32_t dj = upto ? from : carry;
          if (has) carry = last;
          const int32_t j = j0 + u * kN + lane_;
          if (j < total) {
            const star::CellEntry ce = g.cell_e[j + dj];
            id[u] = ce.id, uv[u] = ce.uv;
          }
        }
#pragma unroll 1
        for (int u = 0; u < kInFlight && j0 + u * kN < total; ++u) {
          const int32_t j = j0 + u * kN + lane_;
          if (j < total) fn2(all + j, id[0], uv[0]);
#pragma unroll
          for (int k = 0; k + 1 < kInFlight; ++k) id[k] = id[k + 1], uv[k] = uv[k + 1];
        }
        DevWave::wave_sync();
      }
      all += total;
    }
    return all;
  }
  static constexpr int32_t kNoMark16 = INT32_MIN;
  template <class RowFn, class Fn>
  __device__ void for_rows(const Grid& g, int32_t n, RowFn&& row, Fn&& fn) {
    gather(g, n, row, [&](int32_t, int32_t id, int32_t uv) { fn(id, star::unpack(uv)); });
  }
  __device__ void set_base(const Grid& g, const Region& r) {
    if (n_staged >= 0 && r.x0 == rx0 && r.x1 == rx1 && r.y0 == ry0 && r.y1 == ry1) return;
    rx0 = r.x0, rx1 = r.x1, ry0 = r.y0, ry1 = r.y1;
    int32_t* sid = s_id;
    int32_t* suv = s_uv;
    n_staged = gather(g, r.y1 - r.y0 + 1, star::RegionRows{r}, [&](int32_t j, int32_t id, int32_t uv) {
      if (j < kCap) sid[j] = id, suv[j] = uv;
    });
    DevWave::wave_sync();
  }
  template <class Fn>
  __device__ void for_candidates(const Grid& g, const Region& r, Fn&& fn) {
    if (n_staged >= 0 && n_staged <= kCap && r.x0 == rx0 && r.x1 == rx1 && r.y0 == ry0 && r.y1 == ry1) {
      for (int32_t j = lane_; j < n_staged; j += kN) fn(s_id[j], star::unpack(s_uv[j]));
    } else {
      for_rows(g, r.y1 - r.y0 + 1, star::RegionRows{r}, fn);
    }
  }
};

// Triangles of one star: lane k holds the k-th pending one. The workgroup reserves the
// slots of all its stars' pending triangles at its end, with one atomic on the frame's
// counter (every wavefront adding its own would serialise thousands of same-address
// atomics); a star with more triangles than its group has lanes reserves each full set
// on its own.
constexpr int kFlushSets = 15;  // full sets a 16-lane group's star records for its rasterisation
template <int G>
struct DevOut {
  int lane;   // in the group
  int gbase;  // first lane of the group in the wavefront
  int32_t p;
  sm_tri* T;
  int32_t T_cap;
  int32_t* counter;
  int32_t* counter_copy;  // nullable: the same count in the status copy
  int32_t* err;
  int32_t n = 0, total = 0;
  int32_t my1 = 0, my2 = 0;
  int32_t fl = 0, nfl = 0;  // a wavefront's full sets written so far: lane k holds set k's first slot
  int32_t* fl_list = nullptr;  // a 16-lane group's (nullable, in LDS): [0] its full sets written
                               // so far, [1 + k] set k's first slot (k < kFlushSets)
  __device__ void begin() { n = 0; }
  __device__ void write(int32_t slot) {
    if (lane < n) {
      if (slot + lane < T_cap) T[slot + lane] = sm_tri{p, my1, my2};
      else atomicCAS(err, 0, star::kStarErrCapacity);
    }
  }
  __device__ void flush() {  // a full set, at once
    int32_t slot = 0;
    if (lane == 0) {
      slot = atomicAdd(counter, n);
      if (counter_copy) atomicAdd(counter_copy, n);
    }
    slot = __shfl(slot, gbase);
    write(G == 64 ? uniform(slot) : slot);
    if constexpr (G == 64) {
      if (lane == nfl) fl = slot;
      ++nfl;
    } else {
      if (fl_list && lane == 0) {
        const int32_t k = fl_list[0];
        if (k < kFlushSets) fl_list[1 + k] = slot;
        fl_list[0] = k + 1;
      }
    }
    total += n;
    n = 0;
  }
  __device__ void emit(int32_t i1, int32_t i2) {
    if (lane == n) my1 = i1, my2 = i2;
    if (++n == G) flush();
  }
  // the star's count; its last n triangles wait for the workgroup's reservation
  __device__ int32_t finish() { return total + n; }
};

// Rasterisation of the triangles of a workgroup's stars (the job names D_it), once its
// last walk has ended: the triangles its reservation placed in T[base, base + n), sixteen
// at a time, a 16-lane group each taking every 16th row of one (the waves that finished
// early share the slow stars' long triangles), after each wavefront's full sets written
// earlier (a star with more triangles than lanes). Every pixel is owned by one triangle of
// the mesh, so D_it does not depend on which lanes write it, or when.
__device__ void raster_sets(const StarJob& a, const DevOut<64>& out, int32_t n_support, int lane) {
  const int gi = lane >> 4, rl = lane & 15;
  for (int32_t f = 0; f < out.nfl && f < 64; ++f) {
    const int32_t slot = __builtin_amdgcn_readlane(out.fl, f);
    for (int32_t k0 = 0; k0 < 64; k0 += 4) {
      const int32_t t = slot + k0 + gi;
      if (t < a.T_cap) raster_rows(raster_setup(a.S, n_support, a.T, t, a.W, a.H), rl, 16, a.W, a.D);
    }
  }
}
__device__ void raster_block(const StarJob& a, int32_t base, int32_t n, int32_t n_support) {
  constexpr int kTris = 64 * kStarWaves / 16;  // (a star workgroup: 256 lanes)
  const int rl = threadIdx.x & 15;
  for (int32_t k0 = 0; k0 < n; k0 += kTris) {
    const int32_t k = k0 + (int32_t)(threadIdx.x >> 4);
    if (k < n && base + k < a.T_cap)
      raster_rows(raster_setup(a.S, n_support, a.T, base + k, a.W, a.H), rl, 16, a.W, a.D);
  }
}

__device__ void star_wave(const StarJob& a, int32_t local_wave) {
  __shared__ int32_t s_id[kStarWaves][kStageCap];
  __shared__ int32_t s_uv[kStarWaves][kStageCap];
  __shared__ int32_t s_mark[kStarWaves][DevWave::kN * DevWave::kInFlight];
  __shared__ int32_t s_cnt[kStarWaves];
  __shared__ int32_t s_base, s_sum;
  const int lane = threadIdx.x & 63, wv_i = uniform((int32_t)threadIdx.x >> 6);
  int32_t* status = a.status;
  const int32_t n = status[kMeshSupports];
  const int32_t err0 = status[kMeshErr];
  const int32_t p = local_wave;
  const StarWork& w = a.w;
  DevOut<64> out{lane, 0, p, a.T, a.T_cap, &status[kMeshTris], a.status_copy ? &a.status_copy[kMeshTris] : nullptr,
                 &status[kMeshErr]};
  if (err0 == 0 && p < n && n <= a.w.S_cap) {  // (every wavefront goes on to the barriers)
    const Grid g{w.uv, n, a.W, a.H, w.gw, w.gh, w.cell_start, w.cell_e, w.rows};
    DevWave wv{lane, s_id[wv_i], s_uv[wv_i], s_mark[wv_i]};
    const int32_t r = star::star_of(wv, g, p, out);
    if (r < 0) {  // the frame goes to the host
      out.n = 0;
      if (lane == 0) {
        atomicCAS(&status[kMeshErr], 0, -r);
        if (a.status_copy) atomicCAS(&a.status_copy[kMeshErr], 0, -r);
      }
    } else if (a.D && out.nfl > 0) {
      // the wavefront's own writes to T before its lanes read each other's
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      raster_sets(a, out, n, lane);
    }
  }
  if (lane == 0) s_cnt[wv_i] = out.n;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t sum = 0;
    for (int k = 0; k < kStarWaves; ++k) sum += s_cnt[k];
    int32_t base = 0;
    if (sum > 0) {
      base = atomicAdd(out.counter, sum);
      if (out.counter_copy) atomicAdd(out.counter_copy, sum);
    }
    s_base = base;
    s_sum = sum;
  }
  __syncthreads();
  int32_t off = s_base;
  for (int k = 0; k < wv_i; ++k) off += s_cnt[k];
  out.write(uniform(off));
  if (a.D) {        // (the job's: uniform over the workgroup)
    __syncthreads();  // every wavefront's triangles in T before any lane reads them
    raster_block(a, s_base, s_sum, n);
  }
}

// Sixteen stars per workgroup, one 16-lane group each (the stage-batched solve): the same
// steps as star_wave, the workgroup's triangle slots reserved the same way.
constexpr int kGroupStars = 16;
// grouped stars pay off once the batch's stars far exceed the wavefronts the chip holds
// at once (measured: a 640x480 frame alone is faster a star per wavefront, 64 of them
// 18% faster a star per group; serving batches of a few frames keep a star per wavefront
// for their latency)
constexpr int64_t kGroupedMinCandidates = 65536;
__device__ void star_group16(const StarJob& a, int32_t star0) {
  __shared__ int32_t s_id[kGroupStars][DevGroup16::kCap];
  __shared__ int32_t s_uv[kGroupStars][DevGroup16::kCap];
  __shared__ int32_t s_mark[kGroupStars][DevGroup16::kN * DevGroup16::kInFlight];
  __shared__ int32_t s_cnt[kGroupStars];
  __shared__ int32_t s_base, s_sum;
  __shared__ int32_t s_fl[kGroupStars][1 + kFlushSets];
  const int gi = threadIdx.x >> 4, lane = threadIdx.x & 15, gbase = (threadIdx.x & 63) & ~15;
  int32_t* status = a.status;
  const int32_t n = status[kMeshSupports];
  const int32_t err0 = status[kMeshErr];
  const int32_t p = star0 + gi;
  const StarWork& w = a.w;
  DevOut<16> out{lane, gbase, p, a.T, a.T_cap, &status[kMeshTris],
                 a.status_copy ? &a.status_copy[kMeshTris] : nullptr, &status[kMeshErr]};
  if (a.D) {
    if (lane == 0) s_fl[gi][0] = 0;
    out.fl_list = s_fl[gi];
  }
  if (err0 == 0 && p < n && n <= a.w.S_cap) {  // (every group goes on to the barriers)
    const Grid g{w.uv, n, a.W, a.H, w.gw, w.gh, w.cell_start, w.cell_e, w.rows};
    DevGroup16 wv{lane, gbase, s_id[gi], s_uv[gi], s_mark[gi]};
    const int32_t r = star::star_of(wv, g, p, out);
    if (r < 0) {  // the frame goes to the host
      out.n = 0;
      if (lane == 0) {
        atomicCAS(&status[kMeshErr], 0, -r);
        if (a.status_copy) atomicCAS(&a.status_copy[kMeshErr], 0, -r);
      }
    }
  }
  if (lane == 0) s_cnt[gi] = out.n;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t sum = 0;
    for (int k = 0; k < kGroupStars; ++k) sum += s_cnt[k];
    int32_t base = 0;
    if (sum > 0) {
      base = atomicAdd(out.counter, sum);
      if (out.counter_copy) atomicAdd(out.counter_copy, sum);
    }
    s_base = base;
    s_sum = sum;
  }
  __syncthreads();
  int32_t off = s_base;
  for (int k = 0; k < gi; ++k) off += s_cnt[k];
  out.write(off);
  if (a.D) {        // (the job's: uniform over the workgroup)
    __syncthreads();  // every group's triangles in T before any lane reads them
    // a group's full sets written earlier, a lane per triangle; a star with more of them
    // than the group records sends the frame to the host
    const int32_t nfl = s_fl[gi][0];
    for (int32_t f = 0; f < nfl && f < kFlushSets; ++f) {
      const int32_t t = s_fl[gi][1 + f] + lane;
      if (t < a.T_cap) raster_rows(raster_setup(a.S, n, a.T, t, a.W, a.H), 0, 1, a.W, a.D);
    }
    if (nfl > kFlushSets && lane == 0) {
      atomicCAS(&status[kMeshErr], 0, star::kStarErrSets);
      if (a.status_copy) atomicCAS(&a.status_copy[kMeshErr], 0, star::kStarErrSets);
    }
    raster_block(a, s_base, s_sum, n);
  }
}

__global__ __launch_bounds__(64 * kStarWaves) void k_star(StarJob a) {
  star_wave(a, blockIdx.x * kStarWaves + uniform((int32_t)threadIdx.x >> 6));
}

// the job of workgroup b: the last j with offs[j] <= b
__device__ __forceinline__ int32_t job_of(const int32_t* __restrict__ offs, int32_t n_jobs, int32_t b) {
  int32_t lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// a star per wavefront, as k_star (batches whose stars fit the chip at once)
__global__ __launch_bounds__(64 * kStarWaves) void k_star_many(const StarJob* __restrict__ jobs,
                                                               const int32_t* __restrict__ offs, int32_t n_jobs) {
  const int32_t b = blockIdx.x, j = job_of(offs, n_jobs, b);
  star_wave(jobs[j], (b - offs[j]) * kStarWaves + uniform((int32_t)threadIdx.x >> 6));
}

// a star per 16-lane group (larger batches; three waves per SIMD: the most that fits its
// registers without spilling)
__global__ __launch_bounds__(64 * kStarWaves, 3) void k_star_many16(const StarJob* __restrict__ jobs,
                                                                 const int32_t* __restrict__ offs, int32_t n_jobs) {
  const int32_t b = blockIdx.x, j = job_of(offs, n_jobs, b);
  star_group16(jobs[j], (b - offs[j]) * kGroupStars);
}

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carve {
  size_t o = 0;
  uint8_t* base = nullptr;
  template <class T>
  T* take(size_t n) {
    T* p = base ? (T*)(base + o) : nullptr;
    o = align256(o + n * sizeof(T));
    return p;
  }
};

StarWork carve(Carve& c, int32_t W, int32_t H, int32_t S_cap) {
  StarWork w;
  w.gw = (W + star::kStarCell - 1) / star::kStarCell;
  w.gh = (H + star::kStarCell - 1) / star::kStarCell;
  const size_t cells = (size_t)w.gw * w.gh;
  w.uv = c.take<int32_t>((size_t)S_cap);
  w.cell_start = c.take<int32_t>(cells + 1);
  w.cell_cur = c.take<int32_t>(cells);
  w.cell_e = c.take<star::CellEntry>((size_t)S_cap);
  w.rows = c.take<star::RowExt>((size_t)H);
  w.row_min = c.take<int32_t>((size_t)H);
  w.row_max = c.take<int32_t>((size_t)H);
  w.S_cap = S_cap;
  return w;
}

}  // namespace

bool prep_in_lds(int32_t W, int32_t H) {
  const int64_t cells =
      (int64_t)((W + star::kStarCell - 1) / star::kStarCell) * ((H + star::kStarCell - 1) / star::kStarCell);
  return cells <= kLdsCells && H <= kLdsRows;
}

size_t star_work_bytes(int32_t W, int32_t H, int32_t S_cap) {
  Carve c;
  carve(c, W, H, S_cap);
  return c.o;
}

StarWork star_work_at(void* base, int32_t W, int32_t H, int32_t S_cap) {
  Carve c;
  c.base = (uint8_t*)base;
  return carve(c, W, H, S_cap);
}

int32_t star_blocks(int32_t S_cap) { return (S_cap + kStarWaves - 1) / kStarWaves; }
bool star_grouped(int64_t candidates) { return candidates > kGroupedMinCandidates; }
int32_t star_blocks_many(int32_t S_cap, bool grouped) {
  const int32_t per = grouped ? kGroupStars : kStarWaves;
  return (S_cap + per - 1) / per;
}

hipError_t launch_star(const StarJob& job, hipStream_t s) {
  hipEvent_t e0, e1;
  const bool timed = take_launch_events(&e0, &e1);
  const bool lds = prep_in_lds(job.W, job.H);
  if (timed)
    hipExtLaunchKernelGGL(lds ? k_star_prep<true> : k_star_prep<false>, dim3(1), dim3(kPrepThreads), 0, s, e0,
                          nullptr, 0u, job);
  else
    hipLaunchKernelGGL(lds ? k_star_prep<true> : k_star_prep<false>, dim3(1), dim3(kPrepThreads), 0, s, job);
  if (job.blocks > 0) {
    if (timed)
      hipExtLaunchKernelGGL(k_star, dim3((unsigned)job.blocks), dim3(64 * kStarWaves), 0, s, nullptr, e1, 0u, job);
    else
      hipLaunchKernelGGL(k_star, dim3((unsigned)job.blocks), dim3(64 * kStarWaves), 0, s, job);
  }
  return hipGetLastError();
}

hipError_t launch_star_many(const StarJob* jobs, const int32_t* offs, int32_t n, int32_t total_blocks,
                            bool lds, bool grouped, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipEvent_t e0, e1;
  const bool timed = take_launch_events(&e0, &e1);
  if (timed)
    hipExtLaunchKernelGGL(lds ? k_star_prep_many<true> : k_star_prep_many<false>, dim3((unsigned)n),
                          dim3(kPrepThreads), 0, s, e0, nullptr, 0u, jobs);
  else
    hipLaunchKernelGGL(lds ? k_star_prep_many<true> : k_star_prep_many<false>, dim3((unsigned)n), dim3(kPrepThreads),
                       0, s, jobs);
  if (total_blocks > 0) {
    auto kernel = grouped ? k_star_many16 : k_star_many;
    if (timed)
      hipExtLaunchKernelGGL(kernel, dim3((unsigned)total_blocks), dim3(64 * kStarWaves), 0, s, nullptr, e1, 0u,
                            jobs, offs, n);
    else
      hipLaunchKernelGGL(kernel, dim3((unsigned)total_blocks), dim3(64 * kStarWaves), 0, s, jobs, offs, n);
  }
  return hipGetLastError();
}

}  // namespace sm
