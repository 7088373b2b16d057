// Device kernels of the stereomesh library for gfx950 (CDNA4, wave64).
//
// All per-pixel work is integer or IEEE float with fused multiply-add disabled
// (-ffp-contract=off plus explicit _rn intrinsics where rounding order matters), so
// every output is reproducible bit for bit.
#include "kernels.hpp"
#include "compact.hpp"
#include "raster.hpp"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <climits>
#include <map>
#include <mutex>
#include <tuple>

namespace sm {

// Event pair armed by the host layer for the next launch of this thread: the kernel
// is then dispatched with hipExtLaunchKernelGGL, which timestamps the kernel itself.
namespace {
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
}  // namespace

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_ev_start = start;
  g_ev_stop = stop;
}
bool launch_events_pending() { return g_ev_start != nullptr; }
bool take_launch_events(hipEvent_t* start, hipEvent_t* stop) {
  *start = g_ev_start;
  *stop = g_ev_stop;
  g_ev_start = g_ev_stop = nullptr;
  return *start != nullptr;
}

#define SM_LAUNCH(kernel, grid, block, shmem, stream, ...)                                  \
  do {                                                                                     \
    if (g_ev_start) {                                                                      \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, g_ev_start, g_ev_stop, 0u,  \
                            __VA_ARGS__);                                                  \
      g_ev_start = g_ev_stop = nullptr;                                                    \
    } else {                                                                               \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                  \
    }                                                                                      \
  } while (0)

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    uint32_t y = __shfl_xor(x, off, kWave);
    x = y < x ? y : x;
  }
  return x;
}

// ------------------------------------------------------------------------------------
// Census words + Omega_I (+ optional initialisation of D_f, C_f and the occupancy map).
// Tile of 64 x th output pixels per 256-thread block (th = 8, 16 or 32 rows: a launch-shape
// choice of sm_autotune; by default 8 for one frame's launch, whose few tiles are in
// flight at once, and 16 in the batched census, which has tiles to spare: measured at
// 640x480, 11.0 against 12.5 us alone and 281 against 233 us for 64 frames), staged in LDS
// with its halo.
// ------------------------------------------------------------------------------------
constexpr int kTW = 64, kTHFrame = 8, kTHBatch = 16, kTHMax = 32;

struct CensusArgs {
  CensusJob job[2];
  int32_t W, H, grad_thr, t_hi;
  int32_t th;  // tile rows
  float* D_f;
  uint8_t* C_f;
  uint8_t* occ;
  CensusExtras x;
};

// One 64 x a.th output tile (bx, by) of image jb (left: also Omega_I and the per-frame
// initialisation). `tile` is the block's LDS staging area.
template <int RX, int RY>
__device__ __forceinline__ void census_block(const CensusArgs& a, const CensusJob& jb, bool left, int bx, int by,
                                             uint8_t* tile) {
  constexpr int PW = kTW + 2 * RX;
  const int th = a.th, PH = th + 2 * RY;
  const int W = a.W, H = a.H;
  const int gx0 = bx * kTW - RX, gy0 = by * th - RY;
  // the tile and its halo, every load of a thread in flight before the first LDS store
  constexpr int kStage = ((kTHMax + 2 * RY) * PW + 255) / 256;
  const int tid = threadIdx.y * kTW + threadIdx.x;
  uint8_t px[kStage];
#pragma unroll
  for (int k = 0; k < kStage; ++k) {
    const int i = tid + 256 * k;
    if (i < PH * PW) {
      const int ty = i / PW, tx = i - ty * PW;
      const int gx = min(max(gx0 + tx, 0), W - 1), gy = min(max(gy0 + ty, 0), H - 1);
      px[k] = jb.img[(size_t)gy * jb.stride + gx];
    }
  }
#pragma unroll
  for (int k = 0; k < kStage; ++k) {
    const int i = tid + 256 * k;
    if (i < PH * PW) tile[i] = px[k];
  }
  __syncthreads();
  const int u = bx * kTW + threadIdx.x;
  for (int r = 0; r < th / 4; ++r) {
    const int ly = threadIdx.y + 4 * r;
    const int v = by * th + ly;
    if (v >= H || u >= W) break;
    const size_t idx = (size_t)v * W + u;
    const bool valid = u >= RX && u < W - RX && v >= RY && v < H - RY;
    const uint8_t* c = &tile[(ly + RY) * PW + threadIdx.x + RX];
    uint32_t lo = 0, hi = 0;
    const uint32_t cv = c[0];
#pragma unroll
    for (int dy = -RY; dy <= RY; ++dy) {
#pragma unroll
      for (int dx = -RX; dx <= RX; ++dx) {
        constexpr int kCenter = RY * (2 * RX + 1) + RX;
        const int pos = (dy + RY) * (2 * RX + 1) + (dx + RX);
        if (pos == kCenter) continue;
        const int k = pos < kCenter ? pos : pos - 1;
        const uint32_t bit = (uint32_t)c[dy * PW + dx] < cv;
        if (k < 32) lo |= bit << k;
        else hi |= bit << (k - 32);
      }
    }
    const uint64_t word = valid ? ((uint64_t)hi << 32 | lo) : 0ull;
    jb.census[idx] = word;
    if (jb.omega) {
      uint8_t om = 0;
      if (valid) {
        const int gxx = abs((int)c[1] - (int)c[-1]);
        const int gyy = abs((int)c[PW] - (int)c[-PW]);
        om = (gxx + gyy) >= a.grad_thr;
      }
      jb.omega[idx] = om;
    }
    if (left) {
      if (a.D_f) a.D_f[idx] = 0.0f;
      if (a.C_f) a.C_f[idx] = (uint8_t)a.t_hi;
      if (a.occ) a.occ[idx] = 0;
      if (a.x.D_nan) a.x.D_nan[idx] = __builtin_nanf("");
      if (a.x.grid_slots) {  // support-grid candidate at this pixel
        const int h = a.x.step / 2;
        const int gu = u - h, gv = v - h;
        if (gu >= 0 && gv >= 0 && gu % a.x.step == 0 && gv % a.x.step == 0) {
          const bool cand = valid && jb.omega &&
                            (abs((int)c[1] - (int)c[-1]) + abs((int)c[PW] - (int)c[-PW])) >= a.grad_thr;
          sm_support sp;
          sp.u = (int16_t)u;
          sp.v = (int16_t)v;
          sp.d = cand ? kPending : kRejected;
          a.x.grid_slots[(gv / a.x.step) * a.x.gw + gu / a.x.step] = sp;
        }
      }
    }
  }
  if (a.x.zero && bx == 0 && by == 0 && left) {
    const int t = threadIdx.y * kTW + threadIdx.x;
    if (t < a.x.n_zero) a.x.zero[t] = 0;
  }
}

template <int RX, int RY>
__global__ __launch_bounds__(256) void k_census(CensusArgs a) {
  __shared__ uint8_t tile[(kTHMax + 2 * RY) * (kTW + 2 * RX)];
  census_block<RX, RY>(a, a.job[blockIdx.z], blockIdx.z == 0, blockIdx.x, blockIdx.y, tile);
}

template <int RX, int RY>
hipError_t census_launch(const CensusArgs& a, int n_jobs, hipStream_t s) {
  dim3 grid((a.W + kTW - 1) / kTW, (a.H + a.th - 1) / a.th, n_jobs);
  SM_LAUNCH((k_census<RX, RY>), grid, dim3(kTW, 4, 1), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Candidate slots
// ------------------------------------------------------------------------------------
__global__ void k_grid_slots(const uint8_t* omega, int W, int step, int gw, sm_support* slots, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int gy = i / gw, gx = i - gy * gw;
  const int u = step / 2 + gx * step, v = step / 2 + gy * step;
  sm_support s;
  s.u = (int16_t)u;
  s.v = (int16_t)v;
  s.d = omega[(size_t)v * W + u] ? kPending : kRejected;
  slots[i] = s;
}

__global__ void k_list_slots(const int16_t* uv, int n, sm_support* slots) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  sm_support s;
  s.u = uv[2 * i];
  s.v = uv[2 * i + 1];
  s.d = kPending;
  slots[i] = s;
}

// ------------------------------------------------------------------------------------
// FAST support keypoints sampled from spatial bins (Sec. III-A).
//  * k_fast_score: one thread per pixel; the 16 ring differences d_k = I(ring_k) - I(p)
//    are reduced to the minimum (and maximum) over every arc of 9 by doubling windows
//    (2, 4, 8, then one more element), score = max over arcs of max(min d, -max d), >= 0.
//  * k_fast_select: one 1024-thread workgroup per bin. Pass 1 applies the 3x3
//    suppression and builds a score histogram of the bin's keypoints; the threshold
//    score s* of the per_bin-th best keypoint and the number of keypoints at s* to take
//    follow from it. Pass 2 walks the bin in raster order in 1024-pixel chunks (stopping
//    once the bin is full) and emits the keypoints above s* and the first ones at s*,
//    with block prefix sums (wave ballots) for ranks and output positions, so the
//    output is in raster order.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fast_score(const uint8_t* img, int stride, int W, int H,
                                                    uint8_t* score) {
  const int u = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
  const int v = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (u >= W || v >= H) return;
  int best = 0;
  if (u >= 3 && v >= 3 && u <= W - 4 && v <= H - 4) {
    // radius-3 Bresenham ring, clockwise from the pixel straight above p
    constexpr int kDx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
    constexpr int kDy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};
    const uint8_t* c = img + (size_t)v * stride + u;
    const int ip = c[0];
    int d[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) d[k] = (int)c[kDy[k] * stride + kDx[k]] - ip;
    int lo2[16], hi2[16], lo4[16], hi4[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      lo2[k] = min(d[k], d[(k + 1) & 15]);
      hi2[k] = max(d[k], d[(k + 1) & 15]);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      lo4[k] = min(lo2[k], lo2[(k + 2) & 15]);
      hi4[k] = max(hi2[k], hi2[(k + 2) & 15]);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int lo9 = min(min(lo4[k], lo4[(k + 4) & 15]), d[(k + 8) & 15]);  // arc k .. k+8
      const int hi9 = max(max(hi4[k], hi4[(k + 4) & 15]), d[(k + 8) & 15]);
      best = max(best, max(lo9, -hi9));
    }
  }
  score[(size_t)v * W + u] = (uint8_t)best;
}

struct FastSelectArgs {
  const uint8_t* score;
  int32_t W, H, t, bins_x, bins_y, per_bin;
  sm_support* slots;  // either: per_bin slots per bin, (u, v, kPending) / kRejected
  int16_t* uv;        // or: per_bin (u, v) pairs per bin, (-1, -1) when empty
};

// 3x3 suppression: p (a corner, hence at least 3 px inside the image) is a keypoint when
// earlier raster neighbours score lower and later ones do not score higher.
__device__ __forceinline__ bool fast_keypoint(const uint8_t* score, int W, int u, int v, int sc, int t) {
  if (sc <= t) return false;
  const uint8_t* c = score + (size_t)v * W + u;  // (all eight loads at once: no short circuit)
  const int n0 = c[-W - 1], n1 = c[-W], n2 = c[-W + 1], n3 = c[-1];
  const int n4 = c[1], n5 = c[W - 1], n6 = c[W], n7 = c[W + 1];
  return ((n0 < sc) & (n1 < sc) & (n2 < sc) & (n3 < sc) & (n4 <= sc) & (n5 <= sc) & (n6 <= sc) &
          (n7 <= sc)) != 0;
}

constexpr int kFastThreads = 1024, kFastWaves = kFastThreads / kWave;

// Exclusive prefixes of two flags over the block's threads in thread order, and their
// block totals (one LDS slot per wave and flag, one barrier pair for both).
__device__ __forceinline__ void block_prefix2(bool f0, bool f1, int2* wsum, int& p0, int& p1, int& t0,
                                              int& t1) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  const unsigned long long m0 = __ballot(f0), m1 = __ballot(f1);
  const unsigned long long below = (1ull << lane) - 1ull;
  if (lane == 0) wsum[w] = make_int2(__popcll(m0), __popcll(m1));
  __syncthreads();
  int b0 = 0, b1 = 0;
  t0 = t1 = 0;
#pragma unroll
  for (int k = 0; k < kFastWaves; ++k) {
    const int2 c = wsum[k];
    b0 += k < w ? c.x : 0;
    b1 += k < w ? c.y : 0;
    t0 += c.x;
    t1 += c.y;
  }
  __syncthreads();  // wsum is reused by the next call
  p0 = b0 + __popcll(m0 & below);
  p1 = b1 + __popcll(m1 & below);
}

__global__ __launch_bounds__(kFastThreads) void k_fast_select(FastSelectArgs a) {
  __shared__ int hist[256];
  __shared__ int2 wsum[kFastWaves];
  __shared__ int s_thr, s_take;
  const int b = blockIdx.x;
  const int by = b / a.bins_x, bx = b - by * a.bins_x;
  // pixels with floor(u * bins_x / W) == bx: u in [ceil(bx W / bins_x), ceil((bx+1) W / bins_x))
  const int u0 = (int)(((int64_t)bx * a.W + a.bins_x - 1) / a.bins_x);
  const int u1 = (int)(((int64_t)(bx + 1) * a.W + a.bins_x - 1) / a.bins_x);
  const int v0 = (int)(((int64_t)by * a.H + a.bins_y - 1) / a.bins_y);
  const int v1 = (int)(((int64_t)(by + 1) * a.H + a.bins_y - 1) / a.bins_y);
  const int bw = max(u1 - u0, 0), n = bw * max(v1 - v0, 0);
  if (threadIdx.x < 256) hist[threadIdx.x] = 0;
  __syncthreads();
  constexpr int kHistPer = 4;  // pixels per thread and pass, their loads in flight together
  for (int start = 0; start < n; start += kHistPer * kFastThreads) {
    int sc[kHistPer];
    bool kp[kHistPer];
#pragma unroll
    for (int k = 0; k < kHistPer; ++k) {
      const int i = start + k * kFastThreads + threadIdx.x;
      const int v = v0 + (i < n ? i / bw : 0), u = u0 + (i < n ? i % bw : 0);
      sc[k] = i < n ? a.score[(size_t)v * a.W + u] : 0;
    }
#pragma unroll
    for (int k = 0; k < kHistPer; ++k) {
      const int i = start + k * kFastThreads + threadIdx.x;
      kp[k] = i < n && fast_keypoint(a.score, a.W, u0 + i % bw, v0 + i / bw, sc[k], a.t);
    }
#pragma unroll
    for (int k = 0; k < kHistPer; ++k)
      if (kp[k]) atomicAdd(&hist[sc[k]], 1);
  }
  __syncthreads();  // histogram complete
  if (threadIdx.x == 0) {  // default: every keypoint (score >= 1 > 0) is kept
    s_thr = 0;
    s_take = 0;
  }
  // at_least = number of keypoints scoring >= sc, for sc = 255 - threadIdx.x: an
  // inclusive scan over the histogram read backwards (4 waves of shuffles + LDS)
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  const int sc_t = 255 - threadIdx.x;
  int h = 0, at_least = 0;
  if (threadIdx.x < 256) {
    h = hist[sc_t];
    at_least = h;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int o = __shfl_up(at_least, off, kWave);
      if (lane >= off) at_least += o;
    }
    if (lane == kWave - 1) wsum[w] = make_int2(at_least, 0);
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    for (int k = 0; k < w; ++k) at_least += wsum[k].x;
    // the score of the per_bin-th best keypoint: the only sc with
    // at_least(sc + 1) < per_bin <= at_least(sc)
    if (at_least >= a.per_bin && at_least - h < a.per_bin) {
      s_thr = sc_t;
      s_take = a.per_bin - (at_least - h);
    }
  }
  __syncthreads();
  const int thr = s_thr, take = s_take;
  const size_t out0 = (size_t)b * a.per_bin;
  int base_eq = 0, base_sel = 0;
  constexpr int kSelPer = 4;  // chunks of kFastThreads pixels whose loads go out together
  for (int start0 = 0; start0 < n && base_sel < a.per_bin; start0 += kSelPer * kFastThreads) {  // block-uniform
    int scs[kSelPer];
    bool kps[kSelPer];
#pragma unroll
    for (int k = 0; k < kSelPer; ++k) {
      const int i = start0 + k * kFastThreads + threadIdx.x;
      scs[k] = i < n ? a.score[(size_t)(v0 + i / bw) * a.W + u0 + i % bw] : 0;
    }
#pragma unroll
    for (int k = 0; k < kSelPer; ++k) {
      const int i = start0 + k * kFastThreads + threadIdx.x;
      kps[k] = i < n && fast_keypoint(a.score, a.W, u0 + i % bw, v0 + i / bw, scs[k], a.t);
    }
#pragma unroll
    for (int k = 0; k < kSelPer; ++k) {
      const int start = start0 + k * kFastThreads;
      if (start >= n || base_sel >= a.per_bin) break;  // (block-uniform)
      const int i = start + threadIdx.x;
      const int v = v0 + (i < n ? i / bw : 0), u = u0 + (i < n ? i % bw : 0), sc = scs[k];
      const bool kp = kps[k];
      // keypoints above the threshold are all kept; at the threshold, the first `take` in
      // raster order (their rank needs the prefix of the at-threshold flags)
      const bool above = kp && sc > thr, eq = kp && sc == thr;
      int p_above, p_eq, n_above, n_eq;
      block_prefix2(above, eq, wsum, p_above, p_eq, n_above, n_eq);
      const int rank = base_eq + p_eq;
      const bool eq_sel = eq && rank < take;
      // output position: kept keypoints before this one in raster order
      const int eq_before = min(max(take - base_eq, 0), p_eq);  // kept at-threshold ones before i
      const bool sel = above || eq_sel;
      const int pos = base_sel + p_above + eq_before;
      if (sel) {
        if (a.slots) {
          sm_support sp;
          sp.u = (int16_t)u;
          sp.v = (int16_t)v;
          sp.d = kPending;
          a.slots[out0 + pos] = sp;
        } else {
          a.uv[2 * (out0 + pos)] = (int16_t)u;
          a.uv[2 * (out0 + pos) + 1] = (int16_t)v;
        }
      }
      base_sel += n_above + min(max(take - base_eq, 0), n_eq);
      base_eq += n_eq;
    }
  }
  for (int j = base_sel + threadIdx.x; j < a.per_bin; j += kFastThreads) {  // empty slots
    if (a.slots) {
      sm_support sp;
      sp.u = 0;
      sp.v = 0;
      sp.d = kRejected;
      a.slots[out0 + j] = sp;
    } else {
      a.uv[2 * (out0 + j)] = -1;
      a.uv[2 * (out0 + j) + 1] = -1;
    }
  }
}

// Order-preserving in-place compaction of (u, v) pairs with u >= 0 (one workgroup).
__global__ __launch_bounds__(1024) void k_compact_uv(int16_t* uv, int n, int* n_out) {
  __shared__ int wsum[16];
  __shared__ int wofs[16];
  __shared__ int total;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  int base = 0;
  for (int start = 0; start < n; start += 1024) {
    const int i = start + threadIdx.x;
    int16_t u = -1, v = -1;
    if (i < n) {
      u = uv[2 * i];
      v = uv[2 * i + 1];
    }
    const bool keep = u >= 0;
    const unsigned long long m = __ballot(keep);
    const int pre = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();  // every read of this chunk happened before any write below
    if (threadIdx.x == 0) {
      int acc = 0;
      for (int k = 0; k < 16; ++k) {
        wofs[k] = acc;
        acc += wsum[k];
      }
      total = acc;
    }
    __syncthreads();
    if (keep) {
      uv[2 * (base + wofs[w] + pre)] = u;
      uv[2 * (base + wofs[w] + pre) + 1] = v;
    }
    base += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_out = base;
}

// ------------------------------------------------------------------------------------
// Epipolar matching: a group of G lanes per candidate (G = 64, 32 or 16: 1, 2 or 4
// candidates per wave), the group's lanes over the disparities in ceil(N_D / G) chunks,
// group-shuffle argmin over packed (cost << 8 | d) keys. G is a launch-shape choice
// (sm_autotune), the result does not depend on it.
// ------------------------------------------------------------------------------------
struct MatchArgs {
  const uint64_t* cL;
  const uint64_t* cR;
  int32_t W, H, rx, ry, d_min, d_max, t_hi, uniq, lr_tol;
  sm_support* slots;
  int32_t n;
};

constexpr int kMaxDisp = 256;  // d_max - d_min + 1 (enforced by the parameter checks)

template <int G>
__device__ __forceinline__ uint32_t group_min_u32(uint32_t x) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) {
    const uint32_t y = __shfl_xor(x, off, kWave);
    x = y < x ? y : x;
  }
  return x;
}
// any lane of this lane's group of G
template <int G>
__device__ __forceinline__ bool group_any(bool b, int lane) {
  const uint64_t m = __ballot(b);
  return G == kWave ? m != 0ull : ((m >> (lane & ~(G - 1))) & ((1ull << (G & 63)) - 1)) != 0ull;
}

// Matches left pixel (u, v) (inside the census-valid region); every lane of the group
// must call it with the same (u, v); gl is the lane's index in its group. Returns d* or -1
// when rejected.
template <int G>
__device__ int match_one_g(const MatchArgs& a, int u, int v, int gl, int lane) {
  constexpr int kChunks = kMaxDisp / G;
  const int chunks = (a.d_max - a.d_min + G) / G;
  const int W = a.W;
  const uint64_t* rowL = a.cL + (size_t)v * W;
  const uint64_t* rowR = a.cR + (size_t)v * W;
  const uint64_t wl = rowL[u];
  uint32_t cost[kChunks];
  uint32_t best = 0xffffffffu;
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int d = a.d_min + gl + G * c;
    const bool ok = c < chunks && d <= a.d_max && u - d >= a.rx;
    const uint32_t cs = ok ? (uint32_t)__popcll(wl ^ rowR[u - d]) : 0xffu;
    cost[c] = cs;
    const uint32_t key = ok ? (cs << 8 | (uint32_t)d) : 0xffffffffu;
    best = key < best ? key : best;
  }
  best = group_min_u32<G>(best);
  if (best == 0xffffffffu) return -1;  // no admissible disparity
  const int dstar = (int)(best & 0xffu);
  const uint32_t cstar = best >> 8;
  if (cstar >= (uint32_t)a.t_hi) return -1;
  if (a.uniq > 0) {
    bool bad = false;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const int d = a.d_min + gl + G * c;
      const bool ok = c < chunks && d <= a.d_max && u - d >= a.rx;
      const int dd = d - dstar;
      bad |= ok && (dd >= 2 || dd <= -2) && cost[c] < cstar + (uint32_t)a.uniq;
    }
    if (group_any<G>(bad, lane)) return -1;
  }
  // left-right check from the matched right pixel
  const int ur = u - dstar;
  const uint64_t wr = rowR[ur];
  uint32_t best2 = 0xffffffffu;
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int d = a.d_min + gl + G * c;
    const bool ok = c < chunks && d <= a.d_max && ur + d <= W - 1 - a.rx;
    const uint32_t key = ok ? ((uint32_t)__popcll(wr ^ rowL[ur + d]) << 8 | (uint32_t)d) : 0xffffffffu;
    best2 = key < best2 ? key : best2;
  }
  best2 = group_min_u32<G>(best2);
  const int diff = (int)(best2 & 0xffu) - dstar;
  return (diff <= a.lr_tol && -diff <= a.lr_tol) ? dstar : -1;
}

// one whole wave per pixel (the re-match of a cell)
__device__ __forceinline__ int match_one(const MatchArgs& a, int u, int v, int lane) {
  return match_one_g<kWave>(a, u, v, lane, lane);
}

__device__ __forceinline__ bool match_inside(const MatchArgs& a, int u, int v) {
  return u >= a.rx && u < a.W - a.rx && v >= a.ry && v < a.H - a.ry;
}

// Matches candidate slot `slot` if it is pending (the whole group calls it).
template <int G>
__device__ __forceinline__ void match_slot(const MatchArgs& a, int slot, int lane) {
  const sm_support s = a.slots[slot];
  if (s.d != kPending) return;
  const int gl = lane & (G - 1);
  const int d = match_inside(a, s.u, s.v) ? match_one_g<G>(a, s.u, s.v, gl, lane) : -1;
  if (gl == 0) a.slots[slot].d = d >= 0 ? (float)d : kRejected;
}

// slot of this lane's group: waves of 256-thread blocks, kWave / G groups per wave
template <int G>
__device__ __forceinline__ int match_unit_slot(int wave_unit, int lane) {
  return wave_unit * (kWave / G) + lane / G;
}

template <int G>
__global__ __launch_bounds__(256) void k_match(MatchArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int slot = match_unit_slot<G>(blockIdx.x * 4 + (threadIdx.x >> 6), lane);
  if (slot >= a.n) return;  // (whole groups: a group's lanes share the slot)
  match_slot<G>(a, slot, lane);
}

// Resampling (Alg. 4) fused with the re-match: one wave per cell. Slot c receives the
// confident support of cell c, slot n_cells + c its re-matched invalid pixel; a pixel that
// occ (non-null: the occupancy of the current supports) marks is already a support, so its
// slot stays empty (and is not matched).
__device__ __forceinline__ void rematch_cell(const MatchArgs& a, const uint64_t* cell_g, const uint64_t* cell_b,
                                             const float* D_it, const uint8_t* occ, int n_cells, uint64_t ginit,
                                             uint64_t binit, int c, int lane) {
  const uint64_t g = cell_g[c], b = cell_b[c];
  const bool g_new = g != ginit && !(occ && occ[(uint32_t)g]);
  const bool b_new = b != binit && !(occ && occ[(uint32_t)b]);
  if (lane == 0) {
    sm_support sg;
    if (g_new) {
      const uint32_t idx = (uint32_t)g;
      sg.u = (int16_t)(idx % (uint32_t)a.W);
      sg.v = (int16_t)(idx / (uint32_t)a.W);
      sg.d = D_it[idx];
    } else {
      sg.u = sg.v = 0;
      sg.d = kRejected;
    }
    a.slots[c] = sg;
  }
  sm_support sb;
  sb.u = sb.v = 0;
  sb.d = kRejected;
  if (b_new) {
    const uint32_t idx = (uint32_t)b;
    const int u = (int)(idx % (uint32_t)a.W), v = (int)(idx / (uint32_t)a.W);
    sb.u = (int16_t)u;
    sb.v = (int16_t)v;
    const int d = match_inside(a, u, v) ? match_one(a, u, v, lane) : -1;
    if (d >= 0) sb.d = (float)d;
  }
  if (lane == 0) a.slots[n_cells + c] = sb;
}

__global__ __launch_bounds__(256) void k_rematch_cells(MatchArgs a, const uint64_t* cell_g,
                                                       const uint64_t* cell_b, const float* D_it,
                                                       const uint8_t* occ, int n_cells, uint64_t ginit,
                                                       uint64_t binit, const int32_t* slot_off, int slot_cap) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n_cells) return;
  if (slot_off) {  // region placed after the supports counted on the device
    const int off = *slot_off;
    if (off < 0 || (int64_t)off + 2 * n_cells + 1 > slot_cap) return;  // a failed mesh: nothing to add
    a.slots += off;
  }
  rematch_cell(a, cell_g, cell_b, D_it, occ, n_cells, ginit, binit, c, lane);
}

// ------------------------------------------------------------------------------------
// Order-preserving in-place compaction (one 1024-thread workgroup).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_compact(sm_support* slots, int n, int* n_out, uint8_t* occ,
                                                  int W, int* header, const int32_t* slot_off, int slot_cap) {
  if (slot_off) {  // region after the supports counted on the device; its count in the slot after it
    const int off = *slot_off;
    if (off < 0 || (int64_t)off + n + 1 > slot_cap) return;  // a failed mesh: nothing to compact
    slots += off;
    header = (int*)(slots + n);
  }
  compact_block(slots, n, n_out, occ, W, header);
}

__global__ void k_fill_u8(uint8_t* p, size_t n, uint8_t val) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = val;
}

// p[0, n) = val: 16-byte stores from the first 16-byte boundary on (a grid-stride loop),
// single floats before it and after the last full 16 bytes.
__global__ __launch_bounds__(256) void k_fill_f32(float* p, size_t n, float val) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (size_t)gridDim.x * blockDim.x;
  const size_t head = min((size_t)(((16 - ((uintptr_t)p & 15)) & 15) / 4), n);
  if (tid < head) p[tid] = val;
  float4* q = reinterpret_cast<float4*>(p + head);
  const size_t n4 = (n - head) / 4;
  const float4 v = make_float4(val, val, val, val);
  for (size_t i = tid; i < n4; i += nt) q[i] = v;
  const size_t tail = head + 4 * n4;
  if (tid < n - tail) p[tail + tid] = val;
}

__global__ void k_mark(const sm_support* S, int n, uint8_t* occ, int W, int H) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int u = S[i].u, v = S[i].v;
  if (u >= 0 && u < W && v >= 0 && v < H) occ[(size_t)v * W + u] = 1;
}

// ------------------------------------------------------------------------------------
// Plane fit + rasterisation. Each triangle's rows are dealt to lanes; a lane solves its
// row's owned span exactly from the three edges (ownership of the perturbed point
// (u + eps, v + eps^2)) with no branches, and evaluates the plane along it. Two layouts:
//  * k_raster_wave: one wave per triangle, one lane per row (64 rows at a time). Many
//    short waves: best for small meshes, where the run is launch/latency bound and a
//    large triangle only delays its own wave.
//  * k_raster_group: 4 triangles per wave, 16 lanes per triangle taking its rows in
//    turn (one pass for the typical 10-row triangle of a 10 px support grid): best for
//    large meshes (measured against 2 and 8 triangles per wave, and against staging a
//    workgroup's pixels in an LDS window written out with 16-byte stores, which cut the
//    store instructions but lost more to LDS writes and occupancy).
//    Workgroups are remapped so that each XCD (workgroups are dealt round-robin over
//    the 8 XCDs) takes one contiguous run of the triangle list.
// ------------------------------------------------------------------------------------
constexpr int kXcds = 8;
constexpr int kTriPerWave = 4, kRowLanes = kWave / kTriPerWave;
constexpr int kGroupLayoutMinTris = 16384;
constexpr int kRasterStrideBlocks = 2048;  // 8 per CU

__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b % kXcds, k = b / kXcds, q = nb / kXcds, r = nb % kXcds;
  return x * q + min(x, r) + k;
}

// Triangle t by one wave, one lane per row.
__device__ __forceinline__ void raster_tri_wave(const sm_support* S, int n_support, const sm_tri* T, int t,
                                                int W, int H, float* D, int lane) {
  const RasterTri r = raster_setup(S, n_support, T, t, W, H);
  if (!r.ok) return;
  for (int v = r.vmin + lane; v <= r.vmax; v += kWave) {
    int lo, hi;
    raster_span(r, v, lo, hi);
    raster_row(r, v, lo, hi, D + (size_t)v * W);
  }
}

__global__ __launch_bounds__(256) void k_raster_wave(const sm_support* S, int n_support, const sm_tri* T,
                                                     int n_tris, int W, int H, float* D, const int32_t* counts) {
  const int lane = threadIdx.x & (kWave - 1);
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (counts) {  // counts kept on the device: n_tris is then the launch's upper bound
    n_tris = min(n_tris, counts[kCountTris]);
    n_support = min(n_support, counts[kCountSupports]);
  }
  if (t >= n_tris) return;
  raster_tri_wave(S, n_support, T, t, W, H, D, lane);
}

__global__ __launch_bounds__(256) void k_raster_group(const sm_support* S, int n_support, const sm_tri* T,
                                                      int n_tris, int W, int H, float* D, const int32_t* counts) {
  const int lane = threadIdx.x & (kWave - 1);
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int t = (blk * 4 + (threadIdx.x >> 6)) * kTriPerWave + lane / kRowLanes;
  const int rl = lane % kRowLanes;
  if (counts) {  // counts kept on the device: n_tris is then the launch's upper bound
    n_tris = min(n_tris, counts[kCountTris]);
    n_support = min(n_support, counts[kCountSupports]);
  }
  // lanes are independent; a grid smaller than the triangles strides over them
  for (int tt = t; tt < n_tris; tt += gridDim.x * 4 * kTriPerWave) {
    const RasterTri r = raster_setup(S, n_support, T, tt, W, H);
    if (!r.ok) continue;
    for (int v = r.vmin + rl; v <= r.vmax; v += kRowLanes) {
      int lo, hi;
      raster_span(r, v, lo, hi);
      raster_row(r, v, lo, hi, D + (size_t)v * W);
    }
  }
}

// ------------------------------------------------------------------------------------
// Cost evaluation + refinement. Each 1024-thread workgroup (16 waves) owns whole
// occupancy cells: a tile of cpr cells side by side (cpr = max(1, 64 / sz),
// TW = cpr * sz columns) and crows cell rows (crows = max(1, 16 / sz), TH = crows * sz
// rows). Lanes walk the tile's columns, waves its rows; every thread's pixels lie in
// one cell, so each thread keeps one running minimum per cell array, followed by a
// segmented shuffle minimum across lanes and a minimum across the waves of the same
// cell row through LDS. Cell keys are then written with plain stores (no atomics, no
// reset pass): the packed (cost, raster index) order makes the result the
// first-in-raster-order winner of the sequential definition. The loads that do not
// depend on the pixel's disparity are issued together, so a pixel costs two dependent
// memory round trips.
// ------------------------------------------------------------------------------------
struct ValidateArgs {
  const uint64_t* cL;
  const uint64_t* cR;
  const uint8_t* omega;
  const float* D_it;
  int32_t W, H, rx, d_min, d_max, t_lo, t_hi, levels;
  int32_t sz, Wc, Hc, cpr, TW, TH, crows;
  uint64_t ginit, binit;
  uint8_t* C_it;
  float* D_f;
  uint8_t* C_f;
  uint64_t* cell_g;
  uint64_t* cell_b;
  uint8_t* mask;
  unsigned long long* n_valid;
};

// NW waves per block; a tile of cpr x crows cells, each wave taking every NW-th row.
// The launcher picks NW per frame size: few waves per block (many rows per wave) once
// the grid alone fills the chip, more waves per block on small frames.
template <int NW>
__device__ __forceinline__ void validate_block(const ValidateArgs& a, int bx, int by) {
  __shared__ uint64_t sg[NW][kWave];
  __shared__ uint64_t sb[NW][kWave];
  __shared__ unsigned int s_valid;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_valid = 0;
  const int x0 = bx * a.TW, y0 = by * a.TH;
  const uint64_t none = ~0ull;
  uint64_t kg = none, kb = none;
  unsigned int nvalid = 0;
  // two rows (r, r + NW) per step: both rows' loads are in flight together
  for (int r = w; r < a.TH; r += 2 * NW) {
    for (int c = lane; c < a.TW; c += kWave) {
      const int u = x0 + c;
      if (u >= a.W) break;
      uint32_t idx[2];  // W * H <= 2^26
      bool in[2], om[2];
      float Dv[2];
      uint64_t wl[2], wr[2];
      uint32_t cf[2], cost[2];
      int dd[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int v = y0 + r + k * NW;
        in[k] = r + k * NW < a.TH && v < a.H;
        idx[k] = (uint32_t)(in[k] ? v : 0) * (uint32_t)a.W + (uint32_t)u;
        om[k] = in[k] && a.omega[idx[k]] != 0;
        Dv[k] = in[k] ? a.D_it[idx[k]] : 0.0f;
        wl[k] = in[k] ? a.cL[idx[k]] : 0ull;
        cf[k] = in[k] ? a.C_f[idx[k]] : 0u;
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        dd[k] = -1;
        if (om[k] && isfinite(Dv[k])) {
          const float f = floorf(__fadd_rn(Dv[k], 0.5f));
          if (f >= (float)a.d_min && f <= (float)a.d_max) {
            const int d = (int)f;
            if (u - d >= a.rx) dd[k] = d;
          }
        }
        wr[k] = dd[k] >= 0 ? a.cR[idx[k] - dd[k]] : 0ull;
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (!in[k]) continue;
        cost[k] = dd[k] >= 0 ? (uint32_t)__popcll(wl[k] ^ wr[k]) : 0xffu;
        if (a.levels > 1 && dd[k] >= 0) {  // neighbouring levels d -+ 1 .. (L-1)/2
          for (int dl = 1; dl <= (a.levels - 1) >> 1; ++dl) {
            const int dm = dd[k] - dl, dp = dd[k] + dl;
            if (dm >= a.d_min)
              cost[k] = min(cost[k], (uint32_t)__popcll(wl[k] ^ a.cR[idx[k] - dm]));
            if (dp <= a.d_max && u - dp >= a.rx)
              cost[k] = min(cost[k], (uint32_t)__popcll(wl[k] ^ a.cR[idx[k] - dp]));
          }
        }
        const uint32_t i = idx[k];
        if (a.C_it) a.C_it[i] = (uint8_t)cost[k];
        uint32_t cfk = cf[k];
        if (cost[k] < cfk) {  // never true for 0xff: C_f <= t_hi <= 64
          a.D_f[i] = Dv[k];
          a.C_f[i] = (uint8_t)cost[k];
          cfk = cost[k];
        }
        if (a.mask) {
          const bool mk = om[k] && cfk < (uint32_t)a.t_hi;
          a.mask[i] = mk;
          nvalid += mk;
        }
        if (cost[k] < (uint32_t)a.t_lo) {
          const uint64_t key = (uint64_t)cost[k] << 32 | (uint64_t)i;
          kg = key < kg ? key : kg;
        } else if (cost[k] != 0xffu && cost[k] > (uint32_t)a.t_hi) {
          const uint64_t key = (uint64_t)(255u - cost[k]) << 32 | (uint64_t)i;
          kb = key < kb ? key : kb;
        }
      }
    }
  }
  // segmented minimum over lanes of the same cell column (segments of sz lanes)
  const int seg = a.sz <= kWave ? lane / a.sz : 0;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint64_t og = __shfl_down(kg, off, kWave);
    const uint64_t ob = __shfl_down(kb, off, kWave);
    const int ol = lane + off;
    if (ol < kWave && (a.sz <= kWave ? ol / a.sz : 0) == seg) {
      kg = og < kg ? og : kg;
      kb = ob < kb ? ob : kb;
    }
  }
  sg[w][lane] = kg;
  sb[w][lane] = kb;
  if (a.mask) {  // the wave's count, one LDS atomic per wave
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) nvalid += __shfl_xor(nvalid, off, kWave);
  }
  __syncthreads();  // s_valid initialised, keys visible
  if (a.mask && lane == 0 && nvalid) atomicAdd(&s_valid, nvalid);
  // thread (w, lane): cell row w of the tile, cell column seg (segment heads only)
  const bool head = lane == 0 || (a.sz <= kWave && (lane - 1) / a.sz != seg);
  if (w < a.crows && head && seg < a.cpr) {
    const int cy = by * a.crows + w, cx = bx * a.cpr + seg;
    if (cy < a.Hc && cx < a.Wc) {
      uint64_t g = a.ginit, b = a.binit;
      // the waves whose rows belong to cell row w: rows w*sz .. w*sz+sz-1 are handled by
      // waves (row mod NW); with crows > 1 every wave holds rows of one cell row only
      const int w_lo = a.crows == 1 ? 0 : w * a.sz;
      const int w_hi = a.crows == 1 ? NW : w * a.sz + a.sz;
      for (int q = w_lo; q < w_hi; ++q) {
        g = sg[q][lane] < g ? sg[q][lane] : g;
        b = sb[q][lane] < b ? sb[q][lane] : b;
      }
      a.cell_g[(size_t)cy * a.Wc + cx] = g;
      a.cell_b[(size_t)cy * a.Wc + cx] = b;
    }
  }
  if (a.mask) {
    __syncthreads();
    if (threadIdx.x == 0 && s_valid) atomicAdd(a.n_valid, (unsigned long long)s_valid);
  }
}

template <int NW>
__global__ __launch_bounds__(kWave * NW, 8) void k_validate(ValidateArgs a) {
  validate_block<NW>(a, blockIdx.x, blockIdx.y);
}

inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

// validate launch shape: 2048 waves is 8 per CU, enough to cover HBM latency
constexpr int kValMaxWaves = 16;
constexpr size_t kValMinWaves = 2048;

}  // namespace

__host__ __device__ inline MatchArgs match_args(const uint64_t* cL, const uint64_t* cR, int32_t W, int32_t H,
                                                const sm_params& p, sm_support* slots, int32_t n) {
  MatchArgs a;
  a.cL = cL;
  a.cR = cR;
  a.W = W;
  a.H = H;
  a.rx = (p.census_w - 1) / 2;
  a.ry = (p.census_h - 1) / 2;
  a.d_min = p.d_min;
  a.d_max = p.d_max;
  a.t_hi = p.t_hi;
  a.uniq = p.uniqueness;
  a.lr_tol = p.lr_tol;
  a.slots = slots;
  a.n = n;
  return a;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  SM_LAUNCH(k_fill_u8, dim3(blocks_for(bytes, 256)), dim3(256), 0, s, (uint8_t*)p, bytes,
                     (uint8_t)0);
  return hipGetLastError();
}

hipError_t launch_census(const CensusJob* jobs, int n_jobs, int32_t W, int32_t H, int32_t cw,
                         int32_t ch, int32_t grad_thr, float* D_f, uint8_t* C_f, int32_t t_hi,
                         uint8_t* occ, const CensusExtras* extras, hipStream_t s, int32_t rows) {
  if (rows == 0) rows = census_rows_for(W, H, cw, ch, false);
  if (rows != 8 && rows != 16 && rows != 32) return hipErrorInvalidValue;
  CensusArgs a{};
  a.th = rows;
  if (extras) a.x = *extras;
  for (int i = 0; i < n_jobs; ++i) a.job[i] = jobs[i];
  a.W = W;
  a.H = H;
  a.grad_thr = grad_thr;
  a.t_hi = t_hi;
  a.D_f = D_f;
  a.C_f = C_f;
  a.occ = occ;
  const int rx = (cw - 1) / 2, ry = (ch - 1) / 2;
#define SM_CENSUS_CASE(X, Y) \
  if (rx == X && ry == Y) return census_launch<X, Y>(a, n_jobs, s);
  SM_CENSUS_CASE(1, 1) SM_CENSUS_CASE(1, 2) SM_CENSUS_CASE(1, 3) SM_CENSUS_CASE(1, 4)
  SM_CENSUS_CASE(2, 1) SM_CENSUS_CASE(2, 2) SM_CENSUS_CASE(2, 3) SM_CENSUS_CASE(2, 4)
  SM_CENSUS_CASE(3, 1) SM_CENSUS_CASE(3, 2) SM_CENSUS_CASE(3, 3) SM_CENSUS_CASE(3, 4)
  SM_CENSUS_CASE(4, 1) SM_CENSUS_CASE(4, 2) SM_CENSUS_CASE(4, 3)
#undef SM_CENSUS_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_grid_slots(const uint8_t* omega, int32_t W, int32_t H, int32_t step,
                             sm_support* slots, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int h = step / 2;
  const int gw = (W - 1 - h) / step + 1;
  SM_LAUNCH(k_grid_slots, dim3(blocks_for(n, 256)), dim3(256), 0, s, omega, W, step, gw,
                     slots, n);
  return hipGetLastError();
}

hipError_t launch_fast_score(const uint8_t* img, int32_t stride, int32_t W, int32_t H, uint8_t* score,
                             hipStream_t s) {
  SM_LAUNCH(k_fast_score, dim3(blocks_for(W, kWave), blocks_for(H, 4)), dim3(256), 0, s, img, stride, W, H,
            score);
  return hipGetLastError();
}

hipError_t launch_fast_select(const uint8_t* score, int32_t W, int32_t H, const sm_params& p,
                              sm_support* slots, int16_t* uv, hipStream_t s) {
  FastSelectArgs a;
  a.score = score;
  a.W = W;
  a.H = H;
  a.t = p.fast_threshold;
  a.bins_x = p.fast_bins_x;
  a.bins_y = p.fast_bins_y;
  a.per_bin = p.fast_per_bin;
  a.slots = slots;
  a.uv = uv;
  SM_LAUNCH(k_fast_select, dim3((unsigned)(p.fast_bins_x * p.fast_bins_y)), dim3(kFastThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_compact_uv(int16_t* uv, int32_t n, int32_t* n_out, hipStream_t s) {
  SM_LAUNCH(k_compact_uv, dim3(1), dim3(1024), 0, s, uv, n, n_out);
  return hipGetLastError();
}

hipError_t launch_list_slots(const int16_t* uv, int32_t n, sm_support* slots, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  SM_LAUNCH(k_list_slots, dim3(blocks_for(n, 256)), dim3(256), 0, s, uv, n, slots);
  return hipGetLastError();
}

int32_t match_lanes_for(int32_t W, int32_t H, const sm_params& p) {
  const int32_t tuned = tuned_choice(kTuneMatchLanes, W, H, p.d_max - p.d_min + 1);
  return tuned == 16 || tuned == 32 ? tuned : kWave;
}

int32_t match_units(int32_t n, int32_t lanes) { return (n + kWave / lanes - 1) / (kWave / lanes); }

hipError_t launch_match_lanes(const uint64_t* cL, const uint64_t* cR, int32_t W, int32_t H, const sm_params& p,
                              sm_support* slots, int32_t n, int32_t lanes, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const MatchArgs a = match_args(cL, cR, W, H, p, slots, n);
  const dim3 grid(blocks_for(match_units(n, lanes), 4));
  switch (lanes) {
    case 16: SM_LAUNCH(k_match<16>, grid, dim3(256), 0, s, a); break;
    case 32: SM_LAUNCH(k_match<32>, grid, dim3(256), 0, s, a); break;
    case kWave: SM_LAUNCH(k_match<kWave>, grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_match(const uint64_t* cL, const uint64_t* cR, int32_t W, int32_t H,
                        const sm_params& p, sm_support* slots, int32_t n, hipStream_t s) {
  return launch_match_lanes(cL, cR, W, H, p, slots, n, match_lanes_for(W, H, p), s);
}

hipError_t launch_compact(sm_support* slots, int32_t n, int32_t* n_out, uint8_t* occ, int32_t W,
                          int32_t* header, hipStream_t s, const int32_t* slot_off, int32_t slot_cap) {
  SM_LAUNCH(k_compact, dim3(1), dim3(1024), 0, s, slots, n, n_out, occ, W, header, slot_off, (int)slot_cap);
  return hipGetLastError();
}

hipError_t launch_mark(const sm_support* S, int32_t n, uint8_t* occ, int32_t W, int32_t H,
                       hipStream_t s) {
  const size_t npx = (size_t)W * H;
  SM_LAUNCH(k_fill_u8, dim3(blocks_for(npx, 256)), dim3(256), 0, s, occ, npx, (uint8_t)0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n <= 0) return e;
  SM_LAUNCH(k_mark, dim3(blocks_for(n, 256)), dim3(256), 0, s, S, n, occ, W, H);
  return hipGetLastError();
}

hipError_t launch_fill_nan(float* D, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  SM_LAUNCH(k_fill_f32, dim3(std::min<unsigned>(blocks_for((n + 3) / 4, 256), 8192u)), dim3(256), 0, s, D, n,
            __builtin_nanf(""));
  return hipGetLastError();
}

hipError_t launch_raster_blocks(const sm_support* S, int32_t n_support, const sm_tri* T, int32_t n_tris,
                                int32_t W, int32_t H, float* D_it, hipStream_t s, const int32_t* counts,
                                int32_t max_blocks) {
  if (n_tris <= 0) return hipSuccess;
  if (!counts || max_blocks < 1) return hipErrorInvalidValue;
  const unsigned blocks = std::min<unsigned>(blocks_for(n_tris, 4 * kTriPerWave), (unsigned)max_blocks);
  SM_LAUNCH(k_raster_group, dim3(blocks), dim3(256), 0, s, S, n_support, T, n_tris, W, H, D_it, counts);
  return hipGetLastError();
}

hipError_t launch_raster(const sm_support* S, int32_t n_support, const sm_tri* T, int32_t n_tris,
                         int32_t W, int32_t H, float* D_it, hipStream_t s, const int32_t* counts) {
  if (n_tris <= 0) return hipSuccess;
  if (counts) {  // the count is known on the device only: a bounded grid of the group layout
    const int32_t tuned = tuned_choice(kTuneRasterBlocks, W, H, 0);
    return launch_raster_blocks(S, n_support, T, n_tris, W, H, D_it, s, counts,
                                tuned > 0 ? tuned : kRasterStrideBlocks);
  } else if (n_tris < kGroupLayoutMinTris) {
    SM_LAUNCH(k_raster_wave, dim3(blocks_for(n_tris, 4)), dim3(256), 0, s, S, n_support, T, n_tris, W,
              H, D_it, counts);
  } else {
    SM_LAUNCH(k_raster_group, dim3(blocks_for(n_tris, 4 * kTriPerWave)), dim3(256), 0, s, S, n_support,
              T, n_tris, W, H, D_it, counts);
  }
  return hipGetLastError();
}

hipError_t launch_interpolate(const sm_support* S, int32_t n_support, const sm_tri* T, int32_t n_tris,
                              int32_t W, int32_t H, float* D_it, hipStream_t s) {
  hipError_t e = launch_fill_nan(D_it, (size_t)W * H, s);
  if (e != hipSuccess) return e;
  return launch_raster(S, n_support, T, n_tris, W, H, D_it, s);
}

// Validation arguments of one frame for blocks of nw waves.
__host__ __device__ inline ValidateArgs validate_args(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega,
                                                      const float* D_it, int32_t W, int32_t H, const sm_params& p,
                                                      int32_t sz, int nw, uint8_t* C_it, float* D_f, uint8_t* C_f,
                                                      uint64_t* cell_g, uint64_t* cell_b, uint8_t* mask,
                                                      unsigned long long* n_valid) {
  ValidateArgs a;
  a.cL = cL;
  a.cR = cR;
  a.omega = omega;
  a.D_it = D_it;
  a.W = W;
  a.H = H;
  a.rx = (p.census_w - 1) / 2;
  a.d_min = p.d_min;
  a.d_max = p.d_max;
  a.t_lo = p.t_lo;
  a.t_hi = p.t_hi;
  a.levels = p.levels;
  a.sz = sz;
  a.Wc = (W + sz - 1) / sz;
  a.Hc = (H + sz - 1) / sz;
  a.cpr = sz <= kWave ? kWave / sz : 1;
  a.TW = a.cpr * sz;
  a.crows = sz >= nw ? 1 : nw / sz;
  a.TH = a.crows * sz;
  a.ginit = (uint64_t)p.t_lo << 32;
  a.binit = (uint64_t)(255 - p.t_hi) << 32;
  a.C_it = C_it;
  a.D_f = D_f;
  a.C_f = C_f;
  a.cell_g = cell_g;
  a.cell_b = cell_b;
  a.mask = mask;
  a.n_valid = n_valid;
  return a;
}

int32_t validate_blocks(int32_t W, int32_t H, int32_t sz, int nw) {
  const int cpr = sz <= kWave ? kWave / sz : 1;
  const int crows = sz >= nw ? 1 : nw / sz;
  return (int32_t)(blocks_for(W, cpr * sz) * blocks_for(H, crows * sz));
}

int validate_pick_nw(int64_t (*waves)(int nw, void* ctx), void* ctx) {
  int nw = 1;
  while (nw < kValMaxWaves && waves(nw, ctx) < (int64_t)kValMinWaves) nw *= 2;
  return nw;
}

namespace {
std::mutex g_tune_m;
std::map<std::tuple<int, int32_t, int32_t, int32_t>, int32_t> g_tune;
}  // namespace

int32_t tuned_choice(int kind, int32_t W, int32_t H, int32_t sz) {
  std::lock_guard<std::mutex> lk(g_tune_m);
  const auto it = g_tune.find(std::make_tuple(kind, W, H, sz));
  return it == g_tune.end() ? -1 : it->second;
}

void set_tuned_choice(int kind, int32_t W, int32_t H, int32_t sz, int32_t value) {
  std::lock_guard<std::mutex> lk(g_tune_m);
  if (value == 0) g_tune.erase(std::make_tuple(kind, W, H, sz));
  else g_tune[std::make_tuple(kind, W, H, sz)] = value;
}

hipError_t launch_validate_only(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega,
                                const float* D_it, int32_t W, int32_t H, const sm_params& p,
                                int32_t sz, uint8_t* C_it, float* D_f, uint8_t* C_f,
                                uint64_t* cell_g, uint64_t* cell_b, uint8_t* mask,
                                unsigned long long* n_valid, hipStream_t s) {
  // a measured choice, else the smallest block (most rows per wave) whose grid still
  // holds >= kValMinWaves waves
  struct Ctx {
    int32_t W, H, sz;
  } c{W, H, sz};
  int nw = tuned_choice(kTuneValidateWaves, W, H, sz);
  if (nw < 0)
    nw = validate_pick_nw(
        [](int w, void* x) {
          const Ctx& q = *(const Ctx*)x;
          return (int64_t)validate_blocks(q.W, q.H, q.sz, w) * w;
        },
        &c);
  return launch_validate_nw(cL, cR, omega, D_it, W, H, p, sz, C_it, D_f, C_f, cell_g, cell_b, mask, n_valid, nw, s);
}

hipError_t launch_validate_nw(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega,
                              const float* D_it, int32_t W, int32_t H, const sm_params& p,
                              int32_t sz, uint8_t* C_it, float* D_f, uint8_t* C_f,
                              uint64_t* cell_g, uint64_t* cell_b, uint8_t* mask,
                              unsigned long long* n_valid, int nw, hipStream_t s) {
  if (nw != 1 && nw != 2 && nw != 4 && nw != 8 && nw != 16) return hipErrorInvalidValue;
  const ValidateArgs a = validate_args(cL, cR, omega, D_it, W, H, p, sz, nw, C_it, D_f, C_f, cell_g, cell_b,
                                       mask, n_valid);
  dim3 grid(blocks_for(W, a.TW), blocks_for(H, a.TH));
  switch (nw) {
    case 1: SM_LAUNCH(k_validate<1>, grid, dim3(kWave * 1), 0, s, a); break;
    case 2: SM_LAUNCH(k_validate<2>, grid, dim3(kWave * 2), 0, s, a); break;
    case 4: SM_LAUNCH(k_validate<4>, grid, dim3(kWave * 4), 0, s, a); break;
    case 8: SM_LAUNCH(k_validate<8>, grid, dim3(kWave * 8), 0, s, a); break;
    default: SM_LAUNCH(k_validate<16>, grid, dim3(kWave * 16), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_validate(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega,
                           const float* D_it, int32_t W, int32_t H, const sm_params& p,
                           int32_t sz, uint8_t* C_it, float* D_f, uint8_t* C_f, uint64_t* cell_g,
                           uint64_t* cell_b, uint8_t* mask, unsigned long long* n_valid,
                           hipStream_t s) {
  return launch_validate_only(cL, cR, omega, D_it, W, H, p, sz, C_it, D_f, C_f, cell_g, cell_b, mask,
                              n_valid, s);
}

hipError_t launch_resample(const uint64_t* cL, const uint64_t* cR, const uint64_t* cell_g,
                           const uint64_t* cell_b, const float* D_it, int32_t W, int32_t H, int32_t sz,
                           const sm_params& p, sm_support* slots, const uint8_t* occ, hipStream_t s,
                           const int32_t* slot_off, int32_t slot_cap) {
  const int n_cells = ((W + sz - 1) / sz) * ((H + sz - 1) / sz);
  const uint64_t ginit = (uint64_t)p.t_lo << 32, binit = (uint64_t)(255 - p.t_hi) << 32;
  const MatchArgs a = match_args(cL, cR, W, H, p, slots, 2 * n_cells);
  SM_LAUNCH(k_rematch_cells, dim3(blocks_for(n_cells, 4)), dim3(256), 0, s, a, cell_g, cell_b, D_it, occ,
            n_cells, ginit, binit, slot_off, (int)slot_cap);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Stage-batched kernels: the single-frame device functions above, with work units
// (blocks or waves) mapped to frames by a binary search over the offset array.
// ------------------------------------------------------------------------------------
namespace {

__device__ __forceinline__ int frame_of(const int32_t* off, int n, int unit) {
  int lo = 0, hi = n;  // the last f with off[f] <= unit (frames owning no units are skipped)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= unit) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int RX, int RY>
__global__ __launch_bounds__(256) void k_batch_census(const BatchFrame* F, const int32_t* off, int n) {
  __shared__ uint8_t tile[(kTHMax + 2 * RY) * (kTW + 2 * RX)];
  const int f = frame_of(off, n, blockIdx.x);
  const BatchFrame& fr = F[f];
  const int local = blockIdx.x - off[f];
  const int tx = (fr.W + kTW - 1) / kTW, ty = (fr.H + fr.census_rows - 1) / fr.census_rows;
  const int job = local / (tx * ty), t = local - job * tx * ty;
  CensusArgs a{};  // (the image's job passed on its own: no indexed local array)
  const CensusJob jb = job == 0 ? CensusJob{fr.L, fr.stride, fr.cL, fr.omega} : CensusJob{fr.R, fr.stride, fr.cR, nullptr};
  a.W = fr.W;
  a.H = fr.H;
  a.grad_thr = fr.p.grad_thr;
  a.t_hi = fr.p.t_hi;
  a.th = fr.census_rows;
  a.D_f = fr.D_f;
  a.C_f = fr.C_f;
  a.occ = fr.occ;
  a.x.D_nan = fr.D_it;
  a.x.grid_slots = fr.S;
  a.x.step = fr.p.support_step;
  a.x.gw = fr.gw;
  a.x.zero = fr.counters;
  a.x.n_zero = 16;
  census_block<RX, RY>(a, jb, job == 0, t % tx, t / tx, tile);
}

// a unit is one wave of the frame's candidates, kWave / match_lanes per wave
__global__ __launch_bounds__(256) void k_batch_match(const BatchFrame* F, const int32_t* off, int n, int total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int unit = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (unit >= total) return;
  const int f = frame_of(off, n, unit);
  const BatchFrame& fr = F[f];
  const MatchArgs a = match_args(fr.cL, fr.cR, fr.W, fr.H, fr.p, fr.S, fr.n_grid);
  const int u = unit - off[f];
  if (fr.match_lanes == 16) {
    const int slot = match_unit_slot<16>(u, lane);
    if (slot < a.n) match_slot<16>(a, slot, lane);
  } else if (fr.match_lanes == 32) {
    const int slot = match_unit_slot<32>(u, lane);
    if (slot < a.n) match_slot<32>(a, slot, lane);
  } else {
    const int slot = match_unit_slot<kWave>(u, lane);
    if (slot < a.n) match_slot<kWave>(a, slot, lane);
  }
}

__global__ __launch_bounds__(1024) void k_batch_compact(const BatchFrame* F, int mode) {
  const BatchFrame& fr = F[blockIdx.x];
  if (mode == 0) {
    compact_block(fr.S, fr.n_grid, &fr.counters[0], fr.occ, fr.W, (int32_t*)(fr.S + fr.n_grid));
  } else if (fr.region_n > 0) {
    compact_block(fr.region, fr.region_n, &fr.counters[1], fr.occ, fr.W, (int32_t*)(fr.region + fr.region_n));
  }
}

// Header slot (count) + the compacted supports of frame blockIdx.x into its staging.
__global__ __launch_bounds__(256) void k_batch_pack(const BatchFrame* F, int mode) {
  const BatchFrame& fr = F[blockIdx.x];
  const sm_support* src = mode == 0 ? fr.S : fr.region;
  const int n_slots = mode == 0 ? fr.n_grid : fr.region_n;
  if (!fr.pack || (mode == 1 && n_slots == 0)) return;
  const int count = min(*(const int32_t*)(src + n_slots), fr.pack_cap);
  if (threadIdx.x == 0) *(int32_t*)fr.pack = count;
  for (int i = threadIdx.x; i < count; i += 256) fr.pack[1 + i] = src[i];
}

__global__ __launch_bounds__(256) void k_batch_raster(const BatchFrame* F, const int32_t* off, int n, int total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int unit = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (unit >= total) return;
  const int f = frame_of(off, n, unit);
  const BatchFrame& fr = F[f];
  if (fr.counts) {  // the frame's units stride over its triangles (wave-uniform loop)
    const int units = off[f + 1] - off[f];
    const int n_T = min(fr.T_cap, fr.counts[kCountTris]);
    const int n_S = min(fr.S_cap, fr.counts[kCountSupports]);
    for (int t = unit - off[f]; t < n_T; t += units) raster_tri_wave(fr.S, n_S, fr.T, t, fr.W, fr.H, fr.D_it, lane);
    return;
  }
  raster_tri_wave(fr.S, fr.n_S, fr.T, unit - off[f], fr.W, fr.H, fr.D_it, lane);
}

template <int NW>
__global__ __launch_bounds__(kWave * NW, 8) void k_batch_validate(const BatchFrame* F, const int32_t* off, int n) {
  const int f = frame_of(off, n, blockIdx.x);
  const BatchFrame& fr = F[f];
  const ValidateArgs a = validate_args(fr.cL, fr.cR, fr.omega, fr.D_it, fr.W, fr.H, fr.p, fr.sz, NW, nullptr,
                                       fr.D_f, fr.C_f, fr.cell_g, fr.cell_b, fr.last ? fr.mask : nullptr,
                                       fr.last ? fr.n_valid : nullptr);
  const int local = blockIdx.x - off[f];
  const int gx = (fr.W + a.TW - 1) / a.TW;
  validate_block<NW>(a, local % gx, local / gx);
}

__global__ __launch_bounds__(256) void k_batch_rematch(const BatchFrame* F, const int32_t* off, int n, int total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int unit = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (unit >= total) return;
  const int f = frame_of(off, n, unit);
  const BatchFrame& fr = F[f];
  const int n_cells = fr.region_n / 2;
  sm_support* region = fr.region;
  if (fr.counts) {  // the region follows the supports counted on the device
    const int32_t o = fr.counts[kCountSupports];
    if (o < 0 || (int64_t)o + fr.region_n + 1 > fr.S_cap) return;  // a failed mesh: the frame is redone
    region = fr.S + o;
  }
  const MatchArgs a = match_args(fr.cL, fr.cR, fr.W, fr.H, fr.p, region, fr.region_n);
  rematch_cell(a, fr.cell_g, fr.cell_b, fr.D_it, fr.occ, n_cells, (uint64_t)fr.p.t_lo << 32,
               (uint64_t)(255 - fr.p.t_hi) << 32, unit - off[f], lane);
}

}  // namespace

int32_t census_tiles(int32_t W, int32_t H, int32_t rows) {
  return (int32_t)(blocks_for(W, kTW) * blocks_for(H, (unsigned)rows));
}

int32_t census_rows_for(int32_t W, int32_t H, int32_t cw, int32_t ch, bool batched) {
  const int32_t tuned = tuned_choice(kTuneCensusRows, W, H, ((cw - 1) / 2) << 8 | ((ch - 1) / 2));
  if (tuned == 8 || tuned == 16 || tuned == 32) return tuned;
  return batched ? kTHBatch : kTHFrame;
}

hipError_t launch_batch_census(const BatchFrame* F, const int32_t* off, int32_t n, int32_t total, int rx, int ry,
                               hipStream_t s) {
  if (total <= 0) return hipSuccess;
#define SM_BATCH_CENSUS_CASE(X, Y)                                                                     \
  if (rx == X && ry == Y) {                                                                            \
    SM_LAUNCH((k_batch_census<X, Y>), dim3((unsigned)total), dim3(kTW, 4, 1), 0, s, F, off, (int)n); \
    return hipGetLastError();                                                                          \
  }
  SM_BATCH_CENSUS_CASE(1, 1) SM_BATCH_CENSUS_CASE(1, 2) SM_BATCH_CENSUS_CASE(1, 3) SM_BATCH_CENSUS_CASE(1, 4)
  SM_BATCH_CENSUS_CASE(2, 1) SM_BATCH_CENSUS_CASE(2, 2) SM_BATCH_CENSUS_CASE(2, 3) SM_BATCH_CENSUS_CASE(2, 4)
  SM_BATCH_CENSUS_CASE(3, 1) SM_BATCH_CENSUS_CASE(3, 2) SM_BATCH_CENSUS_CASE(3, 3) SM_BATCH_CENSUS_CASE(3, 4)
  SM_BATCH_CENSUS_CASE(4, 1) SM_BATCH_CENSUS_CASE(4, 2) SM_BATCH_CENSUS_CASE(4, 3)
#undef SM_BATCH_CENSUS_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_batch_match(const BatchFrame* F, const int32_t* off, int32_t n, int32_t total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  SM_LAUNCH(k_batch_match, dim3(blocks_for(total, 4)), dim3(256), 0, s, F, off, (int)n, (int)total);
  return hipGetLastError();
}

hipError_t launch_batch_compact(const BatchFrame* F, int32_t n, int mode, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  SM_LAUNCH(k_batch_compact, dim3((unsigned)n), dim3(1024), 0, s, F, mode);
  return hipGetLastError();
}

hipError_t launch_batch_pack(const BatchFrame* F, int32_t n, int mode, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  SM_LAUNCH(k_batch_pack, dim3((unsigned)n), dim3(256), 0, s, F, mode);
  return hipGetLastError();
}

hipError_t launch_batch_raster(const BatchFrame* F, const int32_t* off, int32_t n, int32_t total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  SM_LAUNCH(k_batch_raster, dim3(blocks_for(total, 4)), dim3(256), 0, s, F, off, (int)n, (int)total);
  return hipGetLastError();
}

hipError_t launch_batch_validate(const BatchFrame* F, const int32_t* off, int32_t n, int32_t total, int nw,
                                 hipStream_t s) {
  if (total <= 0) return hipSuccess;
  const dim3 grid((unsigned)total);
  switch (nw) {
    case 1: SM_LAUNCH(k_batch_validate<1>, grid, dim3(kWave * 1), 0, s, F, off, (int)n); break;
    case 2: SM_LAUNCH(k_batch_validate<2>, grid, dim3(kWave * 2), 0, s, F, off, (int)n); break;
    case 4: SM_LAUNCH(k_batch_validate<4>, grid, dim3(kWave * 4), 0, s, F, off, (int)n); break;
    case 8: SM_LAUNCH(k_batch_validate<8>, grid, dim3(kWave * 8), 0, s, F, off, (int)n); break;
    default: SM_LAUNCH(k_batch_validate<16>, grid, dim3(kWave * 16), 0, s, F, off, (int)n); break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_rematch(const BatchFrame* F, const int32_t* off, int32_t n, int32_t total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  SM_LAUNCH(k_batch_rematch, dim3(blocks_for(total, 4)), dim3(256), 0, s, F, off, (int)n, (int)total);
  return hipGetLastError();
}

}  // namespace sm
