// Shared host-side helpers of the stereomesh library: error state, HIP checks and
// parameter validation. Internal header.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "stereomesh.h"

namespace sm {

// Thread-local message of the last non-OK status.
std::string& last_error();
sm_status fail(sm_status st, const char* fmt, ...);

#define SM_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::sm::fail(SM_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                          \
  } while (0)

#define SM_TRY(expr)                     \
  do {                                   \
    sm_status s_ = (expr);               \
    if (s_ != SM_OK) return s_;          \
  } while (0)

constexpr int kMaxDim = 8192;

inline bool dims_ok(int32_t W, int32_t H) { return W >= 3 && H >= 3 && W <= kMaxDim && H <= kMaxDim; }

inline bool census_ok(int32_t cw, int32_t ch) {
  return cw >= 3 && ch >= 3 && (cw & 1) && (ch & 1) && cw * ch - 1 <= 64 && cw <= 9 && ch <= 9;
}

sm_status check_params(const sm_params* p);
sm_status check_fast_params(const sm_params* p);

// Candidate slots of the FAST detector: fast_per_bin per bin.
inline int64_t fast_slots(const sm_params& p) {
  return (int64_t)p.fast_bins_x * p.fast_bins_y * p.fast_per_bin;
}

inline int32_t occ_size(const sm_params& p, int it) {  // it is 1-based
  int32_t sz = p.sz_occ0;
  for (int k = 1; k < it; ++k) sz = sz / 2 > 1 ? sz / 2 : 1;
  return sz;
}

inline int32_t cells_of(int32_t W, int32_t H, int32_t sz) {
  return ((H + sz - 1) / sz) * ((W + sz - 1) / sz);
}

inline int32_t grid_count(int32_t W, int32_t H, int32_t step) {
  int32_t h = step / 2;
  if (h >= W || h >= H) return 0;
  return ((W - 1 - h) / step + 1) * ((H - 1 - h) / step + 1);
}

// Workspace of one sm_solve frame: byte offsets of its buffers (see sm_solve).
struct Layout {
  size_t cL, cR, omega, occ, D_it, cell_g, cell_b, S, T, counters, score, total;
  int32_t n_grid, S_cap, T_cap, cells_max;  // n_grid: initial candidate slots (grid or FAST)
  // device meshes (host_mesh == 0): the status words and the star kernels' arrays
  bool mesh_on;
  size_t mstatus, mwork;
};
Layout layout_of(int32_t W, int32_t H, const sm_params& p);  // p must have passed check_params
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace sm
