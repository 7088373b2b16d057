// Rasterisation of one triangle into the dense disparity prior D_it (Sec. III-B: the
// plane of each triangle of G(S) through its three supports, Eq. 3, evaluated at the
// pixels it owns): the set-up, the exact column span of each row and the row writes.
// Shared by the raster kernels (kernels.hip) and the star kernel, which rasterises each
// star's triangles as soon as it has found them (star.hip). Internal header.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "stereomesh.h"

namespace sm {

// A triangle ready for rasterisation. Row v of the owned region is the column range
// [lo, hi] = [umin, umax] cut by the three edges. With edge e running from vertex e to
// vertex e + 1 (dx, dy) and E = dx (v - ya) - dy (u - xa), the perturbed point of pixel
// (u, v) is on the triangle's side when E > 0; E = 0 is settled by the perturbation:
// inside for dy < 0, outside for dy > 0, inside for a horizontal edge iff dx > 0. So
// dy < 0 bounds u below by xa + ceil(-dx (v - ya) / -dy), dy > 0 bounds it above by
// xa + ceil(dx (v - ya) / dy) - 1, and a horizontal edge admits rows v >= ya (dx > 0)
// or v < ya (dx < 0), which setup folds into the row range. Each bound is
// ceil((A v + B) / d) + C with per-edge constants.
struct RasterTri {
  int A[3], B[3], C[3], d[3];
  float rc[3];          // 1 / d to within 1 ulp
  int kind[3];          // 0: lower bound on u, 1: upper bound, 2: none (horizontal edge)
  float a, b, d0;       // plane in anchor form
  int u0, v0;           // anchor
  int vmin, vmax, umin, umax;
  bool ok;
};

// Setup of triangle tr (vertex ids into S). Triangles that own nothing (malformed indices,
// vertices outside [0, 8191], not positively oriented, or outside the image) come back
// with ok = false.
__device__ __forceinline__ RasterTri raster_setup_tri(const sm_support* S, int n_support, sm_tri tr, int W,
                                                      int H) {
  RasterTri r = {};
  r.ok = false;
  if ((unsigned)tr.i0 >= (unsigned)n_support || (unsigned)tr.i1 >= (unsigned)n_support ||
      (unsigned)tr.i2 >= (unsigned)n_support)
    return r;
  const sm_support s0 = S[tr.i0], s1 = S[tr.i1], s2 = S[tr.i2];
  const int x[3] = {s0.u, s1.u, s2.u}, y[3] = {s0.v, s1.v, s2.v};
  if ((unsigned)(x[0] | y[0] | x[1] | y[1] | x[2] | y[2]) > 8191u) return r;
  const int du1 = x[1] - x[0], dv1 = y[1] - y[0], du2 = x[2] - x[0], dv2 = y[2] - y[0];
  const int det = du1 * dv2 - du2 * dv1;
  if (det <= 0) return r;
  const double e1 = __dadd_rn((double)s1.d, -(double)s0.d);
  const double e2 = __dadd_rn((double)s2.d, -(double)s0.d);
  const double ddet = (double)det;
  r.a = (float)__ddiv_rn(__dadd_rn(__dmul_rn(e1, (double)dv2), -__dmul_rn(e2, (double)dv1)), ddet);
  r.b = (float)__ddiv_rn(__dadd_rn(__dmul_rn((double)du1, e2), -__dmul_rn((double)du2, e1)), ddet);
  r.d0 = s0.d;
  r.u0 = x[0];
  r.v0 = y[0];
  int vlo = max(min(y[0], min(y[1], y[2])), 0);
  int vhi = min(max(y[0], max(y[1], y[2])), H - 1);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int xa = x[e], ya = y[e], dx = x[(e + 1) % 3] - xa, dy = y[(e + 1) % 3] - ya;
    if (dy == 0) {
      if (dx > 0) vlo = max(vlo, ya);
      else vhi = min(vhi, ya - 1);
      r.A[e] = 0, r.B[e] = 0, r.C[e] = 0, r.d[e] = 1, r.rc[e] = 1.0f, r.kind[e] = 2;
    } else if (dy < 0) {
      r.A[e] = -dx, r.B[e] = dx * ya, r.C[e] = xa, r.d[e] = -dy, r.kind[e] = 0;
    } else {
      r.A[e] = dx, r.B[e] = -dx * ya, r.C[e] = xa - 1, r.d[e] = dy, r.kind[e] = 1;
    }
    if (dy != 0) r.rc[e] = __builtin_amdgcn_rcpf((float)r.d[e]);
  }
  r.vmin = vlo;
  r.vmax = vhi;
  r.umin = max(min(x[0], min(x[1], x[2])), 0);
  r.umax = min(max(x[0], max(x[1], x[2])), W - 1);
  r.ok = r.vmin <= r.vmax && r.umin <= r.umax;
  return r;
}

// ceil((A v + B) / d) + C, given |A v + B| < 2^26, 1 <= d <= 8192 and rc = 1/d within
// 1 ulp: a float estimate (within |q| 2^-22 of the quotient q) corrected once by the
// exact integer remainder. Exact whenever |q| < 2^18, where the remainder cannot wrap;
// larger quotients put the bound beyond any 8192-column image, where an estimate off by
// a few units has the same effect.
__device__ __forceinline__ int edge_bound(int A, int B, int C, int d, float rc, int v) {
  const int n = A * v + B;
  int q = (int)ceilf(__fmul_rn((float)n, rc));
  const int rem = (int)((unsigned)q * (unsigned)d - (unsigned)n);
  q += (rem < 0) - (rem >= d);
  return q + C;
}

// Owned columns [lo, hi] of row v (empty when hi < lo); no branches, so lanes working on
// different triangles stay converged.
__device__ __forceinline__ void raster_span(const RasterTri& r, int v, int& lo, int& hi) {
  lo = r.umin;
  hi = r.umax;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int bound = edge_bound(r.A[e], r.B[e], r.C[e], r.d[e], r.rc[e], v);
    lo = max(lo, r.kind[e] == 0 ? bound : INT_MIN);
    hi = min(hi, r.kind[e] == 1 ? bound : INT_MAX);
  }
}

// D = (d0 + a * (u - u0)) + b * (v - v0), each operation rounded, along [lo, hi] of row
// v; (float)(u - u0) is stepped by exact +1 increments (integers below 2^24).
__device__ __forceinline__ void raster_row(const RasterTri& r, int v, int lo, int hi, float* row) {
  const float tv = __fmul_rn(r.b, (float)(v - r.v0));
  float fu = (float)(lo - r.u0);
  int u = lo;
  for (; u < hi; u += 2) {
    row[u] = __fadd_rn(__fadd_rn(r.d0, __fmul_rn(r.a, fu)), tv);
    row[u + 1] = __fadd_rn(__fadd_rn(r.d0, __fmul_rn(r.a, __fadd_rn(fu, 1.0f))), tv);
    fu = __fadd_rn(fu, 2.0f);
  }
  if (u == hi) row[u] = __fadd_rn(__fadd_rn(r.d0, __fmul_rn(r.a, fu)), tv);
}

// Setup of triangle t of T.
__device__ __forceinline__ RasterTri raster_setup(const sm_support* S, int n_support, const sm_tri* T, int t, int W,
                                                  int H) {
  return raster_setup_tri(S, n_support, T[t], W, H);
}

// The owned rows of r, lanes rl, rl + nl, rl + 2 nl, ... of a group of nl lanes.
__device__ __forceinline__ void raster_rows(const RasterTri& r, int rl, int nl, int W, float* D) {
  if (!r.ok) return;
  for (int v = r.vmin + rl; v <= r.vmax; v += nl) {
    int lo, hi;
    raster_span(r, v, lo, hi);
    raster_row(r, v, lo, hi, D + (size_t)v * W);
  }
}

}  // namespace sm
