// Delaunay triangulation of a frame's supports as independent per-point stars (Sec. III-A,
// the mesh G(S) of Alg. 1): the shared steps of the device kernel (star.hip) and of the
// sequential CPU driver of the tests.
//
// The Delaunay triangulation under the perturbed in-circle test (simulation of simplicity on
// the lifted heights, the rule of predicates.hpp and of the host triangulation) is unique, so
// the triangles around each point -- its star -- can be computed for every point on its own,
// with no shared mesh and no rounds:
//   1. the point's nearest neighbour q (smallest squared distance, then smallest id) is a
//      Delaunay neighbour: the circle with diameter pq holds no other point, not even on its
//      boundary, so it stays empty under any perturbation of the heights;
//   2. around p, counter-clockwise from q: the triangle left of the Delaunay edge p -> a is
//      (p, a, b) with b the point strictly left of p -> a that no other point beats, c
//      beating b when c lies inside the circle through (p, a, b) under the perturbed test.
//      The circles through p and a cut nested caps out of the left half-plane, so this is a
//      total order, any reduction order finds the best, and a point that beats b lies in
//      b's cap. b is the next neighbour; the walk closes when it comes back to q;
//   3. when no point at all lies strictly left of p -> a, that edge is on the convex hull:
//      the walk then goes clockwise from q (the triangle left of a -> p) to the other hull
//      edge.
// Points are found through a bucket grid of kStarCell px cells. The walk takes its
// candidates from the square of cells around p's cell; the best of them, b, is then checked
// against every cell outside the square that b's cap -- the part of the disk through
// (p, a, b) left of the edge -- can reach (band by band of cells, from the disk's exact
// chord and the cap's bounding box, widened by a margin): the best over both is the
// triangle's third vertex, since any point that beats it lies in a cap nested inside b's.
// So the triangles are exact whatever the square; its size only decides how much is
// scanned twice. A step with no candidate in the square takes the best of the frame's row
// extremes (the points with the smallest and the largest u of every pixel row) instead:
// some point lies strictly left of the edge iff some row extreme does, and the hull
// vertices that bound the long triangles of such steps are row extremes, so the cap to
// check is usually tight. A cap that covers far more cells than the square is first
// shrunk by the best of a square of twice the reach (next_vertex). The nearest neighbour
// is taken from a square that certainly holds every point nearer than the one found.
// Each triangle is written once, by its vertex with the smallest raster position (v, u),
// as (i0, i1, i2) counter-clockwise -- the canonical form of sm_tri.
//
// The steps are written for a group of kN lanes (a wavefront of 64 on the device, one lane
// on the host), the WV object: lanes share out the points of a square (wv.for_candidates;
// the walk's square, named by wv.set_base, may be staged) or of a list of cell runs
// (wv.for_rows), and combine their best by its reductions (any, min_u64, reduce_best, and
// pick: a value of the first lane for which a condition holds); every control decision is
// uniform across the group.
#pragma once

#include <cmath>
#include <cstdint>

#include "predicates.hpp"

namespace sm {
namespace star {

using geom::P2;
using geom::incircle_sos;
using geom::orient;

constexpr int32_t kStarCell = 16;      // bucket cell side, px
constexpr int32_t kStarMaxSteps = 4096;  // bound on a walk around one point
constexpr double kDiskMargin = 2.0;      // px added around a disk's computed extent

// error codes of a frame's status word (0: ok); any of them sends the frame's meshes to the host
enum : int32_t {
  kStarOk = 0,
  kStarErrDup = 20,       // two supports on one pixel
  kStarErrSteps = 21,     // a walk around one point did not close within kStarMaxSteps
  kStarErrIndex = 22,     // a point id outside the frame's supports
  kStarErrCapacity = 23,  // more supports or triangles than the frame's arrays hold
  kStarErrSupport = 24,   // a support outside the frame
  kStarErrSets = 25       // a star with more full triangle sets than its 16-lane group records
                          // for their rasterisation
};

// A cell entry: a point id and its packed coordinates.
struct alignas(8) CellEntry {
  int32_t id, uv;
};
// A pixel row's extreme points: smallest and largest u (lo > hi: no point in the row) and
// their ids.
struct alignas(16) RowExt {
  int32_t lo, hi, lo_id, hi_id;
};

struct Grid {
  const int32_t* uv;          // [n] packed coordinates u | v << 16
  int32_t n;
  int32_t W, H;
  int32_t gw, gh;             // cells across / down
  const int32_t* cell_start;   // [gw * gh + 1] first entry of each cell in cell_e
  const CellEntry* cell_e;     // [n] the points ordered by cell (row-major cells)
  const RowExt* rows;          // [H] extreme points of every pixel row
};

__host__ __device__ inline P2 unpack(int32_t w) { return P2{w & 0xffff, (int32_t)((uint32_t)w >> 16)}; }

// Square of cells around p's cell and the radius it certainly covers.
struct Region {
  int32_t k;    // cells around p's cell
  int32_t x0, x1, y0, y1;
  bool full;    // every cell: nothing lies outside
  int64_t R2;   // every point outside lies at distance >= R from p (R2 = R^2)
};

__host__ __device__ inline Region region_of(const Grid& g, P2 P, int32_t k) {
  const int32_t cx = P.x / kStarCell, cy = P.y / kStarCell;
  Region r;
  r.k = k;
  r.x0 = cx - k > 0 ? cx - k : 0;
  r.y0 = cy - k > 0 ? cy - k : 0;
  r.x1 = cx + k < g.gw - 1 ? cx + k : g.gw - 1;
  r.y1 = cy + k < g.gh - 1 ? cy + k : g.gh - 1;
  r.full = r.x0 == 0 && r.y0 == 0 && r.x1 == g.gw - 1 && r.y1 == g.gh - 1;
  int64_t R = INT64_MAX;
  if (r.x0 > 0) R = R < P.x - r.x0 * kStarCell ? R : P.x - r.x0 * kStarCell;
  if (r.y0 > 0) R = R < P.y - r.y0 * kStarCell ? R : P.y - r.y0 * kStarCell;
  if (r.x1 < g.gw - 1) R = R < (r.x1 + 1) * kStarCell - P.x ? R : (r.x1 + 1) * kStarCell - P.x;
  if (r.y1 < g.gh - 1) R = R < (r.y1 + 1) * kStarCell - P.y ? R : (r.y1 + 1) * kStarCell - P.y;
  r.R2 = r.full ? INT64_MAX : R * R;
  return r;
}

// Candidate order of the walk. For C strictly left of x -> y, the circle through (x, y, C)
// has its centre at m + t * perp, with m the midpoint of xy and perp = (-(y-x).y, (y-x).x);
// t(C) = num / den with num = |2C - x - y|^2 - |y - x|^2 (|num| < 2^29) and
// den = 4 (2C - x - y) . perp (0 < den < 2^30), exact in 32-bit integers. The circles
// through x and y cut nested caps out of the left half-plane, the cap growing with t, so C
// beats B (C lies inside the circle through (x, y, B)) exactly when t(C) < t(B), and under
// the perturbation when the two are cocircular.
struct CapKey {
  int32_t num, den;
};
__host__ __device__ inline CapKey cap_key(P2 X, P2 Y, P2 C) {
  const int32_t c2x = 2 * C.x - X.x - Y.x, c2y = 2 * C.y - X.y - Y.y;
  const int32_t ex = Y.x - X.x, ey = Y.y - X.y;
  return CapKey{c2x * c2x + c2y * c2y - (ex * ex + ey * ey), 4 * (ex * c2y - ey * c2x)};
}
// The quotient in single precision, for the scans: num and den rounded to float (2^-24
// relative each), the reciprocal of den (1 ulp on the device, correctly rounded on the
// host) and the product (2^-24): within 5 * 2^-24 of t, relative. Two quotients whose
// single-precision values differ by more than 2^-20 of the larger are thus ordered like the
// exact values; closer ones are compared exactly (beats).
__host__ __device__ inline float cap_tf(P2 X, P2 Y, P2 C) {
  const CapKey k = cap_key(X, Y, C);
#ifdef __HIP_DEVICE_COMPILE__
  return (float)k.num * __builtin_amdgcn_rcpf((float)k.den);
#else
  return (float)k.num * (1.0f / (float)k.den);
#endif
}
// t in double from the exact key (for the disk of a triangle, once per step)
__host__ __device__ inline double cap_t(const CapKey& k) { return (double)k.num / (double)k.den; }
// Does candidate c (single-precision quotient tc) beat the current best b (tb)? b < 0: any
// candidate does. Exact: the float filter decides clear cases, the cross-multiplied keys
// (below 2^59 in 64-bit integers) close ones, the perturbed in-circle test exact ties.
__host__ __device__ inline bool beats(P2 X, P2 Y, int32_t b, P2 B, float tb, int32_t c, P2 C, float tc) {
  if (c < 0) return false;
  if (b < 0) return true;
  const float tol = 0x1p-20f * (fabsf(tb) > fabsf(tc) ? fabsf(tb) : fabsf(tc));
  if (tc < tb - tol) return true;
  if (tc > tb + tol) return false;
  const CapKey kb = cap_key(X, Y, B), kc = cap_key(X, Y, C);
  const int64_t l = (int64_t)kc.num * kb.den, r = (int64_t)kb.num * kc.den;
  if (l != r) return l < r;
  return incircle_sos(X, Y, B, C) > 0;
}

// The best row extreme strictly left of x -> y (ids ix, iy excluded), or -1 when no point
// of the frame lies strictly left of it (then the edge is on the convex hull). Exact: in
// each pixel row the points lie between the row's smallest and largest u, and the open
// half-plane meets a row in an open half-line (or the whole row), so it holds a point of
// the row iff it holds one of those two points.
template <class WV>
__host__ __device__ inline int32_t best_extreme(WV& wv, const Grid& g, int32_t ix, P2 X, int32_t iy, P2 Y,
                                                P2* out) {
  constexpr int kRowsPerLane = 8;  // rows a lane reads at once
  int32_t b = -1;
  P2 B{0, 0};
  float tb = 0.0f;
  for (int32_t v0 = 0; v0 < g.H; v0 += WV::kN * kRowsPerLane) {
    int32_t lo[kRowsPerLane], hi[kRowsPerLane], ilo[kRowsPerLane], ihi[kRowsPerLane];
#pragma unroll
    for (int k = 0; k < kRowsPerLane; ++k) {
      const int32_t v = v0 + k * WV::kN + wv.lane();
      const bool in = v < g.H;
      const RowExt e = in ? g.rows[v] : RowExt{1, 0, -1, -1};
      lo[k] = e.lo, hi[k] = e.hi, ilo[k] = e.lo_id, ihi[k] = e.hi_id;
    }
#pragma unroll
    for (int k = 0; k < kRowsPerLane; ++k) {
      if (lo[k] > hi[k]) continue;  // an empty row
      const int32_t v = v0 + k * WV::kN + wv.lane();
      for (int e = 0; e < 2; ++e) {
        const int32_t id = e ? ihi[k] : ilo[k];
        const P2 C{e ? hi[k] : lo[k], v};
        if (id == ix || id == iy || orient(X, Y, C) <= 0) continue;
        const float tc = cap_tf(X, Y, C);
        if (beats(X, Y, b, B, tb, id, C, tc)) b = id, B = C, tb = tc;
      }
    }
  }
  wv.reduce_best(X, Y, &b, &B, &tb);
  *out = B;
  return b;
}

// A run of cells of one cell row, [x0, x1] of row cy (x0 > x1: none): its entries are
// contiguous in cell_e. Scans visit a list of such runs through the group's
// wv.for_rows(g, n, row, fn), calling fn(id, P) for this lane's share of their points
// (row(i) gives run i; a group may set the runs up in parallel).
struct CellRow {
  int32_t cy, x0, x1;
};
// The runs of square r, one per cell row.
struct RegionRows {
  Region r;
  __host__ __device__ CellRow operator()(int32_t i) const { return CellRow{r.y0 + i, r.x0, r.x1}; }
};

// Cells [*c0, *c1] of cell row cy that can hold a point strictly left of x -> y (a superset:
// the half-plane's bound over the band's rows, widened by a pixel).
__host__ __device__ inline void left_cells(const Grid& g, P2 X, P2 Y, int32_t cy, int32_t* c0, int32_t* c1) {
  const int32_t dx = Y.x - X.x, dy = Y.y - X.y;
  const int32_t v0 = cy * kStarCell, v1 = v0 + kStarCell - 1;
  *c0 = 0;
  *c1 = g.gw - 1;
  if (dy == 0) {  // left is the rows below (dx > 0) or above (dx < 0) the line
    if ((dx > 0 && v1 <= X.y) || (dx < 0 && v0 >= X.y)) *c1 = -1;
    return;
  }
  // on row v the left side is u < bound (dy > 0) or u > bound (dy < 0), bound linear in v
  const double b0 = X.x + (double)dx * (v0 - X.y) / dy, b1 = X.x + (double)dx * (v1 - X.y) / dy;
  if (dy > 0) {
    const double hi = (b0 > b1 ? b0 : b1) + 1.0;
    if (hi < 0.0) *c1 = -1;
    else if (hi < (double)g.gw * kStarCell) *c1 = (int32_t)(hi / kStarCell);
  } else {
    const double lo = (b0 < b1 ? b0 : b1) - 1.0;
    if (lo >= (double)g.gw * kStarCell) *c1 = -1;
    else if (lo > 0.0) *c0 = (int32_t)(lo / kStarCell);
  }
}

// Nearest neighbour of p among the candidates: key (d^2 << 32) | id, ~0 when none, and its
// packed coordinates in *wq; a candidate at distance 0 is reported through *dup.
template <class WV>
__host__ __device__ inline uint64_t nearest(WV& wv, const Grid& g, const Region& r, int32_t p, P2 P, bool* dup,
                                            int32_t* wq) {
  uint64_t best = ~0ull;
  int32_t best_uv = 0;
  bool z = false;
  wv.for_candidates(g, r, [&](int32_t id, P2 C) {
    if (id == p) return;
    const int32_t dx = C.x - P.x, dy = C.y - P.y;
    const uint64_t d2 = (uint64_t)(dx * dx + dy * dy);
    z = z || d2 == 0;
    const uint64_t key = (d2 << 32) | (uint32_t)id;
    if (key < best) best = key, best_uv = C.x | (C.y << 16);
  });
  *dup = wv.any(z);
  const uint64_t m = wv.min_u64(best);
  *wq = wv.pick(best == m, best_uv);
  return m;
}

// The best candidate of square r strictly left of x -> y (ids ix, iy excluded), or -1.
template <class WV>
__host__ __device__ inline int32_t best_left(WV& wv, const Grid& g, const Region& r, int32_t ix, P2 X,
                                             int32_t iy, P2 Y, P2* out) {
  int32_t b = -1;
  P2 B{0, 0};
  float tb = 0.0f;
  auto fn = [&](int32_t id, P2 C) {
    if (id == ix || id == iy || orient(X, Y, C) <= 0) return;
    const float tc = cap_tf(X, Y, C);
    if (beats(X, Y, b, B, tb, id, C, tc)) b = id, B = C, tb = tc;
  };
  wv.for_candidates(g, r, fn);  // the walk's square (possibly staged)
  wv.reduce_best(X, Y, &b, &B, &tb);
  *out = B;
  return b;
}

// Circle through x, y and the point of quotient t: centre m + t * perp, radius
// |centre - x|, in double (relative errors near 1e-16, far inside the margin the scan adds).
struct Disk {
  double cx, cy, r;
};
__host__ __device__ inline Disk disk_of(P2 X, P2 Y, double t) {
  const double cx = 0.5 * (X.x + Y.x) - t * (Y.y - X.y), cy = 0.5 * (X.y + Y.y) + t * (Y.x - X.x);
  const double dx = cx - X.x, dy = cy - X.y;
  return Disk{cx, cy, sqrt(dx * dx + dy * dy)};
}

// The best of b (coordinates *B) and the points strictly left of x -> y (ids ix, iy
// excluded) in n cell runs (rows(i) gives run i).
template <class WV, class RowFn>
__host__ __device__ inline int32_t scan_best(WV& wv, const Grid& g, int32_t n, RowFn&& rows, int32_t ix, P2 X,
                                             int32_t iy, P2 Y, int32_t b, P2* B) {
  int32_t best = b;
  P2 Bb = *B;
  float tbest = b >= 0 ? cap_tf(X, Y, *B) : 0.0f;
  if (n > 0)
    wv.for_rows(g, n, rows, [&](int32_t id, P2 C) {
      if (id == ix || id == iy || orient(X, Y, C) <= 0) return;
      const float tc = cap_tf(X, Y, C);
      if (beats(X, Y, best, Bb, tbest, id, C, tc)) best = id, Bb = C, tbest = tc;
    });
  wv.reduce_best(X, Y, &best, &Bb, &tbest);
  *B = Bb;
  return best;
}

// The part of the closed disk through (x, y, b) left of x -> y -- the circular segment cut
// off by the chord xy, where every point that beats b lies: the disk and the segment's
// bounding box, both widened by the margin m. The box holds x, y and those of the circle's
// four axis extremes that lie on the arc left of the edge (kept when within m of the line
// too).
struct Cap {
  Disk D;
  double m, x0, x1, y0, y1;
};
__host__ __device__ inline Cap cap_of(P2 X, P2 Y, P2 B) {
  Cap c;
  c.D = disk_of(X, Y, cap_t(cap_key(X, Y, B)));
  const Disk& D = c.D;
  c.m = kDiskMargin + 1e-9 * D.r;
  c.x0 = X.x < Y.x ? X.x : Y.x, c.x1 = X.x < Y.x ? Y.x : X.x;
  c.y0 = X.y < Y.y ? X.y : Y.y, c.y1 = X.y < Y.y ? Y.y : X.y;
  const double ex = Y.x - X.x, ey = Y.y - X.y, el = sqrt(ex * ex + ey * ey);
  const double px[4] = {D.cx + D.r, D.cx - D.r, D.cx, D.cx};
  const double py[4] = {D.cy, D.cy, D.cy + D.r, D.cy - D.r};
  for (int k = 0; k < 4; ++k)
    if (ex * (py[k] - X.y) - ey * (px[k] - X.x) > -c.m * el) {  // signed distance left of the line > -m
      c.x0 = px[k] < c.x0 ? px[k] : c.x0;
      c.x1 = px[k] > c.x1 ? px[k] : c.x1;
      c.y0 = py[k] < c.y0 ? py[k] : c.y0;
      c.y1 = py[k] > c.y1 ? py[k] : c.y1;
    }
  c.x0 -= c.m, c.x1 += c.m, c.y0 -= c.m, c.y1 += c.m;
  return c;
}
// A quick sufficient test in single precision: the whole disk through (x, y, b), widened by
// a margin far above the rounding of its centre and radius (relative errors of a few 2^-24
// of the quotient, the coordinates and the radius), lies inside square r.
__host__ __device__ inline bool disk_inside_f(P2 X, P2 Y, P2 B, const Grid& g, const Region& r) {
  if (r.full) return true;
  const CapKey k = cap_key(X, Y, B);
  const float t = (float)k.num / (float)k.den;
  const float ex = (float)(Y.x - X.x), ey = (float)(Y.y - X.y);
  const float cx = 0.5f * (float)(X.x + Y.x) - t * ey, cy = 0.5f * (float)(X.y + Y.y) + t * ex;
  const float dx = cx - (float)X.x, dy = cy - (float)X.y;
  const float rad = sqrtf(dx * dx + dy * dy);
  const float m = kDiskMargin + 1e-4f * (rad + fabsf(cx) + fabsf(cy));
  return (cx - rad - m >= (float)(r.x0 * kStarCell) || r.x0 == 0) &&
         (cx + rad + m < (float)((r.x1 + 1) * kStarCell) || r.x1 == g.gw - 1) &&
         (cy - rad - m >= (float)(r.y0 * kStarCell) || r.y0 == 0) &&
         (cy + rad + m < (float)((r.y1 + 1) * kStarCell) || r.y1 == g.gh - 1);
}
// Cells of the frame that the cap's box covers.
__host__ __device__ inline int64_t cap_cells(const Cap& c, const Grid& g) {
  const double w = (c.x1 < g.W ? c.x1 : g.W) - (c.x0 > 0.0 ? c.x0 : 0.0);
  const double h = (c.y1 < g.H ? c.y1 : g.H) - (c.y0 > 0.0 ? c.y0 : 0.0);
  if (w <= 0.0 || h <= 0.0) return 0;
  return (int64_t)(w / kStarCell + 2.0) * (int64_t)(h / kStarCell + 2.0);
}
// Does the cap lie inside square r (then no point outside r can beat b)?
__host__ __device__ inline bool cap_inside(const Cap& c, const Grid& g, const Region& r) {
  if (r.full) return true;
  return (c.x0 >= (double)r.x0 * kStarCell || r.x0 == 0) && (c.x1 < (double)(r.x1 + 1) * kStarCell || r.x1 == g.gw - 1) &&
         (c.y0 >= (double)r.y0 * kStarCell || r.y0 == 0) && (c.y1 < (double)(r.y1 + 1) * kStarCell || r.y1 == g.gh - 1);
}

// The best point strictly left of x -> y given b, the best of square r: every cell outside
// r that b's cap can reach (the disk's chord over each band of rows, within the cap's box,
// and the cells that can hold a point left of the edge) is scanned too. The best over both
// sets is final, since a point beating it would lie inside its own cap, which is nested
// inside b's.
template <class WV>
__host__ __device__ inline int32_t verify_left(WV& wv, const Grid& g, const Region& r, int32_t ix, P2 X, int32_t iy,
                                               P2 Y, int32_t b, P2* B, const Cap& c) {
  const Disk& D = c.D;
  const double m = c.m;
  const double lim_y = (double)g.gh * kStarCell, lim_x = (double)g.gw * kStarCell;
  const int32_t cy0 = c.y0 <= 0.0 ? 0 : (c.y0 >= lim_y ? g.gh : (int32_t)(c.y0 / kStarCell));
  const int32_t cy1 = c.y1 < 0.0 ? -1 : (c.y1 >= lim_y ? g.gh - 1 : (int32_t)(c.y1 / kStarCell));
  // two runs per band of cells: the band's cells the cap reaches, left and right of the
  // square where the band crosses it (the whole reach as the first run otherwise)
  auto row = [&](int32_t i) -> CellRow {
    const int32_t cy = cy0 + i / 2, seg = i % 2;
    const CellRow none{cy, 1, 0};
    // the disk's extent over this band of rows: its chord at the band's row nearest the centre
    const double y0 = (double)cy * kStarCell, y1 = y0 + kStarCell;
    const double dy = D.cy < y0 ? y0 - D.cy : (D.cy > y1 ? D.cy - y1 : 0.0);
    const double h2 = D.r * D.r - dy * dy;
    if (h2 < -2.0 * m * D.r - m * m) return none;  // (the margin keeps grazing bands)
    const double hw = (h2 > 0.0 ? sqrt(h2) : 0.0) + m;
    const double bx0 = D.cx - hw > c.x0 ? D.cx - hw : c.x0, bx1 = D.cx + hw < c.x1 ? D.cx + hw : c.x1;
    if (bx0 > bx1 || bx1 < 0.0 || bx0 >= lim_x) return none;
    int32_t x0 = bx0 <= 0.0 ? 0 : (int32_t)(bx0 / kStarCell);
    int32_t x1 = bx1 >= lim_x ? g.gw - 1 : (int32_t)(bx1 / kStarCell);
    int32_t c0, c1;  // only the cells that can hold a point left of the edge
    left_cells(g, X, Y, cy, &c0, &c1);
    x0 = x0 > c0 ? x0 : c0;
    x1 = x1 < c1 ? x1 : c1;
    if (x0 > x1) return none;
    if (cy < r.y0 || cy > r.y1) return seg == 0 ? CellRow{cy, x0, x1} : none;
    return seg == 0 ? CellRow{cy, x0, x1 < r.x0 - 1 ? x1 : r.x0 - 1}
                    : CellRow{cy, x0 > r.x1 + 1 ? x0 : r.x1 + 1, x1};
  };
  return scan_best(wv, g, cy1 >= cy0 ? 2 * (cy1 - cy0 + 1) : 0, row, ix, X, iy, Y, b, B);
}

// The cells of square t outside square s (s inside t) that can hold a point left of x -> y,
// two runs per cell row of t.
struct LeftRing {
  const Grid* g;
  Region t, s;
  P2 X, Y;
  __host__ __device__ CellRow operator()(int32_t i) const {
    const int32_t cy = t.y0 + i / 2, seg = i % 2;
    int32_t x0, x1;
    if (cy < s.y0 || cy > s.y1) {
      if (seg) return CellRow{cy, 1, 0};
      x0 = t.x0, x1 = t.x1;
    } else {
      x0 = seg ? s.x1 + 1 : t.x0;
      x1 = seg ? t.x1 : s.x0 - 1;
    }
    int32_t c0, c1;
    left_cells(*g, X, Y, cy, &c0, &c1);
    return CellRow{cy, x0 > c0 ? x0 : c0, x1 < c1 ? x1 : c1};
  }
};

// The third vertex of the triangle left of x -> y, exactly (-1: none, the edge is on the
// hull). Its first candidate is the best of square r or, when r holds none, the best of the
// square around the edge's end other than p or, when that holds none either, the best row
// extreme (on the long triangles of hull vertices it is usually the vertex itself); any
// point left of the edge serves, the checks below find the best. Then,
// with s the square whose points have all been seen (r at first): a cap inside s is final;
// a cap whose box covers no more cells than the square t of twice s's reach (or than
// kBandCells) is checked by its bands outside s (verify_left); a larger one (a poor
// candidate) first takes the best of t's ring around s, which can only shrink it, and the
// check repeats with t as s. *far is set when the answer needed points outside r (a row
// extreme, or cells around r).
constexpr int64_t kBandCells = 512;
template <class WV>
__host__ __device__ inline int32_t next_vertex(WV& wv, const Grid& g, const Region& r, P2 P, int32_t ix, P2 X,
                                               int32_t iy, P2 Y, P2* out, bool* far) {
  *far = false;
  int32_t b = best_left(wv, g, r, ix, X, iy, Y, out);
  if (b < 0) {
    if (r.full) return -1;
    *far = true;
    // the square around the edge's other end first (the long edges of a fan: the vertex
    // is usually next to that end), then the row extremes
    const P2 F = X.x == P.x && X.y == P.y ? Y : X;
    b = best_left(wv, g, region_of(g, F, 1), ix, X, iy, Y, out);
    if (b < 0) b = best_extreme(wv, g, ix, X, iy, Y, out);
    if (b < 0) return -1;  // nothing left of the edge: a hull edge
  }
  if (disk_inside_f(X, Y, *out, g, r)) return b;  // the common case, in single precision
  for (Region s = r;;) {
    const Cap c = cap_of(X, Y, *out);
    if (cap_inside(c, g, s)) return b;
    *far = true;
    const Region t = region_of(g, P, 2 * s.k);
    const int64_t t_cells = (int64_t)(t.x1 - t.x0 + 1) * (t.y1 - t.y0 + 1);
    if (cap_cells(c, g) <= (t_cells > kBandCells ? t_cells : kBandCells))
      return verify_left(wv, g, s, ix, X, iy, Y, b, out, c);
    b = scan_best(wv, g, 2 * (t.y1 - t.y0 + 1), LeftRing{&g, t, s, X, Y}, ix, X, iy, Y, b, out);
    s = t;
  }
}

// Cells around p's cell up to which the walk's square grows: a step that needed points
// outside the square (a vertex across a hole, or a hull fan) doubles it for the steps after
// it, whose vertices are then usually inside (any square gives the same triangles).
// (measured at 640x480: 2, 4 and 8 cut the slowest stars, 4 the most for a wavefront; a
// 16-lane group, whose staging holds half as many candidates, does best with 2)
template <class WV>
__host__ __device__ constexpr int32_t walk_max_k() {
  return WV::kN >= 64 ? 4 : 2;
}

// Triangles of p's star in which p has the smallest raster position, as (p, i1, i2)
// counter-clockwise, handed to out.emit(i1, i2) (uniform calls; out.finish() writes what
// is left). Returns the number of triangles, or -(error code).
template <class WV, class Out>
__host__ __device__ inline int32_t star_of(WV& wv, const Grid& g, int32_t p, Out& out) {
  if (p < 0 || p >= g.n) return -kStarErrIndex;
  const int32_t wp = g.uv[p];
  const P2 P = unpack(wp);
  // the nearest neighbour, from a square that holds every point nearer than it
  Region r;
  uint64_t key = ~0ull;
  int32_t wq = 0;
  for (int32_t k = 1;; k *= 2) {
    r = region_of(g, P, k);
    wv.set_base(g, r);  // the square of the walk, once it holds the nearest neighbour (a
                        // group may stage its points)
    bool dup = false;
    key = nearest(wv, g, r, p, P, &dup, &wq);
    if (dup) return -kStarErrDup;
    if (key == ~0ull && r.full) return 0;  // a lone point
    if (key != ~0ull && (r.full || (int64_t)(key >> 32) < r.R2)) break;
  }
  const int32_t q = (int32_t)(key & 0xffffffffu);
  const P2 Q = unpack(wq);
  out.begin();
  auto emit = [&](int32_t i1, P2 A, int32_t i2, P2 B) {
    if ((uint32_t)wp < (uint32_t)(A.x | (A.y << 16)) && (uint32_t)wp < (uint32_t)(B.x | (B.y << 16)))
      out.emit(i1, i2);  // p is the triangle's i0
  };
  // The triangles p writes are those whose two other vertices come after p in raster
  // order; those vertices lie in a half-plane through p (the rows below p's and its row right
  // of it), so they are one contiguous run of p's neighbours in angular order. The walk goes
  // around p from q one way (counter-clockwise: the triangle of each step lies left of
  // p -> a; clockwise: left of a -> p), then, when needed, from q the other way: it stops
  // at a hull edge, and once past the run's end (for good when q is outside the run: the
  // whole run has been passed). With q outside the run the first way is the one that meets
  // the run's nearer end (the run starts at p's row: counter-clockwise from q's side right
  // of p, clockwise from its left).
  auto later = [&](P2 C) { return (uint32_t)wp < (uint32_t)(C.x | (C.y << 16)); };
  const bool q_in = later(Q);
  bool ccw = q_in || Q.x >= P.x, second = false, in_run = q_in;
  int32_t a = q;
  P2 A = Q;
  for (int32_t steps = 0;; ++steps) {
    if (steps > kStarMaxSteps) return -kStarErrSteps;
    P2 B;
    const int32_t ix = ccw ? p : a, iy = ccw ? a : p;
    const P2 X = ccw ? P : A, Y = ccw ? A : P;
    bool far = false;
    const int32_t b = next_vertex(wv, g, r, P, ix, X, iy, Y, &B, &far);
    if (far && r.k < walk_max_k<WV>() && !r.full) {
      r = region_of(g, P, 2 * r.k);
      wv.set_base(g, r);
    }
    bool turn;
    if (b < 0) {  // a hull edge: the run ends here when q is outside it and it has been met
      if (second || (in_run && !q_in)) break;
      turn = true;
    } else {
      if (ccw) emit(a, A, b, B);
      else emit(b, B, a, A);
      const bool b_in = later(B);
      turn = in_run && !b_in;  // past the run's end this way
      if (turn && (second || !q_in)) break;
      in_run = b_in;
      a = b;
      A = B;
      if (!turn && a == q) break;  // around: an interior point
    }
    if (turn) {  // from q, the other way
      second = true;
      ccw = !ccw;
      a = q;
      A = Q;
      in_run = q_in;
    }
  }
  return out.finish();
}

}  // namespace star
}  // namespace sm
