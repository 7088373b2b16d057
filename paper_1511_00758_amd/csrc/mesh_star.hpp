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
// against every cell that the disk through (p, a, b) reaches outside the square (band by
// band of cells, from the disk's exact chord widened by a margin): the best over both is the
// triangle's third vertex, since any point that beats it lies in a cap nested inside b's.
// So the triangles are exact whatever the square; its size only decides how much is
// scanned twice. A step with no candidate in the square but some point strictly left of the
// edge -- decided exactly from the smallest and largest u of every pixel row holding a
// point -- widens the square for that step until one is found. The nearest neighbour is
// taken from a square that certainly holds every point nearer than the one found.
// Each triangle is written once, by its vertex with the smallest raster position (v, u),
// as (i0, i1, i2) counter-clockwise -- the canonical form of sm_tri.
//
// The steps are written for a group of kN lanes (a wavefront of 64 on the device, one lane
// on the host), the WV object: lanes share out the points of a square (wv.for_candidates;
// the walk's square, named by wv.set_base, may be staged) or of a list of cell runs
// (wv.for_rows), and combine their best by its reductions (any, min_u64, reduce_best);
// every control decision is uniform across the group.
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
  kStarErrSupport = 24    // a support outside the frame
};

struct Grid {
  const int32_t* uv;          // [n] packed coordinates u | v << 16
  int32_t n;
  int32_t W, H;
  int32_t gw, gh;             // cells across / down
  const int32_t* cell_start;  // [gw * gh + 1] first entry of each cell in cell_pts
  const int32_t* cell_pts;    // [n] point ids ordered by cell (row-major cells)
  const int32_t* cell_uv;     // [n] their packed coordinates, in the same order
  const int32_t* row_min;     // [H] smallest u of a point in row v (> 8191: no point)
  const int32_t* row_max;     // [H] largest u (-1: no point)
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
// t(C) = (|2C - x - y|^2 - |y - x|^2) / (4 (2C - x - y) . perp), numerator and denominator
// exact integers in double (below 2^31), the quotient correctly rounded. The circles through
// x and y cut nested caps out of the left half-plane, the cap growing with t, so C beats
// B (C lies inside the circle through (x, y, B)) exactly when t(C) < t(B), and under the
// perturbation when the two are cocircular. Two quotients that differ by more than 2^-50
// of their size are ordered like the exact values; closer ones are decided by the exact
// perturbed in-circle test.
__host__ __device__ inline double cap_t(P2 X, P2 Y, P2 C) {
  const int64_t c2x = 2 * C.x - X.x - Y.x, c2y = 2 * C.y - X.y - Y.y;
  const int64_t ex = Y.x - X.x, ey = Y.y - X.y;
  const int64_t num = c2x * c2x + c2y * c2y - (ex * ex + ey * ey);
  const int64_t den = 4 * (ex * c2y - ey * c2x);  // > 0 for C strictly left of x -> y
  return (double)num / (double)den;
}
// does candidate c (quotient tc) beat the current best b (tb)? b < 0: any candidate does
__host__ __device__ inline bool beats(P2 X, P2 Y, int32_t b, P2 B, double tb, int32_t c, P2 C, double tc) {
  if (c < 0) return false;
  if (b < 0) return true;
  const double tol = 0x1p-50 * (fabs(tb) > fabs(tc) ? fabs(tb) : fabs(tc));
  if (tc < tb - tol) return true;
  if (tc > tb + tol) return false;
  return incircle_sos(X, Y, B, C) > 0;
}

// Is some point of the frame strictly left of x -> y? Exact: in each pixel row the points
// lie between the row's smallest and largest u, and the open half-plane meets a row in an
// open half-line (or the whole row), so it holds a point of the row iff it holds one of
// those two points.
template <class WV>
__host__ __device__ inline bool any_left(WV& wv, const Grid& g, P2 X, P2 Y) {
  constexpr int kRowsPerLane = 8;  // rows a lane reads at once; stops at the first batch with a hit
  for (int32_t v0 = 0; v0 < g.H; v0 += WV::kN * kRowsPerLane) {
    int32_t lo[kRowsPerLane], hi[kRowsPerLane];
#pragma unroll
    for (int k = 0; k < kRowsPerLane; ++k) {
      const int32_t v = v0 + k * WV::kN + wv.lane();
      lo[k] = v < g.H ? g.row_min[v] : 1;
      hi[k] = v < g.H ? g.row_max[v] : 0;
    }
    bool hit = false;
#pragma unroll
    for (int k = 0; k < kRowsPerLane; ++k) {
      const int32_t v = v0 + k * WV::kN + wv.lane();
      hit = hit || (lo[k] <= hi[k] && (orient(X, Y, P2{lo[k], v}) > 0 || orient(X, Y, P2{hi[k], v}) > 0));
    }
    if (wv.any(hit)) return true;
  }
  return false;
}

// A run of cells of one cell row, [x0, x1] of row cy (x0 > x1: none): its entries are
// contiguous in cell_pts and cell_uv. Scans visit a list of such runs through the group's
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

// The runs of square r restricted to the cells that can hold a point left of x -> y.
struct LeftRows {
  const Grid* g;
  Region r;
  P2 X, Y;
  __host__ __device__ CellRow operator()(int32_t i) const {
    const int32_t cy = r.y0 + i;
    int32_t c0, c1;
    left_cells(*g, X, Y, cy, &c0, &c1);
    return CellRow{cy, c0 > r.x0 ? c0 : r.x0, c1 < r.x1 ? c1 : r.x1};
  }
};

// Nearest neighbour of p among the candidates: key (d^2 << 32) | id, ~0 when none; a
// candidate at distance 0 is reported through *dup.
template <class WV>
__host__ __device__ inline uint64_t nearest(WV& wv, const Grid& g, const Region& r, int32_t p, P2 P, bool* dup) {
  uint64_t best = ~0ull;
  bool z = false;
  wv.for_candidates(g, r, [&](int32_t id, P2 C) {
    if (id == p) return;
    const int64_t dx = C.x - P.x, dy = C.y - P.y;
    const uint64_t d2 = (uint64_t)(dx * dx + dy * dy);
    z = z || d2 == 0;
    const uint64_t key = (d2 << 32) | (uint32_t)id;
    best = key < best ? key : best;
  });
  *dup = wv.any(z);
  return wv.min_u64(best);
}

// The best candidate of square r strictly left of x -> y (ids ix, iy excluded), or -1.
template <class WV>
__host__ __device__ inline int32_t best_left(WV& wv, const Grid& g, const Region& r, bool base, int32_t ix, P2 X,
                                             int32_t iy, P2 Y, P2* out, double* t_out) {
  int32_t b = -1;
  P2 B{0, 0};
  double tb = 0.0;
  auto fn = [&](int32_t id, P2 C) {
    if (id == ix || id == iy || orient(X, Y, C) <= 0) return;
    const double tc = cap_t(X, Y, C);
    if (beats(X, Y, b, B, tb, id, C, tc)) b = id, B = C, tb = tc;
  };
  if (base) wv.for_candidates(g, r, fn);  // the walk's square (possibly staged)
  else wv.for_rows(g, r.y1 - r.y0 + 1, LeftRows{&g, r, X, Y}, fn);  // a wider one, its left part
  wv.reduce_best(X, Y, &b, &B, &tb);
  *out = B;
  *t_out = tb;
  return b;
}

// Circle through x, y and the point of quotient t (cap_t): centre m + t * perp, radius
// |centre - x|, in double (relative errors near 1e-16, far inside the margin the scan adds).
struct Disk {
  double cx, cy, r;
};
__host__ __device__ inline Disk disk_of(P2 X, P2 Y, double t) {
  const double cx = 0.5 * (X.x + Y.x) - t * (Y.y - X.y), cy = 0.5 * (X.y + Y.y) + t * (Y.x - X.x);
  const double dx = cx - X.x, dy = cy - X.y;
  return Disk{cx, cy, sqrt(dx * dx + dy * dy)};
}

// The best point strictly left of x -> y given b, the best of square r: every cell that
// the closed disk through (x, y, b) reaches outside r is scanned too. A point beating b lies
// inside that disk (in the left cap); the best over both sets is final, since a point
// beating it would lie inside its own cap, which is nested inside b's.
template <class WV>
__host__ __device__ inline int32_t verify_left(WV& wv, const Grid& g, const Region& r, int32_t ix, P2 X, int32_t iy,
                                               P2 Y, int32_t b, P2* B, double tb) {
  if (r.full) return b;
  const Disk D = disk_of(X, Y, tb);
  const double m = kDiskMargin + 1e-9 * D.r;
  const double fy0 = D.cy - D.r - m, fy1 = D.cy + D.r + m;
  const double fx0 = D.cx - D.r - m, fx1 = D.cx + D.r + m;
  // inside r, with nothing to scan: the common case
  const double sx0 = (double)r.x0 * kStarCell, sx1 = (double)(r.x1 + 1) * kStarCell;
  const double sy0 = (double)r.y0 * kStarCell, sy1 = (double)(r.y1 + 1) * kStarCell;
  if ((fx0 >= sx0 || r.x0 == 0) && (fx1 < sx1 || r.x1 == g.gw - 1) && (fy0 >= sy0 || r.y0 == 0) &&
      (fy1 < sy1 || r.y1 == g.gh - 1))
    return b;
  const double lim_y = (double)g.gh * kStarCell, lim_x = (double)g.gw * kStarCell;
  const int32_t cy0 = fy0 <= 0.0 ? 0 : (fy0 >= lim_y ? g.gh : (int32_t)(fy0 / kStarCell));
  const int32_t cy1 = fy1 < 0.0 ? -1 : (fy1 >= lim_y ? g.gh - 1 : (int32_t)(fy1 / kStarCell));
  // two runs per band of cells: the band's cells the disk reaches, left and right of the
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
    const double bx0 = D.cx - hw, bx1 = D.cx + hw;
    if (bx1 < 0.0 || bx0 >= lim_x) return none;
    int32_t x0 = bx0 <= 0.0 ? 0 : (int32_t)(bx0 / kStarCell);
    int32_t x1 = bx1 >= lim_x ? g.gw - 1 : (int32_t)(bx1 / kStarCell);
    int32_t c0, c1;  // only the disk's part left of the edge can hold a better vertex
    left_cells(g, X, Y, cy, &c0, &c1);
    x0 = x0 > c0 ? x0 : c0;
    x1 = x1 < c1 ? x1 : c1;
    if (x0 > x1) return none;
    if (cy < r.y0 || cy > r.y1) return seg == 0 ? CellRow{cy, x0, x1} : none;
    return seg == 0 ? CellRow{cy, x0, x1 < r.x0 - 1 ? x1 : r.x0 - 1}
                    : CellRow{cy, x0 > r.x1 + 1 ? x0 : r.x1 + 1, x1};
  };
  int32_t best = b;
  P2 Bb = *B;
  double tbest = tb;
  if (cy1 >= cy0)
    wv.for_rows(g, 2 * (cy1 - cy0 + 1), row, [&](int32_t id, P2 C) {
      if (id == ix || id == iy || orient(X, Y, C) <= 0) return;
      const double tc = cap_t(X, Y, C);
      if (beats(X, Y, best, Bb, tbest, id, C, tc)) best = id, Bb = C, tbest = tc;
    });
  wv.reduce_best(X, Y, &best, &Bb, &tbest);
  *B = Bb;
  return best;
}

// The third vertex of the triangle left of x -> y, exactly (-1: none, the edge is on the
// hull). Tries square r first, then squares doubling around p when r holds no candidate
// but some point lies left of the edge. (One call site per step: the device code stays
// small enough for the instruction cache.)
template <class WV>
__host__ __device__ inline int32_t next_vertex(WV& wv, const Grid& g, const Region& r, P2 P, int32_t ix, P2 X,
                                               int32_t iy, P2 Y, P2* out) {
  Region rr = r;
  for (int32_t k = r.k;; k *= 2) {
    if (k != r.k) rr = region_of(g, P, k);
    double tb = 0.0;
    const int32_t b = best_left(wv, g, rr, k == r.k, ix, X, iy, Y, out, &tb);
    if (b >= 0) return verify_left(wv, g, rr, ix, X, iy, Y, b, out, tb);
    if (rr.full) return -1;
    if (k == r.k && !any_left(wv, g, X, Y)) return -1;
  }
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
  for (int32_t k = 1;; k *= 2) {
    r = region_of(g, P, k);
    bool dup = false;
    key = nearest(wv, g, r, p, P, &dup);
    if (dup) return -kStarErrDup;
    if (key == ~0ull && r.full) return 0;  // a lone point
    if (key != ~0ull && (r.full || (int64_t)(key >> 32) < r.R2)) break;
  }
  const int32_t q = (int32_t)(key & 0xffffffffu);
  const P2 Q = unpack(g.uv[q]);
  wv.set_base(g, r);  // the square of the walk (a group may stage its points)
  out.begin();
  auto emit = [&](int32_t i1, P2 A, int32_t i2, P2 B) {
    if ((uint32_t)wp < (uint32_t)(A.x | (A.y << 16)) && (uint32_t)wp < (uint32_t)(B.x | (B.y << 16)))
      out.emit(i1, i2);  // p is the triangle's i0
  };
  // counter-clockwise from q, then (at a hull edge) clockwise from q to the other hull edge;
  // the triangle of each step lies left of p -> a (counter-clockwise) or of a -> p
  bool ccw = true;
  int32_t a = q;
  P2 A = Q;
  for (int32_t steps = 0;; ++steps) {
    if (steps > kStarMaxSteps) return -kStarErrSteps;
    P2 B;
    const int32_t ix = ccw ? p : a, iy = ccw ? a : p;
    const P2 X = ccw ? P : A, Y = ccw ? A : P;
    const int32_t b = next_vertex(wv, g, r, P, ix, X, iy, Y, &B);
    if (b < 0) {
      if (!ccw) break;  // the second hull edge
      ccw = false;      // the first hull edge: back to q, the other way
      a = q;
      A = Q;
      continue;
    }
    if (ccw) emit(a, A, b, B);
    else emit(b, B, a, A);
    a = b;
    A = B;
    if (ccw && a == q) break;  // around: an interior point
  }
  return out.finish();
}

}  // namespace star
}  // namespace sm
