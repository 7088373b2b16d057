// Exact predicates of the device triangulation on packed support coordinates (u and v in
// [0, 8191]): orientation in 32-bit integers and the in-circle test under simulation of
// simplicity on the lifted heights -- the rule the host triangulation and the oracle use
// (Sec. III-A, the Delaunay mesh G(S)), which makes the triangulation unique.
#pragma once

#include <cstdint>

namespace sm {
namespace geom {

struct P2 {
  int32_t x, y;
};

__host__ __device__ inline int sgn64(int64_t x) { return (x > 0) - (x < 0); }

// orientation of (a, b, q): > 0 when q lies left of a -> b; exact for coordinates in [0, 8191]
__host__ __device__ inline int32_t orient(P2 a, P2 b, P2 q) {
  return (b.x - a.x) * (q.y - a.y) - (b.y - a.y) * (q.x - a.x);
}

// Sign of the lifted in-circle determinant of counter-clockwise (a, b, c) and d (> 0: d
// strictly inside the circumcircle). A zero determinant takes the sign of the first
// non-vanishing derivative with respect to the perturbed heights, highest priority (the
// smallest raster position (v, u)) first: d/dz_a = +orient(b, c, d), d/dz_b = -orient(a, c, d),
// d/dz_c = +orient(a, b, d), d/dz_d = -orient(a, b, c).
// Floating-point filter of the in-circle determinant: +1 or -1 when the double evaluation
// proves the sign, 0 when the exact evaluation is needed. Error bound for coordinates in
// [0, 8191] (differences below 2^13): the lifted lengths (< 2^27), the products of a
// difference and a length (< 2^40), the 2x2 minors (< 2^41) and the orientation minor
// (< 2^27) are exact integers in double; each of the three final products is below
// 4 * 8191^4 < 2^54 and rounds by at most 1; their first sum is below 2^55 and rounds by
// at most 2, the second below 2^56 and rounds by at most 4. The computed value is thus
// within 9 of the exact determinant, and a threshold of 64 leaves a wide margin.
__host__ __device__ inline int incircle_filter(P2 a, P2 b, P2 c, P2 d) {
  const double fadx = a.x - d.x, fady = a.y - d.y, fbdx = b.x - d.x, fbdy = b.y - d.y;
  const double fcdx = c.x - d.x, fcdy = c.y - d.y;
  const double fal = fadx * fadx + fady * fady, fbl = fbdx * fbdx + fbdy * fbdy;
  const double fcl = fcdx * fcdx + fcdy * fcdy;
  const double fdet = fadx * (fbdy * fcl - fcdy * fbl) - fady * (fbdx * fcl - fcdx * fbl) +
                      fal * (fbdx * fcdy - fcdx * fbdy);
  if (fdet > 64.0) return 1;
  if (fdet < -64.0) return -1;
  return 0;
}

__host__ __device__ inline int incircle_sos(P2 a, P2 b, P2 c, P2 d) {
  if (const int f = incircle_filter(a, b, c, d)) return f;
  const int64_t adx = a.x - d.x, ady = a.y - d.y;
  const int64_t bdx = b.x - d.x, bdy = b.y - d.y;
  const int64_t cdx = c.x - d.x, cdy = c.y - d.y;
  const int64_t al = adx * adx + ady * ady, bl = bdx * bdx + bdy * bdy, cl = cdx * cdx + cdy * cdy;
  const int64_t det = adx * (bdy * cl - cdy * bl) - ady * (bdx * cl - cdx * bl) + al * (bdx * cdy - cdx * bdy);
  if (det != 0) return sgn64(det);
  // the derivatives, each tagged with its point's raster position, sorted by position
  // (a 4-input network on registers); the first non-zero one decides
  struct D {
    int32_t key, cof;
  };
  auto key = [](P2 q) { return (q.y << 16) | q.x; };
  D e0{key(a), orient(b, c, d)}, e1{key(b), -orient(a, c, d)}, e2{key(c), orient(a, b, d)}, e3{key(d), -orient(a, b, c)};
  auto cx = [](D& x, D& y) {
    if (y.key < x.key) {
      const D t = x;
      x = y;
      y = t;
    }
  };
  cx(e0, e1);
  cx(e2, e3);
  cx(e0, e2);
  cx(e1, e3);
  cx(e1, e2);
  const int32_t cof = e0.cof != 0 ? e0.cof : e1.cof != 0 ? e1.cof : e2.cof != 0 ? e2.cof : e3.cof;
  return cof > 0 ? 1 : (cof < 0 ? -1 : 0);
}

}  // namespace geom
}  // namespace sm
