// Parallel insertion of points into a Delaunay mesh held in flat arrays: the per-item steps
// of the device triangulation (the driver is in mesh.hip).
//
// The mesh has the host triangulation's form: triangle records (v0, v1, v2) counter-
// clockwise, nb[k] = the record across the edge (v[k+1], v[k+2]) opposite v[k], and hull
// edges carried by ghost triangles (y, x, kGhost) for a hull edge x -> y. The points to add
// lie in the closed hull of the mesh (supports found on pixels that the mesh covers).
//
// Insertion runs in rounds of two phases separated by barriers:
//   propose  every pending point finds its live triangle and bids for it (an atomic minimum
//            of a key), a point on an edge also for the triangle across the edge; every
//            triangle on the work list tests its edges with the exact perturbed in-circle
//            predicate (simulation of simplicity on the lifted heights, as on the host) and
//            bids for itself and its neighbour across the first illegal edge;
//   execute  every bid that holds all its triangles is carried out: a point splits its
//            triangle 1 -> 3 or its edge 2 -> 4 (on a hull edge the ghost splits into two
//            ghosts), an illegal edge is flipped; the other bidders retry in the next round
//            and the new solid triangles join the work list with the edges they must test.
// Edges that cannot be illegal are not tested: the spokes of a 1 -> 3 split (the new
// point lies inside the old circumcircle, so each spoke's opposite vertex lies outside the
// circle through the spoke's triangle) and the new diagonal of a flip. An edge's status
// changes only when one of its two triangles is replaced, and every other edge of a new
// triangle is tested, so no illegal edge is missed.
// Keys carry the round number (a newer round bids lower than anything left in vote[]), so
// votes need no clearing; the smallest key of a round holds all its triangles, so every
// round makes progress. Rounds end when no point is pending and no edge is illegal: every
// edge then passes the perturbed empty-circle test, which makes the mesh the unique
// perturbed Delaunay triangulation, the one the host computes for the same points.
//
// Records are never reused: an operation writes new records (at ids above all existing
// ones) and marks the old ones dead, keeping for each old edge the new record that now
// carries it (own) and the list of new records (kids). Links are not patched in the execute
// phase: a link may point at a dead record, and readers follow own[] to the live one
// (resolve), each step to a higher id; pending points follow kids[] the same way
// (locate_live). The propose phase writes resolved links back (both directions). Execute
// phases thus write only records their bid holds and read nothing written in the phase.
// The records of one frame persist from one tessellation to the next.
//
// Coordinates are read packed (u | v << 16, u and v in [0, 8191]), so that orientations
// are exact in 32-bit integers; the in-circle determinant needs 64 bits. Every index read
// from the arrays is range-checked; a broken invariant sets an error code and stops the
// item instead of faulting, and the caller then triangulates on the host.
#pragma once

#include <cstdint>

#include "stereomesh.h"

namespace sm {
namespace mesh {

constexpr int32_t kGhost = -1;
constexpr int32_t kMaxRounds = 4000;  // round numbers fit the 12 key bits (all tessellations of a frame)

enum : int32_t {
  kOk = 0,
  kErrIndex = 1,     // an index outside its array
  kErrOutside = 2,   // a point outside the mesh (in a ghost triangle)
  kErrCapacity = 3,  // more records than the arrays hold
  kErrLink = 4,      // an edge without its twin
  kErrLocate = 5,    // a point in none of the records that replaced its triangle
  kErrRounds = 6,    // insertion did not finish within kMaxRounds
  kErrWalk = 7,      // the initial point location did not end
  kErrList = 8       // a work list overflowed
};

// Point state (pk) besides an edge slot 0..2.
constexpr int32_t kInside = -1;  // bids for a 1 -> 3 split
constexpr int32_t kDup = -2;     // coincides with a mesh vertex: not inserted
constexpr int32_t kDone = -3;    // inserted

struct Mesh {
  const int32_t* uv;    // packed coordinates u | v << 16 per vertex id
  int32_t* tv;          // [cap][3]
  int32_t* tnb;         // [cap][3]
  int32_t* own;         // [cap][3] record carrying old edge k after death (-1: edge removed)
  int32_t* kids;        // [cap][4] records that replaced a dead record (-1 padded)
  int32_t* dead;        // [cap]
  uint64_t* vote;       // [cap]
  int32_t* fk;          // [cap] flip bid: edge slot, -1 none
  int32_t* fs;          // [cap] flip bid: record across the edge
  int32_t* fj;          // [cap] flip bid: slot of the edge in fs
  uint64_t* fkey;       // [cap] flip bid key
  int32_t cap;
  int32_t p0;           // id of the first new point
  int32_t* ploc;        // [n_new] triangle of point p0 + i (possibly dead)
  int32_t* pk;          // [n_new] edge slot, kInside, kDup or kDone
  int32_t* psib;        // [n_new] record across the edge of an edge point
  uint64_t* pkey;       // [n_new]
};

struct P2 {
  int32_t x, y;
};

__host__ __device__ inline int nxt(int k) { return k == 2 ? 0 : k + 1; }
__host__ __device__ inline int prv(int k) { return k == 0 ? 2 : k - 1; }
__host__ __device__ inline int sgn64(int64_t x) { return (x > 0) - (x < 0); }
// Coordinates of vertex p, read through the policy A (LDS or global on the device).
template <class A>
__host__ __device__ inline P2 xy(const Mesh& m, int32_t p) {
  const int32_t w = A::uv(m, p);
  return P2{w & 0xffff, (int32_t)((uint32_t)w >> 16)};
}
__host__ __device__ inline int32_t pack_uv(int32_t u, int32_t v) { return u | (v << 16); }
// x[k] of (x0, x1, x2) by selects (no indexed local array)
template <class T>
__host__ __device__ inline T sel3(int k, T x0, T x1, T x2) { return k == 0 ? x0 : (k == 1 ? x1 : x2); }

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

// Bid of round r: newer rounds bid lower than every older bid left in vote[]; splits (cls 0)
// go before flips (cls 1), which inserts the points in fewer rounds; then the priority,
// then the id, which makes keys unique.
__host__ __device__ inline uint64_t make_key(int32_t round, int32_t cls, uint32_t prio, uint32_t id) {
  return ((uint64_t)(4095 - round) << 52) | ((uint64_t)cls << 51) | ((uint64_t)(prio & 0x7ffffu) << 32) | id;
}

// Slot k of the record (w0, w1, w2) whose edge (w[k+1], w[k+2]) is (x, y), or -1.
__host__ __device__ inline int edge_slot3(int32_t w0, int32_t w1, int32_t w2, int32_t x, int32_t y) {
  return (w1 == x && w2 == y) ? 0 : (w2 == x && w0 == y) ? 1 : (w0 == x && w1 == y) ? 2 : -1;
}
__host__ __device__ inline int edge_slot(const int32_t* v3, int32_t x, int32_t y) {
  return edge_slot3(v3[0], v3[1], v3[2], x, y);
}

__host__ __device__ inline bool rec_ok(int32_t t, int32_t n_rec) { return t >= 0 && t < n_rec; }

// The live record across the edge (x, y) of a live record whose link there is n, or -1 on
// a broken link. Each step of the chain moves to a record created later, so the loop ends
// within n_rec steps.
__host__ __device__ inline int32_t follow(const Mesh& m, int32_t n, int32_t x, int32_t y, int32_t n_rec) {
  while (true) {
    if (!rec_ok(n, n_rec)) return -1;
    if (!m.dead[n]) return n;
    const int j = edge_slot(m.tv + 3 * n, y, x);
    if (j < 0) return -1;
    const int32_t o = m.own[3 * n + j];
    if (o <= n) return -1;
    n = o;
  }
}

__host__ __device__ inline int32_t resolve(const Mesh& m, int32_t t, int k, int32_t n_rec) {
  return follow(m, m.tnb[3 * t + k], m.tv[3 * t + nxt(k)], m.tv[3 * t + prv(k)], n_rec);
}

// True when point q lies in the closed solid record t.
template <class A>
__host__ __device__ inline bool contains(const Mesh& m, int32_t t, P2 q) {
  const int32_t* v = m.tv + 3 * t;
  if (v[2] == kGhost) return false;
  const P2 P = xy<A>(m, v[0]), B = xy<A>(m, v[1]), C = xy<A>(m, v[2]);
  return orient(B, C, q) >= 0 && orient(C, P, q) >= 0 && orient(P, B, q) >= 0;
}

// The live record containing point q, starting from record t (possibly dead), or -1.
template <class A>
__host__ __device__ inline int32_t locate_live(const Mesh& m, int32_t t, P2 q, int32_t n_rec) {
  while (true) {
    if (!rec_ok(t, n_rec)) return -1;
    if (!m.dead[t]) return t;
    int32_t next = -1;
    for (int c = 0; c < 4 && next < 0; ++c) {
      const int32_t k = m.kids[4 * t + c];
      if (k < 0) break;
      if (k > t && rec_ok(k, n_rec) && contains<A>(m, k, q)) next = k;
    }
    t = next;
  }
}

// Visibility walk from live record t to a solid record whose closed interior holds q.
// Returns the record, -1 on an error, -2 when q lies outside the hull. The walk ends in a
// Delaunay mesh; max_steps guards against a broken one.
template <class A>
__host__ __device__ inline int32_t walk(const Mesh& m, int32_t t, P2 q, int32_t n_rec, int32_t max_steps) {
  for (int32_t step = 0; step < max_steps; ++step) {
    if (!rec_ok(t, n_rec)) return -1;
    const int32_t* v = m.tv + 3 * t;
    if (v[2] == kGhost) return -2;
    const P2 P = xy<A>(m, v[0]), B = xy<A>(m, v[1]), C = xy<A>(m, v[2]);
    int k;
    if (orient(B, C, q) < 0) k = 0;
    else if (orient(C, P, q) < 0) k = 1;
    else if (orient(P, B, q) < 0) k = 2;
    else return t;
    t = resolve(m, t, k, n_rec);
  }
  return -1;
}

// Atomics and list appends differ between the device driver and the host emulation; the
// steps below take them from a policy class A with
//   static void vote_min(uint64_t* p, uint64_t v);   atomic minimum
//   static uint64_t vote_get(const uint64_t* p);     read of a value set by vote_min
//   static void vote_set(uint64_t* p, uint64_t v);   store read by later vote_min / vote_get
//   static int32_t push(int32_t* n, int32_t k);      atomic add, returns the old value
//   static void fail(int32_t* err, int32_t code);    records an error
//   static int32_t uv(const Mesh& m, int32_t p);     packed coordinates of vertex p

// propose, pending point p0 + i.
template <class A>
__host__ __device__ inline void propose_point(const Mesh& m, int32_t i, int32_t round, int32_t n_rec, int32_t* err) {
  const P2 q = xy<A>(m, m.p0 + i);
  // the last triangle's state, vertices and links in one go (the common case: still live)
  int32_t t = m.ploc[i];
  if (!rec_ok(t, n_rec)) return A::fail(err, kErrLocate);
  const int32_t dt = m.dead[t];
  int32_t v0 = m.tv[3 * t], v1 = m.tv[3 * t + 1], v2 = m.tv[3 * t + 2];
  int32_t n0 = m.tnb[3 * t], n1 = m.tnb[3 * t + 1], n2 = m.tnb[3 * t + 2];
  if (dt) {
    t = locate_live<A>(m, t, q, n_rec);
    if (t < 0) return A::fail(err, kErrLocate);
    m.ploc[i] = t;
    v0 = m.tv[3 * t], v1 = m.tv[3 * t + 1], v2 = m.tv[3 * t + 2];
    n0 = m.tnb[3 * t], n1 = m.tnb[3 * t + 1], n2 = m.tnb[3 * t + 2];
  }
  const P2 V0 = xy<A>(m, v0), V1 = xy<A>(m, v1), V2 = xy<A>(m, v2);
  const int32_t o0 = orient(V1, V2, q), o1 = orient(V2, V0, q), o2 = orient(V0, V1, q);
  if (o0 < 0 || o1 < 0 || o2 < 0) return A::fail(err, kErrLocate);
  const int zeros = (o0 == 0) + (o1 == 0) + (o2 == 0);
  const int k0 = o0 == 0 ? 0 : (o1 == 0 ? 1 : 2);
  if (zeros >= 2) {  // on a vertex
    m.pk[i] = kDup;
    return;
  }
  // priority: distance to the centroid, so that triangles split near their middle first
  const int64_t cx = (int64_t)V0.x + V1.x + V2.x - 3 * q.x;
  const int64_t cy = (int64_t)V0.y + V1.y + V2.y - 3 * q.y;
  const uint64_t d2 = (uint64_t)(cx * cx + cy * cy);
  const uint32_t prio = d2 >= (1ull << 31) ? 0x7ffffu : (uint32_t)(d2 >> 12);
  const uint64_t key = make_key(round, 0, prio, (uint32_t)i);
  m.pkey[i] = key;
  if (zeros == 0) {
    m.pk[i] = kInside;
    A::vote_min(&m.vote[t], key);
    return;
  }
  const int32_t s = follow(m, sel3(k0, n0, n1, n2), sel3(nxt(k0), v0, v1, v2), sel3(prv(k0), v0, v1, v2), n_rec);
  if (s < 0) return A::fail(err, kErrLink);
  m.pk[i] = k0;
  m.psib[i] = s;
  A::vote_min(&m.vote[t], key);
  A::vote_min(&m.vote[s], key);
}

// Work-list entries: record << 3 | mask of the edge slots still to test.
__host__ __device__ inline int32_t work_entry(int32_t t, int32_t mask) { return (t << 3) | mask; }

template <class A>
__host__ __device__ inline void propose_flip(const Mesh& m, int32_t e, int32_t round, int32_t n_rec, int32_t* err) {
  const int32_t t = e >> 3, mask = e & 7;
  // A round is bound by the latency of dependent loads, so every load is issued as soon
  // as its address is known: the record with its state and links, then the neighbours
  // across all edges to test with their state and vertices; the edges are then tested in
  // slot order, up to the first illegal one.
  const int32_t dt = m.dead[t];
  const int32_t v0 = m.tv[3 * t], v1 = m.tv[3 * t + 1], v2 = m.tv[3 * t + 2];
  const int32_t raw[3] = {m.tnb[3 * t], m.tnb[3 * t + 1], m.tnb[3 * t + 2]};
  m.fk[t] = -1;
  if (dt || v2 == kGhost) return;
  const int32_t ex[3] = {v1, v2, v0}, ey[3] = {v2, v0, v1};  // edge k = (v[k+1], v[k+2])
  // loads without conditions (an index outside the records reads record 0, whose value is
  // then not used), so that they leave back to back
  int32_t dd[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) dd[k] = m.dead[rec_ok(raw[k], n_rec) ? raw[k] : 0];
  int32_t s[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const bool live = rec_ok(raw[k], n_rec) && !dd[k];
    s[k] = !(mask >> k & 1) ? -1 : live ? raw[k] : follow(m, raw[k], ex[k], ey[k], n_rec);
  }
  int32_t w[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int32_t q = s[k] >= 0 ? s[k] : 0;
    w[k][0] = m.tv[3 * q], w[k][1] = m.tv[3 * q + 1], w[k][2] = m.tv[3 * q + 2];
  }
  const P2 V0 = xy<A>(m, v0), V1 = xy<A>(m, v1), V2 = xy<A>(m, v2);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (!(mask >> k & 1)) continue;
    if (s[k] < 0) return A::fail(err, kErrLink);
    const int j = edge_slot3(w[k][0], w[k][1], w[k][2], ey[k], ex[k]);
    if (j < 0) return A::fail(err, kErrLink);
    if (s[k] != raw[k]) m.tnb[3 * t + k] = s[k];
    m.tnb[3 * s[k] + j] = t;
    if (w[k][2] != kGhost && incircle_sos(V0, V1, V2, xy<A>(m, sel3(j, w[k][0], w[k][1], w[k][2]))) > 0) {
      const uint64_t key = make_key(round, 1, 0, (uint32_t)(3 * t + k));
      m.fk[t] = k;
      m.fs[t] = s[k];
      m.fj[t] = j;
      m.fkey[t] = key;
      A::vote_min(&m.vote[t], key);
      A::vote_min(&m.vote[s[k]], key);
      return;
    }
  }
}

// Writes new record id = (a, b, c) with links (n0, n1, n2), alive, unvoted.
template <class A>
__host__ __device__ inline void put(const Mesh& m, int32_t id, int32_t a, int32_t b, int32_t c, int32_t n0, int32_t n1,
                                    int32_t n2) {
  m.tv[3 * id] = a;
  m.tv[3 * id + 1] = b;
  m.tv[3 * id + 2] = c;
  m.tnb[3 * id] = n0;
  m.tnb[3 * id + 1] = n1;
  m.tnb[3 * id + 2] = n2;
  m.dead[id] = 0;
  A::vote_set(&m.vote[id], ~0ull);
}

// Marks record t dead; own0..2 = records now carrying its edges, kids = base .. base+n-1.
__host__ __device__ inline void retire(const Mesh& m, int32_t t, int32_t own0, int32_t own1, int32_t own2, int32_t base,
                                       int n) {
  m.own[3 * t] = own0;
  m.own[3 * t + 1] = own1;
  m.own[3 * t + 2] = own2;
  for (int c = 0; c < 4; ++c) m.kids[4 * t + c] = c < n ? base + c : -1;
  m.dead[t] = 1;
}

// Allocates n records and queues those with edges to test (bits 3c..3c+2 of tests: the
// edge slots of record base + c) for the next round. Returns the first id, or -1.
template <class A>
__host__ __device__ inline int32_t alloc(const Mesh& m, int n, unsigned tests, int32_t* n_rec, int32_t* work,
                                         int32_t* n_work, int32_t work_cap, int32_t* err) {
  const int32_t base = A::push(n_rec, n);
  if (base + n > m.cap) {
    A::fail(err, kErrCapacity);
    return -1;
  }
  int queued = 0;
  for (int c = 0; c < n; ++c) queued += (tests >> (3 * c) & 7u) != 0;
  const int32_t at = A::push(n_work, queued);
  if (at + queued > work_cap) {
    A::fail(err, kErrList);
    return -1;
  }
  int32_t q = at;
  for (int c = 0; c < n; ++c)
    if (tests >> (3 * c) & 7u) work[q++] = work_entry(base + c, (int32_t)(tests >> (3 * c) & 7u));
  return base;
}

// execute, pending point p0 + i: split if its bid holds its triangles, else retry.
template <class A>
__host__ __device__ inline void execute_point(const Mesh& m, int32_t i, int32_t* n_rec, int32_t* pend, int32_t* n_pend,
                                              int32_t pend_cap, int32_t* work, int32_t* n_work, int32_t work_cap,
                                              int32_t* err) {
  // loads issued as soon as their addresses are known: the point's state, then the votes
  // and the records of its triangles
  const int32_t k = m.pk[i];
  const int32_t t = m.ploc[i], s = m.psib[i];
  const uint64_t key = m.pkey[i];
  if (k == kDup || k == kDone) return;
  const bool edge = k != kInside;
  const int32_t sc = edge ? s : t;  // loads without conditions: an interior point reads t twice
  const uint64_t vt = A::vote_get(&m.vote[t]);
  const uint64_t vs = A::vote_get(&m.vote[sc]);
  const int32_t v0 = m.tv[3 * t], v1 = m.tv[3 * t + 1], v2 = m.tv[3 * t + 2];
  const int32_t n0 = m.tnb[3 * t], n1 = m.tnb[3 * t + 1], n2 = m.tnb[3 * t + 2];
  const int32_t w0 = m.tv[3 * sc], w1 = m.tv[3 * sc + 1], w2 = m.tv[3 * sc + 2];
  const int32_t z0 = m.tnb[3 * sc], z1 = m.tnb[3 * sc + 1], z2 = m.tnb[3 * sc + 2];
  if (vt != key || vs != key) {
    const int32_t at = A::push(n_pend, 1);
    if (at >= pend_cap) return A::fail(err, kErrList);
    pend[at] = i;
    return;
  }
  const int32_t p = m.p0 + i;
  if (!edge) {
    // c_i = (v_i, v_i+1, p): its edge opposite p is the old edge opposite v_i-1, the only
    // one to test (slot 2)
    const int32_t b = alloc<A>(m, 3, 0444u, n_rec, work, n_work, work_cap, err);
    if (b < 0) return;
    put<A>(m, b, v0, v1, p, b + 1, b + 2, n2);
    put<A>(m, b + 1, v1, v2, p, b + 2, b, n0);
    put<A>(m, b + 2, v2, v0, p, b, b + 1, n1);
    retire(m, t, b + 1, b + 2, b, b, 3);
  } else {
    // t = (a, b, c) with the edge (b, c) opposite a = slot k; s across it holds (c, b) in
    // slot j opposite d
    const int32_t a = sel3(k, v0, v1, v2), bb = sel3(nxt(k), v0, v1, v2), c = sel3(prv(k), v0, v1, v2);
    const int32_t t_ca = sel3(nxt(k), n0, n1, n2), t_ab = sel3(prv(k), n0, n1, n2);
    const int j = edge_slot3(w0, w1, w2, c, bb);
    if (j < 0) return A::fail(err, kErrLink);
    const int32_t d = sel3(j, w0, w1, w2), s_bd = sel3(nxt(j), z0, z1, z2), s_dc = sel3(prv(j), z0, z1, z2);
    const bool hull = d == kGhost;
    const int32_t r = alloc<A>(m, 4, hull ? 077u : 07777u, n_rec, work, n_work, work_cap, err);
    if (r < 0) return;
    // r = (a, b, p), r+1 = (a, p, c), r+2 = (d, c, p), r+3 = (d, p, b); with d the ghost,
    // r+2 and r+3 are stored rotated so that the ghost sits in slot 2
    put<A>(m, r, a, bb, p, r + 3, r + 1, t_ab);
    put<A>(m, r + 1, a, p, c, r + 2, t_ca, r);
    if (hull) {
      put<A>(m, r + 2, c, p, kGhost, r + 3, s_dc, r + 1);
      put<A>(m, r + 3, p, bb, kGhost, s_bd, r + 2, r);
    } else {
      put<A>(m, r + 2, d, c, p, r + 1, r + 3, s_dc);
      put<A>(m, r + 3, d, p, bb, r, s_bd, r + 2);
    }
    // old edge x of t: opposite a removed, (c, a) -> r + 1, (a, b) -> r; of s: (c, b)
    // removed, (b, d) -> r + 3, (d, c) -> r + 2
    auto own_t = [&](int x) { return x == k ? -1 : (x == nxt(k) ? r + 1 : r); };
    auto own_s = [&](int x) { return x == j ? -1 : (x == nxt(j) ? r + 3 : r + 2); };
    retire(m, t, own_t(0), own_t(1), own_t(2), r, 4);
    retire(m, s, own_s(0), own_s(1), own_s(2), r, 4);
  }
  m.pk[i] = kDone;
}

// execute, work-list record t: flip if its bid holds both records, else retry.
template <class A>
__host__ __device__ inline void execute_flip(const Mesh& m, int32_t e, int32_t* n_rec, int32_t* work_next,
                                             int32_t* n_next, int32_t work_cap, int32_t* err) {
  // loads issued as soon as their addresses are known: the bid with the record, then the
  // votes and the record across the edge
  const int32_t t = e >> 3;
  const int k = m.fk[t];
  const int32_t s = m.fs[t];
  const int j = m.fj[t];
  const uint64_t key = m.fkey[t];
  const uint64_t vt = A::vote_get(&m.vote[t]);
  const int32_t v0 = m.tv[3 * t], v1 = m.tv[3 * t + 1], v2 = m.tv[3 * t + 2];
  const int32_t n0 = m.tnb[3 * t], n1 = m.tnb[3 * t + 1], n2 = m.tnb[3 * t + 2];
  if (k < 0) return;
  const uint64_t vs = A::vote_get(&m.vote[s]);
  const int32_t w0 = m.tv[3 * s], w1 = m.tv[3 * s + 1], w2 = m.tv[3 * s + 2];
  const int32_t z0 = m.tnb[3 * s], z1 = m.tnb[3 * s + 1], z2 = m.tnb[3 * s + 2];
  if (vt != key || vs != key) {
    const int32_t at = A::push(n_next, 1);
    if (at >= work_cap) return A::fail(err, kErrList);
    work_next[at] = e;
    return;
  }
  const int32_t a = sel3(k, v0, v1, v2), b = sel3(nxt(k), v0, v1, v2), c = sel3(prv(k), v0, v1, v2);
  const int32_t d = sel3(j, w0, w1, w2);
  const int32_t s_bd = sel3(nxt(j), z0, z1, z2), s_dc = sel3(prv(j), z0, z1, z2);
  // (a, b, d) and (a, d, c) replace (a, b, c) and (c, b, d); their shared edge (a, d)
  // passes by construction: r tests slots 0 and 2, r + 1 slots 0 and 1
  const int32_t r = alloc<A>(m, 2, 035u, n_rec, work_next, n_next, work_cap, err);
  if (r < 0) return;
  put<A>(m, r, a, b, d, s_bd, r + 1, sel3(prv(k), n0, n1, n2));
  put<A>(m, r + 1, a, d, c, s_dc, sel3(nxt(k), n0, n1, n2), r);
  auto own_t = [&](int x) { return x == k ? -1 : (x == nxt(k) ? r + 1 : r); };
  auto own_s = [&](int x) { return x == j ? -1 : (x == nxt(j) ? r : r + 1); };
  retire(m, t, own_t(0), own_t(1), own_t(2), r, 2);
  retire(m, s, own_s(0), own_s(1), own_s(2), r, 2);
}

// Solid record t as an output triangle: counter-clockwise, first vertex = smallest (v, u).
template <class A>
__host__ __device__ inline sm_tri top_first3(const Mesh& m, int32_t a, int32_t b, int32_t c) {
  const P2 P = xy<A>(m, a), B = xy<A>(m, b), C = xy<A>(m, c);
  const bool b_lt_a = B.y < P.y || (B.y == P.y && B.x < P.x);
  const bool c_lt_a = C.y < P.y || (C.y == P.y && C.x < P.x);
  const bool c_lt_b = C.y < B.y || (C.y == B.y && C.x < B.x);
  if (b_lt_a && !c_lt_b) {
    const int32_t x = a;
    a = b, b = c, c = x;
  } else if (c_lt_a && c_lt_b) {
    const int32_t x = c;
    c = b, b = a, a = x;
  }
  return sm_tri{a, b, c};
}
template <class A>
__host__ __device__ inline sm_tri top_first(const Mesh& m, int32_t t) {
  return top_first3<A>(m, m.tv[3 * t], m.tv[3 * t + 1], m.tv[3 * t + 2]);
}

}  // namespace mesh
}  // namespace sm
