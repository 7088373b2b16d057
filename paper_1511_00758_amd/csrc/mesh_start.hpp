// A first mesh built on the device from supports sorted by raster position (the grid
// supports after compaction are): a valid triangulation of their convex hull, which the
// Lawson flips of mesh_core.hpp then turn into the perturbed Delaunay triangulation.
//
//   rows     every distinct v is a row; rows are contiguous runs of the sorted supports,
//            increasing u inside a row
//   ladders  between two consecutive rows (two horizontal lines) the points are joined by
//            a ladder: walking both rows left to right, each step adds the triangle of the
//            next point of one row and the current point of the other (always valid
//            between parallel lines); strip r holds |row r| + |row r+1| - 2 triangles. The
//            walk is a merge of the two rows by u, so each point finds its own triangle
//            and its place in the strip by a binary search in the other row
//   pockets  the left ends of the rows (bottom to top) and the right ends (top to bottom)
//            are the side chains of the boundary; a stack scan fills every reflex vertex
//            with a triangle, so the boundary becomes the convex hull (collinear points on
//            it stay vertices, as in the host triangulation); the corners at the first and
//            last rows are always convex
//   links    every directed edge goes into a hash table; an edge whose reverse is absent
//            is a hull edge and gets a ghost triangle; ghosts link to the ghosts of the
//            hull edges before and after them
//
// The per-item steps below are shared by the kernel and the CPU tests; atomics come from
// the same policy class as in mesh_core.hpp, plus
//   static uint64_t cas64(uint64_t* p, uint64_t expected, uint64_t desired);  returns old
#pragma once

#include <cstdint>

#include "mesh_core.hpp"

namespace sm {
namespace mesh {

constexpr uint64_t kEmptyEdge = ~0ull;
constexpr int32_t kErrOrder = 9;  // supports not strictly increasing in (v, u)

struct Start {
  int32_t n;           // supports S[0, n)
  int32_t* row_first;  // [n] first support of row r
  int32_t* row_of;     // [n] row of support i
  int32_t* strip_base; // [n] first record of strip r
  int32_t* gh_start;   // [n] ghost of the hull edge starting at vertex x, -1
  int32_t* gh_end;     // [n] ghost of the hull edge ending at vertex x, -1
  int32_t* stack;      // [2][rows] chain scans (left, right)
  uint64_t* keys;      // [hcap] directed edges (x + 1) << 32 | (y + 1)
  int32_t* vals;       // [hcap] 3 * record + slot
  int32_t hcap;        // power of two
};

__host__ __device__ inline uint64_t raster_key(P2 p) { return ((uint64_t)p.y << 16) | (uint64_t)p.x; }

// rows: true when support i starts a row; flags an order error.
template <class A>
__host__ __device__ inline bool row_starts(const Mesh& m, int32_t i, int32_t* err) {
  if (i == 0) return true;
  const P2 a = xy<A>(m, i - 1), b = xy<A>(m, i);
  if (raster_key(a) >= raster_key(b)) A::fail(err, kErrOrder);
  return a.y != b.y;
}

__host__ __device__ inline int32_t ladder_size(const Start& st, int32_t r, int32_t n_rows) {
  const int32_t a0 = st.row_first[r], a1 = st.row_first[r + 1];
  const int32_t b1 = r + 2 < n_rows ? st.row_first[r + 2] : st.n;
  return (a1 - a0 - 1) + (b1 - a1 - 1);
}

// Number of supports q in [lo, hi) of one row with u(q) < X (u(q) <= X when inclusive);
// u increases along a row.
template <class A>
__host__ __device__ inline int32_t rank_in_row(const Mesh& m, int32_t lo, int32_t hi, int32_t X, bool inclusive) {
  int32_t a = lo, b = hi;
  while (a < b) {
    const int32_t mid = (a + b) >> 1;
    const int32_t xm = xy<A>(m, mid).x;
    if (xm < X || (inclusive && xm == X)) a = mid + 1;
    else b = mid;
  }
  return a - lo;
}

// ladders: support i of row r, unless it starts the row, is the next point of a walk step
// in both strips it borders. In strip r (rows r, r + 1) it adds (i - 1, i, B) with B the
// last point of row r + 1 left of it; in strip r - 1 (rows r - 1, r) it adds (A, i, i - 1)
// with A the last point of row r - 1 at or left of it (on a tie the lower row steps
// first). Its triangle's place in the strip is the number of steps before it: the points
// of both rows that come earlier in the merge by u.
template <class A>
__host__ __device__ inline void ladder_point(const Mesh& m, const Start& st, int32_t i, int32_t n_rows) {
  const int32_t r = st.row_of[i];
  const int32_t a0 = st.row_first[r];
  if (i == a0) return;
  const int32_t a1 = r + 1 < n_rows ? st.row_first[r + 1] : st.n;
  const int32_t X = xy<A>(m, i).x;
  if (r + 1 < n_rows) {  // the lower row of strip r; its upper row is [a1, b1)
    const int32_t b1 = r + 2 < n_rows ? st.row_first[r + 2] : st.n;
    const int32_t rank = rank_in_row<A>(m, a1 + 1, b1, X, false);
    const int32_t t = st.strip_base[r] + (i - a0 - 1) + rank;
    m.tv[3 * t] = i - 1, m.tv[3 * t + 1] = i, m.tv[3 * t + 2] = a1 + rank;
  }
  if (r >= 1) {  // the upper row of strip r - 1; its lower row is [c0, a0)
    const int32_t c0 = st.row_first[r - 1];
    const int32_t rank = rank_in_row<A>(m, c0 + 1, a0, X, true);
    const int32_t t = st.strip_base[r - 1] + rank + (i - a0 - 1);
    m.tv[3 * t] = c0 + rank, m.tv[3 * t + 1] = i, m.tv[3 * t + 2] = i - 1;
  }
}

// pockets: scan of one side chain (side 0: row starts, bottom to top; side 1: row ends,
// top to bottom); each reflex vertex gets the triangle (previous, next, vertex). Records
// come from n_rec. Returns false on a capacity error.
template <class A>
__host__ __device__ inline bool pockets(const Mesh& m, const Start& st, int side, int32_t n_rows, int32_t* n_rec,
                                        int32_t* err) {
  int32_t* stk = st.stack + (side ? n_rows : 0);
  auto chain = [&](int32_t q) {  // q-th point of the side chain
    const int32_t r = side ? q : n_rows - 1 - q;
    return side ? (r + 1 < n_rows ? st.row_first[r + 1] : st.n) - 1 : st.row_first[r];
  };
  // the two top entries of the stack stay in registers with their coordinates; the next
  // chain point and its coordinates are read one step ahead
  int32_t top = 0, s1 = -1, s2 = -1;
  P2 c1{0, 0}, c2{0, 0};
  int32_t p = chain(0);
  P2 cp = xy<A>(m, p);
  for (int32_t q = 0; q < n_rows; ++q) {
    const int32_t p_next = q + 1 < n_rows ? chain(q + 1) : p;
    const P2 c_next = xy<A>(m, p_next);
    while (top >= 2 && orient(c2, c1, cp) < 0) {
      const int32_t t = A::push(n_rec, 1);
      if (t >= m.cap) {
        A::fail(err, kErrCapacity);
        return false;
      }
      m.tv[3 * t] = s2, m.tv[3 * t + 1] = p, m.tv[3 * t + 2] = s1;
      --top;
      s1 = s2, c1 = c2;
      if (top >= 2) s2 = stk[top - 2], c2 = xy<A>(m, s2);
    }
    stk[top++] = p;
    s2 = s1, c2 = c1;
    s1 = p, c1 = cp;
    p = p_next, cp = c_next;
  }
  return true;
}

__host__ __device__ inline uint64_t edge_key(int32_t x, int32_t y) {
  return ((uint64_t)(uint32_t)(x + 1) << 32) | (uint32_t)(y + 1);
}

__host__ __device__ inline uint32_t edge_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  return (uint32_t)k;
}

// links, first pass: the directed edge in slot k of solid record t into the table. The
// compare-and-swap at the first slot h of its probe sequence may be issued by the caller
// (old = the key it found), which lets a thread have several edges in flight.
template <class A>
__host__ __device__ inline void edge_insert_from(const Start& st, uint64_t key, int32_t val, uint32_t h, uint64_t old,
                                                 int32_t* err) {
  for (int32_t probe = 1;; ++probe) {
    if (old == kEmptyEdge) {
      st.vals[h] = val;
      return;
    }
    if (old == key) return A::fail(err, kErrLink);  // an edge twice: not a triangulation
    if (probe == st.hcap) return A::fail(err, kErrCapacity);
    h = (h + 1) & (uint32_t)(st.hcap - 1);
    old = A::cas64(&st.keys[h], kEmptyEdge, key);
  }
}

__host__ __device__ inline uint64_t solid_edge_key(const Mesh& m, int32_t t, int k, bool reverse) {
  const int32_t x = m.tv[3 * t + nxt(k)], y = m.tv[3 * t + prv(k)];
  return reverse ? edge_key(y, x) : edge_key(x, y);
}

template <class A>
__host__ __device__ inline void edge_insert(const Mesh& m, const Start& st, int32_t t, int k, int32_t* err) {
  const uint64_t key = solid_edge_key(m, t, k, false);
  const uint32_t h = edge_hash(key) & (uint32_t)(st.hcap - 1);
  edge_insert_from<A>(st, key, 3 * t + k, h, A::cas64(&st.keys[h], kEmptyEdge, key), err);
}

// links, second pass: the slot holding key, probing from slot h whose key cur the caller
// may have read, or -1 when the key is absent.
template <class A>
__host__ __device__ inline int32_t edge_find_from(const Start& st, uint64_t key, uint32_t h, uint64_t cur) {
  for (int32_t probe = 1;; ++probe) {
    if (cur == key) return (int32_t)h;
    if (cur == kEmptyEdge || probe == st.hcap) return -1;
    h = (h + 1) & (uint32_t)(st.hcap - 1);
    cur = A::vote_get(&st.keys[h]);  // written by atomics
  }
}

// The neighbour across slot k of solid record t: the record of the reverse edge (val, from
// its slot in the table), or a new ghost when the reverse edge is absent (slot < 0; a hull
// edge x -> y gets the ghost (y, x, ghost)).
template <class A>
__host__ __device__ inline void edge_link_to(const Mesh& m, const Start& st, int32_t t, int k, int32_t slot,
                                             int32_t val, int32_t* n_rec, int32_t* err) {
  if (slot >= 0) {
    m.tnb[3 * t + k] = val / 3;
    return;
  }
  const int32_t x = m.tv[3 * t + nxt(k)], y = m.tv[3 * t + prv(k)];
  const int32_t g = A::push(n_rec, 1);
  if (g >= m.cap) return A::fail(err, kErrCapacity);
  m.tv[3 * g] = y, m.tv[3 * g + 1] = x, m.tv[3 * g + 2] = kGhost;
  m.tnb[3 * g + 2] = t;
  m.tnb[3 * t + k] = g;
  if (st.gh_start[x] >= 0 || st.gh_end[y] >= 0) return A::fail(err, kErrLink);  // not a simple hull
  st.gh_start[x] = g;
  st.gh_end[y] = g;
}

template <class A>
__host__ __device__ inline void edge_link(const Mesh& m, const Start& st, int32_t t, int k, int32_t* n_rec,
                                          int32_t* err) {
  const uint64_t key = solid_edge_key(m, t, k, true);
  const uint32_t h = edge_hash(key) & (uint32_t)(st.hcap - 1);
  const int32_t slot = edge_find_from<A>(st, key, h, A::vote_get(&st.keys[h]));
  edge_link_to<A>(m, st, t, k, slot, slot >= 0 ? st.vals[slot] : 0, n_rec, err);
}

// links by pairing (in LDS on the device, where the table fits): every undirected edge
// {a, b} has one slot in a table of tcap entries; the first of its two directed edges
// claims the slot, the second finds it and links both records. Slots nobody paired hold
// the hull edges. An entry packs the key a << 15 | b (plus one, so that 0 is empty), the
// record slot 3 * t + k of the claiming edge, its direction and a paired flag.
constexpr int32_t kPairMaxVertices = 1 << 15;

__host__ __device__ inline uint64_t pair_entry(int32_t x, int32_t y, int32_t val) {
  const int32_t a = x < y ? x : y, b = x < y ? y : x;
  const uint64_t key = (((uint64_t)a << 15) | (uint64_t)b) + 1;
  return (key << 32) | ((uint64_t)(uint32_t)val << 2) | ((uint64_t)(x < y) << 1);
}

// The directed edge x -> y in slot k of solid record t (x and y read by the caller, which
// may hold several edges' vertices in flight).
template <class A>
__host__ __device__ inline void pair_edge(const Mesh& m, uint64_t* tab, int32_t tcap, int32_t t, int k, int32_t x,
                                          int32_t y, int32_t* err) {
  const uint64_t mine = pair_entry(x, y, 3 * t + k);
  uint32_t h = edge_hash(mine >> 32) & (uint32_t)(tcap - 1);
  for (int32_t probe = 0; probe < tcap; ++probe) {
    const uint64_t cur = A::cas64(&tab[h], 0, mine);
    if (cur == 0) return;  // claimed: the reverse edge links both
    if ((cur >> 32) == (mine >> 32)) {
      // a third edge on {a, b}, or two in the same direction: not a triangulation
      if ((cur & 1u) || ((cur ^ mine) & 2u) == 0) return A::fail(err, kErrLink);
      if (A::cas64(&tab[h], cur, cur | 1u) != cur) return A::fail(err, kErrLink);
      const int32_t other = (int32_t)((cur >> 2) & 0x3fffffffu);  // 3 * t' + k'
      m.tnb[3 * t + k] = other / 3;
      m.tnb[other] = t;
      return;
    }
    h = (h + 1) & (uint32_t)(tcap - 1);
  }
  A::fail(err, kErrCapacity);
}

// A slot of the table after pairing: an unpaired edge is a hull edge and gets its ghost.
template <class A>
__host__ __device__ inline void pair_hull(const Mesh& m, const Start& st, uint64_t e, int32_t* n_rec, int32_t* err) {
  if (e == 0 || (e & 1u)) return;
  const int32_t val = (int32_t)((e >> 2) & 0x3fffffffu);
  edge_link_to<A>(m, st, val / 3, val % 3, -1, 0, n_rec, err);
}

// Table size for n_solid triangles over n supports: fewer than (3 n_solid + n) / 2
// undirected edges (each solid triangle has three, each interior edge two solid sides,
// and fewer than n lie on the hull); the load stays below 3/4.
__host__ __device__ inline int32_t pair_table_size(int32_t n_solid, int32_t n) {
  const int64_t edges = (3 * (int64_t)n_solid + n) / 2 + 1;
  int32_t c = 1024;
  while ((int64_t)c * 3 < edges * 4 && c < (1 << 26)) c <<= 1;
  return c;
}

// links, third pass: ghost g = (y, x, ghost) of hull edge x -> y links, across (x, ghost),
// to the ghost of the hull edge ending at x and, across (ghost, y), to the one starting at y.
template <class A>
__host__ __device__ inline void ghost_link(const Mesh& m, const Start& st, int32_t g, int32_t* err) {
  const int32_t y = m.tv[3 * g], x = m.tv[3 * g + 1];
  const int32_t before = st.gh_end[x], after = st.gh_start[y];
  if (before < 0 || after < 0) return A::fail(err, kErrLink);
  m.tnb[3 * g] = before;
  m.tnb[3 * g + 1] = after;
}

}  // namespace mesh
}  // namespace sm
