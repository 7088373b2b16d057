// Host Delaunay triangulation of support pixels (see delaunay.hpp).
#include "delaunay.hpp"

#include <algorithm>

namespace sm {

namespace {
inline int sgn(int64_t x) { return (x > 0) - (x < 0); }

// Index of cell (x, y) along a Hilbert curve over a 2^order x 2^order grid of cells.
inline uint32_t hilbert(uint32_t x, uint32_t y, int order) {
  uint32_t d = 0;
  for (uint32_t s = 1u << (order - 1); s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = s - 1 - (x & (s - 1));
        y = s - 1 - (y & (s - 1));
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}
}  // namespace

void Delaunay::reset() {
  pt_.clear();
  ext_.clear();
  vstamp_.clear();
  vfan_.clear();
  tri_.clear();
  alive_.clear();
  free_.clear();
  stamp_.clear();
  pending_.clear();
  gen_ = 0;
  hint_ = -1;
  n_solid_ = 0;
  started_ = false;
}

// Rotates the solid triangle (a, b, c) cyclically (orientation kept) so that its vertex
// with the smallest (y, x) comes first: the triangle is then stored in the orientation
// the output uses, and emitting it needs no search.
void Delaunay::rotate_top(int32_t& a, int32_t& b, int32_t& c) const {
  const Pt A = pt_[a], B = pt_[b], C = pt_[c];
  const bool b_lt_a = B.y < A.y || (B.y == A.y && B.x < A.x);
  const bool c_lt_a = C.y < A.y || (C.y == A.y && C.x < A.x);
  const bool c_lt_b = C.y < B.y || (C.y == B.y && C.x < B.x);
  if (b_lt_a && !c_lt_b) {  // b first
    const int32_t t = a;
    a = b, b = c, c = t;
  } else if (c_lt_a && c_lt_b) {  // c first
    const int32_t t = c;
    c = b, b = a, a = t;
  }
}

int64_t Delaunay::orient(int32_t a, int32_t b, int32_t c) const {
  const Pt A = pt_[a], B = pt_[b], C = pt_[c];
  return int64_t(B.x - A.x) * int64_t(C.y - A.y) - int64_t(B.y - A.y) * int64_t(C.x - A.x);
}

int64_t Delaunay::orient_pt(int32_t a, int32_t b, int64_t x, int64_t y) const {
  const Pt A = pt_[a], B = pt_[b];
  return int64_t(B.x - A.x) * (y - A.y) - int64_t(B.y - A.y) * (x - A.x);
}

// Sign of det[[u, v, u^2+v^2, 1]] over rows a, b, c, d (> 0: d strictly inside the
// circle of counter-clockwise a, b, c). Zero determinants take the sign of the
// derivative with respect to the highest-priority lifted height that does not vanish:
// d/dz_a = +orient(b,c,d), d/dz_b = -orient(a,c,d), d/dz_c = +orient(a,b,d),
// d/dz_d = -orient(a,b,c); priority = smaller (v, u).
int Delaunay::incircle_sos(int32_t a, int32_t b, int32_t c, int32_t d) const {
  const Pt D = pt_[d], A = pt_[a], B = pt_[b], C = pt_[c];
  const int64_t adx = A.x - D.x, ady = A.y - D.y;
  const int64_t bdx = B.x - D.x, bdy = B.y - D.y;
  const int64_t cdx = C.x - D.x, cdy = C.y - D.y;
  const int64_t al = adx * adx + ady * ady;
  const int64_t bl = bdx * bdx + bdy * bdy;
  const int64_t cl = cdx * cdx + cdy * cdy;
  const int64_t det = adx * (bdy * cl - cdy * bl) - ady * (bdx * cl - cdx * bl) + al * (bdx * cdy - cdx * bdy);
  if (det != 0) return sgn(det);
  int32_t ids[4] = {a, b, c, d};
  // order by priority (smaller (v, u) first); insertion sort of 4
  int ord[4] = {0, 1, 2, 3};
  auto key = [&](int k) { return (int64_t(pt_[ids[k]].y) << 16) | int64_t(pt_[ids[k]].x); };
  for (int i = 1; i < 4; ++i)
    for (int j = i; j > 0 && key(ord[j]) < key(ord[j - 1]); --j) std::swap(ord[j], ord[j - 1]);
  for (int k = 0; k < 4; ++k) {
    int64_t cof;
    switch (ord[k]) {
      case 0: cof = orient(b, c, d); break;
      case 1: cof = -orient(a, c, d); break;
      case 2: cof = orient(a, b, d); break;
      default: cof = -orient(a, b, c); break;
    }
    if (cof != 0) return sgn(cof);
  }
  return 0;  // unreachable for a non-degenerate triangle a, b, c
}

bool Delaunay::conflict(int32_t t, int32_t p) const {
  const Tri& T = tri_[t];
  if (T.v[2] != kGhost) return incircle_sos(T.v[0], T.v[1], T.v[2], p) > 0;
  // ghost (y, x, ghost): solid hull edge x -> y with the interior on its left
  const int32_t y = T.v[0], x = T.v[1];
  const int64_t o = orient(x, y, p);
  if (o < 0) return true;
  if (o > 0) return false;
  const int64_t ux = pt_[x].x, uy = pt_[x].y, wx = pt_[y].x, wy = pt_[y].y, qx = pt_[p].x, qy = pt_[p].y;
  const int64_t d1 = (qx - ux) * (wx - ux) + (qy - uy) * (wy - uy);
  const int64_t d2 = (qx - wx) * (ux - wx) + (qy - wy) * (uy - wy);
  return d1 > 0 && d2 > 0;
}

int32_t Delaunay::alloc_tri() {
  int32_t t;
  if (!free_.empty()) {
    t = free_.back();
    free_.pop_back();
    alive_[t] = 1;
  } else {
    t = (int32_t)tri_.size();
    tri_.push_back(Tri{});
    alive_.push_back(1);
    stamp_.push_back(0);
  }
  return t;
}

void Delaunay::free_tri(int32_t t) {
  alive_[t] = 0;
  free_.push_back(t);
}

void Delaunay::start(int32_t a, int32_t b, int32_t c) {
  if (orient(a, b, c) < 0) std::swap(b, c);
  rotate_top(a, b, c);
  const int32_t s = alloc_tri();
  const int32_t g0 = alloc_tri(), g1 = alloc_tri(), g2 = alloc_tri();
  // solid (a, b, c); edges opposite a: b->c, opposite b: c->a, opposite c: a->b
  tri_[s] = Tri{{a, b, c}, {g0, g1, g2}};
  // ghost across b->c is (c, b, G); across c->a is (a, c, G); across a->b is (b, a, G)
  tri_[g0] = Tri{{c, b, kGhost}, {0, 0, s}};
  tri_[g1] = Tri{{a, c, kGhost}, {0, 0, s}};
  tri_[g2] = Tri{{b, a, kGhost}, {0, 0, s}};
  // ghost (y, x, G): nb[0] across x->G, nb[1] across G->y
  // g0 = (c, b): x->G is b->G, shared with the ghost whose edge is G->b: g2 = (b, a)
  tri_[g0].nb[0] = g2;
  tri_[g0].nb[1] = g1;  // G->c shared with c->G of g1 = (a, c)
  tri_[g1].nb[0] = g0;  // c->G shared with G->c of g0
  tri_[g1].nb[1] = g2;  // G->a shared with a->G of g2 = (b, a)
  tri_[g2].nb[0] = g1;  // a->G shared with G->a of g1
  tri_[g2].nb[1] = g0;  // G->b shared with b->G of g0
  n_solid_ = 1;
  hint_ = s;
  started_ = true;
}

int32_t Delaunay::locate(int32_t p, bool* dup) {
  *dup = false;
  int32_t t = hint_;
  if (t < 0 || !alive_[t]) {
    for (t = 0; t < (int32_t)tri_.size() && !alive_[t]; ++t) {
    }
  }
  if (tri_[t].v[2] == kGhost) t = tri_[t].nb[2];
  const int64_t x = pt_[p].x, y = pt_[p].y;
  const size_t limit = 4 * tri_.size() + 64;
  // visibility walk: it cannot cycle in a (perturbed) Delaunay triangulation
  for (size_t step = 0; step < limit; ++step) {
    const Tri& T = tri_[t];
    if (T.v[2] == kGhost) return t;  // entered across a hull edge with p strictly outside
    int next = -1;
    if (orient_pt(T.v[1], T.v[2], x, y) < 0) next = T.nb[0];
    else if (orient_pt(T.v[2], T.v[0], x, y) < 0) next = T.nb[1];
    else if (orient_pt(T.v[0], T.v[1], x, y) < 0) next = T.nb[2];
    if (next < 0) {  // p inside or on the boundary of T
      for (int k = 0; k < 3; ++k)
        if (pt_[T.v[k]].x == x && pt_[T.v[k]].y == y) *dup = true;
      return t;
    }
    t = next;
  }
  // fallback (not expected): scan for any conflicting triangle
  for (int32_t s = 0; s < (int32_t)tri_.size(); ++s) {
    if (!alive_[s]) continue;
    const Tri& T = tri_[s];
    if (T.v[2] != kGhost)
      for (int k = 0; k < 3; ++k)
        if (pt_[T.v[k]].x == x && pt_[T.v[k]].y == y) {
          *dup = true;
          return s;
        }
    if (conflict(s, p)) return s;
  }
  return -1;
}

bool Delaunay::insert_point(int32_t p) {
  bool dup = false;
  const int32_t t0 = locate(p, &dup);
  if (dup || t0 < 0) return false;  // duplicate pixel
  // flood the hole
  if (++gen_ == 0x7fffffffu) {
    std::fill(stamp_.begin(), stamp_.end(), 0u);
    std::fill(vstamp_.begin(), vstamp_.end(), 0u);
    gen_ = 1;
  }
  const uint32_t in_hole = 2 * gen_, outside = 2 * gen_ + 1;
  hole_.clear();
  bnd_.clear();
  stack_.clear();
  stack_.push_back(t0);
  stamp_[t0] = in_hole;
  while (!stack_.empty()) {
    const int32_t t = stack_.back();
    stack_.pop_back();
    hole_.push_back(t);
    for (int i = 0; i < 3; ++i) {
      const int32_t n = tri_[t].nb[i];
      if (stamp_[n] == in_hole) continue;
      bool in = false;
      if (stamp_[n] != outside) {
        in = conflict(n, p);
        stamp_[n] = in ? in_hole : outside;
      }
      if (in) {
        stack_.push_back(n);
      } else {
        bnd_.push_back(Edge{tri_[t].v[(i + 1) % 3], tri_[t].v[(i + 2) % 3], n});
      }
    }
  }
  // fan around p: one triangle per boundary edge a->b; the triangle of edge a->b is
  // remembered at its start vertex a, so its two fan neighbours are found in O(1)
  newt_.clear();
  for (const Edge& e : bnd_) {
    const int32_t t = alloc_tri();
    newt_.push_back(t);
    Tri T;
    // (a, b, p) rotated so a ghost vertex, if any, sits in slot 2
    if (e.b == kGhost) T.v[0] = p, T.v[1] = e.a, T.v[2] = kGhost;
    else if (e.a == kGhost) T.v[0] = e.b, T.v[1] = p, T.v[2] = kGhost;
    else {
      int32_t a = e.a, b = e.b, c = p;
      rotate_top(a, b, c);
      T.v[0] = a, T.v[1] = b, T.v[2] = c;
    }
    T.nb[0] = T.nb[1] = T.nb[2] = -1;
    // across a->b: the outside neighbour
    for (int i = 0; i < 3; ++i)
      if (T.v[(i + 1) % 3] == e.a && T.v[(i + 2) % 3] == e.b) T.nb[i] = e.out;
    tri_[t] = T;
    Tri& O = tri_[e.out];
    for (int i = 0; i < 3; ++i)
      if (O.v[(i + 1) % 3] == e.b && O.v[(i + 2) % 3] == e.a) O.nb[i] = t;
    if (e.a == kGhost) {
      ghost_fan_ = t;
    } else {
      vstamp_[e.a] = gen_;
      vfan_[e.a] = t;
    }
  }
  // link the fan: the triangle of edge a->b meets the triangle of edge b->c across b-p
  for (size_t j = 0; j < bnd_.size(); ++j) {
    const int32_t b = bnd_[j].b;
    const int32_t t1 = newt_[j];
    const int32_t t2 = b == kGhost ? ghost_fan_ : (vstamp_[b] == gen_ ? vfan_[b] : -1);
    if (t2 < 0) continue;  // cannot happen: the hole boundary is a closed cycle
    Tri& A = tri_[t1];
    Tri& B = tri_[t2];
    for (int i = 0; i < 3; ++i)
      if (A.v[(i + 1) % 3] == b && A.v[(i + 2) % 3] == p) A.nb[i] = t2;
    for (int i = 0; i < 3; ++i)
      if (B.v[(i + 1) % 3] == p && B.v[(i + 2) % 3] == b) B.nb[i] = t1;
  }
  int32_t solid_removed = 0, solid_added = 0;
  for (int32_t t : hole_) {
    if (tri_[t].v[2] != kGhost) ++solid_removed;
    free_tri(t);
  }
  for (int32_t t : newt_)
    if (tri_[t].v[2] != kGhost) {
      ++solid_added;
      hint_ = t;
    }
  n_solid_ += solid_added - solid_removed;
  return true;
}

bool Delaunay::insert(int32_t u, int32_t v, int32_t ext) {
  if (u < 0 || v < 0 || u > 8191 || v > 8191) return false;
  const int32_t p = (int32_t)pt_.size();
  pt_.push_back(Pt{u, v});
  ext_.push_back(ext);
  vstamp_.push_back(0);
  vfan_.push_back(-1);
  auto drop_last = [&]() {
    pt_.pop_back();
    ext_.pop_back();
    vstamp_.pop_back();
    vfan_.pop_back();
  };
  if (started_) {
    if (!insert_point(p)) drop_last();  // duplicate: the first occurrence stays
    return true;
  }
  // before the first triangle: keep the points while they are collinear
  for (int32_t q : pending_)
    if (pt_[q].x == u && pt_[q].y == v) {
      drop_last();
      return true;
    }
  if (pending_.size() >= 2 && orient(pending_[0], pending_[1], p) != 0) {
    start(pending_[0], pending_[1], p);
    for (size_t k = 2; k < pending_.size(); ++k) insert_point(pending_[k]);
    pending_.clear();
    return true;
  }
  pending_.push_back(p);
  return true;
}

void Delaunay::order_points(const int32_t* u, const int32_t* v, int32_t n) {
  // Biased randomised insertion order: point i joins round k with probability 2^-(k+1)
  // (k = number of trailing one bits of a xorshift draw, capped at 15); rounds are
  // inserted from the sparsest, each in Hilbert order of 32 px cells. Key = 4 round bits
  // + 16 cell bits, sorted by a stable 3-pass LSD radix sort (input order within a
  // cell), so the order costs O(n).
  constexpr int kCellShift = 5, kOrder = 13 - kCellShift, kCellBits = 2 * kOrder;
  key_.resize(n);
  idx_.resize(n);
  key2_.resize(n);
  idx2_.resize(n);
  uint32_t r = 0x2545f491u;
  for (int32_t i = 0; i < n; ++i) {
    r ^= r << 13;
    r ^= r >> 17;
    r ^= r << 5;
    const uint32_t round = std::min<uint32_t>((uint32_t)__builtin_ctz(~r), 15u);
    const uint32_t cell = hilbert((uint32_t)u[i] >> kCellShift, (uint32_t)v[i] >> kCellShift, kOrder);
    key_[i] = ((15u - round) << kCellBits) | cell;
    idx_[i] = i;
  }
  for (int shift = 0; shift < kCellBits + 4; shift += 8) {
    uint32_t count[257] = {0};
    for (int32_t i = 0; i < n; ++i) ++count[((key_[i] >> shift) & 255u) + 1];
    for (int b = 0; b < 256; ++b) count[b + 1] += count[b];
    for (int32_t i = 0; i < n; ++i) {
      const uint32_t o = count[(key_[i] >> shift) & 255u]++;
      key2_[o] = key_[i];
      idx2_[o] = idx_[i];
    }
    key_.swap(key2_);
    idx_.swap(idx2_);
  }
}

bool Delaunay::insert_many(const int32_t* u, const int32_t* v, const int32_t* ext, int32_t n) {
  for (int32_t i = 0; i < n; ++i)
    if (u[i] < 0 || v[i] < 0 || u[i] > 8191 || v[i] > 8191) return false;
  order_points(u, v, n);
  pt_.reserve(pt_.size() + n);
  ext_.reserve(ext_.size() + n);
  vstamp_.reserve(vstamp_.size() + n);
  vfan_.reserve(vfan_.size() + n);
  for (int32_t k = 0; k < n; ++k) {
    const int32_t i = idx_[k];
    insert(u[i], v[i], ext[i]);
  }
  return true;
}

void Delaunay::emit(std::vector<sm_tri>& out, bool sorted) const {
  const size_t base = out.size();
  for (size_t t = 0; t < tri_.size(); ++t) {
    if (!alive_[t] || tri_[t].v[2] == kGhost) continue;
    const Tri& T = tri_[t];  // stored with its top vertex first
    out.push_back(sm_tri{ext_[T.v[0]], ext_[T.v[1]], ext_[T.v[2]]});
  }
  if (sorted)
    std::sort(out.begin() + base, out.end(), [](const sm_tri& x, const sm_tri& y) {
      if (x.i0 != y.i0) return x.i0 < y.i0;
      if (x.i1 != y.i1) return x.i1 < y.i1;
      return x.i2 < y.i2;
    });
}

}  // namespace sm

namespace sm {

void Delaunay::emit_banded(std::vector<sm_tri>& out, int band_shift) const {
  int32_t max_band = 0;
  for (const Pt& q : pt_) max_band = std::max(max_band, q.y >> band_shift);
  band_count_.assign((size_t)max_band + 2, 0);
  for (size_t t = 0; t < tri_.size(); ++t) {
    if (!alive_[t] || tri_[t].v[2] == kGhost) continue;
    ++band_count_[(pt_[tri_[t].v[0]].y >> band_shift) + 1];  // v[0] is the top vertex
  }
  for (size_t i = 1; i < band_count_.size(); ++i) band_count_[i] += band_count_[i - 1];
  const size_t base = out.size();
  out.resize(base + (size_t)band_count_.back());
  for (size_t t = 0; t < tri_.size(); ++t) {
    if (!alive_[t] || tri_[t].v[2] == kGhost) continue;
    const Tri& T = tri_[t];
    const int32_t slot = band_count_[pt_[T.v[0]].y >> band_shift]++;
    out[base + slot] = sm_tri{ext_[T.v[0]], ext_[T.v[1]], ext_[T.v[2]]};
  }
}

}  // namespace sm
