// Sequential driver of the triangulation code for the CPU tests (Sec. III-A, the Delaunay
// mesh G(S)): the host triangulation (csrc/delaunay.cpp), the device star steps
// (csrc/mesh_star.hpp) run by one lane, and the device predicates (csrc/predicates.hpp).
//
// stdin:  W H n_batches mode, then per batch: count, then count lines "u v"
// stdout: per batch: "batch k n_tris status", then n_tris lines "i0 i1 i2" (sorted): the
//         triangulation of every batch's points so far
//   mode 0: the host triangulation, each batch inserted into the mesh of the earlier ones
//   mode 4: per-point stars from scratch (bucket grid, row extents, one star per point, in
//           shuffled point order: any order must give the same triangles); status 0 or the
//           star steps' error code (no triangles are printed then)
// Mode 3 checks the predicates instead: n_batches lines of four points (a, b, c, d); each
// output line holds the in-circle filter's verdict and the perturbed in-circle sign.
#define __host__
#define __device__
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "delaunay.hpp"
#include "mesh_star.hpp"
#include "predicates.hpp"

using namespace sm;
using geom::P2;

namespace {

// One-lane group for the star steps: reductions are the identity.
struct HostWave {
  static constexpr int kN = 1;
  int lane() const { return 0; }
  bool any(bool b) const { return b; }
  uint64_t min_u64(uint64_t x) const { return x; }
  int32_t pick(bool, int32_t v) const { return v; }
  void reduce_best(P2, P2, int32_t*, P2*, float*) const {}
  template <class RowFn, class Fn>
  void for_rows(const star::Grid& g, int32_t n, RowFn&& row, Fn&& fn) const {
    for (int32_t i = 0; i < n; ++i) {
      const star::CellRow c = row(i);
      if (c.x0 > c.x1) continue;
      for (int32_t e = g.cell_start[c.cy * g.gw + c.x0]; e < g.cell_start[c.cy * g.gw + c.x1 + 1]; ++e)
        fn(g.cell_e[e].id, star::unpack(g.cell_e[e].uv));
    }
  }
  template <class Fn>
  void for_candidates(const star::Grid& g, const star::Region& r, Fn&& fn) const {
    for_rows(g, r.y1 - r.y0 + 1, star::RegionRows{r}, fn);
  }
  void set_base(const star::Grid&, const star::Region&) const {}
};
struct HostOut {  // triangles of one point's star, appended to `all` when it is complete
  std::vector<sm_tri>* all;
  int32_t p;
  std::vector<sm_tri> buf;
  void begin() { buf.clear(); }
  void emit(int32_t i1, int32_t i2) { buf.push_back(sm_tri{p, i1, i2}); }
  int32_t finish() {
    all->insert(all->end(), buf.begin(), buf.end());
    return (int32_t)buf.size();
  }
};

int32_t pack_uv(int32_t u, int32_t v) { return u | (v << 16); }

// Delaunay triangles of points uv[0, n) by per-point stars; status 0 or an error code.
int star_mesh(const std::vector<int32_t>& uv, int W, int H, std::mt19937& rng, std::vector<sm_tri>& out) {
  const int32_t n = (int32_t)uv.size();
  const int32_t C = star::kStarCell, gw = (W + C - 1) / C, gh = (H + C - 1) / C;
  std::vector<int32_t> start(gw * gh + 1, 0);
  std::vector<star::CellEntry> ent(n);
  std::vector<star::RowExt> rows(H, star::RowExt{1 << 30, -1, -1, -1});
  for (int32_t i = 0; i < n; ++i) {
    const P2 q = star::unpack(uv[i]);
    ++start[(q.y / C) * gw + q.x / C + 1];
    star::RowExt& r = rows[q.y];
    if (q.x < r.lo) r.lo = q.x, r.lo_id = i;
    if (q.x > r.hi) r.hi = q.x, r.hi_id = i;
  }
  for (int32_t c = 0; c < gw * gh; ++c) start[c + 1] += start[c];
  std::vector<int32_t> cur(start.begin(), start.end() - 1);
  for (int32_t i = n - 1; i >= 0; --i) {  // any order within a cell gives the same result
    const P2 q = star::unpack(uv[i]);
    const int32_t e = cur[(q.y / C) * gw + q.x / C]++;
    ent[e] = star::CellEntry{i, uv[i]};
  }
  star::Grid g{uv.data(), n, W, H, gw, gh, start.data(), ent.data(), rows.data()};
  std::vector<int32_t> order(n);
  for (int32_t p = 0; p < n; ++p) order[p] = p;
  std::shuffle(order.begin(), order.end(), rng);
  for (const int32_t p : order) {
    HostOut o{&out, p, {}};
    const size_t before = out.size();
    HostWave wv;
    const int32_t r = star::star_of(wv, g, p, o);
    if (r < 0) return -r;
    if (out.size() - before != (size_t)r) return 99;
  }
  return 0;
}

void print_batch(int b, std::vector<sm_tri>& out, int status) {
  std::sort(out.begin(), out.end(), [](const sm_tri& x, const sm_tri& y) {
    if (x.i0 != y.i0) return x.i0 < y.i0;
    if (x.i1 != y.i1) return x.i1 < y.i1;
    return x.i2 < y.i2;
  });
  printf("batch %d %zu %d\n", b, status ? (size_t)0 : out.size(), status);
  if (!status)
    for (const sm_tri& t : out) printf("%d %d %d\n", t.i0, t.i1, t.i2);
}

}  // namespace

int main() {
  int W, H, nb, mode;
  if (scanf("%d %d %d %d", &W, &H, &nb, &mode) != 4) return 2;
  if (mode == 3) {
    for (int k = 0; k < nb; ++k) {
      P2 q[4];
      for (auto& p : q)
        if (scanf("%d %d", &p.x, &p.y) != 2) return 2;
      printf("%d %d\n", geom::incircle_filter(q[0], q[1], q[2], q[3]), geom::incircle_sos(q[0], q[1], q[2], q[3]));
    }
    return 0;
  }
  if (mode != 0 && mode != 4) return 2;
  std::vector<int32_t> uv;
  Delaunay dl;
  std::mt19937 rng(12345);
  for (int b = 0; b < nb; ++b) {
    int n;
    if (scanf("%d", &n) != 1) return 2;
    std::vector<int32_t> u(n), v(n), e(n);
    for (int i = 0; i < n; ++i) {
      if (scanf("%d %d", &u[i], &v[i]) != 2) return 2;
      e[i] = (int32_t)uv.size();
      uv.push_back(pack_uv(u[i], v[i]));
    }
    std::vector<sm_tri> out;
    int status = 0;
    if (mode == 0) {
      if (!dl.insert_many(u.data(), v.data(), e.data(), n)) status = 100;
      else dl.emit(out, true);
    } else {
      status = star_mesh(uv, W, H, rng, out);
    }
    print_batch(b, out, status);
  }
  return 0;
}
