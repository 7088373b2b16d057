// Sequential driver of the device mesh steps (paper_1511_00758_amd/csrc/mesh_core.hpp,
// mesh_start.hpp) for the CPU tests. The first batch of points is triangulated either by
// the host Delaunay and exported (mode 0) or by the device start steps (rows, ladders,
// pockets, edge links, then Lawson flips; points sorted by (v, u); mode 1 links through
// the edge hash table, mode 2 by pairing in a table of undirected edges); every later
// batch is inserted by the same per-item propose / execute steps the GPU kernel runs, one
// item after another in a shuffled order (the GPU runs them concurrently; any order must
// give the same mesh). Prints the solid triangles, top vertex first, after every batch.
//
// stdin:  W H n_batches mode, then per batch: count, then count lines "u v"
// stdout: per batch: "batch k n_tris status", then n_tris lines "i0 i1 i2" (sorted)
// Mode 3 checks the predicates instead: n_batches lines of four points (a, b, c, d); each
// output line holds the in-circle filter's verdict and the perturbed in-circle sign.
// Mode 4 triangulates every batch's points so far from scratch by per-point stars
// (mesh_star.hpp: bucket grid, row extents, one star per point, one lane).
#define __host__
#define __device__
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "delaunay.hpp"
#include "mesh_core.hpp"
#include "mesh_start.hpp"
#include "mesh_star.hpp"

using namespace sm;
using namespace sm::mesh;

namespace {

struct Seq {
  static void vote_min(uint64_t* p, uint64_t v) { *p = v < *p ? v : *p; }
  static uint64_t vote_get(const uint64_t* p) { return *p; }
  static void vote_set(uint64_t* p, uint64_t v) { *p = v; }
  static int32_t push(int32_t* n, int32_t k) {
    const int32_t o = *n;
    *n += k;
    return o;
  }
  static void fail(int32_t* err, int32_t code) {
    if (!*err) *err = code;
  }
  static int32_t uv(const Mesh& m, int32_t p) { return m.uv[p]; }
  static uint64_t cas64(uint64_t* p, uint64_t expected, uint64_t desired) {
    const uint64_t o = *p;
    if (o == expected) *p = desired;
    return o;
  }
};

// One-lane group for the star steps: reductions are the identity.
struct HostWave {
  static constexpr int kN = 1;
  int lane() const { return 0; }
  bool any(bool b) const { return b; }
  uint64_t min_u64(uint64_t x) const { return x; }
  void reduce_best(P2, P2, int32_t*, P2*, double*) const {}
  template <class RowFn, class Fn>
  void for_rows(const star::Grid& g, int32_t n, RowFn&& row, Fn&& fn) const {
    for (int32_t i = 0; i < n; ++i) {
      const star::CellRow c = row(i);
      if (c.x0 > c.x1) continue;
      for (int32_t e = g.cell_start[c.cy * g.gw + c.x0]; e < g.cell_start[c.cy * g.gw + c.x1 + 1]; ++e)
        fn(g.cell_pts[e], star::unpack(g.cell_uv[e]));
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

// Delaunay triangles of points uv[0, n) by per-point stars; status 0 or an error code.
int star_mesh(const std::vector<int32_t>& uv, int W, int H, std::vector<sm_tri>& out) {
  const int32_t n = (int32_t)uv.size();
  const int32_t C = star::kStarCell, gw = (W + C - 1) / C, gh = (H + C - 1) / C;
  std::vector<int32_t> start(gw * gh + 1, 0), pts(n), cuv(n), rmin(H, 1 << 30), rmax(H, -1);
  for (int32_t i = 0; i < n; ++i) {
    const P2 q = star::unpack(uv[i]);
    ++start[(q.y / C) * gw + q.x / C + 1];
    rmin[q.y] = std::min(rmin[q.y], q.x);
    rmax[q.y] = std::max(rmax[q.y], q.x);
  }
  for (int32_t c = 0; c < gw * gh; ++c) start[c + 1] += start[c];
  std::vector<int32_t> cur(start.begin(), start.end() - 1);
  for (int32_t i = n - 1; i >= 0; --i) {  // any order within a cell gives the same result
    const P2 q = star::unpack(uv[i]);
    const int32_t e = cur[(q.y / C) * gw + q.x / C]++;
    pts[e] = i;
    cuv[e] = uv[i];
  }
  star::Grid g{uv.data(), n, W, H, gw, gh, start.data(), pts.data(), cuv.data(), rmin.data(), rmax.data()};
  for (int32_t p = 0; p < n; ++p) {
    HostOut o{&out, p, {}};
    const size_t before = out.size();
    HostWave wv;
    const int32_t r = star::star_of(wv, g, p, o);
    if (r < 0) return -r;
    if (out.size() - before != (size_t)r) return 99;
  }
  return 0;
}

struct Arrays {
  std::vector<int32_t> tv, tnb, own, kids, dead, fk, fs, fj, work[2], pend[2], ploc, pk, psib, uv;
  std::vector<uint64_t> vote, fkey, pkey;
};

}  // namespace

int main() {
  int W, H, nb, mode;
  if (scanf("%d %d %d %d", &W, &H, &nb, &mode) != 4) return 2;
  if (mode == 3) {  // predicates: nb lines "ax ay bx by cx cy dx dy" -> "filter sos"
    for (int k = 0; k < nb; ++k) {
      P2 q[4];
      for (auto& p : q)
        if (scanf("%d %d", &p.x, &p.y) != 2) return 2;
      printf("%d %d\n", incircle_filter(q[0], q[1], q[2], q[3]), incircle_sos(q[0], q[1], q[2], q[3]));
    }
    return 0;
  }
  if (mode == 4) {  // per-point stars over every batch's points so far
    std::vector<int32_t> uv;
    for (int b = 0; b < nb; ++b) {
      int n;
      if (scanf("%d", &n) != 1) return 2;
      for (int i = 0; i < n; ++i) {
        int u, v;
        if (scanf("%d %d", &u, &v) != 2) return 2;
        uv.push_back(pack_uv(u, v));
      }
      std::vector<sm_tri> out;
      const int status = star_mesh(uv, W, H, out);
      std::sort(out.begin(), out.end(), [](const sm_tri& x, const sm_tri& y) {
        if (x.i0 != y.i0) return x.i0 < y.i0;
        if (x.i1 != y.i1) return x.i1 < y.i1;
        return x.i2 < y.i2;
      });
      printf("batch %d %zu %d\n", b, status ? (size_t)0 : out.size(), status);
      if (!status)
        for (const sm_tri& t : out) printf("%d %d %d\n", t.i0, t.i1, t.i2);
    }
    return 0;
  }
  std::vector<sm_support> S;
  std::vector<std::pair<int32_t, int32_t>> range;
  for (int b = 0; b < nb; ++b) {
    int n;
    if (scanf("%d", &n) != 1) return 2;
    const int32_t p0 = (int32_t)S.size();
    for (int i = 0; i < n; ++i) {
      int u, v;
      if (scanf("%d %d", &u, &v) != 2) return 2;
      S.push_back(sm_support{(int16_t)u, (int16_t)v, 0.f});
    }
    range.push_back({p0, (int32_t)S.size()});
  }
  const int32_t n_all = (int32_t)S.size();
  const int32_t cap = 16 * n_all + 1024;
  Arrays a;
  a.tv.assign(3 * (size_t)cap, 0);
  a.tnb.assign(3 * (size_t)cap, 0);
  a.own.assign(3 * (size_t)cap, -1);
  a.kids.assign(4 * (size_t)cap, -1);
  a.dead.assign(cap, 0);
  a.fk.assign(cap, -1);
  a.fs.assign(cap, 0);
  a.fj.assign(cap, 0);
  a.vote.assign(cap, ~0ull);
  a.fkey.assign(cap, 0);
  for (int k = 0; k < 2; ++k) a.work[k].assign(cap, 0);
  a.uv.resize(n_all);
  for (int32_t p = 0; p < n_all; ++p) a.uv[p] = pack_uv(S[p].u, S[p].v);
  Mesh m{a.uv.data(), a.tv.data(), a.tnb.data(), a.own.data(), a.kids.data(), a.dead.data(), a.vote.data(),
         a.fk.data(), a.fs.data(), a.fj.data(), a.fkey.data(), cap, 0, nullptr, nullptr, nullptr, nullptr};
  std::mt19937 rng(12345);
  int32_t n_rec = 0, round_base = 0;
  // rounds of propose / execute over np pending points (pend[0]) and nw work entries (work[0])
  auto rounds = [&](int32_t np, int32_t nw, int32_t err) -> int32_t {
    const int32_t pcap = std::max<int32_t>(np, 1);
    int32_t cur = 0, round = 0;
    std::vector<int32_t> order;
    for (; !err && np + nw > 0; ++round) {
      if (round_base + round >= kMaxRounds) {
        err = kErrRounds;
        break;
      }
      order.resize(np + nw);
      for (int32_t k = 0; k < np + nw; ++k) order[k] = k;
      std::shuffle(order.begin(), order.end(), rng);
      for (int32_t k : order) {
        if (k < np) propose_point<Seq>(m, a.pend[cur][k], round_base + round, n_rec, &err);
        else propose_flip<Seq>(m, a.work[cur][k - np], round_base + round, n_rec, &err);
      }
      if (err) break;
      std::shuffle(order.begin(), order.end(), rng);
      int32_t np2 = 0, nw2 = 0;
      for (int32_t k : order) {
        if (k < np)
          execute_point<Seq>(m, a.pend[cur][k], &n_rec, a.pend[cur ^ 1].data(), &np2, pcap, a.work[cur ^ 1].data(),
                             &nw2, cap, &err);
        else
          execute_flip<Seq>(m, a.work[cur][k - np], &n_rec, a.work[cur ^ 1].data(), &nw2, cap, &err);
      }
      cur ^= 1;
      np = np2;
      nw = nw2;
    }
    round_base += round;
    fprintf(stderr, "rounds %d records %d\n", round, n_rec);
    return err;
  };
  for (int b = 0; b < nb; ++b) {
    const int32_t p0 = range[b].first, n_new = range[b].second - p0;
    int status = 0;
    if (b == 0 && mode >= 1) {
      // device start: rows, ladders, pockets, links, then flips of every solid triangle
      const int32_t n = n_new;
      std::vector<int32_t> row_first(n + 1), row_of(n), strip_base(n + 1), gh_start(n, -1), gh_end(n, -1),
          stk(2 * n + 2);
      int32_t hcap = 1;
      while (hcap < 16 * n + 64) hcap <<= 1;
      std::vector<uint64_t> keys(hcap, kEmptyEdge);
      std::vector<int32_t> vals(hcap, 0);
      Start st{n,           row_first.data(), row_of.data(), strip_base.data(), gh_start.data(),
               gh_end.data(), stk.data(),       keys.data(),   vals.data(),       hcap};
      int32_t err = 0, n_rows = 0;
      for (int32_t i = 0; i < n; ++i) {
        if (row_starts<Seq>(m, i, &err)) row_first[n_rows++] = i;
        row_of[i] = n_rows - 1;
      }
      if (!err && n_rows >= 2) {
        int32_t base = 0;
        for (int32_t r = 0; r + 1 < n_rows; ++r) {
          strip_base[r] = base;
          base += ladder_size(st, r, n_rows);
        }
        std::vector<int32_t> order;
        for (int32_t i = 0; i < n; ++i) order.push_back(i);
        std::shuffle(order.begin(), order.end(), rng);
        for (int32_t i : order) ladder_point<Seq>(m, st, i, n_rows);
        n_rec = base;
        pockets<Seq>(m, st, 1, n_rows, &n_rec, &err);
        pockets<Seq>(m, st, 0, n_rows, &n_rec, &err);
        const int32_t n_solid = n_rec;
        order.clear();
        for (int32_t e = 0; e < 3 * n_solid; ++e) order.push_back(e);
        if (mode == 2) {  // links by pairing each undirected edge's two directed edges
          const int32_t tcap = pair_table_size(n_solid, n);
          std::vector<uint64_t> tab(tcap, 0);
          std::shuffle(order.begin(), order.end(), rng);
          for (int32_t e : order)
            pair_edge<Seq>(m, tab.data(), tcap, e / 3, e % 3, a.tv[3 * (e / 3) + nxt(e % 3)],
                           a.tv[3 * (e / 3) + prv(e % 3)], &err);
          for (int32_t h = 0; h < tcap; ++h) pair_hull<Seq>(m, st, tab[h], &n_rec, &err);
        } else {  // links through the edge hash table
          std::shuffle(order.begin(), order.end(), rng);
          for (int32_t e : order) edge_insert<Seq>(m, st, e / 3, e % 3, &err);
          std::shuffle(order.begin(), order.end(), rng);
          for (int32_t e : order) edge_link<Seq>(m, st, e / 3, e % 3, &n_rec, &err);
        }
        for (int32_t g = n_solid; g < n_rec; ++g) ghost_link<Seq>(m, st, g, &err);
        for (int32_t t = 0; t < n_rec; ++t) a.dead[t] = 0, a.vote[t] = ~0ull;
        int32_t nw = 0;
        for (int32_t t = 0; t < n_solid; ++t) a.work[0][nw++] = work_entry(t, 7);
        if (!err) {
          m.p0 = n;
          err = rounds(0, nw, err);
        }
      } else if (!err) {
        err = 100;  // fewer than two rows: no triangle
      }
      status = err;
      if (err) n_rec = 0;
    } else if (b == 0) {
      Delaunay dl;
      std::vector<int32_t> u, v, e;
      for (int32_t p = 0; p < n_new; ++p) {
        u.push_back(S[p].u);
        v.push_back(S[p].v);
        e.push_back(p);
      }
      dl.insert_many(u.data(), v.data(), e.data(), n_new);
      n_rec = dl.export_mesh(a.tv.data(), a.tnb.data(), cap);
      if (n_rec <= 0) status = 100;
    } else if (n_rec > 0) {
      m.p0 = p0;
      a.ploc.assign(n_new, 0);
      a.pk.assign(n_new, kInside);
      a.psib.assign(n_new, 0);
      a.pkey.assign(n_new, 0);
      for (int k = 0; k < 2; ++k) a.pend[k].assign(n_new + 1, 0);
      m.ploc = a.ploc.data();
      m.pk = a.pk.data();
      m.psib = a.psib.data();
      m.pkey = a.pkey.data();
      int32_t start = -1;  // any live solid record
      for (int32_t t = 0; t < n_rec && start < 0; ++t)
        if (!a.dead[t] && a.tv[3 * t + 2] != kGhost) start = t;
      int32_t err = 0;
      for (int32_t i = 0; i < n_new && !err; ++i) {
        const int32_t t = walk<Seq>(m, start, xy<Seq>(m, p0 + i), n_rec, n_rec + 16);
        if (t < 0) err = t == -2 ? kErrOutside : kErrWalk;
        a.ploc[i] = t;
        a.pend[0][i] = i;
      }
      int32_t err2 = rounds(n_new, 0, err);
      err = err2;
      status = err;
    }
    std::vector<sm_tri> out;
    if (status == 0)
      for (int32_t t = 0; t < n_rec; ++t)
        if (!a.dead[t] && a.tv[3 * t + 2] != kGhost) out.push_back(top_first<Seq>(m, t));
    std::sort(out.begin(), out.end(), [](const sm_tri& x, const sm_tri& y) {
      if (x.i0 != y.i0) return x.i0 < y.i0;
      if (x.i1 != y.i1) return x.i1 < y.i1;
      return x.i2 < y.i2;
    });
    printf("batch %d %zu %d\n", b, out.size(), status);
    for (const sm_tri& t : out) printf("%d %d %d\n", t.i0, t.i1, t.i2);
  }
  return 0;
}
