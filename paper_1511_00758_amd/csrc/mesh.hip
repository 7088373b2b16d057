// Device Delaunay insertion of the resampled supports (tessellation of Sec. III-A for the
// iterations after the first, Alg. 1): the mesh of a frame stays in device memory between
// iterations, so the supports, the mesh and the triangles never cross to the host.
//
// One 1024-thread workgroup runs the whole insertion of a frame (the per-item steps are in
// mesh_core.hpp): packed coordinates into LDS, location hints, a visibility walk per new
// point, rounds of propose / execute separated by workgroup barriers, then the output of
// the live solid triangles. The records of a VGA frame (a few thousand) stay in L2; the
// rounds are latency-bound (a dozen per tessellation, most of them with a few dozen items)
// and one workgroup per frame lets a batch of frames share the chip.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "compact.hpp"
#include "kernels.hpp"
#include "mesh.hpp"
#include "mesh_core.hpp"
#include "mesh_start.hpp"

namespace sm {

namespace {

constexpr int kMeshThreads = 1024;
constexpr int kHintShift = 4;        // 16 x 16 px hint cells
constexpr int kHintBoxCells = 64;    // a record marks every cell of its box up to this many
constexpr int32_t kUvLds = 32768;    // supports whose coordinates fit in LDS (128 KiB)
constexpr int kEdgeBatch = 4;        // edges a thread has in flight while linking the first mesh
constexpr int kOutBatch = 8;         // records a thread has in flight in the output

// Packed coordinates of the frame's supports when they fit (one workgroup per CU).
__shared__ int32_t g_uv[kUvLds];

// Atomics of the per-item steps. One workgroup owns a frame's mesh, so every atomic has
// workgroup scope: it is performed in the L2 of the workgroup's XCD, where the plain
// accesses of the other waves meet it (device scope would send each one to memory).
// Counters and the error code live in LDS. Coordinates come from LDS (kLds) or from the
// global copy.
template <bool kLds>
struct DevA {
  __device__ static void vote_min(uint64_t* p, uint64_t v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ static uint64_t vote_get(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ static void vote_set(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ static int32_t push(int32_t* n, int32_t k) { return atomicAdd(n, k); }
  __device__ static void fail(int32_t* err, int32_t code) { atomicCAS(err, 0, code); }
  __device__ static int32_t uv(const mesh::Mesh& m, int32_t p) { return kLds ? g_uv[p] : m.uv[p]; }
  __device__ static uint64_t cas64(uint64_t* p, uint64_t expected, uint64_t desired) {
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    return expected;  // the value found: desired was stored iff it equals the expected one
  }
};

// Location hints: every 16 x 16 px cell of live solid record t's bounding box (the cells of
// its vertices when the box is large) points at it.
template <class A>
__device__ void mark_hints(const mesh::Mesh& m, int32_t* hint, int gw, int32_t t, int32_t a, int32_t b, int32_t c) {
  using namespace mesh;
  const P2 P = xy<A>(m, a), B = xy<A>(m, b), C = xy<A>(m, c);
  const int x0 = min(min(P.x, B.x), C.x) >> kHintShift, x1 = max(max(P.x, B.x), C.x) >> kHintShift;
  const int y0 = min(min(P.y, B.y), C.y) >> kHintShift, y1 = max(max(P.y, B.y), C.y) >> kHintShift;
  if ((x1 - x0 + 1) * (y1 - y0 + 1) <= kHintBoxCells) {
    for (int y = y0; y <= y1; ++y)
      for (int x = x0; x <= x1; ++x) hint[y * gw + x] = t;
  } else {
    hint[(P.y >> kHintShift) * gw + (P.x >> kHintShift)] = t;
    hint[(B.y >> kHintShift) * gw + (B.x >> kHintShift)] = t;
    hint[(C.y >> kHintShift) * gw + (C.x >> kHintShift)] = t;
  }
}

// Exclusive block-wide prefix sum of one count per thread (every thread calls it).
__device__ void block_scan1(int v, int* wsum, int& excl, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int x = __shfl_up(inc, d);
    if (lane >= d) inc += x;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int k = 0; k < kMeshThreads / 64; ++k) {
    before += k < w ? wsum[k] : 0;
    total += wsum[k];
  }
  __syncthreads();  // wsum is free again
  excl = before + inc - v;
}

template <bool kLds>
__device__ __forceinline__ void mesh_insert_block(const MeshJob& a, int32_t p0, int32_t n_new) {
  using namespace mesh;
  using DA = DevA<kLds>;
  __shared__ int32_t s_np[2], s_nw[2], s_nrec, s_err, s_any, s_ntri, s_next_any;
  __shared__ int s_wsum[kMeshThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63;
  const MeshWork& w = a.w;
  // every thread reads the same control words, so the early exits below are uniform
  const bool start = a.start != 0;
  const bool fresh = !start && a.init_n > 0;
  const int32_t n_rec0 = start ? 0 : (fresh ? a.init_n : a.status[kMeshRecords]);
  const int32_t base_round = start || fresh ? 0 : a.status[kMeshRounds];
  const int32_t tess = start || fresh ? 0 : a.status[kMeshTess];
  const int32_t prior_err = start || fresh ? 0 : a.status[kMeshErr];
  const int32_t n_pts = p0 + n_new;
  auto finish = [&](int32_t n_rec, int32_t n_tri, int32_t err, int32_t rounds) {  // thread 0
    const int32_t words[8] = {n_rec, n_tri, err, rounds, n_new, n_pts, tess + 1, err == 0 ? s_next_any : -1};
    for (int k = 0; k < 8; ++k) {
      a.status[k] = words[k];
      if (a.status_copy) a.status_copy[k] = words[k];
    }
    if (tess >= 0 && tess < 8) {
      a.status[kMeshLog + 2 * tess] = n_pts;
      a.status[kMeshLog + 2 * tess + 1] = n_tri;
      if (a.status_copy) {
        a.status_copy[kMeshLog + 2 * tess] = n_pts;
        a.status_copy[kMeshLog + 2 * tess + 1] = n_tri;
      }
    }
  };
  __syncthreads();
  if (prior_err != 0) {  // an earlier tessellation failed: the frame goes to the host
    if (tid == 0) finish(n_rec0, 0, prior_err, base_round);
    return;
  }
  const bool bad = start ? (p0 != 0 || n_new < 0 || n_pts > w.S_cap)
                         : (n_rec0 <= 0 || n_rec0 > w.cap || n_new < 0 || n_new > w.pcap || p0 < 3 ||
                            n_pts > w.S_cap || base_round < 0 || base_round >= kMaxRounds);
  if (bad || (start && n_new < 3)) {
    if (tid == 0) finish(n_rec0, 0, bad ? kErrCapacity : kMeshErrNoMesh, base_round);
    return;
  }
  if (tid == 0) {
    s_np[0] = start ? 0 : n_new;
    s_nw[0] = 0;
    s_np[1] = s_nw[1] = 0;
    s_nrec = n_rec0;
    s_err = 0;
    // a later tessellation locates its points from the hints the previous one left
    s_any = start || fresh ? -1 : a.status[kMeshAny];
    s_next_any = -1;
    s_ntri = 0;
  }
  const int32_t gw = (a.W + 15) >> kHintShift, gh = (a.H + 15) >> kHintShift;
  int32_t* uv = kLds ? g_uv : w.uv;
  Mesh m;
  m.uv = w.uv;
  m.tv = w.tv;
  m.tnb = w.tnb;
  m.own = w.own;
  m.kids = w.kids;
  m.dead = w.dead;
  m.vote = w.vote;
  m.fk = w.fk;
  m.fs = w.fs;
  m.fj = w.fj;
  m.fkey = w.fkey;
  m.cap = w.cap;
  m.p0 = p0;
  m.ploc = w.ploc;
  m.pk = w.pk;
  m.psib = w.psib;
  m.pkey = w.pkey;
  __syncthreads();

  // packed coordinates (range-checked: the predicates are exact for [0, 8191]); records
  // just written by the host are checked and initialised; hints cleared
  for (int32_t p = tid; p < n_pts; p += kMeshThreads) {
    const sm_support P = a.S[p];
    if (P.u < 0 || P.v < 0 || P.u >= a.W || P.v >= a.H) {
      DA::fail(&s_err, kErrIndex);
      uv[p] = 0;
    } else {
      uv[p] = pack_uv(P.u, P.v);
    }
  }
  if (fresh) {
    for (int32_t t = tid; t < n_rec0; t += kMeshThreads) {
      bool ok = true;
      for (int k = 0; k < 3; ++k) {
        const int32_t v = a.init_tv[3 * t + k], nb = a.init_tnb[3 * t + k];
        ok &= (v >= 0 && v < p0) || (k == 2 && v == kGhost);
        ok &= nb >= 0 && nb < n_rec0;
        w.tv[3 * t + k] = v;
        w.tnb[3 * t + k] = nb;
      }
      if (!ok) DA::fail(&s_err, kErrIndex);
      w.dead[t] = 0;
      DA::vote_set(&w.vote[t], ~0ull);
    }
  }
  // the edge table of a first mesh: 16 slots per support (about 6 directed edges each),
  // within the workspace's table
  int32_t hcap = 1024;
  while (hcap < w.hcap && hcap < 16 * (int64_t)n_new) hcap <<= 1;
  hcap = min(hcap, w.hcap);
  if (fresh)
    for (int32_t c = tid; c < gw * gh; c += kMeshThreads) w.hint[c] = -1;
  if (start) {
    for (int32_t i = tid; i < n_new; i += kMeshThreads) w.gh_start[i] = w.gh_end[i] = -1;
  }
  __syncthreads();

  if (start) {  // the first mesh: rows, ladders, pockets, links (mesh_start.hpp)
    Start st;
    st.n = n_new;
    st.row_first = w.row_first;
    st.row_of = w.row_of;
    st.strip_base = w.strip_base;
    st.gh_start = w.gh_start;
    st.gh_end = w.gh_end;
    st.stack = w.stack;
    st.keys = w.hkeys;
    st.vals = w.hvals;
    st.hcap = hcap;
    // rows: each thread scans a contiguous run of supports
    const int32_t per = (n_new + kMeshThreads - 1) / kMeshThreads;
    const int32_t lo = min(tid * per, n_new), hi = min(lo + per, n_new);
    int cnt = 0;
    for (int32_t i = lo; i < hi; ++i) cnt += row_starts<DA>(m, i, &s_err);
    int base, n_rows;
    block_scan1(cnt, s_wsum, base, n_rows);
    for (int32_t i = lo; i < hi; ++i) {
      if (row_starts<DA>(m, i, &s_err)) w.row_first[base++] = i;
      w.row_of[i] = base - 1;
    }
    __syncthreads();
    if (n_rows < 2 || s_err != 0) {  // uniform: read after the barrier, nothing writes s_err here
      if (tid == 0) finish(0, 0, s_err != 0 ? s_err : kMeshErrNoMesh, 0);
      return;
    }
    // strips: ladder sizes, their prefix sums, the ladders
    const int32_t ns = n_rows - 1;
    const int32_t per2 = (ns + kMeshThreads - 1) / kMeshThreads;
    const int32_t lo2 = min(tid * per2, ns), hi2 = min(lo2 + per2, ns);
    int cnt2 = 0;
    for (int32_t r = lo2; r < hi2; ++r) cnt2 += ladder_size(st, r, n_rows);
    int base2, n_ladder;
    block_scan1(cnt2, s_wsum, base2, n_ladder);
    for (int32_t r = lo2; r < hi2; ++r) {
      w.strip_base[r] = base2;
      base2 += ladder_size(st, r, n_rows);
    }
    if (tid == 0) s_nrec = n_ladder;
    __syncthreads();
    for (int32_t i = tid; i < n_new; i += kMeshThreads) ladder_point<DA>(m, st, i, n_rows);
    // hull pockets: the two side chains, one thread each; the row starts and both stacks
    // sit in LDS after the coordinates when they fit (a branch of its own, so that its
    // accesses compile to LDS instructions)
    const bool chain_lds = kLds && (int64_t)n_new + 3 * (int64_t)n_rows <= kUvLds;
    if (chain_lds)
      for (int32_t r = tid; r < n_rows; r += kMeshThreads) g_uv[n_new + r] = w.row_first[r];
    __syncthreads();
    if (chain_lds) {
      Start sp = st;
      sp.row_first = g_uv + n_new;
      sp.stack = g_uv + n_new + n_rows;
      if (tid == 0) pockets<DA>(m, sp, 1, n_rows, &s_nrec, &s_err);
      if (tid == 64) pockets<DA>(m, sp, 0, n_rows, &s_nrec, &s_err);
    } else {
      if (tid == 0) pockets<DA>(m, st, 1, n_rows, &s_nrec, &s_err);
      if (tid == 64) pockets<DA>(m, st, 0, n_rows, &s_nrec, &s_err);
    }
    __syncthreads();
    const int32_t n_solid = s_nrec;
    if (n_solid == 0 || s_err != 0) {  // every support on one line (or a full array)
      if (tid == 0) finish(0, 0, s_err != 0 ? s_err : kMeshErrNoMesh, 0);
      return;
    }
    const int32_t n_edges = 3 * n_solid;
    // links by pairing in a table in LDS after the coordinates when it fits, else through
    // the edge hash table in global memory
    const int32_t n_even = (n_new + 1) & ~1;  // 8-byte alignment of the table
    const int32_t tcap = pair_table_size(n_solid, n_new);
    const bool pairs = kLds && n_new < kPairMaxVertices && n_even + 2 * (int64_t)tcap <= kUvLds;
    if (pairs) {
      uint64_t* tab = (uint64_t*)(g_uv + n_even);
      for (int32_t h = tid; h < tcap; h += kMeshThreads) tab[h] = 0;
      __syncthreads();
      // each thread holds kEdgeBatch edges' vertices in flight (the loads take no
      // conditions: a missing edge reads edge 0)
      for (int32_t e0 = tid; e0 < n_edges; e0 += kEdgeBatch * kMeshThreads) {
        int32_t ex[kEdgeBatch], ey[kEdgeBatch];
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b) {
          const int32_t e = e0 + b * kMeshThreads, ec = e < n_edges ? e : 0;
          ex[b] = w.tv[3 * (ec / 3) + nxt(ec % 3)];
          ey[b] = w.tv[3 * (ec / 3) + prv(ec % 3)];
        }
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b) {
          const int32_t e = e0 + b * kMeshThreads;
          if (e < n_edges) pair_edge<DA>(m, tab, tcap, e / 3, e % 3, ex[b], ey[b], &s_err);
        }
      }
      __syncthreads();
      for (int32_t h = tid; h < tcap; h += kMeshThreads) pair_hull<DA>(m, st, tab[h], &s_nrec, &s_err);
      __syncthreads();
    } else {
      for (int32_t h = tid; h < hcap; h += kMeshThreads) w.hkeys[h] = kEmptyEdge;
      __syncthreads();
      // every thread keeps kEdgeBatch first probes in flight (compare-and-swap when
      // inserting, a load when looking up the reverse edge), then settles them in order
      // (the loads take no conditions, a missing edge reads edge 0, so that they leave back
      // to back; only the atomics and the settling look at the range)
      for (int32_t e0 = tid; e0 < n_edges; e0 += kEdgeBatch * kMeshThreads) {
        uint64_t key[kEdgeBatch], old[kEdgeBatch];
        uint32_t h[kEdgeBatch];
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b) {
          const int32_t e = e0 + b * kMeshThreads, ec = e < n_edges ? e : 0;
          key[b] = solid_edge_key(m, ec / 3, ec % 3, false);
        }
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b) h[b] = edge_hash(key[b]) & (uint32_t)(hcap - 1);
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b)
          old[b] = e0 + b * kMeshThreads < n_edges ? DA::cas64(&st.keys[h[b]], kEmptyEdge, key[b]) : 0;
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b) {
          const int32_t e = e0 + b * kMeshThreads;
          if (e < n_edges) edge_insert_from<DA>(st, key[b], e, h[b], old[b], &s_err);
        }
      }
      __syncthreads();
      for (int32_t e0 = tid; e0 < n_edges; e0 += kEdgeBatch * kMeshThreads) {
        uint64_t key[kEdgeBatch], cur[kEdgeBatch];
        uint32_t h[kEdgeBatch];
        int32_t slot[kEdgeBatch], val[kEdgeBatch];
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b) {
          const int32_t e = e0 + b * kMeshThreads, ec = e < n_edges ? e : 0;
          key[b] = solid_edge_key(m, ec / 3, ec % 3, true);
        }
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b) {
          h[b] = edge_hash(key[b]) & (uint32_t)(hcap - 1);
          cur[b] = DA::vote_get(&st.keys[h[b]]);
        }
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b) slot[b] = edge_find_from<DA>(st, key[b], h[b], cur[b]);
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b) val[b] = st.vals[slot[b] >= 0 ? slot[b] : 0];
#pragma unroll
        for (int b = 0; b < kEdgeBatch; ++b) {
          const int32_t e = e0 + b * kMeshThreads;
          if (e < n_edges) edge_link_to<DA>(m, st, e / 3, e % 3, slot[b], val[b], &s_nrec, &s_err);
        }
      }
      __syncthreads();
    }
    const int32_t n_all = min(s_nrec, w.cap);
    for (int32_t g = n_solid + tid; g < n_all; g += kMeshThreads) ghost_link<DA>(m, st, g, &s_err);
    for (int32_t t = tid; t < n_all; t += kMeshThreads) {
      w.dead[t] = 0;
      DA::vote_set(&w.vote[t], ~0ull);
    }
    for (int32_t t = tid; t < n_solid; t += kMeshThreads) w.work0[t] = work_entry(t, 7);  // test every edge
    if (tid == 0) s_nw[0] = n_solid;
  }

  // hints of a mesh from the host (a device mesh leaves its hints in its output)
  if (fresh && s_err == 0) {
    for (int32_t t = tid; t < n_rec0; t += kMeshThreads) {
      if (w.dead[t] || w.tv[3 * t + 2] == kGhost) continue;
      mark_hints<DA>(m, w.hint, gw, t, w.tv[3 * t], w.tv[3 * t + 1], w.tv[3 * t + 2]);
      atomicMax(&s_any, t);
    }
  }
  __syncthreads();

  // locate every new point by a visibility walk from the hint of its cell
  if (start) {
  } else if (s_err == 0 && s_any >= 0) {
    for (int32_t i = tid; i < n_new; i += kMeshThreads) {
      const P2 q = xy<DA>(m, p0 + i);
      int32_t h = w.hint[(q.y >> kHintShift) * gw + (q.x >> kHintShift)];
      if (h < 0) h = s_any;
      const int32_t t = walk<DA>(m, h, q, n_rec0, n_rec0 + 16);
      if (t < 0) {
        DA::fail(&s_err, t == -2 ? kErrOutside : kErrWalk);
        continue;
      }
      w.ploc[i] = t;
      w.pk[i] = kInside;
      w.pend0[i] = i;
    }
  } else if (tid == 0 && s_any < 0) {
    DA::fail(&s_err, kErrIndex);
  }

  // rounds of propose / execute; the control values are read between two barriers, so
  // that every thread takes the same decision before any thread can change them
  auto propose_all = [&](int32_t first, int32_t stride, int32_t np, int32_t nw, int32_t n_rec, int32_t gr, int c) {
    const int32_t* pend = c ? w.pend1 : w.pend0;
    const int32_t* work = c ? w.work1 : w.work0;
    for (int32_t it = first; it < np + nw; it += stride) {
      if (it < np) propose_point<DA>(m, pend[it], gr, n_rec, &s_err);
      else propose_flip<DA>(m, work[it - np], gr, n_rec, &s_err);
    }
  };
  auto execute_all = [&](int32_t first, int32_t stride, int32_t np, int32_t nw, int c) {
    const int32_t* pend = c ? w.pend1 : w.pend0;
    const int32_t* work = c ? w.work1 : w.work0;
    int32_t* pend_next = c ? w.pend0 : w.pend1;
    int32_t* work_next = c ? w.work0 : w.work1;
    for (int32_t it = first; it < np + nw; it += stride) {
      if (it < np)
        execute_point<DA>(m, pend[it], &s_nrec, pend_next, &s_np[c ^ 1], w.pcap, work_next, &s_nw[c ^ 1], w.cap,
                          &s_err);
      else
        execute_flip<DA>(m, work[it - np], &s_nrec, work_next, &s_nw[c ^ 1], w.cap, &s_err);
    }
  };
  int cur = 0, round = 0;
  for (;;) {
    __syncthreads();
    const int32_t np = s_np[cur], nw = s_nw[cur], n_rec = s_nrec, err = s_err;
    __syncthreads();
    if (err != 0 || np + nw == 0) break;
    const int32_t gr = base_round + round;
    if (gr >= kMaxRounds) {
      if (tid == 0) s_err = kErrRounds;
      break;
    }
    propose_all(tid, kMeshThreads, np, nw, n_rec, gr, cur);
    if (tid == 0) s_np[cur ^ 1] = s_nw[cur ^ 1] = 0;  // last read before the previous round's work
    __syncthreads();
    if (s_err == 0) execute_all(tid, kMeshThreads, np, nw, cur);  // items only: no barrier depends on this test
    cur ^= 1;
    ++round;
  }
  __syncthreads();
  if (s_err != 0) {
    if (tid == 0) finish(s_nrec, 0, s_err, base_round + round);
    return;
  }

  // output: live solid records as triangles, and the hints of the next tessellation (the
  // walks of this one are over). Each thread has kOutBatch records in flight, state and
  // vertices loaded at once (an index past the records reads record 0, not output); one
  // atomic per wave reserves their slots.
  const bool hints = a.last == 0;
  if (hints)
    for (int32_t c = tid; c < gw * gh; c += kMeshThreads) w.hint[c] = -1;
  __syncthreads();
  const int32_t n_rec = s_nrec;
  for (int32_t base = 0; base < n_rec; base += kOutBatch * kMeshThreads) {  // uniform: the wave scans below
    const int32_t t0 = base + tid;
    unsigned outm = 0;  // bit b: record t0 + b * kMeshThreads is output
    int any = -1;
    int32_t dd[kOutBatch], ov0[kOutBatch], ov1[kOutBatch], ov2[kOutBatch];
#pragma unroll
    for (int b = 0; b < kOutBatch; ++b) {
      const int32_t t = t0 + b * kMeshThreads, tc = t < n_rec ? t : 0;
      dd[b] = w.dead[tc];
      ov0[b] = w.tv[3 * tc], ov1[b] = w.tv[3 * tc + 1], ov2[b] = w.tv[3 * tc + 2];
    }
#pragma unroll
    for (int b = 0; b < kOutBatch; ++b) {
      const int32_t t = t0 + b * kMeshThreads;
      const bool out = t < n_rec && !dd[b] && ov2[b] != kGhost;
      outm |= (unsigned)out << b;
      if (out) any = t;
    }
    const int cnt = __popc(outm);
    int inc = cnt;  // inclusive scan over the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int x = __shfl_up(inc, d);
      if (lane >= d) inc += x;
    }
    int slot = 0;
    if (lane == 63 && inc > 0) slot = atomicAdd(&s_ntri, inc);
    slot = __shfl(slot, 63) + inc - cnt;
    const unsigned long long has = __ballot(any >= 0);  // one record per wave suffices
    if (has && lane == __ffsll((long long)has) - 1) atomicMax(&s_next_any, any);
#pragma nounroll
    for (int b = 0; b < kOutBatch; ++b) {
      // record b's vertices sit in slot 0: the arrays shift down one slot per step, so that
      // every index is a constant and they stay in registers
      const int32_t v0 = ov0[0], v1 = ov1[0], v2 = ov2[0];
#pragma unroll
      for (int k = 0; k + 1 < kOutBatch; ++k) ov0[k] = ov0[k + 1], ov1[k] = ov1[k + 1], ov2[k] = ov2[k + 1];
      if (!(outm >> b & 1u)) continue;
      const int32_t t = t0 + b * kMeshThreads;
      if (slot < a.T_cap) a.T[slot] = top_first3<DA>(m, v0, v1, v2);
      else DA::fail(&s_err, kErrCapacity);
      ++slot;
      if (hints) mark_hints<DA>(m, w.hint, gw, t, v0, v1, v2);
    }
  }
  __syncthreads();
  if (tid == 0) finish(n_rec, s_ntri, s_err, base_round + round);
}

__device__ __forceinline__ void mesh_insert(const MeshJob& a) {
  // the same for every thread: the branches are uniform
  int32_t p0 = a.p0, n_new = 0;
  bool ok = true;
  if (p0 < 0) {  // first new support and its count kept on the device
    p0 = a.status[kMeshSupports];
    ok = p0 >= 3 && p0 < a.w.S_cap && a.n_new_slot >= 0 && (int64_t)p0 + a.n_new_slot < a.w.S_cap;
  }
  // the supports' compaction first, in place (a frame whose earlier tessellation failed is
  // solved again on the host: nothing to compact)
  if (ok && a.compact_n > 0 && (a.start || a.status[kMeshErr] == 0) && (int64_t)p0 + a.compact_n < a.w.S_cap) {
    sm_support* slots = const_cast<sm_support*>(a.S) + p0;
    compact_block(slots, a.compact_n, a.compact_count, a.occ, a.W, (int*)(slots + a.compact_n));
    __syncthreads();
  }
  if (!ok) p0 = 0, n_new = -1;
  else if (a.p0 >= 0) n_new = *a.n_new;
  else n_new = *(const int32_t*)(a.S + p0 + a.n_new_slot);
  if ((int64_t)p0 + n_new <= kUvLds) mesh_insert_block<true>(a, p0, n_new);
  else mesh_insert_block<false>(a, p0, n_new);
}

__global__ __launch_bounds__(kMeshThreads) void k_mesh_insert(MeshJob a) { mesh_insert(a); }

// A pointer read from device memory has no known address space; this one is global, and
// saying so turns its accesses into global (not flat) instructions.
template <class T>
__device__ __forceinline__ T* as_global(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

__global__ __launch_bounds__(kMeshThreads) void k_mesh_insert_many(const MeshJob* __restrict__ jobs) {
  MeshJob a = jobs[blockIdx.x];
  a.S = as_global(a.S);
  a.n_new = as_global(a.n_new);
  a.init_tv = as_global(a.init_tv);
  a.init_tnb = as_global(a.init_tnb);
  a.status = as_global(a.status);
  a.status_copy = as_global(a.status_copy);
  a.T = as_global(a.T);
  a.occ = as_global(a.occ);
  a.compact_count = as_global(a.compact_count);
  MeshWork& w = a.w;
  for (int32_t** q : {&w.tv, &w.tnb, &w.own, &w.kids, &w.dead, &w.fk, &w.fs, &w.fj, &w.work0, &w.work1, &w.ploc,
                      &w.pk, &w.psib, &w.pend0, &w.pend1, &w.uv, &w.hint, &w.row_first, &w.row_of, &w.strip_base,
                      &w.gh_start, &w.gh_end, &w.stack, &w.hvals})
    *q = as_global(*q);
  w.vote = as_global(w.vote);
  w.fkey = as_global(w.fkey);
  w.pkey = as_global(w.pkey);
  w.hkeys = as_global(w.hkeys);
  mesh_insert(a);
}

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carve {
  size_t o = 0;
  uint8_t* base = nullptr;
  template <class T>
  T* take(size_t n) {
    T* p = base ? (T*)(base + o) : nullptr;
    o = align256(o + n * sizeof(T));
    return p;
  }
};

MeshWork carve(Carve& c, int32_t W, int32_t H, int32_t S_cap, int32_t pcap) {
  MeshWork w;
  const int32_t cap = mesh_work_cap(S_cap);
  const size_t nc = (size_t)cap, np = (size_t)pcap;
  w.tv = c.take<int32_t>(3 * nc);
  w.tnb = c.take<int32_t>(3 * nc);
  w.own = c.take<int32_t>(3 * nc);
  w.kids = c.take<int32_t>(4 * nc);
  w.dead = c.take<int32_t>(nc);
  w.fk = c.take<int32_t>(nc);
  w.fs = c.take<int32_t>(nc);
  w.fj = c.take<int32_t>(nc);
  w.work0 = c.take<int32_t>(nc);
  w.work1 = c.take<int32_t>(nc);
  w.vote = c.take<uint64_t>(nc);
  w.fkey = c.take<uint64_t>(nc);
  w.ploc = c.take<int32_t>(np);
  w.pk = c.take<int32_t>(np);
  w.psib = c.take<int32_t>(np);
  w.pend0 = c.take<int32_t>(np);
  w.pend1 = c.take<int32_t>(np);
  w.pkey = c.take<uint64_t>(np);
  w.uv = c.take<int32_t>((size_t)S_cap);
  w.hint = c.take<int32_t>((size_t)((W + 15) >> kHintShift) * ((H + 15) >> kHintShift));
  int32_t hcap = 1024;
  while (hcap < 16 * (int64_t)S_cap && hcap < (1 << 28)) hcap <<= 1;  // 6 directed edges per support, load <= 3/8
  w.row_first = c.take<int32_t>((size_t)S_cap + 1);
  w.row_of = c.take<int32_t>((size_t)S_cap);
  w.strip_base = c.take<int32_t>((size_t)S_cap + 1);
  w.gh_start = c.take<int32_t>((size_t)S_cap);
  w.gh_end = c.take<int32_t>((size_t)S_cap);
  w.stack = c.take<int32_t>(2 * (size_t)S_cap + 2);
  w.hkeys = c.take<uint64_t>((size_t)hcap);
  w.hvals = c.take<int32_t>((size_t)hcap);
  w.cap = cap;
  w.pcap = pcap;
  w.S_cap = S_cap;
  w.hcap = hcap;
  return w;
}

}  // namespace

int32_t mesh_work_cap(int32_t S_cap) {
  const int64_t cap = 8 * (int64_t)S_cap + 4096;  // work-list entries keep record ids below 2^28
  return (int32_t)(cap > (1 << 28) ? (1 << 28) : cap);
}

size_t mesh_work_bytes(int32_t W, int32_t H, int32_t S_cap, int32_t pcap) {
  Carve c;
  carve(c, W, H, S_cap, pcap);
  return c.o;
}

MeshWork mesh_work_at(void* base, int32_t W, int32_t H, int32_t S_cap, int32_t pcap) {
  Carve c;
  c.base = (uint8_t*)base;
  return carve(c, W, H, S_cap, pcap);
}

hipError_t launch_mesh_insert(const MeshJob& job, hipStream_t s) {
  hipEvent_t e0, e1;
  if (take_launch_events(&e0, &e1))
    hipExtLaunchKernelGGL(k_mesh_insert, dim3(1), dim3(kMeshThreads), 0, s, e0, e1, 0u, job);
  else
    hipLaunchKernelGGL(k_mesh_insert, dim3(1), dim3(kMeshThreads), 0, s, job);
  return hipGetLastError();
}

hipError_t launch_mesh_insert_many(const MeshJob* jobs, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipEvent_t e0, e1;
  if (take_launch_events(&e0, &e1))
    hipExtLaunchKernelGGL(k_mesh_insert_many, dim3((unsigned)n), dim3(kMeshThreads), 0, s, e0, e1, 0u, jobs);
  else
    hipLaunchKernelGGL(k_mesh_insert_many, dim3((unsigned)n), dim3(kMeshThreads), 0, s, jobs);
  return hipGetLastError();
}

}  // namespace sm
