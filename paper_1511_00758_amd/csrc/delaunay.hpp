// Host Delaunay triangulation of support pixels (the mesh G(S) of Sec. III-A).
//
// Incremental insertion with an adjacency structure: the point is located by a
// visibility walk from the last created triangle, the triangles whose perturbed
// circumcircle strictly contains it are collected by a flood over neighbours, and
// the hole is re-filled by a fan around the point. Hull edges carry ghost triangles
// (third vertex kGhost) whose conflict region is the open outer half-plane of the
// edge plus the open edge.
//
// Predicates are exact in 64-bit integers for coordinates in [0, 8191]. In-circle
// ties are decided by symbolic perturbation of the lifted heights
// z_i = u_i^2 + v_i^2 + eps_i with eps larger for a smaller raster position (v, u),
// which makes the triangulation unique: the result does not depend on insertion
// order, so points can be added to an existing mesh between iterations.
#pragma once

#include <cstdint>
#include <vector>

#include "stereomesh.h"

namespace sm {

class Delaunay {
 public:
  static constexpr int32_t kGhost = -1;

  void reset();
  // Inserts points (u, v) carrying external indices; duplicates of an existing
  // point are skipped (the first occurrence stays). Returns false if a point lies
  // outside [0, 8191]^2.
  bool insert(int32_t u, int32_t v, int32_t ext);
  // Inserts n points in a biased randomised insertion order (random rounds of doubling
  // size, each round in Hilbert-curve order of 32 px cells): short walks and small
  // holes whatever the input order. Returns false if a point lies outside [0, 8191]^2 (nothing is
  // inserted then).
  bool insert_many(const int32_t* u, const int32_t* v, const int32_t* ext, int32_t n);
  // Appends the solid triangles as external indices, counter-clockwise, first
  // vertex = smallest (v, u). Sorted by (i0, i1, i2) when `sorted`.
  void emit(std::vector<sm_tri>& out, bool sorted) const;
  // Same triangles ordered by the row band (top row >> band_shift) of their first
  // vertex (a counting sort): spatially coherent work for the rasteriser.
  void emit_banded(std::vector<sm_tri>& out, int band_shift) const;
  int32_t n_points() const { return (int32_t)pt_.size(); }
  int32_t n_solid() const { return n_solid_; }

 private:
  struct Tri {
    int32_t v[3];   // vertices (local point ids); v[2] == kGhost for ghost triangles
    int32_t nb[3];  // nb[i]: triangle across the edge opposite v[i]
  };
  struct Pt {
    int32_t x, y;
  };
  std::vector<Pt> pt_;
  std::vector<int32_t> ext_;
  std::vector<uint32_t> vstamp_;   // per point: generation of the fan triangle starting there
  std::vector<int32_t> vfan_;      // per point: that fan triangle
  int32_t ghost_fan_ = -1;         // fan triangle starting at the ghost vertex
  std::vector<Tri> tri_;
  std::vector<uint8_t> alive_;
  std::vector<int32_t> free_;
  std::vector<uint32_t> stamp_;     // flood marks (2*gen: in hole, 2*gen+1: tested, not in hole)
  std::vector<int32_t> pending_;    // points seen before the first non-collinear triple
  std::vector<int32_t> stack_, hole_;
  struct Edge { int32_t a, b, out; };
  std::vector<Edge> bnd_;
  std::vector<int32_t> newt_;
  std::vector<uint32_t> key_, key2_;  // insertion-order keys (radix sort buffers)
  std::vector<int32_t> idx_, idx2_;
  mutable std::vector<int32_t> band_count_;
  uint32_t gen_ = 0;
  int32_t hint_ = -1;
  int32_t n_solid_ = 0;
  bool started_ = false;

  void order_points(const int32_t* u, const int32_t* v, int32_t n);
  int32_t alloc_tri();
  void free_tri(int32_t t);
  bool conflict(int32_t t, int32_t p) const;
  int32_t locate(int32_t p, bool* dup);
  void start(int32_t a, int32_t b, int32_t c);
  bool insert_point(int32_t p);
  int incircle_sos(int32_t a, int32_t b, int32_t c, int32_t d) const;
  int64_t orient(int32_t a, int32_t b, int32_t c) const;
  void rotate_top(int32_t& a, int32_t& b, int32_t& c) const;
  int64_t orient_pt(int32_t a, int32_t b, int64_t x, int64_t y) const;
};

}  // namespace sm
