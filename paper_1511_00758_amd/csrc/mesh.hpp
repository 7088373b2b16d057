// Device mesh insertion: launchers and the per-frame mesh state. Internal header;
// launchers only enqueue work on `stream`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "stereomesh.h"

namespace sm {

// Device Delaunay insertion (mesh.hip): the supports S[p0, p0 + n_new) join the mesh of
// the frame, whose records (the host triangulation's form, vertices as support indices,
// ghosts included) stay in the MeshWork arrays from one tessellation to the next; the
// solid triangles of the result go to T, top vertex first. One 1024-thread workgroup per
// job.
struct MeshWork {  // per-frame arrays: records [cap], new points [pcap], coordinates [S_cap]
  int32_t *tv, *tnb, *own, *kids, *dead, *fk, *fs, *fj, *work0, *work1;
  uint64_t *vote, *fkey;
  int32_t *ploc, *pk, *psib, *pend0, *pend1;
  uint64_t* pkey;
  int32_t* uv;    // packed coordinates when they do not fit in LDS
  int32_t* hint;  // location hints, one per 16 x 16 px cell
  // first mesh built on the device: rows, row of each support, strips, hull ghosts per
  // vertex, chain stacks, edge hash table (hcap entries, a power of two)
  int32_t *row_first, *row_of, *strip_base, *gh_start, *gh_end, *stack;
  uint64_t* hkeys;
  int32_t* hvals;
  int32_t cap, pcap, S_cap, hcap;
};

// Mesh status words (device, kMeshStatusWords x int32), the frame's record of its mesh:
//   [0] records in use
//   [1] triangles written to T
//   [2] error code (0 = ok, else the records are unusable and the caller triangulates on
//       the host; a later insertion keeps the code and writes no triangles)
//   [3] rounds used so far by the frame (keys of later rounds must bid lower)
//   [4] number of new supports read from n_new
//   [5] supports in the mesh so far (p0 + new supports)
//   [6] tessellations done
//   [7] a live solid record (where a point location starts when its cell has no hint)
//   [8 + 2k], [9 + 2k] supports and triangles after tessellation k (k < 8)
enum { kMeshRecords = 0, kMeshTris = 1, kMeshErr = 2, kMeshRounds = 3, kMeshNew = 4, kMeshSupports = 5,
       kMeshTess = 6, kMeshAny = 7, kMeshLog = 8, kMeshStatusWords = 32 };
// error code of a first mesh that cannot exist (fewer than two rows of supports: no
// triangle, or all supports collinear); the host path handles that frame
constexpr int32_t kMeshErrNoMesh = 10;

struct MeshJob {
  const sm_support* S;
  int32_t start;            // 1: build the frame's first mesh from S[0, *n_new) (sorted by
                            //    raster position, p0 = 0), then flip it to Delaunay
  int32_t p0;               // first new support; < 0: status[kMeshSupports] (counted on the device)
  const int32_t* n_new;     // device count of new supports; with p0 < 0 it sits at
  int32_t n_new_slot;       //   S[p0 + n_new_slot] instead
  int32_t last;             // 1: no tessellation follows (the output writes no location hints)
  int32_t compact_n;        // > 0: first compact the slots S[p0, p0 + compact_n) in place (the
  uint8_t* occ;             //   supports' compaction, kernels.hpp, with occupancy occ [H][W]),
  int32_t* compact_count;   //   their count to *compact_count and to the slot after them
  const int32_t* init_tv;   // init_n > 0: the frame's first mesh (records in host form) to
  const int32_t* init_tnb;  //   start from, vertices < p0; may alias w.tv / w.tnb
  int32_t init_n;
  int32_t* status;          // device [kMeshStatusWords], read (unless start or init_n > 0) and written
  int32_t* status_copy;     // nullable: device [kMeshStatusWords], a copy of words 0..7 and of
                            //   the log entries this kernel writes
  sm_tri* T;
  int32_t T_cap;
  int32_t W, H;
  MeshWork w;
};

// Record capacity for a frame of at most S_cap supports (about 5 records per support are
// used; a frame that needs more falls back to the host), bytes of its MeshWork, and the
// carving of a 256-byte aligned block of that size.
int32_t mesh_work_cap(int32_t S_cap);
size_t mesh_work_bytes(int32_t W, int32_t H, int32_t S_cap, int32_t pcap);
MeshWork mesh_work_at(void* base, int32_t W, int32_t H, int32_t S_cap, int32_t pcap);

hipError_t launch_mesh_insert(const MeshJob& job, hipStream_t s);
// one workgroup per job of the device array `jobs`
hipError_t launch_mesh_insert_many(const MeshJob* jobs, int32_t n, hipStream_t s);

}  // namespace sm
