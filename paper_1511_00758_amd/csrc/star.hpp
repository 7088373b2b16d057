// Device Delaunay triangulation by per-point stars (Sec. III-A, the mesh G(S) of Alg. 1;
// the steps are in mesh_star.hpp): launchers and per-frame arrays. Internal header;
// launchers only enqueue work on `stream`.
//
// Each tessellation of a frame is two launches: a preparation kernel (one 1024-thread
// workgroup per frame: the new supports' compaction, packed coordinates, a bucket grid of
// 16 x 16 px cells, the smallest and largest u of every pixel row, the frame's status
// words) and the star kernel (one wavefront per support for one frame, one 16-lane group
// per support for the batched launch; each writes the triangles of its star in which it
// is the first vertex, and, when the job names D_it, rasterises them into it). Nothing is
// kept from one tessellation to the next besides the supports.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mesh_star.hpp"
#include "stereomesh.h"

namespace sm {

// Status words of a frame's meshes (device, kMeshStatusWords x int32):
//   [1] triangles of the current tessellation written to T
//   [2] error code (0 = ok, else the star steps' code, mesh_star.hpp: the caller redoes the
//       frame's meshes on the host; later tessellations keep the code and write nothing)
//   [4] new supports of the current tessellation
//   [5] supports so far
//   [6] tessellations done
//   [8 + 2k], [9 + 2k] supports and triangles of tessellation k (k < 8)
// Words 0, 3 and 7 stay zero. The star kernel counts the triangles in kMeshTris (and in the
// copy) with atomics; a tessellation's log entry gets its supports from the preparation and
// its triangle count from the next preparation, or, for a frame's last tessellation, from
// kMeshTris when the caller reads the words back (star_log_tris).
enum { kMeshTris = 1, kMeshErr = 2, kMeshNew = 4, kMeshSupports = 5, kMeshTess = 6, kMeshLog = 8, kMeshStatusWords = 32 };
inline int32_t star_log_tris(const int32_t* words, int k, int n_tess) {
  return k == n_tess - 1 ? words[kMeshTris] : words[kMeshLog + 2 * k + 1];
}

struct StarWork {  // per-frame arrays
  int32_t* uv;          // [S_cap] packed coordinates u | v << 16
  int32_t* cell_start;  // [cells + 1]
  int32_t* cell_cur;    // [cells] fill cursors
  star::CellEntry* cell_e;  // [S_cap] the supports (id, packed coordinates) ordered by cell
  star::RowExt* rows;       // [H] smallest and largest u of every pixel row and their supports
  int32_t* row_min;         // [H] the preparation's counters when they are not in LDS
  int32_t* row_max;         // [H]
  int32_t gw, gh, S_cap;
};

size_t star_work_bytes(int32_t W, int32_t H, int32_t S_cap);
StarWork star_work_at(void* base, int32_t W, int32_t H, int32_t S_cap);

struct StarJob {
  sm_support* S;
  int32_t first;            // 1: the frame's first tessellation (its supports start at S[0]);
                            // 0: the new supports start at status[kMeshSupports]
  int32_t compact_n;        // > 0: first compact the slots S[p0, p0 + compact_n) in place
  uint8_t* occ;             //   (with occupancy occ [H][W]), their count to *compact_count and
  int32_t* compact_count;   //   to the slot after them
  const int32_t* n_new;     // compact_n == 0: device count of the new supports (NULL: none)
  int32_t* status;          // device [kMeshStatusWords], read (unless first) and written
  int32_t* status_copy;     // nullable: a copy of words 0..7 and of the log
  sm_tri* T;
  int32_t T_cap;
  int32_t W, H;
  int32_t blocks;           // star-kernel workgroups of this frame (star_blocks / star_blocks_many)
  StarWork w;
  float* D = nullptr;       // nullable: D_it [H][W]; the star kernels then rasterise every
                            // triangle they write into it
};

// Star-kernel workgroups for a frame of at most S_cap supports: of launch_star (four stars
// per workgroup, a wavefront each) and of launch_star_many (the same, or sixteen stars, a
// 16-lane group each, when `grouped`); whether a batch whose frames start from
// `candidates` support candidates in total takes the grouped kernel.
int32_t star_blocks(int32_t S_cap);
int32_t star_blocks_many(int32_t S_cap, bool grouped);
bool star_grouped(int64_t candidates);

hipError_t launch_star(const StarJob& job, hipStream_t s);
// the jobs of a device array: preparation, one workgroup per job, then the star kernel over
// every job's supports; offs [n + 1] holds the prefix sums of the jobs' `blocks`; lds: every
// job's frame passes prep_in_lds
hipError_t launch_star_many(const StarJob* jobs, const int32_t* offs, int32_t n, int32_t total_blocks, bool lds,
                            bool grouped, hipStream_t s);
// whether the preparation of a W x H frame keeps its counts in LDS
bool prep_in_lds(int32_t W, int32_t H);

}  // namespace sm
