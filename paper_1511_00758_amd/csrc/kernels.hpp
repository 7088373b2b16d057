// Launchers of the stereomesh device kernels (gfx950). Internal header: every
// launcher only enqueues work on `stream` and returns the launch status; argument
// checking happens in the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "stereomesh.h"

namespace sm {

// Arms a start/stop event pair for the next kernel launch of the calling thread (the
// events then bracket that kernel's execution); pending tells whether it is unused.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool launch_events_pending();
// Hands the armed pair to a launcher outside kernels.hip (and disarms it); false if none.
bool take_launch_events(hipEvent_t* start, hipEvent_t* stop);

// Marker values in sm_support::d for candidate slots (real disparities are >= 0).
constexpr float kPending = -1.0f;   // candidate waiting to be matched
constexpr float kRejected = -2.0f;  // empty slot / rejected candidate

struct CensusJob {
  const uint8_t* img;
  int32_t stride;
  uint64_t* census;
  uint8_t* omega;  // may be null
};

// Per-frame initialisation folded into the census launch (all fields optional).
struct CensusExtras {
  float* D_nan = nullptr;             // [H][W] set to NaN
  sm_support* grid_slots = nullptr;   // support-grid candidate slots (omega-filtered)
  int32_t step = 1, gw = 0;           // grid pitch, grid nodes per row
  int32_t* zero = nullptr;            // words set to 0
  int32_t n_zero = 0;
};

// Census words (+ Omega_I) of one or two images of the same size in one launch.
// When D_f / C_f / occ are non-null they are initialised (0, t_hi, 0) on the way.
hipError_t launch_census(const CensusJob* jobs, int n_jobs, int32_t W, int32_t H, int32_t cw,
                         int32_t ch, int32_t grad_thr, float* D_f, uint8_t* C_f, int32_t t_hi,
                         uint8_t* occ, const CensusExtras* extras, hipStream_t s, int32_t rows = 0);

// Candidate slots: grid nodes (omega-filtered) or an explicit (u, v) list.
hipError_t launch_grid_slots(const uint8_t* omega, int32_t W, int32_t H, int32_t step,
                             sm_support* slots, int32_t n, hipStream_t s);
hipError_t launch_list_slots(const int16_t* uv, int32_t n, sm_support* slots, hipStream_t s);

// FAST keypoints from spatial bins: the score of every pixel, then per bin the kept
// keypoints, per_bin slots per bin (bins row-major, raster order inside a bin). Output
// either as candidate slots (empty ones kRejected) or as (u, v) pairs (empty (-1, -1)),
// which launch_compact_uv packs in order.
hipError_t launch_fast_score(const uint8_t* img, int32_t stride, int32_t W, int32_t H, uint8_t* score,
                             hipStream_t s);
hipError_t launch_fast_select(const uint8_t* score, int32_t W, int32_t H, const sm_params& p,
                              sm_support* slots, int16_t* uv, hipStream_t s);
hipError_t launch_compact_uv(int16_t* uv, int32_t n, int32_t* n_out, hipStream_t s);

// Epipolar matching with left-right check of every pending slot, in place.
// Lanes per candidate of the matcher for a W x H frame with these parameters (16, 32 or
// 64: the sm_autotune choice, else 64), the waves that n candidates take, and the launch
// with an explicit choice (launch_match uses match_lanes_for).
int32_t match_lanes_for(int32_t W, int32_t H, const sm_params& p);
int32_t match_units(int32_t n, int32_t lanes);
hipError_t launch_match_lanes(const uint64_t* cL, const uint64_t* cR, int32_t W, int32_t H, const sm_params& p,
                              sm_support* slots, int32_t n, int32_t lanes, hipStream_t s);
hipError_t launch_match(const uint64_t* cL, const uint64_t* cR, int32_t W, int32_t H,
                        const sm_params& p, sm_support* slots, int32_t n, hipStream_t s);

// Counts kept on the device (the words of a frame's mesh status, mesh.hpp): the triangles
// of the frame's current mesh and the supports it holds.
enum { kCountTris = 1, kCountSupports = 5 };

// Order-preserving in-place compaction of non-marker slots (and, when `occ` is
// non-null, whose pixel is not yet occupied; kept pixels are then marked). The count
// goes to n_out and, when non-null, also to header. With slot_off non-null the slots
// start *slot_off entries after `slots` (a count on the device) and the count also goes
// to the slot after the last one; nothing happens unless those n + 1 slots lie below
// slot_cap.
hipError_t launch_compact(sm_support* slots, int32_t n, int32_t* n_out, uint8_t* occ,
                          int32_t W, int32_t* header, hipStream_t s, const int32_t* slot_off = nullptr,
                          int32_t slot_cap = 0);

// Occupancy map of a support list (cleared first).
hipError_t launch_mark(const sm_support* S, int32_t n, uint8_t* occ, int32_t W, int32_t H,
                       hipStream_t s);

// D_it: NaN fill, then per-triangle plane + rasterisation.
hipError_t launch_interpolate(const sm_support* S, int32_t n_support, const sm_tri* T, int32_t n_tris,
                              int32_t W, int32_t H, float* D_it, hipStream_t s);

// Single-kernel pieces of the two launchers above (for per-kernel timing).
hipError_t launch_fill_nan(float* D, size_t n, hipStream_t s);
// With `counts` non-null, n_tris and n_support are upper bounds and the kernel reads the
// triangle and support counts from counts[kCountTris], counts[kCountSupports].
hipError_t launch_raster(const sm_support* S, int32_t n_support, const sm_tri* T, int32_t n_tris,
                         int32_t W, int32_t H, float* D_it, hipStream_t s, const int32_t* counts = nullptr);
hipError_t launch_validate_only(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega,
                                const float* D_it, int32_t W, int32_t H, const sm_params& p,
                                int32_t sz, uint8_t* C_it, float* D_f, uint8_t* C_f,
                                uint64_t* cell_g, uint64_t* cell_b, uint8_t* mask,
                                unsigned long long* n_valid, hipStream_t s);

// Launch shapes measured by sm_autotune, consulted before the built-in rules (a choice
// changes speed only: every shape gives the same outputs). Keys: the kernel, the frame
// size and, for validation, the occupancy cell size.
enum TuneKind { kTuneValidateWaves = 0, kTuneRasterBlocks = 1, kTuneMatchLanes = 2, kTuneCensusRows = 3 };
int32_t tuned_choice(int kind, int32_t W, int32_t H, int32_t sz);  // -1: none
void set_tuned_choice(int kind, int32_t W, int32_t H, int32_t sz, int32_t value);  // 0: clear
// Validation with a given block size in waves (1, 2, 4, 8 or 16) instead of the rule.
hipError_t launch_validate_nw(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega,
                              const float* D_it, int32_t W, int32_t H, const sm_params& p,
                              int32_t sz, uint8_t* C_it, float* D_f, uint8_t* C_f,
                              uint64_t* cell_g, uint64_t* cell_b, uint8_t* mask,
                              unsigned long long* n_valid, int nw, hipStream_t s);
// Rasterisation with device counts (launch_raster's counts form) on at most max_blocks
// workgroups.
hipError_t launch_raster_blocks(const sm_support* S, int32_t n_support, const sm_tri* T, int32_t n_tris,
                                int32_t W, int32_t H, float* D_it, hipStream_t s, const int32_t* counts,
                                int32_t max_blocks);

// Zero `bytes` bytes (a kernel, so the call is safe inside captured graphs).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// Cost evaluation + refinement; writes every cell key (+ final mask when non-null).
hipError_t launch_validate(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega,
                           const float* D_it, int32_t W, int32_t H, const sm_params& p,
                           int32_t sz, uint8_t* C_it, float* D_f, uint8_t* C_f, uint64_t* cell_g,
                           uint64_t* cell_b, uint8_t* mask, unsigned long long* n_valid,
                           hipStream_t s);

// Resampling fused with the re-match: confident supports of the cells at
// slots[0, cells), re-matched invalid pixels at slots[cells, 2 cells); pixels that occ
// (nullable: the occupancy of the current supports) marks leave their slot empty; with
// slot_off non-null the slots start *slot_off entries after `slots` (nothing happens unless
// the 2 cells + 1 slots lie below slot_cap).
hipError_t launch_resample(const uint64_t* cL, const uint64_t* cR, const uint64_t* cell_g,
                           const uint64_t* cell_b, const float* D_it, int32_t W, int32_t H, int32_t sz,
                           const sm_params& p, sm_support* slots, const uint8_t* occ, hipStream_t s,
                           const int32_t* slot_off = nullptr, int32_t slot_cap = 0);

// ---------------------------------------------------------------------------------
// Stage-batched solve of many frames: every stage is one launch over all frames. The
// batched kernels read per-frame arguments from a device array of BatchFrame and map
// their work units (blocks or waves) to frames through a prefix array `off` of n + 1
// entries (off[0] = 0, frame f owns units off[f] .. off[f+1]-1).
// ---------------------------------------------------------------------------------
struct BatchFrame {
  const uint8_t* L;
  const uint8_t* R;
  int32_t W, H, stride;
  sm_params p;
  uint64_t* cL;
  uint64_t* cR;
  uint8_t* omega;
  uint8_t* occ;
  float* D_it;
  uint64_t* cell_g;
  uint64_t* cell_b;
  sm_support* S;
  int32_t* counters;
  unsigned long long* n_valid;
  float* D_f;
  uint8_t* C_f;
  uint8_t* mask;
  int32_t n_grid, gw;        // grid candidate slots, grid nodes per row
  int32_t match_lanes;       // lanes per candidate of the matcher (match_lanes_for)
  int32_t census_rows;       // rows of a census tile (census_rows_for)
  // state of the current iteration, rewritten before its launches
  const sm_tri* T;
  int32_t n_T, n_S, sz, last;  // last: this iteration writes the mask
  sm_support* region;          // resampling output (2 * cells slots + one header slot)
  int32_t region_n;            // 2 * cells, 0 when the frame does not resample
  sm_support* pack;            // host-bound staging: header slot + up to pack_cap supports
  int32_t pack_cap;
  // counts kept on the device (the frame's mesh status, kCountTris / kCountSupports): when
  // non-null the raster takes n_T and n_S from it (its units stride over the triangles) and
  // the resampling region starts at S + counts[kCountSupports]
  const int32_t* counts;
  int32_t S_cap, T_cap;
};

// census tiles of a W x H image at `rows` rows per tile, and the rows a W x H image with a
// cw x ch window uses (the sm_autotune choice, else 8 in a single frame's launch and 16 in
// the batched census)
int32_t census_tiles(int32_t W, int32_t H, int32_t rows);
int32_t census_rows_for(int32_t W, int32_t H, int32_t cw, int32_t ch, bool batched);
int32_t validate_blocks(int32_t W, int32_t H, int32_t sz, int nw);
// smallest block size (waves) whose batched grid still holds enough waves
int validate_pick_nw(int64_t (*waves)(int nw, void* ctx), void* ctx);

hipError_t launch_batch_census(const BatchFrame* F, const int32_t* off, int32_t n, int32_t total, int rx, int ry,
                               hipStream_t s);
hipError_t launch_batch_match(const BatchFrame* F, const int32_t* off, int32_t n, int32_t total, hipStream_t s);
// mode 0: the grid slots S[0, n_grid); mode 1: the resampling region. One workgroup per frame.
hipError_t launch_batch_compact(const BatchFrame* F, int32_t n, int mode, hipStream_t s);
hipError_t launch_batch_pack(const BatchFrame* F, int32_t n, int mode, hipStream_t s);
hipError_t launch_batch_raster(const BatchFrame* F, const int32_t* off, int32_t n, int32_t total, hipStream_t s);
hipError_t launch_batch_validate(const BatchFrame* F, const int32_t* off, int32_t n, int32_t total, int nw,
                                 hipStream_t s);
hipError_t launch_batch_rematch(const BatchFrame* F, const int32_t* off, int32_t n, int32_t total, hipStream_t s);

}  // namespace sm
