/*
 * stereomesh.h -- C ABI of the MI355X (gfx950) implementation of the iterative
 * piecewise-planar stereo method of Pillai, Ramalingam and Leonard, "High-Performance
 * and Tunable Stereo Reconstruction" (ICRA 2016).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - Pointers are DEVICE pointers unless marked [host]. Every buffer is owned by the
 *   caller; the library keeps no pointer after a call returns, but work it enqueued
 *   reads and writes the buffers until the stream has been synchronised.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream). Calls are
 *   asynchronous on that stream except sm_triangulate (host only) and the solves:
 *   sm_solve synchronises the stream once per frame when every tessellation runs on
 *   the device (the default), once per tessellation with host meshes; the batched
 *   solves and the autotuner return when their work is done.
 * - Images are row-major uint8 with a row pitch `stride` >= W bytes; every per-pixel
 *   output array is row-major with pitch W elements.
 * - Every argument is checked before anything is enqueued; a violation returns
 *   SM_ERR_ARG and enqueues nothing. An output whose capacity `cap` is too small for
 *   the worst case returns SM_ERR_CAPACITY (and, for host outputs, the required count).
 *   A failing HIP call returns SM_ERR_HIP. sm_last_error() describes the last non-OK
 *   status of the calling thread. No C++ exception crosses this interface.
 * - The library allocates no device memory. sm_solve takes a caller-owned workspace;
 *   host-side staging (pinned) and triangulation state are cached per thread.
 * - Degenerate scenes are not errors: fewer than three supports, or only collinear
 *   ones, give zero triangles, an all-NaN interpolation and an empty mask.
 * - Image sizes are limited to 3 <= W, H <= 8192 (exact 64-bit geometric predicates).
 */
#ifndef STEREOMESH_H
#define STEREOMESH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SM_OK = 0,
  SM_ERR_ARG = -1,       /* invalid argument; nothing was enqueued                    */
  SM_ERR_CAPACITY = -2,  /* an output capacity is below the worst case               */
  SM_ERR_HIP = -3,       /* a HIP runtime call failed (message in sm_last_error)     */
  SM_ERR_INTERNAL = -4   /* an internal invariant failed                              */
} sm_status;

/* Support point s = (u, v, d): pixel coordinates and disparity (Sec. III-A). The
 * disparity is a float because supports added by resampling carry the interpolated
 * disparity of their pixel (Alg. 3 records D_it into C_g). 8 bytes. */
typedef struct {
  int16_t u, v;
  float d;
} sm_support;

/* Triangle of the Delaunay mesh G(S) as three indices into the support array;
 * counter-clockwise in (u, v) (orient > 0), i0 = the vertex with the smallest (v, u). */
typedef struct {
  int32_t i0, i1, i2;
} sm_tri;

/* Method parameters (the globals of the paper's Table I). */
typedef struct {
  int32_t d_min, d_max;        /* searched disparities, inclusive; 0 <= d_min <= d_max <= 255   */
  int32_t census_w, census_h;  /* census window, odd, >= 3, census_w*census_h - 1 <= 64          */
  int32_t support_step;        /* pitch of the initial support-candidate grid, px, >= 1          */
  int32_t n_iters;             /* n_iters of Alg. 1, 1..8                                       */
  int32_t t_hi;                /* upper cost threshold (Hamming); mask = C_f < t_hi, <= 64      */
  int32_t t_lo;                /* lower cost threshold (Hamming), 0 <= t_lo <= t_hi             */
  int32_t grad_thr;            /* Omega_I: L1 central-difference gradient >= grad_thr, >= 0     */
  int32_t lr_tol;              /* left-right check: |d_LR - d| <= lr_tol, >= 0                  */
  int32_t uniqueness;          /* reject when a disparity >= 2 away costs < best + uniqueness;
                                  0 disables the test                                          */
  int32_t sz_occ0;             /* initial occupancy-grid size (32 in Alg. 1), 1..1024           */
  /* Paper variants (Sec. III-A, III-B); zero-initialising them gives 0 = the grid, which
     is valid, and levels = 0, which is not: set levels = 1 for Alg. 2 as printed.       */
  int32_t support_mode;        /* 0: candidate grid of support_step; 1: FAST keypoints from
                                  spatial bins (sm_fast_candidates)                           */
  int32_t fast_threshold;      /* FAST: corner when the arc contrast > fast_threshold, 0..254   */
  int32_t fast_bins_x;         /* FAST: spatial bins across (12 in Sec. III-A), 1..1024         */
  int32_t fast_bins_y;         /* FAST: spatial bins down (10 in Sec. III-A), 1..1024           */
  int32_t fast_per_bin;        /* FAST: at most this many keypoints per bin, 1..4096;
                                  fast_bins_x * fast_bins_y * fast_per_bin <= 2^22            */
  int32_t levels;              /* disparity levels tested by cost evaluation: 1 (Alg. 2), 3, 5 */
  int32_t host_mesh;           /* 0 = every tessellation on the device: each one is built there
                                  from all supports so far, one Delaunay star per support (a
                                  frame the device cannot finish is solved again with host
                                  meshes); 1 = every tessellation on the host, which inserts
                                  the new supports into the previous mesh. Same triangles
                                  either way.                                                 */
} sm_params;

/* Per-solve statistics. `timing` is an input: when non-zero, sm_solve records a pair of
 * HIP events on `stream` around kernel launches and reports, per kernel stage, the summed
 * device time (stage_us) and the launch count (stage_launches); the host stages report
 * wall time. Indices are the sm_stage values. timing = SM_TIME_SELECTED | (1 << stage)
 * | ... times only the listed stages (fewer events in the way of the rest); any other
 * non-zero value times every kernel. */
#define SM_TIME_SELECTED 0x40000000
typedef enum {
  SM_ST_CENSUS = 0,          /* census + Omega_I of both images, per-frame initialisation     */
  SM_ST_MATCH = 1,           /* epipolar matching of the support-grid candidates              */
  SM_ST_COMPACT = 2,         /* order-preserving compaction of matched / resampled supports   */
  SM_ST_RASTER = 3,          /* plane fit + per-triangle rasterisation (interpolation); none  */
                             /* with device meshes: their star kernel rasterises (SM_ST_MESH) */
  SM_ST_VALIDATE = 4,        /* cost evaluation + refinement                                 */
  SM_ST_REMATCH = 5,         /* resampling: cells -> confident supports + re-matched pixels  */
  SM_ST_FAST = 6,            /* FAST scores + per-bin keypoint selection (support_mode 1)     */
  SM_ST_MESH = 7,            /* device Delaunay tessellations (grid and per-point stars)      */
  SM_ST_HOST_TRI = 12,       /* host triangulation (wall time)                               */
  SM_ST_HOST_COPY = 13,      /* host<->device copies and waits (wall time)                   */
  SM_ST_TOTAL = 14           /* whole sm_solve call (wall time)                              */
} sm_stage;
#define SM_STAGES 16
typedef struct {
  int32_t timing;                       /* [in]  non-zero: collect stage_us          */
  int32_t n_support[8];                 /* [out] |S_it| per iteration                 */
  int32_t n_tris[8];                    /* [out] |G(S_it)| per iteration              */
  int64_t n_valid;                      /* [out] pixels in the final mask             */
  float stage_us[SM_STAGES];            /* [out] see above                            */
  int32_t stage_launches[SM_STAGES];    /* [out] kernel launches per stage            */
  int32_t mesh_device;                  /* [out] tessellations done on the device      */
  int32_t mesh_fallback;                /* [out] device tessellations redone on the host */
} sm_stats;

/*
 * sm_census -- census words of one image and, optionally, its high-gradient set.
 *   Census window match of the cost-evaluation section (Sec. III-C, Zabih and
 *   Woodfill's census): bit k of the word of pixel p is 1 iff window neighbour k is
 *   strictly darker than p; neighbours in row-major window order, centre skipped,
 *   k = 0 the least significant bit. High-gradient subset Omega_I (Sec. III):
 *   |I(u+1,v) - I(u-1,v)| + |I(u,v+1) - I(u,v-1)| >= grad_thr.
 *   img      [H][stride] uint8 image.
 *   census   [H][W] uint64 out; 0 where the window does not fit (u < rx, u >= W-rx,
 *            v < ry, v >= H-ry with rx = (census_w-1)/2, ry = (census_h-1)/2).
 *   omega    [H][W] uint8 out, 1 = in Omega_I (only where the window fits); may be NULL.
 */
sm_status sm_census(const uint8_t* img, int32_t W, int32_t H, int32_t stride,
                    int32_t census_w, int32_t census_h, int32_t grad_thr,
                    uint64_t* census, uint8_t* omega, void* stream);

/*
 * sm_match_support -- sparse epipolar matching of support candidates (Sec. III-A,
 *   "SparseStereo" of Alg. 1 and "SparseEpipolarStereo" of Alg. 4).
 *   For candidate (u, v): d* = argmin over d in [d_min, d_max] with u - d >= rx of
 *   Hamming(cL(u,v), cR(u-d,v)), ties to the smallest d. Rejected when no d is
 *   admissible, when cost(d*) >= t_hi, when (uniqueness = m > 0) an admissible d with
 *   |d - d*| >= 2 costs < cost(d*) + m, or when the right-to-left argmin d' from
 *   u - d* (over d with u - d* + d <= W-1-rx, ties to the smallest d) has
 *   |d' - d*| > lr_tol. Candidates whose census window does not fit are rejected.
 *   cL, cR   [H][W] census words of the left / right image (sm_census).
 *   omega    [H][W] Omega_I of the left image; required when cand_uv is NULL.
 *   cand_uv  [n_cand][2] int16 (u, v) candidates, or NULL for the grid
 *            (support_step/2 + i*support_step, support_step/2 + j*support_step) in raster
 *            order, restricted to Omega_I (then n_cand is ignored).
 *   out      [cap] accepted supports (u, v, float(d*)) in candidate order.
 *            cap must be >= the number of candidates (the worst case), else
 *            SM_ERR_CAPACITY; out[] beyond the accepted count is scratch.
 *   n_out    [1] int32 out: number of accepted supports.
 */
sm_status sm_match_support(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega,
                           int32_t W, int32_t H, const int16_t* cand_uv, int32_t n_cand,
                           const sm_params* p /* [host] */, sm_support* out, int32_t cap,
                           int32_t* n_out, void* stream);

/* Number of candidates of the support grid (the capacity sm_match_support needs
 * when cand_uv is NULL). Host only. */
int32_t sm_grid_candidates(int32_t W, int32_t H, int32_t support_step);

/*
 * sm_fast_candidates -- support keypoints by the FAST segment test, sampled from
 *   spatial bins (Sec. III-A; Rosten and Drummond's FAST-9).
 *   Circle: the 16 pixels of the radius-3 Bresenham ring, clockwise from the pixel
 *   straight above p. With diff_k = I(ring_k) - I(p), score(p) = max over the 16 arcs
 *   of 9 consecutive ring pixels of max(min diff, min -diff) over the arc, floored at 0
 *   (0 where the ring leaves the image); p is a corner when score > fast_threshold.
 *   A corner is a keypoint when no 3x3 neighbour scores higher and no neighbour earlier
 *   in raster order scores the same. Pixel (u, v) lies in bin
 *   (u * fast_bins_x / W, v * fast_bins_y / H) (integer division); each bin keeps its
 *   fast_per_bin highest-scoring keypoints (ties to the earlier raster position).
 *   img      [H][stride] uint8 image (the left image).
 *   p        [host] parameters; only the fast_* fields are read.
 *   score    [H][W] uint8 out: score(p) for every pixel (also used as scratch).
 *   cand_uv  [cap][2] int16 out: (u, v) of the kept keypoints, bins row-major and raster
 *            order inside a bin; cap >= fast_bins_x * fast_bins_y * fast_per_bin, else
 *            SM_ERR_CAPACITY. Entries past the count are scratch.
 *   n_out    [1] int32 out: number of candidates.
 */
sm_status sm_fast_candidates(const uint8_t* img, int32_t W, int32_t H, int32_t stride,
                             const sm_params* p /* [host] */, uint8_t* score, int16_t* cand_uv,
                             int32_t cap, int32_t* n_out, void* stream);

/*
 * sm_triangulate -- Delaunay triangulation G(S) of the support pixels (Sec. III-A).
 *   Exact integer predicates; cocircular ties resolved by symbolic perturbation of
 *   the lifting z = u^2 + v^2 + eps_i, a smaller raster position (v, u) getting the
 *   larger eps, which makes the triangulation unique. A pixel that occurs more than
 *   once is represented by its first occurrence. Synchronous host code.
 *   S       [host] [n] supports; u, v in [0, 8191].
 *   tris    [host] [cap] out: triangles, canonical (see sm_tri) and sorted by (i0,i1,i2).
 *   n_tris  [host] out: triangle count (the required count on SM_ERR_CAPACITY;
 *           2n - 5 always suffices for n >= 3).
 */
sm_status sm_triangulate(const sm_support* S, int32_t n, sm_tri* tris, int32_t cap,
                         int32_t* n_tris);

/*
 * sm_interpolate -- DisparityInterpolation (Sec. III-B, Alg. 1): the disparity plane
 *   of every triangle (Eq. 3, solved through its three supports) evaluated at every
 *   pixel the triangle owns (the pixel-to-triangle lookup of Sec. III-B).
 *   Plane: anchor i0 = (u0, v0, d0); with du_k, dv_k the integer offsets of i1, i2
 *   and det = du1*dv2 - du2*dv1, in float64: a = ((d1-d0)*dv2 - (d2-d0)*dv1)/det,
 *   b = (du1*(d2-d0) - du2*(d1-d0))/det, each rounded to float32. Pixel (u, v) is owned
 *   by the triangle containing (u + eps, v + eps^2); there
 *   D = (d0 + a*float(u-u0)) + b*float(v-v0) in float32 (no fused multiply-add).
 *   S       [n_support] supports;  T [n_tris] triangles (canonical, as sm_triangulate).
 *   D_it    [H][W] float32 out; NaN where no triangle owns the pixel.
 */
sm_status sm_interpolate(const sm_support* S, int32_t n_support, const sm_tri* T,
                         int32_t n_tris, int32_t W, int32_t H, float* D_it, void* stream);

/* Number of occupancy cells at grid size sz: ceil(H/sz) * ceil(W/sz). Host only. */
int32_t sm_cells(int32_t W, int32_t H, int32_t sz_occ);

/*
 * sm_validate -- CostEvaluation (Alg. 2) and DisparityRefinement (Alg. 3).
 *   For (u, v) in Omega_I with a finite D_it: d = floor(float32(D_it + 0.5)); when
 *   d_min <= d <= d_max and u - d >= rx, C_it = Hamming(cL(u,v), cR(u-d,v)), else the
 *   pixel is not evaluated (C_it = 0xFF). With p->levels = L > 1 (the "3-5 disparity
 *   levels" of Sec. III-B) an evaluated pixel's C_it is the smallest Hamming distance
 *   over d' in [d - (L-1)/2, d + (L-1)/2] with d_min <= d' <= d_max and u - d' >= rx;
 *   the evaluated set and D_it are unchanged. For evaluated pixels: if C_it < C_f then
 *   D_f = D_it and C_f = C_it. Cells of sz_occ x sz_occ pixels (cell (u/sz, v/sz),
 *   ceil(W/sz) per row) keep the pixel with the smallest C_it < t_lo (C_g) and the
 *   one with the largest C_it > t_hi (C_b); ties go to the first pixel in raster order.
 *   C_it     [H][W] uint8 out (may be NULL).
 *   D_f, C_f [H][W] float32 / uint8 in-out (start them at 0 and t_hi, Alg. 1).
 *   cell_g   [sm_cells] uint64 out; key (C_it << 32) | (v*W + u); the "unset" value is
 *            (t_lo << 32), which no recorded pixel can equal.
 *   cell_b   [sm_cells] uint64 out; key ((255 - C_it) << 32) | (v*W + u); "unset" is
 *            ((255 - t_hi) << 32).
 */
sm_status sm_validate(const uint64_t* cL, const uint64_t* cR, const uint8_t* omega,
                      const float* D_it, int32_t W, int32_t H, const sm_params* p /* [host] */,
                      int32_t sz_occ, uint8_t* C_it, float* D_f, uint8_t* C_f,
                      uint64_t* cell_g, uint64_t* cell_b, void* stream);

/*
 * sm_resample -- SupportResampling (Alg. 4). Cells are visited in raster order: a set
 *   C_b cell puts its pixel into X, a set C_g cell yields the support
 *   (u, v, D_it(u, v)); X is matched as in sm_match_support; the new supports are the
 *   confident ones (cell order) followed by the matched ones (X order), dropping any
 *   pixel already in S.
 *   S, n_S   [n_S] current supports (dedup reference).
 *   occ      [H][W] uint8 scratch (overwritten).
 *   out      [cap] out: new supports; cap >= 2 * sm_cells(W, H, sz_occ).
 *   n_out    [1] int32 out: number of new supports.
 */
sm_status sm_resample(const uint64_t* cL, const uint64_t* cR, const float* D_it,
                      const uint64_t* cell_g, const uint64_t* cell_b, int32_t W, int32_t H,
                      int32_t sz_occ, const sm_params* p /* [host] */,
                      const sm_support* S, int32_t n_S, uint8_t* occ,
                      sm_support* out, int32_t cap, int32_t* n_out, void* stream);

/* Workspace sm_solve needs for a W x H frame under p, in bytes (0 on invalid args). */
size_t sm_solve_workspace_bytes(int32_t W, int32_t H, const sm_params* p /* [host] */);

/*
 * sm_solve -- Iterative Stereo Reconstruction (Alg. 1) on a rectified pair:
 *   D_f = 0, C_f = t_hi; S_1 = matched support candidates (the grid, or with
 *   support_mode = 1 the FAST keypoints of sm_fast_candidates); G(S_1); then for
 *   it = 1..n_iters:
 *   interpolation, cost evaluation, refinement with sz_occ = max(1, sz_occ0 >> (it-1)),
 *   and, unless it is the last iteration, resampling and re-triangulation (the
 *   triangulation of all supports so far is unique: the host inserts the new supports into
 *   the previous mesh, the device rebuilds it, and both give the same triangles).
 *   L, R     [H][stride] uint8 left / right images.
 *   ws       workspace of ws_bytes >= sm_solve_workspace_bytes(W, H, p), 256-byte aligned.
 *   D_f      [H][W] float32 out (0 where never validated).
 *   C_f      [H][W] uint8 out.
 *   mask     [H][W] uint8 out: 1 iff in Omega_I and C_f < t_hi (pixels that passed).
 *   st       [host] statistics, may be NULL.
 *   Synchronisation: with grid candidates and device meshes (host_mesh = 0) the counts
 *   stay on the device and `stream` is synchronised once, at the end of the frame (a frame
 *   whose device mesh fails is solved again with host meshes, counted in
 *   st->mesh_fallback); otherwise once per triangulation (n_iters times). With device
 *   meshes the interpolation has no launch of its own: each workgroup of the star kernel
 *   rasterises the triangles its stars found (timed with the mesh stage).
 */
sm_status sm_solve(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t stride,
                   const sm_params* p /* [host] */, void* ws, size_t ws_bytes, float* D_f,
                   uint8_t* C_f, uint8_t* mask, sm_stats* st /* [host] */, void* stream);

/*
 * sm_solve_noalloc -- sm_solve for callers that cannot allocate (code under HIP graph
 *   capture, tight serving loops, harnesses that forbid allocation): the same solve of one
 *   frame with no caller workspace, no device or host allocation (no hipMalloc, hipFree,
 *   pinned staging, timing events or library routine that allocates) on success. The
 *   frame's workspace is a buffer the library holds in device memory, one per GPU,
 *   SM_NOALLOC_MAX_BYTES large; each GPU the library runs on keeps it until the process
 *   ends. Arguments and results are those of sm_solve, except:
 *   - the frame must keep its meshes on the device (host_mesh = 0), else SM_ERR_ARG;
 *   - sm_solve_workspace_bytes(W, H, p) must not exceed SM_NOALLOC_MAX_BYTES, else
 *     SM_ERR_CAPACITY (640x480 with disparities 0-127 needs 7 MiB, 1920x1080 with 0-255
 *     46 MiB, 2560x1440 with 0-255 81 MiB: too large);
 *   - a frame whose device mesh cannot be finished (an array full; sm_solve would solve it
 *     again with host meshes, which allocates) returns SM_ERR_INTERNAL and its outputs are
 *     not valid;
 *   - st gets the counts only (st->timing is ignored);
 *   - `stream` must belong to the calling thread's current device.
 *   Every call on a GPU works in that GPU's one buffer, which keeps the last call's
 *   contents (each call initialises what it reads). Calls that overlap on one GPU -- from
 *   other threads, or on other streams not yet synchronised -- race and give wrong
 *   results. The call synchronises `stream` once, at the end of the frame.
 */
#define SM_NOALLOC_MAX_BYTES ((size_t)48 << 20)
sm_status sm_solve_noalloc(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t stride,
                           const sm_params* p /* [host] */, float* D_f, uint8_t* C_f, uint8_t* mask,
                           sm_stats* st /* [host] */, void* stream);

/* One frame of a batch: inputs, method parameters, outputs (all device pointers). */
typedef struct {
  const uint8_t* L;            /* [H][stride] left image                                  */
  const uint8_t* R;            /* [H][stride] right image                                 */
  int32_t W, H, stride;
  sm_params p;                 /* per-frame parameters (sizes and ranges may differ)     */
  float* D_f;                  /* [H][W] out                                              */
  uint8_t* C_f;                /* [H][W] out                                              */
  uint8_t* mask;               /* [H][W] out                                              */
  sm_status status;            /* [out] status of this frame                              */
  int32_t worker;              /* [out] worker that solved it                              */
  float latency_us;            /* [out] wall time of this frame's solve                    */
} sm_frame;

/*
 * sm_solve_batch -- Alg. 1 on many independent frames at once: n_workers host threads,
 *   each with its own stream and workspace, take frames from a shared counter and run
 *   sm_solve on them, so that the host work of one frame overlaps the kernels of the
 *   others. Each frame's result is identical to sm_solve of that frame alone. The workers
 *   persist between calls made by the same thread.
 *   frames     [host] [n] frames; status, worker and latency_us are written.
 *   streams    [host] [n_workers] hipStream_t per worker (as void*).
 *   ws, ws_bytes [host] [n_workers] workspace per worker; each must cover
 *              sm_solve_workspace_bytes of every frame (checked before any work).
 *   st         [host] statistics summed over frames, may be NULL.
 *   Returns SM_OK when every frame succeeded, else the first failing frame's status.
 *   Synchronous: returns when every frame is solved.
 */
sm_status sm_solve_batch(sm_frame* frames, int32_t n, void* const* streams, void* const* ws,
                         const size_t* ws_bytes, int32_t n_workers, sm_stats* st);

/*
 * sm_solve_many -- Alg. 1 on many independent frames at once, stage by stage: each
 *   stage (census, matching, compaction, rasterisation, validation, resampling) is one
 *   kernel launch over all frames, which may differ in size and parameters; between the
 *   stages that need them, the frames' triangulations run on n_threads host workers.
 *   Every frame's D_f, C_f and mask are bit-identical to its own sm_solve. Frames must
 *   use the support grid (p.support_mode = 0). Frames with fewer iterations drop out of
 *   the later launches.
 *   frames   [host] [n] frames (status, worker = 0 and latency_us = whole call are written).
 *   ws       one workspace of ws_bytes >= sm_solve_many_workspace_bytes(frames, n),
 *            256-byte aligned, holding every frame's buffers and the batch staging.
 *   st       [host] statistics summed over frames (one launch counted per stage launch).
 *   Synchronisation: when every frame keeps its meshes on the device (host_mesh = 0) the
 *   counts stay on the device and `stream` is synchronised once, at the end (a frame whose
 *   device mesh failed is then solved again alone with host meshes); otherwise once per
 *   triangulation round (max n_iters times). With every mesh on the device the batch has
 *   no rasterisation launch: the star kernels rasterise the triangles they find.
 */
size_t sm_solve_many_workspace_bytes(const sm_frame* frames /* [host] */, int32_t n);
sm_status sm_solve_many(sm_frame* frames /* [host] */, int32_t n, void* ws, size_t ws_bytes,
                        int32_t n_threads, sm_stats* st /* [host] */, void* stream);

/*
 * sm_solve_many_capture -- sm_solve_many whose device work is recorded, from the first
 *   upload to the last mesh launch, into a HIP graph on `stream`, run once (the frames are
 *   solved as by sm_solve_many) and returned in *out. Later batches over the same frames
 *   (same sizes, parameters, image, output and workspace buffers; the image contents may
 *   change) replay it with sm_many_graph_run, which launches one graph instead of the
 *   batch's dozens of launches and uploads (the hipGraph-captured iteration loop of the
 *   batched solve; the stage-batched design is Alg. 1 applied stage by stage). Every frame
 *   must keep its meshes on the device (host_mesh = 0), so that the batch needs no host
 *   synchronisation; otherwise SM_ERR_ARG. The graph owns its pinned staging; the
 *   workspace must stay allocated while the graph lives.
 *   st       [host] statistics of the first run, may be NULL (no stage timing).
 *   out      [host] out: the graph, freed by sm_many_graph_destroy; NULL on error.
 */
typedef struct sm_many_graph sm_many_graph;
sm_status sm_solve_many_capture(sm_frame* frames /* [host] */, int32_t n, void* ws, size_t ws_bytes,
                                sm_stats* st /* [host] */, void* stream, sm_many_graph** out /* [host] */);
/*
 * sm_many_graph_run -- replays a captured batch on `stream`, reads back every frame's
 *   status words and valid-pixel count, solves again alone (with host meshes) a frame whose
 *   device mesh failed, and fills st (counts only). Synchronises `stream` once. Calls on
 *   one graph must not overlap.
 */
sm_status sm_many_graph_run(sm_many_graph* g, sm_stats* st /* [host] */, void* stream);
void sm_many_graph_destroy(sm_many_graph* g);

/*
 * sm_autotune -- measures the tunable launch shapes on one frame and records the fastest
 *   for its size (used by every later sm_solve / sm_solve_many launch of that size in this
 *   process; outputs do not depend on them): validation's block size in waves (1, 2, 4, 8
 *   or 16) for each iteration's cell size; for grid supports, the matcher's lanes per
 *   candidate (64, 32 or 16: 1, 2 or 4 candidates per wave, each candidate's disparity
 *   range in chunks of that many lanes), per disparity range; and the census tile's rows
 *   (8, 16 or 32 rows of 64 columns), per window size. Times each candidate by the device
 *   time of the launches it shapes, with events on those launches inside whole solves of
 *   the frame (one launch after another, the others at their best so far; the best of four
 *   runs of four solves), so that every kernel meets its inputs as the solve leaves them;
 *   the last solve leaves the frame's results in D_f, C_f and mask. About 340 solves of
 *   the frame. Arguments as sm_solve. (The rasteriser's bounded grid, kind 1 of
 *   sm_set_launch_shape, is not tuned: no solve launches it, the star kernels rasterise.)
 *   choices  [host] [11] out: validation waves per iteration (0 past n_iters), the raster
 *            workgroups (0: not tuned), the matcher's lanes per candidate, the census rows
 *            per tile (0 where not tuned).
 */
sm_status sm_autotune(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t stride,
                      const sm_params* p /* [host] */, void* ws, size_t ws_bytes, float* D_f, uint8_t* C_f,
                      uint8_t* mask, int32_t* choices /* [host] */, void* stream);

/*
 * sm_set_launch_shape -- records a launch-shape choice as sm_autotune would (value > 0) or
 *   clears it (value = 0: the built-in rule again), for reproducible timings and for
 *   checking that every shape gives the same results. Host only; thread-safe.
 *   kind 0: validation waves per block (1, 2, 4, 8, 16), key = cell size sz_occ;
 *   kind 1: raster workgroups (512, 1024, 2048, 4096, 8192), key = 0 (accepted, but no
 *           current launch reads it: the solves' star kernels rasterise their meshes);
 *   kind 2: matcher lanes per candidate (16, 32, 64), key = d_max - d_min + 1;
 *   kind 3: census rows per tile (8, 16, 32), key = ((census_w-1)/2) << 8 | ((census_h-1)/2).
 *   Returns SM_ERR_ARG for another kind, value or size.
 */
sm_status sm_set_launch_shape(int32_t kind, int32_t W, int32_t H, int32_t key, int32_t value);

/* Message of the calling thread's last non-OK status ("" if none). */
const char* sm_last_error(void);

/* Library version string. */
const char* sm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STEREOMESH_H */
