/*
 * tgv.h -- C ABI of libtgv, the MI355X (gfx950) library for depth-map fusion
 * by TGV minimisation (Out-of-Core Surface Reconstruction via Global TGV
 * Minimization, 2021).
 *
 * The library computes, on one voxel block of the octree at a time:
 *   - depth-map mipmap pyramids (Sec. 3.4),
 *   - per-voxel vote histograms from the depth maps (Sec. 3.4, Algorithm 1),
 *   - the indicator field u minimising the TGV-L1 energy (Eq. 2 with the
 *     symmetric gradient of Eq. 3 and the data weight lambda of Eq. 1) by the
 *     first-order primal-dual method of Sec. 3.2, with u frozen on a border
 *     layer (Sec. 4.5, Fig. 7), and the energy / duality-gap statistics.
 *
 * Conventions for every call:
 *   - Array pointers are DEVICE pointers unless the name ends in _host.
 *     The caller allocates and frees them; the library never frees caller
 *     memory and keeps no pointer to it after the call returns, except
 *     tgv_state_wrap, whose state uses the caller's memory until it is
 *     destroyed.
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*;
 *     NULL = the null stream) unless documented as synchronising.
 *   - Voxel layout: index x + nx * (y + ny * z) (x fastest).
 *   - Errors are returned as tgv_status; no exception crosses the ABI.
 *     tgv_last_error(ctx) gives a message for the last failing call.
 *   - One context per host thread; a context is not re-entrant.  Calls of
 *     one context may use different streams: work that reuses a buffer the
 *     context owns (the camera table of tgv_build_histograms, the block and
 *     tile tables of tgv_solve_batch, the state of a tgv_solve without one)
 *     waits on the device for the previous call's use of it.  Caller-owned
 *     arrays and states used on several streams are ordered by the caller.
 *   - Depth maps hold the camera-frame z (pinhole maps) or the range (360-
 *     degree scans) of the surface seen through each pixel; values that are
 *     not finite or <= 0 mean "no sample".
 *   - Camera models: see tgv_camera (pinhole depth maps of camera-frame z,
 *     equirectangular 360-degree scans of ranges).
 */
#ifndef TGV_H
#define TGV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TGV_OK = 0,
    TGV_E_INVAL = 1,       /* bad argument (null pointer, bad size, bad parameter) */
    TGV_E_NOMEM = 2,       /* device allocation failed */
    TGV_E_DEVICE = 3,      /* a HIP runtime call failed */
    TGV_E_OVERFLOW = 4,    /* a histogram count could exceed 65535 */
    TGV_E_UNSUPPORTED = 5  /* valid request the library does not implement */
} tgv_status;

/* One camera (80 bytes): a depth map seen through a pinhole or a 360-degree
 * scan.  vote: weight of its votes (1 for stereo depth maps, 5 for near
 * noise-free LIDAR scans, Algorithm 1).  model:
 *   TGV_MODEL_PINHOLE: Xc = R X + t (R row-major); the map holds camera-frame
 *     z; pixel column i covers [i, i+1) of px = fx Xc/Zc + cx, row j of
 *     py = fy Yc/Zc + cy; width x height pixels.
 *   TGV_MODEL_SCAN360: an equirectangular 360-degree scan (terrestrial
 *     LIDAR, Sec. 3.1) of width x height pixels (width divisible by 4)
 *     holding ranges (distances from the scanner's centre).  Xc = R X + t
 *     is the direction in the scanner's frame; column c covers azimuths
 *     [2 pi c / width, 2 pi (c + 1) / width) from +x towards +y, row r polar
 *     angles [pi r / height, pi (r + 1) / height) from +z; fx is the map's
 *     pixels per radian (width / (2 pi)), which with the range sets the
 *     pyramid level; fy, cx, cy are unused.  The pixel is decided by sign
 *     tests against tables of the boundary directions: C[i] = cos(2 pi i /
 *     width), S[i] = sin(2 pi i / width) (i < width / 4) and K[j] = cos(pi j
 *     / height) (j < height), each evaluated in double as written
 *     ((6.283185307179586 i) / width, (3.141592653589793 j) / height) and
 *     rounded to float.  The direction is turned by a multiple of -90
 *     degrees into the first quadrant (quadrant 0: x > 0, y >= 0; 1: x <= 0,
 *     y > 0; 2: x < 0, y <= 0; 3: x >= 0, y < 0; the axis x = y = 0 counts
 *     as quadrant 0) giving (x', y'); the column is quadrant * width / 4
 *     plus the number of i in [1, width / 4) with C[i] y' - S[i] x' >= 0,
 *     the row the number of j in [1, height) with z <= K[j] rho, where rho
 *     = sqrt((x^2 + y^2) + z^2) is the voxel's range (every operation
 *     rounded to float on its own). */
typedef struct {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    int32_t vote;
    int32_t model;  /* TGV_MODEL_* */
} tgv_camera;

enum { TGV_MODEL_PINHOLE = 0, TGV_MODEL_SCAN360 = 1 };

/* A regular voxel block: voxel (i, j, k) has centre origin + (idx + 1/2) h.
 * Voxels closer than `halo` cells to a face keep u frozen during a solve
 * (set B of Fig. 7); 0 <= 2 halo < min(nx, ny, nz). */
typedef struct {
    float origin[3];
    float h;
    int32_t nx, ny, nz;
    int32_t halo;
} tgv_grid;

/* Histogram binning (Algorithm 1).  delta: width of the near-surface band in
 * world units (6 voxel radii = 3 h by default, Sec. 3.1); votes with
 * depth - z < -eta_over_delta * delta are dropped (occluded region).
 * rule 0: nearest of num_bins centres spread evenly over [-1, 1] (ends
 * included); rule 1: floor(((a + 1) / 2) num_bins) with a = 1 folded into
 * the last bin.  centers[0..num_bins-1] ascending are the values the solver
 * uses for each bin; 1 <= num_bins <= 8. */
typedef struct {
    int32_t num_bins;
    int32_t rule;
    float centers[8];
    float delta;
    float eta_over_delta;
} tgv_bins;

/* Storage precision of v, p, q in the solver state (u is always float32;
 * arithmetic is float32 in every mode). */
enum { TGV_STORE_F32 = 0, TGV_STORE_F16 = 1, TGV_STORE_BF16 = 2 };

/* Kernel schedule of a solve: FUSED runs one tiled kernel per iteration
 * (primal then dual in one pass over z-marching tiles); SPLIT runs the dual
 * and the primal update as two per-voxel kernels; FUSED_REF runs the fused
 * iteration as a per-voxel kernel; FUSED2 runs two fused iterations per
 * pass over memory (temporal blocking: the second iteration consumes the
 * first one's results from registers and LDS; tile_y in {4, 6, 7}, default
 * 64 x 7 tiles with the chunk depth chosen for the device); AUTO runs FUSED2
 * for a block whose iteration moves more than 48 MiB (when tile_y is 0)
 * and FUSED otherwise.  All of them produce bit-identical results.  A
 * batched solve runs two iterations per persistent launch with FUSED2, and
 * with AUTO when tile_y is 0; one per launch otherwise. */
enum { TGV_SCHED_FUSED = 0, TGV_SCHED_SPLIT = 1, TGV_SCHED_FUSED_REF = 2, TGV_SCHED_FUSED2 = 3, TGV_SCHED_AUTO = 4 };

/* Solver parameters (Eq. 2, Sec. 3.2).  tau, sigma: primal and dual step
 * sizes (> 0); iters >= 0 primal-dual iterations.  tile_y, tile_z: shape of
 * the fused kernel's tiles (64 x tile_y columns, tile_z planes per
 * workgroup); 0 picks the library default: tile_y 8 for a float32 block
 * whose iteration moves more than 256 MiB, else 4; 7 for FUSED2 (and for
 * a batched solve that runs two iterations per launch); 4 for a batched
 * solve with one (tile_y in {4, 8, 12}; in {4, 6, 7} for FUSED2); tile_z
 * from a model of the launch's rounds of resident workgroups (up to 32
 * planes for FUSED; at most 32 for a batched solve). */
typedef struct {
    float alpha0, alpha1, lambda;
    float tau, sigma;
    int32_t iters;
    int32_t storage;   /* TGV_STORE_* */
    int32_t schedule;  /* TGV_SCHED_* */
    int32_t tile_y, tile_z;
    int32_t flags;     /* TGV_FLAG_* */
} tgv_params;

/* flags: TGV_FLAG_GRAPH captures a batched solve's iteration loop in a HIP
 * graph and replays it; TGV_FLAG_TVL1 solves the TV-L1 model of Eq. 1
 * (alpha1 |grad u| + lambda data, i.e. v held at 0 and q unused) instead of
 * the TGV model of Eq. 2: a solve of at least one iteration first sets the
 * state's v and q (both iterates) to 0, whatever they held, and they stay
 * 0.  TGV_FLAG_LEAVE_OPEN (tgv_solve on a caller state without u_io or
 * statistics, tgv_solve_batch without statistics) leaves the state open:
 * iteration n = iters_done has its dual half done and its primal half
 * pending.  The next solve of an open state starts with a pass that
 * completes that primal half fused with the next iteration's dual half, so
 * a long solve cut into calls costs no extra passes; a solve without the
 * flag closes the state (iters 0 closes it without advancing it).  The
 * results are bit-identical to one uninterrupted solve.  An open state
 * cannot be exported or evaluated (tgv_state_export, tgv_energy:
 * TGV_E_INVAL) and continues with the model (TGV or TV-L1) it was opened
 * with; tgv_state_reset and tgv_state_import close it. */
enum { TGV_FLAG_GRAPH = 1, TGV_FLAG_TVL1 = 2, TGV_FLAG_LEAVE_OPEN = 4 };

/* Energy statistics of a state, reduced in float64:
 *   primal = discrete Eq. 2 at (u, v);
 *   dual   = dual bound of the problem restricted to u in [-1, 1] on free
 *            voxels and |v| <= 2 sqrt(3) per voxel;
 *   gap_rel = (primal - dual) / max(primal, 1);
 *   nonfinite = voxels whose u, v, p or q is not finite. */
typedef struct {
    double primal, dual, gap_rel;
    double parts[3];   /* alpha1 term, alpha0 term, data term of primal */
    int64_t nonfinite;
    int64_t iters_done;
} tgv_stats;

typedef struct tgv_ctx tgv_ctx;
typedef struct tgv_state tgv_state;

/* Create a context on HIP device `device` (made current for the call).
 * Returns TGV_E_DEVICE if the device cannot be used. */
tgv_status tgv_create(int device, tgv_ctx **out);
/* Release a context and its workspace (synchronises the device). */
void tgv_destroy(tgv_ctx *ctx);
/* Message of the last failing call on ctx (never NULL; owned by ctx). */
const char *tgv_last_error(const tgv_ctx *ctx);

/* ---- depth-map pyramids (Sec. 3.4) ---------------------------------- */

/* Levels of a W x H pyramid: each level halves each side, rounding up,
 * down to 1 x 1. */
int32_t tgv_pyramid_levels(int32_t W, int32_t H);
/* Floats of one camera's packed pyramid (all levels back to back). */
int64_t tgv_pyramid_floats(int32_t W, int32_t H);
/* Build the pyramids of n_cams depth maps depth[n_cams][H][W] into
 * pyr[n_cams][tgv_pyramid_floats(W, H)].  Level 0 is the input with
 * invalid samples set to 0; a level-(l+1) pixel is the mean of the valid
 * ones among its (up to four) children, summed in the order (2i,2j),
 * (2i+1,2j), (2i,2j+1), (2i+1,2j+1), 0 if none is valid. */
tgv_status tgv_build_pyramids(tgv_ctx *ctx, const float *depth, int32_t n_cams, int32_t W, int32_t H, float *pyr,
                              void *stream);

/* ---- histograms (Sec. 3.4, Algorithm 1) ------------------------------ */

/* Conservative camera cull for a block (host only): writes to keep_host the
 * indices of the cameras whose view may contain a voxel centre of the
 * block (a pinhole camera: its frustum; a 360-degree scan: always), returns
 * their count (or -1 on bad arguments).  Culling never changes a
 * histogram: dropped cameras cast no vote. */
int32_t tgv_cull_cameras(const tgv_camera *cams_host, int32_t n_cams, const tgv_grid *grid, int32_t *keep_host);

/* Vote histograms of every voxel of `grid` from n_cams cameras whose
 * pyramids are packed in pyr (as written by tgv_build_pyramids, all
 * cameras width W and height H).  Output hist[nz][ny][nx][8] uint16: slot
 * k < num_bins counts the votes of bin k, slots >= num_bins are 0.  Per
 * (voxel, camera): project the voxel centre (pinhole) or find its pixel
 * and range (scan); no vote if behind a pinhole camera, outside its image,
 * on an invalid sample or further than eta behind the observed surface;
 * else bin clamp((depth - distance) / delta, -1, 1) by `rule`, where the
 * distance is the camera-frame z (pinhole) or the range (scan).  The level
 * read is floor(log2(h fx / distance)), clamped to the pyramid.  All
 * arithmetic is IEEE binary32 without contraction, so counts are exact and
 * reproducible.  TGV_E_OVERFLOW if the votes of the cameras kept by the
 * cull could sum past 65535. */
tgv_status tgv_build_histograms(tgv_ctx *ctx, const float *pyr, int32_t W, int32_t H, const tgv_camera *cams_host,
                                int32_t n_cams, const tgv_grid *grid, const tgv_bins *bins, uint16_t *hist,
                                void *stream);

/* flags of tgv_build_histograms_ex */
enum { TGV_HIST_ACCUMULATE = 1 };

/* tgv_build_histograms for cameras of different sizes and models (stereo
 * depth maps and 360-degree scans at their own resolutions, fused into one
 * block, Sec. 3.1): camera c is cams_host[c].width x cams_host[c].height
 * and its pyramid (as tgv_build_pyramids writes it at that size) starts at
 * pyr + pyr_offsets_host[c] floats.  flags 0 overwrites hist; with
 * TGV_HIST_ACCUMULATE the votes are added to the counts hist already holds,
 * of which every voxel has at most prior_votes (e.g. the summed votes of
 * earlier calls); TGV_E_OVERFLOW if prior_votes plus the votes of the kept
 * cameras could exceed 65535.  prior_votes must be 0 without the flag. */
tgv_status tgv_build_histograms_ex(tgv_ctx *ctx, const float *pyr, const int64_t *pyr_offsets_host,
                                   const tgv_camera *cams_host, int32_t n_cams, const tgv_grid *grid,
                                   const tgv_bins *bins, int32_t flags, int32_t prior_votes, uint16_t *hist,
                                   void *stream);

/* ---- solver (Eq. 2, Sec. 3.2, Sec. 4.5) ----------------------------- */

/* A resumable solver state for one grid shape and storage precision:
 * u (current and previous iterate), v (same), p, q (double-buffered),
 * held in device memory owned by the state. */
tgv_status tgv_state_create(tgv_ctx *ctx, const tgv_grid *grid, int32_t storage, tgv_state **out);
/* Same, in caller-owned device memory of at least tgv_state_bytes(grid,
 * storage) bytes (256-byte aligned); the state never frees it, and the
 * memory must outlive the state.  Lets a
 * caller keep states in its own pool (a serving loop, a caching allocator)
 * without device-synchronising frees. */
tgv_status tgv_state_wrap(tgv_ctx *ctx, const tgv_grid *grid, int32_t storage, void *mem, int64_t bytes,
                          tgv_state **out);
/* Release a state (frees its memory unless it was wrapped). */
void tgv_state_destroy(tgv_state *st);
/* Device bytes a state of this grid and storage uses. */
int64_t tgv_state_bytes(const tgv_grid *grid, int32_t storage);
/* Reset to a fresh start: u = u0 (interior initial values and the frozen
 * border), v = p = q = 0, iteration count 0. */
tgv_status tgv_state_reset(tgv_ctx *ctx, tgv_state *st, const float *u0, void *stream);
/* Copy the current fields out as float32 (any pointer may be NULL):
 * u[n], v[3][n] (current iterate), u_prev[n], v_prev[3][n] (previous
 * iterate, equal to the current one before the first step), p[3][n],
 * q[6][n] (q order xx yy zz xy xz yz).  Together they are the whole state:
 * importing them into a state resumes the iteration bit for bit (for
 * float32 storage). */
tgv_status tgv_state_export(tgv_ctx *ctx, const tgv_state *st, float *u, float *v, float *u_prev, float *v_prev,
                            float *p, float *q, void *stream);
/* Load a state exported earlier (all six pointers required; values are
 * rounded to the state's storage precision). */
tgv_status tgv_state_import(tgv_ctx *ctx, tgv_state *st, const float *u, const float *v, const float *u_prev,
                            const float *v_prev, const float *p, const float *q, int64_t iters_done, void *stream);

/* Run params->iters primal-dual iterations:
 *   p <- P_alpha1(p + sigma M.(grad ubar - vbar)),  q <- P_alpha0(q + sigma E(vbar)),
 *   u <- prox(u + tau div p) on free voxels (u frozen on the border),
 *   v <- v + tau (M.p + div2 q),  ubar = 2 u_new - u_old,  vbar likewise,
 * where prox is the proximal map of lambda sum_k hist_k |u - c_k|.
 * state == NULL: fresh solve from u_io (initial values + frozen border)
 * in a context-owned state; the result is written back to u_io.
 * state != NULL: the state is advanced (it must match grid and
 * params->storage) and u is written to u_io when u_io != NULL.
 * stats_host != NULL: also reduce the energy statistics of the final
 * state (this synchronises the stream).
 * The gap every k iterations: solve in chunks of k on a state with
 * stats_host set (resuming is bit-identical to one long solve).
 * Blocks with 24 * nx * ny * nz >= 2^31 (about 447^3 voxels) exceed the
 * tiled kernels' 32-bit buffer offsets; their fused passes run the
 * per-voxel fused kernel (same results, slower). */
tgv_status tgv_solve(tgv_ctx *ctx, const tgv_grid *grid, const uint16_t *hist, const tgv_bins *bins,
                     const tgv_params *params, float *u_io, tgv_state *state, tgv_stats *stats_host, void *stream);

/* Bytes of the fixed device workspace of tgv_solve_noalloc (64 MiB): a
 * state of tgv_state_bytes(grid, storage) up to this size, e.g. blocks of
 * up to 645 277 voxels (86^3) with float32 storage, 1 198 372 (106^3) with
 * 16-bit storage. */
#define TGV_NOALLOC_MAX_BYTES (64LL << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): a fresh
 * solve as tgv_solve(ctx, grid, hist, bins, params, u_io, NULL, NULL,
 * stream) gives, bit for bit, whose solver state lives in a fixed device
 * array of TGV_NOALLOC_MAX_BYTES instead of a context-owned allocation.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine) and returns no statistics.  u_io: in = initial values and the
 * frozen border, out = u.  TGV_E_INVAL if the block's state needs more than
 * TGV_NOALLOC_MAX_BYTES (tgv_state_bytes(grid, params->storage)) or on the
 * argument errors of tgv_solve.  Each GPU holds one such array for the
 * life of the process, shared by every context and call on that GPU: calls
 * that overlap on one GPU (other streams, other contexts or threads) race
 * on it and give undefined results; calls in one stream are ordered. */
tgv_status tgv_solve_noalloc(tgv_ctx *ctx, const tgv_grid *grid, const uint16_t *hist, const tgv_bins *bins,
                             const tgv_params *params, float *u_io, void *stream);

/* Batched solve (many uneven blocks, Sec. 4.5: treetop leaves are
 * independent units, and small ones are processed together): advance each
 * of the n states by params->iters iterations.  Every iteration (or
 * pair of iterations, see the schedules) of all blocks is one persistent
 * launch whose workgroups pull tiles from a device work queue (plus a
 * per-block dual step at the start and primal step at the end; blocks too
 * large for 32-bit tile offsets run their own per-voxel launches).  hist: host array of n device pointers (block i's histograms);
 * tile_z_host: per-block z-chunk of the tiles (NULL = params->tile_z or the
 * default: with two iterations per launch, 16, 32 or 64 planes for the whole
 * batch, whichever a plane-step model of the batch's tiles on the device's
 * resident workgroups finds shortest); params->tile_y applies to all blocks.  With TGV_FLAG_GRAPH the
 * iteration loop is captured once in a HIP graph and replayed.  Results are
 * bit-identical to tgv_solve on each state alone.  stats_host: NULL or n
 * entries (synchronises).  All states must use params->storage.  Open and
 * closed states may be mixed: every state advances params->iters
 * iterations (the open ones take one more batched pass than the closed
 * ones, which start with their dual half). */
tgv_status tgv_solve_batch(tgv_ctx *ctx, int32_t n, tgv_state *const *states, const uint16_t *const *hist,
                           const tgv_bins *bins, const tgv_params *params, const int32_t *tile_z_host,
                           tgv_stats *stats_host, void *stream);

/* ---- coarse-to-fine (Sec. 3.2, Sec. 4.5) ------------------------------ */

/* Nearest-parent prolongation: u_fine(i, j, k) = u_coarse(i/2, j/2, k/2)
 * (integer division) for every fine voxel; the coarse grid must have
 * ceil(n/2) voxels per axis.  The indicator of a cube's parent is what the
 * paper freezes on a part's border and starts the finer level from. */
tgv_status tgv_prolongate(tgv_ctx *ctx, const tgv_grid *coarse, const float *u_coarse, const tgv_grid *fine,
                          float *u_fine, void *stream);

/* Coarse-to-fine solve of one block: levels k = levels-1 .. 0 with voxel
 * size h 2^k and ceil(n / 2^k) voxels per axis over the same origin (the
 * band width delta scales with the voxel, Sec. 3.1); each level builds its
 * histograms from the pyramids, starts from the prolongated coarser
 * solution (0 on the coarsest), keeps u frozen on its halo (the finest
 * level uses grid->halo, coarser levels none) and runs params->iters
 * iterations.  The finest u is written to u_out.  Asynchronous on
 * `stream`: the levels' histograms, fields and solver state live in a
 * context-owned workspace that is allocated on the first call and grown
 * (after the previous call's work on it has finished) only when a call
 * needs more; calls on other streams wait on the device for the previous
 * call's use of it. */
tgv_status tgv_solve_coarse_to_fine(tgv_ctx *ctx, const float *pyr, int32_t W, int32_t H, const tgv_camera *cams_host,
                                    int32_t n_cams, const tgv_grid *grid, const tgv_bins *bins,
                                    const tgv_params *params, int32_t levels, float *u_out, void *stream);

/* ---- zero level (Sec. 4.6) ------------------------------------------ */

/* Iso-surface points of u = 0 on a block: for every grid edge between
 * voxel x and x + e_i whose values have different signs (u > 0 against
 * u <= 0), the point origin + (x + 1/2 + t e_i) h with t = u(x) / (u(x) -
 * u(x + e_i)), written as 4 floats (X, Y, Z, i) to points[k], in voxel
 * order then axis order (deterministic).  At most max_points are written
 * (points may be NULL with max_points 0 to only count); *count_host
 * receives the total number of crossings.  Synchronises the stream. */
tgv_status tgv_extract_crossings(tgv_ctx *ctx, const tgv_grid *grid, const float *u, float *points,
                                 int64_t max_points, int64_t *count_host, void *stream);

/* Energy statistics of a state (synchronises the stream). */
tgv_status tgv_energy(tgv_ctx *ctx, const tgv_state *st, const uint16_t *hist, const tgv_bins *bins,
                      const tgv_params *params, tgv_stats *stats_host, void *stream);

/* ---- measurement ------------------------------------------------------ */

/* Copy `bytes` (a multiple of 16; both pointers 16-byte aligned) from src
 * to dst with a plain streaming kernel: every byte read once and written
 * once, the pass the solver kernels' memory rates are measured against.
 * variant selects its shape: bits 0-1 the 16-byte vectors per lane and
 * trip (1, 2, 4, 8), bit 2 non-temporal loads and stores, bits 3-4 the
 * workgroups of 256 lanes per compute unit (2, 4, 8, 16); 0 <= variant <
 * 32.  The buffers must not overlap. */
tgv_status tgv_stream_copy(tgv_ctx *ctx, const void *src, void *dst, int64_t bytes, int32_t variant, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TGV_H */
