/*
 * msplat.h -- C ABI of the MI355X (gfx950) differentiable Gaussian rasterizer.
 *
 * The library implements the data-parallel hot path of Mini-Splatting2-style
 * scene modelling (arXiv 2411.12788): projection of 3D Gaussians to screen,
 * tile binning by a (tile | depth) key sort, front-to-back alpha compositing
 * with rendered argmax index and depth, per-Gaussian importance / area /
 * max-weight accumulation, and the backward pass restricted to an active mask.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: gs_status (0 = GS_OK).  On error nothing has been enqueued
 *    (argument errors) or the HIP error text is available via gs_last_error().
 *  - Ownership: every buffer is allocated and freed by the caller.  Device
 *    pointers (marked [dev]) must stay valid until the enqueued work on
 *    `stream` completes; host pointers (marked [host]) are read before the
 *    call returns.  The library keeps no pointer after return and allocates
 *    nothing: scratch memory arrives as (ws, ws_bytes), sized by the matching
 *    *_workspace_size() query, 256-byte aligned.  (The exceptions:
 *    gs_sort_pairs_static uses a library-owned device array instead, and
 *    gs_bin_count keeps, per host thread and device, a 64-byte pinned host
 *    buffer and an event for its read-back, made on first use and kept until
 *    the process ends.)
 *  - Asynchrony: work is enqueued on `stream` (a hipStream_t; NULL = the null
 *    stream).  Only gs_bin_count and gs_bin synchronise (they return the pair
 *    count).
 *  - Reentrancy: no global mutable state (apart from the diagnostics
 *    gs_sort_set_spin_limit, gs_sort_set_algorithm and
 *    gs_bin_count_set_fold_blocks, and the scratch array of
 *    gs_sort_pairs_static);
 *    concurrent calls on different streams with disjoint buffers are safe.
 *  - Views: V cameras (1 <= V <= GS_MAX_VIEWS) are rendered in one launch per
 *    stage.  A record is one (view, Gaussian) pair, index r = v * n + i.
 *    Per-pixel arrays are indexed by the global pixel id
 *    g = pixel_base[v] + y * width_v + x, pixel_base = prefix sum of width*height;
 *    colour-like arrays are channel-planar: color[c * P + g], P = total pixels.
 *    Tiles are 16x16 pixels; the global tile id is tile_base[v] + ty * tiles_x_v + tx.
 */
#ifndef MSPLAT_H
#define MSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_MAX_VIEWS 32
#define GS_TILE 16
#define GS_REC_FLOATS 16 /* floats per projected record */
#define GS_GRAD2D_FLOATS 9 /* floats per record in the 2D gradient buffer */

typedef enum {
  GS_OK = 0,
  GS_ERR_NULL = -1,        /* a required pointer is NULL */
  GS_ERR_SHAPE = -2,       /* n < 0, V out of range, width/height <= 0 or > 65535, sh_degree not in 0..3 */
  GS_ERR_CAMERA = -3,      /* a camera value is not finite, or fx/fy <= 0 */
  GS_ERR_CAPACITY = -4,    /* ws_bytes (or a count) too small; see the call's notes */
  GS_ERR_DEVICE = -5,      /* HIP reported an error; see gs_last_error() */
  GS_ERR_UNSUPPORTED = -6  /* option value not supported */
} gs_status;

/* depth_mode values: which depth the forward pass writes per pixel.
 * MID     d^mid of the max-weight Gaussian: mid-point of the ray's two
 *         intersections with its 1-sigma ellipsoid (Eq. (2); Sec. 4.1).
 *         When the ray misses the ellipsoid the max-density point along the ray
 *         is written and hit = 0.
 * CENTER  camera depth of the max-weight Gaussian's centre (Sec. 4.1, d^center).
 * BLEND   sum_i w_i z_i (Sec. 4.1, d^blend). */
enum { GS_DEPTH_MID = 0, GS_DEPTH_CENTER = 1, GS_DEPTH_BLEND = 2 };

/* flags */
enum {
  GS_ACCUM_IMPORTANCE = 1, /* gs_render_forward also accumulates (importance, wmax, area) */
  GS_ACCUM_PER_VIEW = 2    /* accumulators are [V][n] instead of [n] summed over views */
};

/* Scene: structure-of-arrays float32 planes, all [dev].
 * means[3][n], scales[3][n] (activated, > 0), quats[4][n] ((w, x, y, z), any
 * non-zero norm; normalised inside), opacity[n] (activated, in [0, 1]),
 * sh[16][3][n] (real SH coefficients, plane k * 3 + channel; only the first
 * (sh_degree + 1)^2 coefficient planes are read).  Sec. 3.1: Gaussian with
 * opacity, centre and covariance Sigma = R(q) diag(s)^2 R(q)^T; colour from SH. */
typedef struct {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacity;
  const float* sh;
  int64_t n;
  int32_t sh_degree;
} gs_scene_t;

/* Pinhole camera [host]: world -> camera rotation R (row-major) and
 * translation t (x_cam = R x_world + t; OpenCV axes: x right, y down, z
 * forward), focal lengths and principal point in pixels; pixel (px, py)
 * samples the continuous image point (px + 0.5, py + 0.5). */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} gs_camera_t;

/* Rasterizer constants.  The paper states none of them; gs_default_opts()
 * gives the 3DGS-lineage values: znear 0.2, low-pass 0.3 (added to the 2D
 * covariance), alpha_max 0.99 (clamp), alpha_min 1/255 (skip), t_min 1e-4
 * (stop before a Gaussian that would take transmittance below it), Jacobian
 * clamp 1.3 x tan(half field of view), black background, MID depth. */
typedef struct {
  float znear, lowpass, alpha_max, alpha_min, t_min, jac_clamp;
  float bg[3];
  int32_t depth_mode;
  int32_t flags;
} gs_opts_t;

/* Projected records [dev], written by gs_project:
 * rec[V * n][16] float: u_hi, v_hi, u_lo, v_lo (screen mean as a float pair,
 *   u = u_hi + u_lo), A, B, C, lo (exponent form of the conic: the 2D Gaussian
 *   times opacity is exp2(lo - A dx^2 - B dx dy - C dy^2), lo = log2 opacity),
 *   r, g, b, opacity, z (camera depth of the centre), a, b, c (conic
 *   [[a, b], [b, c]] = inverse of the 2D covariance with low-pass).  Written
 *   for drawn records only (tiles_touched > 0); other rows keep their bytes.
 * bin[V * n][4] int32: x box (x_lo | x_hi << 16), y box (y_lo | y_hi << 16) in
 *   pixels, clipped to the image; float32 bits of z; tiles_touched (0 = not
 *   drawn: culled, behind the near plane, off-image, or opacity < alpha_min). */
typedef struct {
  float* rec;
  int32_t* bin;
  /* Tile culling at emission (opt-in; 0 = off).  When < 0 it is
   * log2(alpha_cull): gs_project counts, and gs_emit_keys / gs_bin_sort emit,
   * only the tiles of a record's box where exp2(lo - A dx^2 - B dx dy - C dy^2)
   * can reach alpha_cull at a pixel centre of the tile's part of the box (a
   * conservative test: the continuous minimum of the quadratic over that
   * rectangle, with a margin).  Records whose box spans more than
   * GS_TILE_CULL_MAX_TILES tiles keep every tile.  With alpha_cull <= the
   * alpha_min the compositing kernels use, a dropped pair could never have
   * been composited (Sec. 3.1's tile-based rasterizer; the paper's baseline
   * cites tile-based culling of this kind), so every output is unchanged.
   * Set it before gs_project and keep it for the binning calls. */
  float tile_cull_log2_alpha;
} gs_projected_t;
enum { GS_TILE_CULL_MAX_TILES = 64 };

/* Statistics returned by gs_bin_count [host]. */
typedef struct {
  int64_t n_isect;     /* number of (tile, record) pairs */
  int64_t n_visible;   /* records with tiles_touched > 0 */
  uint32_t zbits_min;  /* min / max float32 bits of z over visible records */
  uint32_t zbits_max;
  int32_t tiles_total; /* sum over views of tiles_x * tiles_y */
  int32_t depth_bits;  /* bits kept of (zbits - zbits_min) in the sort key */
  int32_t key_bits;    /* significant bits of the sort key: tile bits + depth_bits */
  int32_t pad;
} gs_bin_stats_t;

/* Forward outputs [dev], P = total pixels over the V views.  Optional
 * pointers may be NULL. */
typedef struct {
  float* color;        /* [3][P] composited colour incl. T_final * bg (Eq. (1)) */
  float* depth;        /* [P] per depth_mode; 0 where nothing was drawn */
  int32_t* imax;       /* [P] Gaussian index of max blend weight (Eq. (2)); -1 if none */
  float* t_final;      /* [P] transmittance after the last included Gaussian */
  uint32_t* last;      /* [P] 1 + position in the tile list of the last included Gaussian */
  uint32_t* n_contrib; /* [P] optional: number of included Gaussians */
  uint8_t* hit;        /* [P] optional: 1 if the pixel ray meets imax's 1-sigma ellipsoid */
} gs_fwd_out_t;

/* Per-Gaussian accumulators [dev]; ADDED to (the caller zeroes them).
 * importance: I_i = sum over pixels of w_i (Sec. 3.2)
 * wmax:       max over pixels of w_i (the w_{i_max} significance criterion, Sec. 5.1)
 * area:       S_i = number of pixels whose imax is i (Eq. (3))
 * Sized [n], or [V][n] with GS_ACCUM_PER_VIEW (per-view visibility, Sec. 5.2).
 * Any of the three may be NULL. */
typedef struct {
  float* importance;
  float* wmax;
  uint32_t* area;
} gs_accum_t;

/* Parameter gradients [dev], same layouts as gs_scene_t (sh is [16][3][n];
 * planes beyond (sh_degree + 1)^2 are written as 0).  Overwritten. */
typedef struct {
  float* means;
  float* scales;
  float* quats;
  float* opacity;
  float* sh;
} gs_grads_t;

/* ---------------------------------------------------------------------- */
const char* gs_last_error(void);      /* thread-local text of the last error */
int32_t gs_version(void);             /* 10000 * major + 100 * minor + patch */
void gs_default_opts(gs_opts_t* opts);

/* Per-view layout helpers [host out]: tiles_x/tiles_y/tile_base/pixel_base
 * arrays of length V (may be NULL), totals returned through the pointers. */
int32_t gs_view_layout(const gs_camera_t* cams, int32_t V, int32_t* tiles_x, int32_t* tiles_y,
                       int32_t* tile_base, int64_t* pixel_base, int32_t* tiles_total, int64_t* pixels_total);

/* a1 -- projection (Sec. 3.1): for every record, camera transform, covariance
 * Sigma = R(q) diag(s^2) R(q)^T, local affine projection
 * Sigma' = J W Sigma W^T J^T + lowpass I, conic, screen mean, SH colour
 * max(0, 0.5 + sum_k c_k Y_k(dir)) with dir from the camera centre, and the
 * pixel box of the ellipse where alpha >= alpha_min.  Computed in double and
 * stored as float.  cull_mask [dev, u8 n] may be NULL; a 0 entry excludes that
 * Gaussian from every view "at the preprocessing stage" (Sec. 5.2). */
int32_t gs_project(const gs_scene_t* scene, const gs_camera_t* cams, int32_t V, const uint8_t* cull_mask,
                   const gs_opts_t* opts, const gs_projected_t* out, void* stream);

/* a2 -- binning count: exclusive scan of tiles_touched into offsets [dev, u32
 * V*n] and the statistics above.  Synchronises `stream` to return *stats: the
 * counting kernel also writes the totals to host-mapped memory and the calling
 * thread polls an event (it spins, holding one core, for the few microseconds
 * of the count).  GS_ERR_CAPACITY if the pair count is 2^30 or more (the
 * sort's limit). */
size_t gs_bin_count_workspace_size(int64_t n_records);
int32_t gs_bin_count(const gs_projected_t* proj, const gs_camera_t* cams, int32_t V, int64_t n,
                     uint32_t* offsets, gs_bin_stats_t* stats, void* ws, size_t ws_bytes, void* stream);

/* a2-a4 -- emit one (tile | depth) key per (tile, record) pair, sort them
 * stably by key (ties keep ascending record order), and find each tile's run.
 * Sec. 3.1: Gaussians are sorted in an approximate depth order by the depth of
 * their centres; here per tile.  vals [dev, u32 n_isect] receives the sorted
 * record indices; ranges [dev, u32 tiles_total][2] receives [start, end) per
 * tile ([0, 0) if empty); keys [dev, u64 n_isect] may be NULL, else receives the
 * sorted keys (global tile << 32) | float32 bits of z; tile_order [dev, u32
 * tiles_total] may be NULL, else receives the processing order described at
 * gs_tile_order. */
size_t gs_bin_sort_workspace_size(int64_t n_isect);
int32_t gs_bin_sort(const gs_projected_t* proj, const gs_camera_t* cams, int32_t V, int64_t n,
                    const uint32_t* offsets, const gs_bin_stats_t* stats, uint64_t* keys, uint32_t* vals,
                    uint32_t* ranges, uint32_t* tile_order, void* ws, size_t ws_bytes, void* stream);

/* a2-a4 in one call: gs_bin_count, then gs_bin_sort when the pairs fit the
 * caller's buffers, with nothing between the pair count's read-back and the
 * sort's first launch (a caller that keeps its buffers from step to step
 * then pays one host round trip per binning).  Arguments as in the two calls;
 * pair_capacity = entries of vals (and of keys, when not NULL); ranges and
 * tile_order hold tiles_total entries (fixed by the cameras); count_ws /
 * sort_ws are the two calls' workspaces.  Returns the first failing call's
 * status, with one addition: GS_ERR_CAPACITY with *stats and offsets valid
 * and stats->n_isect < 2^30 means the pairs did not fit (n_isect >
 * pair_capacity, or sort_ws_bytes < gs_bin_sort_workspace_size(n_isect));
 * nothing was sorted, and the caller grows its buffers and calls gs_bin_sort
 * with the same stats and offsets.  Synchronises `stream` (the pair count). */
int32_t gs_bin(const gs_projected_t* proj, const gs_camera_t* cams, int32_t V, int64_t n, uint32_t* offsets,
               gs_bin_stats_t* stats, uint64_t* keys, uint32_t* vals, int64_t pair_capacity, uint32_t* ranges,
               uint32_t* tile_order, void* count_ws, size_t count_ws_bytes, void* sort_ws, size_t sort_ws_bytes,
               void* stream);

/* Processing order of the tiles for the compositing kernels: tile ids
 * [dev, u32 tiles_total] grouped by the bit length of their list length,
 * longest lists first, ascending tile id inside a group (so the order is a
 * function of the ranges alone).  Work per tile varies by orders of
 * magnitude; starting the long lists first keeps them off the critical path
 * and spreads them over all XCDs.  The compositing kernels also take from the
 * order which tiles to share between four workgroups; that changes results
 * only by float32 rounding, and the same order gives bitwise the same
 * results.  Also produced by gs_bin_sort when tile_order is non-NULL. */
size_t gs_tile_order_workspace_size(void);
int32_t gs_tile_order(const uint32_t* ranges, int32_t tiles_total, uint32_t* tile_order, void* ws, size_t ws_bytes,
                      void* stream);

/* The three stages of gs_bin_sort, exported separately.
 * gs_emit_keys: key = (global tile << depth_shift) | (zbits - zbits_min) for each pair.
 * gs_sort_pairs: in-place stable ascending sort of (keys, vals) on key bits
 *   [0, key_bits) (1..64); ws sized by gs_sort_workspace_size(n); n < 2^30
 *   (GS_ERR_CAPACITY otherwise).
 * gs_tile_ranges: ranges from sorted keys whose tile id is key >> depth_shift;
 *   keys_out (may be NULL; not keys itself: GS_ERR_SHAPE) receives
 *   (tile << 32) | (low bits + zbits_min). */
int32_t gs_emit_keys(const gs_projected_t* proj, const gs_camera_t* cams, int32_t V, int64_t n,
                     const uint32_t* offsets, int32_t depth_shift, uint32_t zbits_min, uint64_t* keys,
                     uint32_t* vals, void* stream);
size_t gs_sort_workspace_size(int64_t n);
int32_t gs_sort_pairs(uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits, void* ws, size_t ws_bytes,
                      void* stream);
int32_t gs_tile_ranges(const uint64_t* keys, int64_t n, int32_t depth_shift, uint32_t zbits_min,
                       int32_t tiles_total, uint32_t* ranges, uint64_t* keys_out, void* stream);

/* Sort status.  The radix sort of gs_bin_sort and gs_sort_pairs waits on
 * other workgroups in bounded loops; a wait that exhausts its bound does not
 * hang but raises an error flag in the first word of the workspace (the
 * workspaces of both calls start with a 512-byte header) and leaves an invalid
 * order.  gs_sort_status synchronises `stream`, reads the flag of the last
 * sort run on the workspace `ws` [dev] and returns GS_OK, or GS_ERR_DEVICE
 * with gs_last_error() saying the order is invalid.  The flag is cleared at
 * the start of every sort on that workspace. */
int32_t gs_sort_status(const void* ws, void* stream);

/* Diagnostic: the number of polls a sort look-back may make before it gives
 * up (default 2^22; 0 makes every look-back give up at once, which exercises
 * the error path above without any wait).  Process-wide; affects sorts
 * enqueued after the call. */
void gs_sort_set_spin_limit(uint32_t polls);

/* Diagnostic: how a radix pass learns where its digits go in the output.
 * GS_SORT_PRESCAN (default): per pass an up-sweep counts each digit per tile
 * of keys and a scan turns the counts into prefixes, then the scatter;
 * no workgroup waits on another.  GS_SORT_LOOKBACK: one kernel per pass, each
 * tile publishes its counts and reads its predecessors' (decoupled look-back,
 * bounded waits reported through gs_sort_status).  Both give the same order.
 * Process-wide; affects sorts enqueued after the call.  GS_ERR_UNSUPPORTED
 * for another value. */
enum { GS_SORT_PRESCAN = 0, GS_SORT_LOOKBACK = 1 };
int32_t gs_sort_set_algorithm(int32_t algorithm);

/* Diagnostic: the largest number of 4096-record blocks for which gs_bin_count
 * runs two kernels (each block of the down-sweep adds the totals of the
 * blocks before it, and the last one publishes the statistics); above it a
 * single-workgroup scan of the block totals runs between the two.  Default
 * 4096 (about 16.7M records; a negative value restores it); 0 always takes
 * the three-kernel path.  Both give the same offsets and statistics.
 * Process-wide; returns the previous value. */
int64_t gs_bin_count_set_fold_blocks(int64_t blocks);

/* Allocation-free sort, for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid allocation).
 * Same result as gs_sort_pairs: in-place stable ascending sort of (keys, vals)
 * [dev, n] on key bits [0, key_bits) (1..64).  The scratch memory is a
 * library-owned device array of fixed size per GPU (sort workspace for
 * GS_SORT_STATIC_MAX_PAIRS pairs, about 14 MB), held until the process ends:
 * n <= GS_SORT_STATIC_MAX_PAIRS, GS_ERR_CAPACITY otherwise.  Runs on the
 * current device; `stream` must belong to it.  All calls on one GPU share the
 * array, so calls that overlap on one GPU (other streams or threads) race.
 * status [dev, u32, may be NULL] receives the sort's status flag once the sort
 * completes on the stream: 0 for a valid order, nonzero when a look-back gave
 * up (see gs_sort_status).  Allocates nothing and does not synchronise. */
#define GS_SORT_STATIC_MAX_PAIRS (1 << 20)
int32_t gs_sort_pairs_static(uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits, uint32_t* status,
                             void* stream);

/* Spatial order: a memory layout of this library, not a step of the method.
 * The Gaussians' index order is free (every result is the same up to a
 * permutation, except that list entries of exactly equal depth keep ascending
 * index order); stored along a Morton (Z-order) curve of their means, the
 * Gaussians a tile's list names sit close together in memory, and the
 * compositing and projection kernels read fewer cache lines.
 * gs_spatial_order: perm [dev, u32 n] receives the stable ascending order of
 * the 30-bit codes of the means [dev, f32 3 x n, planar]; codes [dev, u32 n]
 * may be NULL, else receives the code of Gaussian i at i.  The code, in
 * float32: per axis, lo and hi are the min and max over the Gaussians whose
 * three coordinates are finite, s = 1024 / (hi - lo) (0 when hi = lo), the
 * cell is floor((x - lo) * s), or 1023 when that product is 1023 or more or
 * not a number; bits 3b + 2, 3b + 1 and 3b of the code are bit b of the x, y
 * and z cells.  A Gaussian with a non-finite coordinate gets 2^30 - 1 (it
 * sorts last).  ws [dev] sized by gs_spatial_order_workspace_size(n); its
 * start is a sort workspace (gs_sort_status applies); n < 2^30
 * (GS_ERR_CAPACITY otherwise).  Does not synchronise.
 * gs_permute: dst[p n + i] = src[p n + perm[i]] for planes p < planes and
 * i < n, elements of elem_bytes (1, 2, 4, 8 or 16) bytes [dev, both planar
 * with plane stride n; they may not overlap (GS_ERR_SHAPE)].  An entry
 * perm[i] >= n writes zero bytes at i.  Moves the scene, optimizer state and
 * any other per-Gaussian array into the order perm gives. */
size_t gs_spatial_order_workspace_size(int64_t n);
int32_t gs_spatial_order(const float* means, int64_t n, uint32_t* perm, uint32_t* codes, void* ws, size_t ws_bytes,
                         void* stream);
int32_t gs_permute(const void* src, void* dst, int64_t planes, int64_t n, int32_t elem_bytes, const uint32_t* perm,
                   void* stream);

/* a5 (+a6) -- forward compositing, Eq. (1): per pixel, front to back over its
 * tile's list: alpha = min(alpha_max, opacity * G2D); skip when alpha <
 * alpha_min; stop before a Gaussian whose inclusion would take T below t_min;
 * w = alpha T; C += w c; imax = argmax w (first wins ties, Eq. (2)); depth per
 * depth_mode.  With GS_ACCUM_IMPORTANCE, acc (non-NULL) also receives the
 * importance / wmax / area sums (Sec. 3.2, Eq. (3), Sec. 5.1) of the same pass.
 * tile_order (from gs_bin_sort / gs_tile_order) may be NULL for natural order;
 * the same holds for the other compositing calls below. */
int32_t gs_render_forward(const gs_scene_t* scene, const gs_projected_t* proj, const uint32_t* vals,
                          const uint32_t* ranges, const uint32_t* tile_order, const gs_camera_t* cams, int32_t V,
                          const gs_opts_t* opts, const gs_fwd_out_t* out, const gs_accum_t* acc, void* stream);

/* a6 -- the accumulations alone (same decisions as gs_render_forward; no
 * per-pixel outputs): importance I_i (Sec. 3.2), wmax, area S_i (Eq. (3)).
 * opts->flags may carry GS_ACCUM_PER_VIEW. */
int32_t gs_accumulate_importance(const gs_projected_t* proj, const uint32_t* vals, const uint32_t* ranges,
                                 const uint32_t* tile_order, const gs_camera_t* cams, int32_t V, int64_t n,
                                 const gs_opts_t* opts, const gs_accum_t* acc, void* stream);

/* a7 + a8 -- backward of Eq. (1) and of the projection, restricted to an
 * active mask (region-prioritized optimisation, Sec. 5.2): per pixel, reverse
 * order from `last`, recomputing alpha with the forward's decisions; every
 * Gaussian updates the transmittance and the colour behind it, but only those
 * with active[i] != 0 (all when active == NULL) receive gradient.  dl_dcolor
 * [dev, 3][P]; t_final, last from gs_render_forward.  grad2d [dev, V*n][9]
 * receives d loss / d (u, v, a, b, c, opacity, r, g, b) per record (zeroed
 * first; rows of inactive Gaussians stay 0); grads receives the parameter
 * gradients summed over views (inactive rows 0). */
int32_t gs_render_backward(const gs_scene_t* scene, const gs_projected_t* proj, const uint32_t* vals,
                           const uint32_t* ranges, const uint32_t* tile_order, const gs_camera_t* cams, int32_t V,
                           const gs_opts_t* opts, const float* t_final, const uint32_t* last,
                           const float* dl_dcolor, const uint8_t* active, float* grad2d, const gs_grads_t* grads,
                           void* stream);

/* a7 alone: adds into grad2d (caller zeroes it). */
int32_t gs_render_backward_pixels(const gs_projected_t* proj, const uint32_t* vals, const uint32_t* ranges,
                                  const uint32_t* tile_order, const gs_camera_t* cams, int32_t V, int64_t n,
                                  const gs_opts_t* opts, const float* t_final, const uint32_t* last,
                                  const float* dl_dcolor, const uint8_t* active, float* grad2d, void* stream);

/* a7 with a deterministic reduction (Sec. 2.3 surveys how rasterizers reduce
 * the backward's gradient atomics; this variant orders the reduction instead
 * of only shortening it): the same result as gs_render_backward_pixels up to
 * float32 summation order, added into grad2d, but bitwise the same from run to
 * run for the same inputs and tile_order.  Each 4x4 pixel group's summed
 * partials of an entry are stored in that (entry, group) slot instead of being
 * added with float atomics; then per (tile, entry) the sixteen groups' slots
 * are added in group order, and per record its pairs' sums in emission order
 * (the tiles of its box, row-major, as gs_emit_keys emits them).  offsets
 * [dev, u32 V*n] and n_isect are those of the gs_bin_count call whose pairs
 * vals / ranges hold; ws [dev] sized by gs_render_backward_det_workspace_size
 * (n_isect) (616 bytes per pair: slot masks, sixteen 9-float slots, one
 * 9-float sum); n_isect < 2^32. */
size_t gs_render_backward_det_workspace_size(int64_t n_isect);
int32_t gs_render_backward_pixels_det(const gs_projected_t* proj, const uint32_t* vals, const uint32_t* ranges,
                                      const uint32_t* tile_order, const uint32_t* offsets, const gs_camera_t* cams,
                                      int32_t V, int64_t n, int64_t n_isect, const gs_opts_t* opts,
                                      const float* t_final, const uint32_t* last, const float* dl_dcolor,
                                      const uint8_t* active, float* grad2d, void* ws, size_t ws_bytes,
                                      void* stream);

/* a8 alone: chain rule of gs_project from grad2d to the parameters (written,
 * summed over views; rows with active[i] == 0 written as 0; records with
 * tiles_touched == 0 contribute nothing). */
int32_t gs_project_backward(const gs_scene_t* scene, const gs_projected_t* proj, const gs_camera_t* cams,
                            int32_t V, const gs_opts_t* opts, const float* grad2d, const uint8_t* active,
                            const gs_grads_t* grads, void* stream);

/* Mean absolute error loss and its gradient for a training step:
 * dl_dcolor[k] = sign(color[k] - target[k]) / count; *loss (device float) is
 * ADDED the mean |color - target| (caller zeroes it). */
int32_t gs_l1_loss_grad(const float* color, const float* target, int64_t count, float* dl_dcolor, float* loss,
                        void* stream);

/* Fill `count` 32-bit words with `value` (graph-capture-safe clear). */
int32_t gs_fill_u32(void* dst, uint32_t value, int64_t count, void* stream);

/* ------------------------------------------------------------------------ */
/* Criteria that consume the accumulations: culling and densification.      */
/* ------------------------------------------------------------------------ */

/* Keep-quantile threshold readings (Sec. 5.1 and Sec. 5.2 both filter with a
 * keep quantile of 0.99).  Over the m selected values:
 *  GS_THRESHOLD_MASS  (default reading): sort descending, prefix sums C_k,
 *      total S; tau = x_k for the k with C_k closest to keep * S (smaller k on
 *      a tie), so the values strictly above tau carry about keep of the total.
 *      Values are expected to be >= 0.
 *  GS_THRESHOLD_VALUE: tau = the (1 - keep) quantile of the values, linear
 *      interpolation between order statistics floor(h), floor(h) + 1 with
 *      h = (m - 1)(1 - keep).
 * tau is NaN when nothing is selected; NaN values give unspecified results. */
enum { GS_THRESHOLD_VALUE = 0, GS_THRESHOLD_MASS = 1 };

/* Device workspace of gs_visibility / gs_critical for `problems` thresholds
 * (V views, or 1); reused across calls, no clearing needed. */
size_t gs_select_workspace_size(int32_t problems);

/* Visibility of each view (Sec. 5.2): visible[k][i] = I_i^k > tau_k, where
 * tau_k is the keep-quantile threshold of view k's importances over the
 * Gaussians with I_i^k > 0.  importance [dev, V][n] (GS_ACCUM_PER_VIEW
 * layout); visible [dev, V][n] bytes 0/1 (all written); tau [dev, V] doubles.
 * keep in [0, 1] (GS_ERR_SHAPE otherwise).  The mask feeds gs_project's
 * cull_mask or the backward's `active` (view-dependent culling, Sec. 5.2). */
int32_t gs_visibility(const float* importance, int32_t V, int64_t n, double keep, int32_t mode, uint8_t* visible,
                      double* tau, void* ws, size_t ws_bytes, void* stream);

/* Critical Gaussians (Sec. 5.1): the set G_imax of Gaussians that provide the
 * largest blend weight of at least one pixel (area[i] > 0), filtered by the
 * keep-quantile threshold of their w_max: critical[i] = area[i] > 0 and
 * wmax[i] > tau.  area, wmax [dev, n] as accumulated by the forward pass;
 * critical [dev, n] bytes 0/1; tau [dev, 1] double. */
int32_t gs_critical(const uint32_t* area, const float* wmax, int64_t n, double keep, int32_t mode, uint8_t* critical,
                    double* tau, void* ws, size_t ws_bytes, void* stream);

/* Blur split criterion (Eq. (3)): split[i] = area[i] > theta * H * W, in
 * double precision; the paper's theta is 2e-4.  area [dev, n]; split [dev, n]. */
int32_t gs_blur_split(const uint32_t* area, int64_t n, double theta, int32_t height, int32_t width, uint8_t* split,
                      void* stream);

/* Positional-gradient statistics for the adaptive density control (Sec. 3.2):
 * for each Gaussian and each view where its record touches a tile, adds the
 * norm of d loss / d (u, v) scaled to image coordinates in [-1, 1]
 * (u by W / 2, v by H / 2) to norm_sum[i] and 1 to count[i].  grad2d
 * [dev, V*n][9] from the backward pass; norm_sum [dev, n] float, count
 * [dev, n] uint32, both accumulated (caller zeroes them). */
int32_t gs_grad_stats(const gs_projected_t* proj, const float* grad2d, const gs_camera_t* cams, int32_t V, int64_t n,
                      float* norm_sum, uint32_t* count, void* stream);

/* Writable scene planes [dev] in the gs_scene_t layout with plane stride
 * `capacity` (the output of gs_clone). */
typedef struct {
  float* means;
  float* scales;
  float* quats;
  float* opacity;
  float* sh;
  int64_t capacity;
} gs_scene_out_t;

/* Device workspace of gs_clone for n input Gaussians. */
size_t gs_clone_workspace_size(int64_t n);

/* Aggressive clone into two Gaussians (Sec. 5.1): every row i with
 * select[i] != 0 keeps its centre, rotation and SH and takes opacity
 * a' = 1 - sqrt(1 - a) and scales times a / (2 a' - a'^2 / sqrt 2) (covariance
 * times its square), computed in double; its copy goes to row n + r, r the
 * number of selected rows before i.  Unselected rows are copied unchanged.
 * out->capacity is the plane stride of the output (>= in->n, GS_ERR_CAPACITY
 * otherwise); copies beyond it are dropped, so size it in->n + the number of
 * selected rows.  All 48 SH planes are copied.  *count [dev int64] receives
 * the number of selected rows.  in and out must not overlap. */
int32_t gs_clone(const gs_scene_t* in, const uint8_t* select, const gs_scene_out_t* out, int64_t* count, void* ws,
                 size_t ws_bytes, void* stream);

/* Selection of the adaptive density control inherited from 3DGS (Sec. 3.2):
 * a Gaussian is selected when its mean screen-gradient norm
 * norm_sum[i] / count[i] (as accumulated by gs_grad_stats; computed in
 * double, rows with count 0 are never selected) is >= grad_threshold; a
 * selected Gaussian is cloned when its largest scale is <= scale_threshold
 * (3DGS: percent_dense * scene extent) and split otherwise.  norm_sum, count
 * [dev, n]; scales [dev, 3][n] (scene layout); clone, split [dev, n] bytes
 * 0/1, either may be NULL (not both). */
int32_t gs_densify_select(const float* norm_sum, const uint32_t* count, const float* scales, int64_t n,
                          double grad_threshold, double scale_threshold, uint8_t* clone, uint8_t* split,
                          void* stream);

/* Device workspace of gs_split for n input Gaussians. */
size_t gs_split_workspace_size(int64_t n);

/* Split into two children (the 3DGS split that the blur split of Sec. 4.1,
 * Eq. (3), and the density control apply): every row i with select[i] != 0
 * is replaced by two children c = 0, 1 with centre p + R diag(s) z_c, in
 * double, where R is the rotation of the normalised quaternion (w, x, y, z)
 * (identity for a zero quaternion) and z_c = (normals[c][0][i],
 * normals[c][1][i], normals[c][2][i]) are standard-normal draws supplied by
 * the caller [dev, 2][3][n]; the children's scales are the parent's divided
 * by `factor` (3DGS: 1.6, > 0 or GS_ERR_SHAPE); rotation, opacity and SH are
 * copied.  Output order: the unselected rows in index order (row i goes to
 * i - r, r the number of selected rows before i), then the children of the
 * r-th selected row at (n - m) + 2r + c, m = the number of selected rows,
 * written to *count [dev int64].  out->capacity is the output plane stride
 * (>= in->n, GS_ERR_CAPACITY otherwise; size it n + m); rows beyond it are
 * dropped.  in and out must not overlap. */
int32_t gs_split(const gs_scene_t* in, const uint8_t* select, const float* normals, double factor,
                 const gs_scene_out_t* out, int64_t* count, void* ws, size_t ws_bytes, void* stream);

/* Device workspace of gs_sample for n Gaussians. */
size_t gs_sample_workspace_size(int64_t n);

/* Redundant-Gaussian simplification (Sec. 4.2): intersection preserving keeps
 * the candidates with area[i] > 0 (the rendered indices of some view; all
 * Gaussians when area == NULL), and primitive sampling draws k of them without
 * replacement with probability proportional to importance[i].  The draw uses
 * exponential keys (Efraimidis and Spirakis, 2006): with expo[i] ~ Exp(1)
 * supplied by the caller, the k smallest keys expo[i] / importance[i]
 * (float32, IEEE division; ties to the lower index) are taken; Gaussians with
 * importance <= 0 are never drawn.  selected [dev, n] bytes 0/1 (all
 * written); *count [dev int64] = min(k, number of candidates). */
int32_t gs_sample(const float* importance, const uint32_t* area, const float* expo, int64_t n, int64_t k,
                  uint8_t* selected, int64_t* count, void* ws, size_t ws_bytes, void* stream);

/* Device workspace of gs_depth_points for `pixels` pixels over all views. */
size_t gs_depth_points_workspace_size(int64_t pixels);

/* Depth reinitialisation points (Sec. 4.1): every pixel with imax >= 0 (and
 * hit != 0 when require_hit) whose uniform draw u < rate is lifted to world
 * space, R^T (d ((x - cx) / fx, (y - cy) / fy, 1) - t) at the pixel centre
 * (x, y) = (px + 0.5, py + 0.5) with d its rendered depth (GS_DEPTH_MID is
 * the paper's), in double, and takes the target colour there.  Inputs are
 * [dev] per pixel over the V views in the gs_view_layout order (depth, imax,
 * hit and u [P], target [3][P]).  points and colors [dev, 3][capacity]
 * receive the points in pixel order; those beyond capacity are dropped;
 * *count [dev int64] = the number of qualifying pixels. */
int32_t gs_depth_points(const float* depth, const int32_t* imax, const uint8_t* hit, const float* target,
                        const float* u, const gs_camera_t* cams, int32_t V, double rate, int32_t require_hit,
                        float* points, float* colors, int64_t capacity, int64_t* count, void* ws, size_t ws_bytes,
                        void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MSPLAT_H */
