/*
 * salf.h - C ABI of the sparse-local-field ray-casting renderer for AMD Instinct MI355X (gfx950).
 *
 * The renderer implements the ray-casting mode of "SaLF: Sparse Local Fields for Multi-Sensor
 * Rendering in Real-Time" (arXiv 2507.18713):
 *   - a scene is a sparse set of non-overlapping cubic voxels on an adaptive grid: a regular root
 *     grid of edge s0 whose cells subdivide 8-way up to K levels, only non-empty voxels stored
 *     (Sec. 3.1 "Representation");
 *   - each voxel is a local field giving density and colour at normalized local coordinates
 *     x in [-1, 1]^3 (Sec. 3.1, Eq. 1-2);
 *   - a ray visits the occupied voxels it crosses front to back through an octree that skips
 *     empty space (Sec. 3.2, "Ray-Casting with Octree Acceleration"), samples each ray-voxel
 *     segment at midpoints and alpha-composites with alpha = 1 - exp(-sigma delta) (Eq. 3-4);
 *   - rays come from sensor intrinsics and extrinsics (Sec. 1), including fisheye cameras and
 *     camera and LiDAR rolling shutter (Sec. 5.3), and spinning LiDAR with intensity and an
 *     opacity used for ray drop (Sec. 5.3, Table III);
 *   - training needs the gradient of the rendered outputs (Sec. 4.2, Eq. 7).
 *
 * Conventions for every call
 *   - Every entry point returns salf_status: SALF_OK (0) or a negative error code.  The message
 *     of the last failure on the calling thread is returned by salf_last_error().  No C++
 *     exception crosses this interface.
 *   - GPU work is enqueued asynchronously on the caller's HIP stream (`void* stream` is a
 *     hipStream_t; NULL is the default stream).  Results are valid once that stream has
 *     synchronized.  Faults raised while kernels run surface at the next salf_sync().
 *   - Memory: every device buffer is owned by the caller (for example a torch tensor).  The
 *     library never frees caller memory and allocates no device memory of its own: internal
 *     structures live in caller-provided workspaces whose size is given by *_workspace_size().
 *     Device pointers must belong to the context's device and be 16-byte aligned.
 *   - Host structs passed by pointer are read during the call only.
 *
 * Geometry and units
 *   - World frame: metres, z up.  The scene grid spans origin + [0, root_dims * s0) per axis.
 *   - A voxel is (l, i, j, k): level l in [0, K] (0 = root cells of edge s0, K = finest edge
 *     s_K = s0 / 2^K) and integer coordinates in units of s_l = s0 / 2^l.
 *   - Finest-grid frame ("grid frame"): g = (p - org) * gs with gs = 2^K / s0.  The FP32 rule
 *     that decides which voxels a ray hits is, with every operation rounded to nearest even:
 *       org32 = (float)origin, gs32 = (float)((double)(1 << K) / s0),
 *       og = (o - org32) * gs32, dg = d * gs32, inv = 1 / dg   (per axis, FP32)
 *       an axis is parallel when dg == 0 or inv is infinite; for a parallel axis the voxel's
 *       slab is all t when lo <= og < hi and empty otherwise; for other axes it is
 *       [min(tlo, thi), max(tlo, thi)] with t = (P - og) * inv for the planes P = lo, hi
 *       (lo, hi = the voxel's integer bounds in finest cells);
 *       t_in = max(t_near, slab starts) (a zero t_in is +0), t_out = min(t_far, slab ends);
 *       the ray hits the voxel iff t_in < t_out.
 *     A ray with a non-finite component or with all three axes parallel hits nothing.
 *     Hits are ordered by t_in, which is strictly increasing along a ray.
 *   - Samples: each hit segment [t_in, t_out] is cut into S equal pieces sampled at their
 *     midpoints t_k = t_in + (k + 1/2) (t_out - t_in) / S; S = 1 is the paper's single
 *     midpoint per segment (Sec. 3.1, after Eq. 4).  Each piece is one compositing step.
 *
 * Parameter buffers (FP32, borrowed by a scene; they must outlive it and may be updated in
 * place between renders):
 *   geo [N, 8], rgb [N, 3, 8] (channel-major), intensity [N, 8]   (row = voxel id = upload index)
 *   SALF_FIELD_CORNER: raw logits at the 8 corners c = bx + 2 by + 4 bz (b = 0 on an axis's low
 *     face); density corners are softplus(z), colour and intensity corners sigmoid(z), and the
 *     activated corners are trilinearly interpolated at x.
 *   SALF_FIELD_PAPER (Eq. 1-2): sigma = exp(geo[0:4] . [x, 1]); colour channel ch =
 *     sigmoid(rgb[ch][0:3] . x + rgb[ch][3:7] . gamma(omega)) with the real spherical-harmonic
 *     basis gamma(omega) = (C0, C1 wx, C1 wy, C1 wz), C0 = 1/(2 sqrt(pi)), C1 = sqrt(3)/(2 sqrt(pi)),
 *     omega = the ray direction; intensity = sigmoid(intensity[0:4] . [x, 1]).  Unused entries of
 *     each 8-float row are ignored.
 *   SALF_FIELD_SDF (Eq. 5-6 with Eq. 2): signed distance s = geo[0:4] . [x, 1] and density
 *     sigma = a/2 + a/2 sign(s) (1 - exp(-|s| / b)) with a = exp(geo[4]), b = exp(geo[5]) (the
 *     voxel's SDF-to-density parameters, kept positive through their logarithms); colour and
 *     intensity as SALF_FIELD_PAPER.
 */
#ifndef SALF_H
#define SALF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SALF_ABI_VERSION 1

typedef int32_t salf_status;
enum {
  SALF_OK = 0,
  SALF_ERR_INVALID_ARG = -1,   /* a pointer, size, enum or geometry argument is invalid           */
  SALF_ERR_OUT_OF_MEMORY = -2, /* a caller-provided workspace is too small                          */
  SALF_ERR_DEVICE = -3,        /* a HIP call failed (launch error or a fault surfaced at sync)      */
  SALF_ERR_NOT_FOUND = -4,     /* unknown scene id or ticket                                        */
  SALF_ERR_BUDGET = -5,        /* a serving request alone exceeds the server's memory budget        */
  SALF_ERR_BUSY = -6,          /* the object still has work in flight                               */
  SALF_ERR_UNSUPPORTED = -7,   /* a valid but unimplemented combination                             */
  SALF_ERR_TRUNCATED = -8      /* salf_sync: some ray ran out of its traversal step budget           */
};

enum { SALF_FIELD_CORNER = 0, SALF_FIELD_PAPER = 1, SALF_FIELD_SDF = 2 };
enum { SALF_PINHOLE = 0, SALF_FISHEYE_EQUIDISTANT = 1, SALF_LIDAR_SPINNING = 2 };

#define SALF_MAX_LEVEL 8         /* K <= 8                                                         */
#define SALF_MAX_SAMPLES 32      /* S <= 32                                                        */
#define SALF_MAX_FINE_CELLS (1 << 20) /* root_dims[a] << K must stay below this, per axis           */

typedef struct salf_context salf_context;

/* ------------------------------------------------------------------ library and context */

/* SALF_ABI_VERSION of the loaded library. */
int32_t salf_abi_version(void);

/* Message of the last failed call on this thread ("" if none).  The pointer stays valid until
 * the next failing call on the same thread. */
const char* salf_last_error(void);

/* Create a context bound to HIP device `hip_device`.  *out receives the handle.
 * Errors: INVALID_ARG (bad device or NULL out), DEVICE. */
salf_status salf_create(int32_t hip_device, salf_context** out);

/* Destroy a context and forget its scenes (their workspaces stay owned by the caller).
 * Errors: INVALID_ARG, BUSY (a server created on it is still alive). */
salf_status salf_destroy(salf_context* ctx);

/* Synchronize `stream` and report any fault raised by kernels enqueued on it.  Also reports rays
 * that were cut short: every walk of a ray through a scene (render, backward, trace) takes at most
 * the context's step budget of steps (root-grid steps, leaf passes and octree descents together);
 * a ray that runs out composites only the hits found so far, and the first salf_sync of each
 * context on the device after such a launch has finished returns TRUNCATED with the number of such
 * rays since its previous report (the count is kept per device).  Errors: DEVICE, TRUNCATED. */
salf_status salf_sync(salf_context* ctx, void* stream);

/* Steps a ray's walk may take before it is cut short (default 2^22, far beyond any scene's needs:
 * a walk is bounded by the grid and the voxels it crosses).  Applies to calls made after this one;
 * mainly a diagnostic (a small budget forces the cut-short report).  Errors: INVALID_ARG (< 1). */
salf_status salf_set_step_budget(salf_context* ctx, int32_t steps);

/* ------------------------------------------------------------------ scenes (Sec. 3.1, 3.2) */

typedef struct {
  double origin[3];      /* world position of the grid's min corner (m)                             */
  double root_size;      /* s0, edge of a root cell (m), > 0                                         */
  int32_t root_dims[3];  /* root cells per axis, >= 1                                                */
  int32_t max_level;     /* K in [0, SALF_MAX_LEVEL]                                                 */
  int32_t field;         /* SALF_FIELD_CORNER, SALF_FIELD_PAPER or SALF_FIELD_SDF                    */
  int32_t flags;         /* 0 or SALF_SCENE_PREACTIVATE                                              */
} salf_scene_desc;

/* Corner field only: the build also stores activated corner values (softplus of the density
 * logits, sigmoid of the colour and intensity logits) in the workspace, and forward renders read
 * those instead of activating per hit.  The borrowed logits stay the scene's parameters (the
 * backward reads them); after updating them in place, call salf_scene_refresh before rendering.
 * The workspace grows by 4 B per stored corner value. */
#define SALF_SCENE_PREACTIVATE 1

typedef struct {
  int64_t n_voxels;
  int64_t n_nodes;          /* internal octree nodes built                                          */
  int64_t n_root_cells;     /* root_dims product                                                    */
  int64_t n_occupied_roots; /* root cells holding a voxel or a node                                 */
  size_t workspace_bytes;   /* bytes of the workspace in use                                        */
} salf_scene_stats;

/* Bytes of device workspace salf_scene_create needs for `n_voxels` voxels under `desc`.
 * Errors: INVALID_ARG (bad desc, n_voxels < 0 or > 2^30). */
salf_status salf_scene_workspace_size(const salf_scene_desc* desc, int64_t n_voxels, size_t* bytes);

/* Build the acceleration structure (a dense root grid whose cells point to 8-ary octrees whose
 * leaves are empty or hold one voxel, Sec. 3.2) on the GPU and register the scene.
 *   d_voxels   device int32 [n_voxels, 4] = (l, i, j, k), read during the call only
 *   d_geo      device float [n_voxels, 8]       borrowed (required)
 *   d_rgb      device float [n_voxels, 3, 8]    borrowed (NULL: the scene has no colour)
 *   d_int      device float [n_voxels, 8]       borrowed (NULL: the scene has no intensity)
 *              (a channel is present iff its pointer is non-NULL; with n_voxels == 0 the buffers
 *              are never read, but a non-NULL pointer still declares the channel)
 *   d_workspace, ws_bytes   caller memory of at least salf_scene_workspace_size() bytes; it
 *              holds the structure for the scene's lifetime and must not be touched meanwhile
 *   *scene_id  receives the new scene's id
 * The call blocks until the build has finished on `stream`, so that validation errors can be
 * returned.  Errors: INVALID_ARG (bad desc; a voxel with a level outside [0, K] or coordinates
 * outside the grid; two voxels that overlap or repeat; the message names the first offending
 * voxel index), OUT_OF_MEMORY (ws_bytes too small), DEVICE. */
salf_status salf_scene_create(salf_context* ctx, const salf_scene_desc* desc, int64_t n_voxels,
                              const int32_t* d_voxels, const float* d_geo, const float* d_rgb,
                              const float* d_int, void* d_workspace, size_t ws_bytes, void* stream,
                              int32_t* scene_id);

/* Recompute a SALF_SCENE_PREACTIVATE scene's activated corner values from its borrowed logits
 * (asynchronous on `stream`).  A no-op for other scenes.  Errors: NOT_FOUND, DEVICE. */
salf_status salf_scene_refresh(salf_context* ctx, int32_t scene_id, void* stream);

/* Statistics of a built scene.  Errors: NOT_FOUND. */
salf_status salf_scene_get_stats(salf_context* ctx, int32_t scene_id, salf_scene_stats* out);

/* Dense leaf index (optional; an acceleration of the octree walk of Sec. 3.2, same hits).  For
 * every root cell whose finest voxel level L is in [1, max_level], a 2^L x 2^L x 2^L array (x
 * fastest) of uint32 entries, one per level-L cell, names the octree region that holds that cell
 * (a voxel, or an empty child): bits 0-3 the region's level, bits 4-31 its voxel + 1 (0: empty).
 * Inside such a cell a ray then steps from region to region by one entry read instead of an
 * octree descent per voxel; the reported hits and their intervals are the same.  The memory is
 * caller-allocated: [int32 entry offset per root cell, -1 for cells without an index][entries].
 *
 * Exact bytes of the index of a built scene for `max_level` (copies the root grid to the host;
 * blocking).  Errors: NOT_FOUND, INVALID_ARG (max_level outside [0, SALF_MAX_INDEX_LEVEL], a scene
 * of 2^28 voxels or more), OUT_OF_MEMORY (more than 2^31 entries), DEVICE. */
#define SALF_MAX_INDEX_LEVEL 6
salf_status salf_scene_index_size(salf_context* ctx, int32_t scene_id, int32_t max_level, size_t* bytes);

/* Build the index into d_index (256-byte aligned, >= salf_scene_index_size() bytes, caller-owned,
 * not to be touched while the scene lives or until the index is replaced) on `stream` and block
 * until it is built; later renders, traces and backward passes of the scene use it.  max_level 0
 * drops the index.  Do not call it while work that reads the scene is in flight.  Errors: as
 * salf_scene_index_size, plus INVALID_ARG (misaligned d_index), OUT_OF_MEMORY (bytes too small). */
salf_status salf_scene_build_index(salf_context* ctx, int32_t scene_id, int32_t max_level, void* d_index,
                                   size_t bytes, void* stream);

/* Densification and pruning of a scene's voxel set (Sec. 3.3), producing the voxels and parameters
 * of a new scene (the caller builds it with salf_scene_create).  Voxel v is
 *   pruned  if its edge opacity 1 - exp(-sigma_max edge) is below alpha_min (the paper: 0.001), the
 *           opacity of a path one edge long at sigma_max, the largest of its 8 corner densities
 *           (where every field mode peaks); the paper does not say which opacity it thresholds;
 *   split   else, if level < K and the L1 norm of its colour-field gradient (all 24 colour logits
 *           of the corner field; rgb[ch][0:3] of the paper and SDF fields) exceeds grad_threshold,
 *           into its 8 octree-aligned children (child b = bx + 2 by + 4 bz at (2i + bx, 2j + by,
 *           2k + bz), level + 1), which carry the parent's field exactly: corner logits are the
 *           inverse activations of the parent's activated field at the child corners; affine
 *           forms halve their slopes and move their offsets (the colour's into the SH DC term);
 *   kept    otherwise.
 * Both decisions are taken in FP64.  Outputs keep the input order, children in the order of b. */
typedef struct {
  double grad_threshold;
  double alpha_min;
} salf_refine_opts;

/* Bytes of the device work area salf_refine needs for n_voxels.  Errors: INVALID_ARG. */
salf_status salf_refine_work_size(int64_t n_voxels, size_t* bytes);

/*   d_voxels    device int32 [N, 4], the voxels the scene was built from
 *   d_grad_rgb  device float [N, 3, 8] dL/d(colour parameters), or NULL (no splits)
 *   d_work      work area of salf_refine_work_size(N) bytes
 *   d_*_out     device outputs of `capacity` rows: int32 [cap, 4], float [cap, 8], [cap, 3, 8]
 *               (NULL if the scene has no colour), [cap, 8] (NULL if it has no intensity)
 *   *n_out      receives the refined voxel count.  If it exceeds `capacity`, nothing is written
 *               and OUT_OF_MEMORY is returned (call again with enough rows; capacity 0 queries).
 * Blocks until done on `stream`.  Errors: INVALID_ARG, NOT_FOUND, OUT_OF_MEMORY, DEVICE. */
salf_status salf_refine(salf_context* ctx, int32_t scene_id, const int32_t* d_voxels, const float* d_grad_rgb,
                        const salf_refine_opts* opts, void* d_work, size_t work_bytes, int32_t* d_voxels_out,
                        float* d_geo_out, float* d_rgb_out, float* d_int_out, int64_t capacity, int64_t* n_out,
                        void* stream);

/* Forget a scene.  Its workspace and parameter buffers may be freed by the caller once the
 * work that used them has completed.  Errors: NOT_FOUND. */
salf_status salf_scene_destroy(salf_context* ctx, int32_t scene_id);

/* ------------------------------------------------------------------ sensors (Sec. 1, 5.3) */

typedef struct {
  int32_t model;        /* SALF_PINHOLE | SALF_FISHEYE_EQUIDISTANT | SALF_LIDAR_SPINNING          */
  int32_t width;        /* camera: pixels per row; LiDAR: azimuth steps per sweep (columns)       */
  int32_t height;       /* camera: rows; LiDAR: beams                                              */
  float fx, fy, cx, cy; /* pinhole focal lengths / principal point (px); fisheye: f = fx            */
  float max_theta;      /* fisheye: rays with angle > max_theta from the axis are invalid (rad)   */
  float elev_min, elev_max; /* LiDAR: elevation of beam 0 and of beam height-1 (rad)              */
  float az0;            /* LiDAR: azimuth offset (rad)                                             */
  float t0;             /* time of camera row 0 / LiDAR column 0 (s)                              */
  float dt_line;        /* rolling shutter: time per camera row / LiDAR column (s); 0 = global   */
  float R0[9];          /* sensor-to-world rotation at t0, row-major                              */
  float p0[3];          /* sensor position at t0 (m)                                              */
  float v[3];           /* constant linear velocity (m/s, world)                                  */
  float w[3];           /* constant angular velocity (rad/s, world)                               */
  float t_near, t_far;  /* ray extent (m); 0 <= t_near < t_far; t_far may be +inf                 */
} salf_sensor;
/* Rays (float32, in this order of operations):
 *   pose at time t: p(t) = p0 + v (t - t0), R(t) = Exp([w]x (t - t0)) R0; camera row r is
 *   exposed at t0 + r dt_line, LiDAR column j fires at t0 + j dt_line (all beams together).
 *   pinhole pixel (u, r): d_cam = normalize((u + 1/2 - cx) / fx, (r + 1/2 - cy) / fy, 1)
 *   fisheye (equidistant, r = f theta): x = (u + 1/2 - cx) / f, y = (r + 1/2 - cy) / f,
 *     theta = |(x, y)|, d_cam = (sin theta * x / theta, sin theta * y / theta, cos theta),
 *     valid iff theta <= max_theta; invalid rays render the background with zero opacity
 *   LiDAR beam b, column j: e = elev_min + (elev_max - elev_min) b / (height - 1),
 *     a = az0 + 2 pi (j + 1/2) / width, d_s = (cos e cos a, cos e sin a, sin e)
 *   camera frame: x right, y down, z forward; LiDAR frame: x forward, y left, z up
 *   o = p(t), d = R(t) d_cam.  Ray index: camera r * width + u; LiDAR b * width + j. */

/* Number of rays of a sensor (width * height).  Errors: INVALID_ARG. */
salf_status salf_sensor_ray_count(const salf_sensor* sensor, int64_t* n_rays);

/* Materialize a sensor's rays: d_o, d_d float [n, 3], d_t float [n] (exposure time),
 * d_valid uint8 [n]; any of the four may be NULL.  Errors: INVALID_ARG, DEVICE. */
salf_status salf_generate_rays(salf_context* ctx, const salf_sensor* sensor, float* d_o, float* d_d,
                               float* d_t, uint8_t* d_valid, void* stream);

/* ------------------------------------------------------------------ rendering (Eq. 1-4) */

/* Explicit rays: device float [n, 3] origins and directions (unit length expected; depth is
 * measured in units of |d|).  All rays share [t_near, t_far].  image_width > 0 declares that the
 * rays form an image, row-major with that many rays per row (the last row may be short); the
 * renderer then gives each wave an 8x8 tile of them, as for a camera.  0 = no layout. */
typedef struct {
  const float* o;
  const float* d;
  int64_t n;
  float t_near, t_far;
  int32_t image_width;
  int32_t reserved;      /* must be 0 */
} salf_rays;

typedef struct {
  int32_t samples_per_voxel; /* S in [1, SALF_MAX_SAMPLES]; the workloads use 4, the paper 1        */
  float t_min;               /* a ray stops after the voxel that leaves T < t_min; 0 = never stop */
  float background[3];       /* added as T_end * background to the colour                           */
  int32_t schedule;          /* tile schedule: SALF_SCHEDULE_NONE, _BUILD or _REUSE (see below)      */
  void* d_work;              /* schedule buffer (salf_render_work_size bytes, 256-byte aligned)      */
  size_t work_bytes;         /* its size; both ignored with SALF_SCHEDULE_NONE                      */
  int32_t pieces;            /* lanes per ray: 0 or 1 = one; 2, 4 or 8 = see below                  */
  int32_t reserved;          /* must be 0                                                           */
} salf_render_opts;

/* Rays in pieces (opts->pieces = P in {2, 4, 8}; salf_render and salf_render_static only, other
 * entry points return UNSUPPORTED): P lanes share each ray.  Round by round, each lane walks the
 * next of the ray's occupied root cells in turn and composites it from T = 1 (Eq. 3-4 within the
 * cell); the P partial results are folded front to back into the ray (C += T C_j, D += T D_j,
 * I += T I_j, T *= T_j).  Where the fold would take T below t_min inside a cell, that cell is
 * composited again from the ray's state, so the ray stops after the same voxel as with one lane,
 * up to the FP32 rounding of T; outputs equal the one-lane render's to FP32 rounding, not bit for
 * bit.  The hits are those of the one-lane walk.  For launches with too few rays to fill the GPU
 * (a LiDAR sweep: 2,048 waves of 64 rays against 256 CUs), whose time is that of their longest
 * rays: P times the waves, each ray's cells walked side by side. */

/* Tile schedules.  A render runs one wave per 64-ray tile.  A schedule estimates every tile's
 * cost by walking its centre ray through the root grid (for each occupied root cell, the length
 * of the ray inside the bounds of the cell's voxels divided by the size of its finest voxels,
 * about the voxels it crosses) and orders the tiles heaviest first, which shortens the tail of
 * the launch; a launch whose tiles all fit on the GPU at once keeps its own order.  Outputs are
 * the same bits in any order.
 *   SALF_SCHEDULE_NONE  tiles in index order; d_work is not used
 *   SALF_SCHEDULE_BUILD salf_render / salf_render_backward build the schedule in d_work first
 *   SALF_SCHEDULE_REUSE use the schedule already in d_work (built by salf_render_schedule or an
 *                       earlier BUILD call); a schedule made for another ray layout (sensor size,
 *                       tiling) is ignored.  The scene and pose may differ: only speed depends on it.
 * Calls that may overlap must not share a buffer. */
enum { SALF_SCHEDULE_NONE = 0, SALF_SCHEDULE_BUILD = 1, SALF_SCHEDULE_REUSE = 2 };

/* Device bytes of the schedule buffer of a render of `sensor` or of explicit `rays` (exactly one
 * non-NULL).  Errors: INVALID_ARG. */
salf_status salf_render_work_size(const salf_sensor* sensor, const salf_rays* rays, size_t* bytes);

/* Build the tile schedule of a render of `sensor` or `rays` on scene `scene_id` into opts->d_work
 * (opts->schedule is not used), asynchronously on `stream`.  Errors: INVALID_ARG, NOT_FOUND, DEVICE. */
salf_status salf_render_schedule(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor,
                                 const salf_rays* rays, const salf_render_opts* opts, void* stream);

/* Per-ray outputs, device FP32 unless noted; a NULL pointer means "not wanted".
 *   rgb [n, 3]    C = sum w rgb + T_end * background   (Eq. 3)
 *   depth [n]     D = sum w t_k, expected range along the ray in metres (not divided by O)
 *   opacity [n]   O = 1 - T_end (the LiDAR ray-drop signal)
 *   intensity [n] I = sum w i (LiDAR intensity channel; needs a scene with intensity)
 *   t_end [n]     final transmittance T_end
 *   n_hits [n]    int32, voxels composited (the voxel that crossed t_min included)
 *   hit_voxel, hit_t: the composited hits (salf_render and salf_render_static, one lane per ray):
 *                 hit k of ray r (k < min(n_hits, hit_capacity)) at index k * n + r, hit_voxel
 *                 int32 [hit_capacity, n] its voxel, hit_t float [hit_capacity, n, 2] its t_in and
 *                 t_out; a ray's hits past hit_capacity are not stored (n_hits still counts
 *                 them).  Both or neither; hit_t 8-byte aligned; hit_capacity >= 1 when set.
 *                 salf_render_backward reads a ray's hits from them instead of walking the scene
 *                 again (rays with more hits than were stored are walked).  Other entry points
 *                 refuse them (UNSUPPORTED).
 * Colour needs a scene with colour.  Compositing runs in FP32 with FP32 transmittance. */
typedef struct {
  float* rgb;
  float* depth;
  float* opacity;
  float* intensity;
  float* t_end;
  int32_t* n_hits;
  int32_t* hit_voxel;
  float* hit_t;
  int32_t hit_capacity;
  int32_t reserved;      /* must be 0 */
} salf_outputs;

/* Render one sensor (sensor != NULL, rays == NULL; ray generation is fused into the render
 * kernel) or a batch of explicit rays (sensor == NULL, rays != NULL).  Output arrays have one
 * row per ray in the ray-index order above.  Errors: INVALID_ARG, NOT_FOUND, DEVICE. */
salf_status salf_render(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor,
                        const salf_rays* rays, const salf_render_opts* opts, const salf_outputs* out,
                        void* stream);

/* Render without any caller memory for the tile schedule: as salf_render with
 * opts->schedule = SALF_SCHEDULE_BUILD, except that the schedule is built in a fixed array the
 * library holds on each device (SALF_STATIC_SCHEDULE_BYTES, allocated once per process when the
 * library's code is loaded on that device, kept until the process ends).  For callers that cannot
 * allocate device memory during rendering: code under stream capture, tight serving loops, hosts
 * that forbid allocation.  The call allocates nothing (no hipMalloc, no library allocation);
 * opts->schedule, d_work and work_bytes are ignored.  Every call on a device shares that device's
 * array and overwrites it, so calls that overlap in time on one device (other streams, other
 * threads, other contexts of the device) race and must be serialized by the caller.  Outputs are
 * the same bits as salf_render's.  Errors: as salf_render, plus OUT_OF_MEMORY when the launch has
 * more than SALF_STATIC_SCHEDULE_TILES tiles of 64 rays (the array holds no larger schedule). */
#define SALF_STATIC_SCHEDULE_TILES (1 << 18)
#define SALF_STATIC_SCHEDULE_BYTES (2 * SALF_STATIC_SCHEDULE_TILES * 4 + 2304)
salf_status salf_render_static(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor,
                               const salf_rays* rays, const salf_render_opts* opts, const salf_outputs* out,
                               void* stream);

/* Several sensor renders in one launch: the 64-ray tiles of every item go out in one launch whose
 * waves pull tiles from a shared counter, ordered heaviest first across all items when they number
 * at most 2^17 (item order otherwise), so the long tiles of one sensor (a LiDAR's) start first and
 * the others' fill in around them.  Each item renders to the same bits as salf_render of it (the
 * same device function renders a tile).  Vehicles carry many sensors rendered at one time (Sec. 1).
 * Corner-field scenes only (raw or pre-activated), sensors only (no explicit rays). */
typedef struct {
  int32_t scene_id;
  int32_t reserved;             /* must be 0 */
  const salf_sensor* sensor;    /* read during the call */
  salf_render_opts opts;        /* samples, t_min, background; the schedule fields are not used */
  salf_outputs out;             /* as salf_render */
} salf_render_item;

/* Device bytes of salf_render_multi's work area for n_items items.  Errors: INVALID_ARG. */
salf_status salf_render_multi_work_size(int32_t n_items, size_t* bytes);

/* Render n_items (1..256) items in one launch on `stream`.  d_work: caller memory (256-byte aligned)
 * of salf_render_multi_work_size bytes, not shared by launches that may overlap.  Errors:
 * INVALID_ARG, NOT_FOUND, UNSUPPORTED (a paper-field or SDF scene), DEVICE. */
salf_status salf_render_multi(salf_context* ctx, int32_t n_items, const salf_render_item* items, void* d_work,
                              size_t work_bytes, void* stream);

/* ------------------------------------------------------------------ tile-based splatting (Sec. 3.2) */
/* Rasterization of a global-shutter pinhole frame ("Tile-based Splatting", Sec. 3.2): every voxel
 * is projected (its eight corners; culled when wholly behind the camera or off the image) and
 * listed under each 16 x 16-pixel tile its footprint rectangle overlaps (widened by 0.05 px; a voxel
 * reaching within 1 cm of the camera plane is listed under every tile); each tile's list is sorted
 * front to back; one workgroup per tile stages its voxels' boxes and parameter rows in LDS, and
 * each lane (one pixel) composites the voxels its ray meets under the interval rule, in list
 * order, with the shading and compositing of salf_render (Eq. 1-4).  The depth order is the
 * front-to-back order of the voxel grid seen from the eye (root cells by L1 distance from the
 * eye's root cell, then octant by octant relative to the eye's side of each mid-plane), which is
 * each pixel ray's own hit order, so the outputs are the same bits as salf_render of the sensor.
 * The paper sorts by depth without saying which; a centre-depth order would composite some
 * neighbouring voxels out of order.  A (voxel, tile) pair is one list entry. */

/* Device bytes of salf_render_raster's work area for a frame of `sensor` on scene `scene_id` with
 * up to max_pairs pairs (typically 1-4 per visible voxel).  Uses the device (the sort's temporary
 * storage depends on it).  Errors: INVALID_ARG, NOT_FOUND, UNSUPPORTED (not a global-shutter
 * pinhole), DEVICE. */
salf_status salf_raster_work_size(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor, int64_t max_pairs,
                                  size_t* bytes);

/* Render `sensor` by splatting.  sensor: SALF_PINHOLE whose rays share one pose (dt_line == 0, or v
 * and w zero); opts: samples, t_min and background as salf_render (the schedule fields are
 * ignored); out: as salf_render.  d_work: caller memory (256-byte aligned) of work_bytes.  The call
 * blocks once on `stream` to read the pair count back (the sort's size) and stores it in *n_pairs;
 * if the work area cannot hold that many pairs, nothing is rendered and OUT_OF_MEMORY is returned
 * (size it with salf_raster_work_size(*n_pairs) and call again).  The rest runs asynchronously on
 * `stream`.  Errors: INVALID_ARG, NOT_FOUND, UNSUPPORTED, OUT_OF_MEMORY, DEVICE. */
salf_status salf_render_raster(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor,
                               const salf_render_opts* opts, const salf_outputs* out, void* d_work, size_t work_bytes,
                               int64_t* n_pairs, void* stream);

/* ------------------------------------------------------------------ dynamic actors */
/* An actor: a scene in its own canonical frame placed by a rigid pose, a world point p being the
 * actor point R^T (p - t) (R row-major, orthonormal). */
typedef struct {
  int32_t scene_id;
  float R[9];
  float t[3];
} salf_actor;
#define SALF_MAX_ACTORS 7

/* Render a static scene together with up to SALF_MAX_ACTORS actors (the simulator's merged
 * traversal of a background and its moving actors, Sec. 4.1).  Per ray, each actor's root grid is met in
 * the actor's frame, where the ray is (R^T (o - t), R^T d) formed in FP32 in that order, every
 * operation rounded ((R[i] p0 + R[3 + i] p1) + R[6 + i] p2 per component); a rigid map keeps
 * the ray parameter, so every scene's intervals and depths share it.  The ray walks the static
 * scene up to the first actor box it meets, that actor over its box, the static scene up to the
 * next box, and so on to t_far, compositing every hit in that order as salf_render does.  Actors
 * must not overlap one another or static voxels (the background holds no voxel where an actor
 * is); otherwise hits are composited in that piecewise order, not sorted.  All scenes must use
 * the corner field, all with SALF_SCENE_PREACTIVATE or none, and hold every requested channel.
 * `sensor`/`rays`, `opts` (its schedule is built from the static scene) and `out` as salf_render.
 * Errors: INVALID_ARG, NOT_FOUND, UNSUPPORTED (another field), DEVICE. */
salf_status salf_render_composite(salf_context* ctx, int32_t static_scene_id, int32_t n_actors,
                                  const salf_actor* actors, const salf_sensor* sensor, const salf_rays* rays,
                                  const salf_render_opts* opts, const salf_outputs* out, void* stream);

/* The voxels each explicit ray hits, front to back (Sec. 3.2: the ray-voxel segments a render
 * composites):
 *   apply_early_termination 0: every hit of the ray (opts is not read);
 *                           1: the ray stops after the voxel that leaves T < opts->t_min, with
 *                              opts->samples_per_voxel samples per voxel and transmittance composited
 *                              exactly as salf_render does (only the density decides it), so the
 *                              list is the one a render of these rays shades and d_counts equals its
 *                              n_hits
 *   d_counts int32 [n]: hits of the ray (may exceed max_hits)
 *   d_ids int32 [n, max_hits]: voxel ids (upload index); d_t_in, d_t_out float [n, max_hits]
 * Entries past a ray's count are left untouched.  Errors: INVALID_ARG, NOT_FOUND, DEVICE. */
salf_status salf_trace_hits(salf_context* ctx, int32_t scene_id, const salf_rays* rays, int32_t max_hits,
                            int32_t apply_early_termination, const salf_render_opts* opts, int32_t* d_counts,
                            int32_t* d_ids, float* d_t_in, float* d_t_out, void* stream);

/* ------------------------------------------------------------------ differentiation (Eq. 7) */

/* Upstream gradients dL/d(output), device FP32, NULL = zero. */
typedef struct {
  const float* d_rgb;       /* [n, 3] */
  const float* d_depth;     /* [n]    */
  const float* d_opacity;   /* [n]    */
  const float* d_intensity; /* [n]    */
} salf_grads_in;

/* Gradient of a render w.r.t. the scene's raw parameters, accumulated (+=) into d_dgeo [N, 8],
 * d_drgb [N, 3, 8] and d_dint [N, 8] (NULL = not wanted; the caller zero-fills).  Corner field:
 * w.r.t. the corner logits.  Paper field (Eq. 1-2): w.r.t. the density's slopes and offset
 * (geo[0:4]), each colour channel's slopes and SH coefficients (rgb[ch][0:7]) and the
 * intensity's slopes and offset (int[0:4]); the unused slots receive nothing.
 * `sensor`/`rays`, `opts` and the scene parameters must be those of the forward call, and
 * `saved` must hold its t_end and n_hits (rgb/depth/intensity as well when their gradient is
 * requested).  The kernel re-traverses each ray and recomputes transmittance front to back; no
 * per-sample state is stored.  When `saved` also holds the forward's stored hits (hit_voxel,
 * hit_t, hit_capacity as the forward wrote them), a ray whose hits were all stored is not
 * traversed again: its hits are read in order (a second launch walks the other rays).  A SALF_SCENE_PREACTIVATE scene is read through its stored
 * activated values in both passes (salf_scene_refresh after changing the logits), softplus'
 * being taken as 1 - exp(-softplus); the gradient is w.r.t. the logits either way.  Lanes of a
 * wave that hit the same voxel add their contributions first; the rest is accumulated with FP32
 * atomics, so the summation order (and the last bits) vary between runs.  Errors: INVALID_ARG,
 * NOT_FOUND, DEVICE. */
salf_status salf_render_backward(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor,
                                 const salf_rays* rays, const salf_render_opts* opts,
                                 const salf_outputs* saved, const salf_grads_in* grads, float* d_dgeo,
                                 float* d_drgb, float* d_dint, void* stream);

/* ------------------------------------------------------------------ serving (continuous batching) */
/* A server renders sensor requests (a scene and a sensor each) for many sensors and resident scenes
 * with continuous batching: a scheduler thread inside the library admits queued requests in
 * arrival order as soon as their outputs fit in the caller's HBM pool, and each scheduling cycle
 * launches one batched kernel over every 64-ray tile of all requests admitted since the previous
 * launch; waves pull tiles from a counter, so requests of uneven ray counts share the GPU.  Up
 * to `max_inflight` launches run at once on separate streams, so requests that arrive while
 * others are on the GPU start without waiting for them.  A request's rays render to the same bits
 * as with salf_render (the same device function renders a tile in both).  Multi-sensor vehicles
 * motivate it: the paper notes vehicles carry more than 20 sensors (Sec. 1). */

typedef struct salf_server salf_server;

enum { SALF_OUT_RGB = 1, SALF_OUT_DEPTH = 2, SALF_OUT_OPACITY = 4, SALF_OUT_INTENSITY = 8 };

typedef struct {
  void* d_pool;          /* device memory the outputs of admitted requests are carved from           */
  size_t pool_bytes;     /* the HBM budget for outputs of requests in flight                          */
  void* d_work;          /* device memory for batch descriptors, >= salf_server_work_size() bytes    */
  size_t work_bytes;
  int32_t max_batch;     /* requests per launch, 1..256                                               */
  int32_t max_inflight;  /* launches in flight, 1..4                                                  */
  int64_t max_launch_rays; /* rays per launch under light load: a launch takes admitted requests in
                              order while their rays fit (at least one request), as long as the
                              admitted, unlaunched rays fit in max_inflight such launches; past
                              that backlog, launches take whole batches again.  A request
                              completes when its launch does, so capped launches complete small
                              sensors sooner.  0 = no cap; >= 0                                    */
} salf_server_opts;

typedef struct {
  int64_t submitted, completed, released, launches;
  size_t pool_in_use, pool_peak;   /* bytes of the pool held by admitted, unreleased requests       */
  int32_t queued, inflight;        /* requests waiting for admission / admitted and not yet done   */
} salf_server_stats;

/* Device bytes of the `d_work` buffer for `opts` (max_batch, max_inflight).  Errors: INVALID_ARG. */
salf_status salf_server_work_size(const salf_server_opts* opts, size_t* bytes);

/* Pool bytes a request of `sensor` with outputs `outputs` (SALF_OUT_* mask) occupies.
 * Errors: INVALID_ARG. */
salf_status salf_server_request_bytes(const salf_sensor* sensor, uint32_t outputs, size_t* bytes);

/* Create a server on ctx's device.  Pool and work buffers are caller memory, 256-byte aligned,
 * and must outlive the server.  Errors: INVALID_ARG, DEVICE. */
salf_status salf_server_create(salf_context* ctx, const salf_server_opts* opts, salf_server** out);

/* Queue a render of `sensor` on scene `scene_id` (corner field) with `opts`.  Non-blocking.  The
 * render runs on the server's own streams: work the caller enqueued on another stream that changes
 * the scene (parameter updates, salf_scene_refresh) must have finished before this call (synchronize
 * that stream first).  The scene (its workspace, index and parameter buffers) must stay alive and
 * unchanged until the request is done.  *ticket identifies the request.
 * Errors: INVALID_ARG, NOT_FOUND, UNSUPPORTED (paper or SDF field), BUDGET (its outputs alone exceed the
 * pool). */
salf_status salf_server_submit(salf_server* server, int32_t scene_id, const salf_sensor* sensor,
                               const salf_render_opts* opts, uint32_t outputs, uint64_t* ticket);

/* State of a request: *done = 1 once its outputs are complete in device memory; then `out` (if
 * not NULL) receives device pointers into the pool (rgb [n,3], depth/opacity/intensity [n] as
 * requested; t_end and n_hits NULL).  t_submit / t_done: CLOCK_MONOTONIC seconds at submission
 * and at the moment the scheduler saw the launch finish (t_done = 0 while not done).
 * Errors: NOT_FOUND. */
salf_status salf_server_poll(salf_server* server, uint64_t ticket, int32_t* done, salf_outputs* out,
                             double* t_submit, double* t_done);

/* Block until the request is done or `timeout_s` seconds pass (*done says which).  Errors: NOT_FOUND. */
salf_status salf_server_wait(salf_server* server, uint64_t ticket, double timeout_s, int32_t* done);

/* Return a done request's pool space (its output pointers become invalid); this may admit waiting
 * requests.  Errors: NOT_FOUND, BUSY (not done yet). */
salf_status salf_server_release(salf_server* server, uint64_t ticket);

salf_status salf_server_get_stats(salf_server* server, salf_server_stats* out);

/* Finish every queued and running request, stop the scheduler and free the server's host state
 * (pool and work buffers stay the caller's).  Errors: INVALID_ARG. */
salf_status salf_server_destroy(salf_server* server);

#ifdef __cplusplus
}
#endif

#endif /* SALF_H */
