// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "device.hpp"
#include "salf.h"

namespace salf {

// ---- error reporting (thread-local message; see salf_last_error)
salf_status set_error(salf_status code, const char* fmt, ...);
salf_status check_hip(hipError_t e, const char* what);

// ---- scene workspace layout: [root grid][skip grid][levels][root bounds][nodes][node bounds][bounds scratch][hash keys]
//      [hash values][2 temp grids][counters][voxel boxes][activated corner values, pre-activated scenes only]
struct SceneLayout {
  int64_t n_root;        // root cells
  int64_t node_cap;      // internal nodes the workspace can hold
  int64_t hash_cap;      // hash slots (power of two)
  size_t root_off, skip_off, nodes_off, nbox_off, box_tmp_off, hkeys_off, hvals_off, tmp_off, counters_off;
  size_t order_off;  // node-numbering temporaries (0 when the scene can have no nodes)
  size_t lmax_off;   // finest voxel level per root cell
  size_t rbox_off;   // bounds of each root cell's voxels (uint2 per cell, zero for cells without a node)
  size_t vbox_off;   // each voxel's finest-cell box (int4: min corner, edge), for splatting
  size_t cell_off;   // the traversal's packed root-cell records (int4 per root cell)
  size_t act_geo_off, act_rgb_off, act_int_off;  // pre-activated scenes only (else 0)
  size_t total;
};
bool scene_layout(const salf_scene_desc& d, int64_t n_voxels, SceneLayout* out);

// Build counters written by the build kernels.
struct BuildCounters {
  int32_t error_bits;     // 1: voxel out of range, 2: overlap/duplicate, 4: hash table full
  int32_t first_bad;      // smallest offending voxel index
  int32_t n_nodes;        // internal nodes allocated
  int32_t n_occupied;     // occupied root cells
};

// Activated corner values: dst[i] = softplus(src[i]) for density, sigmoid for colour/intensity.
hipError_t launch_activate(const float* geo, const float* rgb, const float* inten, int64_t n_voxels, float* act_geo,
                           float* act_rgb, float* act_int, hipStream_t stream);

// Densification and pruning (Sec. 3.3) of a scene's n voxels into caller buffers of `capacity`
// rows: *total receives the refined count; nothing is written when it exceeds the capacity.  work:
// refine_work_bytes(n) bytes.  Blocks on `stream`.
size_t refine_work_bytes(int64_t n);
hipError_t launch_refine(const SceneView& v, const salf_scene_desc& d, int64_t n, const int32_t* vox,
                         const float* grad_rgb, double grad_threshold, double alpha_min, void* work,
                         int32_t* vox_out, float* geo_out, float* rgb_out, float* int_out, int64_t capacity,
                         int64_t* total, hipStream_t stream);

// Dense leaf indexes of a built scene: boff[cell] is the first entry of the cell's index or -1.
// Pack the traversal's root-cell records of v (v.cell) from its root codes, voxel bounds, skip
// distances, finest levels and dense-index offsets (v.boff, or none).
hipError_t launch_pack_cells(const SceneView& v, int64_t n_root, hipStream_t stream);
hipError_t launch_index_fill(const SceneView& v, int64_t n_root, const int32_t* boff, uint32_t* entries,
                             hipStream_t stream);

hipError_t launch_scene_build(const salf_scene_desc& d, int64_t n_voxels, const int32_t* voxels,
                              const SceneLayout& L, void* ws, hipStream_t stream);

// ---- rendering
struct RenderParams {
  SceneView scene;
  salf_sensor sensor;
  int32_t use_sensor;
  const float* ro;
  const float* rd;
  int64_t n;
  float t_near, t_far;
  int32_t S;
  float t_min;
  float bg[3];
  salf_outputs out;
  int32_t tiled;             // 1: waves take tiles of 64 rays of an img_w x img_h ray image
  int32_t img_w, img_h;
  int32_t tiles_x, tiles_y;
  int32_t tw_log2;           // tile width 2^tw_log2, height 64 >> tw_log2
  const int32_t* sched;      // optional tile schedule (header + order, see launch_tile_schedule)
  int32_t pieces;            // lanes per ray (1, 2, 4 or 8): > 1 shares each ray's root cells out
};

// int32 entries of the schedule buffer's header
constexpr int kSchedHeader = 64;

// Tiles (waves) of a launch: tiles_x * tiles_y when tiled, else groups of 64 consecutive rays.
__host__ __device__ inline int64_t tile_count(const RenderParams& p) {
  return p.tiled ? (int64_t)p.tiles_x * p.tiles_y : (p.n + 63) / 64;
}

// Logarithmic cost buckets of the tile schedule's counting sort.
constexpr int kCostBuckets = 256;

// Bytes of the tile-schedule buffer for n_tiles tiles (header, cost keys, order, histogram and
// cursors), and the schedule itself: cost estimates and a heaviest-first order of p's tiles
// written to `work`, tagged with p's ray layout.
constexpr size_t tile_work_bytes(int64_t n_tiles) {
  return kSchedHeader * 4 + 2 * ((((size_t)n_tiles * 4) + 255) & ~(size_t)255) + 2 * kCostBuckets * sizeof(uint32_t);
}
hipError_t launch_tile_schedule(const RenderParams& p, void* work, hipStream_t stream);

// Tile shape of a wave: 16 x 4 pixels for a pinhole camera, whose rows near the horizon differ more
// in path length (the distance at which they meet the ground) than its columns do; 32 columns x 2
// beams for a spinning LiDAR, for the same reason; 8 x 8 for a fisheye camera and for explicit
// rays with an image layout.
inline void set_tiling(RenderParams* p, int sensor_model) {
  p->tw_log2 = sensor_model == SALF_LIDAR_SPINNING ? 5 : (sensor_model == SALF_PINHOLE ? 4 : 3);
  const int tw = 1 << p->tw_log2, th = 64 >> p->tw_log2;
  p->tiles_x = (p->img_w + tw - 1) / tw;
  p->tiles_y = (p->img_h + th - 1) / th;
}

hipError_t launch_render(const RenderParams& p, int field, hipStream_t stream);

// A static scene (base.scene) with up to kMaxActors actors, each a scene placed by a rigid pose:
// a world point p is the actor point R^T (p - t) (R row-major).
constexpr int kMaxActors = 7;
struct ActorPose {
  SceneView view;
  float R[9];
  float t[3];
};
struct CompositeParams {
  RenderParams base;
  int32_t n_actors;
  int32_t pad;
  // slot[0]: the static scene, base.scene again (pose unused); slot[1 + a]: actor a.  One array, so
  // that a kernel indexes every walked scene the same way.
  ActorPose slot[kMaxActors + 1];
};
// Corner-field scenes, all with stored activated values (activated) or none.
hipError_t launch_composite(const CompositeParams& cp, bool activated, hipStream_t stream);

// One request of a batched launch (sensor mode, corner field).  variant: bit 0 colour, bit 1
// intensity, bit 2 pre-activated corner values.
struct BatchItem {
  RenderParams p;
  int64_t tile_begin;  // first global tile (wave) of this request
  int32_t variant;
  int32_t pad;
};
// d_items: device array of n_items requests sorted by tile_begin (the first begins at 0);
// d_counter: a zeroed device word the waves pull tiles from; d_sched: a batch schedule built by
// launch_batch_schedule for these items (or null: tiles in request order); variants: bit v set
// when some request has variant v.
hipError_t launch_render_batch(const BatchItem* d_items, int32_t n_items, int64_t n_tiles, uint32_t* d_counter,
                               const int32_t* d_sched, uint32_t variants, hipStream_t stream);
// Heaviest-first schedule of the n_tiles global tiles of a batch, in a buffer of
// tile_work_bytes(kBatchScheduleTiles) bytes.  Larger batches (more than about four 1920x1080
// frames) keep request order: their tail is short next to their length, and interleaving the
// tiles of many frames and scenes costs cache locality.
constexpr int64_t kBatchScheduleTiles = (int64_t)1 << 17;
hipError_t launch_batch_schedule(const BatchItem* d_items, int32_t n_items, int64_t n_tiles, void* work,
                                 hipStream_t stream);
// field < 0: every hit; else (the scene's field) stop after the voxel that leaves T < t_min, with S
// samples per voxel, as the render does.
hipError_t launch_trace(const SceneView& s, const salf_rays& r, int32_t max_hits, int field, int32_t S, float t_min,
                        int32_t* counts, int32_t* ids, float* t_in, float* t_out, hipStream_t stream);
// Total of rays cut short by their step budget on the current device since the library was loaded
// (read on `stream`, which is synchronized).
hipError_t read_cut_rays(hipStream_t stream, uint32_t* total);
// Default steps of a ray's walk (root steps, leaf passes and descents together) before it is cut short.
constexpr int32_t kDefaultStepBudget = 1 << 22;
hipError_t launch_raygen(const salf_sensor& s, float* o, float* d, float* t, uint8_t* valid, hipStream_t stream);

// Tile-based splatting of a global-shutter pinhole frame (raster.hip).
struct RasterParams {
  SceneView scene;
  const int4* vbox;                     // the scene's voxel boxes
  salf_sensor sensor;
  int64_t n_voxels;
  int32_t width, height, tiles_x, tiles_y;
  int32_t S;
  float t_min;
  float bg[3];
  salf_outputs out;
  double R[9], eye[3], fx, fy, cx, cy;  // camera pose and intrinsics for the projection (FP64)
  float og[3];                          // the eye in the FP32 grid frame of the interval rule
  int32_t eye_root[3];                  // its root cell, clamped to [-1, dims]
  int32_t key_bits, tile_bits;          // bits of the depth key and of the tile index in a pair key
  uint32_t* count;                      // [n_voxels + 1] tiles per voxel
  uint64_t* offset;                     // [n_voxels + 1] their exclusive scan
  uint2* rect;                          // [n_voxels] pixel rectangle: u0 | u1 << 16, r0 | r1 << 16
  uint64_t* vkey;                       // [n_voxels] depth key
  uint64_t* keys;                       // [pairs] tile << key_bits | depth key
  uint32_t* vals;                       // [pairs] voxel
};
// Fill the derived fields of p (eye, camera, tiling, key widths) from p->scene and p->sensor.
void raster_prepare(RasterParams* p);
// Work-area bytes for n voxels, n_tiles tiles and max_pairs pairs (queries the sort's temporary
// storage for the current device).
hipError_t raster_work_bytes(int64_t n_voxels, int64_t n_tiles, int64_t max_pairs, size_t* bytes);
// Render p's frame; blocks once on `stream` to read the pair count into *n_pairs and renders
// nothing when it exceeds *capacity, the pairs the work area holds.
hipError_t launch_raster(RasterParams p, int field, void* work, size_t work_bytes, int64_t* n_pairs,
                         int64_t* capacity, hipStream_t stream);
int64_t raster_capacity(int64_t n_voxels, int64_t n_tiles, size_t work_bytes);

struct BackwardParams {
  RenderParams fwd;
  salf_grads_in g;
  float* dgeo;
  float* drgb;
  float* dint;
  const int4* vbox;    // each voxel's finest-cell box (min corner, edge): hits read from fwd.out
  int32_t walk_only_unstored;  // walk only the rays whose hits were not all stored
};
// field: SALF_FIELD_CORNER or SALF_FIELD_PAPER (the scene's)
hipError_t launch_backward(const BackwardParams& p, int field, hipStream_t stream);

// A registered scene (the context's registry).
struct Scene {
  bool live = false;
  salf_scene_desc desc;
  int64_t n = 0;
  SceneLayout layout;
  SceneView view;
  const int4* vbox = nullptr;  // [n] each voxel's finest-cell min corner (x, y, z) and edge (w)
  BuildCounters counters;
};

}  // namespace salf

struct salf_context {
  int device = 0;
  std::mutex mu;
  std::vector<salf::Scene> scenes;
  int servers = 0;  // live servers on this context (under mu); the context outlives them
  void* static_sched = nullptr;  // device address of the library's own schedule array on `device`
  int32_t step_budget = salf::kDefaultStepBudget;  // per-ray walk steps (salf_set_step_budget)
  uint32_t cut_seen = 0;  // rays cut short on the device already reported by this context's salf_sync
};

namespace salf {
// Copy of a live scene's registry entry (under the context lock).  Errors: INVALID_ARG, NOT_FOUND.
salf_status scene_snapshot(salf_context* ctx, int32_t scene_id, Scene* out);
// Validation shared by the entry points.
salf_status validate_sensor(const salf_sensor* s);
salf_status validate_opts(const salf_render_opts* o);
// UNSUPPORTED when o asks for several lanes per ray (entry points whose kernels walk a ray with one lane).
salf_status one_lane_per_ray(const salf_render_opts* o, const char* what);
// The hit-list outputs of out: well formed, and asked only where supported (else UNSUPPORTED, `what`
// naming the entry point); reserved must be 0.
salf_status check_hit_outputs(const salf_outputs* out, bool supported, const char* what);
}  // namespace salf
