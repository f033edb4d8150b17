// C ABI entry points: argument validation, the scene registry and kernel launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "internal.hpp"

namespace salf {

namespace {
thread_local char g_err[512] = "";
}

salf_status set_error(salf_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

salf_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return SALF_OK;
  return set_error(SALF_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace salf

using namespace salf;

namespace {

// RAII guard selecting the context's device for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// The tile-schedule array of salf_render_static: one copy per device, for the process's lifetime.
// Host code never uses this name as an address (on the host it only stands for the symbol): the
// device address is looked up once per context with hipGetSymbolAddress and kept in the context.
static_assert(tile_work_bytes(SALF_STATIC_SCHEDULE_TILES) == SALF_STATIC_SCHEDULE_BYTES, "static schedule size");
static __device__ __align__(256) uint8_t scratch[SALF_STATIC_SCHEDULE_BYTES];

salf_status validate_desc(const salf_scene_desc* d) {
  if (!d) return set_error(SALF_ERR_INVALID_ARG, "scene desc is NULL");
  if (!(d->root_size > 0.0) || !isfinite(d->root_size))
    return set_error(SALF_ERR_INVALID_ARG, "root_size must be finite and > 0");
  if (d->max_level < 0 || d->max_level > SALF_MAX_LEVEL)
    return set_error(SALF_ERR_INVALID_ARG, "max_level %d outside [0, %d]", d->max_level, SALF_MAX_LEVEL);
  for (int a = 0; a < 3; ++a) {
    if (!isfinite(d->origin[a])) return set_error(SALF_ERR_INVALID_ARG, "origin[%d] is not finite", a);
    if (d->root_dims[a] < 1) return set_error(SALF_ERR_INVALID_ARG, "root_dims[%d] must be >= 1", a);
    if (((int64_t)d->root_dims[a] << d->max_level) >= SALF_MAX_FINE_CELLS)
      return set_error(SALF_ERR_INVALID_ARG, "root_dims[%d] << max_level must be < %d", a, SALF_MAX_FINE_CELLS);
  }
  if (d->field != SALF_FIELD_CORNER && d->field != SALF_FIELD_PAPER && d->field != SALF_FIELD_SDF)
    return set_error(SALF_ERR_INVALID_ARG, "unknown field mode %d", d->field);
  if (d->flags & ~SALF_SCENE_PREACTIVATE) return set_error(SALF_ERR_INVALID_ARG, "unknown scene flags %d", d->flags);
  if ((d->flags & SALF_SCENE_PREACTIVATE) && d->field != SALF_FIELD_CORNER)
    return set_error(SALF_ERR_INVALID_ARG, "SALF_SCENE_PREACTIVATE applies to the corner field only");
  return SALF_OK;
}

}  // namespace

salf_status salf::validate_sensor(const salf_sensor* s) {
  if (!s) return set_error(SALF_ERR_INVALID_ARG, "sensor is NULL");
  if (s->model != SALF_PINHOLE && s->model != SALF_FISHEYE_EQUIDISTANT && s->model != SALF_LIDAR_SPINNING)
    return set_error(SALF_ERR_INVALID_ARG, "unknown sensor model %d", s->model);
  if (s->width < 1 || s->height < 1) return set_error(SALF_ERR_INVALID_ARG, "sensor width and height must be >= 1");
  if ((int64_t)s->width * s->height > ((int64_t)1 << 31))
    return set_error(SALF_ERR_INVALID_ARG, "sensor has more than 2^31 rays");
  if (s->model != SALF_LIDAR_SPINNING) {
    if (!(s->fx != 0.0f) || !isfinite(s->fx)) return set_error(SALF_ERR_INVALID_ARG, "fx must be finite and nonzero");
    if (s->model == SALF_PINHOLE && (!(s->fy != 0.0f) || !isfinite(s->fy)))
      return set_error(SALF_ERR_INVALID_ARG, "fy must be finite and nonzero");
  }
  if (!(s->t_near >= 0.0f) || !(s->t_near < s->t_far))
    return set_error(SALF_ERR_INVALID_ARG, "need 0 <= t_near < t_far");
  return SALF_OK;
}

namespace {

salf_status validate_rays(const salf_rays* r) {
  if (!r) return set_error(SALF_ERR_INVALID_ARG, "rays is NULL");
  if (r->n < 0 || r->n > ((int64_t)1 << 31)) return set_error(SALF_ERR_INVALID_ARG, "ray count out of range");
  if (r->n > 0 && (!r->o || !r->d)) return set_error(SALF_ERR_INVALID_ARG, "ray origin/direction pointer is NULL");
  if (!(r->t_near >= 0.0f) || !(r->t_near < r->t_far))
    return set_error(SALF_ERR_INVALID_ARG, "need 0 <= t_near < t_far");
  if (r->image_width < 0 || r->reserved != 0)
    return set_error(SALF_ERR_INVALID_ARG, "image_width must be >= 0 and reserved 0");
  return SALF_OK;
}

}  // namespace

salf_status salf::validate_opts(const salf_render_opts* o) {
  if (!o) return set_error(SALF_ERR_INVALID_ARG, "render opts is NULL");
  if (o->samples_per_voxel < 1 || o->samples_per_voxel > SALF_MAX_SAMPLES)
    return set_error(SALF_ERR_INVALID_ARG, "samples_per_voxel %d outside [1, %d]", o->samples_per_voxel,
                     SALF_MAX_SAMPLES);
  if (!(o->t_min >= 0.0f) || !(o->t_min <= 1.0f)) return set_error(SALF_ERR_INVALID_ARG, "t_min must be in [0, 1]");
  if (o->schedule < SALF_SCHEDULE_NONE || o->schedule > SALF_SCHEDULE_REUSE)
    return set_error(SALF_ERR_INVALID_ARG, "schedule must be SALF_SCHEDULE_NONE, _BUILD or _REUSE");
  if (o->pieces != 0 && o->pieces != 1 && o->pieces != 2 && o->pieces != 4 && o->pieces != 8)
    return set_error(SALF_ERR_INVALID_ARG, "pieces must be 0, 1, 2, 4 or 8");
  if (o->reserved != 0) return set_error(SALF_ERR_INVALID_ARG, "reserved must be 0");
  return SALF_OK;
}

salf_status salf::check_hit_outputs(const salf_outputs* out, bool supported, const char* what) {
  if (!out) return SALF_OK;
  if (out->reserved != 0) return set_error(SALF_ERR_INVALID_ARG, "outputs: reserved must be 0");
  if (!out->hit_voxel && !out->hit_t) return SALF_OK;
  if (!supported) return set_error(SALF_ERR_UNSUPPORTED, "%s store no hit lists", what);
  if (!out->hit_voxel || !out->hit_t) return set_error(SALF_ERR_INVALID_ARG, "hit_voxel and hit_t go together");
  if (out->hit_capacity < 1) return set_error(SALF_ERR_INVALID_ARG, "hit_capacity must be >= 1");
  if (((uintptr_t)out->hit_voxel & 3u) || ((uintptr_t)out->hit_t & 7u))
    return set_error(SALF_ERR_INVALID_ARG, "hit_voxel must be 4-byte and hit_t 8-byte aligned");
  return SALF_OK;
}

salf_status salf::one_lane_per_ray(const salf_render_opts* o, const char* what) {
  if (o && o->pieces > 1) return set_error(SALF_ERR_UNSUPPORTED, "%s walk each ray with one lane (pieces <= 1)", what);
  return SALF_OK;
}

salf_status salf::scene_snapshot(salf_context* ctx, int32_t id, Scene* out) {
  if (!ctx) return set_error(SALF_ERR_INVALID_ARG, "context is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (id < 0 || id >= (int32_t)ctx->scenes.size() || !ctx->scenes[id].live)
    return set_error(SALF_ERR_NOT_FOUND, "no scene with id %d", id);
  *out = ctx->scenes[id];
  out->view.step_budget = ctx->step_budget;
  return SALF_OK;
}

namespace {


// The rays of a launch (sensor or explicit rays) and their tiling.
salf_status ray_layout(const salf_sensor* sensor, const salf_rays* rays, RenderParams* p) {
  salf_status st;
  if ((sensor == nullptr) == (rays == nullptr))
    return set_error(SALF_ERR_INVALID_ARG, "pass exactly one of sensor and rays");
  if (sensor) {
    if ((st = validate_sensor(sensor))) return st;
    p->sensor = *sensor;
    p->use_sensor = 1;
    p->tiled = 1;
    p->img_w = sensor->width;
    p->img_h = sensor->height;
    p->n = (int64_t)sensor->width * sensor->height;
  } else {
    if ((st = validate_rays(rays))) return st;
    p->ro = rays->o;
    p->rd = rays->d;
    p->n = rays->n;
    p->t_near = rays->t_near;
    p->t_far = rays->t_far;
    if (rays->image_width > 0) {
      p->tiled = 1;
      p->img_w = rays->image_width;
      p->img_h = (int32_t)((rays->n + rays->image_width - 1) / rays->image_width);
    }
    if (p->n > 0 && ((((uintptr_t)rays->o) & 3u) || (((uintptr_t)rays->d) & 3u)))
      return set_error(SALF_ERR_INVALID_ARG, "ray buffers must be 4-byte aligned");
  }
  set_tiling(p, sensor ? sensor->model : -1);
  return SALF_OK;
}

// The schedule buffer of opts must hold the schedule of p's tiles.
salf_status check_work(const salf_render_opts* opts, const RenderParams& p) {
  const size_t need = tile_work_bytes(tile_count(p));
  if (!opts->d_work) return set_error(SALF_ERR_INVALID_ARG, "a tile schedule needs a work buffer");
  if (opts->work_bytes < need)
    return set_error(SALF_ERR_INVALID_ARG, "work buffer holds %zu bytes; the tile schedule needs %zu",
                     opts->work_bytes, need);
  if ((uintptr_t)opts->d_work & 255u) return set_error(SALF_ERR_INVALID_ARG, "work buffer must be 256-byte aligned");
  return SALF_OK;
}

// Fill the parts of RenderParams shared by render and backward.
salf_status prepare_render(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor, const salf_rays* rays,
                           const salf_render_opts* opts, RenderParams* p, int* field) {
  Scene sc;
  salf_status st = scene_snapshot(ctx, scene_id, &sc);
  if (st) return st;
  if ((st = validate_opts(opts))) return st;
  memset(p, 0, sizeof(*p));
  if ((st = ray_layout(sensor, rays, p))) return st;
  p->scene = sc.view;
  if (opts->schedule != SALF_SCHEDULE_NONE) {
    if ((st = check_work(opts, *p))) return st;
    p->sched = (const int32_t*)opts->d_work;
  }
  p->S = opts->samples_per_voxel;
  p->t_min = opts->t_min;
  for (int c = 0; c < 3; ++c) p->bg[c] = opts->background[c];
  p->pieces = opts->pieces > 1 ? opts->pieces : 1;
  *field = sc.desc.field;
  return SALF_OK;
}

}  // namespace

namespace {
// Entry offsets of the dense leaf indexes of a scene's root cells whose finest voxel level is in
// [1, max_level] (-1 for the other cells), from the built root grid, and their entry count.
salf_status index_plan(salf_context* ctx, const Scene& sc, int32_t max_level, std::vector<int32_t>* boff,
                       int64_t* entries) {
  const int64_t n_root = sc.layout.n_root;
  std::vector<int32_t> root((size_t)n_root), lmax((size_t)n_root);
  DeviceGuard g(ctx->device);
  if (!g.ok) return set_error(SALF_ERR_DEVICE, "cannot select device %d", ctx->device);
  salf_status st;
  if ((st = check_hip(hipMemcpy(root.data(), sc.view.root, n_root * 4, hipMemcpyDeviceToHost), "copy root grid")))
    return st;
  if ((st = check_hip(hipMemcpy(lmax.data(), sc.view.lmax, n_root * 4, hipMemcpyDeviceToHost), "copy levels")))
    return st;
  boff->assign((size_t)n_root, -1);
  int64_t total = 0;
  for (int64_t i = 0; i < n_root; ++i) {
    if (root[i] < 0 || lmax[i] < 1 || lmax[i] > max_level) continue;
    (*boff)[i] = (int32_t)total;
    total += (int64_t)1 << (3 * lmax[i]);
    if (total > INT32_MAX) return set_error(SALF_ERR_OUT_OF_MEMORY, "dense leaf index exceeds 2^31 entries");
  }
  *entries = total;
  return SALF_OK;
}

size_t index_bytes(int64_t n_root, int64_t entries) { return ((size_t)n_root * 4 + 255) / 256 * 256 + (size_t)entries * 4; }

salf_status check_index_args(salf_context* ctx, int32_t scene_id, int32_t max_level, Scene* sc) {
  salf_status st = scene_snapshot(ctx, scene_id, sc);
  if (st) return st;
  if (max_level < 0 || max_level > SALF_MAX_INDEX_LEVEL)
    return set_error(SALF_ERR_INVALID_ARG, "index level %d outside [0, %d]", max_level, SALF_MAX_INDEX_LEVEL);
  if (sc->n >= ((int64_t)1 << 28)) return set_error(SALF_ERR_INVALID_ARG, "a dense leaf index holds < 2^28 voxels");
  return SALF_OK;
}

// Set a scene's index pointers, under the lock, if the scene is still the one `snap` was taken of
// (it may have been destroyed, and its id reused, while the index was built).
salf_status attach_index(salf_context* ctx, int32_t scene_id, const Scene& snap, const int32_t* boff,
                         const uint32_t* entries) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].live ||
      ctx->scenes[scene_id].view.root != snap.view.root)
    return set_error(SALF_ERR_NOT_FOUND, "scene %d was destroyed while its index was built", scene_id);
  ctx->scenes[scene_id].view.boff = boff;
  ctx->scenes[scene_id].view.cidx = entries;
  return SALF_OK;
}
}  // namespace

extern "C" {

int32_t salf_abi_version(void) { return SALF_ABI_VERSION; }

const char* salf_last_error(void) { return g_err; }

salf_status salf_create(int32_t hip_device, salf_context** out) {
  if (!out) return set_error(SALF_ERR_INVALID_ARG, "out is NULL");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count)
    return set_error(SALF_ERR_INVALID_ARG, "no HIP device %d (found %d)", hip_device, count);
  void* sched = nullptr;
  {
    DeviceGuard g(hip_device);
    if (!g.ok) return set_error(SALF_ERR_DEVICE, "cannot select device %d", hip_device);
    salf_status st = check_hip(hipGetSymbolAddress(&sched, HIP_SYMBOL(scratch)), "static schedule address");
    if (st) return st;
  }
  salf_context* c = new (std::nothrow) salf_context();
  if (!c) return set_error(SALF_ERR_OUT_OF_MEMORY, "host allocation failed");
  c->device = hip_device;
  c->static_sched = sched;
  *out = c;
  return SALF_OK;
}

salf_status salf_destroy(salf_context* ctx) {
  if (!ctx) return set_error(SALF_ERR_INVALID_ARG, "context is NULL");
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->servers > 0) return set_error(SALF_ERR_BUSY, "%d server(s) still use this context", ctx->servers);
  }
  delete ctx;
  return SALF_OK;
}

salf_status salf_sync(salf_context* ctx, void* stream) {
  if (!ctx) return set_error(SALF_ERR_INVALID_ARG, "context is NULL");
  DeviceGuard g(ctx->device);
  salf_status st = check_hip(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
  if (st) return st;
  if ((st = check_hip(hipGetLastError(), "kernel execution"))) return st;
  uint32_t total = 0;
  if ((st = check_hip(read_cut_rays((hipStream_t)stream, &total), "reading the cut-ray count"))) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (total != ctx->cut_seen) {
    const uint32_t fresh = total - ctx->cut_seen;
    ctx->cut_seen = total;
    return set_error(SALF_ERR_TRUNCATED, "%u ray(s) ran out of their traversal step budget (%d steps) and were cut short",
                     fresh, ctx->step_budget);
  }
  return SALF_OK;
}

salf_status salf_set_step_budget(salf_context* ctx, int32_t steps) {
  if (!ctx) return set_error(SALF_ERR_INVALID_ARG, "context is NULL");
  if (steps < 1) return set_error(SALF_ERR_INVALID_ARG, "the step budget must be >= 1");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->step_budget = steps;
  return SALF_OK;
}

salf_status salf_scene_workspace_size(const salf_scene_desc* desc, int64_t n_voxels, size_t* bytes) {
  salf_status st = validate_desc(desc);
  if (st) return st;
  if (!bytes) return set_error(SALF_ERR_INVALID_ARG, "bytes is NULL");
  if (n_voxels < 0 || n_voxels > ((int64_t)1 << 30)) return set_error(SALF_ERR_INVALID_ARG, "n_voxels out of range");
  SceneLayout L;
  scene_layout(*desc, n_voxels, &L);
  *bytes = L.total;
  return SALF_OK;
}

salf_status salf_scene_create(salf_context* ctx, const salf_scene_desc* desc, int64_t n_voxels,
                              const int32_t* d_voxels, const float* d_geo, const float* d_rgb, const float* d_int,
                              void* d_workspace, size_t ws_bytes, void* stream, int32_t* scene_id) {
  if (!ctx) return set_error(SALF_ERR_INVALID_ARG, "context is NULL");
  salf_status st = validate_desc(desc);
  if (st) return st;
  if (!scene_id) return set_error(SALF_ERR_INVALID_ARG, "scene_id is NULL");
  if (n_voxels < 0 || n_voxels > ((int64_t)1 << 30)) return set_error(SALF_ERR_INVALID_ARG, "n_voxels out of range");
  if (n_voxels > 0 && (!d_voxels || !d_geo)) return set_error(SALF_ERR_INVALID_ARG, "voxels and geo are required");
  if (!d_workspace) return set_error(SALF_ERR_INVALID_ARG, "workspace is NULL");
  const void* ptrs[5] = {d_voxels, d_geo, d_rgb, d_int, d_workspace};
  for (const void* q : ptrs)
    if (q && !aligned16(q)) return set_error(SALF_ERR_INVALID_ARG, "device buffers must be 16-byte aligned");
  SceneLayout L;
  scene_layout(*desc, n_voxels, &L);
  if (ws_bytes < L.total)
    return set_error(SALF_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, the scene needs %zu", ws_bytes, L.total);
  DeviceGuard g(ctx->device);
  if (!g.ok) return set_error(SALF_ERR_DEVICE, "cannot select device %d", ctx->device);
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_hip(launch_scene_build(*desc, n_voxels, d_voxels, L, d_workspace, s), "scene build launch")))
    return st;
  BuildCounters c;
  if ((st = check_hip(hipMemcpyAsync(&c, (char*)d_workspace + L.counters_off, sizeof(c), hipMemcpyDeviceToHost, s),
                      "copy build counters")))
    return st;
  if ((st = check_hip(hipStreamSynchronize(s), "scene build"))) return st;
  if (c.error_bits & 1)
    return set_error(SALF_ERR_INVALID_ARG, "voxel %d has a level outside [0, %d] or coordinates outside the grid",
                     c.first_bad, desc->max_level);
  if (c.error_bits & 2)
    return set_error(SALF_ERR_INVALID_ARG, "voxel %d overlaps or repeats another voxel", c.first_bad);
  if (c.error_bits & 4) return set_error(SALF_ERR_OUT_OF_MEMORY, "node table overflow during the scene build");

  Scene sc;
  sc.live = true;
  sc.desc = *desc;
  sc.n = n_voxels;
  sc.layout = L;
  sc.counters = c;
  SceneView& v = sc.view;
  v.root = (const int32_t*)((char*)d_workspace + L.root_off);
  v.nodes = (const int32_t*)((char*)d_workspace + L.nodes_off);
  v.skip = (const uint8_t*)((char*)d_workspace + L.skip_off);
  v.nbox = (const uint2*)((char*)d_workspace + L.nbox_off);
  v.lmax = (const int32_t*)((char*)d_workspace + L.lmax_off);
  v.rbox = (const uint2*)((char*)d_workspace + L.rbox_off);
  sc.vbox = (const int4*)((char*)d_workspace + L.vbox_off);
  v.cell = (const int4*)((char*)d_workspace + L.cell_off);
  v.boff = nullptr;
  v.cidx = nullptr;
  v.act_geo = v.act_rgb = v.act_int = nullptr;
  if (desc->flags & SALF_SCENE_PREACTIVATE) {
    v.act_geo = (const float*)((char*)d_workspace + L.act_geo_off);
    v.act_rgb = d_rgb ? (const float*)((char*)d_workspace + L.act_rgb_off) : nullptr;
    v.act_int = d_int ? (const float*)((char*)d_workspace + L.act_int_off) : nullptr;
    if ((st = check_hip(launch_activate(d_geo, d_rgb, d_int, n_voxels, (float*)v.act_geo, (float*)v.act_rgb,
                                        (float*)v.act_int, s),
                        "activation launch")))
      return st;
  }
  v.geo = d_geo;
  v.rgb = d_rgb;
  v.inten = d_int;
  for (int a = 0; a < 3; ++a) {
    v.dims[a] = desc->root_dims[a];
    v.org[a] = desc->origin[a];
    v.org32[a] = (float)desc->origin[a];
  }
  v.K = desc->max_level;
  v.gs = (double)(1 << desc->max_level) / desc->root_size;
  v.gs32 = (float)v.gs;
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (size_t i = 0; i < ctx->scenes.size(); ++i) {
    if (!ctx->scenes[i].live) {
      ctx->scenes[i] = sc;
      *scene_id = (int32_t)i;
      return SALF_OK;
    }
  }
  ctx->scenes.push_back(sc);
  *scene_id = (int32_t)(ctx->scenes.size() - 1);
  return SALF_OK;
}

salf_status salf_scene_refresh(salf_context* ctx, int32_t scene_id, void* stream) {
  Scene sc;
  salf_status st = scene_snapshot(ctx, scene_id, &sc);
  if (st) return st;
  const SceneView& v = sc.view;
  if (v.act_geo == nullptr) return SALF_OK;
  DeviceGuard g(ctx->device);
  return check_hip(launch_activate(v.geo, v.rgb, v.inten, sc.n, (float*)v.act_geo, (float*)v.act_rgb,
                                   (float*)v.act_int, (hipStream_t)stream),
                   "activation launch");
}

salf_status salf_scene_get_stats(salf_context* ctx, int32_t scene_id, salf_scene_stats* out) {
  Scene sc;
  salf_status st = scene_snapshot(ctx, scene_id, &sc);
  if (st) return st;
  if (!out) return set_error(SALF_ERR_INVALID_ARG, "out is NULL");
  out->n_voxels = sc.n;
  out->n_nodes = sc.counters.n_nodes;
  out->n_root_cells = sc.layout.n_root;
  out->n_occupied_roots = sc.counters.n_occupied;
  out->workspace_bytes = sc.layout.total;
  return SALF_OK;
}

salf_status salf_scene_index_size(salf_context* ctx, int32_t scene_id, int32_t max_level, size_t* bytes) {
  Scene sc;
  salf_status st = check_index_args(ctx, scene_id, max_level, &sc);
  if (st) return st;
  if (!bytes) return set_error(SALF_ERR_INVALID_ARG, "bytes is NULL");
  std::vector<int32_t> boff;
  int64_t entries = 0;
  if ((st = index_plan(ctx, sc, max_level, &boff, &entries))) return st;
  *bytes = index_bytes(sc.layout.n_root, entries);
  return SALF_OK;
}

salf_status salf_scene_build_index(salf_context* ctx, int32_t scene_id, int32_t max_level, void* d_index,
                                   size_t bytes, void* stream) {
  Scene sc;
  salf_status st = check_index_args(ctx, scene_id, max_level, &sc);
  if (st) return st;
  if (max_level == 0) {
    // the traversal's root-cell records lose their index offsets, then the scene its index
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(SALF_ERR_DEVICE, "cannot select device %d", ctx->device);
    SceneView v = sc.view;
    v.boff = nullptr;
    if ((st = check_hip(launch_pack_cells(v, sc.layout.n_root, (hipStream_t)stream), "cell records launch")) ||
        (st = check_hip(hipStreamSynchronize((hipStream_t)stream), "cell records")))
      return st;
    return attach_index(ctx, scene_id, sc, nullptr, nullptr);
  }
  if (!d_index || ((uintptr_t)d_index & 255u)) return set_error(SALF_ERR_INVALID_ARG, "index must be 256-byte aligned");
  std::vector<int32_t> boff;
  int64_t entries = 0;
  if ((st = index_plan(ctx, sc, max_level, &boff, &entries))) return st;
  const int64_t n_root = sc.layout.n_root;
  const size_t need = index_bytes(n_root, entries);
  if (bytes < need) return set_error(SALF_ERR_OUT_OF_MEMORY, "index has %zu bytes, it needs %zu", bytes, need);
  DeviceGuard g(ctx->device);
  if (!g.ok) return set_error(SALF_ERR_DEVICE, "cannot select device %d", ctx->device);
  const hipStream_t s = (hipStream_t)stream;
  int32_t* d_boff = (int32_t*)d_index;
  uint32_t* d_entries = (uint32_t*)((char*)d_index + index_bytes(n_root, 0));
  if ((st = check_hip(hipMemcpyAsync(d_boff, boff.data(), n_root * 4, hipMemcpyHostToDevice, s), "copy index offsets")))
    return st;
  if ((st = check_hip(launch_index_fill(sc.view, n_root, d_boff, d_entries, s), "index launch"))) return st;
  SceneView v = sc.view;
  v.boff = d_boff;
  if ((st = check_hip(launch_pack_cells(v, n_root, s), "cell records launch"))) return st;
  if ((st = check_hip(hipStreamSynchronize(s), "index build"))) return st;
  return attach_index(ctx, scene_id, sc, d_boff, d_entries);
}

salf_status salf_refine_work_size(int64_t n_voxels, size_t* bytes) {
  if (!bytes) return set_error(SALF_ERR_INVALID_ARG, "bytes is NULL");
  if (n_voxels < 0 || n_voxels > ((int64_t)1 << 30)) return set_error(SALF_ERR_INVALID_ARG, "n_voxels out of range");
  *bytes = refine_work_bytes(n_voxels);
  return SALF_OK;
}

salf_status salf_refine(salf_context* ctx, int32_t scene_id, const int32_t* d_voxels, const float* d_grad_rgb,
                        const salf_refine_opts* opts, void* d_work, size_t work_bytes, int32_t* d_voxels_out,
                        float* d_geo_out, float* d_rgb_out, float* d_int_out, int64_t capacity, int64_t* n_out,
                        void* stream) {
  Scene sc;
  salf_status st = scene_snapshot(ctx, scene_id, &sc);
  if (st) return st;
  if (!opts || !n_out) return set_error(SALF_ERR_INVALID_ARG, "opts and n_out are required");
  if (!(opts->grad_threshold >= 0.0) || !(opts->alpha_min >= 0.0) || !(opts->alpha_min <= 1.0))
    return set_error(SALF_ERR_INVALID_ARG, "grad_threshold must be >= 0 and alpha_min in [0, 1]");
  if (capacity < 0) return set_error(SALF_ERR_INVALID_ARG, "capacity must be >= 0");
  const int64_t n = sc.n;
  if (n > 0 && !d_voxels) return set_error(SALF_ERR_INVALID_ARG, "voxels are required");
  if (n > 0 && (!d_work || work_bytes < refine_work_bytes(n)))
    return set_error(SALF_ERR_INVALID_ARG, "work area must hold %zu bytes", refine_work_bytes(n));
  if (capacity > 0 && (!d_voxels_out || !d_geo_out || (sc.view.rgb && !d_rgb_out) || (sc.view.inten && !d_int_out)))
    return set_error(SALF_ERR_INVALID_ARG, "an output the scene needs is NULL");
  DeviceGuard g(ctx->device);
  if (!g.ok) return set_error(SALF_ERR_DEVICE, "cannot select device %d", ctx->device);
  int64_t total = 0;
  if ((st = check_hip(launch_refine(sc.view, sc.desc, n, d_voxels, d_grad_rgb, opts->grad_threshold, opts->alpha_min,
                                    d_work, d_voxels_out, d_geo_out, d_rgb_out, d_int_out, capacity, &total,
                                    (hipStream_t)stream),
                      "refine")))
    return st;
  *n_out = total;
  if (total > capacity)
    return set_error(SALF_ERR_OUT_OF_MEMORY, "the refined scene has %lld voxels, the outputs hold %lld",
                     (long long)total, (long long)capacity);
  return SALF_OK;
}

salf_status salf_scene_destroy(salf_context* ctx, int32_t scene_id) {
  if (!ctx) return set_error(SALF_ERR_INVALID_ARG, "context is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (scene_id < 0 || scene_id >= (int32_t)ctx->scenes.size() || !ctx->scenes[scene_id].live)
    return set_error(SALF_ERR_NOT_FOUND, "no scene with id %d", scene_id);
  ctx->scenes[scene_id].live = false;
  return SALF_OK;
}

salf_status salf_sensor_ray_count(const salf_sensor* sensor, int64_t* n_rays) {
  salf_status st = validate_sensor(sensor);
  if (st) return st;
  if (!n_rays) return set_error(SALF_ERR_INVALID_ARG, "n_rays is NULL");
  *n_rays = (int64_t)sensor->width * sensor->height;
  return SALF_OK;
}

salf_status salf_generate_rays(salf_context* ctx, const salf_sensor* sensor, float* d_o, float* d_d, float* d_t,
                               uint8_t* d_valid, void* stream) {
  if (!ctx) return set_error(SALF_ERR_INVALID_ARG, "context is NULL");
  salf_status st = validate_sensor(sensor);
  if (st) return st;
  DeviceGuard g(ctx->device);
  return check_hip(launch_raygen(*sensor, d_o, d_d, d_t, d_valid, (hipStream_t)stream), "ray generation launch");
}

salf_status salf_render(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor, const salf_rays* rays,
                        const salf_render_opts* opts, const salf_outputs* out, void* stream) {
  RenderParams p;
  int field = 0;
  salf_status st = prepare_render(ctx, scene_id, sensor, rays, opts, &p, &field);
  if (st) return st;
  if (!out) return set_error(SALF_ERR_INVALID_ARG, "outputs is NULL");
  if (out->rgb && !p.scene.rgb) return set_error(SALF_ERR_INVALID_ARG, "colour requested from a scene without colour");
  if (out->intensity && !p.scene.inten)
    return set_error(SALF_ERR_INVALID_ARG, "intensity requested from a scene without intensity");
  if ((st = check_hit_outputs(out, p.pieces <= 1, "renders in pieces"))) return st;
  p.out = *out;
  DeviceGuard g(ctx->device);
  if (opts->schedule == SALF_SCHEDULE_BUILD &&
      (st = check_hip(launch_tile_schedule(p, opts->d_work, (hipStream_t)stream), "tile schedule launch")))
    return st;
  return check_hip(launch_render(p, field, (hipStream_t)stream), "render launch");
}

salf_status salf_render_static(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor, const salf_rays* rays,
                               const salf_render_opts* opts, const salf_outputs* out, void* stream) {
  if (!ctx) return set_error(SALF_ERR_INVALID_ARG, "context is NULL");
  if (!opts) return set_error(SALF_ERR_INVALID_ARG, "render opts is NULL");
  RenderParams lay;
  memset(&lay, 0, sizeof(lay));
  salf_status st = ray_layout(sensor, rays, &lay);
  if (st) return st;
  if (tile_count(lay) > SALF_STATIC_SCHEDULE_TILES)
    return set_error(SALF_ERR_OUT_OF_MEMORY, "the launch has %lld tiles; the static schedule holds at most %d",
                     (long long)tile_count(lay), SALF_STATIC_SCHEDULE_TILES);
  salf_render_opts o = *opts;
  o.schedule = SALF_SCHEDULE_BUILD;
  o.d_work = ctx->static_sched;
  o.work_bytes = SALF_STATIC_SCHEDULE_BYTES;
  return salf_render(ctx, scene_id, sensor, rays, &o, out, stream);
}

}  // extern "C"

namespace {
// The splatting parameters of a frame of `sensor` on scene `scene_id`.
salf_status raster_setup(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor, RasterParams* p, int* field) {
  Scene sc;
  salf_status st = scene_snapshot(ctx, scene_id, &sc);
  if (st) return st;
  if ((st = validate_sensor(sensor))) return st;
  if (sensor->model != SALF_PINHOLE) return set_error(SALF_ERR_UNSUPPORTED, "splatting renders pinhole cameras");
  if (sensor->width > 32767 || sensor->height > 32767)
    return set_error(SALF_ERR_UNSUPPORTED, "splatting renders images of at most 32767 x 32767 pixels");
  const bool still = sensor->v[0] == 0.0f && sensor->v[1] == 0.0f && sensor->v[2] == 0.0f && sensor->w[0] == 0.0f &&
                     sensor->w[1] == 0.0f && sensor->w[2] == 0.0f;
  if (sensor->dt_line != 0.0f && !still)
    return set_error(SALF_ERR_UNSUPPORTED, "splatting needs one pose for every pixel (no rolling-shutter motion)");
  for (int i = 0; i < 3; ++i)
    if (!isfinite(sensor->p0[i])) return set_error(SALF_ERR_INVALID_ARG, "sensor position is not finite");
  memset(p, 0, sizeof(*p));
  p->scene = sc.view;
  p->vbox = sc.vbox;
  p->sensor = *sensor;
  p->n_voxels = sc.n;
  raster_prepare(p);
  if (p->key_bits + p->tile_bits > 64)
    return set_error(SALF_ERR_UNSUPPORTED, "the frame's tiles and the scene's grid need more than 64 key bits");
  *field = sc.desc.field;
  return SALF_OK;
}
}  // namespace

extern "C" {

salf_status salf_raster_work_size(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor, int64_t max_pairs,
                                  size_t* bytes) {
  if (!bytes) return set_error(SALF_ERR_INVALID_ARG, "bytes is NULL");
  if (max_pairs < 0 || max_pairs > (int64_t)UINT32_MAX)
    return set_error(SALF_ERR_INVALID_ARG, "max_pairs must be in [0, 2^32)");
  RasterParams p;
  int field = 0;
  salf_status st = raster_setup(ctx, scene_id, sensor, &p, &field);
  if (st) return st;
  DeviceGuard g(ctx->device);
  return check_hip(raster_work_bytes(p.n_voxels, (int64_t)p.tiles_x * p.tiles_y, max_pairs, bytes),
                   "splatting work size");
}

salf_status salf_render_raster(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor,
                               const salf_render_opts* opts, const salf_outputs* out, void* d_work, size_t work_bytes,
                               int64_t* n_pairs, void* stream) {
  RasterParams p;
  int field = 0;
  salf_status st = raster_setup(ctx, scene_id, sensor, &p, &field);
  if (st) return st;
  if ((st = validate_opts(opts)) || (st = one_lane_per_ray(opts, "splatting renders"))) return st;
  if (!out || !n_pairs) return set_error(SALF_ERR_INVALID_ARG, "outputs and n_pairs are required");
  if ((st = check_hit_outputs(out, false, "splatting renders"))) return st;
  if (out->rgb && !p.scene.rgb) return set_error(SALF_ERR_INVALID_ARG, "colour requested from a scene without colour");
  if (out->intensity && !p.scene.inten)
    return set_error(SALF_ERR_INVALID_ARG, "intensity requested from a scene without intensity");
  if (!d_work || ((uintptr_t)d_work & 255u)) return set_error(SALF_ERR_INVALID_ARG, "work area must be 256-byte aligned");
  p.S = opts->samples_per_voxel;
  p.t_min = opts->t_min;
  for (int c = 0; c < 3; ++c) p.bg[c] = opts->background[c];
  p.out = *out;
  DeviceGuard g(ctx->device);
  int64_t pairs = 0, cap = 0;
  if ((st = check_hip(launch_raster(p, field, d_work, work_bytes, &pairs, &cap, (hipStream_t)stream),
                      "splatting launch")))
    return st;
  *n_pairs = pairs;
  if (pairs > cap)
    return set_error(SALF_ERR_OUT_OF_MEMORY, "the frame has %lld (voxel, tile) pairs; the work area holds %lld",
                     (long long)pairs, (long long)cap);
  return SALF_OK;
}

}  // extern "C"

namespace {
constexpr int32_t kMultiMax = 256;
inline size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }
// Work area of a multi-sensor launch: [items][tile counter][batch schedule].
size_t multi_bytes(int32_t n) {
  return up256((size_t)n * sizeof(BatchItem)) + 256 + up256(tile_work_bytes(kBatchScheduleTiles));
}
}  // namespace

extern "C" {

salf_status salf_render_multi_work_size(int32_t n_items, size_t* bytes) {
  if (!bytes) return set_error(SALF_ERR_INVALID_ARG, "bytes is NULL");
  if (n_items < 1 || n_items > kMultiMax) return set_error(SALF_ERR_INVALID_ARG, "n_items must be in [1, %d]", kMultiMax);
  *bytes = multi_bytes(n_items);
  return SALF_OK;
}

salf_status salf_render_multi(salf_context* ctx, int32_t n_items, const salf_render_item* items, void* d_work,
                              size_t work_bytes, void* stream) {
  if (!ctx) return set_error(SALF_ERR_INVALID_ARG, "context is NULL");
  if (n_items < 1 || n_items > kMultiMax || !items)
    return set_error(SALF_ERR_INVALID_ARG, "n_items must be in [1, %d] with items", kMultiMax);
  if (!d_work || ((uintptr_t)d_work & 255u) || work_bytes < multi_bytes(n_items))
    return set_error(SALF_ERR_INVALID_ARG, "work area must be 256-byte aligned and hold %zu bytes", multi_bytes(n_items));
  std::vector<BatchItem> batch((size_t)n_items);
  int64_t tiles = 0;
  uint32_t variants = 0;
  salf_status st;
  for (int32_t i = 0; i < n_items; ++i) {
    const salf_render_item& it = items[i];
    if (it.reserved != 0 || !it.sensor) return set_error(SALF_ERR_INVALID_ARG, "item %d: reserved != 0 or no sensor", i);
    BatchItem& b = batch[(size_t)i];
    memset(&b, 0, sizeof(b));
    salf_render_opts o = it.opts;
    o.schedule = SALF_SCHEDULE_NONE;
    int field = 0;
    if ((st = one_lane_per_ray(&o, "multi-sensor launches"))) return st;
    if ((st = prepare_render(ctx, it.scene_id, it.sensor, nullptr, &o, &b.p, &field))) return st;
    if (field != SALF_FIELD_CORNER) return set_error(SALF_ERR_UNSUPPORTED, "item %d: multi-sensor launches render corner-field scenes", i);
    if ((st = check_hit_outputs(&it.out, false, "multi-sensor launches"))) return st;
    if (it.out.rgb && !b.p.scene.rgb) return set_error(SALF_ERR_INVALID_ARG, "item %d: colour from a scene without colour", i);
    if (it.out.intensity && !b.p.scene.inten)
      return set_error(SALF_ERR_INVALID_ARG, "item %d: intensity from a scene without intensity", i);
    b.p.out = it.out;
    b.tile_begin = tiles;
    b.variant = (it.out.rgb ? 1 : 0) | (it.out.intensity ? 2 : 0) | (b.p.scene.act_geo ? 4 : 0);
    variants |= 1u << b.variant;
    tiles += tile_count(b.p);
    if (tiles > ((int64_t)1 << 31)) return set_error(SALF_ERR_INVALID_ARG, "more than 2^31 tiles in one launch");
  }
  char* w = (char*)d_work;
  BatchItem* d_items = (BatchItem*)w;
  uint32_t* d_counter = (uint32_t*)(w + up256((size_t)n_items * sizeof(BatchItem)));
  void* d_sched = w + up256((size_t)n_items * sizeof(BatchItem)) + 256;
  DeviceGuard g(ctx->device);
  const hipStream_t s = (hipStream_t)stream;
  static const uint32_t zero = 0;
  if ((st = check_hip(hipMemcpyAsync(d_items, batch.data(), batch.size() * sizeof(BatchItem), hipMemcpyHostToDevice, s),
                      "multi-sensor items copy")))
    return st;
  if ((st = check_hip(hipMemcpyAsync(d_counter, &zero, sizeof(zero), hipMemcpyHostToDevice, s), "counter reset")))
    return st;
  if ((st = check_hip(launch_batch_schedule(d_items, n_items, tiles, d_sched, s), "multi-sensor schedule"))) return st;
  return check_hip(launch_render_batch(d_items, n_items, tiles, d_counter, (const int32_t*)d_sched, variants, s),
                   "multi-sensor launch");
}

salf_status salf_render_schedule(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor,
                                 const salf_rays* rays, const salf_render_opts* opts, void* stream) {
  if (!opts) return set_error(SALF_ERR_INVALID_ARG, "render opts is NULL");
  salf_render_opts o = *opts;
  o.schedule = SALF_SCHEDULE_BUILD;
  RenderParams p;
  int field = 0;
  salf_status st = prepare_render(ctx, scene_id, sensor, rays, &o, &p, &field);
  if (st) return st;
  DeviceGuard g(ctx->device);
  return check_hip(launch_tile_schedule(p, o.d_work, (hipStream_t)stream), "tile schedule launch");
}

salf_status salf_render_work_size(const salf_sensor* sensor, const salf_rays* rays, size_t* bytes) {
  if (!bytes) return set_error(SALF_ERR_INVALID_ARG, "bytes is NULL");
  RenderParams p;
  memset(&p, 0, sizeof(p));
  const salf_status st = ray_layout(sensor, rays, &p);
  if (st) return st;
  *bytes = tile_work_bytes(tile_count(p));
  return SALF_OK;
}

salf_status salf_render_composite(salf_context* ctx, int32_t static_scene_id, int32_t n_actors,
                                  const salf_actor* actors, const salf_sensor* sensor, const salf_rays* rays,
                                  const salf_render_opts* opts, const salf_outputs* out, void* stream) {
  static_assert(SALF_MAX_ACTORS == kMaxActors, "actor count");
  CompositeParams cp;
  memset(&cp, 0, sizeof(cp));
  int field = 0;
  salf_status st = one_lane_per_ray(opts, "renders with actors");
  if (st || (st = prepare_render(ctx, static_scene_id, sensor, rays, opts, &cp.base, &field))) return st;
  if (!out) return set_error(SALF_ERR_INVALID_ARG, "outputs is NULL");
  if ((st = check_hit_outputs(out, false, "renders with actors"))) return st;
  if (n_actors < 0 || n_actors > SALF_MAX_ACTORS || (n_actors > 0 && !actors))
    return set_error(SALF_ERR_INVALID_ARG, "n_actors %d outside [0, %d] or actors NULL", n_actors, SALF_MAX_ACTORS);
  const bool act = cp.base.scene.act_geo != nullptr;
  auto check = [&](const SceneView& v, int fld) -> salf_status {
    if (fld != SALF_FIELD_CORNER) return set_error(SALF_ERR_UNSUPPORTED, "actors render corner-field scenes only");
    if ((v.act_geo != nullptr) != act)
      return set_error(SALF_ERR_INVALID_ARG, "all scenes must be pre-activated, or none");
    if (out->rgb && !v.rgb) return set_error(SALF_ERR_INVALID_ARG, "colour requested from a scene without colour");
    if (out->intensity && !v.inten)
      return set_error(SALF_ERR_INVALID_ARG, "intensity requested from a scene without intensity");
    return SALF_OK;
  };
  if ((st = check(cp.base.scene, field))) return st;
  cp.n_actors = n_actors;
  cp.slot[0].view = cp.base.scene;
  for (int a = 0; a < n_actors; ++a) {
    Scene sc;
    if ((st = scene_snapshot(ctx, actors[a].scene_id, &sc))) return st;
    if ((st = check(sc.view, sc.desc.field))) return st;
    for (int k = 0; k < 9; ++k)
      if (!isfinite(actors[a].R[k])) return set_error(SALF_ERR_INVALID_ARG, "actor %d pose is not finite", a);
    for (int k = 0; k < 3; ++k)
      if (!isfinite(actors[a].t[k])) return set_error(SALF_ERR_INVALID_ARG, "actor %d pose is not finite", a);
    ActorPose& sa = cp.slot[1 + a];
    sa.view = sc.view;
    memcpy(sa.R, actors[a].R, sizeof(sa.R));
    memcpy(sa.t, actors[a].t, sizeof(sa.t));
  }
  cp.base.out = *out;
  DeviceGuard g(ctx->device);
  if (opts->schedule == SALF_SCHEDULE_BUILD &&
      (st = check_hip(launch_tile_schedule(cp.base, opts->d_work, (hipStream_t)stream), "tile schedule launch")))
    return st;
  if (n_actors == 0)  // the same bits as the actor kernel, from the plain render kernel
    return check_hip(launch_render(cp.base, field, (hipStream_t)stream), "render launch");
  return check_hip(launch_composite(cp, act, (hipStream_t)stream), "composite launch");
}

salf_status salf_trace_hits(salf_context* ctx, int32_t scene_id, const salf_rays* rays, int32_t max_hits,
                            int32_t apply_early_termination, const salf_render_opts* opts, int32_t* d_counts,
                            int32_t* d_ids, float* d_t_in, float* d_t_out, void* stream) {
  Scene sc;
  salf_status st = scene_snapshot(ctx, scene_id, &sc);
  if (st) return st;
  if ((st = validate_rays(rays))) return st;
  if (max_hits < 0) return set_error(SALF_ERR_INVALID_ARG, "max_hits must be >= 0");
  if (rays->n > 0 && (!d_counts || (max_hits > 0 && (!d_ids || !d_t_in || !d_t_out))))
    return set_error(SALF_ERR_INVALID_ARG, "output pointer is NULL");
  int field = -1, S = 1;
  float t_min = 0.0f;
  if (apply_early_termination) {
    if ((st = validate_opts(opts))) return st;
    field = sc.desc.field;
    S = opts->samples_per_voxel;
    t_min = opts->t_min;
  }
  DeviceGuard g(ctx->device);
  return check_hip(launch_trace(sc.view, *rays, max_hits, field, S, t_min, d_counts, d_ids, d_t_in, d_t_out,
                                (hipStream_t)stream),
                   "trace launch");
}

salf_status salf_render_backward(salf_context* ctx, int32_t scene_id, const salf_sensor* sensor, const salf_rays* rays,
                                 const salf_render_opts* opts, const salf_outputs* saved, const salf_grads_in* grads,
                                 float* d_dgeo, float* d_drgb, float* d_dint, void* stream) {
  BackwardParams b;
  int field = 0;
  salf_status st = one_lane_per_ray(opts, "backward passes");
  if (st || (st = prepare_render(ctx, scene_id, sensor, rays, opts, &b.fwd, &field))) return st;
  if (!saved || !grads) return set_error(SALF_ERR_INVALID_ARG, "saved outputs and gradients are required");
  if (!saved->t_end || !saved->n_hits) return set_error(SALF_ERR_INVALID_ARG, "saved t_end and n_hits are required");
  if (grads->d_rgb && (!saved->rgb || !b.fwd.scene.rgb))
    return set_error(SALF_ERR_INVALID_ARG, "colour gradient needs the saved colour and a scene with colour");
  if (grads->d_depth && !saved->depth) return set_error(SALF_ERR_INVALID_ARG, "depth gradient needs the saved depth");
  if (grads->d_intensity && (!saved->intensity || !b.fwd.scene.inten))
    return set_error(SALF_ERR_INVALID_ARG, "intensity gradient needs the saved intensity and a scene with intensity");
  if (d_drgb && !b.fwd.scene.rgb) return set_error(SALF_ERR_INVALID_ARG, "scene has no colour parameters");
  if (d_dint && !b.fwd.scene.inten) return set_error(SALF_ERR_INVALID_ARG, "scene has no intensity parameters");
  if ((st = check_hit_outputs(saved, true, ""))) return st;
  b.fwd.out = *saved;
  b.g = *grads;
  b.dgeo = d_dgeo;
  b.drgb = d_drgb;
  b.dint = d_dint;
  b.vbox = nullptr;
  b.walk_only_unstored = 0;
  if (saved->hit_voxel) {
    Scene sc;
    if ((st = scene_snapshot(ctx, scene_id, &sc))) return st;
    b.vbox = sc.vbox;
  }
  DeviceGuard g(ctx->device);
  if (opts->schedule == SALF_SCHEDULE_BUILD &&
      (st = check_hip(launch_tile_schedule(b.fwd, opts->d_work, (hipStream_t)stream), "tile schedule launch")))
    return st;
  return check_hip(launch_backward(b, field, (hipStream_t)stream), "backward launch");
}

}  // extern "C"
