// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device.hpp"
#include "salf.h"

namespace salf {

// ---- error reporting (thread-local message; see salf_last_error)
salf_status set_error(salf_status code, const char* fmt, ...);
salf_status check_hip(hipError_t e, const char* what);

// ---- scene workspace layout: [root grid][skip grid][nodes][hash keys][hash values][2 temp grids][counters]
struct SceneLayout {
  int64_t n_root;        // root cells
  int64_t node_cap;      // internal nodes the workspace can hold
  int64_t hash_cap;      // hash slots (power of two)
  size_t root_off, skip_off, nodes_off, hkeys_off, hvals_off, tmp_off, counters_off;
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
  int32_t tiled;             // 1: waves take 8x8 tiles of an img_w x img_h ray image
  int32_t img_w, img_h;
  int32_t tiles_x, tiles_y;
};

hipError_t launch_render(const RenderParams& p, int field, hipStream_t stream);
hipError_t launch_trace(const SceneView& s, const salf_rays& r, int32_t max_hits, int32_t* counts, int32_t* ids,
                        float* t_in, float* t_out, hipStream_t stream);
hipError_t launch_raygen(const salf_sensor& s, float* o, float* d, float* t, uint8_t* valid, hipStream_t stream);

struct BackwardParams {
  RenderParams fwd;
  salf_grads_in g;
  float* dgeo;
  float* drgb;
  float* dint;
};
hipError_t launch_backward(const BackwardParams& p, hipStream_t stream);

}  // namespace salf
