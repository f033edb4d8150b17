// Device-side building blocks of the renderer (gfx950, wave64).
//
//  * the FP32 ray/voxel interval rule in the finest-grid frame (the hit definition of salf.h);
//  * front-to-back traversal of the occupied voxels of a ray: a root-grid walk plus an octree
//    descent that skips empty space (Sec. 3.2, octree ray casting), driven by a single running
//    parameter t so that every voxel is reported with exactly the interval the rule defines;
//  * sensor ray generation (pinhole, equidistant fisheye, spinning LiDAR, rolling shutter);
//  * local field evaluation (corner-interpolated mode, and Eq. 1-2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "salf.h"

namespace salf {

constexpr int32_t kEmpty = -1;          // empty cell / child
__host__ __device__ inline bool is_leaf_code(int32_t c) { return c <= -2; }
__host__ __device__ inline int32_t leaf_code(int32_t voxel) { return -2 - voxel; }
__host__ __device__ inline int32_t leaf_voxel(int32_t code) { return -2 - code; }

// Everything a kernel needs to know about a built scene (passed by value).
struct SceneView {
  const int32_t* root;   // [Dz][Dy][Dx] cell codes: kEmpty, node index (>= 0) or leaf code
  const int32_t* nodes;  // [n_nodes][8] child codes
  const float* geo;      // [N][8]
  const float* rgb;      // [N][3][8] or null
  const float* inten;    // [N][8] or null
  int32_t dims[3];       // root cells per axis
  int32_t K;             // finest level
  float org32[3];        // grid origin, FP32
  float gs32;            // finest cells per metre, FP32
  double org[3];         // grid origin, FP64
  double gs;             // finest cells per metre, FP64
};

// ----------------------------------------------------------------------------- interval rule
// t at which the ray crosses the grid plane P of one axis: (P - og) * inv, each op rounded,
// never fused.
__device__ __forceinline__ float plane_t(float P, float og, float inv) {
#pragma clang fp contract(off)
  return (P - og) * inv;
}

// Per-ray grid-frame state.
struct RayFrame {
  float og[3], inv[3];
  int par;          // bit a set: axis a is parallel
  double ogd[3];    // FP64 grid-frame origin and direction for sample positions
  double dgd[3];
  float t_near, t_far;
  bool valid;
};

__device__ inline RayFrame make_frame(const SceneView& s, const float o[3], const float d[3], float t_near,
                                      float t_far) {
#pragma clang fp contract(off)
  RayFrame f;
  f.par = 0;
  bool finite = true;
  for (int a = 0; a < 3; ++a) {
    finite = finite && isfinite(o[a]) && isfinite(d[a]);
    f.og[a] = (o[a] - s.org32[a]) * s.gs32;
    const float dg = d[a] * s.gs32;
    f.inv[a] = 1.0f / dg;  // correctly rounded division (HIP default)
    if (dg == 0.0f || isinf(f.inv[a])) f.par |= 1 << a;
    f.ogd[a] = ((double)o[a] - s.org[a]) * s.gs;
    f.dgd[a] = (double)d[a] * s.gs;
  }
  f.valid = finite && f.par != 7;
  f.t_near = t_near;
  f.t_far = t_far;
  return f;
}

// Interval of the axis-aligned box [lo, hi) (finest-cell integers) under the rule.  Returns
// false for a parallel axis outside the slab; otherwise t_in/t_out (t_in canonical +0).
__device__ __forceinline__ bool box_interval(const RayFrame& f, const int32_t lo[3], const int32_t hi[3],
                                             float& t_in, float& t_out) {
  float a0 = f.t_near, a1 = f.t_far;
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (f.par & (1 << a)) {
      ok = ok && ((float)lo[a] <= f.og[a]) && (f.og[a] < (float)hi[a]);
    } else {
      const float ta = plane_t((float)lo[a], f.og[a], f.inv[a]);
      const float tb = plane_t((float)hi[a], f.og[a], f.inv[a]);
      a0 = fmaxf(a0, fminf(ta, tb));
      a1 = fminf(a1, fmaxf(ta, tb));
    }
  }
  t_in = (a0 == 0.0f) ? 0.0f : a0;
  t_out = a1;
  return ok;
}

// ----------------------------------------------------------------------------- traversal
// Calls visit(voxel, lo[3], size, t_in, t_out) for every voxel the ray hits, in increasing
// t_in, until visit returns false.  lo/size are in finest cells.
//
// The walk keeps a running parameter t.  At root level it maintains, per axis, the root-cell
// index whose slab [t_a(entry plane), t_a(exit plane)) contains t; inside an occupied root
// cell it descends, per level, to the child whose per-axis half-open slabs contain t (compare
// t with the FP32 crossing of the mid plane).  Because every slab bound is the same FP32
// plane crossing the rule uses, the leaf found contains t in the rule's sense, its t_in is t,
// and its t_out (> t) is where the walk continues; voxels are found exactly once and none is
// missed.  Each step strictly increases t, and a step budget bounds the loop regardless.
template <typename Visit>
__device__ inline void traverse(const SceneView& s, const RayFrame& f, Visit&& visit) {
  if (!f.valid) return;
  const int K = s.K;
  int32_t glo[3] = {0, 0, 0};
  int32_t ghi[3] = {s.dims[0] << K, s.dims[1] << K, s.dims[2] << K};
  float t_enter, t_exit;
  if (!box_interval(f, glo, ghi, t_enter, t_exit)) return;
  if (!(t_enter < t_exit)) return;

  int k[3], step[3];
  float nxt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int D = s.dims[a];
    if (f.par & (1 << a)) {
      int c = (int)f.og[a] >> K;  // og in [0, D << K) here
      k[a] = c < 0 ? 0 : (c >= D ? D - 1 : c);
      step[a] = 0;
      nxt[a] = INFINITY;
      continue;
    }
    // guess the cell at t_enter, then correct it against the rule's plane crossings
    const float pos = f.og[a] + t_enter * (1.0f / f.inv[a]);
    int c = (int)floorf(pos) >> K;
    c = c < 0 ? 0 : (c >= D ? D - 1 : c);
    if (f.inv[a] > 0.0f) {
      while (c > 0 && plane_t((float)(c << K), f.og[a], f.inv[a]) > t_enter) --c;
      while (c < D - 1 && plane_t((float)((c + 1) << K), f.og[a], f.inv[a]) <= t_enter) ++c;
      step[a] = 1;
      nxt[a] = plane_t((float)((c + 1) << K), f.og[a], f.inv[a]);
    } else {
      while (c < D - 1 && plane_t((float)((c + 1) << K), f.og[a], f.inv[a]) > t_enter) ++c;
      while (c > 0 && plane_t((float)(c << K), f.og[a], f.inv[a]) <= t_enter) --c;
      step[a] = -1;
      nxt[a] = plane_t((float)(c << K), f.og[a], f.inv[a]);
    }
    k[a] = c;
  }

  int budget = 1 << 22;
  float t = t_enter;
  const int32_t N0 = 1 << K;
  while (budget-- > 0) {
    const float cell_exit = fminf(fminf(nxt[0], nxt[1]), fminf(nxt[2], t_exit));
    const int32_t code = s.root[((int64_t)k[2] * s.dims[1] + k[1]) * s.dims[0] + k[0]];
    if (code != kEmpty) {
      const int32_t rlo[3] = {k[0] << K, k[1] << K, k[2] << K};
      if (is_leaf_code(code)) {
        const int32_t hi[3] = {rlo[0] + N0, rlo[1] + N0, rlo[2] + N0};
        float ti, to;
        box_interval(f, rlo, hi, ti, to);
        if (ti < to && !visit(leaf_voxel(code), rlo, N0, ti, to)) return;
      } else {
        float tc = t;
        while (tc < cell_exit && budget-- > 0) {
          int32_t node = code, size = N0, c8 = 0, child = kEmpty;
          int32_t lo[3] = {rlo[0], rlo[1], rlo[2]};
          for (int depth = 0; depth < K; ++depth) {
            const int32_t half = size >> 1;
            c8 = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const int32_t mid = lo[a] + half;
              bool upper;
              if (f.par & (1 << a)) {
                upper = f.og[a] >= (float)mid;
              } else {
                const bool past = plane_t((float)mid, f.og[a], f.inv[a]) <= tc;
                upper = (f.inv[a] > 0.0f) ? past : !past;
              }
              if (upper) {
                lo[a] = mid;
                c8 |= 1 << a;
              }
            }
            size = half;
            child = s.nodes[(int64_t)node * 8 + c8];
            if (child >= 0) {
              node = child;
              child = kEmpty;  // a node below the finest level would be malformed: treat as empty
              continue;
            }
            break;
          }
          // leaf cell [lo, lo + size): where the ray leaves it
          float to = f.t_far;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            if (f.par & (1 << a)) continue;
            const int32_t P = (f.inv[a] > 0.0f) ? lo[a] + size : lo[a];
            to = fminf(to, plane_t((float)P, f.og[a], f.inv[a]));
          }
          if (is_leaf_code(child)) {
            const int32_t hi[3] = {lo[0] + size, lo[1] + size, lo[2] + size};
            float ti, tv;
            box_interval(f, lo, hi, ti, tv);
            if (ti < tv && !visit(leaf_voxel(child), lo, size, ti, tv)) return;
          }
          if (!(to > tc)) break;  // cannot happen under the rule; guards against a stall
          tc = to;
        }
      }
    }
    if (!(cell_exit < t_exit)) return;
    t = cell_exit;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      while (step[a] != 0 && nxt[a] <= t) {
        k[a] += step[a];
        if (k[a] < 0 || k[a] >= s.dims[a]) return;
        const int32_t P = (step[a] > 0) ? (k[a] + 1) << K : k[a] << K;
        nxt[a] = plane_t((float)P, f.og[a], f.inv[a]);
      }
    }
  }
}

// ----------------------------------------------------------------------------- sensors
__device__ inline void rotate_rodrigues(const float w[3], float dt, float v[3]) {
  const float wx = w[0], wy = w[1], wz = w[2];
  const float wn = sqrtf(wx * wx + wy * wy + wz * wz);
  const float th = wn * dt;
  if (th == 0.0f) return;
  const float kx = wx / wn, ky = wy / wn, kz = wz / wn;
  float sn, cs;
  sincosf(th, &sn, &cs);
  const float cx = ky * v[2] - kz * v[1], cy = kz * v[0] - kx * v[2], cz = kx * v[1] - ky * v[0];
  const float kd = (kx * v[0] + ky * v[1] + kz * v[2]) * (1.0f - cs);
  const float r0 = v[0] * cs + cx * sn + kx * kd;
  const float r1 = v[1] * cs + cy * sn + ky * kd;
  const float r2 = v[2] * cs + cz * sn + kz * kd;
  v[0] = r0;
  v[1] = r1;
  v[2] = r2;
}

// Ray (o, d) and exposure time of pixel/beam (col, row) of a sensor; false for an invalid ray.
__device__ inline bool sensor_ray(const salf_sensor& s, int col, int row, float o[3], float d[3], float& t) {
  float dl[3];
  bool valid = true;
  int line;
  if (s.model == SALF_LIDAR_SPINNING) {
    const float e = (s.height > 1) ? s.elev_min + (s.elev_max - s.elev_min) * ((float)row / (float)(s.height - 1))
                                   : s.elev_min;
    const float az = s.az0 + 6.28318530717958647692f * (((float)col + 0.5f) / (float)s.width);
    float se, ce, sa, ca;
    sincosf(e, &se, &ce);
    sincosf(az, &sa, &ca);
    dl[0] = ce * ca;
    dl[1] = ce * sa;
    dl[2] = se;
    line = col;
  } else if (s.model == SALF_PINHOLE) {
    const float x = ((float)col + 0.5f - s.cx) / s.fx;
    const float y = ((float)row + 0.5f - s.cy) / s.fy;
    const float rn = 1.0f / sqrtf(x * x + y * y + 1.0f);
    dl[0] = x * rn;
    dl[1] = y * rn;
    dl[2] = rn;
    line = row;
  } else {  // equidistant fisheye
    const float x = ((float)col + 0.5f - s.cx) / s.fx;
    const float y = ((float)row + 0.5f - s.cy) / s.fx;
    const float th = sqrtf(x * x + y * y);
    valid = th <= s.max_theta;
    float sn, cs;
    sincosf(th, &sn, &cs);
    const float sc = th > 0.0f ? sn / th : 1.0f;
    dl[0] = x * sc;
    dl[1] = y * sc;
    dl[2] = cs;
    line = row;
  }
  const float dt = (float)line * s.dt_line;
  t = s.t0 + dt;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d[a] = s.R0[3 * a + 0] * dl[0] + s.R0[3 * a + 1] * dl[1] + s.R0[3 * a + 2] * dl[2];
    o[a] = s.p0[a] + s.v[a] * dt;
  }
  rotate_rodrigues(s.w, dt, d);
  if (!valid) d[0] = d[1] = d[2] = 0.0f;
  return valid;
}

// ----------------------------------------------------------------------------- fields
__device__ __forceinline__ float softplus_f(float z) {
  return fmaxf(z, 0.0f) + __logf(1.0f + __expf(-fabsf(z)));
}
__device__ __forceinline__ float sigmoid_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// Trilinear corner weights at x in [-1, 1]^3 (corner c = bx + 2 by + 4 bz).
__device__ __forceinline__ void corner_weights(const float x[3], float w[8]) {
  const float lx = 0.5f - 0.5f * x[0], hx = 0.5f + 0.5f * x[0];
  const float ly = 0.5f - 0.5f * x[1], hy = 0.5f + 0.5f * x[1];
  const float lz = 0.5f - 0.5f * x[2], hz = 0.5f + 0.5f * x[2];
  const float a0 = ly * lz, a1 = hy * lz, a2 = ly * hz, a3 = hy * hz;
  w[0] = lx * a0; w[1] = hx * a0; w[2] = lx * a1; w[3] = hx * a1;
  w[4] = lx * a2; w[5] = hx * a2; w[6] = lx * a3; w[7] = hx * a3;
}

constexpr float kShC0 = 0.28209479177387814f;
constexpr float kShC1 = 0.48860251190291992f;

}  // namespace salf
