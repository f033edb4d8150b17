// Device-side building blocks of the renderer (gfx950, wave64).
//
//  * the FP32 ray/voxel interval rule in the finest-grid frame (the hit definition of salf.h);
//  * front-to-back traversal of the occupied voxels of a ray: a root-grid walk that jumps over
//    empty space plus an octree walk with a per-lane node stack (Sec. 3.2, octree ray casting),
//    shaped so that the lanes of a wave report their hits at one convergent point;
//  * sensor ray generation (pinhole, equidistant fisheye, spinning LiDAR, rolling shutter);
//  * local field evaluation (corner-interpolated mode, and Eq. 1-2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "salf.h"

namespace salf {

constexpr int32_t kEmpty = -1;          // empty cell / child
// Field variants of the render kernels: the two of salf.h plus the corner field read from stored
// activated corner values.
constexpr int kFieldCornerActivated = 2;
// The SDF variant's render kernels (SALF_FIELD_SDF scenes).
constexpr int kFieldSdf = 3;
__host__ __device__ inline bool is_leaf_code(int32_t c) { return c <= -2; }
__host__ __device__ inline int32_t leaf_code(int32_t voxel) { return -2 - voxel; }
__host__ __device__ inline int32_t leaf_voxel(int32_t code) { return -2 - code; }

// Everything a kernel needs to know about a built scene (passed by value).
struct SceneView {
  const int32_t* root;   // [Dz][Dy][Dx] cell codes: kEmpty, node index (>= 0) or leaf code
  const int32_t* nodes;  // [n_nodes][8] child codes
  const uint2* nbox;     // [n_nodes] bounds of each node's voxels relative to the node's min corner:
                         // bytes (lo_x, lo_y, lo_z) in .x and (hi_x - 1, hi_y - 1, hi_z - 1) in .y
  const float* geo;      // [N][8]
  const float* rgb;      // [N][3][8] or null
  const float* inten;    // [N][8] or null
  const uint8_t* skip;   // [Dz][Dy][Dx] Chebyshev distance (in root cells, capped) to the nearest
                         // occupied root cell; 0 = occupied.  Null: no empty-space skipping.
  const int32_t* lmax;   // [Dz][Dy][Dx] finest voxel level in each root cell
  const uint2* rbox;     // [Dz][Dy][Dx] nbox of each root cell's node (zero for other cells)
  const int32_t* boff;   // [Dz][Dy][Dx] first entry of each root cell's dense leaf index, or -1;
                         // null: no index
  const uint32_t* cidx;  // dense leaf indexes (see kIdx* below)
  const int4* cell;      // [Dz][Dy][Dx] what a root step reads, in one 16-byte record: x the code,
                         // y boff (-1 without an index), z rbox.x | skip << 24, w rbox.y | lmax << 24
  const float* act_geo;  // activated corner values (pre-activated corner scenes), same layouts as
  const float* act_rgb;  // geo / rgb / inten; null otherwise
  const float* act_int;
  int32_t dims[3];       // root cells per axis
  int32_t K;             // finest level
  float org32[3];        // grid origin, FP32
  float gs32;            // finest cells per metre, FP32
  double org[3];         // grid origin, FP64
  double gs;             // finest cells per metre, FP64
  int32_t step_budget;   // walk steps a ray may take before it is cut short (and reported)
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
  float og[3], dg[3], inv[3];
  float o[3], d[3];  // the ray as given (FP32); sample positions are formed from it in FP64
  int par;           // bit a set: axis a is parallel
  float t_near, t_far;
  bool valid;
};

__device__ inline RayFrame make_frame(const SceneView& s, const float o[3], const float d[3], float t_near,
                                      float t_far) {
#pragma clang fp contract(off)
  RayFrame f;
  f.par = 0;
  bool finite = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    finite = finite && isfinite(o[a]) && isfinite(d[a]);
    f.o[a] = o[a];
    f.d[a] = d[a];
    f.og[a] = (o[a] - s.org32[a]) * s.gs32;
    const float dg = d[a] * s.gs32;
    f.dg[a] = dg;
    f.inv[a] = 1.0f / dg;  // correctly rounded division (HIP default)
    if (dg == 0.0f || isinf(f.inv[a])) f.par |= 1 << a;
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
// Root cell index of a non-parallel axis whose half-open slab contains t under the rule, and
// the crossing where the ray leaves it.  The position guess is corrected against the rule's
// own plane crossings, which are monotone in the plane.
__device__ __forceinline__ void locate_axis(const RayFrame& f, int a, float t, int D, int K, int& k, float& nxt) {
  const float pos = f.og[a] + t * f.dg[a];
  int c = (int)floorf(pos) >> K;
  c = c < 0 ? 0 : (c >= D ? D - 1 : c);
  const float og = f.og[a], inv = f.inv[a];
  if (inv > 0.0f) {
    while (c > 0 && plane_t((float)(c << K), og, inv) > t) --c;
    while (c < D - 1 && plane_t((float)((c + 1) << K), og, inv) <= t) ++c;
    nxt = plane_t((float)((c + 1) << K), og, inv);
  } else {
    while (c < D - 1 && plane_t((float)((c + 1) << K), og, inv) > t) ++c;
    while (c > 0 && plane_t((float)(c << K), og, inv) <= t) --c;
    nxt = plane_t((float)(c << K), og, inv);
  }
  k = c;
}

// Where the ray leaves the box [lo, lo + size) (finest cells): the smallest exit-plane crossing.
__device__ __forceinline__ float box_exit(const RayFrame& f, const int32_t lo[3], int32_t size) {
  float to = f.t_far;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (f.par & (1 << a)) continue;
    const int32_t P = (f.inv[a] > 0.0f) ? lo[a] + size : lo[a];
    to = fminf(to, plane_t((float)P, f.og[a], f.inv[a]));
  }
  return to;
}

// Root-walk state of one axis: the root-cell index holding t, the step direction (0 for a
// parallel axis) and the crossing where the ray leaves that cell.
struct RootAxis {
  int k, step;
  float nxt;
};

template <int A>
__device__ __forceinline__ void root_axis_init(const RayFrame& f, const SceneView& s, float t, RootAxis& r) {
  if (f.par & (1 << A)) {
    const int c = (int)f.og[A] >> s.K;  // og in [0, D << K) for a parallel axis that hits the grid
    r.k = c < 0 ? 0 : (c >= s.dims[A] ? s.dims[A] - 1 : c);
    r.step = 0;
    r.nxt = INFINITY;
  } else {
    locate_axis(f, A, t, s.dims[A], s.K, r.k, r.nxt);
    r.step = f.inv[A] > 0.0f ? 1 : -1;
  }
}

// Step the axis past every cell whose exit crossing is <= t; false if the walk leaves the grid.
template <int A>
__device__ __forceinline__ bool root_axis_advance(const RayFrame& f, const SceneView& s, float t, RootAxis& r) {
  if (r.step == 0) return true;
  while (r.nxt <= t) {
    r.k += r.step;
    if (r.k < 0 || r.k >= s.dims[A]) return false;
    const int32_t P = (r.step > 0) ? (r.k + 1) << s.K : r.k << s.K;
    r.nxt = plane_t((float)P, f.og[A], f.inv[A]);
  }
  return true;
}

// Crossing where the ray leaves, along axis A, the cube of root cells within distance d - 1.
template <int A>
__device__ __forceinline__ float cube_exit(const RayFrame& f, const SceneView& s, const RootAxis& r, int d) {
  if (r.step == 0) return INFINITY;
  int P = (r.step > 0) ? r.k + d : r.k - (d - 1);
  P = P < 0 ? 0 : (P > s.dims[A] ? s.dims[A] : P);
  return plane_t((float)(P << s.K), f.og[A], f.inv[A]);
}

// The rule's interval of the bounds of a node's voxels (packed relative to the node's min corner
// `lo`); false if the ray misses them.  Every voxel of the node lies inside these bounds, so a
// voxel's entry crossing is never before b_in.
__device__ __forceinline__ bool node_bounds(const RayFrame& f, const int32_t lo[3], const uint2 b, float& b_in,
                                            float& b_out) {
  const int32_t blo[3] = {lo[0] + (int32_t)(b.x & 255u), lo[1] + (int32_t)((b.x >> 8) & 255u),
                          lo[2] + (int32_t)((b.x >> 16) & 255u)};
  const int32_t bhi[3] = {lo[0] + (int32_t)(b.y & 255u) + 1, lo[1] + (int32_t)((b.y >> 8) & 255u) + 1,
                          lo[2] + (int32_t)((b.y >> 16) & 255u) + 1};
  return box_interval(f, blo, bhi, b_in, b_out) && b_in < b_out;
}

// Child code c8 of the 8 held in two int4 registers, by selects (no indexed register access).
__device__ __forceinline__ int32_t pick8(const int4 a, const int4 b, int c8) {
  const bool z = (c8 & 4) != 0, y = (c8 & 2) != 0, x = (c8 & 1) != 0;
  const int32_t q0 = z ? b.x : a.x, q1 = z ? b.y : a.y, q2 = z ? b.z : a.z, q3 = z ? b.w : a.w;
  const int32_t lo = x ? q1 : q0, hi = x ? q3 : q2;
  return y ? hi : lo;
}

// One voxel hit: id, finest-cell box and the rule's interval.
struct Hit {
  int32_t voxel;
  int32_t lo[3];
  int32_t size;
  float t_in, t_out;
};

// Sample geometry of a hit segment: the position at t_in relative to the voxel's min corner and
// the step between samples, in finest cells, formed in FP64 from the FP32 ray and then kept in
// FP32 (small numbers, so far-away samples keep full precision); the piece length delta and the
// scale sc = 1 / size to unit-cube coordinates u = (rel + (k + 1/2) stp) sc, u = (x + 1) / 2 for
// the local x in [-1, 1].  rS = 1 / S.
__device__ __forceinline__ void segment_frame(const SceneView& s, const RayFrame& f, const Hit& h, double rS,
                                              float rel[3], float stp[3], float& delta, float& sc) {
  const double ti = (double)h.t_in;
  const double dtS = ((double)h.t_out - ti) * rS;
  delta = (float)dtS;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double ogd = ((double)f.o[a] - s.org[a]) * s.gs;
    const double dgd = (double)f.d[a] * s.gs;
    rel[a] = (float)fma(ti, dgd, ogd - (double)h.lo[a]);
    stp[a] = (float)(dtS * dgd);
  }
  sc = __builtin_amdgcn_rcpf((float)h.size);  // exact: size is a power of two
}

// The ray's own FP64 terms of segment_frame, (o - org) gs and d gs per axis, formed once per ray
// with the same operations and kept (in LDS) at seg[a * stride] and seg[(3 + a) * stride]:
// segment_frame_of then takes the same values per hit, so its results are the same bits, with
// a third of the FP64 instructions (half-rate on the VALU) per hit.
__device__ __forceinline__ void segment_ray_terms(const SceneView& s, const RayFrame& f, double* seg, int stride) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    seg[a * stride] = ((double)f.o[a] - s.org[a]) * s.gs;
    seg[(3 + a) * stride] = (double)f.d[a] * s.gs;
  }
}

__device__ __forceinline__ void segment_frame_of(const double* seg, int stride, const Hit& h, double rS,
                                                 float rel[3], float stp[3], float& delta, float& sc) {
  const double ti = (double)h.t_in;
  const double dtS = ((double)h.t_out - ti) * rS;
  delta = (float)dtS;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double ogd = seg[a * stride];
    const double dgd = seg[(3 + a) * stride];
    rel[a] = (float)fma(ti, dgd, ogd - (double)h.lo[a]);
    stp[a] = (float)(dtS * dgd);
  }
  sc = __builtin_amdgcn_rcpf((float)h.size);
}

// Unit-cube coordinate of sample k (midpoint k + 1/2) along one axis, clamped to [0, 1].
__device__ __forceinline__ float sample_u(float rel, float stp, float fk, float sc) {
  return __builtin_amdgcn_fmed3f(fmaf(fk, stp, rel) * sc, 0.0f, 1.0f);
}

// Dense leaf index of a root cell whose finest voxel level is L: 2^L x 2^L x 2^L entries (x
// fastest), one per cell of level L, each naming the region of the cell's octree that holds it:
// bits 0-3 the region's level (1..L), bits 4-31 its voxel + 1 (0: an empty region).
constexpr int kIdxLevelBits = 4;
constexpr uint32_t kIdxLevelMask = 15u;

// Index of the level-L cell of one axis (edge 2^sh finest cells, root cell min corner lo) whose
// half-open slab holds tc under the rule, and the crossing where the ray leaves it; the same
// predicate as the octree descent's mid-plane tests (monotone crossings), found from a position
// guess corrected against the crossings.
__device__ __forceinline__ void locate_fine(const RayFrame& f, int a, float tc, int32_t lo, int sh, int R, int& c,
                                            float& nxt) {
  const float og = f.og[a], inv = f.inv[a];
  if (f.par & (1 << a)) {
    c = ((int32_t)floorf(og) - lo) >> sh;
    c = c < 0 ? 0 : (c >= R ? R - 1 : c);
    nxt = INFINITY;
    return;
  }
  c = ((int32_t)floorf(og + tc * f.dg[a]) - lo) >> sh;
  c = c < 0 ? 0 : (c >= R ? R - 1 : c);
  if (inv > 0.0f) {
    while (c > 0 && plane_t((float)(lo + (c << sh)), og, inv) > tc) --c;
    while (c < R - 1 && plane_t((float)(lo + ((c + 1) << sh)), og, inv) <= tc) ++c;
    nxt = plane_t((float)(lo + ((c + 1) << sh)), og, inv);
  } else {
    while (c < R - 1 && plane_t((float)(lo + ((c + 1) << sh)), og, inv) > tc) ++c;
    while (c > 0 && plane_t((float)(lo + (c << sh)), og, inv) <= tc) --c;
    nxt = plane_t((float)(lo + (c << sh)), og, inv);
  }
}

// Step one axis's level-L cell index past every crossing <= tc (the index stays in [0, R)).
__device__ __forceinline__ void step_fine(const RayFrame& f, int a, float tc, int32_t lo, int sh, int R, int& c,
                                          float& nxt) {
  if (f.par & (1 << a)) return;
  const float og = f.og[a], inv = f.inv[a];
  if (inv > 0.0f) {
    while (nxt <= tc && c < R - 1) {
      ++c;
      nxt = plane_t((float)(lo + ((c + 1) << sh)), og, inv);
    }
  } else {
    while (nxt <= tc && c > 0) {
      --c;
      nxt = plane_t((float)(lo + (c << sh)), og, inv);
    }
  }
}

// The leaf loop of a root cell with a dense leaf index: each pass reads the entry of the level-L
// cell holding tc, reports the region if it is a voxel, moves tc to the region's exit crossing and
// steps the per-axis cell indices past it.  Same passes as the octree walk, minus its descents and
// pops.  False if visit asked to stop.
template <typename Visit>
__device__ __forceinline__ bool index_walk(const SceneView& s, const RayFrame& f, const int32_t lo[3], int L,
                                           const uint32_t* idx, float tc, float cell_end, int& budget, Hit& h,
                                           Visit&& visit) {
  if (!(tc < cell_end)) return true;
  const int sh = s.K - L;
  const int R = 1 << L;
  int c0, c1, c2;
  float n0, n1, n2;
  locate_fine(f, 0, tc, lo[0], sh, R, c0, n0);
  locate_fine(f, 1, tc, lo[1], sh, R, c1, n1);
  locate_fine(f, 2, tc, lo[2], sh, R, c2, n2);
  uint32_t e = idx[(((c2 << L) + c1) << L) + c0];
  while (budget-- > 0) {
    const int rs = L - (int)(e & kIdxLevelMask);  // log2 of the region's edge in level-L cells
    const int32_t size = (1 << (rs + sh));
    h.lo[0] = lo[0] + ((c0 >> rs) << (rs + sh));
    h.lo[1] = lo[1] + ((c1 >> rs) << (rs + sh));
    h.lo[2] = lo[2] + ((c2 >> rs) << (rs + sh));
    // a level-L region's exit planes are the ones the per-axis crossings already hold
    const float to = rs == 0 ? fminf(fminf(n0, n1), fminf(n2, f.t_far)) : box_exit(f, h.lo, size);
    // step to the next region and start reading its entry before this one is shaded
    const bool more = to > tc && to < cell_end;  // (to > tc always holds under the rule)
    uint32_t e_next = 0;
    if (more) {
      step_fine(f, 0, to, lo[0], sh, R, c0, n0);
      step_fine(f, 1, to, lo[1], sh, R, c1, n1);
      step_fine(f, 2, to, lo[2], sh, R, c2, n2);
      e_next = idx[(((c2 << L) + c1) << L) + c0];
    }
    if (e >> kIdxLevelBits) {
      h.voxel = (int32_t)(e >> kIdxLevelBits) - 1;
      h.size = size;
      h.t_in = tc;
      h.t_out = to;
      if (!visit(h)) return false;
    }
    if (!more) return true;
    tc = to;
    e = e_next;
  }
  return true;
}

// The leaf loop of a root cell without a dense leaf index, from tc to cell_end: each pass descends
// from the cell's node (code) to the leaf holding tc, reports the leaf if it holds a voxel, moves tc
// to the leaf's exit crossing and pops the nodes tc has left.  lo: the cell's min corner (changed);
// stk: the lane's node stack.  False if visit asked to stop.
template <typename Visit>
__device__ __forceinline__ bool octree_walk(const SceneView& s, const RayFrame& f, int32_t lo[3], int32_t code,
                                            float tc, float cell_end, int32_t* stk, int stride, int& budget, Hit& h,
                                            Visit&& visit) {
  const int K = s.K;
  int depth = 0;
  int32_t size = 1 << K;
  stk[0] = code;
  const int4* np = reinterpret_cast<const int4*>(s.nodes + (int64_t)code * 8);
  int4 c0 = np[0], c1 = np[1];
  while (tc < cell_end && budget-- > 0) {
    // (1) descend to the leaf holding tc
    int32_t clo[3], half, child;
    for (;;) {
      half = size >> 1;
      int c8 = 0;
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
        clo[a] = upper ? mid : lo[a];
        c8 |= upper ? (1 << a) : 0;
      }
      child = pick8(c0, c1, c8);
      // internal children exist only above the finest level; deeper would be malformed: empty
      if (child < 0 || depth + 1 >= K) break;
      // an internal node: enter it where the ray meets its voxels' bounds, or pass it like an
      // empty leaf if they lie behind tc or off the ray
      np = reinterpret_cast<const int4*>(s.nodes + (int64_t)child * 8);
      const int4 n0 = np[0], n1 = np[1];
      float c_in, c_out;
      const bool hit = node_bounds(f, clo, s.nbox[child], c_in, c_out);
      const float c_tc = fmaxf(tc, c_in);
      if (!hit || !(c_tc < c_out)) {
        child = kEmpty;
        break;
      }
      tc = c_tc;
      ++depth;
      stk[depth * stride] = child;
      size = half;
      lo[0] = clo[0];
      lo[1] = clo[1];
      lo[2] = clo[2];
      c0 = n0;
      c1 = n1;
    }
    // (2) the leaf [clo, clo + half): report a voxel
    const float to = box_exit(f, clo, half);
    if (is_leaf_code(child)) {
      h.voxel = leaf_voxel(child);
      h.lo[0] = clo[0];
      h.lo[1] = clo[1];
      h.lo[2] = clo[2];
      h.size = half;
      h.t_in = tc;
      h.t_out = to;
      if (!visit(h)) return false;
    }
    // (3) advance and leave every node that no longer holds tc
    if (!(to > tc)) break;  // cannot happen under the rule; guards against a stall
    tc = to;
    if (!(tc < cell_end)) break;
    bool popped = false;
    while (depth > 0 && !(tc < box_exit(f, lo, size))) {
      --depth;
      size <<= 1;
      lo[0] &= ~(size - 1);
      lo[1] &= ~(size - 1);
      lo[2] &= ~(size - 1);
      popped = true;
    }
    if (popped) {
      np = reinterpret_cast<const int4*>(s.nodes + (int64_t)stk[depth * stride] * 8);
      c0 = np[0];
      c1 = np[1];
    }
  }
  return true;
}

// Front-to-back walk over the voxels a ray hits: calls visit(hit) for each, in increasing t_in,
// until visit returns false.  Each voxel is reported exactly once with the rule's interval.
//
// The walk keeps one running parameter t.  At root level it keeps, per axis, the root-cell index
// whose slab [crossing of its entry plane, crossing of its exit plane) contains t; an empty root
// cell whose Chebyshev distance to occupied cells is d > 1 lets the walk jump to where the ray
// leaves the empty cube of radius d - 1 around it (every cell the ray meets before that is in the
// cube).  Inside an occupied root cell, each pass of the leaf loop (1) descends from the current
// node to the leaf holding t, choosing at every level the octant whose half-open slabs contain t
// (t against the mid-plane crossings) and pushing internal nodes on a per-lane stack (LDS,
// stk[depth * stride]); (2) reports the leaf if it holds a voxel; (3) moves t to the leaf's exit
// crossing and pops every node that t has left.  All lanes of a wave therefore report at most one
// voxel per pass, at the same point of the loop, which keeps shading convergent.
//
// Every bound is a crossing the rule itself computes.  The leaf found contains t, so its t_in
// (the largest of its entry crossings and t_near) is exactly t, and its t_out is its exit crossing
// capped by t_far: neither needs recomputing.  t strictly increases, and a step budget
// (s.step_budget) bounds the walk regardless; a walk that runs out of it ends early and calls
// cut() (off the hot path: only there), so the ray's truncation is reported, not silent.
template <typename Visit, typename Cut>
__device__ inline void traverse(const SceneView& s, const RayFrame& f, int32_t* stk, int stride, Visit&& visit,
                                Cut&& cut) {
  if (!f.valid) return;
  const int K = s.K;
  float t, t_exit;
  {
    const int32_t glo[3] = {0, 0, 0};
    const int32_t ghi[3] = {s.dims[0] << K, s.dims[1] << K, s.dims[2] << K};
    if (!box_interval(f, glo, ghi, t, t_exit)) return;
    if (!(t < t_exit)) return;
  }
  RootAxis ax, ay, az;
  root_axis_init<0>(f, s, t, ax);
  root_axis_init<1>(f, s, t, ay);
  root_axis_init<2>(f, s, t, az);
  const int32_t N0 = 1 << K;
  int budget = s.step_budget;
  Hit h;
  while (budget-- > 0) {
    const float cell_exit = fminf(fminf(ax.nxt, ay.nxt), fminf(az.nxt, t_exit));
    const int64_t lin = ((int64_t)az.k * s.dims[1] + ay.k) * s.dims[0] + ax.k;
    // the cell's code, index offset, voxel bounds, skip distance and finest level: one record
    const int4 rec = s.cell[lin];
    const int32_t code = rec.x;
    const int32_t bo = rec.y;
    const uint2 rb = make_uint2((uint32_t)rec.z, (uint32_t)rec.w);  // node_bounds reads the low 3 bytes
    const int dskip = (int)((uint32_t)rec.z >> 24);
    float t_next = cell_exit;
    if (code >= 0) {
      // octree of this root cell, entered where the ray meets the bounds of its voxels
      int32_t lo[3] = {ax.k << K, ay.k << K, az.k << K};
      float b_in, b_out;
      const bool meets = node_bounds(f, lo, rb, b_in, b_out);
      float tc = fmaxf(t, b_in);
      const float cell_end = fminf(cell_exit, b_out);
      if (!meets) tc = cell_end;
      if (bo >= 0) {
        if (!index_walk(s, f, lo, (int)((uint32_t)rec.w >> 24), s.cidx + bo, tc, cell_end, budget, h, visit)) return;
      } else if (!octree_walk(s, f, lo, code, tc, cell_end, stk, stride, budget, h, visit)) {
        return;
      }
      if (budget <= 0) break;  // the cell's walk used up the budget: the ray is cut short
    } else if (is_leaf_code(code)) {
      // a level-0 voxel fills the root cell: it holds t, so its interval is [t, cell_exit]
      h.voxel = leaf_voxel(code);
      h.lo[0] = ax.k << K;
      h.lo[1] = ay.k << K;
      h.lo[2] = az.k << K;
      h.size = N0;
      h.t_in = t;
      h.t_out = cell_exit;
      if (!visit(h)) return;
    } else if (dskip > 1) {  // leave the empty cube of radius dskip - 1 around this cell
      t_next = fminf(fminf(cube_exit<0>(f, s, ax, dskip), cube_exit<1>(f, s, ay, dskip)),
                     fminf(cube_exit<2>(f, s, az, dskip), t_exit));
    }
    if (!(t_next < t_exit)) return;
    t = t_next;
    if (!root_axis_advance<0>(f, s, t, ax) || !root_axis_advance<1>(f, s, t, ay) ||
        !root_axis_advance<2>(f, s, t, az))
      return;
  }
  cut();  // the step budget ran out
}


// ---- a ray's root cells shared out among several lanes
// A root cell holding voxels, as the root walk meets it: what its leaf loop needs.
struct CellJob {
  int32_t lo[3];       // the cell's min corner (finest cells)
  int32_t code;        // its node (>= 0), or the leaf code of a voxel that fills it
  int32_t bo, lmax;    // its dense leaf index (first entry, or -1) and finest voxel level
  float tc, cell_end;  // the leaf loop's range (a filling voxel: its interval)
};

// Root-walk state of a ray between occupied cells: t at the current cell, where the ray leaves
// the grid, and the per-axis cell indices.  The walk is over once t reaches t_exit.
struct RootWalk {
  float t, t_exit;
  RootAxis ax, ay, az;
};

// Start the root walk where the ray enters the grid; false if it misses the grid.
__device__ __forceinline__ bool root_walk_begin(const SceneView& s, const RayFrame& f, RootWalk& w) {
  if (!f.valid) return false;
  const int K = s.K;
  const int32_t glo[3] = {0, 0, 0};
  const int32_t ghi[3] = {s.dims[0] << K, s.dims[1] << K, s.dims[2] << K};
  if (!box_interval(f, glo, ghi, w.t, w.t_exit) || !(w.t < w.t_exit)) return false;
  root_axis_init<0>(f, s, w.t, w.ax);
  root_axis_init<1>(f, s, w.t, w.ay);
  root_axis_init<2>(f, s, w.t, w.az);
  return true;
}

// Move the walk to t_next (the current cell's exit, or the exit of an empty cube around it).
__device__ __forceinline__ void root_walk_step(const SceneView& s, const RayFrame& f, RootWalk& w, float t_next) {
  if (!(t_next < w.t_exit)) {
    w.t = w.t_exit;
    return;
  }
  w.t = t_next;
  if (!root_axis_advance<0>(f, s, w.t, w.ax) || !root_axis_advance<1>(f, s, w.t, w.ay) ||
      !root_axis_advance<2>(f, s, w.t, w.az))
    w.t = w.t_exit;
}

// Pass `skip` occupied root cells, then describe the next one in job and leave the walk just past
// it.  Returns 1 with a job, 0 if the ray leaves the grid first, -1 if the step budget runs out.
// The steps, crossings and cell ranges are those of traverse, so every lane that walks the same
// ray meets the same occupied cells in the same order and the leaf loops find the same hits.
__device__ __forceinline__ int root_walk_next(const SceneView& s, const RayFrame& f, RootWalk& w, int skip,
                                              int& budget, CellJob& job) {
  const int K = s.K;
  if (!(w.t < w.t_exit)) return 0;
  while (budget-- > 0) {
    const float cell_exit = fminf(fminf(w.ax.nxt, w.ay.nxt), fminf(w.az.nxt, w.t_exit));
    const int64_t lin = ((int64_t)w.az.k * s.dims[1] + w.ay.k) * s.dims[0] + w.ax.k;
    const int4 rec = s.cell[lin];
    const int32_t code = rec.x;
    float t_next = cell_exit;
    if (code >= 0 || is_leaf_code(code)) {
      if (skip == 0) {
        job.lo[0] = w.ax.k << K;
        job.lo[1] = w.ay.k << K;
        job.lo[2] = w.az.k << K;
        job.code = code;
        job.bo = -1;
        job.lmax = 0;
        job.tc = w.t;
        job.cell_end = cell_exit;
        if (code >= 0) {
          float b_in, b_out;
          const bool meets = node_bounds(f, job.lo, make_uint2((uint32_t)rec.z, (uint32_t)rec.w), b_in, b_out);
          job.cell_end = fminf(cell_exit, b_out);
          job.tc = meets ? fmaxf(w.t, b_in) : job.cell_end;
          job.bo = rec.y;
          if (job.bo >= 0) job.lmax = (int32_t)((uint32_t)rec.w >> 24);
        }
        root_walk_step(s, f, w, cell_exit);
        return 1;
      }
      --skip;
    } else {
      const int dskip = (int)((uint32_t)rec.z >> 24);
      if (dskip > 1)
        t_next = fminf(fminf(cube_exit<0>(f, s, w.ax, dskip), cube_exit<1>(f, s, w.ay, dskip)),
                       fminf(cube_exit<2>(f, s, w.az, dskip), w.t_exit));
    }
    root_walk_step(s, f, w, t_next);
    if (!(w.t < w.t_exit)) return 0;
  }
  return -1;
}

// The leaf loop of one job: visit(hit) for each voxel of the cell the ray hits, in order, as
// traverse reports them.  False if visit asked to stop.
template <typename Visit>
__device__ __forceinline__ bool walk_cell(const SceneView& s, const RayFrame& f, const CellJob& job, int32_t* stk,
                                          int stride, int& budget, Hit& h, Visit&& visit) {
  if (is_leaf_code(job.code)) {
    h.voxel = leaf_voxel(job.code);
    h.lo[0] = job.lo[0];
    h.lo[1] = job.lo[1];
    h.lo[2] = job.lo[2];
    h.size = 1 << s.K;
    h.t_in = job.tc;
    h.t_out = job.cell_end;
    return visit(h);
  }
  if (job.bo >= 0)
    return index_walk(s, f, job.lo, job.lmax, s.cidx + job.bo, job.tc, job.cell_end, budget, h, visit);
  int32_t lo[3] = {job.lo[0], job.lo[1], job.lo[2]};
  return octree_walk(s, f, lo, job.code, job.tc, job.cell_end, stk, stride, budget, h, visit);
}

// Estimated number of voxels a ray crosses, from the root grid alone (used to schedule tiles):
// for every occupied root cell on the ray, the length inside the bounds of the cell's voxels
// times 2^(finest level in the cell) / root-cell size, plus a quarter per root cell visited.
// Only the part of the ray's path through the grid between fractions lo and hi of its length is
// walked, so that several lanes can share one ray.
__device__ inline float root_cost(const SceneView& s, const RayFrame& f, float lo, float hi) {
  if (!f.valid) return 0.0f;
  const int K = s.K;
  float t, t_exit;
  {
    const int32_t glo[3] = {0, 0, 0};
    const int32_t ghi[3] = {s.dims[0] << K, s.dims[1] << K, s.dims[2] << K};
    if (!box_interval(f, glo, ghi, t, t_exit) || !(t < t_exit)) return 0.0f;
    const float span = t_exit - t;
    const float t1 = hi >= 1.0f ? t_exit : t + span * hi;
    t = t + span * lo;
    t_exit = t1;
    if (!(t < t_exit)) return 0.0f;
  }
  RootAxis ax, ay, az;
  root_axis_init<0>(f, s, t, ax);
  root_axis_init<1>(f, s, t, ay);
  root_axis_init<2>(f, s, t, az);
  float len = 0.0f;
  int steps = 0;
  while (steps < (1 << 16)) {
    ++steps;
    const float cell_exit = fminf(fminf(ax.nxt, ay.nxt), fminf(az.nxt, t_exit));
    const int64_t lin = ((int64_t)az.k * s.dims[1] + ay.k) * s.dims[0] + ax.k;
    const int32_t code = s.root[lin];
    float t_next = cell_exit;
    if (code >= 0) {
      const int32_t lo[3] = {ax.k << K, ay.k << K, az.k << K};
      float b_in, b_out;
      if (node_bounds(f, lo, s.rbox[lin], b_in, b_out)) {
        const float l = fminf(b_out, cell_exit) - fmaxf(b_in, t);
        if (l > 0.0f) len += l * (float)(1 << s.lmax[lin]);
      }
    } else if (is_leaf_code(code)) {
      len += cell_exit - t;
    } else if (s.skip != nullptr) {
      const int d = s.skip[lin];
      if (d > 1)
        t_next = fminf(fminf(cube_exit<0>(f, s, ax, d), cube_exit<1>(f, s, ay, d)),
                       fminf(cube_exit<2>(f, s, az, d), t_exit));
    }
    if (!(t_next < t_exit)) break;
    t = t_next;
    if (!root_axis_advance<0>(f, s, t, ax) || !root_axis_advance<1>(f, s, t, ay) ||
        !root_axis_advance<2>(f, s, t, az))
      break;
  }
  return len * s.gs32 / (float)(1 << K) + 0.25f * (float)steps;
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
// Dot product of trilinear weights with 8 corner values, as a chain of fused multiply-adds.
__device__ __forceinline__ float dot8(const float w[8], const float c[8]) {
  float a = w[0] * c[0];
#pragma unroll
  for (int i = 1; i < 8; ++i) a = fmaf(w[i], c[i], a);
  return a;
}

__device__ __forceinline__ float softplus_f(float z) {
  return fmaxf(z, 0.0f) + __logf(1.0f + __expf(-fabsf(z)));
}
__device__ __forceinline__ float sigmoid_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// Trilinear corner weights at unit-cube coordinates u in [0, 1]^3 (u = (x + 1) / 2 for the local
// x in [-1, 1]; corner c = bx + 2 by + 4 bz).
__device__ __forceinline__ void corner_weights(const float u[3], float w[8]) {
  const float hx = u[0], lx = 1.0f - hx;
  const float hy = u[1], ly = 1.0f - hy;
  const float hz = u[2], lz = 1.0f - hz;
  const float a0 = ly * lz, a1 = hy * lz, a2 = ly * hz, a3 = hy * hz;
  w[0] = lx * a0; w[1] = hx * a0; w[2] = lx * a1; w[3] = hx * a1;
  w[4] = lx * a2; w[5] = hx * a2; w[6] = lx * a3; w[7] = hx * a3;
}

constexpr float kShC0 = 0.28209479177387814f;
constexpr float kShC1 = 0.48860251190291992f;

}  // namespace salf
