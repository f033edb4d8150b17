// Forward rendering: per ray, front-to-back traversal of the occupied voxels it hits, S midpoint
// samples of each voxel's local field per segment, and alpha compositing of colour, depth,
// intensity and opacity with FP32 transmittance and early termination (Eq. 1-4, Sec. 3.2).
//
// Work mapping: one lane per ray.  In sensor mode a wave64 covers a tile of 64 neighbouring rays
// (16x4 pixels of a pinhole camera, 8x8 of a fisheye, 32 columns x 2 beams of a LiDAR) so that
// the lanes of a wave walk nearby voxels and share their parameter cache lines; ray generation is
// fused (no ray buffer in HBM).  The per-tile render kernels run one wave per workgroup; the
// backward and the persistent serving kernel run four.
#include <string.h>

#include <atomic>

#include "internal.hpp"
#include "shade.hpp"

namespace salf {
namespace {

constexpr int kThreads = 256;

// Rays whose walk ran out of its step budget on this device, since the library was loaded (never
// reset; read by salf_sync).  Walks are cut short only on pathological input, so the atomic is
// off the hot path.
__device__ uint32_t g_cut_rays;
__device__ __forceinline__ void note_cut() { atomicAdd(&g_cut_rays, 1u); }

// The ray of this lane of wave `wave` (tiled: the wave's tile; else 64 consecutive rays): its
// index and grid frame.  Returns false for lanes without a ray.
__device__ __forceinline__ bool lane_ray(const RenderParams& p, int64_t wave, int lane, int64_t& ray, float d[3],
                                         RayFrame& f) {
  int col = 0, row = 0;
  if (p.tiled) {
    const int tx = (int)(wave % p.tiles_x), ty = (int)(wave / p.tiles_x);
    col = tx * (1 << p.tw_log2) + (lane & ((1 << p.tw_log2) - 1));
    row = ty * (64 >> p.tw_log2) + (lane >> p.tw_log2);
    if (ty >= p.tiles_y || col >= p.img_w || row >= p.img_h) return false;
    ray = (int64_t)row * p.img_w + col;
    if (ray >= p.n) return false;
  } else {
    ray = wave * 64 + lane;
    if (ray >= p.n) return false;
  }
  float o[3];
  bool valid = true;
  float tn = p.t_near, tf = p.t_far;
  if (p.use_sensor) {
    float tt;
    valid = sensor_ray(p.sensor, col, row, o, d, tt);
    tn = p.sensor.t_near;
    tf = p.sensor.t_far;
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      o[a] = p.ro[ray * 3 + a];
      d[a] = p.rd[ray * 3 + a];
    }
  }
  f = make_frame(p.scene, o, d, tn, tf);
  if (!valid) f.valid = false;
  return true;
}

// Tile rendered by wave w of a launch: the schedule's entry when p carries a schedule built for
// this launch's ray layout (its header must match), else w.
__device__ __forceinline__ int64_t scheduled_tile(const RenderParams& p, int64_t w) {
  const int64_t nt = tile_count(p);
  if (p.sched == nullptr || w >= nt) return w;
  const int32_t* h = p.sched;
  if (h[0] != (int32_t)nt || h[1] != (p.tiled | (p.tw_log2 << 8)) || h[2] != p.img_w) return w;
  const int32_t t = h[kSchedHeader + h[3] + w];
  return (t >= 0 && t < nt) ? (int64_t)t : w;
}

// Render the rays of one wave (tile `wave` of p) and store their outputs.  stk: this lane's node
// stack (stride kThreads).  Shared by the single-request kernel and the batched kernel, so a ray
// renders to the same bits alone or in a batch.  p_is_kernarg: p is the kernel's only argument;
// the output pointers and background are then read again from the argument block after the walk
// (an opaque copy of its address keeps the compiler from loading them up front), rather than held
// in scalar registers through it: those are short in the walk, and every extra value there is
// spilled and reloaded inside its loops.
template <int FIELD, bool RGB, bool INT, bool p_is_kernarg = false, bool HITS = false>
__device__ __forceinline__ void render_wave(const RenderParams& p, int64_t wave, int32_t* stk, double* seg,
                                            int stride = kThreads) {
  int64_t ray;
  float d[3];
  RayFrame f;
  if (!lane_ray(p, wave, threadIdx.x & 63, ray, d, f)) return;
  if (f.valid) segment_ray_terms(p.scene, f, seg, stride);
  float sh[4] = {kShC0, kShC1 * d[0], kShC1 * d[1], kShC1 * d[2]};
  Accum acc;
  acc.T = 1.0f;
  acc.C[0] = acc.C[1] = acc.C[2] = 0.0f;
  acc.D = acc.I = 0.0f;
  acc.n = 0;
  const int S = p.S;
  const double rS = 1.0 / S;
  const float t_min = p.t_min;
  bool cut = false;
  traverse(p.scene, f, stk, stride, [&](const Hit& h) -> bool {
    // every visited voxel is shaded, so the hit's index is the count before shading; stored before
    // the shading, whose arithmetic then covers the stores' latency (the next step's loads would
    // otherwise wait for them)
    if (HITS && acc.n < p.out.hit_capacity) {
      // hit k of the ray at k * n + ray: the lanes of a wave store neighbouring entries
      const int64_t at = (int64_t)acc.n * p.n + ray;
      p.out.hit_voxel[at] = h.voxel;
      reinterpret_cast<float2*>(p.out.hit_t)[at] = make_float2(h.t_in, h.t_out);
    }
    return shade_voxel<FIELD, RGB, INT>(p.scene, f, sh, h, S, rS, t_min, acc, seg, stride);
  }, [&] { cut = true; });
  const RenderParams* q = &p;
  if (p_is_kernarg) {
    q = (const RenderParams*)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(q));
  }
  const salf_outputs& out = q->out;
  if (out.rgb) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) out.rgb[ray * 3 + ch] = fmaf(acc.T, q->bg[ch], acc.C[ch]);
  }
  if (out.depth) out.depth[ray] = acc.D;
  if (out.opacity) out.opacity[ray] = 1.0f - acc.T;
  if (out.intensity) out.intensity[ray] = acc.I;
  if (out.t_end) out.t_end[ray] = acc.T;
  if (out.n_hits) out.n_hits[ray] = acc.n;
  // Counted after the stores: the report stays out of the traversal loop's register budget.
  if (cut) note_cut();
}

// At most 168 VGPRs, so that three waves fit each SIMD: the heavier variants (raw logits, colour
// and intensity) would otherwise take a few more registers and drop to two waves, which costs far
// more than the few spills the cap causes.
#define SALF_RENDER_OCCUPANCY __attribute__((amdgpu_waves_per_eu(3)))

// One wave per workgroup.  Waves of one launch differ in length by an order of magnitude (tiles on
// the horizon against sky or near ground); a workgroup of four waves holds its compute unit's
// slots until all four are placed, and the slot a finished wave frees stays idle until enough
// are free for a whole new workgroup, while a one-wave workgroup takes any free slot at once.
constexpr int kRenderThreads = 64;

template <int FIELD, bool RGB, bool INT, bool HITS>
__global__ __launch_bounds__(kRenderThreads) SALF_RENDER_OCCUPANCY void render_kernel(RenderParams p) {
  __shared__ int32_t stk[SALF_MAX_LEVEL * kRenderThreads];
  __shared__ double seg[6 * kRenderThreads];
  const int64_t w = blockIdx.x;
  render_wave<FIELD, RGB, INT, true, HITS>(p, scheduled_tile(p, w), stk + threadIdx.x, seg + threadIdx.x,
                                           kRenderThreads);
}

// ---- one ray in pieces
// P consecutive lanes (P = 2, 4 or 8) share one ray: round by round, lane g walks the ray's
// (rP + g)-th occupied root cell and composites it from T = 1; the P partial results are then
// folded front to back (C += T C_j, D += T D_j, I += T I_j, T *= T_j) into the ray's state, which
// every lane of the group holds.  Where the fold would leave T below t_min inside a cell, that
// cell's lane walks it again from the ray's state with the stopping rule, so the ray stops after
// the voxel a one-lane walk stops after (up to the rounding of T).  For launches with too few rays
// to fill the GPU: a long ray's cells are walked side by side instead of one after another.
template <int FIELD, bool RGB, bool INT>
__global__ __launch_bounds__(kRenderThreads) void render_split_kernel(RenderParams p) {
  __shared__ int32_t stk[SALF_MAX_LEVEL * kRenderThreads];
  const int P = p.pieces;
  const int lane = threadIdx.x & 63;
  const int g = lane & (P - 1);
  const int base = lane - g;
  const int64_t w = (blockIdx.x * (int64_t)kRenderThreads + threadIdx.x) >> 6;
  int64_t ray;
  float d[3];
  RayFrame f;
  // split wave w covers lanes (w % P) * 64 / P ... of the one-lane layout's wave w / P
  if (!lane_ray(p, scheduled_tile(p, w / P), (int)(w % P) * (64 / P) + lane / P, ray, d, f)) return;
  const SceneView& s = p.scene;
  const float sh[4] = {kShC0, kShC1 * d[0], kShC1 * d[1], kShC1 * d[2]};
  const int S = p.S;
  const double rS = 1.0 / S;
  const float t_min = p.t_min;
  int32_t* my_stk = stk + threadIdx.x;
  Accum acc;
  acc.T = 1.0f;
  acc.C[0] = acc.C[1] = acc.C[2] = 0.0f;
  acc.D = acc.I = 0.0f;
  acc.n = 0;
  int budget = s.step_budget;
  RootWalk rw;
  bool walking = root_walk_begin(s, f, rw);
  bool cut = false;
  int skip = g;
  for (;;) {
    CellJob job;
    bool has = false;
    if (walking) {
      const int r = root_walk_next(s, f, rw, skip, budget, job);
      has = r > 0;
      walking = r > 0;
      cut = cut || r < 0;
    }
    skip = P - 1;
    Accum part;
    part.T = 1.0f;
    part.C[0] = part.C[1] = part.C[2] = 0.0f;
    part.D = part.I = 0.0f;
    part.n = 0;
    if (has) {
      Hit h;
      // a partial may stop once its own T < t_min: the ray's T (no larger) is below it too
      walk_cell(s, f, job, my_stk, kRenderThreads, budget, h, [&](const Hit& x) -> bool {
        return shade_voxel<FIELD, RGB, INT>(s, f, sh, x, S, rS, t_min, part);
      });
      if (budget <= 0) {
        cut = true;
        walking = false;
      }
    }
    // fold the group's partials in cell order (every lane of the group computes the same)
    bool any = false, stop = false;
    for (int j = 0; j < P; ++j) {
      const int src = base + j;
      if (__shfl((int)has, src) == 0) continue;
      any = true;
      const float pT = __shfl(part.T, src);
      if (acc.T * pT < t_min) {
        // the ray stops inside cell j: its lane walks the cell again from the ray's state
        if (g == j) {
          Hit h;
          int again = s.step_budget;
          walk_cell(s, f, job, my_stk, kRenderThreads, again, h, [&](const Hit& x) -> bool {
            return shade_voxel<FIELD, RGB, INT>(s, f, sh, x, S, rS, t_min, acc);
          });
        }
        acc.T = __shfl(acc.T, src);
        if (RGB) {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) acc.C[ch] = __shfl(acc.C[ch], src);
        }
        acc.D = __shfl(acc.D, src);
        if (INT) acc.I = __shfl(acc.I, src);
        acc.n = __shfl(acc.n, src);
        if (acc.T < t_min) {
          stop = true;
          break;
        }
        continue;
      }
      if (RGB) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) acc.C[ch] = fmaf(acc.T, __shfl(part.C[ch], src), acc.C[ch]);
      }
      acc.D = fmaf(acc.T, __shfl(part.D, src), acc.D);
      if (INT) acc.I = fmaf(acc.T, __shfl(part.I, src), acc.I);
      acc.n += __shfl(part.n, src);
      acc.T *= pT;
    }
    if (stop || !any) break;
  }
  bool cut_any = false;
  for (int j = 0; j < P; ++j) cut_any = cut_any || __shfl((int)cut, base + j) != 0;
  if (g != 0) return;
  const salf_outputs& out = p.out;
  if (out.rgb) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) out.rgb[ray * 3 + ch] = fmaf(acc.T, p.bg[ch], acc.C[ch]);
  }
  if (out.depth) out.depth[ray] = acc.D;
  if (out.opacity) out.opacity[ray] = 1.0f - acc.T;
  if (out.intensity) out.intensity[ray] = acc.I;
  if (out.t_end) out.t_end[ray] = acc.T;
  if (out.n_hits) out.n_hits[ray] = acc.n;
  if (cut_any) note_cut();
}

// ---- a static scene with dynamic actors (merged traversal)
// The ray in an actor's frame: R^T (o - t), R^T d, each operation rounded in this order.
__device__ __forceinline__ void actor_ray(const ActorPose& a, const float o[3], const float d[3], float oa[3],
                                          float da[3]) {
  const float p[3] = {o[0] - a.t[0], o[1] - a.t[1], o[2] - a.t[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    oa[i] = (a.R[i] * p[0] + a.R[3 + i] * p[1]) + a.R[6 + i] * p[2];
    da[i] = (a.R[i] * d[0] + a.R[3 + i] * d[1]) + a.R[6 + i] * d[2];
  }
}

// Each lane finds the actor boxes its ray meets, then walks the static scene up to the next box,
// the actor inside it (in its frame), and so on, compositing every hit in that order; shading and
// compositing are those of render_wave.
template <int FIELD, bool RGB, bool INT>
__global__ __launch_bounds__(kRenderThreads) void composite_kernel(CompositeParams cp) {
  __shared__ int32_t stk[SALF_MAX_LEVEL * kRenderThreads];
  const RenderParams& p = cp.base;
  const int64_t wave = (blockIdx.x * (int64_t)kRenderThreads + threadIdx.x) >> 6;
  int64_t ray;
  float dir[3];
  RayFrame f;
  if (!lane_ray(p, scheduled_tile(p, wave), threadIdx.x & 63, ray, dir, f)) return;
  const float sh[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // (corner field: no view-dependent term)
  // each lane's actor-box intervals, kept in LDS rather than registers (read once per piece)
  __shared__ float a_in[kMaxActors][kRenderThreads], a_out[kMaxActors][kRenderThreads];
  const int lt = threadIdx.x;
#pragma unroll
  for (int a = 0; a < kMaxActors; ++a) {
    a_in[a][lt] = INFINITY;
    a_out[a][lt] = -INFINITY;
    if (a < cp.n_actors && f.valid) {
      const ActorPose& sa = cp.slot[1 + a];
      float oa[3], da[3];
      actor_ray(sa, f.o, f.d, oa, da);
      const RayFrame fa = make_frame(sa.view, oa, da, f.t_near, f.t_far);
      const int K = sa.view.K;
      const int32_t glo[3] = {0, 0, 0};
      const int32_t ghi[3] = {sa.view.dims[0] << K, sa.view.dims[1] << K,
                              sa.view.dims[2] << K};
      float ti, to;
      if (fa.valid && box_interval(fa, glo, ghi, ti, to) && ti < to) {
        a_in[a][lt] = ti;
        a_out[a][lt] = to;
      }
    }
  }
  Accum acc;
  acc.T = 1.0f;
  acc.C[0] = acc.C[1] = acc.C[2] = 0.0f;
  acc.D = acc.I = 0.0f;
  acc.n = 0;
  const int S = p.S;
  const double rS = 1.0 / S;
  const float t_min = p.t_min;
  bool alive = f.valid;
  // Pieces of the ray, front to back: the static scene from cur up to the next actor box, then that
  // actor inside its box.  Each round every live lane picks its next piece; the wave then runs
  // over the scene slots (static, actor 0, 1, ...) in step, the lanes whose piece is in slot k
  // walking it, so that the walked scene is uniform and one walk serves every slot.
  __shared__ float ray_o[3][kRenderThreads], ray_d[3][kRenderThreads], ray_tf[kRenderThreads];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ray_o[a][lt] = f.o[a];
    ray_d[a][lt] = f.d[a];
  }
  ray_tf[lt] = f.t_far;
  float cur = f.t_near;
  uint32_t done = 0;
  bool ray_done = !alive;
  for (int round = 0; round <= 2 * kMaxActors + 1 && !ray_done; ++round) {
    // the next actor box along the ray (smallest entry, ties by index)
    int nxt = -1;
    float nin = INFINITY, nout = -INFINITY;
#pragma unroll
    for (int a = 0; a < kMaxActors; ++a) {
      const float ti = a_in[a][lt];
      if (!((done >> a) & 1u) && ti < nin) {
        nin = ti;
        nout = a_out[a][lt];
        nxt = a;
      }
    }
    // this round's piece: the static scene up to the next box if any is left, else the actor
    const float s_end = nxt >= 0 ? nin : ray_tf[lt];
    int slot;
    float t0, t1;
    if (cur < s_end) {
      slot = 0;
      t0 = cur;
      t1 = s_end;
      cur = s_end;
    } else if (nxt >= 0) {
      slot = 1 + nxt;
      t0 = nin;
      t1 = nout;
      done |= 1u << nxt;
      cur = fmaxf(cur, nout);
    } else {
      ray_done = true;
      continue;
    }
#pragma unroll 1
    for (int k = 0; k <= cp.n_actors; ++k) {
      if (k != slot) continue;
      const SceneView& sv = cp.slot[k].view;
      // the frame is rebuilt per piece (the static one as the lane built it, make_frame being a
      // function of its arguments), so that only the ray itself stays live across pieces
      float o[3], d[3], oa[3], da[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        o[a] = ray_o[a][lt];
        d[a] = ray_d[a][lt];
      }
      if (k == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          oa[a] = o[a];
          da[a] = d[a];
        }
      } else {
        actor_ray(cp.slot[k], o, d, oa, da);
      }
      const RayFrame fr = make_frame(sv, oa, da, t0, t1);
      traverse(sv, fr, stk + threadIdx.x, kRenderThreads, [&](const Hit& h) -> bool {
        alive = shade_voxel<FIELD, RGB, INT>(sv, fr, sh, h, S, rS, t_min, acc);
        return alive;
      }, note_cut);
    }
    if (!alive) ray_done = true;
  }
  const salf_outputs& out = p.out;
  if (out.rgb) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) out.rgb[ray * 3 + ch] = fmaf(acc.T, p.bg[ch], acc.C[ch]);
  }
  if (out.depth) out.depth[ray] = acc.D;
  if (out.opacity) out.opacity[ray] = 1.0f - acc.T;
  if (out.intensity) out.intensity[ray] = acc.I;
  if (out.t_end) out.t_end[ray] = acc.T;
  if (out.n_hits) out.n_hits[ray] = acc.n;
}

// Request of global tile `tile` in a batch (items sorted by tile_begin, the first at 0).
__device__ __forceinline__ int find_item(const BatchItem* items, int32_t n_items, int64_t tile) {
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].tile_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ----------------------------------------------------------------------------- tile schedule
// Heaviest tiles first (longest-processing-time-first list scheduling).  A tile's cost is the
// root-grid estimate of its centre ray, quantized to kCostBuckets logarithmic buckets; a counting
// sort over the buckets writes the order (block-local histograms in LDS, one global atomic per
// block and bucket).  Ties are placed in arbitrary order, which changes the schedule only, never
// a ray's result.  A launch whose tiles all fit on the GPU at once keeps its own order (sorting
// would only crowd the heavy tiles onto the same compute units): its schedule holds no order.

// Header of the schedule buffer: [0] tiles (0 = no order), [1] tiled | tw_log2 << 8, [2] img_w,
// [3] offset of the order (int32 entries after the header); then keys, order, histogram, cursors.
__global__ void sched_init(int32_t* h, int32_t n_tiles, int32_t layout, int32_t img_w, int32_t order_off,
                           uint32_t* hist) {
  for (int i = threadIdx.x; i < 2 * kCostBuckets; i += blockDim.x) hist[i] = 0u;
  if (threadIdx.x == 0) {
    h[0] = n_tiles;
    h[1] = layout;
    h[2] = img_w;
    h[3] = order_off;
  }
}

// kCostLanes lanes per tile walk consecutive pieces of its centre ray; the tile's cost is their sum.
constexpr int kCostLanes = 8;

// Tiles of one launch (items == nullptr) or the global tiles of a batch of requests.
__global__ __launch_bounds__(kThreads) void tile_cost_kernel(RenderParams p, const BatchItem* items, int32_t n_items,
                                                             int64_t n_tiles, uint32_t* key, uint32_t* hist) {
  static_assert(kThreads == kCostBuckets, "one thread per bucket");
  __shared__ uint32_t local[kCostBuckets];
  local[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t tile = (blockIdx.x * (int64_t)kThreads + threadIdx.x) / kCostLanes;
  const int piece = threadIdx.x % kCostLanes;
  float cost = 0.0f;
  if (tile < n_tiles) {
    const RenderParams* q = &p;
    int64_t lt = tile;
    if (items != nullptr) {
      const int r = find_item(items, n_items, tile);
      q = &items[r].p;
      lt = tile - items[r].tile_begin;
    }
    const int tw = q->tiled ? 1 << q->tw_log2 : 64, th = q->tiled ? 64 >> q->tw_log2 : 1;
    int64_t ray;
    float d[3];
    RayFrame f;
    if (lane_ray(*q, lt, (th / 2) * tw + tw / 2, ray, d, f) || lane_ray(*q, lt, 0, ray, d, f))
      cost = root_cost(q->scene, f, (float)piece / kCostLanes, (float)(piece + 1) / kCostLanes);
  }
#pragma unroll
  for (int m = 1; m < kCostLanes; m <<= 1) cost += __shfl_xor(cost, m);
  if (tile < n_tiles && piece == 0) {
    const int b = (int)(__log2f(1.0f + cost) * 16.0f);
    const uint32_t bucket = (uint32_t)(b < 0 ? 0 : (b >= kCostBuckets ? kCostBuckets - 1 : b));
    key[tile] = bucket;
    atomicAdd(&local[bucket], 1u);
  }
  __syncthreads();
  if (local[threadIdx.x]) atomicAdd(&hist[threadIdx.x], local[threadIdx.x]);
}

__global__ __launch_bounds__(kThreads) void tile_order_kernel(const uint32_t* key, int64_t n_tiles,
                                                              const uint32_t* hist, uint32_t* cursor, int32_t* order) {
  __shared__ uint32_t above[kCostBuckets], local[kCostBuckets], base[kCostBuckets];
  // above[b] = tiles in buckets heavier than b: an exclusive scan from the heaviest bucket down
  const int t = threadIdx.x;
  const uint32_t own = hist[kCostBuckets - 1 - t];
  above[t] = own;
  local[t] = 0u;
  __syncthreads();
  for (int off = 1; off < kCostBuckets; off <<= 1) {
    const uint32_t add = t >= off ? above[t - off] : 0u;
    __syncthreads();
    above[t] += add;
    __syncthreads();
  }
  const uint32_t excl = above[t] - own;
  __syncthreads();
  above[kCostBuckets - 1 - t] = excl;
  // this block's tiles: rank within their bucket in the block, then one range per bucket
  const int64_t tile = blockIdx.x * (int64_t)kThreads + t;
  uint32_t b = 0u, rank = 0u;
  if (tile < n_tiles) {
    b = key[tile];
    rank = atomicAdd(&local[b], 1u);
  }
  __syncthreads();
  if (local[t]) base[t] = atomicAdd(&cursor[t], local[t]);
  __syncthreads();
  if (tile < n_tiles) order[above[b] + base[b] + rank] = (int32_t)tile;
}

// Batched render of several requests in one launch: a grid sized to the GPU's resident capacity
// whose waves pull global tile numbers from a counter until every tile of every request is done
// (each wave's exit condition is that counter passing the tile count).  The request of a tile is
// found by binary search over the requests' first tiles; its shading variant is uniform per wave.
// MASK (bit v: variant v) names the variants the kernel is built for: each one inlined adds to the
// registers the whole kernel holds, so launches whose requests use fewer variants get a kernel
// with only those.  The kernel for pre-activated colour and intensity requests (cameras and LiDARs
// together, the common serving mix) is capped at three waves per SIMD: it would take 194 VGPRs
// (two waves); the cap spills 18 of them and is faster by about 14% in the serving loop.
template <uint32_t MASK>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(MASK == 0x60u ? 3 : 1))) void render_batch_kernel(const BatchItem* items, int32_t n_items,
                                                                int64_t n_tiles, uint32_t* counter,
                                                                const int32_t* sched) {
  __shared__ int32_t stk[SALF_MAX_LEVEL * kThreads];
  __shared__ double seg[6 * kThreads];
  const int lane = threadIdx.x & 63;
  const bool ordered = sched != nullptr && sched[0] == (int32_t)n_tiles;
  for (;;) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(counter, 1u);
    const int64_t slot = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)t);
    if (slot >= n_tiles) break;
    int64_t tile = slot;
    if (ordered) {
      const int32_t o = sched[kSchedHeader + sched[3] + slot];
      if (o >= 0 && o < n_tiles) tile = o;
    }
    const BatchItem& b = items[find_item(items, n_items, tile)];
    const int64_t w = tile - b.tile_begin;
    const int v = b.variant;
    if constexpr ((MASK & 0x01u) != 0) if (v == 0) render_wave<SALF_FIELD_CORNER, false, false>(b.p, w, stk + threadIdx.x, seg + threadIdx.x);
    if constexpr ((MASK & 0x02u) != 0) if (v == 1) render_wave<SALF_FIELD_CORNER, true, false>(b.p, w, stk + threadIdx.x, seg + threadIdx.x);
    if constexpr ((MASK & 0x04u) != 0) if (v == 2) render_wave<SALF_FIELD_CORNER, false, true>(b.p, w, stk + threadIdx.x, seg + threadIdx.x);
    if constexpr ((MASK & 0x08u) != 0) if (v == 3) render_wave<SALF_FIELD_CORNER, true, true>(b.p, w, stk + threadIdx.x, seg + threadIdx.x);
    if constexpr ((MASK & 0x10u) != 0) if (v == 4) render_wave<kFieldCornerActivated, false, false>(b.p, w, stk + threadIdx.x, seg + threadIdx.x);
    if constexpr ((MASK & 0x20u) != 0) if (v == 5) render_wave<kFieldCornerActivated, true, false>(b.p, w, stk + threadIdx.x, seg + threadIdx.x);
    if constexpr ((MASK & 0x40u) != 0) if (v == 6) render_wave<kFieldCornerActivated, false, true>(b.p, w, stk + threadIdx.x, seg + threadIdx.x);
    if constexpr ((MASK & 0x80u) != 0) if (v == 7) render_wave<kFieldCornerActivated, true, true>(b.p, w, stk + threadIdx.x, seg + threadIdx.x);
  }
}

// Hit lists of explicit rays.  FIELD >= 0: with the render's early termination, each ray stopping
// after the voxel that leaves T < t_min, T composited exactly as the render composites it (the
// density alone decides it); FIELD < 0: every hit.
template <int FIELD>
__global__ __launch_bounds__(kThreads) void trace_kernel(SceneView s, salf_rays r, int32_t max_hits, int32_t S,
                                                         float t_min, int32_t* counts, int32_t* ids, float* t_in,
                                                         float* t_out) {
  const int64_t ray = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (ray >= r.n) return;
  float o[3], d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o[a] = r.o[ray * 3 + a];
    d[a] = r.d[ray * 3 + a];
  }
  const RayFrame f = make_frame(s, o, d, r.t_near, r.t_far);
  int32_t n = 0;
  const int64_t base = ray * (int64_t)max_hits;
  __shared__ int32_t stk[SALF_MAX_LEVEL * kThreads];
  const float sh[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  const double rS = 1.0 / S;
  Accum acc;
  acc.T = 1.0f;
  acc.C[0] = acc.C[1] = acc.C[2] = 0.0f;
  acc.D = acc.I = 0.0f;
  acc.n = 0;
  traverse(s, f, stk + threadIdx.x, kThreads, [&](const Hit& h) -> bool {
    if (n < max_hits) {
      ids[base + n] = h.voxel;
      t_in[base + n] = h.t_in;
      t_out[base + n] = h.t_out;
    }
    ++n;
    if constexpr (FIELD >= 0) return shade_voxel<FIELD, false, false>(s, f, sh, h, S, rS, t_min, acc);
    return true;
  }, note_cut);
  counts[ray] = n;
}

__global__ __launch_bounds__(kThreads) void raygen_kernel(salf_sensor s, float* o, float* d, float* t, uint8_t* valid) {
  const int64_t ray = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  const int64_t n = (int64_t)s.width * s.height;
  if (ray >= n) return;
  const int col = (int)(ray % s.width), row = (int)(ray / s.width);
  float ro[3], rd[3], tt;
  const bool ok = sensor_ray(s, col, row, ro, rd, tt);
  if (o) {
#pragma unroll
    for (int a = 0; a < 3; ++a) o[ray * 3 + a] = ro[a];
  }
  if (d) {
#pragma unroll
    for (int a = 0; a < 3; ++a) d[ray * 3 + a] = rd[a];
  }
  if (t) t[ray] = tt;
  if (valid) valid[ray] = ok ? 1 : 0;
}

// Backward of the corner-field render (the derivation is the one of the oracle's gradient):
// with w_j = T_j - T_{j+1} and the suffix sums of a ray formed by prefix subtraction from the
// saved outputs (sum_{k>j} w_k c_k + T_end bg = C - sum_{k<=j} w_k c_k, likewise for D and I),
//   dL/dtau_j = gC.(T_{j+1} c_j - sufC_j) + gD (T_{j+1} t_j - sufD_j) + gI (T_{j+1} i_j - sufI_j)
//               + gO T_end,
// dsigma_j = dL/dtau_j * delta_j, dc_j = gC w_j, di_j = gI w_j; corner logits get these times
// the trilinear weight and the activation's derivative (softplus' = sigmoid, sigmoid' = s(1-s)).
// Transmittance is recomputed front to back; the ray stops after the saved number of voxels.
// PAPER: the field of Eq. 1-2 (raw parameters; ACT is false), with SDF its density replaced by
// Eq. 5-6; else the corner field.
// HITS: the forward stored each ray's hits (fwd.out.hit_voxel, hit_t), and the kernel reads them
// instead of walking the scene: only rays whose hits were all stored; a second launch without
// HITS (walk_only_unstored) walks the others.
template <bool RGB, bool INT, bool ACT, bool PAPER, bool SDF, bool HITS>
__global__ __launch_bounds__(kThreads) void backward_kernel(BackwardParams b) {
  const RenderParams& p = b.fwd;
  int64_t ray;
  float dir[3];
  RayFrame f;
  const int64_t w = (blockIdx.x * (int64_t)kThreads + threadIdx.x) >> 6;
  if (!lane_ray(p, scheduled_tile(p, w), threadIdx.x & 63, ray, dir, f)) return;
  const int32_t n_stop = p.out.n_hits[ray];
  if (n_stop <= 0) return;
  if (HITS ? n_stop > p.out.hit_capacity : (b.walk_only_unstored && n_stop <= p.out.hit_capacity)) return;
  const float T_end = p.out.t_end[ray];
  float gC[3] = {0.0f, 0.0f, 0.0f}, Cs[3] = {0.0f, 0.0f, 0.0f};
  if (RGB) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      gC[ch] = b.g.d_rgb[ray * 3 + ch];
      Cs[ch] = p.out.rgb[ray * 3 + ch];
    }
  }
  const float gD = b.g.d_depth ? b.g.d_depth[ray] : 0.0f;
  const float Ds = b.g.d_depth ? p.out.depth[ray] : 0.0f;
  const float gI = INT ? b.g.d_intensity[ray] : 0.0f;
  const float Is = INT ? p.out.intensity[ray] : 0.0f;
  const float gOT = (b.g.d_opacity ? b.g.d_opacity[ray] : 0.0f) * T_end;
  const SceneView& s = p.scene;
  const int S = p.S;
  const double rS = 1.0 / S;
  float T = 1.0f, PC[3] = {0.0f, 0.0f, 0.0f}, PD = 0.0f, PI = 0.0f;
  int32_t count = 0;
  // per-wave gradient rows in LDS, [row][lane] with a stride of 65 so that the lanes summing
  // different rows of one lane's column hit different banks
  constexpr int kIntRow = RGB ? 32 : 8;
  constexpr int kRows = kIntRow + (INT ? 8 : 0);
  constexpr int kRedStride = 65;
  __shared__ float red_all[(kThreads / 64) * kRows * kRedStride];
  float* red = red_all + (threadIdx.x >> 6) * (kRows * kRedStride);
  // per-wave list of the lanes whose voxel no other lane of the pass hit, and their voxels
  __shared__ int32_t one_all[2 * kThreads];
  int32_t* one_lane = one_all + (threadIdx.x >> 6) * 128;
  int32_t* one_vox = one_lane + 64;
  const int lane = threadIdx.x & 63;
  __shared__ int32_t stk[SALF_MAX_LEVEL * kThreads];
  // degree-1 SH basis of the ray direction (paper field), as in the forward
  const float shb[4] = {kShC0, kShC1 * dir[0], kShC1 * dir[1], kShC1 * dir[2]};
  const auto visit = [&](const Hit& h) -> bool {
    const int32_t v = h.voxel;
    const float ti = h.t_in;
    // activated corner values (stored ones when the scene keeps them, else from the logits); for
    // the paper field the raw parameters
    float sp[8], cr[3][8], ci[8];
    if constexpr (PAPER) {
      const float4* gp = reinterpret_cast<const float4*>(s.geo + (int64_t)v * 8);
      const float4 g0 = gp[0];
      sp[0] = g0.x; sp[1] = g0.y; sp[2] = g0.z; sp[3] = g0.w;
      if (SDF) {
        const float4 g1 = gp[1];
        sp[4] = 0.5f * __expf(g1.x);  // a / 2
        sp[5] = __expf(-g1.y);        // 1 / b
      }
      if (RGB) {
        const float4* cp = reinterpret_cast<const float4*>(s.rgb + (int64_t)v * 24);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          const float4 a = cp[2 * ch], q = cp[2 * ch + 1];
          cr[ch][0] = a.x; cr[ch][1] = a.y; cr[ch][2] = a.z; cr[ch][3] = a.w;
          cr[ch][4] = q.x; cr[ch][5] = q.y; cr[ch][6] = q.z;
          // the view-dependent term of the colour logit, as the forward forms it
          cr[ch][7] = fmaf(cr[ch][3], shb[0], fmaf(cr[ch][4], shb[1], fmaf(cr[ch][5], shb[2], cr[ch][6] * shb[3])));
        }
      }
      if (INT) {
        const float4 a = reinterpret_cast<const float4*>(s.inten + (int64_t)v * 8)[0];
        ci[0] = a.x; ci[1] = a.y; ci[2] = a.z; ci[3] = a.w;
      }
    } else {
      const float4* gp = reinterpret_cast<const float4*>((ACT ? s.act_geo : s.geo) + (int64_t)v * 8);
      const float4 g0 = gp[0], g1 = gp[1];
      const float g[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
#pragma unroll
      for (int i = 0; i < 8; ++i) sp[i] = ACT ? g[i] : softplus_f(g[i]);
    if (RGB) {
      const float4* cp = reinterpret_cast<const float4*>((ACT ? s.act_rgb : s.rgb) + (int64_t)v * 24);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float4 a = cp[2 * ch], q = cp[2 * ch + 1];
        const float z[8] = {a.x, a.y, a.z, a.w, q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) cr[ch][i] = ACT ? z[i] : sigmoid_f(z[i]);
      }
    }
    if (INT) {
      const float4* ip = reinterpret_cast<const float4*>((ACT ? s.act_int : s.inten) + (int64_t)v * 8);
      const float4 a = ip[0], q = ip[1];
      const float z[8] = {a.x, a.y, a.z, a.w, q.x, q.y, q.z, q.w};
#pragma unroll
      for (int i = 0; i < 8; ++i) ci[i] = ACT ? z[i] : sigmoid_f(z[i]);
    }
    }
    float rel[3], stp[3], delta, sc;
    segment_frame(s, f, h, rS, rel, stp, delta, sc);
    // ag: dL/d(corner density) before the activation; aw: sum over samples of weight x corner
    // weight, which times a channel's output gradient is that channel's corner gradient
    float ag[8], aw[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) ag[i] = aw[i] = 0.0f;
    // paper field: per channel, the colour logit's gradient times (x, 1)
    float pc[3][4];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) pc[ch][0] = pc[ch][1] = pc[ch][2] = pc[ch][3] = 0.0f;
    for (int k = 0; k < S; ++k) {
      const float fk = (float)k + 0.5f;
      float u[3], w[8], x[3], sdq = 0.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a) u[a] = sample_u(rel[a], stp[a], fk, sc);
      // the forward's arithmetic, operation for operation, so T matches it bit for bit (the colour and
      // intensity prefix sums, formed per sample here, agree with its per-voxel dot products up to
      // FP32 rounding)
      float sigma, col[3] = {0.0f, 0.0f, 0.0f}, inten = 0.0f;
      if constexpr (PAPER) {
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] = fmaf(2.0f, u[a], -1.0f);
        sdq = fmaf(sp[0], x[0], fmaf(sp[1], x[1], fmaf(sp[2], x[2], sp[3])));
        sigma = SDF ? sdf_sigma(sdq, sp[4], sp[5]) : __expf(sdq);
        if (RGB) {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch)
            col[ch] = sigmoid_f(fmaf(cr[ch][0], x[0], fmaf(cr[ch][1], x[1], fmaf(cr[ch][2], x[2], cr[ch][7]))));
        }
        if (INT) inten = sigmoid_f(fmaf(ci[0], x[0], fmaf(ci[1], x[1], fmaf(ci[2], x[2], ci[3]))));
      } else {
        corner_weights(u, w);
        sigma = dot8(w, sp);
        if (RGB) {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) col[ch] = dot8(w, cr[ch]);
        }
        if (INT) inten = dot8(w, ci);
      }
      const float e = __expf(-sigma * delta);
      const float wgt = T * (1.0f - e);
      const float Tn = T * e;
      const float tk = fmaf(fk, delta, ti);
      float dtau = gOT;
      if (RGB) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          PC[ch] = fmaf(wgt, col[ch], PC[ch]);
          dtau = fmaf(gC[ch], fmaf(Tn, col[ch], -(Cs[ch] - PC[ch])), dtau);
        }
      }
      PD = fmaf(wgt, tk, PD);
      dtau = fmaf(gD, fmaf(Tn, tk, -(Ds - PD)), dtau);
      if (INT) {
        PI = fmaf(wgt, inten, PI);
        dtau = fmaf(gI, fmaf(Tn, inten, -(Is - PI)), dtau);
      }
      const float dsig = dtau * delta;
      if constexpr (PAPER) {
        // ag[0:4]: d/d(density parameters) = dsig sigma (x, 1); aw[ch * 2 + 0:1] hold no corner
        // weights here: aw[0:3] and pc: d/d(colour logit) x (x, 1) per channel, pi likewise
        // d(sigma)/d(affine form): sigma itself, or for the SDF density (a / 2b) exp(-|s| / b)
        float ds;
        if (SDF) {
          const float e = __expf(-fabsf(sdq) * sp[5]);
          ds = dsig * (sp[4] * sp[5] * e);
          ag[4] = fmaf(dsig, sigma, ag[4]);                       // d/d(log a) = sigma
          ag[5] = fmaf(dsig, -(sp[4] * sdq * sp[5] * e), ag[5]);  // d/d(log b)
        } else {
          ds = dsig * sigma;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) ag[a] = fmaf(ds, x[a], ag[a]);
        ag[3] += ds;
        if (RGB) {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            const float gl = gC[ch] * wgt * (col[ch] * (1.0f - col[ch]));
#pragma unroll
            for (int a = 0; a < 3; ++a) pc[ch][a] = fmaf(gl, x[a], pc[ch][a]);
            pc[ch][3] += gl;
          }
        }
        if (INT) {
          const float gl = gI * wgt * (inten * (1.0f - inten));
#pragma unroll
          for (int a = 0; a < 3; ++a) aw[a] = fmaf(gl, x[a], aw[a]);
          aw[3] += gl;
        }
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          ag[i] = fmaf(dsig, w[i], ag[i]);
          aw[i] = fmaf(wgt, w[i], aw[i]);
        }
      }
      T = Tn;
    }
    // this lane's gradient row for the voxel (activation derivative applied): 8 density corners,
    // then 24 colour and 8 intensity corners when present.  softplus' = sigmoid, and
    // sigmoid(z) = 1 - exp(-softplus(z)), from the activated value either way.  The paper
    // field's rows follow its record layout (density a, b; per channel A, then the SH
    // coefficients B times the basis; intensity a, b), zero in the unused slots.
    if constexpr (PAPER) {
#pragma unroll
      for (int i = 0; i < 8; ++i) red[i * kRedStride + lane] = i < (SDF ? 6 : 4) ? ag[i] : 0.0f;
      if (RGB) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
#pragma unroll
          for (int i = 0; i < 8; ++i)
            red[(8 + ch * 8 + i) * kRedStride + lane] =
                i < 3 ? pc[ch][i] : (i < 7 ? pc[ch][3] * shb[i - 3] : 0.0f);
      }
      if (INT) {
#pragma unroll
        for (int i = 0; i < 8; ++i) red[(kIntRow + i) * kRedStride + lane] = i < 4 ? aw[i] : 0.0f;
      }
    } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) red[i * kRedStride + lane] = ag[i] * -expm1f(-sp[i]);
    if (RGB) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int i = 0; i < 8; ++i)
          red[(8 + ch * 8 + i) * kRedStride + lane] = (gC[ch] * aw[i]) * (cr[ch][i] * (1.0f - cr[ch][i]));
    }
    if (INT) {
#pragma unroll
      for (int i = 0; i < 8; ++i) red[(kIntRow + i) * kRedStride + lane] = (gI * aw[i]) * (ci[i] * (1.0f - ci[i]));
    }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Lanes that hit the same voxel at this point form a group; the group's rows are added over
    // its members and sent out with one atomic per value, instead of one atomic per value and
    // lane on the same addresses.
    uint64_t pending = __ballot(1), mine = 0;
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const int32_t vl = __shfl(v, leader);
      const uint64_t m = __ballot(v == vl) & pending;
      if (v == vl) mine = m;
      pending &= ~m;
    }
    const int size = __popcll(mine);
    const uint64_t below = (1ull << lane) - 1ull;
    const uint64_t ones = __ballot(size == 1);
    if constexpr (HITS) {
      if (size == 1) {
        const int r = __popcll(ones & below);
        one_lane[r] = lane;
        one_vox[r] = v;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // row j of voxel w (nullptr: not wanted, or a slot the paper field's record does not use)
    const auto row_dst = [&](int32_t w, int j) -> float* {
      if (PAPER && (j < 8 ? j >= (SDF ? 6 : 4) : (RGB && j < 32 ? ((j - 8) & 7) == 7 : j - kIntRow >= 4))) return nullptr;
      return j < 8 ? (b.dgeo ? b.dgeo + (int64_t)w * 8 + j : nullptr)
                   : (RGB && j < 32 ? (b.drgb ? b.drgb + (int64_t)w * 24 + (j - 8) : nullptr)
                                    : (b.dint ? b.dint + (int64_t)w * 8 + (j - kIntRow) : nullptr));
    };
    const uint64_t act = __ballot(1);
    const int nact = __popcll(act), me = __popcll(act & below);
    // voxels that no other lane of the pass hit: their rows go out as they are.  Reading stored
    // hits, the lanes run in lock step and most of the wave is in every pass: the lanes take
    // consecutive (voxel, row) pairs, so that one atomic instruction writes whole rows of one or
    // two voxels (a few memory requests) instead of one value of each lane's own voxel (one
    // request per lane).  Walking, fewer lanes share a pass and each sends its own rows.
    if constexpr (HITS) {
      const int n_one = __popcll(ones) * kRows;
      for (int t = me; t < n_one; t += nact) {
        const int k = t / kRows, j = t - k * kRows;
        float* dst = row_dst(one_vox[k], j);
        if (dst) unsafeAtomicAdd(dst, red[j * kRedStride + one_lane[k]]);
      }
    } else if (size == 1) {
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        float* dst = row_dst(v, j);
        if (dst) unsafeAtomicAdd(dst, red[j * kRedStride + lane]);
      }
    }
    // the groups of two or more lanes, one at a time, every lane of the pass helping: a group's
    // member mask is uniform, so its members are walked with scalar instructions while each lane
    // adds one row over them
    for (uint64_t heads = __ballot(size > 1 && (mine & below) == 0); heads; heads &= heads - 1ull) {
      const int ld = __ffsll((long long)heads) - 1;
      const uint32_t m_lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mine, ld);
      const uint32_t m_hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mine >> 32), ld);
      const uint64_t members = (uint64_t)m_lo | ((uint64_t)m_hi << 32);
      const int32_t vg = __builtin_amdgcn_readlane(v, ld);
      for (int j = me; j < kRows; j += nact) {
        float* dst = row_dst(vg, j);
        if (!dst) continue;
        float sum = 0.0f;
        for (uint64_t m = members; m; m &= m - 1ull) sum += red[j * kRedStride + (__ffsll((long long)m) - 1)];
        unsafeAtomicAdd(dst, sum);
      }
    }
    return ++count < n_stop;
  };
  if constexpr (HITS) {
    const int32_t* hv = p.out.hit_voxel;
    const float2* ht = reinterpret_cast<const float2*>(p.out.hit_t);
    for (int32_t k = 0; k < n_stop; ++k) {
      const int64_t at = (int64_t)k * p.n + ray;
      Hit h;
      h.voxel = hv[at];
      const float2 t = ht[at];
      h.t_in = t.x;
      h.t_out = t.y;
      const int4 bx = b.vbox[h.voxel];
      h.lo[0] = bx.x;
      h.lo[1] = bx.y;
      h.lo[2] = bx.z;
      h.size = bx.w;
      visit(h);
    }
  } else {
    traverse(s, f, stk + threadIdx.x, kThreads, visit, note_cut);
  }
}

template <int FIELD>
hipError_t launch_field(const RenderParams& p, unsigned blocks, hipStream_t stream) {
  const bool rgb = p.out.rgb != nullptr, in = p.out.intensity != nullptr;
  if (p.pieces > 1) {
    blocks *= (unsigned)p.pieces;
    if (rgb && in) render_split_kernel<FIELD, true, true><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
    else if (rgb) render_split_kernel<FIELD, true, false><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
    else if (in) render_split_kernel<FIELD, false, true><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
    else render_split_kernel<FIELD, false, false><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
    return hipGetLastError();
  }
  if (p.out.hit_voxel != nullptr) {
    if (rgb && in) render_kernel<FIELD, true, true, true><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
    else if (rgb) render_kernel<FIELD, true, false, true><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
    else if (in) render_kernel<FIELD, false, true, true><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
    else render_kernel<FIELD, false, false, true><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
    return hipGetLastError();
  }
  if (rgb && in) render_kernel<FIELD, true, true, false><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
  else if (rgb) render_kernel<FIELD, true, false, false><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
  else if (in) render_kernel<FIELD, false, true, false><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
  else render_kernel<FIELD, false, false, false><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace

namespace {
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

namespace {
// Schedule of the tiles of one launch (items == nullptr: p's tiles) or of a batch of requests.
hipError_t schedule_tiles(const RenderParams& p, const BatchItem* items, int32_t n_items, int64_t n_tiles,
                          int64_t capacity, void* work, hipStream_t stream) {
  // waves the GPU holds at once: 4 SIMDs per compute unit, 4 waves each at the render kernels'
  // register use (per device, queried once; concurrent first calls only repeat the query)
  static std::atomic<int> resident[64];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int held = (dev >= 0 && dev < 64) ? resident[dev].load(std::memory_order_relaxed) : 0;
  if (held == 0) {
    int cus = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    held = 16 * (cus > 0 ? cus : 1);
    if (dev >= 0 && dev < 64) resident[dev].store(held, std::memory_order_relaxed);
  }
  // no order for a launch that fits on the GPU at once or exceeds the buffer's capacity; the
  // buffer then holds only the header and the (unused) histograms
  const bool sort = n_tiles > 1 && n_tiles <= capacity && n_tiles > held;
  const int64_t lay = sort ? n_tiles : 0;
  char* w = (char*)work;
  int32_t* hdr = (int32_t*)w;
  uint32_t* key = (uint32_t*)(w + kSchedHeader * 4);
  int32_t* order = (int32_t*)(w + kSchedHeader * 4 + align256((size_t)lay * 4));
  uint32_t* hist = (uint32_t*)(w + kSchedHeader * 4 + 2 * align256((size_t)lay * 4));
  uint32_t* cursor = hist + kCostBuckets;
  const int32_t order_off = (int32_t)(align256((size_t)lay * 4) / 4);
  sched_init<<<1, 256, 0, stream>>>(hdr, sort ? (int32_t)n_tiles : 0, p.tiled | (p.tw_log2 << 8), p.img_w, order_off,
                                    hist);
  if (sort) {
    const unsigned blocks = (unsigned)((n_tiles + kThreads - 1) / kThreads);
    tile_cost_kernel<<<(unsigned)((n_tiles * kCostLanes + kThreads - 1) / kThreads), kThreads, 0, stream>>>(
        p, items, n_items, n_tiles, key, hist);
    tile_order_kernel<<<blocks, kThreads, 0, stream>>>(key, n_tiles, hist, cursor, order);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tile_schedule(const RenderParams& p, void* work, hipStream_t stream) {
  const int64_t n_tiles = tile_count(p);
  return schedule_tiles(p, nullptr, 0, n_tiles, n_tiles, work, stream);
}

hipError_t launch_batch_schedule(const BatchItem* d_items, int32_t n_items, int64_t n_tiles, void* work,
                                 hipStream_t stream) {
  RenderParams none;
  memset(&none, 0, sizeof(none));
  return schedule_tiles(none, d_items, n_items, n_tiles, kBatchScheduleTiles, work, stream);
}

hipError_t launch_composite(const CompositeParams& cp, bool activated, hipStream_t stream) {
  const RenderParams& p = cp.base;
  const int64_t threads = p.tiled ? (int64_t)p.tiles_x * p.tiles_y * 64 : p.n;
  if (threads <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((threads + kThreads - 1) / kThreads);
  const bool rgb = p.out.rgb != nullptr, in = p.out.intensity != nullptr;
  constexpr int A = kFieldCornerActivated, C = SALF_FIELD_CORNER;
  if (activated) {
    if (rgb && in) composite_kernel<A, true, true><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(cp);
    else if (rgb) composite_kernel<A, true, false><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(cp);
    else if (in) composite_kernel<A, false, true><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(cp);
    else composite_kernel<A, false, false><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(cp);
  } else {
    if (rgb && in) composite_kernel<C, true, true><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(cp);
    else if (rgb) composite_kernel<C, true, false><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(cp);
    else if (in) composite_kernel<C, false, true><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(cp);
    else composite_kernel<C, false, false><<<blocks * (kThreads / kRenderThreads), kRenderThreads, 0, stream>>>(cp);
  }
  return hipGetLastError();
}

hipError_t launch_render(const RenderParams& p, int field, hipStream_t stream) {
  const int64_t threads = p.tiled ? (int64_t)p.tiles_x * p.tiles_y * 64 : p.n;
  if (threads <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((threads + kThreads - 1) / kThreads);
  if (field == SALF_FIELD_PAPER) return launch_field<SALF_FIELD_PAPER>(p, blocks, stream);
  if (field == SALF_FIELD_SDF) return launch_field<kFieldSdf>(p, blocks, stream);
  if (p.scene.act_geo != nullptr) return launch_field<kFieldCornerActivated>(p, blocks, stream);
  return launch_field<SALF_FIELD_CORNER>(p, blocks, stream);
}

namespace {
// Kernels of the batched launch, each built for a set of variants: pre-activated colour-only and
// intensity-only requests (cameras and LiDARs), every pre-activated variant, every variant.
constexpr uint32_t kBatchMasks[3] = {0x60u, 0xF0u, 0xFFu};

template <uint32_t MASK>
hipError_t launch_batch_mask(int slot, const BatchItem* d_items, int32_t n_items, int64_t n_tiles,
                             uint32_t* d_counter, const int32_t* d_sched, hipStream_t stream) {
  // blocks of this kernel the whole GPU keeps resident (per device and kernel, queried once)
  static std::atomic<int> resident[3][64];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int resident_blocks = (dev >= 0 && dev < 64) ? resident[slot][dev].load(std::memory_order_relaxed) : 0;
  if (resident_blocks == 0) {
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, render_batch_kernel<MASK>, kThreads, 0);
    if (e != hipSuccess) return e;
    resident_blocks = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
    if (dev >= 0 && dev < 64) resident[slot][dev].store(resident_blocks, std::memory_order_relaxed);
  }
  const int64_t want = (n_tiles + 3) / 4;  // 4 waves per block
  const unsigned blocks = (unsigned)(want < resident_blocks ? want : resident_blocks);
  render_batch_kernel<MASK><<<blocks, kThreads, 0, stream>>>(d_items, n_items, n_tiles, d_counter, d_sched);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_render_batch(const BatchItem* d_items, int32_t n_items, int64_t n_tiles, uint32_t* d_counter,
                               const int32_t* d_sched, uint32_t variants, hipStream_t stream) {
  if (n_items <= 0 || n_tiles <= 0) return hipSuccess;
  if ((variants & ~kBatchMasks[0]) == 0)
    return launch_batch_mask<kBatchMasks[0]>(0, d_items, n_items, n_tiles, d_counter, d_sched, stream);
  if ((variants & ~kBatchMasks[1]) == 0)
    return launch_batch_mask<kBatchMasks[1]>(1, d_items, n_items, n_tiles, d_counter, d_sched, stream);
  return launch_batch_mask<kBatchMasks[2]>(2, d_items, n_items, n_tiles, d_counter, d_sched, stream);
}

namespace {
template <bool HITS>
hipError_t launch_backward_pass(const BackwardParams& b, int field, unsigned blocks, hipStream_t stream) {
  const bool rgb = b.g.d_rgb != nullptr, in = b.g.d_intensity != nullptr;
  const RenderParams& p = b.fwd;
  if (field == SALF_FIELD_SDF) {
    if (rgb && in) backward_kernel<true, true, false, true, true, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else if (rgb) backward_kernel<true, false, false, true, true, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else if (in) backward_kernel<false, true, false, true, true, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else backward_kernel<false, false, false, true, true, HITS><<<blocks, kThreads, 0, stream>>>(b);
  } else if (field == SALF_FIELD_PAPER) {
    if (rgb && in) backward_kernel<true, true, false, true, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else if (rgb) backward_kernel<true, false, false, true, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else if (in) backward_kernel<false, true, false, true, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else backward_kernel<false, false, false, true, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
  } else if (p.scene.act_geo != nullptr) {
    if (rgb && in) backward_kernel<true, true, true, false, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else if (rgb) backward_kernel<true, false, true, false, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else if (in) backward_kernel<false, true, true, false, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else backward_kernel<false, false, true, false, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
  } else {
    if (rgb && in) backward_kernel<true, true, false, false, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else if (rgb) backward_kernel<true, false, false, false, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else if (in) backward_kernel<false, true, false, false, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
    else backward_kernel<false, false, false, false, false, HITS><<<blocks, kThreads, 0, stream>>>(b);
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_backward(const BackwardParams& b, int field, hipStream_t stream) {
  const RenderParams& p = b.fwd;
  const int64_t threads = p.tiled ? (int64_t)p.tiles_x * p.tiles_y * 64 : p.n;
  if (threads <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((threads + kThreads - 1) / kThreads);
  if (p.out.hit_voxel == nullptr || b.vbox == nullptr) return launch_backward_pass<false>(b, field, blocks, stream);
  // stored hits: every ray whose hits were all stored, then a walk of the others
  hipError_t e = launch_backward_pass<true>(b, field, blocks, stream);
  if (e != hipSuccess) return e;
  BackwardParams rest = b;
  rest.walk_only_unstored = 1;
  return launch_backward_pass<false>(rest, field, blocks, stream);
}

hipError_t launch_trace(const SceneView& s, const salf_rays& r, int32_t max_hits, int field, int32_t S, float t_min,
                        int32_t* counts, int32_t* ids, float* t_in, float* t_out, hipStream_t stream) {
  if (r.n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((r.n + kThreads - 1) / kThreads);
  if (field < 0)
    trace_kernel<-1><<<blocks, kThreads, 0, stream>>>(s, r, max_hits, S, t_min, counts, ids, t_in, t_out);
  else if (field == SALF_FIELD_PAPER)
    trace_kernel<SALF_FIELD_PAPER><<<blocks, kThreads, 0, stream>>>(s, r, max_hits, S, t_min, counts, ids, t_in, t_out);
  else if (field == SALF_FIELD_SDF)
    trace_kernel<kFieldSdf><<<blocks, kThreads, 0, stream>>>(s, r, max_hits, S, t_min, counts, ids, t_in, t_out);
  else if (s.act_geo != nullptr)
    trace_kernel<kFieldCornerActivated><<<blocks, kThreads, 0, stream>>>(s, r, max_hits, S, t_min, counts, ids, t_in,
                                                                         t_out);
  else
    trace_kernel<SALF_FIELD_CORNER><<<blocks, kThreads, 0, stream>>>(s, r, max_hits, S, t_min, counts, ids, t_in,
                                                                     t_out);
  return hipGetLastError();
}

hipError_t read_cut_rays(hipStream_t stream, uint32_t* total) {
  hipError_t e = hipMemcpyFromSymbolAsync(total, HIP_SYMBOL(g_cut_rays), sizeof(uint32_t), 0, hipMemcpyDeviceToHost,
                                          stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return e;
}

hipError_t launch_raygen(const salf_sensor& s, float* o, float* d, float* t, uint8_t* valid, hipStream_t stream) {
  const int64_t n = (int64_t)s.width * s.height;
  if (n <= 0) return hipSuccess;
  raygen_kernel<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, stream>>>(s, o, d, t, valid);
  return hipGetLastError();
}

}  // namespace salf
