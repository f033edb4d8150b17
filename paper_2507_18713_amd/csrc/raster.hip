// Tile-based splatting of the voxels onto a global-shutter pinhole image (Sec. 3.2 "Tile-based
// Splatting"): project and cull every voxel, list it under every 16x16-pixel tile its footprint
// overlaps, sort each tile's list front to back, and let one workgroup per tile stage its voxels'
// boxes and parameters in LDS chunk by chunk while each of its 256 lanes (one pixel) composites the
// voxels its ray meets.
//
// The depth order is the front-to-back order of the voxel grid seen from the eye: the L1 distance
// in root cells from the eye's root cell, then the octant digits of each level relative to the
// eye's side of the node's mid-planes.  It strictly increases along the hits of every ray from the
// eye, so a pixel composites exactly the hits a ray cast of its ray finds, in the same order, with
// the same interval rule and shading arithmetic (shade.hpp): the outputs are the ray cast's bits.
//
// Steps per frame: count (tiles per voxel) -> exclusive scan -> the pair count read back to the
// host (the one synchronization: the sort's size is a host argument) -> emit (tile, key) pairs ->
// radix sort -> tile ranges -> the tile kernel.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "internal.hpp"
#include "shade.hpp"

namespace salf {
namespace {

constexpr int kTile = 16;          // pixels per tile side (one workgroup of 256 lanes per tile)
constexpr int kChunk = 128;        // voxels staged in LDS per round
constexpr double kZNear = 1e-2;    // metres: a voxel reaching closer to the camera plane covers the image
// Pixels added around each projected rectangle, so that every pixel whose float32 ray meets the
// voxel lies inside it: the rays' directions are within ~1e-6 rad of the exact pixel-centre ray
// (a few thousandths of a pixel at the focal lengths of full-HD and 4K frames), 0.05 px is ten
// times that.
constexpr double kMargin = 0.05;

// Inclusive pixel rectangle of voxel box b (finest cells: min corner, edge), or false when culled:
// every corner behind the camera plane, or a rectangle off the image.  A voxel reaching closer
// than kZNear covers the whole image.  FP64, widened by kMargin for rays that graze the voxel.
__device__ __forceinline__ bool footprint(const RasterParams& p, const int4 b, int& px0, int& py0, int& px1,
                                          int& py1) {
  const SceneView& s = p.scene;
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  bool front = false, near = false;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const double g[3] = {(double)(b.x + ((c & 1) ? b.w : 0)), (double)(b.y + ((c & 2) ? b.w : 0)),
                         (double)(b.z + ((c & 4) ? b.w : 0))};
    double d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = s.org[a] + g[a] / s.gs - p.eye[a];
    // camera frame: R^T d (R row-major, sensor to world)
    const double X = p.R[0] * d[0] + p.R[3] * d[1] + p.R[6] * d[2];
    const double Y = p.R[1] * d[0] + p.R[4] * d[1] + p.R[7] * d[2];
    const double Z = p.R[2] * d[0] + p.R[5] * d[1] + p.R[8] * d[2];
    front = front || Z > 0.0;
    near = near || Z < kZNear;
    if (Z >= kZNear) {
      const double x = p.cx + p.fx * X / Z, y = p.cy + p.fy * Y / Z;
      xmin = fmin(xmin, x);
      xmax = fmax(xmax, x);
      ymin = fmin(ymin, y);
      ymax = fmax(ymax, y);
    }
  }
  if (!front) return false;
  if (near) {
    px0 = py0 = 0;
    px1 = p.width - 1;
    py1 = p.height - 1;
    return true;
  }
  // the pixels whose centre (u + 1/2) lies in the widened rectangle; none: no pixel ray meets it
  const double u0 = ceil(xmin - 0.5 - kMargin), u1 = floor(xmax - 0.5 + kMargin);
  const double r0 = ceil(ymin - 0.5 - kMargin), r1 = floor(ymax - 0.5 + kMargin);
  if (u0 > u1 || r0 > r1) return false;
  if (u1 < 0.0 || r1 < 0.0 || u0 > (double)(p.width - 1) || r0 > (double)(p.height - 1)) return false;
  px0 = (int)fmax(u0, 0.0);
  px1 = (int)fmin(u1, (double)(p.width - 1));
  py0 = (int)fmax(r0, 0.0);
  py1 = (int)fmin(r1, (double)(p.height - 1));
  return true;
}

// Front-to-back key of a voxel box seen from the eye (og: the eye in the FP32 grid frame of the
// interval rule, eye_root: its root cell clamped to one cell outside the grid).
__device__ __forceinline__ uint64_t depth_key(const RasterParams& p, const int4 b) {
  const int K = p.scene.K;
  const int lo[3] = {b.x, b.y, b.z};
  uint64_t l1 = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int r = lo[a] >> K;
    l1 += (uint64_t)(r >= p.eye_root[a] ? r - p.eye_root[a] : p.eye_root[a] - r);
  }
  const int level = K - (31 - __clz(b.w));
  uint64_t digits = 0;
  for (int j = 1; j <= level; ++j) {
    const int half = 1 << (K - j);
    uint32_t rel = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int mid = ((lo[a] >> (K - j + 1)) << (K - j + 1)) + half;
      const uint32_t bit = (uint32_t)(lo[a] >> (K - j)) & 1u;
      const uint32_t eye = p.og[a] >= (float)mid ? 1u : 0u;
      rel |= (bit ^ eye) << a;
    }
    digits |= (uint64_t)rel << (3 * (K - j));
  }
  return (l1 << (3 * K)) | digits;
}

// Tiles per voxel, the voxel's pixel rectangle (u0 | u1 << 16, r0 | r1 << 16: the tile kernel's
// per-pixel pre-test, and the tiles it is listed under) and its depth key.
__global__ void raster_count_kernel(RasterParams p) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v > p.n_voxels) return;
  uint32_t n = 0;
  int px0, py0, px1, py1;
  if (v < p.n_voxels && footprint(p, p.vbox[v], px0, py0, px1, py1)) {
    n = (uint32_t)((px1 / kTile - px0 / kTile + 1) * (py1 / kTile - py0 / kTile + 1));
    p.rect[v] = make_uint2((uint32_t)px0 | ((uint32_t)px1 << 16), (uint32_t)py0 | ((uint32_t)py1 << 16));
    p.vkey[v] = depth_key(p, p.vbox[v]);
  }
  p.count[v] = n;  // count[n_voxels] = 0 closes the scan
}

// One thread per pair: its voxel is the last one whose scan offset is at most the pair's index
// (voxels without pairs share their successor's offset and are passed over), the pair's tile the
// k-th of the voxel's tile rectangle, row by row.  Writes are coalesced whatever the footprints.
__global__ void raster_emit_kernel(RasterParams p, int64_t n_pairs) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_pairs) return;
  int64_t lo = 0, hi = p.n_voxels - 1;  // offset[lo] <= i < offset[n_voxels]
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (p.offset[mid] <= (uint64_t)i) lo = mid;
    else hi = mid - 1;
  }
  const int64_t v = lo;
  const uint32_t k = (uint32_t)((uint64_t)i - p.offset[v]);
  const uint2 rc = p.rect[v];
  const int tx0 = (int)(rc.x & 0xffffu) / kTile, tx1 = (int)(rc.x >> 16) / kTile;
  const int ty0 = (int)(rc.y & 0xffffu) / kTile;
  const uint32_t w = (uint32_t)(tx1 - tx0 + 1);
  const int tx = tx0 + (int)(k % w), ty = ty0 + (int)(k / w);
  p.keys[i] = ((uint64_t)(ty * p.tiles_x + tx) << p.key_bits) | p.vkey[v];
  p.vals[i] = (uint32_t)v;
}

// Tiles heaviest first: key ~(list length), so that an ascending sort puts the longest lists first
// (the launch's tail is its longest tiles; starting them first shortens it).
__global__ void raster_length_kernel(const uint2* range, int64_t n_tiles, uint32_t* key, uint32_t* tile) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const uint2 r = range[t];
  key[t] = ~(r.y - r.x);
  tile[t] = (uint32_t)t;
}

__global__ void raster_range_kernel(const uint64_t* keys, int64_t n_pairs, int key_bits, int64_t n_tiles,
                                    uint2* range) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_pairs) return;
  const uint64_t t = keys[i] >> key_bits;
  if (t >= (uint64_t)n_tiles) return;
  if (i == 0 || (keys[i - 1] >> key_bits) != t) range[t].x = (uint32_t)i;
  if (i == n_pairs - 1 || (keys[i + 1] >> key_bits) != t) range[t].y = (uint32_t)(i + 1);
}

__global__ void raster_clear_kernel(uint2* range, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) range[i] = make_uint2(0u, 0u);
}

// One workgroup per tile, one lane per pixel.  Each round stages kChunk voxels of the tile's sorted
// list (ids, boxes, parameter rows) in LDS, then every live pixel tests its ray against them in
// order and composites the hits; the tile stops once every pixel has stopped.
template <int FIELD, bool RGB, bool INT>
__global__ __launch_bounds__(kTile * kTile) void raster_tile_kernel(RasterParams p, const uint32_t* vals,
                                                                     const uint2* range, const uint32_t* order) {
  constexpr bool kAct = FIELD == kFieldCornerActivated;
  const SceneView& s = p.scene;
  const int tile = (int)order[blockIdx.x];
  const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
  const int lane = threadIdx.x;
  const int col = tx * kTile + (lane % kTile), row = ty * kTile + (lane / kTile);
  const bool in_image = col < p.width && row < p.height;
  float o[3], d[3], tt;
  bool valid = sensor_ray(p.sensor, in_image ? col : 0, in_image ? row : 0, o, d, tt);
  RayFrame f = make_frame(s, o, d, p.sensor.t_near, p.sensor.t_far);
  if (!valid) f.valid = false;
  const float sh[4] = {kShC0, kShC1 * d[0], kShC1 * d[1], kShC1 * d[2]};
  Accum acc;
  acc.T = 1.0f;
  acc.C[0] = acc.C[1] = acc.C[2] = 0.0f;
  acc.D = acc.I = 0.0f;
  acc.n = 0;
  const int S = p.S;
  const double rS = 1.0 / S;
  bool alive = in_image && f.valid;

  __shared__ int32_t ids[kChunk];
  __shared__ int4 boxes[kChunk];
  __shared__ uint2 rects[kChunk];
  __shared__ float4 rows[kChunk * 8];                   // geo [8] then rgb [3][8] per voxel
  __shared__ float4 irows[INT ? kChunk * 2 : 1];       // intensity [8] per voxel
  const float* geo = kAct ? s.act_geo : s.geo;
  const float* rgb = kAct ? s.act_rgb : s.rgb;
  const float* itn = kAct ? s.act_int : s.inten;
  const uint2 rg = range[tile];
  for (uint32_t c = rg.x; c < rg.y; c += kChunk) {
    const int m = (int)(rg.y - c < (uint32_t)kChunk ? rg.y - c : (uint32_t)kChunk);
    if (lane < m) {
      const int32_t v = (int32_t)vals[c + lane];
      ids[lane] = v;
      boxes[lane] = p.vbox[v];
      rects[lane] = p.rect[v];
    }
    __syncthreads();
    // 8 lanes per voxel copy its 128-byte row (2 float4 of density, 6 of colour)
    for (int q = lane; q < m * 8; q += kTile * kTile) {
      const int j = q >> 3, part = q & 7;
      const int64_t v = ids[j];
      float4 val = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (part < 2) val = reinterpret_cast<const float4*>(geo + v * 8)[part];
      else if (RGB) val = reinterpret_cast<const float4*>(rgb + v * 24)[part - 2];
      rows[q] = val;
    }
    if (INT) {
      for (int q = lane; q < m * 2; q += kTile * kTile)
        irows[q] = reinterpret_cast<const float4*>(itn + (int64_t)ids[q >> 1] * 8)[q & 1];
    }
    __syncthreads();
    // (1) the staged voxels whose pixel rectangle holds this pixel, as a bit mask: the same cheap
    // test on every lane, so the wave stays converged; most listed voxels cover few of a tile's
    // pixels.  (2) each lane then walks only its own candidates, in list order, with the interval
    // rule and the shading: a wave pays for its busiest lane, not for the union of its lanes.
    uint32_t cand[kChunk / 32];
#pragma unroll
    for (int w = 0; w < kChunk / 32; ++w) {
      uint32_t bits = 0u;
      for (int b = 0; b < 32; ++b) {
        const int j = w * 32 + b;
        const uint2 rc = rects[j];
        const bool in = j < m && col >= (int)(rc.x & 0xffffu) && col <= (int)(rc.x >> 16) &&
                        row >= (int)(rc.y & 0xffffu) && row <= (int)(rc.y >> 16);
        bits |= in ? (1u << b) : 0u;
      }
      cand[w] = alive ? bits : 0u;
    }
#pragma unroll
    for (int w = 0; w < kChunk / 32; ++w) {
      uint32_t bits = cand[w];
      while (bits != 0u && alive) {
        const int j = w * 32 + (__ffs((int)bits) - 1);
        bits &= bits - 1u;
        const int4 b = boxes[j];
        Hit h;
        h.lo[0] = b.x;
        h.lo[1] = b.y;
        h.lo[2] = b.z;
        h.size = b.w;
        const int32_t hi[3] = {b.x + b.w, b.y + b.w, b.z + b.w};
        if (!box_interval(f, h.lo, hi, h.t_in, h.t_out) || !(h.t_in < h.t_out)) continue;
        h.voxel = ids[j];
        const float* row_p = reinterpret_cast<const float*>(rows + j * 8);
        const float* irow_p = INT ? reinterpret_cast<const float*>(irows + j * 2) : nullptr;
        if (!shade_rows<FIELD, RGB, INT>(s, f, sh, h, S, rS, p.t_min, acc, row_p, row_p + 8, irow_p)) alive = false;
      }
    }
    if (__syncthreads_count(alive ? 1 : 0) == 0) break;  // (also the barrier before the next round's loads)
  }
  if (!in_image) return;
  const int64_t ray = (int64_t)row * p.width + col;
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

template <int FIELD>
hipError_t launch_tiles(const RasterParams& p, const uint32_t* vals, const uint2* range, const uint32_t* order,
                        hipStream_t stream) {
  const unsigned blocks = (unsigned)(p.tiles_x * p.tiles_y);
  const bool rgb = p.out.rgb != nullptr, in = p.out.intensity != nullptr;
  if (rgb && in) raster_tile_kernel<FIELD, true, true><<<blocks, kTile * kTile, 0, stream>>>(p, vals, range, order);
  else if (rgb) raster_tile_kernel<FIELD, true, false><<<blocks, kTile * kTile, 0, stream>>>(p, vals, range, order);
  else if (in) raster_tile_kernel<FIELD, false, true><<<blocks, kTile * kTile, 0, stream>>>(p, vals, range, order);
  else raster_tile_kernel<FIELD, false, false><<<blocks, kTile * kTile, 0, stream>>>(p, vals, range, order);
  return hipGetLastError();
}

inline size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int bit_width(uint64_t x) { return x == 0 ? 0 : 64 - __builtin_clzll(x); }

// Work-area layout for n voxels, `tiles` tiles and up to `pairs` (voxel, tile) pairs.
struct RasterLayout {
  size_t count, offset, rect, vkey, keys_a, keys_b, vals_a, vals_b, range, tile_sort, temp, temp_bytes, total;
};

hipError_t raster_layout(int64_t n, int64_t tiles, int64_t pairs, RasterLayout* L) {
  size_t scan_bytes = 0, sort_bytes = 0, tile_bytes = 0;
  hipError_t e = rocprim::exclusive_scan(nullptr, scan_bytes, (const uint32_t*)nullptr, (uint64_t*)nullptr,
                                         (uint64_t)0, (size_t)(n + 1), rocprim::plus<uint64_t>());
  if (e != hipSuccess) return e;
  e = rocprim::radix_sort_pairs(nullptr, sort_bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                (const uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)(pairs > 0 ? pairs : 1));
  if (e != hipSuccess) return e;
  e = rocprim::radix_sort_pairs(nullptr, tile_bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                (const uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)(tiles > 0 ? tiles : 1));
  if (e != hipSuccess) return e;
  if (tile_bytes > sort_bytes) sort_bytes = tile_bytes;
  size_t off = 0;
  L->count = off;
  off = up256(off + (size_t)(n + 1) * 4);
  L->offset = off;
  off = up256(off + (size_t)(n + 1) * 8);
  L->rect = off;
  off = up256(off + (size_t)n * 8);
  L->vkey = off;
  off = up256(off + (size_t)n * 8);
  L->keys_a = off;
  off = up256(off + (size_t)pairs * 8);
  L->keys_b = off;
  off = up256(off + (size_t)pairs * 8);
  L->vals_a = off;
  off = up256(off + (size_t)pairs * 4);
  L->vals_b = off;
  off = up256(off + (size_t)pairs * 4);
  L->range = off;
  off = up256(off + (size_t)tiles * 8);
  L->tile_sort = off;  // tile keys, tile ids, sorted keys, order: 4 arrays of uint32
  off = up256(off + (size_t)tiles * 16);
  L->temp = off;
  L->temp_bytes = scan_bytes > sort_bytes ? scan_bytes : sort_bytes;
  off = up256(off + L->temp_bytes);
  L->total = off;
  return hipSuccess;
}

inline unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t raster_work_bytes(int64_t n_voxels, int64_t n_tiles, int64_t max_pairs, size_t* bytes) {
  RasterLayout L;
  const hipError_t e = raster_layout(n_voxels, n_tiles, max_pairs, &L);
  if (e == hipSuccess) *bytes = L.total;
  return e;
}

int64_t raster_capacity(int64_t n_voxels, int64_t n_tiles, size_t work_bytes) {
  // the largest pair count whose layout fits (the layout grows with the pairs)
  int64_t lo = 0, hi = (int64_t)(work_bytes / 24) + 1;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    size_t need = 0;
    if (raster_work_bytes(n_voxels, n_tiles, mid, &need) == hipSuccess && need <= work_bytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

void raster_prepare(RasterParams* p) {
  // the eye in the FP32 grid frame, as the interval rule forms a ray origin (each op rounded)
  const SceneView& s = p->scene;
  const int K = s.K;
  for (int a = 0; a < 3; ++a) {
    const float og = (p->sensor.p0[a] - s.org32[a]) * s.gs32;
    p->og[a] = og;
    p->eye[a] = (double)p->sensor.p0[a];
    const float fl = floorf(og);
    int c = fl < -1e9f ? -(1 << 30) : (fl > 1e9f ? (1 << 30) : (int)fl);
    c = c >> K;  // arithmetic shift: the floor of the root-cell index, negatives included
    p->eye_root[a] = c < -1 ? -1 : (c > s.dims[a] ? s.dims[a] : c);
  }
  for (int i = 0; i < 9; ++i) p->R[i] = (double)p->sensor.R0[i];
  p->fx = p->sensor.fx;
  p->fy = p->sensor.fy;
  p->cx = p->sensor.cx;
  p->cy = p->sensor.cy;
  p->width = p->sensor.width;
  p->height = p->sensor.height;
  p->tiles_x = (p->width + kTile - 1) / kTile;
  p->tiles_y = (p->height + kTile - 1) / kTile;
  uint64_t max_l1 = 0;
  for (int a = 0; a < 3; ++a) {
    const int e = p->eye_root[a];
    max_l1 += (uint64_t)(e > s.dims[a] - 1 - e ? e + 1 : s.dims[a] - e);
  }
  p->key_bits = 3 * K + bit_width(max_l1);
  p->tile_bits = bit_width((uint64_t)p->tiles_x * p->tiles_y);  // room for the one-past-the-last tile
}

hipError_t launch_raster(RasterParams p, int field, void* work, size_t work_bytes, int64_t* n_pairs,
                         int64_t* capacity, hipStream_t stream) {
  const int64_t n = p.n_voxels;
  const int64_t tiles = (int64_t)p.tiles_x * p.tiles_y;
  int64_t cap = raster_capacity(n, tiles, work_bytes);
  if (cap > (int64_t)UINT32_MAX) cap = (int64_t)UINT32_MAX;  // list positions are 32-bit
  *capacity = cap;
  RasterLayout L;
  hipError_t e = raster_layout(n, tiles, cap, &L);
  if (e != hipSuccess) return e;
  char* w = (char*)work;
  p.count = (uint32_t*)(w + L.count);
  p.offset = (uint64_t*)(w + L.offset);
  p.rect = (uint2*)(w + L.rect);
  p.vkey = (uint64_t*)(w + L.vkey);
  p.keys = (uint64_t*)(w + L.keys_a);
  p.vals = (uint32_t*)(w + L.vals_a);
  uint64_t* keys_b = (uint64_t*)(w + L.keys_b);
  uint32_t* vals_b = (uint32_t*)(w + L.vals_b);
  uint2* range = (uint2*)(w + L.range);
  const int T = 256;
  raster_count_kernel<<<blocks_of(n + 1, T), T, 0, stream>>>(p);
  size_t tb = L.temp_bytes;
  e = rocprim::exclusive_scan(w + L.temp, tb, p.count, p.offset, (uint64_t)0, (size_t)(n + 1),
                              rocprim::plus<uint64_t>(), stream);
  if (e != hipSuccess) return e;
  uint64_t total = 0;
  if ((e = hipMemcpyAsync(&total, p.offset + n, sizeof(total), hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
  *n_pairs = (int64_t)total;
  if ((int64_t)total > cap) return hipSuccess;  // the caller reports the shortfall
  raster_clear_kernel<<<blocks_of(tiles, T), T, 0, stream>>>(range, tiles);
  if (total > 0) {
    raster_emit_kernel<<<blocks_of((int64_t)total, T), T, 0, stream>>>(p, (int64_t)total);
    tb = L.temp_bytes;
    e = rocprim::radix_sort_pairs(w + L.temp, tb, p.keys, keys_b, p.vals, vals_b, (size_t)total, 0u,
                                  (unsigned)(p.key_bits + p.tile_bits), stream);
    if (e != hipSuccess) return e;
    raster_range_kernel<<<blocks_of((int64_t)total, T), T, 0, stream>>>(keys_b, (int64_t)total, p.key_bits, tiles,
                                                                         range);
  }
  // the tile order: longest lists first
  uint32_t* tkey = (uint32_t*)(w + L.tile_sort);
  uint32_t* tid = tkey + tiles;
  uint32_t* tkey_sorted = tid + tiles;
  uint32_t* order = tkey_sorted + tiles;
  raster_length_kernel<<<blocks_of(tiles, T), T, 0, stream>>>(range, tiles, tkey, tid);
  tb = L.temp_bytes;
  e = rocprim::radix_sort_pairs(w + L.temp, tb, tkey, tkey_sorted, tid, order, (size_t)tiles, 0u, 32u, stream);
  if (e != hipSuccess) return e;
  if (field == SALF_FIELD_PAPER) return launch_tiles<SALF_FIELD_PAPER>(p, vals_b, range, order, stream);
  if (field == SALF_FIELD_SDF) return launch_tiles<kFieldSdf>(p, vals_b, range, order, stream);
  if (p.scene.act_geo != nullptr) return launch_tiles<kFieldCornerActivated>(p, vals_b, range, order, stream);
  return launch_tiles<SALF_FIELD_CORNER>(p, vals_b, range, order, stream);
}

}  // namespace salf
