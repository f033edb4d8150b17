// Acceleration-structure build on the GPU: a dense root grid whose occupied cells hold either a
// level-0 voxel or an 8-ary octree, whose non-leaf nodes point to their 8 sub-volumes and whose
// leaves hold "empty" or a voxel (Sec. 3.2, octree ray casting).
//
// Build, one thread per voxel or hash slot:
//   1. fill: root grid and node children <- empty, hash keys <- unused
//   2. insert: validate each voxel (level and coordinates in range) and insert the keys of its
//      ancestors (depth m = 0 .. l-1, coordinates >> (l - m)) into an open-addressing hash set,
//      keeping per node the smallest index of a voxel below it (its first voxel)
//   3. number: nodes are numbered in the order (first voxel, depth).  The nodes whose first voxel
//      is v are ancestors of v at consecutive depths d0(v) .. l_v - 1, so a node's index is
//      offset(v) + depth - d0(v), with offset an exclusive scan of the counts l_v - d0(v).  For
//      voxels uploaded in Morton order of their corners this is the depth-first pre-order of every
//      octree (siblings' subtrees are contiguous), and for any order it is deterministic.
//   4. link: write each ancestor's index into its parent's child slot (or the root grid) and the
//      voxel's leaf code into its own slot, all by compare-and-swap from "empty".  Two voxels that
//      overlap or repeat make two different values compete for one slot; the loser is reported.
#include "internal.hpp"

namespace salf {
namespace {

constexpr uint64_t kNoKey = ~0ull;

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

__device__ __forceinline__ uint64_t node_key(int depth, int32_t x, int32_t y, int32_t z) {
  return ((uint64_t)depth << 60) | ((uint64_t)x << 40) | ((uint64_t)y << 20) | (uint64_t)z;
}

__global__ void fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_u64(uint64_t* p, uint64_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void init_counters(BuildCounters* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->error_bits = 0;
    c->first_bad = 0x7fffffff;
    c->n_nodes = 0;
    c->n_occupied = 0;
  }
}

struct BuildArgs {
  const int32_t* vox;
  int64_t n;
  int32_t dims[3];
  int32_t K;
  int32_t* root;
  int32_t* nodes;
  uint64_t* hkeys;
  int32_t* hvals;
  int64_t hcap;
  int64_t node_cap;
  BuildCounters* cnt;
  int32_t* lmax;     // [n_root] finest voxel level in each root cell (0 if empty)
  int32_t* box_tmp;  // [node_cap][6] absolute finest bounds of each node's voxels (min lo, max hi)
  uint2* nbox;       // [node_cap] packed bounds relative to the node
  int32_t* d0;       // [n] shallowest depth of a node whose first voxel is v (numbering only)
  int32_t* offs;     // [n] first node index of those nodes (numbering only)
};

__device__ __forceinline__ void report(BuildCounters* c, int bit, int32_t v) {
  atomicOr(&c->error_bits, bit);
  atomicMin(&c->first_bad, v);
}

__device__ __forceinline__ bool voxel_ok(const BuildArgs& a, int32_t l, int32_t i, int32_t j, int32_t k) {
  if (l < 0 || l > a.K) return false;
  return i >= 0 && j >= 0 && k >= 0 && i < (a.dims[0] << l) && j < (a.dims[1] << l) && k < (a.dims[2] << l);
}

// Slot of `key` (inserted if new), or -1 if the table is full.
__device__ int64_t hash_insert(const BuildArgs& a, uint64_t key) {
  uint64_t h = mix64(key) & (uint64_t)(a.hcap - 1);
  for (int64_t probe = 0; probe < a.hcap; ++probe) {
    const uint64_t prev = atomicCAS((unsigned long long*)&a.hkeys[h], (unsigned long long)kNoKey,
                                    (unsigned long long)key);
    if (prev == kNoKey || prev == key) return (int64_t)h;
    h = (h + 1) & (uint64_t)(a.hcap - 1);
  }
  return -1;
}

__device__ int32_t hash_find(const BuildArgs& a, uint64_t key) {
  uint64_t h = mix64(key) & (uint64_t)(a.hcap - 1);
  for (int64_t probe = 0; probe < a.hcap; ++probe) {
    const uint64_t k = a.hkeys[h];
    if (k == key) return a.hvals[h];
    if (k == kNoKey) return -1;
    h = (h + 1) & (uint64_t)(a.hcap - 1);
  }
  return -1;
}

__global__ void insert_kernel(BuildArgs a) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= a.n) return;
  const int4 q = reinterpret_cast<const int4*>(a.vox)[v];
  const int32_t l = q.x;
  if (!voxel_ok(a, l, q.y, q.z, q.w)) {
    report(a.cnt, 1, (int32_t)v);
    return;
  }
  for (int m = 0; m < l; ++m) {
    const int sh = l - m;
    const int64_t slot = hash_insert(a, node_key(m, q.y >> sh, q.z >> sh, q.w >> sh));
    if (slot < 0) {
      report(a.cnt, 4, (int32_t)v);
      return;
    }
    atomicMin(&a.hvals[slot], (int32_t)v);
  }
}

// Each voxel's finest-cell box: min corner and edge (2^(K - l) cells).
__global__ void vbox_kernel(const int32_t* vox, int64_t n, int K, int4* vbox) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int4 q = reinterpret_cast<const int4*>(vox)[v];
  const int sh = K - q.x;
  vbox[v] = make_int4(q.y << sh, q.z << sh, q.w << sh, 1 << sh);
}

// d0(v) <- l_v (no node yet), 0 for an invalid voxel
__global__ void d0_init(BuildArgs a) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= a.n) return;
  const int4 q = reinterpret_cast<const int4*>(a.vox)[v];
  a.d0[v] = voxel_ok(a, q.x, q.y, q.z, q.w) ? q.x : 0;
}

// d0(first voxel) <- min(depth) over the nodes
__global__ void d0_min(BuildArgs a) {
  const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h >= a.hcap) return;
  const uint64_t key = a.hkeys[h];
  if (key == kNoKey) return;
  const int32_t v = a.hvals[h];
  if (v < 0 || v >= a.n) return;
  atomicMin(&a.d0[v], (int32_t)(key >> 60));
}

// offs(v) <- number of nodes whose first voxel is v
__global__ void node_counts(BuildArgs a) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= a.n) return;
  const int4 q = reinterpret_cast<const int4*>(a.vox)[v];
  a.offs[v] = voxel_ok(a, q.x, q.y, q.z, q.w) ? q.x - a.d0[v] : 0;
}

__global__ void number_kernel(BuildArgs a) {
  const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h >= a.hcap) return;
  const uint64_t key = a.hkeys[h];
  if (key == kNoKey) return;
  const int32_t v = a.hvals[h];
  int32_t id = -1;
  if (v >= 0 && v < a.n) {
    const int64_t i = (int64_t)a.offs[v] + (int32_t)(key >> 60) - a.d0[v];
    if (i >= 0 && i < a.node_cap) id = (int32_t)i;
  }
  a.hvals[h] = id;
  if (id < 0) report(a.cnt, 4, 0);
  atomicAdd(&a.cnt->n_nodes, 1);
}

// In-place exclusive prefix sum of int32 values, 2048 per block; sums[b] <- the block's total.
constexpr int kScanThreads = 256, kScanItems = 8, kScanBlock = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void scan_blocks(int32_t* x, int64_t n, int32_t* sums) {
  __shared__ int32_t part[kScanThreads];
  const int64_t base = blockIdx.x * (int64_t)kScanBlock + threadIdx.x * kScanItems;
  int32_t v[kScanItems], tot = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? x[base + i] : 0;
    tot += v[i];
  }
  part[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {  // inclusive Hillis-Steele scan of the partials
    const int32_t add = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int32_t run = part[threadIdx.x] - tot;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) x[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = part[threadIdx.x];
}

__global__ void scan_add(int32_t* x, int64_t n, const int32_t* sums) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] += sums[i / kScanBlock];
}

__device__ __forceinline__ bool claim(int32_t* slot, int32_t value) {
  const int32_t old = atomicCAS(slot, kEmpty, value);
  return old == kEmpty || old == value;
}

__global__ void link_kernel(BuildArgs a) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= a.n) return;
  const int4 q = reinterpret_cast<const int4*>(a.vox)[v];
  const int32_t l = q.x;
  if (!voxel_ok(a, l, q.y, q.z, q.w)) return;
  int32_t parent = -1;  // node index of the depth m-1 ancestor
  for (int m = 0; m <= l; ++m) {
    const int sh = l - m;
    const int32_t x = q.y >> sh, y = q.z >> sh, z = q.w >> sh;
    int32_t value;
    if (m == l) {
      value = leaf_code((int32_t)v);
    } else {
      value = hash_find(a, node_key(m, x, y, z));
      if (value < 0) {
        report(a.cnt, 4, (int32_t)v);
        return;
      }
    }
    int32_t* slot;
    if (m == 0) {
      const int64_t cell = ((int64_t)z * a.dims[1] + y) * a.dims[0] + x;
      slot = &a.root[cell];
      atomicMax(&a.lmax[cell], l);
    } else {
      slot = &a.nodes[(int64_t)parent * 8 + ((x & 1) | ((y & 1) << 1) | ((z & 1) << 2))];
    }
    if (!claim(slot, value)) {
      report(a.cnt, 2, (int32_t)v);
      return;
    }
    if (m < l) {  // grow the ancestor's bounds of occupied content by this voxel
      const int sh_f = a.K - l;
      const int32_t vlo[3] = {q.y << sh_f, q.z << sh_f, q.w << sh_f};
      int32_t* b = a.box_tmp + (int64_t)value * 6;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        atomicMin(&b[ax], vlo[ax]);
        atomicMax(&b[3 + ax], vlo[ax] + (1 << sh_f));
      }
    }
    parent = value;
  }
}

// Chebyshev distance from every root cell to the nearest occupied one (0 = occupied), capped at
// kSkipCap, by three separable passes: along x, then y, then z, each taking
// d(c) = min over |j| <= cap of max(|j|, d_prev(c + j e_axis)).
constexpr int kSkipCap = 24;

__global__ void skip_pass(const int32_t* root, const uint8_t* in, uint8_t* out, int axis, int32_t dx, int32_t dy,
                          int32_t dz) {
  const int64_t n = (int64_t)dx * dy * dz;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t x = (int32_t)(i % dx), y = (int32_t)((i / dx) % dy), z = (int32_t)(i / ((int64_t)dx * dy));
  const int32_t c = axis == 0 ? x : (axis == 1 ? y : z);
  const int32_t D = axis == 0 ? dx : (axis == 1 ? dy : dz);
  const int64_t stride = axis == 0 ? 1 : (axis == 1 ? dx : (int64_t)dx * dy);
  int best = kSkipCap + 1;
  for (int j = -kSkipCap; j <= kSkipCap; ++j) {
    const int32_t q = c + j;
    if (q < 0 || q >= D) continue;
    const int64_t qi = i + (int64_t)j * stride;
    const int prev = (axis == 0) ? (root[qi] != kEmpty ? 0 : kSkipCap + 1) : (int)in[qi];
    const int aj = j < 0 ? -j : j;
    const int v = prev > aj ? prev : aj;
    best = v < best ? v : best;
  }
  out[i] = (uint8_t)best;
}

__global__ void box_init(int32_t* b, int64_t n_nodes) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_nodes; i += (int64_t)gridDim.x * blockDim.x) {
    b[i * 6 + 0] = b[i * 6 + 1] = b[i * 6 + 2] = 0x7fffffff;
    b[i * 6 + 3] = b[i * 6 + 4] = b[i * 6 + 5] = -0x7fffffff;
  }
}

// Pack every node's bounds relative to the node's min corner: bytes (lo_x, lo_y, lo_z) and
// (hi_x - 1, hi_y - 1, hi_z - 1), each in [0, 255] since a node spans at most 2^K <= 256 cells.
// The node's own box comes from its hash key (depth, coordinates at that depth).
__global__ void box_pack(BuildArgs a) {
  const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h >= a.hcap) return;
  const uint64_t key = a.hkeys[h];
  if (key == kNoKey) return;
  const int32_t id = a.hvals[h];
  if (id < 0) return;
  const int depth = (int)(key >> 60);
  const int sh = a.K - depth;
  const int32_t nlo[3] = {(int32_t)((key >> 40) & 0xFFFFF) << sh, (int32_t)((key >> 20) & 0xFFFFF) << sh,
                          (int32_t)(key & 0xFFFFF) << sh};
  const int32_t* b = a.box_tmp + (int64_t)id * 6;
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    lo |= (uint32_t)(b[ax] - nlo[ax]) << (8 * ax);
    hi |= (uint32_t)(b[3 + ax] - 1 - nlo[ax]) << (8 * ax);
  }
  a.nbox[id] = make_uint2(lo, hi);
}

// Bounds of each root cell's voxels (its root node's), indexed by cell, so that a walk can read
// them together with the cell's code.
__global__ void root_box_kernel(const int32_t* root, const uint2* nbox, uint2* rbox, int64_t n_root) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_root; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = root[i];
    rbox[i] = c >= 0 ? nbox[c] : make_uint2(0u, 0u);
  }
}

__global__ void count_roots(const int32_t* root, int64_t n, BuildCounters* c) {
  int32_t mine = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    mine += root[i] != kEmpty;
  if (mine) atomicAdd(&c->n_occupied, mine);
}

// one thread per item (n <= 2^31 here, so the grid fits in gridDim.x)
inline unsigned blocks_for(int64_t n, int threads) {
  const int64_t b = (n + threads - 1) / threads;
  return (unsigned)(b < 1 ? 1 : b);
}

// int32 entries of block sums an exclusive scan of n values needs (all levels)
int64_t scan_temp(int64_t n) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  return nb + (nb > 1 ? scan_temp(nb) : 0);
}

void launch_scan(int32_t* x, int64_t n, int32_t* tmp, hipStream_t stream) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  scan_blocks<<<(unsigned)nb, kScanThreads, 0, stream>>>(x, n, tmp);
  if (nb > 1) {
    launch_scan(tmp, nb, tmp + nb, stream);
    scan_add<<<blocks_for(n, 256), 256, 0, stream>>>(x, n, tmp);
  }
}

}  // namespace

bool scene_layout(const salf_scene_desc& d, int64_t n, SceneLayout* L) {
  const int K = d.max_level;
  int64_t n_root = (int64_t)d.root_dims[0] * d.root_dims[1] * d.root_dims[2];
  // every voxel adds at most K ancestors; no depth can hold more nodes than it has cells
  int64_t geo_cap = 0, cells = n_root;
  for (int m = 0; m < K; ++m) {
    geo_cap += cells;
    if (geo_cap > ((int64_t)1 << 40)) break;
    cells *= 8;
  }
  int64_t node_cap = n * (int64_t)K;
  if (geo_cap < node_cap) node_cap = geo_cap;
  int64_t hcap = 1024;
  while (hcap < 2 * node_cap) hcap <<= 1;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off = 0;
  L->n_root = n_root;
  L->node_cap = node_cap;
  L->hash_cap = hcap;
  L->root_off = off;
  off = up(off + (size_t)n_root * 4);
  L->skip_off = off;
  off = up(off + (size_t)n_root);
  L->lmax_off = off;
  off = up(off + (size_t)n_root * 4);
  L->rbox_off = off;
  off = up(off + (size_t)n_root * 8);
  L->nodes_off = off;
  off = up(off + (size_t)node_cap * 32);
  L->nbox_off = off;
  off = up(off + (size_t)node_cap * 8);
  L->box_tmp_off = off;
  off = up(off + (size_t)node_cap * 24);
  L->hkeys_off = off;
  off = up(off + (size_t)hcap * 8);
  L->hvals_off = off;
  off = up(off + (size_t)hcap * 4);
  L->tmp_off = off;
  off = up(off + (size_t)n_root * 2);
  L->order_off = 0;
  if (K > 0 && n > 0) {  // node numbering: d0 [n], offsets [n], scan block sums
    L->order_off = off;
    off = up(off + (size_t)(2 * n + scan_temp(n)) * 4);
  }
  L->counters_off = off;
  off = up(off + sizeof(BuildCounters));
  L->vbox_off = off;
  off = up(off + (size_t)n * 16);
  L->act_geo_off = L->act_rgb_off = L->act_int_off = 0;
  if (d.flags & SALF_SCENE_PREACTIVATE) {
    L->act_geo_off = off;
    off = up(off + (size_t)n * 8 * 4);
    L->act_rgb_off = off;
    off = up(off + (size_t)n * 24 * 4);
    L->act_int_off = off;
    off = up(off + (size_t)n * 8 * 4);
  }
  L->cell_off = off;
  off = up(off + (size_t)n_root * 16);
  L->total = off;
  return true;
}

namespace {
// Dense leaf index of every root cell with boff[cell] >= 0 (one workgroup per cell): each entry
// descends the cell's octree to the region that holds its level-L cell (the first child on the
// way that is a voxel or empty) and records that region's level and voxel.
__global__ void index_fill_kernel(const int32_t* root, const int32_t* nodes, const int32_t* lmax,
                                  const int32_t* boff, int64_t cell0, uint32_t* entries) {
  const int64_t cell = cell0 + blockIdx.x;
  const int32_t off = boff[cell];
  if (off < 0) return;
  const int L = lmax[cell];
  const int32_t code = root[cell];
  const int32_t n = 1 << (3 * L);
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const int32_t x = i & ((1 << L) - 1), y = (i >> L) & ((1 << L) - 1), z = i >> (2 * L);
    int32_t node = code;
    uint32_t e = (uint32_t)L;  // a malformed tree (an internal node at level L) reads as empty
    for (int d = 0; d < L; ++d) {
      const int b = L - 1 - d;
      const int c8 = ((x >> b) & 1) | (((y >> b) & 1) << 1) | (((z >> b) & 1) << 2);
      const int32_t ch = nodes[(int64_t)node * 8 + c8];
      if (is_leaf_code(ch)) {
        e = ((uint32_t)(leaf_voxel(ch) + 1) << kIdxLevelBits) | (uint32_t)(d + 1);
        break;
      }
      if (ch < 0) {
        e = (uint32_t)(d + 1);
        break;
      }
      node = ch;
    }
    entries[(int64_t)off + i] = e;
  }
}

// Corner activations for pre-activated scenes (the same functions the render kernels apply).
__global__ void activate_kernel(const float* src, float* dst, int64_t n, int softplus) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = softplus ? softplus_f(src[i]) : sigmoid_f(src[i]);
}
}  // namespace

hipError_t launch_activate(const float* geo, const float* rgb, const float* inten, int64_t n, float* act_geo,
                           float* act_rgb, float* act_int, hipStream_t stream) {
  const int T = 256;
  auto grid = [](int64_t m) { return (unsigned)((m + 255) / 256 > 8192 ? 8192 : (m + 255) / 256); };
  if (n <= 0) return hipSuccess;
  activate_kernel<<<grid(n * 8), T, 0, stream>>>(geo, act_geo, n * 8, 1);
  if (rgb) activate_kernel<<<grid(n * 24), T, 0, stream>>>(rgb, act_rgb, n * 24, 0);
  if (inten) activate_kernel<<<grid(n * 8), T, 0, stream>>>(inten, act_int, n * 8, 0);
  return hipGetLastError();
}

namespace {
// ---- densification and pruning (Sec. 3.3)
struct RefineArgs {
  const int32_t* vox;       // [n, 4] (l, i, j, k)
  const float* geo;         // [n, 8]
  const float* rgb;         // [n, 3, 8] or null
  const float* inten;       // [n, 8] or null
  const float* grad_rgb;    // [n, 3, 8] or null (no splits)
  int64_t n;
  int32_t K, field;
  double s0, grad_threshold, alpha_min;
};

__device__ __forceinline__ double softplus64(double z) { return fmax(z, 0.0) + log1p(exp(-fabs(z))); }
__device__ __forceinline__ double sigmoid64(double z) { return 1.0 / (1.0 + exp(-z)); }

// Largest density of a voxel: the largest corner density (trilinear of non-negative corner
// values; exp of an affine form; Eq. 6, monotone in an affine signed distance).
__device__ double sigma_max64(const float* g, int field) {
  double m = 0.0;
  for (int c = 0; c < 8; ++c) {
    double sig;
    if (field == SALF_FIELD_CORNER) {
      sig = softplus64(g[c]);
    } else {
      const double q = (c & 1 ? 1.0 : -1.0) * g[0] + (c & 2 ? 1.0 : -1.0) * g[1] + (c & 4 ? 1.0 : -1.0) * g[2] + g[3];
      if (field == SALF_FIELD_SDF) {
        const double a = exp((double)g[4]), b = exp((double)g[5]);
        const double e = 1.0 - exp(-fabs(q) / b);
        sig = a / 2.0 + a / 2.0 * (q > 0.0 ? e : (q < 0.0 ? -e : 0.0));
      } else {
        sig = exp(q);
      }
    }
    m = fmax(m, sig);
  }
  return m;
}

// Output rows of voxel v: 0 (pruned), 1 (kept) or 8 (split), in float64 as the decision's
// definition states them.
__global__ void refine_count_kernel(RefineArgs a, int32_t* count) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= a.n) return;
  // the caller's voxels are those the scene was built from (levels in [0, K]); clamp anyway so
  // that a wrong array cannot shift out of range
  const int lvl = min(max(a.vox[v * 4], 0), a.K);
  const double edge = a.s0 / (double)(1 << lvl);
  const double alpha = -expm1(-sigma_max64(a.geo + v * 8, a.field) * edge);
  int32_t c = 1;
  if (alpha < a.alpha_min) {
    c = 0;
  } else if (lvl < a.K && a.grad_rgb != nullptr) {
    double l1 = 0.0;
    for (int ch = 0; ch < 3; ++ch)
      for (int i = 0; i < (a.field == SALF_FIELD_CORNER ? 8 : 3); ++i) l1 += fabs((double)a.grad_rgb[v * 24 + ch * 8 + i]);
    if (l1 > a.grad_threshold) c = 8;
  }
  count[v] = c;
}

__device__ __forceinline__ float logit64(double q, double q1) { return (float)(log(q) - log(q1)); }

// Writes each voxel's output rows at its offset (offs: exclusive scan of the counts, total: their
// sum).  Children carry the parent's field exactly: corner logits are the inverse activations of
// the parent's activated field at the child corners; affine forms halve their slopes and move
// their offsets (the colour's into the SH DC coefficient, times 1 / C0).
__global__ void refine_emit_kernel(RefineArgs a, const int32_t* offs, int64_t total, int32_t* vox_out,
                                   float* geo_out, float* rgb_out, float* int_out) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= a.n) return;
  const int64_t o = offs[v];
  const int64_t c = (v + 1 < a.n ? (int64_t)offs[v + 1] : total) - o;
  const int32_t* vx = a.vox + v * 4;
  const float* g = a.geo + v * 8;
  const float* r = a.rgb ? a.rgb + v * 24 : nullptr;
  const float* it = a.inten ? a.inten + v * 8 : nullptr;
  if (c == 1) {
    for (int t = 0; t < 4; ++t) vox_out[o * 4 + t] = vx[t];
    for (int t = 0; t < 8; ++t) geo_out[o * 8 + t] = g[t];
    if (r && rgb_out) for (int t = 0; t < 24; ++t) rgb_out[o * 24 + t] = r[t];
    if (it && int_out) for (int t = 0; t < 8; ++t) int_out[o * 8 + t] = it[t];
    return;
  }
  if (c != 8) return;
  for (int b = 0; b < 8; ++b) {
    const int64_t q = o + b;
    const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
    vox_out[q * 4 + 0] = vx[0] + 1;
    vox_out[q * 4 + 1] = 2 * vx[1] + bx;
    vox_out[q * 4 + 2] = 2 * vx[2] + by;
    vox_out[q * 4 + 3] = 2 * vx[3] + bz;
    const double ob[3] = {bx - 0.5, by - 0.5, bz - 0.5};
    if (a.field == SALF_FIELD_CORNER) {
      for (int k = 0; k < 8; ++k) {
        // child corner k in the parent's unit coordinates u = (x_p + 1) / 2 (0, 1/2 or 1)
        double w[8];
        const double u[3] = {((k & 1 ? 1.0 : -1.0) / 2.0 + ob[0] + 1.0) / 2.0,
                             ((k & 2 ? 1.0 : -1.0) / 2.0 + ob[1] + 1.0) / 2.0,
                             ((k & 4 ? 1.0 : -1.0) / 2.0 + ob[2] + 1.0) / 2.0};
        for (int p = 0; p < 8; ++p)
          w[p] = (p & 1 ? u[0] : 1.0 - u[0]) * (p & 2 ? u[1] : 1.0 - u[1]) * (p & 4 ? u[2] : 1.0 - u[2]);
        double y = 0.0;
        for (int p = 0; p < 8; ++p) y += w[p] * softplus64(g[p]);
        geo_out[q * 8 + k] = (float)log(expm1(y));
        if (r && rgb_out) {
          for (int ch = 0; ch < 3; ++ch) {
            double s1 = 0.0, s0 = 0.0;  // the interpolated value and its complement, each accurate
            for (int p = 0; p < 8; ++p) {
              s1 += w[p] * sigmoid64(r[ch * 8 + p]);
              s0 += w[p] * sigmoid64(-(double)r[ch * 8 + p]);
            }
            rgb_out[q * 24 + ch * 8 + k] = logit64(s1, s0);
          }
        }
        if (it && int_out) {
          double s1 = 0.0, s0 = 0.0;
          for (int p = 0; p < 8; ++p) {
            s1 += w[p] * sigmoid64(it[p]);
            s0 += w[p] * sigmoid64(-(double)it[p]);
          }
          int_out[q * 8 + k] = logit64(s1, s0);
        }
      }
    } else {
      constexpr double kC0 = 0.28209479177387814;
      for (int t = 0; t < 8; ++t) geo_out[q * 8 + t] = g[t];
      geo_out[q * 8 + 0] = (float)(g[0] / 2.0);
      geo_out[q * 8 + 1] = (float)(g[1] / 2.0);
      geo_out[q * 8 + 2] = (float)(g[2] / 2.0);
      geo_out[q * 8 + 3] = (float)(g[3] + g[0] * ob[0] + g[1] * ob[1] + g[2] * ob[2]);
      if (r && rgb_out) {
        for (int ch = 0; ch < 3; ++ch) {
          const float* rc = r + ch * 8;
          float* oc = rgb_out + q * 24 + ch * 8;
          for (int t = 0; t < 8; ++t) oc[t] = rc[t];
          oc[0] = (float)(rc[0] / 2.0);
          oc[1] = (float)(rc[1] / 2.0);
          oc[2] = (float)(rc[2] / 2.0);
          oc[3] = (float)(rc[3] + (rc[0] * ob[0] + rc[1] * ob[1] + rc[2] * ob[2]) / kC0);
        }
      }
      if (it && int_out) {
        for (int t = 0; t < 8; ++t) int_out[q * 8 + t] = it[t];
        int_out[q * 8 + 0] = (float)(it[0] / 2.0);
        int_out[q * 8 + 1] = (float)(it[1] / 2.0);
        int_out[q * 8 + 2] = (float)(it[2] / 2.0);
        int_out[q * 8 + 3] = (float)(it[3] + it[0] * ob[0] + it[1] * ob[1] + it[2] * ob[2]);
      }
    }
  }
}
}  // namespace

size_t refine_work_bytes(int64_t n) { return ((size_t)(n + scan_temp(n > 0 ? n : 1)) * 4 + 255) / 256 * 256; }

hipError_t launch_refine(const SceneView& v, const salf_scene_desc& d, int64_t n, const int32_t* vox,
                         const float* grad_rgb, double grad_threshold, double alpha_min, void* work,
                         int32_t* vox_out, float* geo_out, float* rgb_out, float* int_out, int64_t capacity,
                         int64_t* total, hipStream_t stream) {
  *total = 0;
  if (n <= 0) return hipSuccess;
  RefineArgs a;
  a.vox = vox;
  a.geo = v.geo;
  a.rgb = v.rgb;
  a.inten = v.inten;
  a.grad_rgb = grad_rgb;
  a.n = n;
  a.K = d.max_level;
  a.field = d.field;
  a.s0 = d.root_size;
  a.grad_threshold = grad_threshold;
  a.alpha_min = alpha_min;
  int32_t* count = (int32_t*)work;
  refine_count_kernel<<<blocks_for(n, 256), 256, 0, stream>>>(a, count);
  int32_t last[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(&last[0], count + n - 1, 4, hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return e;
  launch_scan(count, n, count + n, stream);
  if ((e = hipMemcpyAsync(&last[1], count + n - 1, 4, hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
  *total = (int64_t)last[0] + last[1];
  if (*total > capacity) return hipSuccess;
  refine_emit_kernel<<<blocks_for(n, 256), 256, 0, stream>>>(a, count, *total, vox_out, geo_out, rgb_out, int_out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamSynchronize(stream);
}

namespace {
__global__ void pack_cells_kernel(const int32_t* root, const uint2* rbox, const uint8_t* skip, const int32_t* lmax,
                                  const int32_t* boff, int64_t n_root, int4* cell) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_root) return;
  const uint2 b = rbox[i];
  const uint32_t sk = skip != nullptr ? (uint32_t)skip[i] : 0u;
  const uint32_t lm = (uint32_t)lmax[i] & 255u;
  cell[i] = make_int4(root[i], boff != nullptr ? boff[i] : -1, (int32_t)((b.x & 0xffffffu) | (sk << 24)),
                      (int32_t)((b.y & 0xffffffu) | (lm << 24)));
}
}  // namespace

hipError_t launch_pack_cells(const SceneView& v, int64_t n_root, hipStream_t stream) {
  if (n_root <= 0) return hipSuccess;
  pack_cells_kernel<<<blocks_for(n_root, 256), 256, 0, stream>>>(v.root, v.rbox, v.skip, v.lmax, v.boff, n_root,
                                                                  const_cast<int4*>(v.cell));
  return hipGetLastError();
}

hipError_t launch_index_fill(const SceneView& v, int64_t n_root, const int32_t* boff, uint32_t* entries,
                             hipStream_t stream) {
  for (int64_t c0 = 0; c0 < n_root; c0 += (int64_t)1 << 30) {
    const int64_t m = n_root - c0 < ((int64_t)1 << 30) ? n_root - c0 : ((int64_t)1 << 30);
    index_fill_kernel<<<(unsigned)m, 256, 0, stream>>>(v.root, v.nodes, v.lmax, boff, c0, entries);
  }
  return hipGetLastError();
}

hipError_t launch_scene_build(const salf_scene_desc& d, int64_t n, const int32_t* voxels, const SceneLayout& L,
                              void* ws, hipStream_t stream) {
  char* base = (char*)ws;
  BuildArgs a;
  a.vox = voxels;
  a.n = n;
  for (int i = 0; i < 3; ++i) a.dims[i] = d.root_dims[i];
  a.K = d.max_level;
  a.root = (int32_t*)(base + L.root_off);
  a.nodes = (int32_t*)(base + L.nodes_off);
  a.hkeys = (uint64_t*)(base + L.hkeys_off);
  a.hvals = (int32_t*)(base + L.hvals_off);
  a.hcap = L.hash_cap;
  a.node_cap = L.node_cap;
  a.cnt = (BuildCounters*)(base + L.counters_off);
  a.box_tmp = (int32_t*)(base + L.box_tmp_off);
  a.lmax = (int32_t*)(base + L.lmax_off);
  a.nbox = (uint2*)(base + L.nbox_off);
  a.d0 = L.order_off ? (int32_t*)(base + L.order_off) : nullptr;
  a.offs = L.order_off ? a.d0 + n : nullptr;
  const int T = 256;
  fill_i32<<<blocks_for(L.n_root, T), T, 0, stream>>>(a.root, kEmpty, L.n_root);
  fill_i32<<<blocks_for(L.n_root, T), T, 0, stream>>>(a.lmax, 0, L.n_root);
  if (L.node_cap > 0) box_init<<<blocks_for(L.node_cap, T) > 8192 ? 8192 : blocks_for(L.node_cap, T), T, 0, stream>>>(
      a.box_tmp, L.node_cap);
  if (L.node_cap > 0) fill_i32<<<blocks_for(L.node_cap * 8, T), T, 0, stream>>>(a.nodes, kEmpty, L.node_cap * 8);
  fill_u64<<<blocks_for(L.hash_cap, T), T, 0, stream>>>(a.hkeys, kNoKey, L.hash_cap);
  fill_i32<<<blocks_for(L.hash_cap, T), T, 0, stream>>>(a.hvals, 0x7fffffff, L.hash_cap);
  init_counters<<<1, 64, 0, stream>>>(a.cnt);
  if (n > 0) insert_kernel<<<blocks_for(n, T), T, 0, stream>>>(a);
  if (a.d0 != nullptr) {
    const unsigned hb = (unsigned)((L.hash_cap + T - 1) / T);
    d0_init<<<blocks_for(n, T), T, 0, stream>>>(a);
    d0_min<<<hb, T, 0, stream>>>(a);
    node_counts<<<blocks_for(n, T), T, 0, stream>>>(a);
    launch_scan(a.offs, n, a.offs + n, stream);
    number_kernel<<<hb, T, 0, stream>>>(a);
  }
  if (n > 0) link_kernel<<<blocks_for(n, T), T, 0, stream>>>(a);
  box_pack<<<(unsigned)((L.hash_cap + T - 1) / T), T, 0, stream>>>(a);
  root_box_kernel<<<blocks_for(L.n_root, T) > 8192 ? 8192 : blocks_for(L.n_root, T), T, 0, stream>>>(
      a.root, a.nbox, (uint2*)(base + L.rbox_off), L.n_root);
  {
    uint8_t* skip = (uint8_t*)(base + L.skip_off);
    uint8_t* t0 = (uint8_t*)(base + L.tmp_off);
    uint8_t* t1 = t0 + L.n_root;
    const unsigned nb = blocks_for(L.n_root, T);
    skip_pass<<<nb, T, 0, stream>>>(a.root, nullptr, t0, 0, a.dims[0], a.dims[1], a.dims[2]);
    skip_pass<<<nb, T, 0, stream>>>(a.root, t0, t1, 1, a.dims[0], a.dims[1], a.dims[2]);
    skip_pass<<<nb, T, 0, stream>>>(a.root, t1, skip, 2, a.dims[0], a.dims[1], a.dims[2]);
  }
  count_roots<<<blocks_for(L.n_root, T) > 1024 ? 1024 : blocks_for(L.n_root, T), T, 0, stream>>>(a.root, L.n_root,
                                                                                                  a.cnt);
  // (a voxel outside [0, K] fails the build before its box is read)
  if (n > 0) vbox_kernel<<<blocks_for(n, T), T, 0, stream>>>(voxels, n, a.K, (int4*)(base + L.vbox_off));
  pack_cells_kernel<<<blocks_for(L.n_root, T), T, 0, stream>>>(a.root, (const uint2*)(base + L.rbox_off),
                                                               (const uint8_t*)(base + L.skip_off), a.lmax, nullptr,
                                                               L.n_root, (int4*)(base + L.cell_off));
  return hipGetLastError();
}

}  // namespace salf
