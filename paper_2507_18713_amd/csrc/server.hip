// Serving with continuous batching (the salf_server_* entry points).
//
// A scheduler thread owns the GPU side of the server.  Each cycle it
//   1. retires launches whose completion event has fired (their requests become done),
//   2. admits queued requests in arrival order while their outputs fit in the HBM pool (first fit;
//      a request that does not fit blocks the ones behind it, so admission stays FIFO),
//   3. if a launch slot is free, launches one batched kernel over every tile of the requests
//      admitted since the previous launch (up to max_batch requests and, while the backlog is
//      short, max_launch_rays rays) on that slot's stream.
// With several slots, a batch starts while earlier ones are still running, so requests that arrive
// while the GPU is busy overlap with them instead of waiting for a drain.
#include <string.h>
#include <time.h>

#include <condition_variable>
#include <iterator>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "internal.hpp"

namespace salf {
namespace {

double now_s() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

constexpr size_t kAlign = 256;
constexpr int kMaxBatch = 256;
constexpr int kMaxInflight = 4;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Offsets of a request's outputs inside its pool block (SIZE_MAX = not requested).
struct OutLayout {
  size_t rgb, depth, opacity, intensity, total;
};

OutLayout out_layout(int64_t n, uint32_t mask) {
  OutLayout L;
  size_t off = 0;
  auto take = [&](bool on, size_t bytes) {
    if (!on) return (size_t)-1;
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.rgb = take(mask & SALF_OUT_RGB, (size_t)n * 12);
  L.depth = take(mask & SALF_OUT_DEPTH, (size_t)n * 4);
  L.opacity = take(mask & SALF_OUT_OPACITY, (size_t)n * 4);
  L.intensity = take(mask & SALF_OUT_INTENSITY, (size_t)n * 4);
  L.total = off > 0 ? off : kAlign;
  return L;
}

// First-fit allocator over [0, size) with coalescing of freed neighbours.
class Pool {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
    in_use = peak = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      in_use += bytes;
      if (in_use > peak) peak = in_use;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    in_use -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  size_t in_use = 0, peak = 0;

 private:
  std::map<size_t, size_t> free_;
};

enum State { kQueued = 0, kAdmitted = 1, kRunning = 2, kDone = 3 };

struct Request {
  uint64_t ticket = 0;
  RenderParams p;
  int32_t variant = 0;
  uint32_t outputs = 0;
  int64_t n_tiles = 0;
  OutLayout lay;
  size_t off = 0;
  double t_submit = 0.0, t_done = 0.0;
  int state = kQueued;
  salf_status error = SALF_OK;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets;
  std::vector<BatchItem> items;  // host copy; kept until the launch has finished
  uint32_t zero = 0;
  BatchItem* d_items = nullptr;
  uint32_t* d_counter = nullptr;
  void* d_sched = nullptr;  // heaviest-first order of the launch's tiles
};

size_t slot_bytes(int max_batch) {
  return align_up((size_t)max_batch * sizeof(BatchItem)) + kAlign + align_up(tile_work_bytes(kBatchScheduleTiles));
}

}  // namespace
}  // namespace salf

using namespace salf;

struct salf_server {
  salf_context* ctx = nullptr;
  int device = 0;
  salf_server_opts opts;
  char* pool_base = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stopping = false;
  std::deque<uint64_t> queue, admitted;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  Pool pool;
  std::vector<Slot> slots;
  int64_t submitted = 0, completed = 0, released = 0, launches = 0;

  void run();
  bool launch(Slot& s);
};

bool salf_server::launch(Slot& s) {
  s.items.clear();
  s.tickets.clear();
  int64_t tiles = 0, rays = 0;
  uint32_t variants = 0;
  // the ray cap holds while the admitted backlog fits in max_inflight capped launches; past that
  // the GPU is the bottleneck and whole batches keep it fuller (fewer launch tails)
  int64_t cap = opts.max_launch_rays;
  if (cap > 0) {
    int64_t backlog = 0;
    for (uint64_t tk : admitted) backlog += reqs[tk].p.n;
    if (backlog > (int64_t)opts.max_inflight * cap) cap = 0;
  }
  while (!admitted.empty() && (int)s.items.size() < opts.max_batch) {
    Request& r = reqs[admitted.front()];
    if (!s.items.empty() && tiles + r.n_tiles > ((int64_t)1 << 30)) break;
    if (!s.items.empty() && cap > 0 && rays + r.p.n > cap) break;
    rays += r.p.n;
    BatchItem b;
    b.p = r.p;
    b.tile_begin = tiles;
    b.variant = r.variant;
    b.pad = 0;
    variants |= 1u << (r.variant & 7);
    s.items.push_back(b);
    s.tickets.push_back(r.ticket);
    tiles += r.n_tiles;
    r.state = kRunning;
    admitted.pop_front();
  }
  if (s.items.empty()) return false;
  hipError_t e = hipMemcpyAsync(s.d_items, s.items.data(), s.items.size() * sizeof(BatchItem), hipMemcpyHostToDevice,
                                s.stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s.d_counter, &s.zero, sizeof(uint32_t), hipMemcpyHostToDevice, s.stream);
  if (e == hipSuccess) e = launch_batch_schedule(s.d_items, (int32_t)s.items.size(), tiles, s.d_sched, s.stream);
  if (e == hipSuccess)
    e = launch_render_batch(s.d_items, (int32_t)s.items.size(), tiles, s.d_counter, (const int32_t*)s.d_sched,
                            variants, s.stream);
  if (e == hipSuccess) e = hipEventRecord(s.event, s.stream);
  if (e != hipSuccess) {
    const double t = now_s();
    for (uint64_t tk : s.tickets) {
      Request& r = reqs[tk];
      r.state = kDone;
      r.t_done = t;
      r.error = SALF_ERR_DEVICE;
      ++completed;
    }
    s.tickets.clear();
    cv_done.notify_all();
    return true;
  }
  s.busy = true;
  ++launches;
  return true;
}

void salf_server::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool progress = false;
    for (Slot& s : slots) {  // 1. retire finished launches
      if (!s.busy) continue;
      const hipError_t e = hipEventQuery(s.event);
      if (e == hipErrorNotReady) continue;
      const double t = now_s();
      for (uint64_t tk : s.tickets) {
        Request& r = reqs[tk];
        r.state = kDone;
        r.t_done = t;
        if (e != hipSuccess) r.error = SALF_ERR_DEVICE;
        ++completed;
      }
      s.tickets.clear();
      s.busy = false;
      progress = true;
    }
    if (progress) cv_done.notify_all();
    while (!queue.empty()) {  // 2. admit in arrival order while the pool has room
      Request& r = reqs[queue.front()];
      size_t off = 0;
      if (!pool.alloc(r.lay.total, &off)) break;
      r.off = off;
      char* base = pool_base + off;
      r.p.out.rgb = r.lay.rgb == (size_t)-1 ? nullptr : (float*)(base + r.lay.rgb);
      r.p.out.depth = r.lay.depth == (size_t)-1 ? nullptr : (float*)(base + r.lay.depth);
      r.p.out.opacity = r.lay.opacity == (size_t)-1 ? nullptr : (float*)(base + r.lay.opacity);
      r.p.out.intensity = r.lay.intensity == (size_t)-1 ? nullptr : (float*)(base + r.lay.intensity);
      r.state = kAdmitted;
      admitted.push_back(r.ticket);
      queue.pop_front();
      progress = true;
    }
    if (!admitted.empty()) {  // 3. launch everything admitted on a free slot
      for (Slot& s : slots) {
        if (s.busy) continue;
        if (launch(s)) progress = true;
        break;
      }
    }
    bool running = false;
    for (const Slot& s : slots) running = running || s.busy;
    if (stopping && queue.empty() && admitted.empty() && !running) break;
    if (!progress) cv_work.wait_for(lk, std::chrono::microseconds(running ? 20 : 2000));
  }
}

extern "C" {

salf_status salf_server_work_size(const salf_server_opts* opts, size_t* bytes) {
  if (!opts || !bytes) return set_error(SALF_ERR_INVALID_ARG, "NULL argument");
  if (opts->max_batch < 1 || opts->max_batch > kMaxBatch)
    return set_error(SALF_ERR_INVALID_ARG, "max_batch must be in [1, %d]", kMaxBatch);
  if (opts->max_inflight < 1 || opts->max_inflight > kMaxInflight)
    return set_error(SALF_ERR_INVALID_ARG, "max_inflight must be in [1, %d]", kMaxInflight);
  if (opts->max_launch_rays < 0) return set_error(SALF_ERR_INVALID_ARG, "max_launch_rays must be >= 0");
  *bytes = (size_t)opts->max_inflight * slot_bytes(opts->max_batch);
  return SALF_OK;
}

salf_status salf_server_request_bytes(const salf_sensor* sensor, uint32_t outputs, size_t* bytes) {
  salf_status st = validate_sensor(sensor);
  if (st) return st;
  if (!bytes) return set_error(SALF_ERR_INVALID_ARG, "bytes is NULL");
  if (outputs == 0 || (outputs & ~15u)) return set_error(SALF_ERR_INVALID_ARG, "bad output mask %u", outputs);
  *bytes = out_layout((int64_t)sensor->width * sensor->height, outputs).total;
  return SALF_OK;
}

salf_status salf_server_create(salf_context* ctx, const salf_server_opts* opts, salf_server** out) {
  if (!ctx || !opts || !out) return set_error(SALF_ERR_INVALID_ARG, "NULL argument");
  size_t need = 0;
  salf_status st = salf_server_work_size(opts, &need);
  if (st) return st;
  if (!opts->d_pool || opts->pool_bytes < kAlign || ((uintptr_t)opts->d_pool & (kAlign - 1)))
    return set_error(SALF_ERR_INVALID_ARG, "pool must be a 256-byte aligned buffer of at least 256 bytes");
  if (!opts->d_work || opts->work_bytes < need || ((uintptr_t)opts->d_work & (kAlign - 1)))
    return set_error(SALF_ERR_INVALID_ARG, "work buffer must be 256-byte aligned and hold %zu bytes", need);
  salf_server* s = new (std::nothrow) salf_server();
  if (!s) return set_error(SALF_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->ctx = ctx;
  s->device = ctx->device;
  s->opts = *opts;
  s->pool_base = (char*)opts->d_pool;
  s->pool.reset(opts->pool_bytes & ~(kAlign - 1));
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  s->slots.resize(opts->max_inflight);
  for (int i = 0; i < opts->max_inflight; ++i) {
    Slot& sl = s->slots[i];
    char* w = (char*)opts->d_work + (size_t)i * slot_bytes(opts->max_batch);
    sl.d_items = (BatchItem*)w;
    sl.d_counter = (uint32_t*)(w + align_up((size_t)opts->max_batch * sizeof(BatchItem)));
    sl.d_sched = w + align_up((size_t)opts->max_batch * sizeof(BatchItem)) + kAlign;
    hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.event, hipEventDisableTiming);
    if (e != hipSuccess) {
      for (Slot& q : s->slots) {
        if (q.event) (void)hipEventDestroy(q.event);
        if (q.stream) (void)hipStreamDestroy(q.stream);
      }
      delete s;
      if (prev >= 0) (void)hipSetDevice(prev);
      return check_hip(e, "server stream/event creation");
    }
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ++ctx->servers;
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return SALF_OK;
}

salf_status salf_server_submit(salf_server* server, int32_t scene_id, const salf_sensor* sensor,
                               const salf_render_opts* opts, uint32_t outputs, uint64_t* ticket) {
  if (!server || !ticket) return set_error(SALF_ERR_INVALID_ARG, "NULL argument");
  salf_status st = validate_sensor(sensor);
  if (st) return st;
  if ((st = validate_opts(opts)) || (st = one_lane_per_ray(opts, "served requests"))) return st;
  if (outputs == 0 || (outputs & ~15u)) return set_error(SALF_ERR_INVALID_ARG, "bad output mask %u", outputs);
  Scene sc;
  if ((st = scene_snapshot(server->ctx, scene_id, &sc))) return st;
  if (sc.desc.field != SALF_FIELD_CORNER)
    return set_error(SALF_ERR_UNSUPPORTED, "the server renders corner-field scenes");
  if ((outputs & SALF_OUT_RGB) && !sc.view.rgb) return set_error(SALF_ERR_INVALID_ARG, "scene has no colour");
  if ((outputs & SALF_OUT_INTENSITY) && !sc.view.inten)
    return set_error(SALF_ERR_INVALID_ARG, "scene has no intensity");
  Request r;
  const int64_t n = (int64_t)sensor->width * sensor->height;
  r.lay = out_layout(n, outputs);
  if (r.lay.total > server->opts.pool_bytes)
    return set_error(SALF_ERR_BUDGET, "request needs %zu pool bytes, the pool holds %zu", r.lay.total,
                     server->opts.pool_bytes);
  memset(&r.p, 0, sizeof(r.p));
  r.p.scene = sc.view;
  r.p.sensor = *sensor;
  r.p.use_sensor = 1;
  r.p.tiled = 1;
  r.p.img_w = sensor->width;
  r.p.img_h = sensor->height;
  set_tiling(&r.p, sensor->model);
  r.p.n = n;
  r.p.S = opts->samples_per_voxel;
  r.p.t_min = opts->t_min;
  for (int c = 0; c < 3; ++c) r.p.bg[c] = opts->background[c];
  r.variant = ((outputs & SALF_OUT_RGB) ? 1 : 0) | ((outputs & SALF_OUT_INTENSITY) ? 2 : 0) |
              (sc.view.act_geo ? 4 : 0);
  r.outputs = outputs;
  r.n_tiles = (int64_t)r.p.tiles_x * r.p.tiles_y;
  r.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(server->mu);
    if (server->stopping) return set_error(SALF_ERR_BUSY, "server is shutting down");
    r.ticket = server->next_ticket++;
    *ticket = r.ticket;
    server->queue.push_back(r.ticket);
    server->reqs.emplace(r.ticket, r);
    ++server->submitted;
  }
  server->cv_work.notify_one();
  return SALF_OK;
}

salf_status salf_server_poll(salf_server* server, uint64_t ticket, int32_t* done, salf_outputs* out, double* t_submit,
                             double* t_done) {
  if (!server) return set_error(SALF_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(server->mu);
  auto it = server->reqs.find(ticket);
  if (it == server->reqs.end()) return set_error(SALF_ERR_NOT_FOUND, "no request with ticket %llu",
                                                 (unsigned long long)ticket);
  const Request& r = it->second;
  const bool fin = r.state == kDone;
  if (done) *done = fin ? 1 : 0;
  if (t_submit) *t_submit = r.t_submit;
  if (t_done) *t_done = fin ? r.t_done : 0.0;
  if (out) {
    memset(out, 0, sizeof(*out));
    if (fin) {
      out->rgb = r.p.out.rgb;
      out->depth = r.p.out.depth;
      out->opacity = r.p.out.opacity;
      out->intensity = r.p.out.intensity;
    }
  }
  if (fin && r.error) return set_error(r.error, "the launch of request %llu failed", (unsigned long long)ticket);
  return SALF_OK;
}

salf_status salf_server_wait(salf_server* server, uint64_t ticket, double timeout_s, int32_t* done) {
  if (!server) return set_error(SALF_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(server->mu);
  auto fin = [&] {
    auto it = server->reqs.find(ticket);
    return it == server->reqs.end() || it->second.state == kDone;
  };
  if (server->reqs.find(ticket) == server->reqs.end())
    return set_error(SALF_ERR_NOT_FOUND, "no request with ticket %llu", (unsigned long long)ticket);
  const bool ok = server->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s < 0 ? 0 : timeout_s), fin);
  if (done) *done = ok ? 1 : 0;
  return SALF_OK;
}

salf_status salf_server_release(salf_server* server, uint64_t ticket) {
  if (!server) return set_error(SALF_ERR_INVALID_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(server->mu);
    auto it = server->reqs.find(ticket);
    if (it == server->reqs.end())
      return set_error(SALF_ERR_NOT_FOUND, "no request with ticket %llu", (unsigned long long)ticket);
    if (it->second.state != kDone)
      return set_error(SALF_ERR_BUSY, "request %llu is not done", (unsigned long long)ticket);
    server->pool.release(it->second.off, it->second.lay.total);
    server->reqs.erase(it);
    ++server->released;
  }
  server->cv_work.notify_one();
  return SALF_OK;
}

salf_status salf_server_get_stats(salf_server* server, salf_server_stats* out) {
  if (!server || !out) return set_error(SALF_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(server->mu);
  out->submitted = server->submitted;
  out->completed = server->completed;
  out->released = server->released;
  out->launches = server->launches;
  out->pool_in_use = server->pool.in_use;
  out->pool_peak = server->pool.peak;
  out->queued = (int32_t)server->queue.size();
  int32_t inflight = 0;
  for (const auto& kv : server->reqs)
    if (kv.second.state == kAdmitted || kv.second.state == kRunning) ++inflight;
  out->inflight = inflight;
  return SALF_OK;
}

salf_status salf_server_destroy(salf_server* server) {
  if (!server) return set_error(SALF_ERR_INVALID_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(server->mu);
    server->stopping = true;
  }
  server->cv_work.notify_one();
  if (server->worker.joinable()) server->worker.join();
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(server->device);
  for (Slot& s : server->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    if (s.event) (void)hipEventDestroy(s.event);
    if (s.stream) (void)hipStreamDestroy(s.stream);
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  {
    std::lock_guard<std::mutex> lk(server->ctx->mu);
    --server->ctx->servers;
  }
  delete server;
  return SALF_OK;
}

}  // extern "C"
