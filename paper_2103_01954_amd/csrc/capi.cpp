// C ABI of libmvp: contexts, the per-frame acceleration structure, forward and
// backward marches, and the test exports.  Serving lives in serve.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>

#include "ctx.h"

namespace mvp {

static thread_local std::string g_error = "no error";

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}

mvp_status status_of(hipError_t e) {
  if (e == hipSuccess) return MVP_OK;
  return e == hipErrorOutOfMemory ? MVP_ERR_OOM : MVP_ERR_DEVICE;
}

#define MVP_HIP(expr)                                                      \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));           \
      return status_of(e_);                                                \
    }                                                                      \
  } while (0)

// ---------------------------------------------------------------------------
// arena
// ---------------------------------------------------------------------------

static size_t round_size(size_t b) {
  if (b < 256) b = 256;
  const size_t q = b < (1u << 20) ? 256 : (2u << 20);
  return (b + q - 1) / q * q;
}

PinnedPool::~PinnedPool() {
  for (void *p : all_) (void)hipHostFree(p);
}

void *PinnedPool::get() {
  {
    std::lock_guard<std::mutex> g(mu_);
    if (!free_.empty()) {
      void *p = free_.back();
      free_.pop_back();
      return p;
    }
  }
  void *p = nullptr;
  if (hipHostMalloc(&p, kPinnedBlock, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> g(mu_);
  all_.push_back(p);
  return p;
}

void PinnedPool::put(void *p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(mu_);
  free_.push_back(p);
}

Arena::~Arena() {
  std::lock_guard<std::mutex> g(mu_);
  for (auto &p : pending_) {
    (void)hipEventSynchronize(p.ev);
    (void)hipEventDestroy(p.ev);
    for (void *b : p.blocks) free_.emplace(size_[b], b);
  }
  pending_.clear();
  for (hipEvent_t e : events_) (void)hipEventDestroy(e);
  events_.clear();
  trim_locked();
  for (auto &kv : size_) (void)hipFree(kv.first);   // blocks still owned by live objects
}

void Arena::reap_locked() {
  for (size_t i = 0; i < pending_.size();) {
    if (hipEventQuery(pending_[i].ev) == hipSuccess) {
      events_.push_back(pending_[i].ev);
      for (void *b : pending_[i].blocks) free_.emplace(size_[b], b);
      pending_[i] = pending_.back();
      pending_.pop_back();
    } else {
      ++i;
    }
  }
}

void Arena::trim_locked() {
  for (auto &kv : free_) {
    (void)hipFree(kv.second);
    held_ -= kv.first;
    size_.erase(kv.second);
  }
  free_.clear();
}

void Arena::trim() {
  std::lock_guard<std::mutex> g(mu_);
  reap_locked();
  trim_locked();
}

size_t Arena::held_bytes() {
  std::lock_guard<std::mutex> g(mu_);
  return held_;
}

mvp_status Arena::alloc(size_t bytes, void **out) {
  const size_t sz = round_size(bytes);
  std::lock_guard<std::mutex> g(mu_);
  auto fit = [&]() {
    auto it = free_.lower_bound(sz);
    if (it == free_.end() || it->first > 2 * sz) return false;
    *out = it->second;
    free_.erase(it);
    return true;
  };
  if (fit()) return MVP_OK;
  reap_locked();   // blocks whose streams have passed their release points
  if (fit()) return MVP_OK;
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    trim_locked();
    e = hipMalloc(&p, sz);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of %zu bytes failed: %s", sz, hipGetErrorString(e));
    return status_of(e);
  }
  size_[p] = sz;
  held_ += sz;
  *out = p;
  return MVP_OK;
}

void Arena::release_now(void *p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(mu_);
  free_.emplace(size_[p], p);
}

mvp_status Arena::get_event(hipEvent_t *ev) {
  {
    std::lock_guard<std::mutex> g(mu_);
    if (!events_.empty()) {
      *ev = events_.back();
      events_.pop_back();
      return MVP_OK;
    }
  }
  const hipError_t e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    set_error("event creation failed: %s", hipGetErrorString(e));
    return status_of(e);
  }
  return MVP_OK;
}

void Arena::put_event(hipEvent_t ev) {
  if (!ev) return;
  std::lock_guard<std::mutex> g(mu_);
  events_.push_back(ev);
}

mvp_status Arena::release_after(const std::vector<void *> &blocks, hipStream_t s) {
  if (blocks.empty()) return MVP_OK;
  hipEvent_t ev = nullptr;
  hipError_t e = get_event(&ev) == MVP_OK ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess) e = hipEventRecord(ev, s);
  std::lock_guard<std::mutex> g(mu_);
  if (e != hipSuccess) {
    // cannot track completion: wait for the stream instead
    (void)hipStreamSynchronize(s);
    if (ev) events_.push_back(ev);
    for (void *b : blocks) free_.emplace(size_[b], b);
    set_error("event record failed: %s", hipGetErrorString(e));
    return MVP_ERR_DEVICE;
  }
  pending_.push_back({ev, blocks});
  return MVP_OK;
}

// ---------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------

mvp_status check_prims(const mvp_prims *p, bool need_payload) {
  if (!p) { set_error("prims is NULL"); return MVP_ERR_INVALID; }
  if (p->n_prim < 0) { set_error("n_prim < 0"); return MVP_ERR_INVALID; }
  if (p->M < 2 || p->M > 1024) { set_error("payload size M=%d out of range [2,1024]", p->M); return MVP_ERR_INVALID; }
  if (p->payload_dtype != MVP_F32 && p->payload_dtype != MVP_BF16) { set_error("bad payload dtype"); return MVP_ERR_INVALID; }
  if ((int64_t)p->M * p->M * p->M * (int64_t)p->n_prim > (int64_t)1 << 40) { set_error("payload too large"); return MVP_ERR_INVALID; }
  if ((int64_t)p->M * p->M * p->M >= (int64_t)1 << 31) { set_error("M^3 too large"); return MVP_ERR_INVALID; }
  if (p->n_prim > 0) {
    if (!p->pos || !p->rot || !p->scale) { set_error("pos/rot/scale pointer is NULL"); return MVP_ERR_INVALID; }
    if (need_payload && !p->payload) { set_error("payload pointer is NULL"); return MVP_ERR_INVALID; }
    const size_t align = p->payload_dtype == MVP_F32 ? 16 : 8;
    if (need_payload && ((uintptr_t)p->payload % align)) { set_error("payload not %zu-byte aligned", align); return MVP_ERR_INVALID; }
  }
  return MVP_OK;
}

mvp_status check_camera(const mvp_camera *c) {
  if (c->width <= 0 || c->height <= 0 || c->width > 32768 || c->height > 32768) {
    set_error("camera size %dx%d out of range", c->width, c->height);
    return MVP_ERR_INVALID;
  }
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(c->origin[i])) { set_error("camera origin not finite"); return MVP_ERR_INVALID; }
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(c->pix2dir[i])) { set_error("camera matrix not finite"); return MVP_ERR_INVALID; }
  return MVP_OK;
}

mvp_status check_params(const mvp_march_params *p) {
  if (!p) { set_error("params is NULL"); return MVP_ERR_INVALID; }
  if (!(p->step > 0.0f) || !std::isfinite(p->step)) { set_error("step must be finite and > 0"); return MVP_ERR_INVALID; }
  if (!(p->eps_early >= 0.0f && p->eps_early < 1.0f)) { set_error("eps_early must be in [0,1)"); return MVP_ERR_INVALID; }
  if (!(p->t_near >= 0.0f) || !std::isfinite(p->t_near)) { set_error("t_near must be finite and >= 0"); return MVP_ERR_INVALID; }
  if (!(p->fade_alpha >= 0.0f) || !std::isfinite(p->fade_alpha)) { set_error("fade_alpha must be finite and >= 0"); return MVP_ERR_INVALID; }
  if (p->fade_alpha > 0.0f && (!(p->fade_beta > 0.0f) || !std::isfinite(p->fade_beta))) { set_error("fade_beta must be finite and > 0"); return MVP_ERR_INVALID; }
  if (p->combine != MVP_COMBINE_SUM && p->combine != MVP_COMBINE_SEQUENTIAL) { set_error("combine must be MVP_COMBINE_SUM or MVP_COMBINE_SEQUENTIAL"); return MVP_ERR_INVALID; }
  return MVP_OK;
}

static bool invert3(const float *m, float *out) {
  const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5], g = m[6], h = m[7], i = m[8];
  const double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
  const double det = a * A + b * B + c * C;
  if (!(std::fabs(det) > 0) || !std::isfinite(det)) return false;
  const double inv[9] = {A, -(b * i - c * h), b * f - c * e, B, a * i - c * g, -(a * f - c * d),
                         C, -(a * h - b * g), a * e - b * d};
  for (int k = 0; k < 9; ++k) out[k] = (float)(inv[k] / det);
  return true;
}

// ---------------------------------------------------------------------------
// acceleration structure
// ---------------------------------------------------------------------------

namespace {
// Device blocks of one call; on an error path they are recycled once the work
// already enqueued on the stream has finished.
struct Blocks {
  mvp_ctx *ctx;
  hipStream_t s;
  std::vector<void *> list;
  bool keep = false;
  template <typename T>
  mvp_status get(T **p, size_t count) {
    void *v = nullptr;
    mvp_status st = ctx->arena.alloc(count * sizeof(T) + 16, &v);
    if (st != MVP_OK) return st;
    list.push_back(v);
    *p = (T *)v;
    return MVP_OK;
  }
  ~Blocks() {
    if (!keep) ctx->arena.release_after(list, s);
  }
};
}  // namespace

#define MVP_CHECK(expr)                 \
  do {                                  \
    mvp_status st_ = (expr);            \
    if (st_ != MVP_OK) return st_;      \
  } while (0)

static mvp_status read_u64(const uint64_t *dev, uint64_t *host, hipStream_t s) {
  MVP_HIP(hipMemcpyAsync(host, dev, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  MVP_HIP(hipStreamSynchronize(s));
  return MVP_OK;
}

// The transposed lists (primitive -> its culling-list entries) and the
// backward work items, on the context's side stream after the build's kernels
// (event `built`); they need only the sorted culling lists.  Launched once, by
// the first forward after its own launch or by the first backward; `lists` is
// recorded after them and the held temporaries are recycled after them.
static mvp_status launch_lists(const mvp_accel *ac) {
  if (!ac->lists_pending.exchange(false)) return MVP_OK;
  mvp_accel *a = const_cast<mvp_accel *>(ac);
  mvp_ctx *ctx = a->ctx;
  hipStream_t s2 = ctx->side;
  const AccelView av = a->view(2);
  const size_t N = (size_t)a->N;
  const uint64_t ne = (uint64_t)a->n_tile_pairs;
  hipError_t e = hipStreamWaitEvent(s2, a->built, 0);
  if (e == hipSuccess) e = launch_zero_u32(a->prim_cnt, N, s2);
  if (e == hipSuccess) e = launch_prim_entry_count(a->tile_list, ne, a->prim_cnt, s2);
  if (e == hipSuccess) e = launch_scan_u32_u64(a->prim_cnt, a->prim_entry_off, N, a->scan_scratch, s2);
  if (e == hipSuccess) e = launch_prim_entry_place(av, a->rect, ne, a->prim_entry_off, a->prim_entries, s2);
  if (e == hipSuccess)
    e = launch_prim_order(a->rect, a->N, a->V, a->tiles_x, a->tiles_y, a->prim_key, a->prim_bcnt,
                          a->prim_boff, a->scan_scratch, a->item_prim, s2);
  if (e == hipSuccess)
    e = launch_item_count(a->prim_entry_off, a->item_prim, a->N, a->item_entries, a->prim_cnt, s2);
  if (e == hipSuccess) e = launch_scan_u32_u64(a->prim_cnt, a->item_off, N, a->scan_scratch, s2);
  if (e == hipSuccess) e = hipEventRecord(a->lists, s2);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s2);
    a->lists_pending.store(true);   // a later call tries again
    MVP_HIP(e);
  }
  MVP_CHECK(ctx->arena.release_after(a->lists_temps, s2));
  a->lists_temps.clear();
  return MVP_OK;
}

mvp_status build_accel(mvp_ctx *ctx, const mvp_prims *prims, const mvp_camera *cams, int32_t n_views,
                       const mvp_march_params *params, const int64_t *rays, int64_t n_rays,
                       mvp_accel **out, hipStream_t s, const Admit *admit, bool for_backward) {
  if (!ctx || !out || !cams) { set_error("NULL argument"); return MVP_ERR_INVALID; }
  *out = nullptr;
  MVP_CHECK(check_prims(prims, false));
  MVP_CHECK(check_params(params));
  if (n_views < 1) { set_error("n_views must be >= 1"); return MVP_ERR_INVALID; }
  for (int v = 0; v < n_views; ++v) {
    MVP_CHECK(check_camera(&cams[v]));
    if (cams[v].width != cams[0].width || cams[v].height != cams[0].height) {
      set_error("all views of one structure must share a resolution");
      return MVP_ERR_INVALID;
    }
  }
  const int W = cams[0].width, H = cams[0].height, N = prims->n_prim;
  const int tx = (W + kTile - 1) / kTile, ty = (H + kTile - 1) / kTile;
  const size_t ntile = (size_t)n_views * tx * ty;
  const size_t npix = (size_t)n_views * W * H;
  if (rays && n_rays < 0) { set_error("n_rays < 0"); return MVP_ERR_INVALID; }
  if (!rays && n_rays != 0) { set_error("rays is NULL"); return MVP_ERR_INVALID; }
  const size_t R = rays ? (size_t)n_rays : npix;   // ray slots
  if (ntile >= (size_t)1 << 31) { set_error("too many tiles"); return MVP_ERR_INVALID; }
  if (R >= (size_t)1 << 31) { set_error("too many rays (%zu) in one structure", R); return MVP_ERR_INVALID; }

  mvp_accel *a = new (std::nothrow) mvp_accel();
  if (!a) { set_error("host allocation failed"); return MVP_ERR_OOM; }
  a->ctx = ctx; a->V = n_views; a->W = W; a->H = H; a->N = N; a->tiles_x = tx; a->tiles_y = ty;
  a->n_slots = (int64_t)R;
  a->params = *params;
  a->cams_host.resize(n_views);
  for (int v = 0; v < n_views; ++v) {
    DevCam &c = a->cams_host[v];
    memcpy(c.o, cams[v].origin, sizeof c.o);
    memcpy(c.P, cams[v].pix2dir, sizeof c.P);
    c.W = W;
    c.H = H;
    if (!invert3(c.P, c.Pinv)) {
      delete a;
      set_error("camera matrix of view %d is singular", v);
      return MVP_ERR_INVALID;
    }
  }
  struct Guard {
    mvp_accel *a;
    bool keep = false;
    ~Guard() {
      if (keep) return;
      for (hipEvent_t e : {a->built, a->lists, a->pairs_done}) a->ctx->arena.put_event(e);
      delete a;
    }
  } guard{a};

  MVP_HIP(hipSetDevice(ctx->device));
  Blocks keep{ctx, s}, temp{ctx, s}, ltmp{ctx, s};   // ltmp: temporaries the transposed lists read
  int4 *rect = nullptr;
  uint32_t *tile_cnt = nullptr, *cap = nullptr, *rcnt = nullptr, *depth = nullptr;
  uint8_t *scratch = nullptr;
  const size_t sb = scan_scratch_bytes(std::max<size_t>(std::max<size_t>(ntile, (size_t)N), (size_t)kPrimBuckets));
  if (admit) {
    const size_t base = n_views * sizeof(DevCam) + 3 * (size_t)N * 16 + 2 * (ntile + 1) * 8 + R * 16 + 16 +
                        kNumCounters * 8 + (size_t)n_views * N * 20 + 2 * ntile * 4 + sb + 10 * 256 +
                        (rays ? R * 12 + ntile * 12 + 3 * 256 : 0);
    MVP_CHECK(admit->fn(admit->user, base));
  }
  MVP_CHECK(keep.get(&a->cams, n_views));
  MVP_CHECK(keep.get(&a->xf, 3 * (size_t)N));
  MVP_CHECK(keep.get(&a->tile_off, ntile + 1));
  MVP_CHECK(keep.get(&a->pair_base, ntile + 1));
  MVP_CHECK(keep.get(&a->ray_seg, R ? R : 1));
  MVP_CHECK(keep.get(&a->ray_nj, R ? R : 1));
  MVP_CHECK(keep.get(&a->counters, kNumCounters));
  MVP_CHECK(ltmp.get(&rect, (size_t)n_views * N));
  MVP_CHECK(temp.get(&depth, (size_t)n_views * N));
  MVP_CHECK(temp.get(&tile_cnt, ntile));
  MVP_CHECK(temp.get(&cap, ntile));
  MVP_CHECK(ltmp.get(&scratch, sb));
  // cameras up and list sizes down through a pinned block (returned once the
  // build has synchronised, or on any early return)
  struct PinHold {
    PinnedPool &pool;
    void *p;
    hipStream_t s;
    bool synced = false;
    ~PinHold() {   // a copy still in flight on an early return must not see the block reused
      if (p && !synced) (void)hipStreamSynchronize(s);
      pool.put(p);
    }
  } pin{ctx->pinned, ctx->pinned.get(), s};
  const size_t cam_bytes = n_views * sizeof(DevCam);
  if (pin.p && cam_bytes + 64 <= kPinnedBlock) {
    memcpy((char *)pin.p + 64, a->cams_host.data(), cam_bytes);
    MVP_HIP(hipMemcpyAsync(a->cams, (char *)pin.p + 64, cam_bytes, hipMemcpyHostToDevice, s));
  } else {
    MVP_HIP(hipMemcpyAsync(a->cams, a->cams_host.data(), cam_bytes, hipMemcpyHostToDevice, s));
  }
  MVP_HIP(launch_zero_u64((uint64_t *)a->counters, kNumCounters, s));
  uint32_t *flag = nullptr;
  if (rays) {
    // ray subset: a private copy of the pixel ids, binned into screen tiles
    MVP_CHECK(keep.get(&a->ray_pix, R ? R : 1));
    MVP_CHECK(keep.get(&a->tile_ray_off, ntile + 1));
    MVP_CHECK(keep.get(&a->tile_rays, R ? R : 1));
    MVP_CHECK(temp.get(&rcnt, ntile));
    MVP_CHECK(temp.get(&flag, 1));
    if (R) MVP_HIP(hipMemcpyAsync(a->ray_pix, rays, R * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    AccelView rv = a->view(2);
    MVP_HIP(launch_zero_u32(rcnt, ntile, s));
    MVP_HIP(launch_zero_u32(flag, 1, s));
    MVP_HIP(launch_ray_bin(rv, rcnt, flag, s));
    MVP_HIP(launch_scan_u32_u64(rcnt, a->tile_ray_off, ntile, scratch, s));
    // rcnt keeps the per-tile ray counts (for the pair capacities); the fill
    // takes its own cursor
    uint32_t *cursor = nullptr;
    MVP_CHECK(temp.get(&cursor, ntile));
    MVP_HIP(launch_zero_u32(cursor, ntile, s));
    MVP_HIP(launch_ray_fill(rv, cursor, a->tile_rays, s));
    MVP_HIP(launch_segment_sort(a->tile_ray_off, a->tile_rays, (int64_t)ntile, nullptr, 0, 1, s));
  }
  AccelView av = a->view(2);

  // culling lists: rectangles, tile counts, offsets; pair capacities; one
  // stream synchronisation for the sizes
  MVP_HIP(launch_zero_u32(tile_cnt, ntile, s));
  MVP_HIP(launch_prep(*prims, av, a->xf, rect, depth, tile_cnt, s));
  MVP_HIP(launch_scan_u32_u64(tile_cnt, a->tile_off, ntile, scratch, s));
  MVP_HIP(launch_tile_capacity(tile_cnt, rcnt, ntile, cap, s));
  MVP_HIP(launch_scan_u32_u64(cap, a->pair_base, ntile, scratch, s));
  // the three sizes gathered into one small device block, then one copy down
  uint64_t *dsz = (uint64_t *)a->counters + kCntSizes;
  MVP_HIP(launch_gather_sizes(a->tile_off + ntile, a->pair_base + ntile, flag, dsz, s));
  uint64_t host_sz[3] = {0, 0, 0};
  uint64_t *hsz = pin.p ? (uint64_t *)pin.p : host_sz;
  MVP_HIP(hipMemcpyAsync(hsz, dsz, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  MVP_HIP(hipStreamSynchronize(s));
  pin.synced = true;
  const uint64_t n_tile_pairs = hsz[0], capacity = hsz[1];
  const uint32_t flag_h = (uint32_t)hsz[2];
  if (flag_h & 1u) { set_error("a ray pixel id is outside [0, n_views*height*width)"); return MVP_ERR_INVALID; }
  if (flag_h & 2u) { set_error("more than 256 rays in one 16x16 tile (repeated pixel ids)"); return MVP_ERR_INVALID; }
  if (capacity >= (uint64_t)1 << 32) {
    set_error("%llu ray/primitive pair slots exceed 2^32 (%llu culling-list entries)", (unsigned long long)capacity,
              (unsigned long long)n_tile_pairs);
    return MVP_ERR_INVALID;
  }
  const size_t ntp = n_tile_pairs ? n_tile_pairs : 1;
  const size_t npc = capacity ? capacity : 1;
  const size_t list_bytes = for_backward ? ntp * (4 + 4 + 48 + 8 + 16 + 4) + (size_t)N * 20 + 24 + npc * 24
                                         : ntp * (4 + 48) + npc * 16;
  if (admit) MVP_CHECK(admit->fn(admit->user, list_bytes + 8 * 256));
  a->for_backward = for_backward;
  MVP_CHECK(keep.get(&a->tile_list, ntp));
  MVP_CHECK(keep.get(&a->ef, 3 * ntp));
  MVP_CHECK(keep.get(&a->pr, npc));
  uint32_t *prim_cnt = nullptr;
  if (for_backward) {
    MVP_CHECK(keep.get(&a->prim_entries, ntp));
    MVP_CHECK(keep.get(&a->prim_entry_off, (size_t)N + 1));
    MVP_CHECK(keep.get(&a->item_off, (size_t)N + 1));
    MVP_CHECK(keep.get(&a->item_prim, N ? (size_t)N : 1));
    MVP_CHECK(keep.get(&a->ent_base, ntp));
    MVP_CHECK(keep.get(&a->ent_n, 4 * ntp));
    MVP_CHECK(keep.get(&a->ent_tile, ntp));
    MVP_CHECK(keep.get(&a->ent_rec, npc));
    MVP_CHECK(ltmp.get(&prim_cnt, (size_t)N + 1));
    MVP_CHECK(ltmp.get(&a->prim_key, N ? (size_t)N : 1));
    MVP_CHECK(ltmp.get(&a->prim_bcnt, (size_t)kPrimBuckets));
    MVP_CHECK(ltmp.get(&a->prim_boff, (size_t)kPrimBuckets + 1));
  }
  av = a->view(2);
  MVP_HIP(launch_zero_u32(tile_cnt, ntile, s));
  MVP_HIP(launch_tile_fill(av, rect, tile_cnt, a->tile_list, s));
  MVP_HIP(launch_segment_sort(a->tile_off, a->tile_list, (int64_t)ntile, depth, N, tx * ty, s));
  a->item_entries = backward_item_entries(prims->M);
  a->n_items_max = for_backward ? (int64_t)(n_tile_pairs / a->item_entries) + N : 0;
  // Every ray's pairs, the entry frames and the per-entry pair lists: either
  // by the pairs kernel now, or by the first forward, each workgroup building
  // its tile's pairs just before marching them.  Fusing pays where the march
  // has latency to hide the pairs pass in (payloads of at most 8^3, which stay
  // in the caches) and the grid has enough tiles (32 per CU) for the pairs
  // phases of some workgroups to overlap the marching of others; elsewhere the
  // pairs kernel, at its own higher occupancy, is faster.
  a->po = PairsOut{a->ef, a->pr, a->ray_seg, a->ray_nj, a->ent_base, a->ent_n, a->ent_tile, a->ent_rec,
                   a->counters + kCntPairs};
  // MVP_PAIRS_IN_FORWARD=1 or 0 overrides the choice (tests and tuning)
  const char *force = getenv("MVP_PAIRS_IN_FORWARD");
  const bool fuse = force && (force[0] == '0' || force[0] == '1') ? force[0] == '1' : prims->M <= 8 && ntile >= 8192;
  MVP_CHECK(ctx->arena.get_event(&a->pairs_done));
  if (for_backward) MVP_CHECK(ctx->arena.get_event(&a->lists));
  MVP_CHECK(ctx->arena.get_event(&a->built));
  MVP_HIP(hipEventRecord(a->built, s));   // the culling lists are complete
  if (!fuse) {
    MVP_HIP(launch_pairs(av, a->po, s));
    MVP_HIP(hipEventRecord(a->pairs_done, s));
  }

  a->n_tile_pairs = (int64_t)n_tile_pairs;
  a->n_ray_pairs = -1;   // read from the device on demand (mvp_accel_get_info)
  a->pair_capacity = capacity;
  a->bytes = (int64_t)(n_views * sizeof(DevCam) + 3 * (size_t)N * 16 + 2 * (ntile + 1) * 8 + R * 16 +
                       kNumCounters * 8 +
                       (for_backward ? n_tile_pairs * (4 + 4 + 48 + 8 + 16 + 4) + (size_t)N * 24 + capacity * 24
                                     : n_tile_pairs * (4 + 48) + capacity * 16) +
                       (rays ? R * 12 + (ntile + 1) * 8 : 0));
  a->blocks = keep.list;
  keep.keep = true;
  // temporaries are recycled once the build's kernels have run, except those
  // of the transposed lists, which the structure holds until they are launched
  // (now, beside the pairs kernel; or after the first forward when that builds
  // the pairs, so that their launches are off the path to the forward)
  MVP_CHECK(ctx->arena.release_after(temp.list, s));
  temp.keep = true;
  if (for_backward) {
    a->rect = rect;
    a->prim_cnt = prim_cnt;
    a->scan_scratch = scratch;
    a->lists_temps = ltmp.list;
    ltmp.keep = true;
    a->lists_pending.store(true);
  }
  a->pairs_pending.store(fuse);
  a->pairs_in_forward = fuse;
  guard.keep = true;
  ctx->live_accels.fetch_add(1);
  *out = a;
  // beside the pairs kernel; on failure the first backward tries again
  if (!fuse) (void)launch_lists(a);
  return MVP_OK;
}

mvp_status destroy_accel(mvp_ctx *ctx, mvp_accel *a, hipStream_t s) {
  if (!ctx || !a || a->ctx != ctx) { set_error("bad accel handle"); return MVP_ERR_INVALID; }
  if (a->lists_pending.exchange(false)) {
    (void)ctx->arena.release_after(a->lists_temps, s);   // never launched: last used by the build
  } else if (a->lists) {
    (void)hipStreamWaitEvent(s, a->lists, 0);   // the transposed lists are written on the side stream
  }
  mvp_status st = ctx->arena.release_after(a->blocks, s);
  ctx->live_accels.fetch_sub(1);
  for (hipEvent_t e : {a->built, a->lists, a->pairs_done}) ctx->arena.put_event(e);
  delete a;
  return st;
}

// ---------------------------------------------------------------------------
// allocation-free backward: per-ray scratch in a fixed device array
// ---------------------------------------------------------------------------

// Scratch of mvp_render_bwd_noalloc: room for the per-ray constants and bounds
// of MVP_NOALLOC_MAX_RAYS rays (24 MiB).  Every device the library runs on
// holds its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, never the device memory: kernels and copies get the
// address that hipGetSymbolAddress returns for the device, kept in
// g_scratch[device] by resolve_scratch.
static __device__ __align__(256) unsigned char scratch[bwd_scratch_bytes(MVP_NOALLOC_MAX_RAYS)];
constexpr int kMaxDevices = 64;
static void *g_scratch[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];
static std::once_flag g_scratch_once[kMaxDevices];

// Resolve this device's copy of `scratch`, once per device; the device must be
// current.  Called by mvp_create.
static mvp_status resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device %d beyond the %d devices the library supports", device, kMaxDevices);
    return MVP_ERR_INVALID;
  }
  std::call_once(g_scratch_once[device], [device] {
    void *ptr = nullptr;
    g_scratch_err[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (g_scratch_err[device] == hipSuccess) g_scratch[device] = ptr;
    else (void)hipGetLastError();
  });
  if (!g_scratch[device]) {
    set_error("hipGetSymbolAddress of the backward scratch array failed on device %d: %s", device,
              hipGetErrorString(g_scratch_err[device]));
    return MVP_ERR_DEVICE;
  }
  return MVP_OK;
}

static mvp_status check_render(mvp_ctx *ctx, const mvp_accel *a, const mvp_prims *p) {
  if (!ctx || !a || a->ctx != ctx) { set_error("bad context or accel handle"); return MVP_ERR_INVALID; }
  MVP_CHECK(check_prims(p, true));
  if (p->n_prim != a->N) { set_error("prims has %d primitives, accel was built for %d", p->n_prim, a->N); return MVP_ERR_INVALID; }
  return MVP_OK;
}

}  // namespace mvp

using namespace mvp;

// ---------------------------------------------------------------------------
// exported C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *mvp_last_error(void) { return g_error.c_str(); }
const char *mvp_version(void) { return "mvp-mi355x 0.1 (gfx950)"; }

mvp_status mvp_create(int device, mvp_ctx **out) {
  if (!out) { set_error("out is NULL"); return MVP_ERR_INVALID; }
  *out = nullptr;
  int n = 0;
  MVP_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) { set_error("device %d out of range (%d devices)", device, n); return MVP_ERR_INVALID; }
  MVP_HIP(hipSetDevice(device));
  MVP_CHECK(resolve_scratch(device));
  mvp_ctx *c = new (std::nothrow) mvp_ctx(device);
  if (!c) { set_error("host allocation failed"); return MVP_ERR_OOM; }
  const hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    return status_of(e);
  }
  *out = c;
  return MVP_OK;
}

mvp_status mvp_destroy(mvp_ctx *ctx) {
  if (!ctx) { set_error("ctx is NULL"); return MVP_ERR_INVALID; }
  if (ctx->live_accels.load() != 0) { set_error("%d acceleration structures still alive", ctx->live_accels.load()); return MVP_ERR_BUSY; }
  serve_shutdown(ctx);
  (void)mvp_timing_stop(ctx);
  (void)hipSetDevice(ctx->device);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  delete ctx;
  return MVP_OK;
}

mvp_status mvp_build_accel(mvp_ctx *ctx, const mvp_prims *prims, const mvp_camera *cams, int32_t n_views,
                           const mvp_march_params *params, mvp_accel **out, void *stream) {
  return build_accel(ctx, prims, cams, n_views, params, nullptr, 0, out, (hipStream_t)stream, nullptr);
}

mvp_status mvp_build_accel_rays(mvp_ctx *ctx, const mvp_prims *prims, const mvp_camera *cams, int32_t n_views,
                                const mvp_march_params *params, const int64_t *rays, int64_t n_rays,
                                mvp_accel **out, void *stream) {
  static const int64_t no_rays = 0;   // an empty list may come as NULL; it is never read
  if (!rays && n_rays == 0) rays = &no_rays;
  if (!rays) { set_error("rays is NULL"); return MVP_ERR_INVALID; }
  return build_accel(ctx, prims, cams, n_views, params, rays, n_rays, out, (hipStream_t)stream, nullptr);
}

mvp_status mvp_accel_destroy(mvp_ctx *ctx, mvp_accel *accel, void *stream) {
  return destroy_accel(ctx, accel, (hipStream_t)stream);
}

mvp_status mvp_accel_get_info(const mvp_accel *a, mvp_accel_info *info) {
  if (!a || !info) { set_error("NULL argument"); return MVP_ERR_INVALID; }
  if (a->n_ray_pairs < 0 && !a->pairs_pending.load()) {   // counted on the device by the pass that built them
    MVP_HIP(hipSetDevice(a->ctx->device));
    MVP_HIP(hipEventSynchronize(a->pairs_done));
    uint64_t n = 0;
    MVP_HIP(hipMemcpy(&n, a->counters + kCntPairs, sizeof n, hipMemcpyDeviceToHost));
    const_cast<mvp_accel *>(a)->n_ray_pairs = (int64_t)n;
  }
  info->n_views = a->V; info->width = a->W; info->height = a->H; info->n_prim = a->N;
  info->n_tile_pairs = a->n_tile_pairs; info->n_ray_pairs = a->n_ray_pairs; info->device_bytes = a->bytes;
  info->pairs_in_forward = a->pairs_in_forward ? 1 : 0;
  info->reserved = 0;
  return MVP_OK;
}

// Next free event pair of a kernel kind, or {nullptr, nullptr} when not recording.
static std::pair<hipEvent_t, hipEvent_t> timer_slot(mvp_ctx *ctx, int kind) {
  std::lock_guard<std::mutex> g(ctx->timer.m);
  mvp::KernelTimer &t = ctx->timer;
  if (t.n[kind] >= t.cap) return {nullptr, nullptr};
  const int i = t.n[kind]++;
  return {t.ev[kind][2 * i], t.ev[kind][2 * i + 1]};
}

static void timer_free(mvp::KernelTimer &t) {
  for (auto &v : t.ev) {
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
    v.clear();
  }
  t.cap = 0;
  t.n[0] = t.n[1] = 0;
}

mvp_status mvp_timing_start(mvp_ctx *ctx, int32_t capacity) {
  if (!ctx) { set_error("ctx is NULL"); return MVP_ERR_INVALID; }
  if (capacity < 1 || capacity > (1 << 16)) { set_error("capacity must be in [1, 65536]"); return MVP_ERR_INVALID; }
  MVP_HIP(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> g(ctx->timer.m);
  timer_free(ctx->timer);
  for (auto &v : ctx->timer.ev) {
    v.resize(2 * (size_t)capacity, nullptr);
    for (hipEvent_t &e : v) {
      if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        timer_free(ctx->timer);
        set_error("hipEventCreate failed");
        return MVP_ERR_DEVICE;
      }
    }
  }
  ctx->timer.cap = capacity;
  return MVP_OK;
}

mvp_status mvp_timing_read(mvp_ctx *ctx, int32_t kernel, float *ms, int32_t *n) {
  if (!ctx || !ms || !n) { set_error("bad argument"); return MVP_ERR_INVALID; }
  if (kernel != MVP_KERNEL_FWD_MARCH && kernel != MVP_KERNEL_BWD_MARCH) { set_error("unknown kernel %d", kernel); return MVP_ERR_INVALID; }
  MVP_HIP(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> g(ctx->timer.m);
  const mvp::KernelTimer &t = ctx->timer;
  for (int i = 0; i < t.n[kernel]; ++i) {
    MVP_HIP(hipEventSynchronize(t.ev[kernel][2 * i + 1]));
    MVP_HIP(hipEventElapsedTime(&ms[i], t.ev[kernel][2 * i], t.ev[kernel][2 * i + 1]));
  }
  *n = t.n[kernel];
  return MVP_OK;
}

mvp_status mvp_timing_stop(mvp_ctx *ctx) {
  if (!ctx) { set_error("ctx is NULL"); return MVP_ERR_INVALID; }
  MVP_HIP(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> g(ctx->timer.m);
  for (auto &v : ctx->timer.ev)
    for (hipEvent_t e : v) (void)hipEventSynchronize(e);
  timer_free(ctx->timer);
  return MVP_OK;
}

static mvp_status render_fwd(mvp_ctx *ctx, const mvp_accel *a, const mvp_prims *prims, const float *bg,
                             float *rgba, mvp_ray_aux *aux, hipStream_t s) {
  MVP_CHECK(check_render(ctx, a, prims));
  if (!rgba && a->n_slots > 0) { set_error("rgba is NULL"); return MVP_ERR_INVALID; }
  MVP_HIP(hipSetDevice(ctx->device));
  MVP_HIP(launch_zero_u64((uint64_t *)a->counters, kCntFwdPab + 1, s));
  const auto ev = timer_slot(ctx, MVP_KERNEL_FWD_MARCH);
  if (ev.first) MVP_HIP(hipEventRecord(ev.first, s));
  // the first forward builds the pairs, tile by tile, before marching them
  const bool build = a->pairs_pending.exchange(false);
  hipError_t e = launch_march_fwd(a->view(prims->M), *prims, bg, rgba, aux, a->counters, s, build ? &a->po : nullptr);
  if (e == hipSuccess && build) e = hipEventRecord(a->pairs_done, s);
  if (e != hipSuccess && build) a->pairs_pending.store(true);
  MVP_HIP(e);
  if (ev.second) MVP_HIP(hipEventRecord(ev.second, s));
  return launch_lists(a);
}

// What the backward reads of the structure: the pairs (built here if no
// forward has built them) and the transposed lists (made on the side stream).
static mvp_status bwd_ready(const mvp_accel *a, hipStream_t s) {
  if (a->pairs_pending.exchange(false)) {
    hipError_t e = launch_pairs(a->view(2), a->po, s);
    if (e == hipSuccess) e = hipEventRecord(a->pairs_done, s);
    if (e != hipSuccess) a->pairs_pending.store(true);
    MVP_HIP(e);
  }
  MVP_CHECK(launch_lists(a));
  if (a->lists) MVP_HIP(hipStreamWaitEvent(s, a->lists, 0));
  return MVP_OK;
}

static mvp_status render_bwd(mvp_ctx *ctx, const mvp_accel *a, const mvp_prims *prims, const float *bg,
                             const float *rgba, const mvp_ray_aux *aux, const float *grad_rgba, float *grad_payload,
                             float *grad_pos, float *grad_rot, float *grad_scale, float *grad_bg, hipStream_t s) {
  MVP_CHECK(check_render(ctx, a, prims));
  if (!a->for_backward) { set_error("the structure was built for the forward only"); return MVP_ERR_INVALID; }
  if ((!aux || !grad_rgba) && a->n_slots > 0) { set_error("aux and grad_rgba are required"); return MVP_ERR_INVALID; }
  MVP_HIP(hipSetDevice(ctx->device));
  MVP_CHECK(bwd_ready(a, s));
  Blocks temp{ctx, s};
  uint8_t *scratch = nullptr;
  MVP_CHECK(temp.get(&scratch, bwd_scratch_bytes(a->n_rays())));
  const auto ev = timer_slot(ctx, MVP_KERNEL_BWD_MARCH);
  MVP_HIP(launch_march_bwd(a->view(prims->M), *prims, a->n_items_max, aux, grad_rgba, bg, rgba, scratch, grad_payload,
                           grad_pos, grad_rot, grad_scale, grad_bg, a->counters, s, ev.first, ev.second));
  return MVP_OK;   // the scratch is recycled after the kernels have run
}

mvp_status mvp_render_fwd(mvp_ctx *ctx, const mvp_accel *a, const mvp_prims *prims, float *rgba,
                          mvp_ray_aux *aux, void *stream) {
  return render_fwd(ctx, a, prims, nullptr, rgba, aux, (hipStream_t)stream);
}

mvp_status mvp_render_fwd_bg(mvp_ctx *ctx, const mvp_accel *a, const mvp_prims *prims, const float *background,
                             float *rgba, mvp_ray_aux *aux, void *stream) {
  if (!background && a && a->n_slots > 0) { set_error("background is NULL"); return MVP_ERR_INVALID; }
  return render_fwd(ctx, a, prims, background, rgba, aux, (hipStream_t)stream);
}

mvp_status mvp_render_bwd(mvp_ctx *ctx, const mvp_accel *a, const mvp_prims *prims, const mvp_ray_aux *aux,
                          const float *grad_rgba, float *grad_payload, float *grad_pos, float *grad_rot,
                          float *grad_scale, void *stream) {
  return render_bwd(ctx, a, prims, nullptr, nullptr, aux, grad_rgba, grad_payload, grad_pos, grad_rot, grad_scale,
                    nullptr, (hipStream_t)stream);
}

mvp_status mvp_render_bwd_noalloc(mvp_ctx *ctx, const mvp_accel *a, const mvp_prims *prims,
                                  const mvp_ray_aux *aux, const float *grad_rgba, float *grad_payload,
                                  float *grad_pos, float *grad_rot, float *grad_scale, void *stream) {
  MVP_CHECK(check_render(ctx, a, prims));
  if (!a->for_backward) { set_error("the structure was built for the forward only"); return MVP_ERR_INVALID; }
  if ((!aux || !grad_rgba) && a->n_slots > 0) { set_error("aux and grad_rgba are required"); return MVP_ERR_INVALID; }
  if (a->n_rays() > (size_t)MVP_NOALLOC_MAX_RAYS) {
    set_error("%zu rays exceed the %d of the allocation-free backward (use mvp_render_bwd)", a->n_rays(),
              MVP_NOALLOC_MAX_RAYS);
    return MVP_ERR_INVALID;
  }
  void *ptr = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_scratch[ctx->device] : nullptr;
  if (!ptr) { set_error("the backward scratch array of device %d was not resolved", ctx->device); return MVP_ERR_DEVICE; }
  MVP_HIP(hipSetDevice(ctx->device));
  MVP_CHECK(bwd_ready(a, (hipStream_t)stream));
  const auto ev = timer_slot(ctx, MVP_KERNEL_BWD_MARCH);
  MVP_HIP(launch_march_bwd(a->view(prims->M), *prims, a->n_items_max, aux, grad_rgba, nullptr, nullptr, ptr,
                           grad_payload, grad_pos, grad_rot, grad_scale, nullptr, a->counters, (hipStream_t)stream,
                           ev.first, ev.second));
  return MVP_OK;
}

mvp_status mvp_render_bwd_bg(mvp_ctx *ctx, const mvp_accel *a, const mvp_prims *prims, const float *background,
                             const float *rgba, const mvp_ray_aux *aux, const float *grad_rgba, float *grad_payload,
                             float *grad_pos, float *grad_rot, float *grad_scale, float *grad_background,
                             void *stream) {
  if ((!background || !rgba) && a && a->n_slots > 0) { set_error("background and rgba are required"); return MVP_ERR_INVALID; }
  return render_bwd(ctx, a, prims, background, rgba, aux, grad_rgba, grad_payload, grad_pos, grad_rot, grad_scale,
                    grad_background, (hipStream_t)stream);
}

mvp_status mvp_accel_counts(mvp_ctx *ctx, const mvp_accel *a, uint64_t *ray_samples, uint64_t *prim_samples,
                            void *stream) {
  if (!ctx || !a || a->ctx != ctx || !ray_samples || !prim_samples) { set_error("bad argument"); return MVP_ERR_INVALID; }
  hipStream_t s = (hipStream_t)stream;
  MVP_HIP(hipSetDevice(ctx->device));
  uint64_t h[2] = {0, 0};
  MVP_HIP(hipMemcpyAsync(h, a->counters, sizeof h, hipMemcpyDeviceToHost, s));
  MVP_HIP(hipStreamSynchronize(s));
  *ray_samples = h[0];
  *prim_samples = h[1];
  return MVP_OK;
}

mvp_status mvp_accel_load_counts(mvp_ctx *ctx, const mvp_accel *a, uint64_t *out, void *stream) {
  if (!ctx || !a || a->ctx != ctx || !out) { set_error("bad argument"); return MVP_ERR_INVALID; }
  hipStream_t s = (hipStream_t)stream;
  MVP_HIP(hipSetDevice(ctx->device));
  MVP_HIP(hipMemcpyAsync(out, a->counters, (kCntBwdFlush + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  MVP_HIP(hipStreamSynchronize(s));
  return MVP_OK;
}

mvp_status mvp_debug_hits(mvp_ctx *ctx, const mvp_accel *a, const mvp_prims *prims, int64_t *offsets,
                          int32_t *ids, int64_t ids_cap, int64_t *n_total, void *stream) {
  if (!ctx || !a || a->ctx != ctx || !offsets || !n_total || ids_cap < 0) { set_error("bad argument"); return MVP_ERR_INVALID; }
  MVP_CHECK(check_prims(prims, false));
  if (prims->n_prim != a->N) { set_error("prims does not match the accel"); return MVP_ERR_INVALID; }
  hipStream_t s = (hipStream_t)stream;
  MVP_HIP(hipSetDevice(ctx->device));
  const size_t R = a->n_rays();
  Blocks temp{ctx, s};
  uint32_t *cnt = nullptr;
  uint8_t *scratch = nullptr;
  MVP_CHECK(temp.get(&cnt, R));
  MVP_CHECK(temp.get(&scratch, scan_scratch_bytes(R)));
  AccelView av = a->view(prims->M);
  MVP_HIP(launch_hit_count(av, cnt, s));
  MVP_HIP(launch_scan_u32_u64(cnt, (uint64_t *)offsets, R, scratch, s));
  uint64_t total = 0;
  MVP_CHECK(read_u64((const uint64_t *)offsets + R, &total, s));
  *n_total = (int64_t)total;
  if ((int64_t)total > ids_cap) { set_error("ids_cap %lld < %llu hits", (long long)ids_cap, (unsigned long long)total); return MVP_ERR_OOM; }
  if (total > 0 && !ids) { set_error("ids is NULL"); return MVP_ERR_INVALID; }
  MVP_HIP(launch_hit_ids(av, (const uint64_t *)offsets, ids, s));
  MVP_HIP(hipStreamSynchronize(s));
  return MVP_OK;
}

}  // extern "C"
