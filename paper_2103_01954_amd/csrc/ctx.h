// Host-side runtime objects behind the C ABI: error state, the caching device
// memory arena, contexts and acceleration structures.
#pragma once

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace mvp {

// Record a message for mvp_last_error() on this thread.
void set_error(const char *fmt, ...);
mvp_status status_of(hipError_t e);

// Caching allocator for library-owned device memory.  Blocks released with a
// stream go back to the cache only after the work enqueued on that stream has
// finished (an event is recorded at release time), so memory can be recycled
// across frames without synchronising the device.
class Arena {
 public:
  explicit Arena(int device) : device_(device) {}
  ~Arena();
  mvp_status alloc(size_t bytes, void **out);
  // recycle after the work already enqueued on `s` completes
  mvp_status release_after(const std::vector<void *> &blocks, hipStream_t s);
  void release_now(void *p);
  size_t held_bytes();
  void trim();
  // Events without timing, recycled (creating one costs microseconds of host
  // time on the build's path).  An event handed back may still be pending:
  // recording it again later is fine.
  mvp_status get_event(hipEvent_t *ev);
  void put_event(hipEvent_t ev);

 private:
  struct Pending {
    hipEvent_t ev;
    std::vector<void *> blocks;
  };
  void reap_locked();
  void trim_locked();
  int device_;
  std::mutex mu_;
  std::multimap<size_t, void *> free_;
  std::unordered_map<void *, size_t> size_;
  std::vector<Pending> pending_;
  std::vector<hipEvent_t> events_;
  size_t held_ = 0;
};

// Small pinned host blocks for the build's transfers (cameras up, list sizes
// down), so that they are direct DMA copies rather than copies staged through
// the runtime's own buffers.  Blocks are kPinnedBlock bytes, allocated on
// first use and kept until the context is destroyed.
constexpr size_t kPinnedBlock = 64 * 1024;
class PinnedPool {
 public:
  ~PinnedPool();
  void *get();            // nullptr if pinned memory cannot be allocated
  void put(void *p);
 private:
  std::mutex mu_;
  std::vector<void *> free_, all_;
};

class Server;  // serving scheduler (serve.cpp)

}  // namespace mvp

namespace mvp {
// HIP event pairs around the march kernels (benchmark timing).
struct KernelTimer {
  std::mutex m;
  int cap = 0;
  std::vector<hipEvent_t> ev[2];   // per kernel kind: start/stop of launch i at 2i, 2i+1
  int n[2] = {0, 0};
};
}  // namespace mvp

struct mvp_ctx {
  int device = 0;
  hipStream_t side = nullptr;   // second stream for build work that can overlap the pairs kernel
  mvp::Arena arena;
  mvp::PinnedPool pinned;
  mvp::KernelTimer timer;
  std::atomic<int> live_accels{0};
  mvp::Server *server = nullptr;
  explicit mvp_ctx(int dev) : device(dev), arena(dev) {}
};

struct mvp_accel {
  mvp_ctx *ctx = nullptr;
  int32_t V = 0, W = 0, H = 0, N = 0, tiles_x = 0, tiles_y = 0;
  mvp_march_params params{};
  std::vector<mvp::DevCam> cams_host;
  mvp::DevCam *cams = nullptr;
  float4 *xf = nullptr;
  uint64_t *tile_off = nullptr;
  uint32_t *tile_list = nullptr;
  uint64_t *prim_entry_off = nullptr;
  uint32_t *prim_entries = nullptr;
  uint64_t *item_off = nullptr;
  uint32_t *item_prim = nullptr;
  int64_t n_items_max = 0;             // upper bound on the backward work items
  int32_t item_entries = 64;           // culling-list entries per backward work item
  float4 *ef = nullptr;                // entry frames
  uint64_t *pair_base = nullptr;       // per tile
  uint64_t *ray_seg = nullptr;         // per ray slot
  int2 *ray_nj = nullptr;              // per ray slot
  int4 *pr = nullptr;                  // pair records
  uint64_t *ent_base = nullptr;        // per culling-list entry
  uint32_t *ent_n = nullptr;
  uint32_t *ent_tile = nullptr;
  uint2 *ent_rec = nullptr;            // per-entry pair lists
  uint64_t pair_capacity = 0;
  bool for_backward = true;            // false: no per-entry or transposed lists (forward only)
  bool pairs_in_forward = false;       // the first forward builds the pairs
  hipEvent_t built = nullptr;          // recorded on the build's stream after its kernels
  hipEvent_t lists = nullptr;          // recorded on the side stream once the transposed lists are built
  // The per-ray pairs are built by the first forward (each workgroup builds its
  // tile's pairs, then marches them) or, if a backward comes first, by the
  // pairs kernel; pairs_done is recorded after whichever did it.
  mvp::PairsOut po{};
  mutable std::atomic<bool> pairs_pending{false};
  mutable hipEvent_t pairs_done = nullptr;
  // The transposed lists are built on the context's side stream, launched
  // after the first forward (so that their launches are off the path from
  // the build to the forward) or by the first backward; until then the
  // structure keeps the temporaries they read.
  mutable std::atomic<bool> lists_pending{false};
  std::vector<void *> lists_temps;
  int4 *rect = nullptr;
  uint32_t *prim_cnt = nullptr;
  uint8_t *scan_scratch = nullptr;
  uint32_t *prim_key = nullptr, *prim_bcnt = nullptr;   // the backward's primitive order (launch_prim_order)
  uint64_t *prim_boff = nullptr;
  int64_t n_slots = 0;                 // rays: V*H*W (full frames) or the subset size
  int64_t *ray_pix = nullptr;          // subset only: pixel id of each ray slot
  uint64_t *tile_ray_off = nullptr;    // subset only
  uint32_t *tile_rays = nullptr;       // subset only
  unsigned long long *counters = nullptr;
  int64_t n_tile_pairs = 0, n_ray_pairs = 0, bytes = 0;
  std::vector<void *> blocks;

  mvp::AccelView view(int M) const {
    mvp::AccelView v{};
    v.V = V; v.W = W; v.H = H; v.N = N; v.M = M;
    v.tiles_x = tiles_x; v.tiles_y = tiles_y;
    v.step = params.step; v.eps = params.eps_early; v.t_near = params.t_near;
    v.fade_alpha = params.fade_alpha; v.fade_beta = params.fade_beta; v.combine = params.combine;
    v.cams = cams; v.xf = xf; v.tile_off = tile_off; v.tile_list = tile_list;
    v.prim_entry_off = prim_entry_off; v.prim_entries = prim_entries; v.item_off = item_off; v.item_prim = item_prim;
    v.item_entries = item_entries;
    v.ef = ef; v.pair_base = pair_base; v.ray_seg = ray_seg; v.ray_nj = ray_nj; v.pr = pr;
    v.ent_base = ent_base; v.ent_n = ent_n; v.ent_tile = ent_tile; v.ent_rec = ent_rec;
    v.n_slots = n_slots; v.ray_pix = ray_pix; v.tile_ray_off = tile_ray_off; v.tile_rays = tile_rays;
    return v;
  }
  size_t n_rays() const { return (size_t)n_slots; }
};

namespace mvp {
// Build / check helpers shared with the serving scheduler.
mvp_status check_prims(const mvp_prims *p, bool need_payload);
mvp_status check_camera(const mvp_camera *c);
mvp_status check_params(const mvp_march_params *p);
// Optional admission hook: called before each group of device allocations of a
// build with the number of bytes about to be allocated; a non-OK status aborts
// the build.
struct Admit {
  mvp_status (*fn)(void *user, size_t bytes);
  void *user;
};
// rays == nullptr: every pixel of every view; else n_rays device pixel ids.
// for_backward == false builds only what the forward reads (no per-entry pair
// lists, no transposed lists): the serving loop's structures.
mvp_status build_accel(mvp_ctx *ctx, const mvp_prims *prims, const mvp_camera *cams, int32_t n_views,
                       const mvp_march_params *params, const int64_t *rays, int64_t n_rays,
                       mvp_accel **out, hipStream_t s, const Admit *admit, bool for_backward = true);
mvp_status destroy_accel(mvp_ctx *ctx, mvp_accel *a, hipStream_t s);
// stop the serving scheduler of a context (waits for its work)
void serve_shutdown(mvp_ctx *ctx);
}  // namespace mvp
