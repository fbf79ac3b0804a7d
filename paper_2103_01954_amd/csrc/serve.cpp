// Serving: resident scenes and continuous batching of render requests.
//
// Requests are queued by mvp_submit and admitted in arrival order by a
// scheduler thread, which hands each one to a free slot.  Every slot owns a
// HIP stream and a worker thread that builds the request's culling structure
// and launches its forward march on that stream, so the builds of different
// requests (with their host round trips) and the marches of admitted requests
// all overlap on the device.  Device memory is reserved against the budget in
// three steps as the build sizes the structure (fixed buffers, tile lists,
// ray/primitive pairs).  A build whose next step does not fit waits while
// other requests are running; when none is running, the oldest waiting build
// keeps its memory and younger builds give theirs back and return to the
// front of the queue, so builds cannot wait on each other forever; a request
// that does not fit even alone fails.  While a build waits for memory no new
// build starts (admission stays in arrival order).  A host callback enqueued
// behind each request's forward stamps its completion time.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>

#include "ctx.h"

namespace mvp {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

class Server {
 public:
  Server(mvp_ctx *ctx, size_t budget, int n_slots);
  ~Server();
  mvp_status scene_create(const mvp_prims *src, uint64_t *id);
  mvp_status scene_release(uint64_t id);
  mvp_status submit(const mvp_request *r, uint64_t *ticket);
  mvp_status poll(uint64_t t, int32_t *state, double *ts, double *tstart, double *td);
  mvp_status samples(uint64_t t, uint64_t *ray, uint64_t *prim);
  mvp_status wait(uint64_t t, double timeout_s);
  mvp_status ticket_release(uint64_t t);
  size_t budget() const { return budget_; }

 private:
  struct Scene {
    mvp_prims prims{};
    std::vector<void *> blocks;
    size_t bytes = 0;
    int pending = 0;   // queued or running requests
  };
  struct Ticket {
    mvp_request req{};
    int32_t state = 0;   // 0 queued, 1 running, 2 done, 3 failed
    double t_submit = 0, t_start = 0, t_done = 0;
    uint64_t ray_samples = 0, prim_samples = 0;   // of the forward, once done
  };
  enum : int { kFree = 0, kBuilding = 1, kRunning = 2 };
  struct Slot {
    Server *srv = nullptr;
    hipStream_t stream = nullptr;
    int state = kFree;                 // guarded by mu_
    bool has_work = false;             // a ticket handed over, not yet picked up (mu_)
    bool waiting = false;              // its build waits for memory (mu_)
    std::atomic<bool> finished{false};
    double t_finish = 0;
    uint64_t *h_counts = nullptr;      // pinned: the forward's ray- and prim-sample counts
    uint64_t ray_samples = 0, prim_samples = 0;
    uint64_t ticket = 0;
    mvp_accel *accel = nullptr;
    size_t reserved = 0;
    std::thread worker;
  };
  static void host_done(void *p);
  static mvp_status admit_cb(void *user, size_t bytes);
  void run();
  void work(Slot &slot);
  bool reap_locked();
  void release_slot_locked(Slot &slot);

  mvp_ctx *ctx_;
  size_t budget_;
  size_t used_ = 0;   // resident scenes + reservations of building and running requests
  std::vector<std::unique_ptr<Slot>> slots_;
  std::mutex mu_;
  std::condition_variable cv_;        // scheduler and admission wake-ups
  std::condition_variable work_cv_;   // slot workers
  std::condition_variable done_cv_;   // ticket completions
  std::deque<uint64_t> queue_;
  std::unordered_map<uint64_t, Ticket> tickets_;
  std::unordered_map<uint64_t, Scene> scenes_;
  uint64_t next_ticket_ = 1, next_scene_ = 1;
  bool stop_ = false;
  hipStream_t copy_stream_ = nullptr; // scene uploads
  std::thread thread_;
};

Server::Server(mvp_ctx *ctx, size_t budget, int n_slots) : ctx_(ctx), budget_(budget) {
  (void)hipSetDevice(ctx->device);
  for (int i = 0; i < n_slots; ++i) {
    slots_.emplace_back(new Slot());
    Slot &s = *slots_.back();
    s.srv = this;
    (void)hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    s.h_counts = (uint64_t *)ctx->pinned.get();   // nullptr: the counts are reported as 0
  }
  (void)hipStreamCreateWithFlags(&copy_stream_, hipStreamNonBlocking);
  for (auto &s : slots_) {
    Slot *sp = s.get();
    s->worker = std::thread([this, sp] { work(*sp); });
  }
  thread_ = std::thread([this] { run(); });
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  thread_.join();     // returns once the queue is empty and every slot is free
  work_cv_.notify_all();
  for (auto &s : slots_) s->worker.join();
  (void)hipSetDevice(ctx_->device);
  for (auto &s : slots_) {
    if (s->stream) {
      (void)hipStreamSynchronize(s->stream);
      if (s->accel) destroy_accel(ctx_, s->accel, s->stream);
      (void)hipStreamDestroy(s->stream);
    }
    ctx_->pinned.put(s->h_counts);
  }
  for (auto &kv : scenes_) ctx_->arena.release_after(kv.second.blocks, copy_stream_);
  (void)hipStreamSynchronize(copy_stream_);
  (void)hipStreamDestroy(copy_stream_);
}

void Server::host_done(void *p) {
  Slot *s = (Slot *)p;
  s->t_finish = now_s();
  // the copy of the counts was enqueued before this callback on the same stream
  s->ray_samples = s->h_counts ? s->h_counts[0] : 0;
  s->prim_samples = s->h_counts ? s->h_counts[1] : 0;
  s->finished.store(true);
  Server *srv = s->srv;
  { std::lock_guard<std::mutex> g(srv->mu_); }
  srv->cv_.notify_all();
}

void Server::release_slot_locked(Slot &slot) {
  if (slot.accel) destroy_accel(ctx_, slot.accel, slot.stream);
  slot.accel = nullptr;
  used_ -= slot.reserved;
  slot.reserved = 0;
  slot.state = kFree;
  slot.finished.store(false);
}

// complete finished requests; returns true if any slot was freed
bool Server::reap_locked() {
  bool any = false;
  for (auto &sp : slots_) {
    Slot &s = *sp;
    if (s.state != kRunning || !s.finished.load()) continue;
    auto it = tickets_.find(s.ticket);
    if (it != tickets_.end()) {
      it->second.state = 2;
      it->second.t_done = s.t_finish;
      it->second.ray_samples = s.ray_samples;
      it->second.prim_samples = s.prim_samples;
      auto sc = scenes_.find(it->second.req.scene_id);
      if (sc != scenes_.end()) --sc->second.pending;
    }
    release_slot_locked(s);
    any = true;
  }
  if (any) {
    done_cv_.notify_all();
    cv_.notify_all();
  }
  return any;
}

// Called (from a slot worker, without the lock) before each group of
// allocations of the build in progress.  MVP_ERR_BUSY tells the build to give
// way to an older one (see the top of the file).
mvp_status Server::admit_cb(void *user, size_t bytes) {
  Slot *me = (Slot *)user;
  Server *srv = me->srv;
  std::unique_lock<std::mutex> lk(srv->mu_);
  while (srv->used_ + bytes > srv->budget_) {
    bool running = false, older_waiting = false, younger = false;
    for (auto &sp : srv->slots_) {
      const Slot &s = *sp;
      if (&s == me) continue;
      if (s.state == kRunning) running = true;
      if (s.state == kBuilding && s.ticket < me->ticket && s.waiting) older_waiting = true;
      if (s.state == kBuilding && s.ticket > me->ticket) younger = true;
    }
    if (!running && older_waiting) {
      me->waiting = false;
      set_error("build gives way to an older request waiting for memory");
      return MVP_ERR_BUSY;
    }
    if (!running && !younger && !older_waiting) {
      bool older = false;
      for (auto &sp : srv->slots_)
        if (sp.get() != me && sp->state == kBuilding) older = true;
      if (!older) {
        me->waiting = false;
        set_error("request needs %zu bytes beyond the serving budget (%zu of %zu in use)", bytes, srv->used_,
                  srv->budget_);
        return MVP_ERR_OOM;
      }
    }
    if (!me->waiting) {
      me->waiting = true;
      srv->cv_.notify_all();   // builds of other slots re-check who waits
    }
    if (!srv->reap_locked()) srv->cv_.wait_for(lk, std::chrono::microseconds(200));
  }
  me->waiting = false;
  srv->used_ += bytes;
  me->reserved += bytes;
  return MVP_OK;
}

// Slot worker: build the handed-over request and launch its forward.
void Server::work(Slot &slot) {
  (void)hipSetDevice(ctx_->device);
  std::unique_lock<std::mutex> lk(mu_);
  while (true) {
    work_cv_.wait(lk, [&] { return slot.has_work || stop_; });
    if (!slot.has_work) break;   // stopping
    slot.has_work = false;
    const uint64_t t = slot.ticket;
    Ticket &tk = tickets_[t];
    tk.t_start = now_s();
    const mvp_request req = tk.req;
    const mvp_prims prims = scenes_.find(req.scene_id)->second.prims;
    lk.unlock();
    Admit admit{&Server::admit_cb, &slot};
    mvp_accel *a = nullptr;
    mvp_status st = build_accel(ctx_, &prims, &req.cam, 1, &req.params, nullptr, 0, &a, slot.stream, &admit,
                                 /*for_backward=*/false);
    if (st == MVP_OK) {
      slot.accel = a;
      hipError_t e = launch_zero_u64((uint64_t *)a->counters, kCntFwdPab + 1, slot.stream);
      if (e == hipSuccess)
        e = launch_march_fwd(a->view(prims.M), prims, nullptr, req.rgba_out, nullptr, a->counters, slot.stream,
                             a->pairs_pending.exchange(false) ? &a->po : nullptr);
      if (e == hipSuccess && slot.h_counts)   // counters [0] ray-samples, [1] prim-samples of the forward
        e = hipMemcpyAsync(slot.h_counts, a->counters, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, slot.stream);
      if (e == hipSuccess) e = hipLaunchHostFunc(slot.stream, &Server::host_done, &slot);
      if (e != hipSuccess) {
        set_error("launch failed: %s", hipGetErrorString(e));
        st = MVP_ERR_DEVICE;
      }
    }
    if (st != MVP_OK) (void)hipStreamSynchronize(slot.stream);
    lk.lock();
    slot.waiting = false;
    Ticket &tk2 = tickets_[t];   // the map may have rehashed meanwhile
    if (st == MVP_OK) {
      slot.state = kRunning;
    } else if (st == MVP_ERR_BUSY) {
      // gave way to an older build: back to the front of the queue
      release_slot_locked(slot);
      tk2.state = 0;
      queue_.push_front(t);
    } else {
      release_slot_locked(slot);
      tk2.state = 3;
      tk2.t_done = now_s();
      auto sc = scenes_.find(req.scene_id);
      if (sc != scenes_.end()) --sc->second.pending;
      done_cv_.notify_all();
    }
    cv_.notify_all();
  }
}

void Server::run() {
  (void)hipSetDevice(ctx_->device);
  std::unique_lock<std::mutex> lk(mu_);
  while (true) {
    reap_locked();
    bool busy = false, blocked = false;
    Slot *free_slot = nullptr;
    for (auto &sp : slots_) {
      Slot &s = *sp;
      busy |= s.state != kFree || s.has_work;
      blocked |= s.waiting;
      if (!free_slot && s.state == kFree && !s.has_work) free_slot = &s;
    }
    if (stop_ && !busy && queue_.empty()) break;
    if (free_slot && !blocked && !queue_.empty()) {
      const uint64_t t = queue_.front();
      queue_.pop_front();
      tickets_[t].state = 1;
      free_slot->state = kBuilding;
      free_slot->ticket = t;
      free_slot->reserved = 0;
      free_slot->finished.store(false);
      free_slot->has_work = true;
      work_cv_.notify_all();
      continue;
    }
    cv_.wait_for(lk, std::chrono::milliseconds(5));
  }
}

mvp_status Server::scene_create(const mvp_prims *src, uint64_t *id) {
  mvp_status st = check_prims(src, true);
  if (st != MVP_OK) return st;
  const size_t n = (size_t)src->n_prim, m3 = (size_t)src->M * src->M * src->M;
  const size_t pay_bytes = n * m3 * 4 * (src->payload_dtype == MVP_BF16 ? 2 : 4);
  const size_t bytes = n * 15 * 4 + pay_bytes + 4 * 256;
  {
    std::lock_guard<std::mutex> g(mu_);
    if (used_ + bytes > budget_) {
      set_error("scene of %zu bytes does not fit the serving budget (%zu of %zu in use)", bytes, used_, budget_);
      return MVP_ERR_OOM;
    }
    used_ += bytes;
  }
  Scene sc;
  sc.bytes = bytes;
  sc.prims = *src;
  auto fail = [&](mvp_status s) {
    for (void *b : sc.blocks) ctx_->arena.release_now(b);
    std::lock_guard<std::mutex> g(mu_);
    used_ -= bytes;
    return s;
  };
  void *p[4] = {nullptr, nullptr, nullptr, nullptr};
  const size_t sz[4] = {n * 12 + 16, n * 36 + 16, n * 12 + 16, pay_bytes + 16};
  for (int i = 0; i < 4; ++i) {
    st = ctx_->arena.alloc(sz[i], &p[i]);
    if (st != MVP_OK) return fail(st);
    sc.blocks.push_back(p[i]);
  }
  (void)hipSetDevice(ctx_->device);
  hipStream_t s = copy_stream_;
  const void *srcs[4] = {src->pos, src->rot, src->scale, src->payload};
  for (int i = 0; i < 4; ++i) {
    if (sz[i] > 16 && hipMemcpyAsync(p[i], srcs[i], sz[i] - 16, hipMemcpyDeviceToDevice, s) != hipSuccess) {
      set_error("scene copy failed");
      return fail(MVP_ERR_DEVICE);
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    set_error("scene copy failed");
    return fail(MVP_ERR_DEVICE);
  }
  sc.prims.pos = (const float *)p[0];
  sc.prims.rot = (const float *)p[1];
  sc.prims.scale = (const float *)p[2];
  sc.prims.payload = p[3];
  std::lock_guard<std::mutex> g(mu_);
  *id = next_scene_++;
  scenes_[*id] = std::move(sc);
  return MVP_OK;
}

mvp_status Server::scene_release(uint64_t id) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = scenes_.find(id);
  if (it == scenes_.end()) { set_error("unknown scene %llu", (unsigned long long)id); return MVP_ERR_INVALID; }
  if (it->second.pending) { set_error("scene has %d pending requests", it->second.pending); return MVP_ERR_BUSY; }
  ctx_->arena.release_after(it->second.blocks, copy_stream_);
  used_ -= it->second.bytes;
  scenes_.erase(it);
  return MVP_OK;
}

mvp_status Server::submit(const mvp_request *r, uint64_t *ticket) {
  if (!r || !ticket || !r->rgba_out) { set_error("NULL argument"); return MVP_ERR_INVALID; }
  mvp_status st = check_camera(&r->cam);
  if (st == MVP_OK) st = check_params(&r->params);
  if (st != MVP_OK) return st;
  {
    std::lock_guard<std::mutex> g(mu_);
    auto it = scenes_.find(r->scene_id);
    if (it == scenes_.end()) { set_error("unknown scene %llu", (unsigned long long)r->scene_id); return MVP_ERR_INVALID; }
    ++it->second.pending;
    const uint64_t t = next_ticket_++;
    Ticket tk;
    tk.req = *r;
    tk.t_submit = now_s();
    tickets_[t] = tk;
    queue_.push_back(t);
    *ticket = t;
  }
  cv_.notify_all();
  return MVP_OK;
}

mvp_status Server::poll(uint64_t t, int32_t *state, double *ts, double *tstart, double *td) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = tickets_.find(t);
  if (it == tickets_.end()) { set_error("unknown ticket %llu", (unsigned long long)t); return MVP_ERR_INVALID; }
  if (state) *state = it->second.state;
  if (ts) *ts = it->second.t_submit;
  if (tstart) *tstart = it->second.t_start;
  if (td) *td = it->second.t_done;
  return MVP_OK;
}

mvp_status Server::samples(uint64_t t, uint64_t *ray, uint64_t *prim) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = tickets_.find(t);
  if (it == tickets_.end()) { set_error("unknown ticket %llu", (unsigned long long)t); return MVP_ERR_INVALID; }
  if (it->second.state != 2) { set_error("ticket %llu is not done", (unsigned long long)t); return MVP_ERR_NOT_READY; }
  if (ray) *ray = it->second.ray_samples;
  if (prim) *prim = it->second.prim_samples;
  return MVP_OK;
}

mvp_status Server::wait(uint64_t t, double timeout_s) {
  std::unique_lock<std::mutex> lk(mu_);
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  while (true) {
    auto it = tickets_.find(t);
    if (it == tickets_.end()) { set_error("unknown ticket %llu", (unsigned long long)t); return MVP_ERR_INVALID; }
    if (it->second.state >= 2) return it->second.state == 2 ? MVP_OK : MVP_ERR_DEVICE;
    if (done_cv_.wait_until(lk, deadline) == std::cv_status::timeout) {
      it = tickets_.find(t);
      if (it != tickets_.end() && it->second.state >= 2) return it->second.state == 2 ? MVP_OK : MVP_ERR_DEVICE;
      set_error("timeout");
      return MVP_ERR_NOT_READY;
    }
  }
}

mvp_status Server::ticket_release(uint64_t t) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = tickets_.find(t);
  if (it == tickets_.end()) { set_error("unknown ticket %llu", (unsigned long long)t); return MVP_ERR_INVALID; }
  if (it->second.state < 2) { set_error("ticket still pending"); return MVP_ERR_BUSY; }
  tickets_.erase(it);
  return MVP_OK;
}

static constexpr size_t kDefaultBudget = (size_t)32 << 30;
static constexpr int kDefaultSlots = 4;

static Server *server_of(mvp_ctx *ctx) {
  if (!ctx->server) ctx->server = new Server(ctx, kDefaultBudget, kDefaultSlots);
  return ctx->server;
}

}  // namespace mvp

using namespace mvp;

void mvp::serve_shutdown(mvp_ctx *ctx) {
  delete ctx->server;
  ctx->server = nullptr;
}

extern "C" {

mvp_status mvp_serve_configure(mvp_ctx *ctx, size_t budget_bytes, int32_t n_slots) {
  if (!ctx || n_slots < 1 || n_slots > 32 || budget_bytes == 0) { set_error("bad argument"); return MVP_ERR_INVALID; }
  if (ctx->server) { set_error("serving already configured"); return MVP_ERR_BUSY; }
  ctx->server = new Server(ctx, budget_bytes, n_slots);
  return MVP_OK;
}

mvp_status mvp_scene_create(mvp_ctx *ctx, const mvp_prims *src, uint64_t *scene_id) {
  if (!ctx || !scene_id) { set_error("NULL argument"); return MVP_ERR_INVALID; }
  return server_of(ctx)->scene_create(src, scene_id);
}

mvp_status mvp_scene_release(mvp_ctx *ctx, uint64_t scene_id) {
  if (!ctx || !ctx->server) { set_error("no serving state"); return MVP_ERR_INVALID; }
  return ctx->server->scene_release(scene_id);
}

mvp_status mvp_submit(mvp_ctx *ctx, const mvp_request *req, uint64_t *ticket) {
  if (!ctx || !ctx->server) { set_error("no resident scene"); return MVP_ERR_INVALID; }
  return ctx->server->submit(req, ticket);
}

mvp_status mvp_poll(mvp_ctx *ctx, uint64_t ticket, int32_t *state, double *t_submit, double *t_done) {
  if (!ctx || !ctx->server) { set_error("no serving state"); return MVP_ERR_INVALID; }
  return ctx->server->poll(ticket, state, t_submit, nullptr, t_done);
}

mvp_status mvp_ticket_times(mvp_ctx *ctx, uint64_t ticket, double *t_submit, double *t_start, double *t_done) {
  if (!ctx || !ctx->server) { set_error("no serving state"); return MVP_ERR_INVALID; }
  return ctx->server->poll(ticket, nullptr, t_submit, t_start, t_done);
}

mvp_status mvp_ticket_samples(mvp_ctx *ctx, uint64_t ticket, uint64_t *ray_samples, uint64_t *prim_samples) {
  if (!ctx || !ctx->server) { set_error("no serving state"); return MVP_ERR_INVALID; }
  return ctx->server->samples(ticket, ray_samples, prim_samples);
}

double mvp_clock(void) { return now_s(); }

mvp_status mvp_wait(mvp_ctx *ctx, uint64_t ticket, double timeout_s) {
  if (!ctx || !ctx->server) { set_error("no serving state"); return MVP_ERR_INVALID; }
  return ctx->server->wait(ticket, timeout_s);
}

mvp_status mvp_ticket_release(mvp_ctx *ctx, uint64_t ticket) {
  if (!ctx || !ctx->server) { set_error("no serving state"); return MVP_ERR_INVALID; }
  return ctx->server->ticket_release(ticket);
}

}  // extern "C"
