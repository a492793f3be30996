// Continuous-batching server: requests wait in a FIFO queue, are admitted by
// device-memory footprint into a first-fit arena, and are packed into batches
// (one launch of the fused kernel over a (request, pixel block) tile list and
// one convolution launch per batch).  Several batches are in flight on
// separate streams; new requests keep being admitted while others run.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "jt_host.hpp"
#include "jt_kernels.hpp"

using namespace jt;
using Clock = std::chrono::steady_clock;

namespace {

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

// First-fit allocator over [0, size).
struct Arena {
  size_t size = 0, in_use = 0, peak = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t n) {
    size = n;
    free_.clear();
    if (n) free_[0] = n;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t o = it->first, rest = it->second - n;
      free_.erase(it);
      if (rest) free_[o + n] = rest;
      *off = o;
      in_use += n;
      peak = std::max(peak, in_use);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    in_use -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Req {
  uint64_t ticket = 0;
  GridC g;
  MacroC mc;
  LightC src, ll;
  const SubRec* table = nullptr;
  int nsub = 0, nloop = 0;
  const float* psf = nullptr;
  int k = 0;
  float* out = nullptr;
  size_t footprint = 0;
  double pairs = 0;
  int state = JT_TICKET_QUEUED;
  Clock::time_point t_submit, t_done;
};

struct Batch {
  std::vector<Req*> reqs;
  size_t off = 0, bytes = 0;
  double pairs = 0;
  int stream = 0;
  std::atomic<bool> done{false};
  bool failed = false;
  Clock::time_point t_done;
  Clock::time_point sim_done;
  jt_server* srv = nullptr;
};

// Conservative device bytes of one request inside a batch block.
size_t request_footprint(const GridC& g, int k) {
  const long npix = (long)g.nx * g.ny;
  const long ppb_min = std::max(1, 64 / g.s2);
  const long tiles = (npix + ppb_min - 1) / ppb_min;
  const long ctiles = k ? (long)conv_tiles_x(g.nx) * conv_tiles_y(g.ny) : 0;
  return a256(sizeof(ImageDesc)) + a256(sizeof(ConvDesc)) + a256(8 * tiles) + a256(16 * ctiles) +
         (k ? a256(4 * npix) : 0);
}

double request_pairs(const GridC& g, int nloop) {
  return (double)g.nx * g.ny * g.s2 * (double)(nloop + 16);
}

}  // namespace

struct jt_server {
  jt_ctx* ctx = nullptr;  // null: simulated device
  jt_server_cfg cfg{};
  double sim_rate = 0;
  std::mutex mu;
  std::condition_variable cv;       // wakes the scheduling thread
  std::condition_variable done_cv;  // wakes waiters
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> tickets;
  std::deque<std::unique_ptr<Batch>> inflight;
  Arena arena;
  char* arena_dev = nullptr;
  std::vector<hipStream_t> streams;
  int next_stream = 0;
  uint64_t next_ticket = 1;
  jt_server_stats st{};
  Clock::time_point sim_free;
  bool stop = false;
  std::thread thread;

  void run();
  void launch_ready();
  void complete_finished();
  jt_status launch_hip(Batch& b);
};

namespace {

// Runs on a HIP runtime thread when the stream reaches the end of the batch.
// The batch may be freed by the scheduler as soon as `done` is set, so it is
// not touched afterwards; the server outlives the callback because
// jt_server_destroy synchronises every stream before freeing it.
void on_batch_done(void* p) {
  Batch* b = (Batch*)p;
  jt_server* srv = b->srv;
  b->t_done = Clock::now();
  b->done.store(true, std::memory_order_release);
  srv->cv.notify_all();
}

}  // namespace

jt_status jt_server::launch_hip(Batch& b) {
  JT_TRY(ctx_enter(ctx));
  hipStream_t s = streams[b.stream];
  // one split for the whole tile list
  long subpix = 0;
  int max_nloop = 0, max_s2 = 1, kmax = 0;
  for (Req* r : b.reqs) {
    subpix += (long)r->g.nx * r->g.ny * r->g.s2;
    max_nloop = std::max(max_nloop, r->nloop);
    max_s2 = std::max(max_s2, r->g.s2);
    kmax = std::max(kmax, r->k);
  }
  const int split = pick_split(subpix, max_s2, max_nloop);
  // longest tiles first
  std::vector<Req*> order(b.reqs);
  std::stable_sort(order.begin(), order.end(), [](Req* x, Req* y) { return x->nloop > y->nloop; });
  const size_t n = order.size();
  std::vector<ImageDesc> descs(n);
  std::vector<ConvDesc> cdescs;
  std::vector<int2> tiles;
  std::vector<int4> ctiles;
  // block layout: descs | conv descs | tiles | conv tiles | images
  size_t img_total = 0;
  for (Req* r : order) img_total += r->k ? a256(4 * (size_t)r->g.nx * r->g.ny) : 0;
  size_t ntiles = 0, nctiles = 0, ncon = 0;
  for (Req* r : order) {
    const int ppb = (256 / split) / r->g.s2;
    ntiles += ((long)r->g.nx * r->g.ny + ppb - 1) / ppb;
    if (r->k) {
      nctiles += (size_t)conv_tiles_x(r->g.nx) * conv_tiles_y(r->g.ny);
      ++ncon;
    }
  }
  const size_t o_cd = a256(sizeof(ImageDesc) * n);
  const size_t o_t = o_cd + a256(sizeof(ConvDesc) * ncon);
  const size_t o_ct = o_t + a256(sizeof(int2) * ntiles);
  const size_t o_img = o_ct + a256(sizeof(int4) * nctiles);
  if (o_img + img_total > b.bytes) return fail(JT_EDEVICE, "server: batch block too small (internal)");
  char* base = arena_dev + b.off;
  size_t img_off = o_img;
  for (size_t i = 0; i < n; ++i) {
    Req* r = order[i];
    ImageDesc& D = descs[i];
    std::memset(&D, 0, sizeof(D));
    D.g = r->g;
    D.g.ppb = (256 / split) / r->g.s2;
    D.mc = r->mc;
    D.src = r->src;
    D.ll = r->ll;
    D.sub = r->table ? r->table : ctx_empty_table(ctx);
    D.nloop = r->nloop;
    const int bpi = (r->g.nx * r->g.ny + D.g.ppb - 1) / D.g.ppb;
    for (int blk = 0; blk < bpi; ++blk) tiles.push_back(make_int2((int)i, blk));
    if (r->k) {
      D.img = (float*)(base + img_off);
      img_off += a256(4 * (size_t)r->g.nx * r->g.ny);
      const int ci = (int)cdescs.size();
      cdescs.push_back(ConvDesc{D.img, r->out, r->psf, r->g.nx, r->g.ny, r->k, 0});
      for (int ty = 0; ty < conv_tiles_y(r->g.ny); ++ty)
        for (int tx = 0; tx < conv_tiles_x(r->g.nx); ++tx) ctiles.push_back(make_int4(ci, tx, ty, 0));
    } else {
      D.img = r->out;
    }
  }
  std::vector<char> host(o_img, 0);
  std::memcpy(host.data(), descs.data(), sizeof(ImageDesc) * n);
  if (ncon) std::memcpy(host.data() + o_cd, cdescs.data(), sizeof(ConvDesc) * ncon);
  std::memcpy(host.data() + o_t, tiles.data(), sizeof(int2) * ntiles);
  if (nctiles) std::memcpy(host.data() + o_ct, ctiles.data(), sizeof(int4) * nctiles);
  JT_TRY(ctx_upload(ctx, s, base, host.data(), o_img));
  JT_TRY(timed_launch(ctx, JT_K_SIM, s, [&] {
    return launch_simulate_desc(split, (const ImageDesc*)base, (const int2*)(base + o_t), (int)ntiles, 0, s);
  }, "server simulate"));
  if (ncon)
    JT_TRY(timed_launch(ctx, JT_K_CONV, s, [&] {
      return launch_conv_desc((const ConvDesc*)(base + o_cd), (const int4*)(base + o_ct), (int)nctiles, kmax, s);
    }, "server convolve"));
  return check_hip(hipLaunchHostFunc(s, on_batch_done, &b), "hipLaunchHostFunc");
}

// Called with mu held.
void jt_server::complete_finished() {
  const auto now = Clock::now();
  bool any = false;
  for (auto it = inflight.begin(); it != inflight.end();) {
    Batch& b = **it;
    const bool fin = ctx ? b.done.load(std::memory_order_acquire) : (now >= b.sim_done);
    if (!fin) {
      ++it;
      continue;
    }
    const auto t = ctx ? b.t_done : b.sim_done;
    for (Req* r : b.reqs) {
      r->state = b.failed ? JT_TICKET_FAILED : JT_TICKET_DONE;
      r->t_done = t;
      if (b.failed) ++st.failed; else ++st.completed;
    }
    arena.release(b.off, b.bytes);
    it = inflight.erase(it);
    any = true;
  }
  if (any) done_cv.notify_all();
}

// Called with mu held: forms batches from the queue head while slots and
// arena space allow.
void jt_server::launch_ready() {
  while (!stop && (int)inflight.size() < cfg.max_inflight_batches && !queue.empty()) {
    std::vector<Req*> pick;
    double pairs = 0;
    size_t bytes = 0;
    for (Req* r : queue) {
      if ((int)pick.size() >= cfg.max_batch_images) break;
      if (!pick.empty() && pairs + r->pairs > cfg.max_batch_pairs) break;
      pick.push_back(r);
      pairs += r->pairs;
      bytes += r->footprint;
    }
    size_t off = 0;
    while (!pick.empty() && !arena.alloc(bytes, &off)) {
      bytes -= pick.back()->footprint;
      pairs -= pick.back()->pairs;
      pick.pop_back();
    }
    if (pick.empty()) return;  // the head does not fit yet: wait for completions
    for (size_t i = 0; i < pick.size(); ++i) queue.pop_front();
    auto bp = std::make_unique<Batch>();
    Batch& b = *bp;
    b.reqs = pick;
    b.off = off;
    b.bytes = bytes;
    b.pairs = pairs;
    b.srv = this;
    b.stream = next_stream;
    next_stream = (next_stream + 1) % std::max(1, (int)streams.size());
    for (Req* r : pick) r->state = JT_TICKET_RUNNING;
    ++st.batches;
    if (ctx) {
      if (launch_hip(b) != JT_OK) {
        // no completion callback was queued: let whatever was launched finish
        // before the batch's arena block can be reused
        (void)hipStreamSynchronize(streams[b.stream]);
        b.failed = true;
        b.t_done = Clock::now();
        b.done.store(true);
      }
    } else {
      const auto now = Clock::now();
      const double dur = pairs / sim_rate + 20e-6;
      const auto start = std::max(now, sim_free);
      b.sim_done = start + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(dur));
      sim_free = b.sim_done;
      st.device_seconds += dur;
    }
    inflight.push_back(std::move(bp));
  }
}

void jt_server::run() {
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    complete_finished();
    launch_ready();
    if (stop && inflight.empty()) break;
    if (inflight.empty()) {
      cv.wait(lk, [&] { return stop || !queue.empty(); });
    } else if (!ctx) {
      auto next = inflight.front()->sim_done;
      for (auto& b : inflight) next = std::min(next, b->sim_done);
      cv.wait_until(lk, next);
    } else {
      // woken by batch callbacks and submissions; the timeout covers a
      // notification that lands between the check and the wait
      cv.wait_for(lk, std::chrono::microseconds(500));
    }
  }
}

namespace {

jt_status check_cfg(const jt_server_cfg* c) {
  if (!c) return fail(JT_EINVAL, "server: null config");
  if (c->hbm_budget_bytes == 0 || c->max_batch_images < 1 || !(c->max_batch_pairs > 0) ||
      c->max_inflight_batches < 1 || c->n_streams < 1 || c->n_streams > 16)
    return fail(JT_EINVAL, "server: bad config");
  return JT_OK;
}

jt_status start(jt_server* s) {
  s->arena.init(s->cfg.hbm_budget_bytes);
  s->st.arena_bytes = s->cfg.hbm_budget_bytes;
  s->sim_free = Clock::now();
  s->thread = std::thread([s] { s->run(); });
  return JT_OK;
}

}  // namespace

extern "C" jt_status jt_server_create(jt_ctx* ctx, const jt_server_cfg* cfg, jt_server** out) {
  JT_TRY(ctx_enter(ctx));
  JT_TRY(check_cfg(cfg));
  if (!out) return fail(JT_EINVAL, "server: null output");
  auto s = std::make_unique<jt_server>();
  s->ctx = ctx;
  s->cfg = *cfg;
  JT_TRY(check_hip(hipMalloc((void**)&s->arena_dev, cfg->hbm_budget_bytes), "hipMalloc(server arena)"));
  for (int i = 0; i < cfg->n_streams; ++i) {
    hipStream_t st = nullptr;
    jt_status e = check_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
    if (e != JT_OK) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      (void)hipFree(s->arena_dev);
      return e;
    }
    s->streams.push_back(st);
  }
  JT_TRY(start(s.get()));
  *out = s.release();
  return JT_OK;
}

extern "C" jt_status jt_server_create_simulated(const jt_server_cfg* cfg, double pairs_per_second, jt_server** out) {
  JT_TRY(check_cfg(cfg));
  if (!out || !(pairs_per_second > 0)) return fail(JT_EINVAL, "server: bad simulated rate or output");
  auto s = std::make_unique<jt_server>();
  s->cfg = *cfg;
  s->sim_rate = pairs_per_second;
  JT_TRY(start(s.get()));
  *out = s.release();
  return JT_OK;
}

extern "C" jt_status jt_server_submit(jt_server* srv, const jt_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket) return fail(JT_EINVAL, "server submit: null argument");
  auto r = std::make_unique<Req>();
  JT_TRY(make_grid(&req->grid, r->g));
  jt_lens lens;
  std::memset(&lens, 0, sizeof(lens));
  lens.has_sie = req->has_sie;
  lens.sie = req->sie;
  lens.has_shear = req->has_shear;
  lens.shear = req->shear;
  JT_TRY(make_macro(&lens, r->mc));
  JT_TRY(make_light(&req->src, r->src, "source"));
  JT_TRY(make_light(&req->lens_light, r->ll, "lens light"));
  if (!req->out) return fail(JT_EINVAL, "server submit: null output");
  r->out = req->out;
  if (srv->ctx) {
    if (req->subhalo_handle) JT_TRY(ctx_subhalo_handle(srv->ctx, req->subhalo_handle, &r->table, &r->nsub));
    if (req->psf_handle) JT_TRY(jt_psf_pointer(srv->ctx, req->psf_handle, &r->psf, &r->k));
  } else {
    r->nsub = (int)req->subhalo_handle;
    r->k = (int)req->psf_handle;
    if (r->k && r->k % 2 == 0) return fail(JT_EINVAL, "server submit: even PSF side");
  }
  if (r->k > JT_MAX_PSF) return fail(JT_EUNSUPPORTED, "server submit: PSF side %d > %d", r->k, JT_MAX_PSF);
  r->nloop = subhalo_loop_count(r->nsub);
  r->footprint = request_footprint(r->g, r->k);
  r->pairs = request_pairs(r->g, r->nloop);
  if (r->footprint > srv->arena.size)
    return fail(JT_ENOMEM, "server submit: request needs %zu bytes, arena holds %zu", r->footprint, srv->arena.size);
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return fail(JT_ECANCELLED, "server submit: server is stopping");
  r->ticket = srv->next_ticket++;
  r->t_submit = Clock::now();
  *ticket = r->ticket;
  srv->queue.push_back(r.get());
  srv->tickets[r->ticket] = std::move(r);
  ++srv->st.submitted;
  srv->cv.notify_all();
  return JT_OK;
}

extern "C" jt_status jt_server_poll(jt_server* srv, uint64_t ticket, int* state) {
  if (!srv || !state) return fail(JT_EINVAL, "server poll: null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return fail(JT_EINVAL, "server poll: unknown ticket %llu", (unsigned long long)ticket);
  *state = it->second->state;
  return JT_OK;
}

extern "C" jt_status jt_server_wait(jt_server* srv, uint64_t ticket, double timeout_s, double* latency_s) {
  if (!srv) return fail(JT_EINVAL, "server wait: null server");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return fail(JT_EINVAL, "server wait: unknown ticket %llu", (unsigned long long)ticket);
  Req* r = it->second.get();
  auto final_state = [&] { return r->state >= JT_TICKET_DONE; };
  if (timeout_s < 0) {
    srv->done_cv.wait(lk, final_state);
  } else if (!srv->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), final_state)) {
    return fail(JT_EBUSY, "server wait: ticket %llu still pending", (unsigned long long)ticket);
  }
  const int state = r->state;
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  srv->tickets.erase(it);
  if (state == JT_TICKET_CANCELLED) return fail(JT_ECANCELLED, "ticket %llu cancelled", (unsigned long long)ticket);
  if (state == JT_TICKET_FAILED) return fail(JT_EDEVICE, "ticket %llu failed on the device", (unsigned long long)ticket);
  return JT_OK;
}

extern "C" jt_status jt_server_cancel(jt_server* srv, uint64_t ticket) {
  if (!srv) return fail(JT_EINVAL, "server cancel: null server");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return fail(JT_EINVAL, "server cancel: unknown ticket %llu", (unsigned long long)ticket);
  Req* r = it->second.get();
  if (r->state == JT_TICKET_RUNNING) return fail(JT_EBUSY, "server cancel: ticket is running");
  if (r->state != JT_TICKET_QUEUED) return fail(JT_EINVAL, "server cancel: ticket already finished");
  srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), r));
  r->state = JT_TICKET_CANCELLED;
  r->t_done = Clock::now();
  ++srv->st.cancelled;
  srv->done_cv.notify_all();
  srv->cv.notify_all();
  return JT_OK;
}

extern "C" jt_status jt_server_get_stats(jt_server* srv, jt_server_stats* stats) {
  if (!srv || !stats) return fail(JT_EINVAL, "server stats: null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  *stats = srv->st;
  stats->arena_in_use = srv->arena.in_use;
  stats->arena_peak = srv->arena.peak;
  return JT_OK;
}

extern "C" void jt_server_destroy(jt_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    for (Req* r : srv->queue) {
      r->state = JT_TICKET_CANCELLED;
      r->t_done = Clock::now();
      ++srv->st.cancelled;
    }
    srv->queue.clear();
    srv->cv.notify_all();
    srv->done_cv.notify_all();
  }
  if (srv->thread.joinable()) srv->thread.join();
  if (srv->ctx) {
    (void)hipSetDevice(srv->ctx->device);
    for (auto s : srv->streams) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
    if (srv->arena_dev) (void)hipFree(srv->arena_dev);
  }
  delete srv;
}
