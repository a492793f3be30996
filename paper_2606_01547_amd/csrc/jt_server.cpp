// Continuous-batching server: requests wait in a FIFO queue, are admitted by
// device-memory footprint into a first-fit arena, and are packed into batches
// (one launch of the fused kernel over a (request, pixel block) tile list and
// one convolution launch per batch).  Several batches are in flight on
// separate streams; new requests keep being admitted while others run.
//
// A request whose work exceeds the per-batch cap and that has more than two
// minimum chunks of pixel blocks runs in chunks instead (a smaller one over
// the cap forms a batch of its own): each chunk is a launch of at least
// kChunkMinBlocks blocks (about what the chip holds at once in 256-thread
// blocks, so a chunk is dispatched almost as soon as it is queued and the
// batches of other streams get in between) and otherwise about the cap, all on one stream
// with two chunks queued at a time, and the convolution follows as a launch of
// its own once every chunk has completed.  The hardware dispatches every
// workgroup of a queued kernel before it turns to another queue, but switches
// at kernel boundaries of one queue: batches of the requests behind a large
// one therefore start at the next chunk boundary instead of after the whole
// image.  While whole requests are queued or running, chunks shrink to 768
// blocks, three eighths of a round of wave slots, one at a time
// (kChunkSharedBlocks), so the small batches always find most of the chip
// open.
//
// A batch that fails on the device (its completion event reports an error,
// or its launch fails) puts the server in a failed state: a device fault can
// leave any memory the device touched untrustworthy, so every request in
// flight or queued then fails (JT_EDEVICE), chunked requests stop launching
// chunks, and new submissions are refused.  Destroying the server cancels the
// queue and the chunked requests in progress (their chunks on the device are
// waited for, then their tickets read CANCELLED).
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
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "jt_host.hpp"
#include "jt_kernels.hpp"

using namespace jt;
using Clock = std::chrono::steady_clock;

namespace {

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

// Smallest chunk of a chunked request: 2048 blocks of 4 waves, one full round
// of wave slots on 256 CUs at 8 waves per SIMD.
constexpr int kChunkMinBlocks = 2048;
// While whole requests wait in the queue or run, a chunked request takes
// chunks of at most this many blocks (three eighths of a round of wave
// slots), one at a time, so that most of the chip stays open to the small
// batches: the blocks of a large image each run for milliseconds, and the
// hardware hands a freed slot to whichever queue's kernel is next, so a
// full-round chunk would hold the whole chip for one block lifetime per chunk.
// Measured: 512 blocks starve the large images at full load, 1024 leave the
// small requests a longer tail at half load.  With nothing else to run the
// request goes back to full chunks, two queued.
constexpr int kChunkSharedBlocks = 768;

// A truncated-NFW pair costs about 1.55 NFW pairs of GPU time (headline image:
// 2.08 ms against 1.33 ms); the work caps count it so.
constexpr double kTnfwPairCost = 1.55;

// Pinned host memory for the batches' descriptor uploads.  Each batch keeps its
// own slice until it completes, so forming a batch never waits for a copy
// queued behind earlier work on the same stream.
constexpr size_t kStagingBytes = 64u << 20;

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
  const void* table = nullptr;     // SubRec records, or TRec when tnfw
  bool tnfw = false;
  int nsub = 0, nloop = 0;
  const float* psf = nullptr;
  int k = 0;
  float* out = nullptr;
  size_t footprint = 0;
  double pairs = 0;
  int state = JT_TICKET_QUEUED;
  Clock::time_point t_submit, t_launch, t_done;
  // chunked (large) requests
  bool chunked = false;
  int split = 1, ppb = 1;          // fixed block shape of all its chunks
  int blocks = 0, next_block = 0;  // pixel blocks in all, first not yet launched
  int chunk_blocks = 1;            // blocks per chunk
  int chunks_inflight = 0;
  bool conv_launched = false;
  bool failed = false;
  int stream = 0;                  // every chunk runs on this stream
  size_t img_off = 0, img_bytes = 0;  // arena block of its unconvolved image
};

struct Batch {
  size_t st_off = 0, st_bytes = 0; // slice of the pinned staging arena
  std::vector<Req*> reqs;          // whole requests, or the one chunked request
  bool chunk = false;              // a chunk of reqs[0]: blocks [blk0, blk1)
  int blk0 = 0, blk1 = 0;
  bool conv = false;               // the convolution of chunked request reqs[0]
  size_t off = 0, bytes = 0;
  double pairs = 0;
  int stream = 0;
  hipEvent_t ev = nullptr;         // recorded after the batch's last kernel
  bool done = false;               // set when the launch failed
  bool failed = false;
  Clock::time_point t_done;
  Clock::time_point sim_done;      // simulated device: completion time once known
  double sim_left = 0;             // simulated device: seconds of work left alone on the device
  bool sim_fin = false;
  jt_server* srv = nullptr;
};

// Conservative device bytes of one request inside a batch block.
size_t request_footprint(const GridC& g, int k) {
  const long npix = (long)g.nx * g.ny;
  const long ppb_min = std::max(1, 64 / g.s2);
  const long tiles = (npix + ppb_min - 1) / ppb_min;
  const long ctiles = k ? (long)conv_tiles_x(g.nx, conv_shape(g.nx, g.ny, k)) * conv_tiles_y(g.ny) : 0;
  return a256(sizeof(ImageDesc)) + a256(sizeof(ConvDesc)) + a256(8 * tiles) + a256(16 * ctiles) +
         (k ? a256(4 * npix) : 0);
}

double request_pairs(const GridC& g, int nloop) {
  return (double)g.nx * g.ny * g.s2 * (double)(nloop + 16);
}

// Host-side header of a request inside a batch: its footprint without the
// unconvolved image (descriptors and tile lists, uploaded through staging).
size_t header_bytes(const Req* r) {
  return r->footprint - (r->k ? a256(4 * (size_t)r->g.nx * r->g.ny) : 0);
}

// Device bytes of one chunk batch (descriptor and tile list) and of the
// convolution batch of a chunked request (descriptor and tiles).
size_t chunk_footprint(int chunk_blocks) {
  return a256(sizeof(ImageDesc)) + a256(8 * (size_t)chunk_blocks);
}

size_t conv_footprint(const GridC& g, int k) {
  return a256(sizeof(ConvDesc)) + a256(16 * (size_t)conv_tiles_x(g.nx, conv_shape(g.nx, g.ny, k)) * conv_tiles_y(g.ny));
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
  std::vector<Req*> active;         // chunked requests in progress
  size_t rr = 0;                    // round robin over them
  int chunk_batches = 0;            // their chunk and convolution batches in flight
  Arena stage;                      // offsets into stage_host
  char* stage_host = nullptr;
  std::vector<hipEvent_t> events;   // completion events not in use
  uint64_t next_ticket = 1;
  jt_server_stats st{};
  Clock::time_point sim_last;       // simulated device: last advance
  bool stop = false;
  int waiters = 0;                  // threads inside jt_server_wait
  bool broken = false;              // a batch failed on the device: no more work
  std::string broken_why;
  uint64_t sim_fail_batch = 0;      // simulated device: launch index (1-based) that fails
  std::thread thread;

  void run();
  void sim_advance(Clock::time_point now);
  double sim_next_completion();
  void launch_ready();
  void complete_finished();
  void finish_request(Req* r, bool failed, Clock::time_point t);
  void cancel_request(Req* r, Clock::time_point t);
  void fail_all(const char* why);
  void retire_stopped_chunked(Clock::time_point t);
  bool launch_batch(std::unique_ptr<Batch> bp);
  jt_status launch_hip(Batch& b);
  jt_status launch_chunk_hip(Batch& b);
  jt_status launch_conv_hip(Batch& b);
  jt_status upload(Batch& b, const char* host, size_t bytes, void* dev, hipStream_t s);
  int small_stream();
};

// Copies the batch's header bytes through its staging slice.
jt_status jt_server::upload(Batch& b, const char* host, size_t bytes, void* dev, hipStream_t s) {
  if (bytes > b.st_bytes) return fail(JT_EDEVICE, "server: staging slice too small (internal)");
  std::memcpy(stage_host + b.st_off, host, bytes);
  return check_hip(hipMemcpyAsync(dev, stage_host + b.st_off, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync(batch)");
}

jt_status jt_server::launch_hip(Batch& b) {
  JT_TRY(ctx_enter(ctx));
  hipStream_t s = streams[b.stream];
  // one split for the whole tile list
  long subpix = 0;
  int max_nloop = 0, max_s2 = 1;
  for (Req* r : b.reqs) {
    subpix += (long)r->g.nx * r->g.ny * r->g.s2;
    max_nloop = std::max(max_nloop, r->nloop);
    max_s2 = std::max(max_s2, r->g.s2);
  }
  const int split = pick_split(subpix, max_s2, max_nloop);
  // longest tiles first
  std::vector<Req*> order(b.reqs);
  std::stable_sort(order.begin(), order.end(), [](Req* x, Req* y) { return x->nloop > y->nloop; });
  const size_t n = order.size();
  std::vector<ImageDesc> descs(n);
  std::vector<ConvDesc> cdescs;
  std::vector<int2> tiles;
  // convolution tiles by the shape kind each request alone would take (one
  // launch per kind), and the LDS each launch needs
  std::vector<int4> ctiles[3];
  size_t clds[3] = {0, 0, 0};
  // block layout: descs | conv descs | tiles | conv tiles | images
  size_t img_total = 0;
  for (Req* r : order) img_total += r->k ? a256(4 * (size_t)r->g.nx * r->g.ny) : 0;
  size_t ntiles = 0, nctiles = 0, ncon = 0;
  bool extra = false;
  for (Req* r : order) {
    const int ppb = split_lanes(split) / r->g.s2;
    ntiles += ((long)r->g.nx * r->g.ny + ppb - 1) / ppb;
    extra = extra || light_has_extra(r->src) || light_has_extra(r->ll);
    if (r->k) {
      nctiles += (size_t)conv_tiles_x(r->g.nx, conv_shape(r->g.nx, r->g.ny, r->k)) * conv_tiles_y(r->g.ny);
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
    D.g.ppb = split_lanes(split) / r->g.s2;
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
      // the shape the request alone would get, so its image does not depend
      // on what else the batch holds
      const ConvShape sh = conv_shape(r->g.nx, r->g.ny, r->k);
      cdescs.push_back(ConvDesc{D.img, r->out, r->psf, r->g.nx, r->g.ny, r->k, sh.t});
      const int kind = conv_shape_kind(sh);
      clds[kind] = std::max(clds[kind], conv_lds_bytes(r->k, sh));
      for (int ty = 0; ty < conv_tiles_y(r->g.ny); ++ty)
        for (int tx = 0; tx < conv_tiles_x(r->g.nx, sh); ++tx) ctiles[kind].push_back(make_int4(ci, tx, ty, 0));
    } else {
      D.img = r->out;
    }
  }
  std::vector<char> host(o_img, 0);
  std::memcpy(host.data(), descs.data(), sizeof(ImageDesc) * n);
  if (ncon) std::memcpy(host.data() + o_cd, cdescs.data(), sizeof(ConvDesc) * ncon);
  std::memcpy(host.data() + o_t, tiles.data(), sizeof(int2) * ntiles);
  size_t ct_off[3], nct_all = 0;
  for (int kind = 0; kind < 3; ++kind) {
    ct_off[kind] = nct_all;
    if (!ctiles[kind].empty())
      std::memcpy(host.data() + o_ct + sizeof(int4) * nct_all, ctiles[kind].data(), sizeof(int4) * ctiles[kind].size());
    nct_all += ctiles[kind].size();
  }
  JT_TRY(upload(b, host.data(), o_img, base, s));
  JT_TRY(timed_launch(ctx, JT_K_SIM, s, [&] {
    return launch_simulate_desc(split, order[0]->tnfw, extra, false, (const ImageDesc*)base, (const int2*)(base + o_t), (int)ntiles,
                                0, s);
  }, "server simulate"));
  for (int kind = 0; kind < 3; ++kind) {
    if (ctiles[kind].empty()) continue;
    const int4* tl = (const int4*)(base + o_ct) + ct_off[kind];
    JT_TRY(timed_launch(ctx, JT_K_CONV, s, [&] {
      return launch_conv_desc(kind, (const ConvDesc*)(base + o_cd), tl, (int)ctiles[kind].size(), clds[kind], s);
    }, "server convolve"));
  }
  return check_hip(hipEventRecord(b.ev, s), "hipEventRecord(batch)");
}

jt_status jt_server::launch_chunk_hip(Batch& b) {
  JT_TRY(ctx_enter(ctx));
  Req* r = b.reqs[0];
  hipStream_t s = streams[b.stream];
  const int nt = b.blk1 - b.blk0;
  const size_t o_t = a256(sizeof(ImageDesc));
  const size_t end = o_t + a256(sizeof(int2) * (size_t)nt);
  if (end > b.bytes) return fail(JT_EDEVICE, "server: chunk block too small (internal)");
  char* base = arena_dev + b.off;
  std::vector<char> host(end, 0);
  ImageDesc& D = *(ImageDesc*)host.data();
  D.g = r->g;
  D.g.ppb = r->ppb;
  D.mc = r->mc;
  D.src = r->src;
  D.ll = r->ll;
  D.sub = r->table ? r->table : ctx_empty_table(ctx);
  D.nloop = r->nloop;
  D.img = r->k ? (float*)(arena_dev + r->img_off) : r->out;
  int2* tl = (int2*)(host.data() + o_t);
  for (int i = 0; i < nt; ++i) tl[i] = make_int2(0, b.blk0 + i);
  JT_TRY(upload(b, host.data(), end, base, s));
  JT_TRY(timed_launch(ctx, JT_K_SIM, s, [&] {
    return launch_simulate_desc(r->split, r->tnfw, light_has_extra(r->src) || light_has_extra(r->ll), false, (const ImageDesc*)base,
                                (const int2*)(base + o_t), nt, 0, s);
  }, "server simulate chunk"));
  return check_hip(hipEventRecord(b.ev, s), "hipEventRecord(batch)");
}

jt_status jt_server::launch_conv_hip(Batch& b) {
  JT_TRY(ctx_enter(ctx));
  Req* r = b.reqs[0];
  hipStream_t s = streams[b.stream];
  const ConvShape sh = conv_shape(r->g.nx, r->g.ny, r->k);
  const long nct = (long)conv_tiles_x(r->g.nx, sh) * conv_tiles_y(r->g.ny);
  const size_t o_ct = a256(sizeof(ConvDesc));
  const size_t end = o_ct + a256(sizeof(int4) * (size_t)nct);
  if (end > b.bytes) return fail(JT_EDEVICE, "server: convolution block too small (internal)");
  char* base = arena_dev + b.off;
  std::vector<char> host(end, 0);
  *(ConvDesc*)host.data() = ConvDesc{(const float*)(arena_dev + r->img_off), r->out, r->psf, r->g.nx, r->g.ny, r->k,
                                     sh.t};
  int4* ct = (int4*)(host.data() + o_ct);
  long j = 0;
  for (int ty = 0; ty < conv_tiles_y(r->g.ny); ++ty)
    for (int tx = 0; tx < conv_tiles_x(r->g.nx, sh); ++tx) ct[j++] = make_int4(0, tx, ty, 0);
  JT_TRY(upload(b, host.data(), end, base, s));
  JT_TRY(timed_launch(ctx, JT_K_CONV, s, [&] {
    return launch_conv_desc(conv_shape_kind(sh), (const ConvDesc*)base, (const int4*)(base + o_ct), (int)nct,
                            conv_lds_bytes(r->k, sh), s);
  }, "server convolve"));
  return check_hip(hipEventRecord(b.ev, s), "hipEventRecord(batch)");
}

// Simulated device, called with mu held: the first unfinished batch of each
// stream runs, and the running batches share the device equally (a stream's
// batches run in order, different streams overlap).
void jt_server::sim_advance(Clock::time_point now) {
  double dt = std::chrono::duration<double>(now - sim_last).count();
  auto at = sim_last;
  sim_last = now;
  for (;;) {
    std::vector<Batch*> run;
    std::vector<int> seen;
    for (auto& bp : inflight) {
      Batch* b = bp.get();
      if (b->sim_fin || std::find(seen.begin(), seen.end(), b->stream) != seen.end()) {
        if (!b->sim_fin) continue;
        continue;
      }
      seen.push_back(b->stream);
      run.push_back(b);
    }
    if (run.empty() || dt <= 0) return;
    const double n = (double)run.size();
    double first = run[0]->sim_left;
    for (Batch* b : run) first = std::min(first, b->sim_left);
    const double t_first = first * n;          // wall time until the first finishes
    const double step = std::min(t_first, dt);
    for (Batch* b : run) b->sim_left -= step / n;
    at += std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(step));
    dt -= step;
    bool any = false;
    for (Batch* b : run)
      if (b->sim_left <= 1e-12) {
        b->sim_fin = true;
        b->sim_done = at;
        any = true;
      }
    if (!any) return;
  }
}

// Simulated device: wall seconds until the next running batch finishes.
double jt_server::sim_next_completion() {
  std::vector<int> seen;
  double best = 1.0, n = 0;
  std::vector<double> left;
  for (auto& bp : inflight) {
    Batch* b = bp.get();
    if (b->sim_fin || std::find(seen.begin(), seen.end(), b->stream) != seen.end()) continue;
    seen.push_back(b->stream);
    left.push_back(b->sim_left);
  }
  n = (double)left.size();
  for (double l : left) best = std::min(best, l * n);
  return left.empty() ? 1e-3 : best;
}

// Called with mu held: a request leaves the device.
void jt_server::finish_request(Req* r, bool failed, Clock::time_point t) {
  r->state = failed ? JT_TICKET_FAILED : JT_TICKET_DONE;
  r->t_done = t;
  if (failed) ++st.failed; else ++st.completed;
  const double w = std::chrono::duration<double>(r->t_launch - r->t_submit).count();
  st.wait_seconds += w;
  st.max_wait_seconds = std::max(st.max_wait_seconds, w);
  st.run_seconds += std::chrono::duration<double>(t - r->t_launch).count();
}

// Called with mu held: a request ends without running to completion.
void jt_server::cancel_request(Req* r, Clock::time_point t) {
  r->state = JT_TICKET_CANCELLED;
  r->t_done = t;
  ++st.cancelled;
}

// Called with mu held, on the first failed batch: the queue fails at once,
// chunked requests stop launching chunks (they fail once nothing of theirs
// runs), and every batch still in flight will report failure.
void jt_server::fail_all(const char* why) {
  if (broken) return;
  broken = true;
  broken_why = why;
  const auto now = Clock::now();
  for (Req* r : queue) {
    r->t_launch = now;
    finish_request(r, true, now);
  }
  queue.clear();
  for (Req* r : active) r->failed = true;
  done_cv.notify_all();
}

// Called with mu held once stopping: chunked requests with nothing on the
// device end as cancelled (a request whose convolution was launched finishes
// normally when it completes).
void jt_server::retire_stopped_chunked(Clock::time_point t) {
  for (auto it = active.begin(); it != active.end();) {
    Req* r = *it;
    if (r->chunks_inflight == 0 && !r->conv_launched) {
      if (r->failed) finish_request(r, true, t); else cancel_request(r, t);
      if (r->img_bytes) arena.release(r->img_off, r->img_bytes);
      it = active.erase(it);
      done_cv.notify_all();
    } else {
      ++it;
    }
  }
}

// Called with mu held.
void jt_server::complete_finished() {
  const auto now = Clock::now();
  if (!ctx) sim_advance(now);
  bool any = false;
  for (auto it = inflight.begin(); it != inflight.end();) {
    Batch& b = **it;
    bool fin = false;
    if (!ctx) {
      fin = b.sim_fin;
    } else if (b.done) {
      fin = true;
    } else {
      // completion is polled from the stream's event: a host callback on the
      // stream was seen to wait for the other streams' queued work
      const hipError_t q = hipEventQuery(b.ev);
      if (q == hipSuccess) {
        fin = true;
        b.t_done = now;
      } else if (q != hipErrorNotReady) {
        (void)hipGetLastError();
        fin = true;
        b.failed = true;
        b.t_done = now;
      }
    }
    if (!fin) {
      ++it;
      continue;
    }
    if (b.ev) events.push_back(b.ev);
    const auto t = ctx ? b.t_done : b.sim_done;
    if (b.failed) fail_all("a batch failed on the device");
    if (broken) b.failed = true;
    if (b.chunk || b.conv) {
      --chunk_batches;
      Req* r = b.reqs[0];
      if (b.chunk) --r->chunks_inflight;
      if (b.failed) r->failed = true;
      // done after its convolution (or last chunk without a PSF), or after a
      // failure once nothing of it runs
      const bool chunks_done = r->next_block == r->blocks && r->chunks_inflight == 0;
      const bool over = b.conv || (r->failed && r->chunks_inflight == 0) || (chunks_done && !r->k);
      if (over) {
        finish_request(r, r->failed, t);
        if (r->img_bytes) arena.release(r->img_off, r->img_bytes);
        active.erase(std::find(active.begin(), active.end(), r));
      }
    } else {
      for (Req* r : b.reqs) finish_request(r, b.failed, t);
    }
    arena.release(b.off, b.bytes);
    if (b.st_bytes) stage.release(b.st_off, b.st_bytes);
    it = inflight.erase(it);
    any = true;
  }
  if (any) done_cv.notify_all();
}

// Stream of the next batch of whole requests: round robin, avoiding the
// streams of chunked requests in progress when another is free.
int jt_server::small_stream() {
  const int n = std::max(1, cfg.n_streams);
  int sidx = next_stream;
  for (int t = 0; t < n; ++t) {
    const int c = (next_stream + t) % n;
    bool used = false;
    for (Req* a : active) used |= a->stream == c;
    if (!used) {
      sidx = c;
      break;
    }
  }
  next_stream = (sidx + 1) % n;
  return sidx;
}

// Called with mu held: launches (or, on the simulated device, schedules) a
// formed batch; false when the launch failed.
bool jt_server::launch_batch(std::unique_ptr<Batch> bp) {
  Batch& b = *bp;
  b.srv = this;
  ++st.batches;
  bool ok = true;
  if (ctx) {
    if (!events.empty()) {
      b.ev = events.back();
      events.pop_back();
    } else if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) {
      b.ev = nullptr;
    }
  }
  if (ctx && !b.ev) {
    b.failed = true;
    b.t_done = Clock::now();
    b.done = true;
    ok = false;
  } else if (ctx) {
    if ((b.chunk ? launch_chunk_hip(b) : b.conv ? launch_conv_hip(b) : launch_hip(b)) != JT_OK) {
      // no completion callback was queued: let whatever was launched finish
      // before the batch's arena block can be reused
      (void)hipStreamSynchronize(streams[b.stream]);
      b.failed = true;
      b.t_done = Clock::now();
      b.done = true;
      ok = false;
    }
  } else {
    const auto now = Clock::now();
    const double dur = b.pairs / sim_rate + 20e-6;
    sim_advance(now);
    b.sim_left = dur;
    st.device_seconds += dur;
    // an injected failure shows when the batch completes, as a device error would
    if (sim_fail_batch && st.batches == sim_fail_batch) b.failed = true;
  }
  inflight.push_back(std::move(bp));
  return ok;
}

// Called with mu held: forms batches while slots and arena space allow.
// Chunked requests in progress get their next chunks first (round robin, at
// most two queued each, leaving one slot for batches of whole requests); then
// whole requests are taken from the queue head up to the caps (a request over
// the work cap that is not chunked forms a batch of its own).  A chunked
// request at the head is started while fewer than max(1, n_streams - 1) are
// in progress, and otherwise waits there (FIFO).
void jt_server::launch_ready() {
  // staging slices exist only on a real device
  auto take_stage = [&](size_t n, size_t* o) { return !ctx || n == 0 || stage.alloc(n, o); };
  const int n_streams = std::max(1, cfg.n_streams);
  const int max_active = std::max(1, n_streams - 1);
  const int max_chunk_batches = std::max(1, cfg.max_inflight_batches - 1);
  while (!stop && !broken && (int)inflight.size() < cfg.max_inflight_batches) {
    // next chunk of a chunked request, or its convolution once every chunk
    // has completed
    Req* r = nullptr;
    bool conv = false;
    // whole requests queued or on the device: chunks share the chip
    const bool shared = !queue.empty() || (int)inflight.size() > chunk_batches;
    const int chunk_depth = shared ? 1 : 2;
    if (chunk_batches < max_chunk_batches) {
      for (size_t i = 0; i < active.size() && !r; ++i) {
        Req* a = active[(rr + i) % active.size()];
        if (a->failed) continue;
        if (a->next_block < a->blocks && a->chunks_inflight < chunk_depth) {
          r = a;
        } else if (a->k && !a->conv_launched && a->next_block == a->blocks && a->chunks_inflight == 0) {
          r = a;
          conv = true;
        }
        if (r) rr = (rr + i + 1) % active.size();
      }
    }
    if (r) {
      const int cb = shared ? std::min(r->chunk_blocks, kChunkSharedBlocks) : r->chunk_blocks;
      const int b0 = r->next_block, b1 = conv ? b0 : std::min(r->blocks, b0 + cb);
      const size_t bytes = conv ? conv_footprint(r->g, r->k) : chunk_footprint(b1 - b0);
      size_t off = 0, so = 0;
      if (!arena.alloc(bytes, &off)) return;
      if (!take_stage(bytes, &so)) {
        arena.release(off, bytes);
        return;
      }
      auto bp = std::make_unique<Batch>();
      bp->st_off = so;
      bp->st_bytes = ctx ? bytes : 0;
      bp->reqs = {r};
      bp->off = off;
      bp->bytes = bytes;
      bp->stream = r->stream;
      if (conv) {
        bp->conv = true;
        r->conv_launched = true;
      } else {
        bp->chunk = true;
        bp->blk0 = b0;
        bp->blk1 = b1;
        bp->pairs = r->pairs * (double)(b1 - b0) / r->blocks;
        r->next_block = b1;
        ++r->chunks_inflight;
      }
      ++chunk_batches;
      if (!launch_batch(std::move(bp))) r->failed = true;
      continue;
    }
    if (queue.empty()) return;
    Req* head = queue.front();
    if (head->chunked) {
      if ((int)active.size() >= max_active) return;  // FIFO behind it
      // start the chunked request: its image block and stream
      size_t off = 0;
      const size_t img = head->k ? a256(4 * (size_t)head->g.nx * head->g.ny) : 0;
      if (img && !arena.alloc(img, &off)) return;
      head->img_off = off;
      head->img_bytes = img;
      // a stream no other chunked request uses
      int sidx = next_stream;
      for (int t = 0; t < n_streams; ++t) {
        const int c = (next_stream + t) % n_streams;
        bool used = false;
        for (Req* a : active) used |= a->stream == c;
        if (!used) {
          sidx = c;
          break;
        }
      }
      head->stream = sidx;
      next_stream = (sidx + 1) % n_streams;
      head->state = JT_TICKET_RUNNING;
      head->t_launch = Clock::now();
      queue.pop_front();
      active.push_back(head);
      continue;
    }
    std::vector<Req*> pick;
    double pairs = 0;
    size_t bytes = 0, hbytes = 0;
    for (Req* r : queue) {
      if ((int)pick.size() >= cfg.max_batch_images) break;
      if (r->chunked) break;  // it waits at its place
      if (!pick.empty() && pairs + r->pairs > cfg.max_batch_pairs) break;
      if (!pick.empty() && r->tnfw != pick[0]->tnfw) break;  // one subhalo profile per launch
      pick.push_back(r);
      pairs += r->pairs;
      bytes += r->footprint;
      hbytes += header_bytes(r);
    }
    size_t off = 0, so = 0;
    while (!pick.empty()) {
      if (arena.alloc(bytes, &off)) {
        if (take_stage(hbytes, &so)) break;
        arena.release(off, bytes);
      }
      bytes -= pick.back()->footprint;
      hbytes -= header_bytes(pick.back());
      pairs -= pick.back()->pairs;
      pick.pop_back();
    }
    if (pick.empty()) return;  // the head does not fit yet: wait for completions
    for (size_t i = 0; i < pick.size(); ++i) queue.pop_front();
    auto bp = std::make_unique<Batch>();
    bp->st_off = so;
    bp->st_bytes = ctx ? hbytes : 0;
    bp->reqs = pick;
    bp->off = off;
    bp->bytes = bytes;
    bp->pairs = pairs;
    bp->stream = small_stream();
    const auto tl = Clock::now();
    for (Req* r : pick) {
      r->state = JT_TICKET_RUNNING;
      r->t_launch = tl;
    }
    launch_batch(std::move(bp));
  }
}

void jt_server::run() {
  if (ctx) (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    complete_finished();
    launch_ready();
    if (stop || broken) retire_stopped_chunked(Clock::now());
    if (stop && inflight.empty()) break;
    if (inflight.empty()) {
      cv.wait(lk, [&] { return stop || !queue.empty(); });
    } else if (!ctx) {
      const double dt = sim_next_completion();
      cv.wait_for(lk, std::chrono::duration<double>(std::max(dt, 1e-6)));
    } else {
      // woken by submissions; in-flight batches are polled every 200 us
      cv.wait_for(lk, std::chrono::microseconds(200));
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
  s->stage.init(kStagingBytes);
  s->st.arena_bytes = s->cfg.hbm_budget_bytes;
  s->sim_last = Clock::now();
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
  jt_status hs = check_hip(hipHostMalloc((void**)&s->stage_host, kStagingBytes, hipHostMallocDefault),
                           "hipHostMalloc(server staging)");
  if (hs != JT_OK) {
    (void)hipFree(s->arena_dev);
    return hs;
  }
  for (int i = 0; i < cfg->n_streams; ++i) {
    hipStream_t st = nullptr;
    jt_status e = check_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
    if (e != JT_OK) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      (void)hipFree(s->arena_dev);
      (void)hipHostFree(s->stage_host);
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
  lens.has_epl = req->has_epl;
  lens.epl = req->epl;
  JT_TRY(make_macro(&lens, r->mc));
  JT_TRY(make_light(&req->src, r->src, "source"));
  JT_TRY(make_light(&req->lens_light, r->ll, "lens light"));
  if (!req->out) return fail(JT_EINVAL, "server submit: null output");
  r->out = req->out;
  if (srv->ctx) {
    if (req->subhalo_handle) {
      const void* tab = nullptr;
      JT_TRY(ctx_subhalo_handle(srv->ctx, req->subhalo_handle, &tab, &r->nsub, &r->tnfw));
      r->table = tab;
    }
    if (req->psf_handle) JT_TRY(jt_psf_pointer(srv->ctx, req->psf_handle, &r->psf, &r->k));
  } else {
    r->nsub = (int)req->subhalo_handle;
    r->k = (int)req->psf_handle;
    if (r->k && r->k % 2 == 0) return fail(JT_EINVAL, "server submit: even PSF side");
  }
  if (r->k > JT_MAX_PSF) return fail(JT_EUNSUPPORTED, "server submit: PSF side %d > %d", r->k, JT_MAX_PSF);
  r->nloop = subhalo_loop_count(r->nsub);
  r->pairs = request_pairs(r->g, r->nloop) * (r->tnfw ? kTnfwPairCost : 1.0);
  // block shape as the request would run alone; chunked when over the work
  // cap and large enough for more than two minimum chunks, otherwise a
  // request over the cap runs as a batch of its own
  r->split = pick_split((long)r->g.nx * r->g.ny * r->g.s2, r->g.s2, r->nloop);
  r->ppb = split_lanes(r->split) / r->g.s2;
  r->blocks = (int)(((long)r->g.nx * r->g.ny + r->ppb - 1) / r->ppb);
  r->chunked = r->pairs > srv->cfg.max_batch_pairs && r->blocks > 2 * kChunkMinBlocks;
  if (r->chunked) {
    const double per_block = r->pairs / r->blocks;
    r->chunk_blocks = (int)std::max((double)kChunkMinBlocks, std::floor(srv->cfg.max_batch_pairs / per_block));
    r->footprint = (r->k ? a256(4 * (size_t)r->g.nx * r->g.ny) : 0) +
                   std::max(2 * chunk_footprint(std::min(r->blocks, r->chunk_blocks)), r->k ? conv_footprint(r->g, r->k) : 0);
  } else {
    r->footprint = request_footprint(r->g, r->k);
  }
  const size_t hdr = r->chunked ? (r->k ? conv_footprint(r->g, r->k) : 0) : header_bytes(r.get());
  if (hdr > kStagingBytes)
    return fail(JT_ENOMEM, "server submit: request descriptors need %zu bytes of staging, %zu available", hdr,
                kStagingBytes);
  if (r->footprint > srv->arena.size)
    return fail(JT_ENOMEM, "server submit: request needs %zu bytes, arena holds %zu", r->footprint, srv->arena.size);
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return fail(JT_ECANCELLED, "server submit: server is stopping");
  if (srv->broken)
    return fail(JT_EDEVICE, "server submit: refused after a device failure (%s); create a new server",
                srv->broken_why.c_str());
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
  // jt_server_destroy waits until no thread is in here
  ++srv->waiters;
  bool ended = true;
  if (timeout_s < 0)
    srv->done_cv.wait(lk, final_state);
  else
    ended = srv->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), final_state);
  --srv->waiters;
  srv->done_cv.notify_all();
  if (!ended) return fail(JT_EBUSY, "server wait: ticket %llu still pending", (unsigned long long)ticket);
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

extern "C" jt_status jt_server_simulate_failure(jt_server* srv, uint64_t batch) {
  if (!srv) return fail(JT_EINVAL, "server failure injection: null server");
  if (srv->ctx) return fail(JT_EINVAL, "server failure injection: simulated servers only");
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->sim_fail_batch = batch;
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
  {
    // every ticket is final now; let threads still in jt_server_wait leave
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->done_cv.notify_all();
    srv->done_cv.wait(lk, [&] { return srv->waiters == 0; });
  }
  if (srv->ctx) {
    (void)hipSetDevice(srv->ctx->device);
    for (auto s : srv->streams) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
    for (auto e : srv->events) (void)hipEventDestroy(e);
    if (srv->arena_dev) (void)hipFree(srv->arena_dev);
    if (srv->stage_host) (void)hipHostFree(srv->stage_host);
  }
  delete srv;
}
