// Stress driver for the continuous-batching server on its simulated device
// (no GPU), through the C ABI only: concurrent submitters and waiters,
// cancellation racing the scheduler, an injected device failure, and
// destruction with queued work, a chunked request in progress and threads
// still waiting.  Built against host-sanitized builds of the library
// (AddressSanitizer + UndefinedBehaviorSanitizer, ThreadSanitizer) by
// paper_2606_01547_amd/csrc/build_sanitized.sh; exits non-zero on a failed
// check, and the sanitizers abort on a finding.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "jt.h"

#define CHECK(cond)                                                                     \
  do {                                                                                  \
    if (!(cond)) {                                                                      \
      std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #cond, jt_last_error()); \
      std::exit(1);                                                                     \
    }                                                                                   \
  } while (0)

namespace {

jt_sersic g_src{10.0, 0.2, 2.0, 0.8, 0.3, 0.05, -0.02};

jt_request request(int npix, int s, int nsub, int k) {
  jt_request r{};
  r.grid = jt_grid{npix, npix, s, 0.05, 0.0, 0.0};
  r.has_sie = 1;
  r.sie = jt_sie{1.1, 0.8, 0.4, 0.01, -0.02};
  r.has_shear = 1;
  r.shear = jt_shear{0.02, -0.01};
  r.subhalo_handle = (uint64_t)nsub;   // simulated server: subhalo count
  r.psf_handle = (uint64_t)k;          // simulated server: PSF side
  r.src.n = 1;
  r.src.c = &g_src;
  r.out = reinterpret_cast<float*>(16);   // never touched by the simulated device
  return r;
}

jt_server* make(int inflight, int images, double cap, double rate, int streams = 2) {
  jt_server_cfg cfg{64u << 20, images, cap, inflight, streams};
  jt_server* s = nullptr;
  CHECK(jt_server_create_simulated(&cfg, rate, &s) == JT_OK);
  return s;
}

void concurrent_submitters() {
  jt_server* s = make(3, 16, 5e8, 1e11, 3);
  std::atomic<int> done{0};
  std::vector<std::thread> th;
  for (int w = 0; w < 4; ++w)
    th.emplace_back([&, w] {
      std::vector<uint64_t> mine;
      for (int i = 0; i < 50; ++i) {
        jt_request r = request(32 + 16 * ((w + i) % 4), 1 + 2 * (i % 2), 10 * (i % 7), (i % 3) ? 11 : 0);
        uint64_t t = 0;
        CHECK(jt_server_submit(s, &r, &t) == JT_OK);
        mine.push_back(t);
        int st = -1;
        CHECK(jt_server_poll(s, t, &st) == JT_OK);
      }
      for (uint64_t t : mine) {
        double lat = 0;
        CHECK(jt_server_wait(s, t, 30.0, &lat) == JT_OK);
        CHECK(lat >= 0);
        done.fetch_add(1);
      }
    });
  for (auto& t : th) t.join();
  jt_server_stats st{};
  CHECK(jt_server_get_stats(s, &st) == JT_OK);
  CHECK(done.load() == 200 && st.completed == 200 && st.arena_in_use == 0);
  jt_server_destroy(s);
}

void cancel_races_the_scheduler() {
  jt_server* s = make(1, 1, 5e8, 1e10);
  std::vector<uint64_t> t(40);
  for (auto& x : t) {
    jt_request r = request(64, 3, 500, 11);
    CHECK(jt_server_submit(s, &r, &x) == JT_OK);
  }
  std::thread canceller([&] {
    for (size_t i = 1; i < t.size(); i += 2) {
      const jt_status c = jt_server_cancel(s, t[i]);
      CHECK(c == JT_OK || c == JT_EBUSY || c == JT_EINVAL);
    }
  });
  int ok = 0, cancelled = 0;
  for (size_t i = 0; i < t.size(); i += 2) {
    CHECK(jt_server_wait(s, t[i], 30.0, nullptr) == JT_OK);
    ++ok;
  }
  canceller.join();
  for (size_t i = 1; i < t.size(); i += 2) {
    const jt_status w = jt_server_wait(s, t[i], 30.0, nullptr);
    CHECK(w == JT_OK || w == JT_ECANCELLED);
    (w == JT_OK ? ok : cancelled) += 1;
  }
  jt_server_stats st{};
  CHECK(jt_server_get_stats(s, &st) == JT_OK);
  CHECK((int)st.completed == ok && (int)st.cancelled == cancelled && ok + cancelled == 40);
  jt_server_destroy(s);
}

void injected_failure() {
  jt_server* s = make(2, 1, 5e8, 1e9);
  CHECK(jt_server_simulate_failure(s, 4) == JT_OK);
  std::vector<uint64_t> t(12);
  for (auto& x : t) {
    jt_request r = request(100, 1, 1000, 11);
    CHECK(jt_server_submit(s, &r, &x) == JT_OK);
  }
  std::vector<std::thread> waiters;
  std::atomic<int> ok{0}, failed{0};
  for (size_t i = 0; i < t.size(); ++i)
    waiters.emplace_back([&, i] {
      const jt_status w = jt_server_wait(s, t[i], 30.0, nullptr);
      CHECK(w == JT_OK || w == JT_EDEVICE);
      (w == JT_OK ? ok : failed).fetch_add(1);
    });
  for (auto& w : waiters) w.join();
  CHECK(ok.load() == 3 && failed.load() == 9);
  jt_request r = request(32, 1, 0, 0);
  uint64_t x = 0;
  CHECK(jt_server_submit(s, &r, &x) == JT_EDEVICE);
  jt_server_stats st{};
  CHECK(jt_server_get_stats(s, &st) == JT_OK);
  CHECK(st.arena_in_use == 0 && st.failed == 9);
  jt_server_destroy(s);
}

void destroy_with_work_everywhere() {
  // a chunked request in progress, whole requests queued behind it, and
  // threads waiting on all of them while the server is destroyed
  jt_server* s = make(3, 4, 1e7, 1e10);
  std::vector<uint64_t> t;
  jt_request big = request(1200, 3, 2000, 21);
  uint64_t tb = 0;
  CHECK(jt_server_submit(s, &big, &tb) == JT_OK);
  t.push_back(tb);
  for (int i = 0; i < 20; ++i) {
    jt_request r = request(200, 3, 5000, 11);
    uint64_t x = 0;
    CHECK(jt_server_submit(s, &r, &x) == JT_OK);
    t.push_back(x);
  }
  int st = JT_TICKET_QUEUED;
  for (int i = 0; i < 5000 && st != JT_TICKET_RUNNING; ++i) {
    CHECK(jt_server_poll(s, tb, &st) == JT_OK);
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  }
  CHECK(st == JT_TICKET_RUNNING);
  std::atomic<int> started{0}, returned{0}, cancelled{0};
  std::vector<std::thread> waiters;
  for (uint64_t x : t)
    waiters.emplace_back([&, x] {
      started.fetch_add(1);
      const jt_status w = jt_server_wait(s, x, -1.0, nullptr);
      CHECK(w == JT_OK || w == JT_ECANCELLED);
      if (w == JT_ECANCELLED) cancelled.fetch_add(1);
      returned.fetch_add(1);
    });
  while (started.load() < (int)t.size()) std::this_thread::yield();
  std::this_thread::sleep_for(std::chrono::milliseconds(50));   // every waiter is inside jt_server_wait
  const auto t0 = std::chrono::steady_clock::now();
  jt_server_destroy(s);
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (auto& w : waiters) w.join();
  CHECK(returned.load() == (int)t.size());
  CHECK(cancelled.load() >= 1);                 // the chunked request at least
  CHECK(sec < 10.0);
}

}  // namespace

int main() {
  concurrent_submitters();
  std::puts("concurrent submitters: ok");
  cancel_races_the_scheduler();
  std::puts("cancellation: ok");
  injected_failure();
  std::puts("injected failure: ok");
  destroy_with_work_everywhere();
  std::puts("destroy with work pending: ok");
  return 0;
}
