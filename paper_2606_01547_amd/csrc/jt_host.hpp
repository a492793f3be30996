// Internal host-side declarations of libjt: the context, error helpers,
// parameter preparation (FP64 -> FP32 kernel constants) and timed launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/jt.h"
#include "jt_device.hpp"

#define JT_TRY(expr)            \
  do {                          \
    jt_status _s = (expr);      \
    if (_s != JT_OK) return _s; \
  } while (0)

struct Buffer {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Resident {
  int kind = 0;  // 1 = NFW subhalo table, 2 = PSF, 3 = TNFW subhalo table
  void* dev = nullptr;
  int n = 0;     // subhalos (kind 1) or PSF side k (kind 2)
};

struct Staging {
  void* host = nullptr;       // pinned
  size_t bytes = 0;
  hipEvent_t done = nullptr;  // recorded after the last copy out of `host`
  bool pending = false;
};

struct EventRec {
  hipEvent_t a, b;
  int id;
};

struct jt_ctx {
  int device = 0;
  std::mutex mu;
  std::map<hipStream_t, Buffer> ws;      // per-stream workspace
  std::map<hipStream_t, Buffer> ws_aux;  // per-stream second workspace (FFT buffers)
  std::map<hipStream_t, Staging> stage;  // per-stream pinned upload buffer
  std::map<int, void*> twiddles;         // FFT length -> device exp(-2 pi i t / N), t < N
  std::map<uint64_t, Resident> handles;
  uint64_t next_handle = 1;
  jt::SubRec* empty_table = nullptr;  // padding records for lenses without subhalos
  bool prof = false;
  std::vector<EventRec> pending;
  std::vector<hipEvent_t> free_events;
  double prof_ms[JT_K_COUNT] = {0};
  int prof_n[JT_K_COUNT] = {0};
};

namespace jt {

// [a, a + n) and [b, b + m) share an element (null pointers share none).
inline bool overlap(const float* a, size_t n, const float* b, size_t m) {
  if (!a || !b || n == 0 || m == 0) return false;
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + sizeof(float) * m && pb < pa + sizeof(float) * n;
}

jt_status fail(jt_status st, const char* fmt, ...);
jt_status check_hip(hipError_t e, const char* what);
jt_status ctx_enter(jt_ctx* ctx);
jt_status ctx_workspace(jt_ctx* ctx, hipStream_t stream, size_t bytes, void** out);
// A second per-stream workspace, independent of the first (a call can hold
// both: e.g. the unconvolved image in one and FFT buffers in the other).
jt_status ctx_workspace_aux(jt_ctx* ctx, hipStream_t stream, size_t bytes, void** out);
// Asynchronous host -> device copy of `bytes` through the stream's pinned
// staging buffer (the previous copy out of it is waited for first).
jt_status ctx_upload(jt_ctx* ctx, hipStream_t stream, void* dev_dst, const void* host_src, size_t bytes);
// Device twiddle table of an FFT length (built on first use, kept by ctx).
jt_status ctx_twiddles(jt_ctx* ctx, int N, const double2** out);
// A resident subhalo table: records (SubRec, or TRec when *tnfw), count.
jt_status ctx_subhalo_handle(jt_ctx* ctx, uint64_t h, const void** table, int* n, bool* tnfw);
const SubRec* ctx_empty_table(jt_ctx* ctx);
// Looks up the calling device's static scratch array for
// jt_simulate_image_noalloc (once per device; the device must be current).
jt_status noalloc_scratch_init(int device);
hipEvent_t take_event(jt_ctx* ctx);
void drain_events(jt_ctx* ctx);

// Timed launch: records HIP events around `launch` on `st` when profiling is on.
template <class F>
jt_status timed_launch(jt_ctx* ctx, int id, hipStream_t st, F&& launch, const char* what) {
  hipEvent_t a = nullptr, b = nullptr;
  bool prof;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    prof = ctx->prof;
    if (prof) {
      if (ctx->pending.size() > 4096) drain_events(ctx);
      a = take_event(ctx);
      b = take_event(ctx);
      if (!a || !b) prof = false;
    }
  }
  if (prof) (void)hipEventRecord(a, st);
  hipError_t e = launch();
  if (prof) {
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->pending.push_back({a, b, id});
  }
  return check_hip(e, what);
}

// ---- parameter preparation (jt_params.cpp) ----
jt_status make_macro(const jt_lens* lens, MacroC& out);
jt_status make_light(const jt_light* light, LightC& out, const char* which);
jt_status make_grid(const jt_grid* grid, GridC& out);
// Median-defining b_n: the root b of P(2n, b) = 1/2 (regularised lower
// incomplete gamma), by safeguarded Newton iteration.
double sersic_bn_exact(double n);
// Regularised lower incomplete gamma P(a, x).
double gamma_p(double a, double x);
// Packed subhalo table (with padding records) from host FP32 SoA; validates.
jt_status pack_subhalos_host(int n, const float* x, const float* y, const float* rs, const float* ars,
                             std::vector<SubRec>& out);
// Validates host FP32 SoA of truncated subhalos (r_trunc > 0); their table
// is packed on the device by the same kernel as a device SoA's, so that both
// give bit-identical records.
jt_status validate_tnfw_host(int n, const float* x, const float* y, const float* rs, const float* ars,
                             const float* rt);
// Bytes of the packed table the device SoA of `lens` needs (0 with a handle or
// no subhalos), 256-byte aligned.
size_t subhalo_scratch_bytes(const jt_lens* lens);

// Resolves the subhalo table of a lens: resident handle, or device SoA packed
// into `scratch` (room for subhalo_table_records(n) records) by the prep
// kernel, or the context's empty table.  *nloop = loop count (multiple of 4).
jt_status resolve_subhalos(jt_ctx* ctx, const jt_lens* lens, void* scratch, hipStream_t st,
                           const void** table, int* nloop, bool* tnfw);

}  // namespace jt
