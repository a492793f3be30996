// libjt host runtime: argument validation, FP64 parameter preparation, device
// workspace and resident tables, kernel timing, and the C ABI of include/jt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/jt.h"
#include "jt_host.hpp"
#include "jt_kernels.hpp"

using namespace jt;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace {
thread_local std::string g_last_error;
}

namespace jt {
jt_status fail(jt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

jt_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return JT_OK;
  if (e == hipErrorOutOfMemory) return fail(JT_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(JT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}
}  // namespace jt

extern "C" const char* jt_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* jt_version(void) { return "libjt 0.1 (gfx950)"; }

extern "C" double jt_sersic_bn(double n, int exact) {
  if (!(n >= 0.2 && n <= 10.0)) return std::nan("");
  return exact ? sersic_bn_exact(n) : 1.9992 * n - 0.3271;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
namespace jt {

jt_status ctx_enter(jt_ctx* ctx) {
  if (!ctx) return fail(JT_EINVAL, "null context");
  return check_hip(hipSetDevice(ctx->device), "hipSetDevice");
}

// Workspace of at least `bytes` for `stream`; grows (after synchronising the
// stream) when too small.
static jt_status grow_buffer(Buffer& b, hipStream_t stream, size_t bytes, void** out);

jt_status ctx_workspace(jt_ctx* ctx, hipStream_t stream, size_t bytes, void** out) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  return grow_buffer(ctx->ws[stream], stream, bytes, out);
}

jt_status ctx_workspace_aux(jt_ctx* ctx, hipStream_t stream, size_t bytes, void** out) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  return grow_buffer(ctx->ws_aux[stream], stream, bytes, out);
}

static jt_status grow_buffer(Buffer& b, hipStream_t stream, size_t bytes, void** out) {
  if (b.bytes < bytes) {
    if (b.p) {
      JT_TRY(check_hip(hipStreamSynchronize(stream), "workspace sync"));
      JT_TRY(check_hip(hipFree(b.p), "hipFree"));
      b.p = nullptr;
      b.bytes = 0;
    }
    size_t cap = std::max<size_t>(bytes, 1 << 20);
    cap = (cap + 4095) & ~size_t(4095);
    JT_TRY(check_hip(hipMalloc(&b.p, cap), "hipMalloc(workspace)"));
    b.bytes = cap;
  }
  *out = b.p;
  return JT_OK;
}

jt_status ctx_upload(jt_ctx* ctx, hipStream_t stream, void* dev_dst, const void* host_src, size_t bytes) {
  if (bytes == 0) return JT_OK;
  std::lock_guard<std::mutex> lk(ctx->mu);
  Staging& sg = ctx->stage[stream];
  if (sg.pending) {
    JT_TRY(check_hip(hipEventSynchronize(sg.done), "staging wait"));
    sg.pending = false;
  }
  if (sg.bytes < bytes) {
    if (sg.host) JT_TRY(check_hip(hipHostFree(sg.host), "hipHostFree"));
    sg.host = nullptr;
    sg.bytes = 0;
    const size_t cap = std::max<size_t>(bytes, 1 << 16);
    JT_TRY(check_hip(hipHostMalloc(&sg.host, cap, hipHostMallocDefault), "hipHostMalloc(staging)"));
    sg.bytes = cap;
  }
  if (!sg.done) JT_TRY(check_hip(hipEventCreateWithFlags(&sg.done, hipEventDisableTiming), "hipEventCreate"));
  std::memcpy(sg.host, host_src, bytes);
  JT_TRY(check_hip(hipMemcpyAsync(dev_dst, sg.host, bytes, hipMemcpyHostToDevice, stream), "staged upload"));
  JT_TRY(check_hip(hipEventRecord(sg.done, stream), "staging event"));
  sg.pending = true;
  return JT_OK;
}

jt_status ctx_twiddles(jt_ctx* ctx, int N, const double2** out) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->twiddles.find(N);
  if (it == ctx->twiddles.end()) {
    std::vector<double2> tw(N);
    const double two_pi = 6.283185307179586476925286766559;
    for (int t = 0; t < N; ++t) {
      const double a = two_pi * (double)t / (double)N;
      tw[t] = make_double2(std::cos(a), -std::sin(a));
    }
    void* dev = nullptr;
    JT_TRY(check_hip(hipMalloc(&dev, sizeof(double2) * tw.size()), "hipMalloc(twiddles)"));
    jt_status st = check_hip(hipMemcpy(dev, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice),
                             "hipMemcpy(twiddles)");
    if (st != JT_OK) {
      (void)hipFree(dev);
      return st;
    }
    it = ctx->twiddles.emplace(N, dev).first;
  }
  *out = (const double2*)it->second;
  return JT_OK;
}

hipEvent_t take_event(jt_ctx* ctx) {
  if (!ctx->free_events.empty()) {
    hipEvent_t e = ctx->free_events.back();
    ctx->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void drain_events(jt_ctx* ctx) {
  for (auto& r : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      ctx->prof_ms[r.id] += ms;
      ctx->prof_n[r.id] += 1;
    }
    ctx->free_events.push_back(r.a);
    ctx->free_events.push_back(r.b);
  }
  ctx->pending.clear();
}

}  // namespace jt

extern "C" jt_status jt_create(int device, jt_ctx** out) {
  if (!out) return fail(JT_EINVAL, "jt_create: null output pointer");
  *out = nullptr;
  int count = 0;
  JT_TRY(check_hip(hipGetDeviceCount(&count), "hipGetDeviceCount"));
  if (device < 0 || device >= count) return fail(JT_EINVAL, "jt_create: device %d of %d", device, count);
  JT_TRY(check_hip(hipSetDevice(device), "hipSetDevice"));
  JT_TRY(noalloc_scratch_init(device));
  jt_ctx* ctx = new jt_ctx();
  ctx->device = device;
  const int rec = subhalo_table_records(0);
  std::vector<SubRec> pad(rec, kSubRecPad);
  jt_status st = check_hip(hipMalloc(&ctx->empty_table, rec * sizeof(SubRec)), "hipMalloc(empty table)");
  if (st == JT_OK)
    st = check_hip(hipMemcpy(ctx->empty_table, pad.data(), rec * sizeof(SubRec), hipMemcpyHostToDevice),
                   "hipMemcpy(empty table)");
  if (st != JT_OK) {
    if (ctx->empty_table) (void)hipFree(ctx->empty_table);
    delete ctx;
    return st;
  }
  *out = ctx;
  return JT_OK;
}

extern "C" void jt_destroy(jt_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    drain_events(ctx);
    for (auto e : ctx->free_events) (void)hipEventDestroy(e);
    for (auto& kv : ctx->ws)
      if (kv.second.p) (void)hipFree(kv.second.p);
    for (auto& kv : ctx->ws_aux)
      if (kv.second.p) (void)hipFree(kv.second.p);
    for (auto& kv : ctx->handles)
      if (kv.second.dev) (void)hipFree(kv.second.dev);
    for (auto& kv : ctx->twiddles) (void)hipFree(kv.second);
    for (auto& kv : ctx->stage) {
      if (kv.second.host) (void)hipHostFree(kv.second.host);
      if (kv.second.done) (void)hipEventDestroy(kv.second.done);
    }
  }
  if (ctx->empty_table) (void)hipFree(ctx->empty_table);
  delete ctx;
}

extern "C" jt_status jt_sync(jt_ctx* ctx, hipStream_t stream) {
  JT_TRY(ctx_enter(ctx));
  JT_TRY(check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize"));
  return check_hip(hipGetLastError(), "device error");
}

// ---------------------------------------------------------------------------
// resident tables
// ---------------------------------------------------------------------------
extern "C" jt_status jt_upload_subhalos(jt_ctx* ctx, int n, const float* x, const float* y,
                                        const float* Rs, const float* alpha_Rs, uint64_t* handle) {
  JT_TRY(ctx_enter(ctx));
  if (!handle) return fail(JT_EINVAL, "jt_upload_subhalos: null handle pointer");
  if (n < 0) return fail(JT_EINVAL, "jt_upload_subhalos: n = %d", n);
  if (n > 0 && (!x || !y || !Rs || !alpha_Rs)) return fail(JT_EINVAL, "jt_upload_subhalos: null array");
  std::vector<SubRec> tab;
  JT_TRY(pack_subhalos_host(n, x, y, Rs, alpha_Rs, tab));
  void* dev = nullptr;
  JT_TRY(check_hip(hipMalloc(&dev, tab.size() * sizeof(SubRec)), "hipMalloc(subhalos)"));
  jt_status st = check_hip(hipMemcpy(dev, tab.data(), tab.size() * sizeof(SubRec), hipMemcpyHostToDevice),
                           "hipMemcpy(subhalos)");
  if (st != JT_OK) {
    (void)hipFree(dev);
    return st;
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  const uint64_t h = ctx->next_handle++;
  ctx->handles[h] = Resident{1, dev, n};
  *handle = h;
  return JT_OK;
}

extern "C" jt_status jt_upload_tnfw(jt_ctx* ctx, int n, const float* x, const float* y, const float* Rs,
                                    const float* alpha_Rs, const float* r_trunc, uint64_t* handle) {
  JT_TRY(ctx_enter(ctx));
  if (!handle) return fail(JT_EINVAL, "jt_upload_tnfw: null handle pointer");
  if (n < 0) return fail(JT_EINVAL, "jt_upload_tnfw: n = %d", n);
  if (n > 0 && (!x || !y || !Rs || !alpha_Rs || !r_trunc)) return fail(JT_EINVAL, "jt_upload_tnfw: null array");
  JT_TRY(validate_tnfw_host(n, x, y, Rs, alpha_Rs, r_trunc));
  // the records (with their far-field fits) are derived on the device by the
  // prep kernel, exactly as for a device SoA
  void* dev = nullptr;
  float* soa = nullptr;
  JT_TRY(check_hip(hipMalloc(&dev, (size_t)subhalo_table_records(n) * sizeof(TRec)), "hipMalloc(tnfw)"));
  jt_status st = JT_OK;
  if (n > 0) st = check_hip(hipMalloc((void**)&soa, 5 * sizeof(float) * (size_t)n), "hipMalloc(tnfw staging)");
  const float* cols[5] = {x, y, Rs, alpha_Rs, r_trunc};
  for (int c = 0; c < 5 && st == JT_OK && n > 0; ++c)
    st = check_hip(hipMemcpy(soa + (size_t)c * n, cols[c], sizeof(float) * (size_t)n, hipMemcpyHostToDevice),
                   "hipMemcpy(tnfw)");
  if (st == JT_OK)
    st = check_hip(launch_prep_tnfw(n, soa, soa + n, soa + 2 * (size_t)n, soa + 3 * (size_t)n,
                                    soa + 4 * (size_t)n, (TRec*)dev, nullptr),
                   "prep_tnfw");
  if (st == JT_OK) st = check_hip(hipStreamSynchronize(nullptr), "prep_tnfw sync");
  if (soa) (void)hipFree(soa);
  if (st != JT_OK) {
    (void)hipFree(dev);
    return st;
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  const uint64_t h = ctx->next_handle++;
  ctx->handles[h] = Resident{3, dev, n};
  *handle = h;
  return JT_OK;
}

extern "C" jt_status jt_upload_psf(jt_ctx* ctx, const float* psf, int k, uint64_t* handle) {
  JT_TRY(ctx_enter(ctx));
  if (!handle || !psf) return fail(JT_EINVAL, "jt_upload_psf: null pointer");
  if (k < 1 || k % 2 == 0 || k > 4095) return fail(JT_EINVAL, "jt_upload_psf: PSF side %d must be odd", k);
  for (long i = 0; i < (long)k * k; ++i)
    if (!std::isfinite(psf[i])) return fail(JT_EINVAL, "jt_upload_psf: non-finite PSF value");
  void* dev = nullptr;
  const size_t bytes = sizeof(float) * (size_t)k * k;
  JT_TRY(check_hip(hipMalloc(&dev, bytes), "hipMalloc(psf)"));
  jt_status st = check_hip(hipMemcpy(dev, psf, bytes, hipMemcpyHostToDevice), "hipMemcpy(psf)");
  if (st != JT_OK) {
    (void)hipFree(dev);
    return st;
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  const uint64_t h = ctx->next_handle++;
  ctx->handles[h] = Resident{2, dev, k};
  *handle = h;
  return JT_OK;
}

extern "C" jt_status jt_psf_pointer(jt_ctx* ctx, uint64_t handle, const float** dev_psf, int* k) {
  if (!ctx || !dev_psf || !k) return fail(JT_EINVAL, "jt_psf_pointer: null pointer");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->handles.find(handle);
  if (it == ctx->handles.end() || it->second.kind != 2) return fail(JT_EINVAL, "unknown PSF handle %llu", (unsigned long long)handle);
  *dev_psf = (const float*)it->second.dev;
  *k = it->second.n;
  return JT_OK;
}

extern "C" jt_status jt_release(jt_ctx* ctx, uint64_t handle) {
  JT_TRY(ctx_enter(ctx));
  void* dev = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->handles.find(handle);
    if (it == ctx->handles.end()) return fail(JT_EINVAL, "unknown handle %llu", (unsigned long long)handle);
    dev = it->second.dev;
    ctx->handles.erase(it);
  }
  JT_TRY(check_hip(hipDeviceSynchronize(), "jt_release sync"));
  return check_hip(hipFree(dev), "hipFree(handle)");
}

namespace jt {
jt_status ctx_subhalo_handle(jt_ctx* ctx, uint64_t h, const void** table, int* n, bool* tnfw) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->handles.find(h);
  if (it == ctx->handles.end() || (it->second.kind != 1 && it->second.kind != 3))
    return fail(JT_EINVAL, "unknown subhalo handle %llu", (unsigned long long)h);
  *table = it->second.dev;
  *n = it->second.n;
  *tnfw = it->second.kind == 3;
  return JT_OK;
}

const SubRec* ctx_empty_table(jt_ctx* ctx) { return ctx->empty_table; }

}  // namespace jt

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
extern "C" jt_status jt_profile_enable(jt_ctx* ctx, int on) {
  JT_TRY(ctx_enter(ctx));
  std::lock_guard<std::mutex> lk(ctx->mu);
  drain_events(ctx);
  ctx->prof = on != 0;
  for (int i = 0; i < JT_K_COUNT; ++i) {
    ctx->prof_ms[i] = 0.0;
    ctx->prof_n[i] = 0;
  }
  return JT_OK;
}

extern "C" jt_status jt_profile_read(jt_ctx* ctx, int id, double* total_ms, int* launches) {
  JT_TRY(ctx_enter(ctx));
  if (id < 0 || id >= JT_K_COUNT || !total_ms || !launches) return fail(JT_EINVAL, "jt_profile_read: bad argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  drain_events(ctx);
  *total_ms = ctx->prof_ms[id];
  *launches = ctx->prof_n[id];
  return JT_OK;
}
