// Allocation-free fused simulation: jt_simulate_image_noalloc.
//
// The same kernels as jt_simulate_image (subhalo-table derivation, fused
// steps 1-2 with the supersample average, direct PSF convolution), with the
// two intermediate buffers -- the packed subhalo table and the unconvolved
// image -- carved from one file-scope device array instead of the context's
// workspace.  Nothing here calls hipMalloc, hipFree, hipEventCreate or any
// other allocating routine, so the call suits code under stream capture and
// loops that must not allocate.
//
// The array is one per device (each device that loads the code object holds
// its own copy for the life of the process).  Host code never names it after
// set-up: jt_create looks up its device address once per device with
// hipGetSymbolAddress, and kernels receive that address.  Every call on a
// device shares the device's array, so two calls that overlap on one device
// (different streams, or threads without ordering) race on it; calls on one
// stream are ordered and safe.  Nothing in the array needs to start at zero:
// the prep kernel writes every table record it later reads and the fused
// kernel writes every pixel of the unconvolved image.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/jt.h"
#include "jt_host.hpp"
#include "jt_kernels.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)JT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace jt {

// Looks up this device's copy of the array (the device must be current).
// Called by jt_create; later calls for the same device return at once.
jt_status noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(JT_EUNSUPPORTED, "static scratch: device %d", device);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_done[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_err[device] = e;
    g_ptr[device] = e == hipSuccess ? p : nullptr;
    g_done[device] = true;
  }
  if (g_err[device] != hipSuccess) return check_hip(g_err[device], "hipGetSymbolAddress(static scratch)");
  return JT_OK;
}

static jt_status noalloc_scratch(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= kMaxDevices || !g_done[device] || !g_ptr[device])
    return fail(JT_EDEVICE, "static scratch of device %d is unavailable (%s)", device,
                device >= 0 && device < kMaxDevices && g_done[device] ? hipGetErrorString(g_err[device])
                                                                       : "not looked up");
  *out = g_ptr[device];
  return JT_OK;
}

}  // namespace jt

using namespace jt;

extern "C" jt_status jt_simulate_image_noalloc(jt_ctx* ctx, const jt_grid* grid, const jt_lens* lens,
                                               const jt_light* src, const jt_light* lens_light, const float* psf,
                                               int k, float* out, hipStream_t stream) {
  JT_TRY(ctx_enter(ctx));
  GridC g;
  MacroC mc;
  LightC s, l;
  JT_TRY(make_grid(grid, g));
  JT_TRY(make_macro(lens, mc));
  JT_TRY(make_light(src, s, "source"));
  JT_TRY(make_light(lens_light, l, "lens light"));
  if (!out) return fail(JT_EINVAL, "simulate_noalloc: null output");
  if ((psf == nullptr) != (k == 0)) return fail(JT_EINVAL, "simulate_noalloc: psf and k must be given together");
  if (psf && (k < 1 || k % 2 == 0)) return fail(JT_EINVAL, "simulate_noalloc: PSF side %d must be odd", k);
  if (psf && k > JT_MAX_PSF)
    return fail(JT_EUNSUPPORTED, "simulate_noalloc: direct convolution only, k <= %d (got %d)", JT_MAX_PSF, k);
  if (psf && overlap(out, (size_t)g.nx * g.ny, psf, (size_t)k * k))
    return fail(JT_EINVAL, "simulate_noalloc: output overlaps the PSF");
  // scratch: [subhalo table][unconvolved image], each 256-byte aligned
  const size_t tab_bytes = subhalo_scratch_bytes(lens);
  const size_t img_bytes = psf ? ((sizeof(float) * (size_t)g.nx * g.ny + 255) & ~size_t(255)) : 0;
  if (tab_bytes + img_bytes > kScratchBytes)
    return fail(JT_EUNSUPPORTED,
                "simulate_noalloc: needs %zu bytes of static scratch (subhalo table %zu + image %zu), "
                "more than its %zu",
                tab_bytes + img_bytes, tab_bytes, img_bytes, kScratchBytes);
  void* base = nullptr;
  JT_TRY(noalloc_scratch(ctx->device, &base));
  char* ws = (char*)base;
  // the subhalo table: a resident handle, the caller's SoA packed into the
  // scratch, or the context's empty table
  const void* tab = nullptr;
  int nloop = 0;
  bool tnfw = false;
  if (lens->subhalo_handle) {
    int n = 0;
    JT_TRY(ctx_subhalo_handle(ctx, lens->subhalo_handle, &tab, &n, &tnfw));
    nloop = subhalo_loop_count(n);
  } else if (lens->nfw.n > 0) {
    const jt_nfw& sh = lens->nfw;
    if (sh.r_trunc) {
      JT_TRY(check_hip(launch_prep_tnfw(sh.n, sh.x, sh.y, sh.Rs, sh.alpha_Rs, sh.r_trunc, (TRec*)ws, stream),
                       "simulate_noalloc: prep_tnfw"));
      tnfw = true;
    } else {
      JT_TRY(check_hip(launch_prep_subhalos(sh.n, sh.x, sh.y, sh.Rs, sh.alpha_Rs, (SubRec*)ws, stream),
                       "simulate_noalloc: prep_subhalos"));
    }
    tab = ws;
    nloop = subhalo_loop_count(sh.n);
  } else {
    tab = ctx_empty_table(ctx);
  }
  float* img = psf ? (float*)(ws + tab_bytes) : out;
  JT_TRY(check_hip(launch_simulate(g, mc, tnfw, tab, nloop, s, l, img, stream), "simulate_noalloc: simulate"));
  if (!psf) return JT_OK;
  return check_hip(launch_conv_direct(img, g.nx, g.ny, psf, k, out, stream), "simulate_noalloc: conv_direct");
}
