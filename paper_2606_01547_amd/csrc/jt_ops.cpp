// The compute entry points of the C ABI: ray shooting, surface brightness,
// convolution and the fused simulation.  Each validates its arguments (no
// launch on error) and enqueues kernels on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "jt_host.hpp"
#include "jt_kernels.hpp"

using namespace jt;

namespace {

jt_status ray_common(bool alpha, jt_ctx* ctx, int n, const float* x, const float* y, const jt_lens* lens,
                     float* ox, float* oy, hipStream_t st) {
  JT_TRY(ctx_enter(ctx));
  if (n < 0) return fail(JT_EINVAL, "ray_shoot: n = %d", n);
  MacroC mc;
  JT_TRY(make_macro(lens, mc));
  if (n == 0) return JT_OK;
  if (!x || !y || !ox || !oy) return fail(JT_EINVAL, "ray_shoot: null array");
  const size_t N = (size_t)n;
  if (overlap(ox, N, x, N) || overlap(ox, N, y, N) || overlap(oy, N, x, N) || overlap(oy, N, y, N) ||
      overlap(ox, N, oy, N))
    return fail(JT_EINVAL, "ray_shoot: outputs overlap the inputs or each other");
  void* scratch = nullptr;
  const size_t tab_bytes = subhalo_scratch_bytes(lens);
  if (tab_bytes) JT_TRY(ctx_workspace(ctx, st, tab_bytes, &scratch));
  const void* tab = nullptr;
  int nloop = 0;
  bool tnfw = false;
  JT_TRY(resolve_subhalos(ctx, lens, scratch, st, &tab, &nloop, &tnfw));
  return timed_launch(ctx, JT_K_RAY, st,
                      [&] { return launch_ray_shoot(alpha, tnfw, n, x, y, mc, tab, nloop, ox, oy, st); },
                      "ray_shoot");
}

jt_status check_conv_args(const float* img, int nx, int ny, const float* psf, int k, const float* out) {
  if (!img || !out || !psf) return fail(JT_EINVAL, "convolve: null pointer");
  if (nx < 1 || ny < 1) return fail(JT_EINVAL, "convolve: %d x %d image", nx, ny);
  if (k < 1 || k % 2 == 0) return fail(JT_EINVAL, "convolve: PSF side %d must be odd", k);
  const size_t npix = (size_t)std::max(nx, 0) * (size_t)std::max(ny, 0);
  if (overlap(out, npix, img, npix) || overlap(out, npix, psf, (size_t)k * k))
    return fail(JT_EINVAL, "convolve: output overlaps the image or the PSF");
  if ((double)nx * ny > 2147483647.0) return fail(JT_EUNSUPPORTED, "convolve: image too large");
  return JT_OK;
}

}  // namespace

namespace jt {
// Direct or FFT for method 0: the FFT path once its modelled time is lower,
// or when the direct path cannot take k.
bool conv_prefers_fft(int nx, int ny, int k) {
  const bool fft_ok = fft_size_for(nx, k) <= kFftMaxN && fft_size_for(ny, k) <= kFftMaxN;
  if (!fft_ok) return false;
  if (k > JT_MAX_PSF) return true;
  const ConvShape sh = conv_shape(nx, ny, k);
  const double waves = (double)conv_tiles_x(nx, sh) * conv_tiles_y(ny) * sh.nc * sh.s;
  const double rate = std::min(kConvMfmaMacPerS, waves * kConvMfmaMacPerWaveS);
  const double macs = (double)nx * ny * (16.0 + k - 1) * (double)((k + 3) & ~3);
  const double direct_s = kConvDirectFixedS + macs / rate;
  const double N2 = (double)fft_size_for(nx, k) * fft_size_for(ny, k);
  const double fft_s = kConvFftFixedS + N2 / kConvFftPointsPerS;
  return fft_s < direct_s;
}
}  // namespace jt

namespace {

jt_status convolve_on(jt_ctx* ctx, const float* img, int nx, int ny, const float* psf, int k, int method,
                      float* out, hipStream_t st) {
  if (method < 0 || method > 2) return fail(JT_EINVAL, "convolve: method %d", method);
  if (method == 0) method = conv_prefers_fft(nx, ny, k) ? 2 : 1;
  if (method == 1) {
    if (k > JT_MAX_PSF) return fail(JT_EUNSUPPORTED, "convolve: direct path supports k <= %d", JT_MAX_PSF);
    return timed_launch(ctx, JT_K_CONV, st,
                        [&] { return launch_conv_direct(img, nx, ny, psf, k, out, st); }, "conv_direct");
  }
  const int Nx = fft_size_for(nx, k), Ny = fft_size_for(ny, k);
  if (Nx > kFftMaxN || Ny > kFftMaxN)
    return fail(JT_EUNSUPPORTED, "convolve: FFT path supports padded sizes up to %d", kFftMaxN);
  const double2 *twx = nullptr, *twy = nullptr;
  JT_TRY(ctx_twiddles(ctx, Nx, &twx));
  JT_TRY(ctx_twiddles(ctx, Ny, &twy));
  void* ws = nullptr;
  JT_TRY(ctx_workspace_aux(ctx, st, fft_workspace_bytes(nx, ny, k), &ws));
  return timed_launch(ctx, JT_K_CONV, st,
                      [&] { return launch_fft_convolve(img, nx, ny, psf, k, out, ws, twx, twy, st); }, "conv_fft");
}

}  // namespace

extern "C" jt_status jt_ray_shoot(jt_ctx* ctx, int n, const float* x, const float* y, const jt_lens* lens,
                                  float* bx, float* by, hipStream_t stream) {
  return ray_common(false, ctx, n, x, y, lens, bx, by, stream);
}

extern "C" jt_status jt_deflection(jt_ctx* ctx, int n, const float* x, const float* y, const jt_lens* lens,
                                   float* ax, float* ay, hipStream_t stream) {
  return ray_common(true, ctx, n, x, y, lens, ax, ay, stream);
}

extern "C" jt_status jt_source_sb(jt_ctx* ctx, int n, const float* x, const float* y, const float* bx,
                                  const float* by, const jt_light* src, const jt_light* lens_light, float* sb,
                                  hipStream_t stream) {
  JT_TRY(ctx_enter(ctx));
  if (n < 0) return fail(JT_EINVAL, "source_sb: n = %d", n);
  LightC s, l;
  JT_TRY(make_light(src, s, "source"));
  JT_TRY(make_light(lens_light, l, "lens light"));
  if (n == 0) return JT_OK;
  if (!sb) return fail(JT_EINVAL, "source_sb: null output");
  if (light_any(s) && (!bx || !by)) return fail(JT_EINVAL, "source_sb: null traced coordinates");
  if (light_any(l) && (!x || !y)) return fail(JT_EINVAL, "source_sb: null image-plane coordinates");
  // in place is fine (each element is read before its own output is written)
  for (const float* p : {light_any(s) ? bx : nullptr, light_any(s) ? by : nullptr, light_any(l) ? x : nullptr,
                         light_any(l) ? y : nullptr})
    if (p != sb && overlap(sb, (size_t)n, p, (size_t)n))
      return fail(JT_EINVAL, "source_sb: output overlaps an input without being it");
  const float* zx = bx ? bx : x;  // unused when the matching list is empty
  const float* zy = by ? by : y;
  return timed_launch(ctx, JT_K_SB, stream,
                      [&] { return launch_source_sb(n, x ? x : zx, y ? y : zy, zx, zy, s, l, sb, stream); },
                      "source_sb");
}

extern "C" jt_status jt_convolve(jt_ctx* ctx, const float* img, int nx, int ny, const float* psf, int k,
                                 int method, float* out, hipStream_t stream) {
  JT_TRY(ctx_enter(ctx));
  JT_TRY(check_conv_args(img, nx, ny, psf, k, out));
  return convolve_on(ctx, img, nx, ny, psf, k, method, out, stream);
}

extern "C" int jt_convolve_auto_method(int nx, int ny, int k) {
  if (nx < 1 || ny < 1 || k < 1 || k % 2 == 0) return 0;
  if (conv_prefers_fft(nx, ny, k)) return 2;
  return k <= JT_MAX_PSF ? 1 : 0;
}

extern "C" jt_status jt_simulate_image(jt_ctx* ctx, const jt_grid* grid, const jt_lens* lens,
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
  if (!out) return fail(JT_EINVAL, "simulate: null output");
  if ((psf == nullptr) != (k == 0)) return fail(JT_EINVAL, "simulate: psf and k must be given together");
  if (psf && (k < 1 || k % 2 == 0)) return fail(JT_EINVAL, "simulate: PSF side %d must be odd", k);
  if (psf && overlap(out, (size_t)g.nx * g.ny, psf, (size_t)k * k))
    return fail(JT_EINVAL, "simulate: output overlaps the PSF");
  // workspace: [subhalo table][unconvolved image]
  const size_t tab_bytes = subhalo_scratch_bytes(lens);
  const size_t img_bytes = psf ? sizeof(float) * (size_t)g.nx * g.ny : 0;
  char* ws = nullptr;
  if (tab_bytes + img_bytes > 0) {
    void* p = nullptr;
    JT_TRY(ctx_workspace(ctx, stream, tab_bytes + img_bytes, &p));
    ws = (char*)p;
  }
  const void* tab = nullptr;
  int nloop = 0;
  bool tnfw = false;
  JT_TRY(resolve_subhalos(ctx, lens, tab_bytes ? ws : nullptr, stream, &tab, &nloop, &tnfw));
  float* img = psf ? (float*)(ws + tab_bytes) : out;
  JT_TRY(timed_launch(ctx, JT_K_SIM, stream,
                      [&] { return launch_simulate(g, mc, tnfw, tab, nloop, s, l, img, stream); }, "simulate"));
  if (!psf) return JT_OK;
  return convolve_on(ctx, img, g.nx, g.ny, psf, k, 0, out, stream);
}

extern "C" jt_status jt_linear_amplitudes(jt_ctx* ctx, const jt_grid* grid, const jt_lens* lens,
                                          const jt_light* src, const jt_light* lens_light, const float* psf, int k,
                                          const float* data, const float* inv_var, double* amps, float* model,
                                          double* logL, hipStream_t stream) {
  JT_TRY(ctx_enter(ctx));
  GridC g;
  MacroC mc;
  LightC s, l;
  JT_TRY(make_grid(grid, g));
  JT_TRY(make_macro(lens, mc));
  JT_TRY(make_light(src, s, "source"));
  JT_TRY(make_light(lens_light, l, "lens light"));
  const int n = s.n + l.n;
  if (s.ng | s.ncs | s.nsh | l.ng | l.ncs | l.nsh)
    return fail(JT_EUNSUPPORTED, "linear amplitudes: Sersic components only");
  if (n < 1) return fail(JT_EINVAL, "linear amplitudes: no light component");
  if (n > kMaxBasis) return fail(JT_EUNSUPPORTED, "linear amplitudes: %d components (max %d)", n, kMaxBasis);
  if (!data || !inv_var || !amps) return fail(JT_EINVAL, "linear amplitudes: null data, weights or amplitudes");
  if ((psf == nullptr) != (k == 0)) return fail(JT_EINVAL, "linear amplitudes: psf and k must be given together");
  if (psf && (k < 1 || k % 2 == 0)) return fail(JT_EINVAL, "linear amplitudes: PSF side %d must be odd", k);
  const long npix = (long)g.nx * g.ny;
  if ((double)npix * n > 2147483647.0) return fail(JT_EUNSUPPORTED, "linear amplitudes: basis too large");
  // workspace: [subhalo table][basis n x npix][convolved basis][solver partials]
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t tab_bytes = subhalo_scratch_bytes(lens);
  const size_t basis_bytes = al(sizeof(float) * (size_t)n * npix);
  const size_t conv_bytes = psf ? basis_bytes : 0;
  const size_t part_bytes = al(sizeof(double) * (size_t)kLinBlocks * (kLinTerms + 1));
  void* p = nullptr;
  JT_TRY(ctx_workspace(ctx, stream, tab_bytes + basis_bytes + conv_bytes + part_bytes, &p));
  char* ws = (char*)p;
  float* basis = (float*)(ws + tab_bytes);
  float* conv = psf ? (float*)(ws + tab_bytes + basis_bytes) : basis;
  double* part = (double*)(ws + tab_bytes + basis_bytes + conv_bytes);
  const void* tab = nullptr;
  int nloop = 0;
  bool tnfw = false;
  JT_TRY(resolve_subhalos(ctx, lens, tab_bytes ? ws : nullptr, stream, &tab, &nloop, &tnfw));
  JT_TRY(timed_launch(ctx, JT_K_SIM, stream,
                      [&] { return launch_simulate_basis(g, mc, tnfw, tab, nloop, s, l, basis, stream); },
                      "simulate_basis"));
  if (psf) {
    if (!conv_prefers_fft(g.nx, g.ny, k) && k <= JT_MAX_PSF) {
      JT_TRY(timed_launch(ctx, JT_K_CONV, stream, [&] {
        return launch_conv_direct_batched(false, n, basis, npix, g.nx, g.ny, psf, k, conv, npix, stream);
      }, "conv_basis"));
    } else {
      for (int j = 0; j < n; ++j)
        JT_TRY(convolve_on(ctx, basis + (size_t)j * npix, g.nx, g.ny, psf, k, 2, conv + (size_t)j * npix, stream));
    }
  }
  return check_hip(launch_linear_solve((int)npix, n, conv, data, inv_var, part, amps, model, logL, stream),
                   "linear_solve");
}
