// Batches of parameter draws: batched forward images, the chi^2
// log-likelihood and its hand-written adjoint (host side).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "jt_host.hpp"
#include "jt_kernels.hpp"

using namespace jt;

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Carve {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    T* p = (T*)(base + off);
    off += align256(count * sizeof(T));
    return p;
  }
};

// Everything a batch launch needs on the host: one ImageDesc per draw.
struct Batch {
  GridC g;
  int B = 0, n = 0, nloop = 0, records = 0, npix = 0, nsubpix = 0;
  int split = 1, bpi = 0, P = 0;
  bool epl = false, tnfw = false;   // EPL main deflector; truncated subhalos
  size_t rec_bytes = sizeof(SubRec);
  std::vector<ImageDesc> descs;
};

jt_status check_draws(const jt_draws* d, bool for_grad) {
  if (!d) return fail(JT_EINVAL, "null draws");
  if (d->B < 1) return fail(JT_EINVAL, "draws: B = %d", d->B);
  if ((!d->sie && !d->epl) || !d->shear) return fail(JT_EINVAL, "draws: null main-deflector or shear array");
  if (d->n_sub < 0) return fail(JT_EINVAL, "draws: n_sub = %d", d->n_sub);
  if (d->n_sub > 0 && (!d->sub_x || !d->sub_y || !d->sub_Rs || !d->sub_alpha_Rs))
    return fail(JT_EINVAL, "draws: null subhalo array");
  if (d->n_src < 0 || d->n_ll < 0) return fail(JT_EINVAL, "draws: negative component count");
  if (d->n_src > JT_MAX_SERSIC || d->n_ll > JT_MAX_SERSIC) return fail(JT_EUNSUPPORTED, "draws: too many components");
  if ((d->n_src > 0 && !d->src) || (d->n_ll > 0 && !d->ll)) return fail(JT_EINVAL, "draws: null Sersic array");
  if (for_grad && d->n_src + d->n_ll > 3)
    return fail(JT_EUNSUPPORTED, "gradient: %d Sersic components (max 3)", d->n_src + d->n_ll);
  return JT_OK;
}

jt_status make_batch(const jt_grid* grid, const jt_draws* d, bool for_grad, Batch& bt) {
  JT_TRY(check_draws(d, for_grad));
  JT_TRY(make_grid(grid, bt.g));
  bt.B = d->B;
  bt.n = d->n_sub;
  bt.nloop = subhalo_loop_count(bt.n);
  bt.records = subhalo_table_records(bt.n);
  bt.npix = bt.g.nx * bt.g.ny;
  bt.nsubpix = bt.npix * bt.g.s2;
  if ((double)bt.B * bt.nsubpix > 2147483647.0) return fail(JT_EUNSUPPORTED, "batch: too many sub-pixels");
  bt.split = pick_split((long)bt.B * bt.nsubpix, bt.g.s2, bt.nloop);
  bt.g.ppb = split_lanes(bt.split) / bt.g.s2;
  bt.bpi = (bt.npix + bt.g.ppb - 1) / bt.g.ppb;
  bt.epl = d->epl != nullptr;
  bt.tnfw = d->n_sub > 0 && d->sub_r_trunc != nullptr;
  bt.rec_bytes = bt.tnfw ? sizeof(TRec) : sizeof(SubRec);
  bt.P = (bt.epl ? 8 : 7) + 7 * (d->n_src + d->n_ll);
  bt.descs.resize(bt.B);
  for (int b = 0; b < bt.B; ++b) {
    jt_lens lens;
    std::memset(&lens, 0, sizeof(lens));
    if (bt.epl) {
      lens.has_epl = 1;
      lens.epl = d->epl[b];
    } else {
      lens.has_sie = 1;
      lens.sie = d->sie[b];
    }
    lens.has_shear = 1;
    lens.shear = d->shear[b];
    ImageDesc& D = bt.descs[b];
    std::memset(&D, 0, sizeof(D));
    JT_TRY(make_macro(&lens, D.mc));
    jt_light src{d->n_src, d->n_src ? d->src + (size_t)b * d->n_src : nullptr, 0};
    jt_light ll{d->n_ll, d->n_ll ? d->ll + (size_t)b * d->n_ll : nullptr, 0};
    JT_TRY(make_light(&src, D.src, "source"));
    JT_TRY(make_light(&ll, D.ll, "lens light"));
    D.g = bt.g;
    D.nloop = bt.nloop;
  }
  return JT_OK;
}

// Forward images: tables, descriptors, fused kernel, convolution.  Fills the
// device pointers of the descriptors from the carved workspace and uploads
// them.  model_u / model: [B][npix].
jt_status run_forward(jt_ctx* ctx, Batch& bt, const jt_draws* d, const float* psf, int k, void* tables,
                      ImageDesc* ddescs, float* model_u, float* model, hipStream_t st, float2* beta = nullptr) {
  for (int b = 0; b < bt.B; ++b) {
    bt.descs[b].sub = bt.n > 0 ? (const void*)((const char*)tables + bt.rec_bytes * (size_t)b * bt.records)
                               : (const void*)ctx_empty_table(ctx);
    bt.descs[b].img = model_u + (size_t)b * bt.npix;
    bt.descs[b].beta = beta ? beta + (size_t)b * bt.nsubpix : nullptr;
  }
  JT_TRY(ctx_upload(ctx, st, ddescs, bt.descs.data(), sizeof(ImageDesc) * bt.B));
  if (bt.n > 0 && bt.tnfw)
    JT_TRY(timed_launch(ctx, JT_K_PREP, st, [&] {
      return launch_prep_tnfw_batched(bt.B, bt.n, d->sub_x, d->sub_y, d->sub_Rs, d->sub_alpha_Rs, d->sub_r_trunc,
                                      false, (TRec*)tables, st);
    }, "prep_tnfw_batched"));
  else if (bt.n > 0)
    JT_TRY(timed_launch(ctx, JT_K_PREP, st, [&] {
      return launch_prep_subhalos_batched(bt.B, bt.n, d->sub_x, d->sub_y, d->sub_Rs, d->sub_alpha_Rs,
                                          (SubRec*)tables, st);
    }, "prep_subhalos_batched"));
  JT_TRY(timed_launch(ctx, JT_K_SIM, st, [&] {
    return launch_simulate_desc(bt.split, bt.tnfw, false, beta != nullptr, ddescs, nullptr, bt.B * bt.bpi, bt.bpi,
                                st);
  }, "simulate_batch"));
  if (psf && model != model_u)
    JT_TRY(timed_launch(ctx, JT_K_CONV, st, [&] {
      return launch_conv_direct_batched(false, bt.B, model_u, bt.npix, bt.g.nx, bt.g.ny, psf, k, model, bt.npix, st);
    }, "conv_batch"));
  return JT_OK;
}

jt_status check_psf(const float* psf, int k) {
  if ((psf == nullptr) != (k == 0)) return fail(JT_EINVAL, "psf and k must be given together");
  if (psf && (k < 1 || k % 2 == 0)) return fail(JT_EINVAL, "PSF side %d must be odd", k);
  if (k > JT_MAX_PSF) return fail(JT_EUNSUPPORTED, "direct convolution supports k <= %d", JT_MAX_PSF);
  return JT_OK;
}

}  // namespace

extern "C" jt_status jt_simulate_batch(jt_ctx* ctx, const jt_grid* grid, const jt_draws* draws, const float* psf,
                                       int k, float* out, hipStream_t stream) {
  JT_TRY(ctx_enter(ctx));
  Batch bt;
  JT_TRY(make_batch(grid, draws, false, bt));
  JT_TRY(check_psf(psf, k));
  if (!out) return fail(JT_EINVAL, "simulate_batch: null output");
  if (psf) {   // the convolution reads the PSF while it writes out
    const uintptr_t po = (uintptr_t)out, pp = (uintptr_t)psf;
    const size_t no = sizeof(float) * (size_t)bt.B * bt.npix, np = sizeof(float) * (size_t)k * k;
    if (po < pp + np && pp < po + no) return fail(JT_EINVAL, "simulate_batch: output overlaps the PSF");
  }
  const size_t bytes = align256(sizeof(ImageDesc) * bt.B) + align256(bt.rec_bytes * (size_t)bt.B * bt.records) +
                       align256(sizeof(float) * (size_t)bt.B * bt.npix);
  void* ws = nullptr;
  JT_TRY(ctx_workspace(ctx, stream, bytes, &ws));
  Carve cv{(char*)ws};
  ImageDesc* dd = cv.take<ImageDesc>(bt.B);
  void* tables = cv.take<char>(bt.rec_bytes * (size_t)bt.B * bt.records);
  float* mu = psf ? cv.take<float>((size_t)bt.B * bt.npix) : out;
  return run_forward(ctx, bt, draws, psf, k, tables, dd, mu, psf ? out : mu, stream);
}

namespace {

jt_status chi2_common(jt_ctx* ctx, const jt_grid* grid, const jt_draws* draws, const float* psf, int k,
                      const float* data, const float* inv_var, double* logL, float* g_macro, float* g_sub,
                      bool grad, hipStream_t st, bool keep = false) {
  JT_TRY(ctx_enter(ctx));
  Batch bt;
  JT_TRY(make_batch(grid, draws, grad, bt));
  JT_TRY(check_psf(psf, k));
  if (!data || !inv_var) return fail(JT_EINVAL, "chi2: null data or inverse variance");
  if (grad && !g_macro) return fail(JT_EINVAL, "chi2_grad: null g_macro");
  if (grad && bt.n > 0 && !g_sub) return fail(JT_EINVAL, "chi2_grad: null g_sub with n_sub > 0");
  if (!grad && !logL) return fail(JT_EINVAL, "chi2: null logL");
  const size_t BN = (size_t)bt.B * bt.npix;
  const int nres = (bt.npix + 255) / 256;
  const int nrec_loop = (bt.nsubpix + 3) & ~3;
  const int rec_stride = nrec_loop + 4;
  const int rec_parts = bt.tnfw ? kRecPartsTnfwHost + 1 : kRecPartsHost;   // + the truncated near pass
  size_t bytes = align256(sizeof(ImageDesc) * bt.B) + align256(bt.rec_bytes * (size_t)bt.B * bt.records) +
                 3 * align256(sizeof(float) * BN) + align256(sizeof(float) * (size_t)bt.B * nres);
  if (grad)
    bytes += align256(sizeof(float) * BN) + align256(sizeof(float4) * (size_t)bt.B * rec_stride) +
             align256(sizeof(float) * (size_t)bt.B * bt.bpi * bt.P) +
             align256(sizeof(float) * (size_t)rec_parts * bt.B * bt.n * 3) +
             (keep ? align256(sizeof(float2) * (size_t)bt.B * bt.nsubpix) : 0) +
             (bt.tnfw ? align256(sizeof(TRec) * (size_t)bt.B * bt.records) : 0);
  void* ws = nullptr;
  JT_TRY(ctx_workspace(ctx, st, bytes, &ws));
  Carve cv{(char*)ws};
  ImageDesc* dd = cv.take<ImageDesc>(bt.B);
  void* tables = cv.take<char>(bt.rec_bytes * (size_t)bt.B * bt.records);
  float* mu = cv.take<float>(BN);
  float* model = psf ? cv.take<float>(BN) : mu;
  float* resid = cv.take<float>(BN);
  float* lpart = cv.take<float>((size_t)bt.B * nres);
  // the kept variant of the gradient reads the forward's traced positions back
  // instead of recomputing them
  float2* beta = keep ? cv.take<float2>((size_t)bt.B * bt.nsubpix) : nullptr;
  JT_TRY(run_forward(ctx, bt, draws, psf, k, tables, dd, mu, model, st, beta));
  int nb = 0;
  JT_TRY(timed_launch(ctx, JT_K_GRAD, st, [&] {
    return launch_residual(bt.B, bt.npix, model, data, inv_var, resid, lpart, &nb, st);
  }, "residual"));
  if (!grad)
    return timed_launch(ctx, JT_K_GRAD, st, [&] {
      return launch_grad_finalize(bt.B, 0, 0, nullptr, nullptr, nres, lpart, logL, 0, 0, nullptr, nullptr, st);
    }, "chi2_finalize");
  float* lamU = psf ? cv.take<float>(BN) : resid;
  float4* rec = cv.take<float4>((size_t)bt.B * rec_stride);
  float* part = cv.take<float>((size_t)bt.B * bt.bpi * bt.P);
  float* gpart = cv.take<float>((size_t)rec_parts * bt.B * bt.n * 3);
  if (psf)
    JT_TRY(timed_launch(ctx, JT_K_CONV, st, [&] {
      return launch_conv_direct_batched(true, bt.B, resid, bt.npix, bt.g.nx, bt.g.ny, psf, k, lamU, bt.npix, st);
    }, "conv_adjoint"));
  JT_TRY(timed_launch(ctx, JT_K_GRAD, st, [&] {
    return launch_grad_pixel(bt.split, keep, bt.tnfw, bt.epl, bt.B, bt.bpi, dd, lamU, rec, rec_stride, part, bt.P,
                             st);
  }, "grad_pixel"));
  if (bt.tnfw) {
    // per-lane constants of the truncated subhalos, for alpha_Rs = 1
    TRec* utab = cv.take<TRec>((size_t)bt.B * bt.records);
    JT_TRY(timed_launch(ctx, JT_K_PREP, st, [&] {
      return launch_prep_tnfw_batched(bt.B, bt.n, draws->sub_x, draws->sub_y, draws->sub_Rs, draws->sub_alpha_Rs,
                                      draws->sub_r_trunc, true, utab, st);
    }, "prep_tnfw_unit"));
    JT_TRY(timed_launch(ctx, JT_K_GRAD, st, [&] {
      return launch_grad_subhalo_tnfw(bt.B, bt.n, utab, bt.records, draws->sub_alpha_Rs, rec, rec_stride, nrec_loop,
                                      bt.g, gpart, st);
    }, "grad_subhalo_tnfw"));
  } else {
    JT_TRY(timed_launch(ctx, JT_K_GRAD, st, [&] {
      return launch_grad_subhalo(bt.B, bt.n, draws->sub_x, draws->sub_y, draws->sub_Rs, draws->sub_alpha_Rs, rec,
                                 rec_stride, nrec_loop, gpart, st);
    }, "grad_subhalo"));
  }
  return timed_launch(ctx, JT_K_GRAD, st, [&] {
    return launch_grad_finalize(bt.B, bt.P, bt.bpi, part, g_macro, nres, lpart, logL, bt.n, rec_parts, gpart,
                                bt.n > 0 ? g_sub : nullptr, st);
  }, "grad_finalize");
}

}  // namespace

extern "C" jt_status jt_chi2(jt_ctx* ctx, const jt_grid* grid, const jt_draws* draws, const float* psf, int k,
                             const float* data, const float* inv_var, double* logL, hipStream_t stream) {
  return chi2_common(ctx, grid, draws, psf, k, data, inv_var, logL, nullptr, nullptr, false, stream);
}

extern "C" jt_status jt_chi2_grad(jt_ctx* ctx, const jt_grid* grid, const jt_draws* draws, const float* psf,
                                  int k, const float* data, const float* inv_var, double* logL, float* g_macro,
                                  float* g_sub, hipStream_t stream) {
  return chi2_common(ctx, grid, draws, psf, k, data, inv_var, logL, g_macro, g_sub, true, stream);
}

extern "C" jt_status jt_chi2_grad_kept(jt_ctx* ctx, const jt_grid* grid, const jt_draws* draws, const float* psf,
                                       int k, const float* data, const float* inv_var, double* logL, float* g_macro,
                                       float* g_sub, hipStream_t stream) {
  return chi2_common(ctx, grid, draws, psf, k, data, inv_var, logL, g_macro, g_sub, true, stream, true);
}
