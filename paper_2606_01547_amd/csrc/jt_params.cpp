// Host parameter preparation: validates the ABI structs and turns FP64
// parameters into the FP32 constants the kernels consume.
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "jt_host.hpp"
#include "jt_kernels.hpp"

namespace jt {

namespace {
bool finite(double v) { return std::isfinite(v); }
}  // namespace

// ---------------------------------------------------------------------------
// regularised incomplete gamma and the exact Sersic b_n
// ---------------------------------------------------------------------------
// P(a, x) by its power series for x < a + 1 (Abramowitz & Stegun 6.5.29) and
// otherwise through Q = 1 - P from Legendre's continued fraction
// (A&S 6.5.31), evaluated with the modified Lentz method.
double gamma_p(double a, double x) {
  if (!(x > 0.0)) return 0.0;
  const double lpref = a * std::log(x) - x - std::lgamma(a);
  if (x < a + 1.0) {
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 100000; ++n) {
      term *= x / (a + n);
      sum += term;
      if (std::fabs(term) < std::fabs(sum) * 1e-17) break;
    }
    return sum * std::exp(lpref);
  }
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 100000; ++i) {
    const double an = -i * (i - a);
    b += 2.0;
    d = an * d + b;
    if (std::fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (std::fabs(del - 1.0) < 1e-16) break;
  }
  return 1.0 - std::exp(lpref) * h;
}

double sersic_bn_exact(double n) {
  const double a = 2.0 * n;
  double lo = 0.0, hi = std::numeric_limits<double>::infinity();
  double b = std::fmax(a - 1.0 / 3.0 + 8.0 / (405.0 * a), 1e-3);
  for (int it = 0; it < 200; ++it) {
    const double f = gamma_p(a, b) - 0.5;
    if (f > 0.0) hi = b; else lo = b;
    const double dens = std::exp((a - 1.0) * std::log(b) - b - std::lgamma(a));
    double nb = b - f / dens;
    if (!(nb > lo && nb < hi)) nb = std::isinf(hi) ? 2.0 * b + 1.0 : 0.5 * (lo + hi);
    if (std::fabs(nb - b) <= 1e-15 * b) return nb;
    b = nb;
  }
  return b;
}

// ---------------------------------------------------------------------------
// lens
// ---------------------------------------------------------------------------
jt_status make_macro(const jt_lens* lens, MacroC& m) {
  std::memset(&m, 0, sizeof(m));
  if (!lens) return fail(JT_EINVAL, "null lens");
  if (lens->has_sie) {
    const jt_sie& s = lens->sie;
    if (!finite(s.theta_E) || !finite(s.q) || !finite(s.phi) || !finite(s.cx) || !finite(s.cy))
      return fail(JT_EINVAL, "SIE: non-finite parameter");
    if (s.theta_E < 0.0) return fail(JT_EINVAL, "SIE: theta_E = %g < 0", s.theta_E);
    if (!(s.q > 0.0 && s.q <= 1.0)) return fail(JT_EINVAL, "SIE: q = %g not in (0, 1]", s.q);
    const double f = std::sqrt((1.0 - s.q) * (1.0 + s.q));
    const double pref = s.theta_E * std::sqrt(s.q);
    m.has_sie = 1;
    m.sie_series = f < 1e-3;
    m.cx = (float)s.cx;
    m.cy = (float)s.cy;
    m.cphi = (float)std::cos(s.phi);
    m.sphi = (float)std::sin(s.phi);
    m.q2 = (float)(s.q * s.q);
    m.f = (float)f;
    m.dcx = s.cx;
    m.dcy = s.cy;
    m.dcphi = std::cos(s.phi);
    m.dsphi = std::sin(s.phi);
    m.dq2 = s.q * s.q;
    m.df = f;
    m.dpref = pref;
    m.dpref_f = f > 0.0 ? pref / f : 0.0;
    m.theta_E = (float)s.theta_E;
    m.q = (float)s.q;
    m.sqrt_q = (float)std::sqrt(s.q);
  }
  if (lens->has_epl) {
    const jt_epl& e = lens->epl;
    if (!finite(e.theta_E) || !finite(e.gamma) || !finite(e.q) || !finite(e.phi) || !finite(e.cx) || !finite(e.cy))
      return fail(JT_EINVAL, "EPL: non-finite parameter");
    if (e.theta_E < 0.0) return fail(JT_EINVAL, "EPL: theta_E = %g < 0", e.theta_E);
    if (!(e.gamma > 1.0 && e.gamma < 3.0)) return fail(JT_EINVAL, "EPL: gamma = %g not in (1, 3)", e.gamma);
    if (!(e.q > 0.0 && e.q <= 1.0)) return fail(JT_EINVAL, "EPL: q = %g not in (0, 1]", e.q);
    if (e.q < 0.05) return fail(JT_EUNSUPPORTED, "EPL: q = %g below 0.05 (series too long)", e.q);
    const double t = e.gamma - 1.0, b = e.theta_E * std::sqrt(e.q);
    m.has_epl = e.theta_E > 0.0;
    m.ecx = e.cx;
    m.ecy = e.cy;
    m.ecphi = std::cos(e.phi);
    m.esphi = std::sin(e.phi);
    m.eq = e.q;
    m.ef = (1.0 - e.q) / (1.0 + e.q);
    m.e2mt = 2.0 - t;
    m.eb = b;
    m.etm1 = t - 1.0;
    m.epref = 2.0 * b / (1.0 + e.q);
    m.e_te = e.theta_E;
    m.e_gamma = e.gamma;
    m.e_phi = e.phi;
  }
  if (lens->has_shear) {
    if (!finite(lens->shear.gamma1) || !finite(lens->shear.gamma2))
      return fail(JT_EINVAL, "shear: non-finite parameter");
    m.has_shear = 1;
    m.g1 = (float)lens->shear.gamma1;
    m.g2 = (float)lens->shear.gamma2;
    m.dg1 = lens->shear.gamma1;
    m.dg2 = lens->shear.gamma2;
  }
  const jt_point_masses& pm = lens->pm;
  if (pm.n < 0 || pm.n > JT_MAX_POINT_MASS)
    return fail(pm.n < 0 ? JT_EINVAL : JT_EUNSUPPORTED, "point masses: n = %d (max %d)", pm.n, JT_MAX_POINT_MASS);
  if (pm.n > 0 && (!pm.x || !pm.y || !pm.theta_E)) return fail(JT_EINVAL, "point masses: null array");
  for (int k = 0; k < pm.n; ++k) {
    if (!finite(pm.x[k]) || !finite(pm.y[k]) || !finite(pm.theta_E[k]))
      return fail(JT_EINVAL, "point mass %d: non-finite parameter", k);
    m.pm_x[k] = pm.x[k];
    m.pm_y[k] = pm.y[k];
    m.pm_te2[k] = pm.theta_E[k] * pm.theta_E[k];
  }
  m.npm = pm.n;
  if (lens->nfw.n < 0) return fail(JT_EINVAL, "NFW: n = %d", lens->nfw.n);
  if (!lens->subhalo_handle && lens->nfw.n > 0 &&
      (!lens->nfw.x || !lens->nfw.y || !lens->nfw.Rs || !lens->nfw.alpha_Rs))
    return fail(JT_EINVAL, "NFW: null device array");
  return JT_OK;
}

jt_status pack_subhalos_host(int n, const float* x, const float* y, const float* rs, const float* ars,
                             std::vector<SubRec>& out) {
  out.assign(subhalo_table_records(n), kSubRecPad);
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || !std::isfinite(ars[i]))
      return fail(JT_EINVAL, "subhalo %d: non-finite parameter", i);
    if (!(rs[i] > 0.0f) || !std::isfinite(rs[i])) return fail(JT_EINVAL, "subhalo %d: Rs = %g", i, (double)rs[i]);
    out[i] = make_subrec(x[i], y[i], rs[i], ars[i]);
  }
  return JT_OK;
}

jt_status validate_tnfw_host(int n, const float* x, const float* y, const float* rs, const float* ars,
                             const float* rt) {
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || !std::isfinite(ars[i]))
      return fail(JT_EINVAL, "subhalo %d: non-finite parameter", i);
    if (!(rs[i] > 0.0f) || !std::isfinite(rs[i])) return fail(JT_EINVAL, "subhalo %d: Rs = %g", i, (double)rs[i]);
    if (!(rt[i] > 0.0f) || !std::isfinite(rt[i]))
      return fail(JT_EINVAL, "subhalo %d: r_trunc = %g", i, (double)rt[i]);
  }
  return JT_OK;
}

size_t subhalo_scratch_bytes(const jt_lens* lens) {
  if (lens->subhalo_handle || lens->nfw.n <= 0) return 0;
  const size_t rec = lens->nfw.r_trunc ? sizeof(TRec) : sizeof(SubRec);
  return (rec * (size_t)subhalo_table_records(lens->nfw.n) + 255) & ~size_t(255);
}

jt_status resolve_subhalos(jt_ctx* ctx, const jt_lens* lens, void* scratch, hipStream_t st, const void** table,
                           int* nloop, bool* tnfw) {
  *tnfw = false;
  if (lens->subhalo_handle) {
    int n = 0;
    JT_TRY(ctx_subhalo_handle(ctx, lens->subhalo_handle, table, &n, tnfw));
    *nloop = subhalo_loop_count(n);
    return JT_OK;
  }
  const jt_nfw& s = lens->nfw;
  if (s.n > 0) {
    if (!scratch) return fail(JT_EINVAL, "internal: no scratch for the subhalo table");
    if (s.r_trunc) {
      JT_TRY(timed_launch(ctx, JT_K_PREP, st,
                          [&] { return launch_prep_tnfw(s.n, s.x, s.y, s.Rs, s.alpha_Rs, s.r_trunc, (TRec*)scratch, st); },
                          "prep_tnfw"));
      *tnfw = true;
    } else {
      JT_TRY(timed_launch(ctx, JT_K_PREP, st,
                          [&] { return launch_prep_subhalos(s.n, s.x, s.y, s.Rs, s.alpha_Rs, (SubRec*)scratch, st); },
                          "prep_subhalos"));
    }
    *table = scratch;
    *nloop = subhalo_loop_count(s.n);
    return JT_OK;
  }
  *table = ctx_empty_table(ctx);
  *nloop = 0;
  return JT_OK;
}

// ---------------------------------------------------------------------------
// light
// ---------------------------------------------------------------------------
namespace {
void set_frame(double phi, double q, double cx, double cy, float& fcx, float& fcy, float& cphi, float& sphi, float& fq,
               float& inv_q) {
  fcx = (float)cx;
  fcy = (float)cy;
  cphi = (float)std::cos(phi);
  sphi = (float)std::sin(phi);
  fq = (float)q;
  inv_q = (float)(1.0 / q);
}
}  // namespace

jt_status make_light(const jt_light* light, LightC& out, const char* which) {
  std::memset(&out, 0, sizeof(out));
  if (!light) return JT_OK;
  if (light->n < 0 || light->n_gauss < 0 || light->n_core < 0)
    return fail(JT_EINVAL, "%s: negative component count", which);
  if (light->n > JT_MAX_SERSIC) return fail(JT_EUNSUPPORTED, "%s: %d components (max %d)", which, light->n, JT_MAX_SERSIC);
  if (light->n > 0 && !light->c) return fail(JT_EINVAL, "%s: null component array", which);
  for (int k = 0; k < light->n; ++k) {
    const jt_sersic& c = light->c[k];
    if (!finite(c.amp) || !finite(c.R_sersic) || !finite(c.n_sersic) || !finite(c.q) || !finite(c.phi) ||
        !finite(c.cx) || !finite(c.cy))
      return fail(JT_EINVAL, "%s[%d]: non-finite parameter", which, k);
    if (!(c.R_sersic > 0.0)) return fail(JT_EINVAL, "%s[%d]: R_sersic = %g", which, k, c.R_sersic);
    if (!(c.n_sersic >= 0.2 && c.n_sersic <= 10.0)) return fail(JT_EINVAL, "%s[%d]: n_sersic = %g not in [0.2, 10]", which, k, c.n_sersic);
    if (!(c.q > 0.0 && c.q <= 1.0)) return fail(JT_EINVAL, "%s[%d]: q = %g not in (0, 1]", which, k, c.q);
    const double b = light->bn_exact ? sersic_bn_exact(c.n_sersic) : 1.9992 * c.n_sersic - 0.3271;
    SersicC& o = out.c[k];
    set_frame(c.phi, c.q, c.cx, c.cy, o.cx, o.cy, o.cphi, o.sphi, o.q, o.inv_q);
    o.inv_r2 = (float)(1.0 / (c.R_sersic * c.R_sersic));
    o.e = (float)(0.5 / c.n_sersic);
    o.kb = (float)(b / kLn2d);
    o.amp = (float)c.amp;
    o.R = (float)c.R_sersic;
    o.n = (float)c.n_sersic;
    o.b = (float)b;
  }
  out.n = light->n;
  // Gaussians
  if (light->n_gauss > kMaxGauss)
    return fail(JT_EUNSUPPORTED, "%s: %d Gaussians (max %d)", which, light->n_gauss, kMaxGauss);
  if (light->n_gauss > 0 && !light->gauss) return fail(JT_EINVAL, "%s: null Gaussian array", which);
  for (int k = 0; k < light->n_gauss; ++k) {
    const jt_gaussian& c = light->gauss[k];
    if (!finite(c.amp) || !finite(c.sigma) || !finite(c.q) || !finite(c.phi) || !finite(c.cx) || !finite(c.cy))
      return fail(JT_EINVAL, "%s Gaussian %d: non-finite parameter", which, k);
    if (!(c.sigma > 0.0)) return fail(JT_EINVAL, "%s Gaussian %d: sigma = %g", which, k, c.sigma);
    if (!(c.q > 0.0 && c.q <= 1.0)) return fail(JT_EINVAL, "%s Gaussian %d: q = %g not in (0, 1]", which, k, c.q);
    GaussC& o = out.g[k];
    set_frame(c.phi, c.q, c.cx, c.cy, o.cx, o.cy, o.cphi, o.sphi, o.q, o.inv_q);
    o.k = (float)(1.0 / (kLn2d * 2.0 * c.sigma * c.sigma));
    o.norm = (float)(c.amp / (2.0 * M_PI * c.sigma * c.sigma));
  }
  out.ng = light->n_gauss;
  // core-Sersic components
  if (light->n_core > kMaxCore)
    return fail(JT_EUNSUPPORTED, "%s: %d core-Sersic components (max %d)", which, light->n_core, kMaxCore);
  if (light->n_core > 0 && !light->core) return fail(JT_EINVAL, "%s: null core-Sersic array", which);
  for (int k = 0; k < light->n_core; ++k) {
    const jt_core_sersic& c = light->core[k];
    if (!finite(c.amp) || !finite(c.R_sersic) || !finite(c.R_b) || !finite(c.n_sersic) || !finite(c.gamma) ||
        !finite(c.alpha) || !finite(c.q) || !finite(c.phi) || !finite(c.cx) || !finite(c.cy))
      return fail(JT_EINVAL, "%s core-Sersic %d: non-finite parameter", which, k);
    if (!(c.R_sersic > 0.0) || !(c.R_b > 0.0)) return fail(JT_EINVAL, "%s core-Sersic %d: radii must be > 0", which, k);
    if (!(c.n_sersic >= 0.2 && c.n_sersic <= 10.0)) return fail(JT_EINVAL, "%s core-Sersic %d: n_sersic = %g", which, k, c.n_sersic);
    if (!(c.gamma >= 0.0 && c.gamma < 2.0)) return fail(JT_EINVAL, "%s core-Sersic %d: gamma = %g not in [0, 2)", which, k, c.gamma);
    if (!(c.alpha > 0.0 && c.alpha <= 20.0)) return fail(JT_EINVAL, "%s core-Sersic %d: alpha = %g not in (0, 20]", which, k, c.alpha);
    if (!(c.q > 0.0 && c.q <= 1.0)) return fail(JT_EINVAL, "%s core-Sersic %d: q = %g not in (0, 1]", which, k, c.q);
    const double b = light->bn_exact ? sersic_bn_exact(c.n_sersic) : 1.9992 * c.n_sersic - 0.3271;
    CoreC& o = out.cs[k];
    set_frame(c.phi, c.q, c.cx, c.cy, o.cx, o.cy, o.cphi, o.sphi, o.q, o.inv_q);
    o.half_alpha = (float)(0.5 * c.alpha);
    o.lRb = (float)(c.alpha * std::log2(c.R_b));
    o.lRe = (float)(c.alpha * std::log2(c.R_sersic));
    o.g_over_a = (float)(c.gamma / c.alpha);
    o.e = (float)(1.0 / (c.n_sersic * c.alpha));
    o.kb = (float)(b / kLn2d);
    o.amp = (float)c.amp;
    o.R2_floor = (float)(1e-12 * c.R_b * c.R_b);
  }
  out.ncs = light->n_core;
  // shapelets
  if (light->shapelets) {
    const jt_shapelets& c = *light->shapelets;
    if (c.n_max < 0 || c.n_max > kShapeletMaxN)
      return fail(JT_EUNSUPPORTED, "%s shapelets: n_max = %d not in [0, %d]", which, c.n_max, kShapeletMaxN);
    if (!(c.beta > 0.0) || !finite(c.beta) || !finite(c.cx) || !finite(c.cy))
      return fail(JT_EINVAL, "%s shapelets: bad beta or centre", which);
    if (!c.coeff) return fail(JT_EINVAL, "%s shapelets: null coefficients", which);
    const int m = (c.n_max + 1) * (c.n_max + 2) / 2;
    for (int i = 0; i < m; ++i)
      if (!finite(c.coeff[i])) return fail(JT_EINVAL, "%s shapelets: non-finite coefficient %d", which, i);
    ShapeC& o = out.sh;
    o.cx = (float)c.cx;
    o.cy = (float)c.cy;
    o.inv_beta = (float)(1.0 / c.beta);
    o.scale = (float)(1.0 / (std::sqrt(M_PI) * c.beta));
    for (int i = 0; i < m; ++i) o.coeff[i] = (float)c.coeff[i];
    out.nsh = 1;
  }
  return JT_OK;
}

// ---------------------------------------------------------------------------
// grid
// ---------------------------------------------------------------------------
jt_status make_grid(const jt_grid* g, GridC& out) {
  std::memset(&out, 0, sizeof(out));
  if (!g) return fail(JT_EINVAL, "null grid");
  if (g->nx < 1 || g->ny < 1) return fail(JT_EINVAL, "grid: %d x %d pixels", g->nx, g->ny);
  if (g->supersample < 1 || g->supersample > 16) return fail(JT_EINVAL, "grid: supersample %d not in [1, 16]", g->supersample);
  if (!(g->pixel_scale > 0.0) || !finite(g->pixel_scale) || !finite(g->x0) || !finite(g->y0))
    return fail(JT_EINVAL, "grid: bad pixel scale or centre");
  const double npix = (double)g->nx * g->ny;
  if (npix * g->supersample * g->supersample > 2147483647.0)
    return fail(JT_EUNSUPPORTED, "grid: %g sub-pixels exceed the 32-bit index range", npix * g->supersample * g->supersample);
  out.nx = g->nx;
  out.ny = g->ny;
  out.s = g->supersample;
  out.s2 = g->supersample * g->supersample;
  out.ppb = 256 / out.s2;
  out.step = g->pixel_scale / g->supersample;
  out.ox = g->x0 - 0.5 * g->pixel_scale * g->nx;
  out.oy = g->y0 - 0.5 * g->pixel_scale * g->ny;
  out.area_over_s2 = (float)(g->pixel_scale * g->pixel_scale / out.s2);
  return JT_OK;
}

}  // namespace jt
