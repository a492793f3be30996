// Device-side building blocks of the lensed-image simulation (gfx950).
//
// Everything here is evaluated per image-plane (sub-)pixel: the macro-lens
// deflection (SIE + external shear + test point masses, FP64, once per
// sub-pixel), the NFW subhalo pair term (FP32, the hot loop), and the
// elliptical Sersic surface brightness (FP32).  Kernel-constant structs are
// filled on the host in FP64; the FP32 ones are rounded once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jt {

constexpr int kMaxSersic = 8;
constexpr int kMaxBasis = 8;     // light components of the linear amplitude solver
constexpr int kMaxPointMass = 16;
constexpr float kLn2 = 0.69314718055994530942f;
constexpr double kLn2d = 0.69314718055994530942;

#include "nfw_poly.inc"
#include "atan_poly.inc"

// Mean relative errors of gfx950's log2 and rsq instructions (measured over 4M
// arguments in [1e-6, 1e6]: log2 sits 0.466 ulp low).  Their products with a
// sum of tens of thousands of same-signed NFW terms would otherwise bias the
// deflection by ~5e-8 of its size.  The subhalo record's amplitude carries
// kNfwRecScale = (ln2/2)(1 - kLog2Bias)(1 - 2 kRsqBias) and the far-field
// polynomial is fitted to P/(1 - kLog2Bias), which removes both means at no
// cost; the near-field forms are rescaled by kNfwNearScale to the same units.
constexpr double kLog2Bias = -4.08e-8;
constexpr double kRsqBias = -7.4e-9;
constexpr double kNfwRecScale = 0.5 * kLn2d * (1.0 - kLog2Bias) * (1.0 - 2.0 * kRsqBias);
constexpr float kNfwNearScale = (float)(1.0 / ((1.0 - kLog2Bias) * (1.0 - 2.0 * kRsqBias)));

// Launch shape of the subhalo sum: `split` wave-groups share the records of
// one set of sub-pixels; a group has split_lanes(split) lanes (a multiple of
// the wave size, so record reads are wave-uniform) and a block
// split_threads(split) threads.
__host__ __device__ constexpr int split_lanes(int split) { return split <= 4 ? 256 / split : 64; }
__host__ __device__ constexpr int split_threads(int split) { return split <= 4 ? 256 : 64 * split; }

// ---------------------------------------------------------------------------
// kernel constants
// ---------------------------------------------------------------------------
struct MacroC {
  int has_sie, sie_series, has_shear, npm, has_epl;
  // FP32 copies for the adjoint's SIE and shear partials
  float cx, cy, cphi, sphi, q2, f;
  float theta_E, q, sqrt_q;
  float g1, g2;
  // FP64 constants of the deflection.  SIE: rotate into the major-axis frame
  // about (cx, cy); psi = sqrt(q^2 x'^2 + y'^2); pref = theta_E sqrt(q),
  // pref_f = pref / f, f = sqrt(1 - q^2)
  double dcx, dcy, dcphi, dsphi, dq2, df, dpref, dpref_f;
  double dg1, dg2;
  // EPL: the same rotation about (ecx, ecy); R = sqrt(q^2 x'^2 + y'^2);
  // alpha' = epref (eb / R)^etm1 * Omega, Omega the series of the
  // hypergeometric factor with ratio -ef (2n - e2mt)/(2n + e2mt) e^{2 i varphi}
  double ecx, ecy, ecphi, esphi, eq, ef, e2mt, eb, etm1, epref;
  double e_te, e_gamma, e_phi;   // theta_E, gamma, phi themselves (the adjoint's partials)
  double pm_x[kMaxPointMass], pm_y[kMaxPointMass], pm_te2[kMaxPointMass];
};

struct SersicC {
  float cx, cy, cphi, sphi;
  float q, inv_q;        // R^2 = q x'^2 + y'^2 / q
  float inv_r2;          // 1 / R_sersic^2
  float e;               // 1 / (2 n): (R/R_s)^(1/n) = exp2(e * log2(R^2 / R_s^2))
  float kb;              // b_n * log2(e): I = amp * exp2(kb * (1 - t))
  float amp;
  float R, n, b;         // R_sersic, n, b_n (used by the adjoint)
};

// Elliptical Gaussian: I = norm exp2(-k R^2), norm = amp/(2 pi sigma^2),
// k = log2(e)/(2 sigma^2), R^2 as the Sersic's.
struct GaussC {
  float cx, cy, cphi, sphi, q, inv_q, k, norm;
};

// Core-Sersic in base-2 logarithms: lRb = alpha log2 R_b, lRe = alpha log2 R_e,
// half_alpha = alpha/2, g_over_a = gamma/alpha, e = 1/(n alpha),
// kb = b_n log2(e); R^2 floored at R2_floor = (1e-6 R_b)^2.
struct CoreC {
  float cx, cy, cphi, sphi, q, inv_q;
  float half_alpha, lRb, lRe, g_over_a, e, kb, amp, R2_floor;
};

// Cartesian shapelets up to order kShapeletMaxN: coefficients by n = n1 + n2,
// then n2 (zero beyond the set's n_max); scale = pi^(-1/2)/beta.
constexpr int kShapeletMaxN = 10;
constexpr int kShapeletCoeffs = (kShapeletMaxN + 1) * (kShapeletMaxN + 2) / 2;
struct ShapeC {
  float cx, cy, inv_beta, scale;
  float coeff[kShapeletCoeffs];
};
constexpr int kMaxGauss = 8;
constexpr int kMaxCore = 2;

struct LightC {
  int n;
  SersicC c[kMaxSersic];
  int ng, ncs, nsh;      // Gaussians, core-Sersic components, shapelet sets (0 or 1)
  GaussC g[kMaxGauss];
  CoreC cs[kMaxCore];
  ShapeC sh;
};

// Implicit sub-pixel grid: theta = origin + step * (m + 1/2) along each axis,
// m = pixel * s + sub-pixel; origin and step in FP64 so that theta is the
// correctly rounded FP32 value of the exact grid.
struct GridC {
  int nx, ny, s, s2;
  int ppb;               // whole pixels per wave-group: floor(split_lanes(split) / s^2)
  double ox, oy, step;   // ox = x0 - d nx / 2, step = d / s
  float area_over_s2;    // d^2 / s^2
};

// One image of a batched launch: grid, lens and light constants, its subhalo
// table and its unconvolved output.  Read from device memory with
// wave-uniform indices.
struct ImageDesc;

// Packed subhalo record: centre and the two derived constants of the pair term
// alpha = c2 * g'(x) / Xq * (dx, dy), Xq = x^2/4 = r^2 c1, c1 = 1/(4 Rs^2),
// with g in units of ln2/2 (g' = g / (ln2/2)) and the factor carried by
// c2 = kNfwRecScale alpha_Rs / (4 (1 - ln 2) Rs).  Folding the constant into c2
// (one FP64 product rounded per subhalo) keeps its FP32 rounding from biasing
// every term the same way.  The quarters are exact (powers of two), so
// 4 c1 = 1/Rs^2 and 4 c2 are the unscaled constants rounded once.
struct __align__(16) SubRec {
  float x, y, c1, c2;
};

// The record of one subhalo (host and device use the same roundings).
__host__ __device__ inline SubRec make_subrec(float x, float y, float rs, float ars) {
  const double r = rs;
  return SubRec{x, y, (float)(0.25 * (1.0 / (r * r))),
                (float)(0.25 * (kNfwRecScale * (double)ars / ((1.0 - kLn2d) * r)))};
}
// Padding record: far away, zero amplitude.
constexpr SubRec kSubRecPad{1e18f, 1e18f, 0.25f, 0.0f};

// Truncated NFW record (Baltz, Marshall & Oguri 2009, truncation exponent 1):
// centre, c1 = 1/Rs^2, tau = r_trunc/Rs with tau^2 and 1/tau, and
// c2 = alpha_Rs/((1 - ln 2) Rs) * tau^2/(tau^2 + 1)^2, each rounded once from
// FP64; then the far-field form: for x^2 = r^2 c1 >= Xf the pair term is
// c2 T(x) = y^2 sum_k a_k u^k, y = 1/x, u = y k1 - 1 (see tnfw_far_fit).
constexpr int kTnfwFarDeg = 10;
// In the fused kernels the first 48 bytes (through k1 and a_2) are read
// through scalar loads and the last 32 (a_3 .. a_10) staged through LDS.
struct __align__(16) TRec {
  float x, y, c1, Xf, tau, t2, itau, c2;
  float k1, a[kTnfwFarDeg + 1];
};
static_assert(sizeof(TRec) == 80, "TRec is read as 12 scalar floats and two float4s");

struct ImageDesc {
  GridC g;               // g.ppb matches the launch's wave split
  MacroC mc;
  LightC src, ll;
  const void* sub;       // subhalo_table_records(n) records: SubRec, or TRec in a TNFW launch
  int nloop;             // loop count (multiple of 4)
  float* img;            // unconvolved image [ny][nx]
  float2* beta;          // traced sub-pixel positions [ny * nx][s^2] kept for the adjoint, or null
};

// One convolution of a heterogeneous batch: out = psf * img ([ny][nx], odd k).
struct ConvDesc {
  const float* img;
  float* out;
  const float* psf;
  int nx, ny, k;
  int t;                 // input rows per staged chunk: conv_shape(nx, ny, k).t
};

// ---------------------------------------------------------------------------
// macro lens
// ---------------------------------------------------------------------------
// FP64, once per sub-pixel: the FP32 representation of angles of tens of
// arcseconds (|theta|, |alpha| up to ~20") would otherwise dominate the error
// of beta = theta - alpha.
// EPL deflection (Tessore & Metcalf 2015) in FP64, in the major-axis frame:
// with e^{i varphi} = (q x' + i y')/R, alpha' = 2b/(1+q) (b/R)^(t-1) Omega,
// Omega = sum_n w_n, w_0 = e^{i varphi},
// w_n = -f (2n - (2-t))/(2n + (2-t)) e^{2 i varphi} w_{n-1}, f = (1-q)/(1+q):
// the power series of the Gauss hypergeometric factor, summed until a term no
// longer changes the sum in double precision.  0 at R = 0.
constexpr int kEplMaxTerms = 1000;

__device__ __forceinline__ void epl_deflection64(const MacroC& m, double tx, double ty, double& ax, double& ay) {
  const double dx = tx - m.ecx, dy = ty - m.ecy;
  const double xp = m.ecphi * dx + m.esphi * dy;
  const double yp = m.ecphi * dy - m.esphi * dx;
  const double qx = m.eq * xp;
  const double R = sqrt(qx * qx + yp * yp);
  ax = 0.0;
  ay = 0.0;
  if (!(R > 0.0)) return;
  const double iR = 1.0 / R;
  const double c = qx * iR, s = yp * iR;
  const double c2 = c * c - s * s, s2 = 2.0 * c * s;
  double wr = c, wi = s, sr = c, si = s;
  for (int n = 1; n < kEplMaxTerms; ++n) {
    const double k = -m.ef * (2.0 * n - m.e2mt) / (2.0 * n + m.e2mt);
    const double nr = k * (c2 * wr - s2 * wi);
    const double ni = k * (s2 * wr + c2 * wi);
    wr = nr;
    wi = ni;
    sr += nr;
    si += ni;
    if (fabs(nr) + fabs(ni) <= 0x1p-56 * (fabs(sr) + fabs(si))) break;
  }
  const double a = m.epref * pow(m.eb * iR, m.etm1);
  const double axp = a * sr, ayp = a * si;
  ax = m.ecphi * axp - m.esphi * ayp;
  ay = m.esphi * axp + m.ecphi * ayp;
}

__device__ __forceinline__ void macro_deflection64(const MacroC& m, double tx, double ty, double& ax, double& ay) {
  ax = 0.0;
  ay = 0.0;
  if (m.has_sie) {
    const double dx = tx - m.dcx, dy = ty - m.dcy;
    const double xp = m.dcphi * dx + m.dsphi * dy;
    const double yp = m.dcphi * dy - m.dsphi * dx;
    const double psi = sqrt(m.dq2 * xp * xp + yp * yp);
    double axp = 0.0, ayp = 0.0;
    if (psi > 0.0) {
      const double ipsi = 1.0 / psi;
      if (m.sie_series) {
        // atan(z)/z and atanh(z)/z by their Taylor series for f < 1e-3 (|z| < f)
        const double zx = m.df * xp * ipsi, zy = m.df * yp * ipsi;
        const double zx2 = zx * zx, zy2 = zy * zy;
        axp = m.dpref * xp * ipsi * (1.0 + zx2 * (-1.0 / 3.0 + zx2 * (0.2 - zx2 / 7.0)));
        ayp = m.dpref * yp * ipsi * (1.0 + zy2 * (1.0 / 3.0 + zy2 * (0.2 + zy2 / 7.0)));
      } else {
        axp = m.dpref_f * atan(m.df * xp * ipsi);
        ayp = m.dpref_f * atanh(m.df * yp * ipsi);
      }
    }
    ax = m.dcphi * axp - m.dsphi * ayp;
    ay = m.dsphi * axp + m.dcphi * ayp;
  }
  if (m.has_epl) {
    double ex, ey;
    epl_deflection64(m, tx, ty, ex, ey);
    ax += ex;
    ay += ey;
  }
  if (m.has_shear) {
    ax += m.dg1 * tx + m.dg2 * ty;
    ay += m.dg2 * tx - m.dg1 * ty;
  }
  for (int k = 0; k < m.npm; ++k) {
    const double dx = tx - m.pm_x[k], dy = ty - m.pm_y[k];
    const double r2 = dx * dx + dy * dy;
    const double fac = r2 > 0.0 ? m.pm_te2[k] / r2 : 0.0;
    ax += fac * dx;
    ay += fac * dy;
  }
}

// ---------------------------------------------------------------------------
// NFW pair term
// ---------------------------------------------------------------------------
// The pair kernel works with the quarter squared radius Xq = x^2/4 (the
// record carries c1/4), lq = log2(Xq) and yq = rsq(Xq) = 2/x, and returns
// hq = g'(x)/Xq = 4 g'(x)/x^2 (the record carries c2/4), g' = g/(ln2/2).
//
// Near field, x^2 = 4 Xq < 1 (rare pairs), with hardware transcendentals and
// forms that avoid cancellation.  In these units ln(x/2) = (ln2/2) lq exactly:
//   x^2 >= 0.81: F = sum_k (-u)^k/(2k+1), u = x^2 - 1 in [-0.19, 0), and
//                g' = lq + F / (ln2/2);
//   x^2 <  0.81: g = [-L x^2/(1+w) + log1p(-x^2/(2(1+w)))]/w, L = ln(x/2),
//                w = sqrt(1 - x^2), with log1p(t) = t ln(1+t)/((1+t) - 1)
//                (exact t when 1 + t rounds to 1);
// 0 at x = 0.
__device__ __forceinline__ float nfw_near_hq(float Xq, float lq) {
  constexpr float kInvA = (float)(2.0 / kLn2d);   // 1 / (ln2/2)
  const float X2 = 4.0f * Xq;
  const float Lp = lq;                             // ln(x/2) / (ln2/2)
  float g;
  if (X2 >= 0.81f) {
    const float u = X2 - 1.0f;
    // F / (ln2/2): coefficients (2/ln2)/(2k+1), each rounded once
    float F = (float)(2.0 / kLn2d / 21.0);
    F = fmaf(F, -u, (float)(2.0 / kLn2d / 19.0));
    F = fmaf(F, -u, (float)(2.0 / kLn2d / 17.0));
    F = fmaf(F, -u, (float)(2.0 / kLn2d / 15.0));
    F = fmaf(F, -u, (float)(2.0 / kLn2d / 13.0));
    F = fmaf(F, -u, (float)(2.0 / kLn2d / 11.0));
    F = fmaf(F, -u, (float)(2.0 / kLn2d / 9.0));
    F = fmaf(F, -u, (float)(2.0 / kLn2d / 7.0));
    F = fmaf(F, -u, (float)(2.0 / kLn2d / 5.0));
    F = fmaf(F, -u, (float)(2.0 / kLn2d / 3.0));
    F = fmaf(F, -u, kInvA);
    g = Lp + F;
  } else {
    const float w = __builtin_amdgcn_sqrtf(1.0f - X2);
    const float ropw = __builtin_amdgcn_rcpf(1.0f + w);
    const float t = -0.5f * X2 * ropw;
    const float u = 1.0f + t;
    // log1p(t) / (ln2/2) = 2 log2(1+t) t / ((1+t) - 1)
    const float lp = (u == 1.0f) ? t * kInvA : 2.0f * __builtin_amdgcn_logf(u) * t * __builtin_amdgcn_rcpf(u - 1.0f);
    g = fmaf(-Lp * X2, ropw, lp) * __builtin_amdgcn_rcpf(w);
  }
  return Xq > 0.f ? g * kNfwNearScale * __builtin_amdgcn_rcpf(Xq) : 0.f;
}

// Far field, x >= 1: g' = lq + yq R(yq) with R the fitted polynomial in the
// shifted form (the constant -2 of g' is what log2(x^2/4) = log2(x^2) - 2
// absorbs), and hq = g' yq^2.  The short form uses the fit on
// [0, kNfwFastY] in y = 1/x only.
__device__ __forceinline__ float nfw_far_hq(float lq, float yq) {
  float p = kNfwR[0];
#pragma unroll
  for (int i = 1; i < JT_NFW_POLY_DEGREE; ++i) p = fmaf(p, yq, kNfwR[i]);
  return fmaf(p, yq, lq) * (yq * yq);
}

__device__ __forceinline__ float nfw_far_hq_short(float lq, float yq) {
  float p = kNfwRFast[0];
#pragma unroll
  for (int i = 1; i < JT_NFW_FAST_DEGREE; ++i) p = fmaf(p, yq, kNfwRFast[i]);
  return fmaf(p, yq, lq) * (yq * yq);
}

// Four (sub-pixel, subhalo) pairs: adds alpha_k, k = 0..3, to (sx, sy), with
// X = Xq, l = lq and y = yq of the quarter-radius form above.  When
// y = 2 Rs/r < kNfwFastYq for all four (distant subhalos: nearly every
// group) the short polynomial is used; otherwise the full one, and a second
// branch recomputes the rare near-field (x < 1) terms.  The choice is made
// per lane from its own four pairs, so a sub-pixel's result does not depend
// on which sub-pixels share its wave; in practice the lanes of a wave agree
// and the branches are uniform.
__device__ __forceinline__ void nfw_pairs4(float tx, float ty, const SubRec& s0, const SubRec& s1,
                                           const SubRec& s2, const SubRec& s3, float& sx,
                                           float& sy) {
  const float dx0 = tx - s0.x, dy0 = ty - s0.y;
  const float dx1 = tx - s1.x, dy1 = ty - s1.y;
  const float dx2 = tx - s2.x, dy2 = ty - s2.y;
  const float dx3 = tx - s3.x, dy3 = ty - s3.y;
  const float X0 = fmaf(dy0, dy0, dx0 * dx0) * s0.c1;
  const float X1 = fmaf(dy1, dy1, dx1 * dx1) * s1.c1;
  const float X2 = fmaf(dy2, dy2, dx2 * dx2) * s2.c1;
  const float X3 = fmaf(dy3, dy3, dx3 * dx3) * s3.c1;
  const float l0 = __builtin_amdgcn_logf(X0);
  const float l1 = __builtin_amdgcn_logf(X1);
  const float l2 = __builtin_amdgcn_logf(X2);
  const float l3 = __builtin_amdgcn_logf(X3);
  const float y0 = __builtin_amdgcn_rsqf(X0);
  const float y1 = __builtin_amdgcn_rsqf(X1);
  const float y2 = __builtin_amdgcn_rsqf(X2);
  const float y3 = __builtin_amdgcn_rsqf(X3);
  float h0, h1, h2, h3;
  if (fmaxf(fmaxf(y0, y1), fmaxf(y2, y3)) < kNfwFastYq) {
    h0 = nfw_far_hq_short(l0, y0);
    h1 = nfw_far_hq_short(l1, y1);
    h2 = nfw_far_hq_short(l2, y2);
    h3 = nfw_far_hq_short(l3, y3);
  } else {
    h0 = nfw_far_hq(l0, y0);
    h1 = nfw_far_hq(l1, y1);
    h2 = nfw_far_hq(l2, y2);
    h3 = nfw_far_hq(l3, y3);
    if (fminf(fminf(X0, X1), fminf(X2, X3)) < 0.25f) {
      if (X0 < 0.25f) h0 = nfw_near_hq(X0, l0);
      if (X1 < 0.25f) h1 = nfw_near_hq(X1, l1);
      if (X2 < 0.25f) h2 = nfw_near_hq(X2, l2);
      if (X3 < 0.25f) h3 = nfw_near_hq(X3, l3);
    }
  }
  sx = fmaf(h0 * s0.c2, dx0, sx);
  sy = fmaf(h0 * s0.c2, dy0, sy);
  sx = fmaf(h1 * s1.c2, dx1, sx);
  sy = fmaf(h1 * s1.c2, dy1, sy);
  sx = fmaf(h2 * s2.c2, dx2, sx);
  sy = fmaf(h2 * s2.c2, dy2, sy);
  sx = fmaf(h3 * s3.c2, dx3, sx);
  sy = fmaf(h3 * s3.c2, dy3, sy);
}

// ---------------------------------------------------------------------------
// TNFW pair term
// ---------------------------------------------------------------------------
// log(1 + z) from the hardware log2, accurate for small z as well:
// z ln(1+z) / ((1+z) - 1) (exact z when 1 + z rounds to 1).
__device__ __forceinline__ float log1p_fast(float z) {
  const float w = 1.0f + z;
  const float d = w - 1.0f;
  return d == 0.0f ? z : __builtin_amdgcn_logf(w) * kLn2 * z * __builtin_amdgcn_rcpf(d);
}

// atan(z) for z >= 0: z A(z^2) on [0, 1], pi/2 - atan(1/z) above.
__device__ __forceinline__ float atan_pos(float z, float iz) {
  const float m = fminf(z, iz);
  const float t = m * m;
  float p = kAtanP[0];
#pragma unroll
  for (int k = 1; k <= JT_ATAN_POLY_DEGREE; ++k) p = fmaf(p, t, kAtanP[k]);
  p *= m;
  return z > 1.0f ? 1.57079632679489661923f - p : p;
}

// FP64 T(x) = G(x, tau) / (A x^2) = (tau^2 - 1) P1 + P2 of the truncated
// profile (A = tau^2/(tau^2 + 1)^2, the regrouping of tnfw_T_general below) for
// X2 = x^2 >= 1.2, the form without cancelling differences.
__host__ __device__ inline double tnfw_T64_far(double X2, double tau) {
  constexpr double kPiD = 3.14159265358979323846;
  const double t2 = tau * tau;
  const double x = sqrt(X2), s = sqrt(t2 + X2), sp = s + tau;
  const double u = sqrt(X2 - 1.0);
  const double a = atan(1.0 / u);
  const double g = (0.5 * log(X2) - kLn2d) + (0.5 * kPiD - a) / u;     // ln(x/2) + F(x)
  const double P2 = (kPiD * (tau + (t2 + 1.0) / (s + u)) / sp - 2.0 * a) / u;
  const double z1 = (tau + t2 / (s + x)) / x;                            // -ln(x/sp) = log1p(z1)
  const double z2 = 0.5 * X2 / (tau * sp);                               // ln(sp/(2 tau)) = log1p(z2)
  const double P1 = (g - log1p(z2)) / X2 - log1p(z1) / (tau * sp);
  return (t2 - 1.0) * P1 + P2;
}

// Far field of the truncated pair term as a polynomial in 1/x: for
// x >= x_f = max(kTnfwFarX tau, kTnfwFarMin), W(y) = T(1/y) / y^2 is analytic
// in y = 1/x on [0, 1/x_f] (its nearest singularities are y = -1 and
// y = +-i/tau), so the interpolant at kTnfwFarDeg + 1 Chebyshev points of that
// interval, written as a polynomial in u = 2 y x_f - 1 in [-1, 1], matches it
// to about 3e-8 relative for tau in [0.4, 1e4] (degree 12 would give 3e-9;
// the FP32 Horner evaluation adds about 1e-7 either way).  The record stores
// Xf = x_f^2, k1 = 2 x_f and a_k = c2 (1 - 2 kRsqBias) m_k, m_k the
// interpolant's monomial coefficients (the factor removes the mean bias of the
// hardware rsq that forms y^2).  The pair then costs one reciprocal square
// root and a degree-10 polynomial instead of nine transcendentals.  x_f =
// 0.75 tau (down from 1.5 tau with degree 8) leaves about a third as many
// pairs to the general form for two more FMAs each.
constexpr double kTnfwFarX = 0.75;
constexpr double kTnfwFarMin = 1.5;
__host__ __device__ inline void tnfw_far_fit(double tau, double c2, TRec& r) {
  constexpr double kPiD = 3.14159265358979323846;
  constexpr int N = kTnfwFarDeg + 1;
  const double xf = kTnfwFarX * tau > kTnfwFarMin ? kTnfwFarX * tau : kTnfwFarMin;
  double f[N], uj[N], tj[N], tjm1[N];
  for (int j = 0; j < N; ++j) {
    uj[j] = cos(kPiD * (2 * j + 1) / (2 * N));
    const double y = 0.5 * (uj[j] + 1.0) / xf;
    const double X2 = 1.0 / (y * y);
    f[j] = tnfw_T64_far(X2, tau) * X2;
    tjm1[j] = 1.0;      // T_0(u_j)
    tj[j] = uj[j];      // T_1(u_j)
  }
  // Chebyshev coefficients of the interpolant (T_k(u_j) by the recurrence
  // T_{k+1} = 2 u T_k - T_{k-1}), then its monomial form in u by the same
  // recurrence on coefficient vectors
  double m[N], tkm1[N], tk[N], tkp1[N];
  for (int i = 0; i < N; ++i) m[i] = tkm1[i] = tk[i] = 0.0;
  tkm1[0] = 1.0;   // T_0
  tk[1] = 1.0;     // T_1
  for (int k = 0; k < N; ++k) {
    double c = 0.0;
    for (int j = 0; j < N; ++j) {
      const double t = k == 0 ? tjm1[j] : tj[j];
      c += f[j] * t;
      if (k >= 1) {
        const double nxt = 2.0 * uj[j] * tj[j] - tjm1[j];
        tjm1[j] = tj[j];
        tj[j] = nxt;
      }
    }
    c *= (k == 0 ? 1.0 : 2.0) / N;
    const double* tkk = k == 0 ? tkm1 : tk;
    for (int i = 0; i < N; ++i) m[i] += c * tkk[i];
    if (k >= 1) {
      for (int i = 0; i < N; ++i) tkp1[i] = (i > 0 ? 2.0 * tk[i - 1] : 0.0) - tkm1[i];
      for (int i = 0; i < N; ++i) {
        tkm1[i] = tk[i];
        tk[i] = tkp1[i];
      }
    }
  }
  const double scale = c2 * (1.0 - 2.0 * kRsqBias);
  r.Xf = (float)(xf * xf);
  r.k1 = (float)(2.0 * xf);
  for (int i = 0; i < N; ++i) r.a[i] = (float)(scale * m[i]);
}

// The record of one truncated subhalo (c2 includes A; every value rounded
// once from FP64).
__host__ __device__ inline TRec make_trec(float x, float y, float rs, float ars, float rt) {
  const double r = rs, tau = (double)rt / r, t2 = tau * tau;
  const double c2 = (double)ars / ((1.0 - kLn2d) * r) * t2 / ((t2 + 1.0) * (t2 + 1.0));
  TRec out;
  out.x = x;
  out.y = y;
  out.c1 = (float)(1.0 / (r * r));
  out.c2 = (float)c2;
  out.tau = (float)tau;
  out.t2 = (float)t2;
  out.itau = (float)(1.0 / tau);
  tnfw_far_fit(tau, c2, out);
  return out;
}

// Padding record: far away, zero amplitude (both forms give an exact zero).
__host__ __device__ inline TRec trec_pad() {
  TRec out;
  out.x = out.y = 1e18f;
  out.c1 = 1.0f;
  out.c2 = 0.0f;
  out.tau = out.t2 = out.itau = 1.0f;
  out.Xf = 0.0f;
  out.k1 = 0.0f;
  for (int i = 0; i <= kTnfwFarDeg; ++i) out.a[i] = 0.0f;
  return out;
}

// With x^2 = X2, s = sqrt(tau^2 + x^2), sp = s + tau, the projected mass of
// the truncated profile regrouped so that no step cancels catastrophically:
//   G/x^2 = A [ (tau^2 - 1) P1 + P2 ],  A = tau^2/(tau^2 + 1)^2 (in c2),
//   P1 = (g - ln(sp/(2 tau))) / x^2 + L / (tau sp),
//   P2 = 2F - pi/sp,
// g = ln(x/2) + F the NFW function, L = ln(x/sp) = -log1p((tau + tau^2/(s+x))/x)
// and ln(sp/(2 tau)) = log1p(x^2/(2 tau sp)).  F and g by branch:
//   x^2 < 0.8:  g = [-ln(x/2) x^2/(1+w) + log1p(-x^2/(2(1+w)))]/w, w = sqrt(1-x^2);
//   x^2 < 1.2:  F = sum_k (-v)^k/(2k+1), v = x^2 - 1;
//   otherwise:  u = sqrt(x^2 - 1), a = atan(1/u), F = (pi/2 - a)/u, and
//               P2 = pi (tau + (tau^2+1)/(s+u)) / (u sp) - 2a/u, which avoids
//               the cancellation of 2F against pi/sp far from the centre.
// Hardware rsq, sqrt, rcp and log2 (about one ulp each, none of them in a
// cancelling difference; nine per distant pair, reciprocals shared where two
// are needed) and the polynomial arctangent.  0 at the centre
// (X2 below 1e-30, where the term is below 1e-28 of alpha_Rs).
// The general form, for 1e-30 < X2: returns T = (tau^2 - 1) P1 + P2 (the
// pair term is c2 T) and also F(x), s = sqrt(tau^2 + x^2) and
// lp1 = log1p(z1) = -ln(x/(s + tau)), which the adjoint's derivative uses.
__device__ __forceinline__ float tnfw_T_general(float X2, const TRec& r, float& F, float& s, float& lp1) {
  constexpr float kPi = 3.14159265358979323846f;
  constexpr float kHalfPi = 1.57079632679489661923f;
  const float ix = __builtin_amdgcn_rsqf(X2);
  const float x = X2 * ix;
  s = __builtin_amdgcn_sqrtf(r.t2 + X2);
  const float sp = s + r.tau;
  const float isp = __builtin_amdgcn_rcpf(sp);
  const float Lh = fmaf(__builtin_amdgcn_logf(X2), 0.5f * kLn2, -kLn2);   // ln(x/2)
  const float spx = s + x;
  float g, P2, isx;   // isx = 1/(s + x)
  if (X2 < 0.8f) {
    const float w = __builtin_amdgcn_sqrtf(1.0f - X2);
    const float i1w = __builtin_amdgcn_rcpf(1.0f + w);
    g = (-Lh * X2 * i1w + log1p_fast(-0.5f * X2 * i1w)) * __builtin_amdgcn_rcpf(w);
    F = g - Lh;
    P2 = fmaf(2.0f, F, -kPi * isp);
    isx = __builtin_amdgcn_rcpf(spx);
  } else if (X2 < 1.2f) {
    const float v = -(X2 - 1.0f);
    F = 1.0f / 21.0f;
    F = fmaf(F, v, 1.0f / 19.0f);
    F = fmaf(F, v, 1.0f / 17.0f);
    F = fmaf(F, v, 1.0f / 15.0f);
    F = fmaf(F, v, 1.0f / 13.0f);
    F = fmaf(F, v, 1.0f / 11.0f);
    F = fmaf(F, v, 1.0f / 9.0f);
    F = fmaf(F, v, 1.0f / 7.0f);
    F = fmaf(F, v, 1.0f / 5.0f);
    F = fmaf(F, v, 1.0f / 3.0f);
    F = fmaf(F, v, 1.0f);
    g = Lh + F;
    P2 = fmaf(2.0f, F, -kPi * isp);
    isx = __builtin_amdgcn_rcpf(spx);
  } else {
    const float v1 = X2 - 1.0f;
    const float iu = __builtin_amdgcn_rsqf(v1);
    const float u = v1 * iu;
    const float a = atan_pos(iu, u);
    F = (kHalfPi - a) * iu;
    g = Lh + F;
    const float spu = s + u;
    const float r2 = __builtin_amdgcn_rcpf(spu * spx);    // 1/(s+u) and 1/(s+x) from one reciprocal
    isx = r2 * spu;
    P2 = (kPi * fmaf(r.t2 + 1.0f, r2 * spx, r.tau) * isp - 2.0f * a) * iu;
  }
  // L = -log1p(z1) and the log1p(z2) of P1, both as z ln(1+z)/((1+z) - 1)
  // with one reciprocal for the two quotients (an exact z where 1 + z rounds
  // to 1)
  const float z1 = fmaf(r.t2, isx, r.tau) * ix;
  const float z2 = 0.5f * X2 * r.itau * isp;
  const float w1 = 1.0f + z1, w2 = 1.0f + z2;
  const float d1 = w1 - 1.0f, d2 = w2 - 1.0f;
  const float e1 = d1 == 0.0f ? 1.0f : d1, e2 = d2 == 0.0f ? 1.0f : d2;
  const float rd = __builtin_amdgcn_rcpf(e1 * e2);
  lp1 = d1 == 0.0f ? z1 : __builtin_amdgcn_logf(w1) * kLn2 * z1 * (rd * e2);
  const float lp2 = d2 == 0.0f ? z2 : __builtin_amdgcn_logf(w2) * kLn2 * z2 * (rd * e1);
  const float P1 = (g - lp2) * (ix * ix) - lp1 * r.itau * isp;
  return fmaf(r.t2 - 1.0f, P1, P2);
}

// Far field of the truncated pair term (tnfw_far_fit), X2 >= r.Xf:
// h = y^2 sum_k a_k u^k.
__device__ __forceinline__ float tnfw_far_h(float X2, const TRec& r) {
  const float yy = __builtin_amdgcn_rsqf(X2);
  const float u = fmaf(yy, r.k1, -1.0f);
  float p = r.a[kTnfwFarDeg];
#pragma unroll
  for (int k = kTnfwFarDeg - 1; k >= 0; --k) p = fmaf(p, u, r.a[k]);
  return p * (yy * yy);
}

// Pair terms of two consecutive truncated-subhalo records a, b at one
// sub-pixel, added to (sx, sy) in that order.  The far form is evaluated by
// every lane, without a branch (a wave's lanes are neighbouring sub-pixels,
// nearly always all far), and replaced where X2 < Xf; a pair at the centre
// itself (X2 <= 1e-30) adds 0.  One exec-masked region covers both records'
// general forms: an if/else per pair cost more scalar instructions and
// branches than the far form's arithmetic, and a region per pair twice the
// mask instructions of this one.
__device__ __forceinline__ void tnfw_pair2(float tx, float ty, const TRec& a, const TRec& b, float& sx,
                                           float& sy) {
  const float dxa = tx - a.x, dya = ty - a.y;
  const float dxb = tx - b.x, dyb = ty - b.y;
  const float Xa = fmaf(dya, dya, dxa * dxa) * a.c1;
  const float Xb = fmaf(dyb, dyb, dxb * dxb) * b.c1;
  float ha = tnfw_far_h(Xa, a);
  float hb = tnfw_far_h(Xb, b);
  const bool na = Xa < a.Xf, nb = Xb < b.Xf;
  if (na || nb) {
    float F, s, lp1;
    if (na) ha = Xa > 1e-30f ? a.c2 * tnfw_T_general(Xa, a, F, s, lp1) : 0.0f;
    if (nb) hb = Xb > 1e-30f ? b.c2 * tnfw_T_general(Xb, b, F, s, lp1) : 0.0f;
  }
  sx = fmaf(ha, dxa, sx);
  sy = fmaf(ha, dya, sy);
  sx = fmaf(hb, dxb, sx);
  sy = fmaf(hb, dyb, sy);
}

// Knuth's TwoSum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum_acc(float& hi, float& lo, float v) {
  const float s = hi + v;
  const float bp = s - hi;
  const float e = (hi - (s - bp)) + (v - bp);
  hi = s;
  lo += e;
}

// ---------------------------------------------------------------------------
// Sersic light
// ---------------------------------------------------------------------------
// One Sersic component at unit amplitude.
__device__ __forceinline__ float sersic_unit(const SersicC& c, float x, float y) {
  const float dx = x - c.cx, dy = y - c.cy;
  const float xp = fmaf(c.cphi, dx, c.sphi * dy);
  const float yp = fmaf(c.cphi, dy, -c.sphi * dx);
  const float R2 = fmaf(c.q, xp * xp, c.inv_q * (yp * yp));
  const float t = __builtin_amdgcn_exp2f(c.e * __builtin_amdgcn_logf(R2 * c.inv_r2));
  return __builtin_amdgcn_exp2f(fmaf(-c.kb, t, c.kb));
}

__device__ __forceinline__ float sersic_sum(const LightC& L, float x, float y) {
  float acc = 0.f;
  for (int k = 0; k < L.n; ++k) acc = fmaf(L.c[k].amp, sersic_unit(L.c[k], x, y), acc);
  return acc;
}

__device__ __forceinline__ float shapelet_sum(const ShapeC& s, float x, float y) {
  constexpr float kHalfLog2e = 0.72134752044448170368f;   // log2(e)/2
  const float u = (x - s.cx) * s.inv_beta, v = (y - s.cy) * s.inv_beta;
  // phi_n(v) / pi^(-1/4) by the normalised Hermite recurrence
  float pv[kShapeletMaxN + 1];
  pv[0] = __builtin_amdgcn_exp2f(-kHalfLog2e * v * v);
  pv[1] = 1.41421356237309504880f * v * pv[0];
#pragma unroll
  for (int n = 1; n < kShapeletMaxN; ++n)
    pv[n + 1] = fmaf((float)__builtin_sqrt(2.0 / (n + 1)) * v, pv[n], -(float)__builtin_sqrt((double)n / (n + 1)) * pv[n - 1]);
  float pu_prev = 0.f, pu = __builtin_amdgcn_exp2f(-kHalfLog2e * u * u);
  float acc = 0.f;
#pragma unroll
  for (int n1 = 0; n1 <= kShapeletMaxN; ++n1) {
    float row = 0.f;
#pragma unroll
    for (int n2 = 0; n1 + n2 <= kShapeletMaxN; ++n2) {
      const int n = n1 + n2;
      row = fmaf(s.coeff[n * (n + 1) / 2 + n2], pv[n2], row);
    }
    acc = fmaf(pu, row, acc);
    const float next = n1 == 0 ? 1.41421356237309504880f * u * pu
                               : fmaf((float)__builtin_sqrt(2.0 / (n1 + 1)) * u, pu,
                                      -(float)__builtin_sqrt((double)n1 / (n1 + 1)) * pu_prev);
    pu_prev = pu;
    pu = next;
  }
  return acc * s.scale;
}

// The profiles beyond the Sersic: Gaussians, core-Sersic components and a
// shapelet set.
__device__ __forceinline__ float light_extra(const LightC& L, float x, float y) {
  float acc = 0.f;
  for (int k = 0; k < L.ng; ++k) {
    const GaussC& c = L.g[k];
    const float dx = x - c.cx, dy = y - c.cy;
    const float xp = fmaf(c.cphi, dx, c.sphi * dy);
    const float yp = fmaf(c.cphi, dy, -c.sphi * dx);
    const float R2 = fmaf(c.q, xp * xp, c.inv_q * (yp * yp));
    acc = fmaf(c.norm, __builtin_amdgcn_exp2f(-c.k * R2), acc);
  }
  for (int k = 0; k < L.ncs; ++k) {
    const CoreC& c = L.cs[k];
    const float dx = x - c.cx, dy = y - c.cy;
    const float xp = fmaf(c.cphi, dx, c.sphi * dy);
    const float yp = fmaf(c.cphi, dy, -c.sphi * dx);
    const float R2 = fmaxf(fmaf(c.q, xp * xp, c.inv_q * (yp * yp)), c.R2_floor);
    const float lRa = c.half_alpha * __builtin_amdgcn_logf(R2);                    // log2 R^alpha
    const float lsum = fmaxf(lRa, c.lRb) + __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(-fabsf(lRa - c.lRb)));
    const float inner = __builtin_amdgcn_exp2f(c.g_over_a * (lsum - lRa));
    const float t = __builtin_amdgcn_exp2f(c.e * (lsum - c.lRe));
    acc = fmaf(c.amp * inner, __builtin_amdgcn_exp2f(fmaf(-c.kb, t, c.kb)), acc);
  }
  if (L.nsh) acc += shapelet_sum(L.sh, x, y);
  return acc;
}

__host__ __device__ __forceinline__ bool light_any(const LightC& L) { return (L.n | L.ng | L.ncs | L.nsh) != 0; }
__host__ __device__ __forceinline__ bool light_has_extra(const LightC& L) { return (L.ng | L.ncs | L.nsh) != 0; }

// Every light component of a list at (x, y).  Kernels instantiated with
// kExtra = false see Sersic components only: the extra profiles' code (and
// the scalar registers its constants take) stays out of them.
template <bool kExtra = true>
__device__ __forceinline__ float light_sum(const LightC& L, float x, float y) {
  float acc = sersic_sum(L, x, y);
  if (kExtra && light_has_extra(L)) acc += light_extra(L, x, y);
  return acc;
}

}  // namespace jt
