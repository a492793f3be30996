// Hand-written adjoint of the chi^2 image log-likelihood (gfx950, FP32).
//
//   log L = -1/2 sum_i w_i (m_i - d_i)^2,  m = K * U,  U = pixel-area mean of
//   the sub-pixel surface brightness I(theta, beta(theta)).
//
// Reverse pass, per parameter draw:
//   r = -w (m - d)                         k_residual (+ log L block partials)
//   lambda_U = K correlated with r         k_conv_direct<flip>
//   lambda   = lambda_U * d^2 / s^2 per sub-pixel; beta recomputed by the
//   forward's canonical subhalo sum (or, in the kept variant, the forward
//   launch's own traced position, 8 bytes per sub-pixel), G = lambda *
//   dI/dbeta; Sersic, SIE and shear parameter partials are reduced per
//   block                                             k_grad_pixel
//   subhalo (x, y, alpha_Rs) gradients: a subhalo-major pass over the
//   sub-pixel records (theta, G)                      k_grad_subhalo
//   (truncated subhalos: the far pairs so, the near
//   pairs by a wave per subhalo over its box)         k_grad_subhalo_tnfw(_near)
//   fixed-order sums of the partials                  k_grad_finalize
// Every sum has a fixed order (no atomics), so gradients are reproducible.
#include "jt_device.hpp"
#include "jt_kernels.hpp"
#include "jt_sum.hpp"

namespace jt {

// Parts of the subhalo-major pass over sub-pixel records (summed in order).
constexpr int kRecParts = kRecPartsHost;
constexpr int kRecPartsTnfw = kRecPartsTnfwHost;
// Subhalos per block of that pass: its waves read the same records, so a
// block of several waves shares them through its CU's scalar cache.
constexpr int kSubhaloBlock = 256;

constexpr float kCapaccioliSlope = 1.9992f;   // d b_n / d n of the Capaccioli fit

// ---------------------------------------------------------------------------
// Sersic value and its partials.  d[0..6] = dI / d(amp, R, n, q, phi, cx, cy);
// (gx, gy) = dI / d(x, y) at the evaluation point.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float sersic_grad(const SersicC& c, float x, float y, float d[7], float& gx,
                                             float& gy) {
  const float dx = x - c.cx, dy = y - c.cy;
  const float xp = fmaf(c.cphi, dx, c.sphi * dy);
  const float yp = fmaf(c.cphi, dy, -c.sphi * dx);
  const float R2 = fmaf(c.q, xp * xp, c.inv_q * (yp * yp));
  const float lr = __builtin_amdgcn_logf(R2 * c.inv_r2);          // log2(R^2 / R_s^2)
  const float t = __builtin_amdgcn_exp2f(c.e * lr);                // (R / R_s)^(1/n)
  const float E = __builtin_amdgcn_exp2f(fmaf(-c.kb, t, c.kb));    // exp(-b (t - 1))
  const float I = c.amp * E;
  const bool pos = R2 > 0.f;
  const float dIdR2 = pos ? -c.b * I * c.e * t / R2 : 0.f;         // dI/dt * dt/dR^2
  d[0] = E;
  d[1] = c.b * I * t / (c.n * c.R);
  const float tl = pos ? t * lr * kLn2 : 0.f;                       // t ln(R^2/R_s^2)
  d[2] = -I * (kCapaccioliSlope * (t - 1.0f) - c.b * tl * 0.5f / (c.n * c.n));
  d[3] = dIdR2 * (xp * xp - yp * yp * c.inv_q * c.inv_q);
  d[4] = dIdR2 * 2.0f * xp * yp * (c.q - c.inv_q);
  gx = dIdR2 * 2.0f * (c.q * xp * c.cphi - yp * c.inv_q * c.sphi);
  gy = dIdR2 * 2.0f * (c.q * xp * c.sphi + yp * c.inv_q * c.cphi);
  d[5] = -gx;
  d[6] = -gy;
  return I;
}

// T(t) = atan(sqrt t)/sqrt t and dT/dt; Hh(s) = atanh(sqrt s)/sqrt s and
// dHh/ds.  Series below 0.05 (truncation < 1e-9), closed forms above.
__device__ __forceinline__ void atan_ratio(float t, float& T, float& dT) {
  if (t < 0.05f) {
    T = fmaf(t, fmaf(t, fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.0f / 13, -1.0f / 11), 1.0f / 9), -1.0f / 7), 1.0f / 5),
                     -1.0f / 3), 1.0f);
    dT = fmaf(t, fmaf(t, fmaf(t, fmaf(t, fmaf(t, 6.0f / 13, -5.0f / 11), 4.0f / 9), -3.0f / 7), 2.0f / 5),
              -1.0f / 3);
  } else {
    const float r = sqrtf(t);
    T = atanf(r) / r;
    dT = (1.0f / (1.0f + t) - T) / (2.0f * t);
  }
}

__device__ __forceinline__ void atanh_ratio(float s, float& H, float& dH) {
  if (s < 0.05f) {
    H = fmaf(s, fmaf(s, fmaf(s, fmaf(s, fmaf(s, fmaf(s, 1.0f / 13, 1.0f / 11), 1.0f / 9), 1.0f / 7), 1.0f / 5),
                     1.0f / 3), 1.0f);
    dH = fmaf(s, fmaf(s, fmaf(s, fmaf(s, fmaf(s, 6.0f / 13, 5.0f / 11), 4.0f / 9), 3.0f / 7), 2.0f / 5),
              1.0f / 3);
  } else {
    const float r = sqrtf(s);
    H = atanhf(r) / r;
    dH = (1.0f / (1.0f - s) - H) / (2.0f * s);
  }
}

// Contributions -G . d alpha_SIE / d p to d log L / d p for
// p = (theta_E, q, phi, cx, cy), from the Jacobian of the primed-frame
// deflection alpha'(u) = theta_E sqrt(q) (x'/psi T(t), y'/psi Hh(s)),
// t = f^2 x'^2/psi^2, s = f^2 y'^2/psi^2:
//   d alpha'/d u = theta_E sqrt(q)/(psi r^2) [[y'^2, -x'y'], [-x'y', x'^2]].
__device__ __forceinline__ void sie_grad(const MacroC& m, float tx, float ty, float Gx, float Gy, float out[5]) {
  const float dx = tx - m.cx, dy = ty - m.cy;
  const float xp = fmaf(m.cphi, dx, m.sphi * dy);
  const float yp = fmaf(m.cphi, dy, -m.sphi * dx);
  const float psi2 = fmaf(m.q2, xp * xp, yp * yp);
  const float r2 = fmaf(xp, xp, yp * yp);
  if (!(psi2 > 0.f)) {
    for (int i = 0; i < 5; ++i) out[i] = 0.f;
    return;
  }
  const float psi = sqrtf(psi2);
  const float ipsi = 1.0f / psi;
  const float f2 = m.f * m.f;
  const float t = f2 * xp * xp / psi2, s = f2 * yp * yp / psi2;
  float T, dT, H, dH;
  atan_ratio(t, T, dT);
  atanh_ratio(s, H, dH);
  // primed-frame G
  const float Gpx = fmaf(m.cphi, Gx, m.sphi * Gy);
  const float Gpy = fmaf(m.cphi, Gy, -m.sphi * Gx);
  const float ax1 = m.sqrt_q * xp * ipsi * T;   // alpha'_x / theta_E
  const float ay1 = m.sqrt_q * yp * ipsi * H;   // alpha'_y / theta_E
  out[0] = -(Gpx * ax1 + Gpy * ay1);
  // q
  const float ipsi3 = ipsi * ipsi * ipsi;
  const float lead = (psi2 - 2.0f * m.q2 * xp * xp) * ipsi3 * 0.5f / m.sqrt_q;
  const float dts = -2.0f * m.q * r2 * ipsi3 * ipsi;   // d(t, s)/dq = dts * (x'^2, y'^2)
  const float dax = m.theta_E * (xp * lead * T + m.sqrt_q * xp * ipsi * dT * dts * xp * xp);
  const float day = m.theta_E * (yp * lead * H + m.sqrt_q * yp * ipsi * dH * dts * yp * yp);
  out[1] = -(Gpx * dax + Gpy * day);
  // phi: d alpha/d phi = R (J alpha' - H' J u), H' J u = theta_E sqrt(q)/psi (-y', x')
  const float a = m.theta_E * m.sqrt_q * ipsi;
  const float vx = -m.theta_E * ay1 + a * yp;
  const float vy = m.theta_E * ax1 - a * xp;
  out[2] = -(Gpx * vx + Gpy * vy);
  // centre: d log L/d c = G . H e = G' . H' (R^T e)
  const float k = m.theta_E * m.sqrt_q * ipsi / (r2 > 0.f ? r2 : 1.0f) * (Gpx * yp - Gpy * xp);
  out[3] = k * fmaf(yp, m.cphi, xp * m.sphi);
  out[4] = k * fmaf(yp, m.sphi, -xp * m.cphi);
}

// ---------------------------------------------------------------------------
// EPL partials by forward-mode differentiation in FP64: the forward's series
// evaluated on numbers carrying their derivatives with respect to
// (theta_E, gamma, q, phi, cx, cy).
// ---------------------------------------------------------------------------
struct Dual6 {
  double v, d[6];
};

__device__ __forceinline__ Dual6 dnum(double v, int var) {
  Dual6 r;
  r.v = v;
#pragma unroll
  for (int i = 0; i < 6; ++i) r.d[i] = i == var ? 1.0 : 0.0;
  return r;
}
__device__ __forceinline__ Dual6 operator+(const Dual6& a, const Dual6& b) {
  Dual6 r;
  r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < 6; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
__device__ __forceinline__ Dual6 operator-(const Dual6& a, const Dual6& b) {
  Dual6 r;
  r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < 6; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
__device__ __forceinline__ Dual6 operator*(const Dual6& a, const Dual6& b) {
  Dual6 r;
  r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < 6; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
__device__ __forceinline__ Dual6 operator*(double s, const Dual6& a) {
  Dual6 r;
  r.v = s * a.v;
#pragma unroll
  for (int i = 0; i < 6; ++i) r.d[i] = s * a.d[i];
  return r;
}
__device__ __forceinline__ Dual6 operator+(double s, const Dual6& a) {
  Dual6 r = a;
  r.v += s;
  return r;
}
__device__ __forceinline__ Dual6 inv(const Dual6& a) {   // 1/a
  const double i = 1.0 / a.v, i2 = -i * i;
  Dual6 r;
  r.v = i;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.d[k] = i2 * a.d[k];
  return r;
}
__device__ __forceinline__ Dual6 fn(const Dual6& a, double f, double df) {   // chain rule
  Dual6 r;
  r.v = f;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.d[k] = df * a.d[k];
  return r;
}
__device__ __forceinline__ Dual6 dsqrt(const Dual6& a) {
  const double s = sqrt(a.v);
  return fn(a, s, 0.5 / s);
}
__device__ __forceinline__ Dual6 dlog(const Dual6& a) { return fn(a, log(a.v), 1.0 / a.v); }
__device__ __forceinline__ Dual6 dexp(const Dual6& a) {
  const double e = exp(a.v);
  return fn(a, e, e);
}

// Contributions -G . d alpha_EPL / d p to d log L / d p for
// p = (theta_E, gamma, q, phi, cx, cy) at the image-plane point (tx, ty):
// the forward's deflection (epl_deflection64: the series of the
// hypergeometric factor, the same terms and stopping rule) on dual numbers.
__device__ void epl_grad(const MacroC& m, double tx, double ty, float Gx, float Gy, float out[6]) {
  const Dual6 q = dnum(m.eq, 2), ph = dnum(m.e_phi, 3);
  const Dual6 c = fn(ph, cos(m.e_phi), -sin(m.e_phi)), s = fn(ph, sin(m.e_phi), cos(m.e_phi));
  const Dual6 dx = tx + (-1.0 * dnum(m.ecx, 4)), dy = ty + (-1.0 * dnum(m.ecy, 5));
  const Dual6 xp = c * dx + s * dy, yp = c * dy - s * dx;
  const Dual6 qx = q * xp;
  const Dual6 R2 = qx * qx + yp * yp;
#pragma unroll
  for (int i = 0; i < 6; ++i) out[i] = 0.f;
  if (!(R2.v > 0.0)) return;
  const Dual6 iR = inv(dsqrt(R2));
  const Dual6 er = qx * iR, ei = yp * iR;
  const Dual6 c2 = er * er - ei * ei, s2 = 2.0 * (er * ei);
  const Dual6 f = (1.0 + (-1.0 * q)) * inv(1.0 + q);
  const Dual6 e2mt = 3.0 + (-1.0 * dnum(m.e_gamma, 1));   // 2 - t, t = gamma - 1
  Dual6 wr = er, wi = ei, sr = er, si = ei;
  for (int n = 1; n < kEplMaxTerms; ++n) {
    const Dual6 k = (-1.0 * f) * ((2.0 * n) + (-1.0 * e2mt)) * inv((2.0 * n) + e2mt);
    const Dual6 nr = k * (c2 * wr - s2 * wi);
    const Dual6 ni = k * (s2 * wr + c2 * wi);
    wr = nr;
    wi = ni;
    sr = sr + nr;
    si = si + ni;
    if (fabs(nr.v) + fabs(ni.v) <= 0x1p-56 * (fabs(sr.v) + fabs(si.v))) break;
  }
  const Dual6 b = dnum(m.e_te, 0) * dsqrt(q);
  const Dual6 tm1 = -2.0 + dnum(m.e_gamma, 1);            // t - 1
  const Dual6 a = 2.0 * b * inv(1.0 + q) * dexp(tm1 * dlog(b * iR));
  const Dual6 axp = a * sr, ayp = a * si;
  const Dual6 ax = c * axp - s * ayp, ay = s * axp + c * ayp;
#pragma unroll
  for (int i = 0; i < 6; ++i) out[i] = (float)(-((double)Gx * ax.d[i] + (double)Gy * ay.d[i]));
}

// ---------------------------------------------------------------------------
// residual weights and log-likelihood block partials
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_residual(int npix, const float* __restrict__ model,
                                                 const float* __restrict__ data, const float* __restrict__ w,
                                                 float* __restrict__ resid, float* __restrict__ part) {
  __shared__ float red[256];
  const int b = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  float v = 0.f;
  if (i < npix) {
    const float diff = model[(size_t)b * npix + i] - data[i];
    resid[(size_t)b * npix + i] = -w[i] * diff;
    v = -0.5f * w[i] * diff * diff;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// per-sub-pixel adjoint
// ---------------------------------------------------------------------------
constexpr int kGradMaxP = 8 + 7 * 3;   // EPL 6 (SIE 5) + shear 2 + 7 per Sersic component (<= 3)

// Deterministic sum of v over one wave (xor butterfly, fixed pattern).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// kEpl: the draws' main deflector is an EPL (partials by epl_grad, macro row
// [EPL 6, shear 2, Sersic ...]) instead of an SIE ([SIE 5, shear 2, ...]);
// P: the subhalo pair kernel of the recomputed deflection.
template <int kSplit, bool kKept, class P_ = NfwPairs, bool kEpl = false>
__global__ __launch_bounds__(split_threads(kSplit)) void k_grad_pixel(const ImageDesc* __restrict__ descs, int bpi,
                                                                     const float* __restrict__ lamU,
                                                                     float4* __restrict__ rec, int rec_stride,
                                                                     float* __restrict__ part, int P) {
  __shared__ RangeScratch<kSplit> scratch;   // the recomputed subhalo sum
  __shared__ float wsum[4][kGradMaxP];
  constexpr int kW = split_lanes(kSplit);
  const int di = blockIdx.x / bpi;
  const int blk = blockIdx.x - di * bpi;
  const ImageDesc& d = descs[di];
  const GridC& g = d.g;
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / kW);
  const int t = threadIdx.x - grp * kW;
  const int lp = t / g.s2;
  const int si = t - lp * g.s2;
  const int npix = g.nx * g.ny;
  const int p = blk * g.ppb + lp;
  const bool valid = (lp < g.ppb) && (p < npix);
  const int pp = valid ? p : 0;
  const int row = pp / g.nx, col = pp - (pp / g.nx) * g.nx;
  const int a = si / g.s, b = si - (si / g.s) * g.s;
  const double tx64 = g.ox + g.step * ((double)(col * g.s + b) + 0.5);
  const double ty64 = g.oy + g.step * ((double)(row * g.s + a) + 0.5);
  const float tx = (float)tx64, ty = (float)ty64;
  double sx = 0.0, sy = 0.0;
  if (!kKept) {
    subhalo_ranges<kSplit, P_>(tx, ty, d.sub, d.nloop, grp, t, scratch, sx, sy);
    __syncthreads();
  }
  float c[kGradMaxP];
#pragma unroll
  for (int i = 0; i < kGradMaxP; ++i) c[i] = 0.f;
  if (grp == 0) {
    float bx, by;
    if (kKept) {
      // the traced position the forward launch kept for this sub-pixel
      const float2 bb = d.beta[(size_t)pp * g.s2 + si];
      bx = bb.x;
      by = bb.y;
    } else {
      // recomputed: the same canonical sum as the forward, so the same bits
      double ax, ay;
      total_deflection64<kSplit>(d.mc, tx64, ty64, scratch, t, sx, sy, ax, ay);
      bx = (float)(tx64 - ax);
      by = (float)(ty64 - ay);
    }
    const float lam = valid ? lamU[(size_t)di * npix + pp] * g.area_over_s2 : 0.f;
    float Gx = 0.f, Gy = 0.f, dd[7], gx, gy;
    const int ns = d.src.n, nl = d.ll.n;
    constexpr int kM = kEpl ? 6 : 5;   // main-deflector parameters
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k < ns) {
        sersic_grad(d.src.c[k], bx, by, dd, gx, gy);
#pragma unroll
        for (int m = 0; m < 7; ++m) c[kM + 2 + 7 * k + m] = lam * dd[m];
        Gx = fmaf(lam, gx, Gx);
        Gy = fmaf(lam, gy, Gy);
      } else if (k < ns + nl) {
        sersic_grad(d.ll.c[k - ns], tx, ty, dd, gx, gy);
#pragma unroll
        for (int m = 0; m < 7; ++m) c[kM + 2 + 7 * k + m] = lam * dd[m];
      }
    }
    // the EPL's partials (slots 0..5) are written afterwards by k_grad_epl,
    // from the (theta, G) records, so that this kernel keeps the pair loop's
    // register budget
    if (!kEpl && d.mc.has_sie) sie_grad(d.mc, tx, ty, Gx, Gy, c);
    c[kM] = -(Gx * tx - Gy * ty);
    c[kM + 1] = -(Gx * ty + Gy * tx);
    if (valid) rec[(size_t)di * rec_stride + (size_t)pp * g.s2 + si] = make_float4(tx, ty, Gx, Gy);
  }
  // padding records past the last sub-pixel: G = 0 and a finite x^2 for any
  // subhalo, so they contribute exactly zero
  if (blk == 0 && threadIdx.x < 8) {
    const int first = npix * g.s2;
    const int idx = first + threadIdx.x;
    if (idx < rec_stride) rec[(size_t)di * rec_stride + idx] = make_float4(1e4f, 1e4f, 0.f, 0.f);
  }
  const int wave = threadIdx.x >> 6;
  constexpr int kWaves0 = kW / 64;   // waves of group 0
#pragma unroll
  for (int i = 0; i < kGradMaxP; ++i) {
    if (i < P && wave < kWaves0) {
      const float s = wave_sum(c[i]);
      if ((threadIdx.x & 63) == 0) wsum[wave][i] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < P) {
    float acc = 0.f;
    for (int w = 0; w < kWaves0; ++w) acc += wsum[w][threadIdx.x];
    part[((size_t)di * bpi + blk) * P + threadIdx.x] = acc;
  }
}

// The EPL main deflector's partials per block, in the block decomposition of
// k_grad_pixel (its first wave-group's sub-pixels, its wave order): reads each
// sub-pixel's (theta, G) record and overwrites slots 0..5 of the block's
// partials.  The dual-number arithmetic needs about 200 VGPRs, which is why it
// is not part of k_grad_pixel's pair loop.
template <int kSplit>
__global__ __launch_bounds__(split_lanes(kSplit)) void k_grad_epl(const ImageDesc* __restrict__ descs, int bpi,
                                                                   const float4* __restrict__ rec, int rec_stride,
                                                                   float* __restrict__ part, int P) {
  __shared__ float wsum[4][6];
  constexpr int kW = split_lanes(kSplit);
  const int di = blockIdx.x / bpi;
  const int blk = blockIdx.x - di * bpi;
  const ImageDesc& d = descs[di];
  const GridC& g = d.g;
  const int t = threadIdx.x;
  const int lp = t / g.s2;
  const int si = t - lp * g.s2;
  const int npix = g.nx * g.ny;
  const int p = blk * g.ppb + lp;
  const bool valid = (lp < g.ppb) && (p < npix);
  float c[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid && d.mc.has_epl) {
    const int row = p / g.nx, col = p - (p / g.nx) * g.nx;
    const int a = si / g.s, b = si - (si / g.s) * g.s;
    const double tx64 = g.ox + g.step * ((double)(col * g.s + b) + 0.5);
    const double ty64 = g.oy + g.step * ((double)(row * g.s + a) + 0.5);
    const float4 r = rec[(size_t)di * rec_stride + (size_t)p * g.s2 + si];
    epl_grad(d.mc, tx64, ty64, r.z, r.w, c);
  }
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float v = wave_sum(c[i]);
    if ((threadIdx.x & 63) == 0) wsum[wave][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    float acc = 0.f;
    for (int w = 0; w < kW / 64; ++w) acc += wsum[w][threadIdx.x];
    part[((size_t)di * bpi + blk) * P + threadIdx.x] = acc;
  }
}

// ---------------------------------------------------------------------------
// subhalo-major pass
// ---------------------------------------------------------------------------
// h = g/x^2 and dh/d(x^2) for the NFW term, X2 = x^2, in the forward's units
// (g divided by kNfwRecScale, which each record's c2 carries).  Far
// (X2 >= 1.2): the fitted polynomial, psi = (ln2/2)(1 - kLog2Bias) P,
// F = psi + ln 2 and dg/dX2 = (1 - F)/(2 (X2 - 1)).  Near: series in
// u = X2 - 1 (X2 >= 0.81), the log1p form below, 0 at X2 = 0; both in units
// of ln2/2, then rescaled by kNfwNearScale.
__device__ __forceinline__ void nfw_h_dh_near(float X2, float& h, float& dh) {
  if (!(X2 > 0.f)) {
    h = 0.f;
    dh = 0.f;
    return;
  }
  constexpr float kInvA = (float)(2.0 / kLn2d);    // 1 / (ln2/2)
  constexpr float kInvLn2 = (float)(1.0 / kLn2d);
  const float l2 = __builtin_amdgcn_logf(X2);
  const float Lp = l2 - 2.0f;                       // ln(x/2) / (ln2/2)
  const float iX2 = __builtin_amdgcn_rcpf(X2);
  if (X2 >= 0.81f) {
    const float u = X2 - 1.0f;
    float F = 1.0f / 25.0f;   // F = sum_{k=0..12} (-u)^k / (2k+1)
    F = fmaf(F, -u, 1.0f / 23.0f);
    F = fmaf(F, -u, 1.0f / 21.0f);
    F = fmaf(F, -u, 1.0f / 19.0f);
    F = fmaf(F, -u, 1.0f / 17.0f);
    F = fmaf(F, -u, 1.0f / 15.0f);
    F = fmaf(F, -u, 1.0f / 13.0f);
    F = fmaf(F, -u, 1.0f / 11.0f);
    F = fmaf(F, -u, 1.0f / 9.0f);
    F = fmaf(F, -u, 1.0f / 7.0f);
    F = fmaf(F, -u, 1.0f / 5.0f);
    F = fmaf(F, -u, 1.0f / 3.0f);
    F = fmaf(F, -u, 1.0f);
    // S = (1 - F)/u = sum_{j=0..11} (-1)^j u^j / (2j+3)
    float S = -1.0f / 25.0f;
    S = fmaf(S, u, 1.0f / 23.0f);
    S = fmaf(S, u, -1.0f / 21.0f);
    S = fmaf(S, u, 1.0f / 19.0f);
    S = fmaf(S, u, -1.0f / 17.0f);
    S = fmaf(S, u, 1.0f / 15.0f);
    S = fmaf(S, u, -1.0f / 13.0f);
    S = fmaf(S, u, 1.0f / 11.0f);
    S = fmaf(S, u, -1.0f / 9.0f);
    S = fmaf(S, u, 1.0f / 7.0f);
    S = fmaf(S, u, -1.0f / 5.0f);
    S = fmaf(S, u, 1.0f / 3.0f);
    h = fmaf(F, kInvA, Lp) * iX2;
    dh = fmaf(S, kInvLn2, -h) * iX2;
    h *= kNfwNearScale;
    dh *= kNfwNearScale;
  } else {
    const float w = __builtin_amdgcn_sqrtf(1.0f - X2);
    const float ropw = __builtin_amdgcn_rcpf(1.0f + w);
    const float tt = -0.5f * X2 * ropw;
    const float uu = 1.0f + tt;
    const float lp = (uu == 1.0f) ? tt * kInvA : 2.0f * __builtin_amdgcn_logf(uu) * tt * __builtin_amdgcn_rcpf(uu - 1.0f);
    const float iw = __builtin_amdgcn_rcpf(w);
    const float g = fmaf(-Lp * X2, ropw, lp) * iw;
    // F = atanh(w)/w = ln((1+w)^2 / X2) / (2 w)
    const float F = kLn2 * (2.0f * __builtin_amdgcn_logf(1.0f + w) - l2) * 0.5f * iw;
    h = g * iX2;
    dh = ((1.0f - F) * kInvLn2 / (X2 - 1.0f) - h) * iX2;
    h *= kNfwNearScale;
    dh *= kNfwNearScale;
  }
}

// Far field (X2 >= 1.2) from l2 = log2(X2), y2 = 1/X2, the fitted
// polynomial p = P(y) (psi = (ln2/2)(1 - kLog2Bias) P, F = psi + ln 2) and
// inv = 1/(X2 - 1): h = (l2 + p) y2, dh/d(X2) = ((1 - F)/(2 (X2 - 1)) - h) y2.
__device__ __forceinline__ void nfw_h_dh_far(float l2, float y2, float p, float inv, float& h, float& dh) {
  constexpr float kA1 = (float)(0.5 * kLn2d * (1.0 - kLog2Bias));   // psi = kA1 * P
  constexpr float kInv2U = (float)(0.5 / kNfwRecScale);
  h = (l2 + p) * y2;
  const float oneF = fmaf(-kA1, p, (float)(1.0 - kLn2d));           // 1 - F
  dh = fmaf(oneF * kInv2U, inv, -h) * y2;
}

// grid (ceil(n / kSubhaloBlock), B, kRecParts); lane = subhalo k of draw b, read from
// the draws' SoA [B][n] (x, y, Rs, alpha_Rs).  Writes the part partial
// (x, y, alpha_Rs) gradients to gpart[q][b][k][3].
__global__ __launch_bounds__(kSubhaloBlock) void k_grad_subhalo(const float* __restrict__ sub_x, const float* __restrict__ sub_y,
                                                    const float* __restrict__ sub_rs, const float* __restrict__ sub_ars,
                                                    const float4* __restrict__ rec, int rec_stride,
                                                    int nrec_loop, int n, float* __restrict__ gpart) {
  const int b = blockIdx.y, q = blockIdx.z, B = gridDim.y;
  const int k = blockIdx.x * kSubhaloBlock + threadIdx.x;
  const bool valid = k < n;
  const size_t j = (size_t)b * n + (valid ? k : 0);
  const float x0 = sub_x[j], y0 = sub_y[j];
  // c1 = 1/Rs^2 and c2 = kNfwRecScale alpha_Rs / ((1 - ln 2) Rs), each rounded once
  const double rs = sub_rs[j];
  const float c1 = (float)(1.0 / (rs * rs));
  const float c2 = (float)(kNfwRecScale * (double)sub_ars[j] / ((1.0 - kLn2d) * rs));
  // alpha / alpha_Rs = c2n * h * d  (h in units of ln2/2)
  const float c2n = sqrtf(c1) * (float)(kNfwRecScale / (1.0 - kLn2d));
  const float c1x2 = 2.0f * c1;
  const float4* __restrict__ r = rec + (size_t)b * rec_stride;
  const int kb = part_bound(nrec_loop, kRecParts, q), ke = part_bound(nrec_loop, kRecParts, q + 1);
  float hx = 0.f, lx = 0.f, hy = 0.f, ly = 0.f, ha = 0.f, la = 0.f;
  float4 n0 = r[kb], n1 = r[kb + 1], n2 = r[kb + 2], n3 = r[kb + 3];
  for (int j0 = kb; j0 < ke; j0 += 64) {
    const int jend = min(j0 + 64, ke);
    float px = 0.f, py = 0.f, pa = 0.f;
    for (int j = j0; j < jend; j += 4) {
      const float4 rr[4] = {n0, n1, n2, n3};
      n0 = r[j + 4];
      n1 = r[j + 5];
      n2 = r[j + 6];
      n3 = r[j + 7];
      float dx[4], dy[4], X[4], y[4], l2[4], y2[4], p[4], inv[4], h[4], dh[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        dx[m] = rr[m].x - x0;
        dy[m] = rr[m].y - y0;
        X[m] = fmaf(dy[m], dy[m], dx[m] * dx[m]) * c1;
        y[m] = __builtin_amdgcn_rsqf(X[m]);
        l2[m] = __builtin_amdgcn_logf(X[m]);
        y2[m] = y[m] * y[m];
      }
      // lanes are different subhalos, so a wave seldom agrees on the short
      // far-field form: one polynomial for every pair keeps the wave coherent
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        float q = kNfwP[0];
#pragma unroll
        for (int i = 1; i <= JT_NFW_POLY_DEGREE; ++i) q = fmaf(q, y[m], kNfwP[i]);
        p[m] = q;
        inv[m] = __builtin_amdgcn_rcpf(X[m] - 1.0f);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) nfw_h_dh_far(l2[m], y2[m], p[m], inv[m], h[m], dh[m]);
      if (__builtin_expect(fminf(fminf(X[0], X[1]), fminf(X[2], X[3])) < 1.2f, 0)) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
          if (X[m] < 1.2f) nfw_h_dh_near(X[m], h[m], dh[m]);
      }
      // c2, -c2n and the 2 c1 of e are applied once per subhalo below
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const float GD = fmaf(rr[m].z, dx[m], rr[m].w * dy[m]);
        const float e = c1x2 * dh[m] * GD;
        px = fmaf(e, dx[m], fmaf(h[m], rr[m].z, px));
        py = fmaf(e, dy[m], fmaf(h[m], rr[m].w, py));
        pa = fmaf(h[m], GD, pa);
      }
    }
    two_sum_acc(hx, lx, px);
    two_sum_acc(hy, ly, py);
    two_sum_acc(ha, la, pa);
  }
  if (valid) {
    float* o = gpart + (((size_t)q * B + b) * n + k) * 3;
    o[0] = c2 * (hx + lx);
    o[1] = c2 * (hy + ly);
    o[2] = -c2n * (ha + la);
  }
}

// h = c2 T(x) and dh = dh/d(X2) of the truncated pair term for the record r
// (X2 = x^2 = r^2 c1).  Far field (X2 >= Xf, the record's polynomial
// W(u) = sum a_k u^k, u = y k1 - 1, y = 1/x): h = y^2 W and, with
// dy/dX2 = -y^3/2, dh = -y^4 (W + (k1 y / 2) W'(u)).
__device__ __forceinline__ void tnfw_h_dh_far(float X2, const TRec& r, float& h, float& dh) {
  {
    const float y = __builtin_amdgcn_rsqf(X2);
    const float u = fmaf(y, r.k1, -1.0f);
    float p = r.a[kTnfwFarDeg], dp = 0.f;
#pragma unroll
    for (int k = kTnfwFarDeg - 1; k >= 0; --k) {
      dp = fmaf(dp, u, p);
      p = fmaf(p, u, r.a[k]);
    }
    const float y2 = y * y;
    h = p * y2;
    dh = -(y2 * y2) * fmaf(0.5f * r.k1 * y, dp, p);
  }
}

// The same for X2 < Xf: the general form, and from the projected mass's
// derivative -- the surface density of the truncated profile (Baltz, Marshall
// & Oguri 2009) --
//   dG/dX2 = (A/2) K,  K = (tau^2 + 1)(1 - F)/(x^2 - 1) + 2F - pi/s
//                          + (tau^2 - 1) L/(tau s),  L = ln(x/(s + tau)),
// dh = (c2 K/2 - h)/X2 (c2 carries A).  (1 - F)/(x^2 - 1) is the series
// 1/3 - v/5 + v^2/7 - ... in v = x^2 - 1 near x = 1.  0 at the centre.
__device__ __forceinline__ void tnfw_h_dh_near(float X2, const TRec& r, float& h, float& dh) {
  constexpr float kPi = 3.14159265358979323846f;
  if (!(X2 > 1e-30f)) {
    h = 0.f;
    dh = 0.f;
    return;
  }
  float F, s, lp1;
  h = r.c2 * tnfw_T_general(X2, r, F, s, lp1);
  const float v = X2 - 1.0f;
  float oneF;   // (1 - F)/(x^2 - 1)
  if (fabsf(v) < 0.2f) {
    float S = -1.0f / 25.0f;
    S = fmaf(S, v, 1.0f / 23.0f);
    S = fmaf(S, v, -1.0f / 21.0f);
    S = fmaf(S, v, 1.0f / 19.0f);
    S = fmaf(S, v, -1.0f / 17.0f);
    S = fmaf(S, v, 1.0f / 15.0f);
    S = fmaf(S, v, -1.0f / 13.0f);
    S = fmaf(S, v, 1.0f / 11.0f);
    S = fmaf(S, v, -1.0f / 9.0f);
    S = fmaf(S, v, 1.0f / 7.0f);
    S = fmaf(S, v, -1.0f / 5.0f);
    oneF = fmaf(S, v, 1.0f / 3.0f);
  } else {
    oneF = (1.0f - F) * __builtin_amdgcn_rcpf(v);
  }
  const float is = __builtin_amdgcn_rcpf(s);
  const float K = fmaf(r.t2 + 1.0f, oneF, fmaf(2.0f, F, -kPi * is)) - (r.t2 - 1.0f) * lp1 * r.itau * is;
  dh = fmaf(0.5f * r.c2, K, -h) * __builtin_amdgcn_rcpf(X2);
}

// The subhalo-major pass for truncated subhalos, far pairs: as k_grad_subhalo,
// with each lane's record read from the draw's table built for alpha_Rs = 1
// (utab [B][records]), so that the sums are per unit alpha_Rs: d log L/d(x, y)
// is alpha_Rs times them and d log L/d alpha_Rs is minus the h G.d sum.  Every
// lane evaluates the far form, and pairs with X2 < Xf add zero here: the lanes
// of a wave are different subhalos, so a general form evaluated here would run
// for the whole wave wherever any of its 64 subhalos is near, and
// k_grad_subhalo_tnfw_near takes those pairs instead.
__global__ __launch_bounds__(kSubhaloBlock) void k_grad_subhalo_tnfw(const TRec* __restrict__ utab, int records,
                                                                    const float* __restrict__ sub_ars,
                                                                    const float4* __restrict__ rec, int rec_stride,
                                                                    int nrec_loop, int n, float* __restrict__ gpart) {
  const int b = blockIdx.y, q = blockIdx.z, B = gridDim.y;
  // the lane block rotates with the draw and the part, so that consecutive
  // blocks of a draw spread over the XCDs
  const int xb = (int)((blockIdx.x + blockIdx.y + blockIdx.z) % gridDim.x);
  const int k = xb * kSubhaloBlock + threadIdx.x;
  const bool valid = k < n;
  const TRec R = utab[(size_t)b * records + (valid ? k : 0)];
  const float c1x2 = 2.0f * R.c1;
  const float4* __restrict__ r = rec + (size_t)b * rec_stride;
  const int kb = part_bound(nrec_loop, kRecPartsTnfw, q), ke = part_bound(nrec_loop, kRecPartsTnfw, q + 1);
  float hx = 0.f, lx = 0.f, hy = 0.f, ly = 0.f, ha = 0.f, la = 0.f;
  for (int j0 = kb; j0 < ke; j0 += 64) {
    const int jend = min(j0 + 64, ke);
    float px = 0.f, py = 0.f, pa = 0.f;
    for (int j = j0; j < jend; ++j) {
      const float4 rr = r[j];
      const float dx = rr.x - R.x, dy = rr.y - R.y;
      const float X2 = fmaf(dy, dy, dx * dx) * R.c1;
      float h, dh;
      tnfw_h_dh_far(X2, R, h, dh);
      const bool far = !(X2 < R.Xf);
      h = far ? h : 0.0f;
      dh = far ? dh : 0.0f;
      const float GD = fmaf(rr.z, dx, rr.w * dy);
      const float e = c1x2 * dh * GD;
      px = fmaf(e, dx, fmaf(h, rr.z, px));
      py = fmaf(e, dy, fmaf(h, rr.w, py));
      pa = fmaf(h, GD, pa);
    }
    two_sum_acc(hx, lx, px);
    two_sum_acc(hy, ly, py);
    two_sum_acc(ha, la, pa);
  }
  if (valid) {
    const float ars = sub_ars[(size_t)b * n + k];
    float* o = gpart + (((size_t)q * B + b) * n + k) * 3;
    o[0] = ars * (hx + lx);
    o[1] = ars * (hy + ly);
    o[2] = -(ha + la);
  }
}

// The near pairs of the truncated subhalos (X2 < Xf, within
// rho = (Xf / c1)^(1/2) of the centre), which the far pass leaves out: one
// wave per (subhalo k, draw b) visits the box of the sub-pixel grid around the
// centre (rho widened by 0.1% and two sub-pixels, so that no pair the X2 test
// admits lies outside it), lane l the box cells l, l + 64, ...; the same X2
// test as the far pass decides each pair, so every pair is counted by exactly
// one of the two passes, and the lanes of a wave run the general form
// together.  The lane sums are added in a fixed butterfly order and written as
// part kRecPartsTnfw of gpart.  rec holds the sub-pixel records
// [b][pixel * s^2 + sub-pixel]; g is the draws' common grid.
__global__ __launch_bounds__(64) void k_grad_subhalo_tnfw_near(const TRec* __restrict__ utab, int records,
                                                              const float* __restrict__ sub_ars,
                                                              const float4* __restrict__ rec, int rec_stride, GridC g,
                                                              int n, float* __restrict__ gpart) {
  const int k = blockIdx.x, b = blockIdx.y, B = gridDim.y;
  const int lane = threadIdx.x;
  const TRec R = utab[(size_t)b * records + k];
  const int W = g.nx * g.s, H = g.ny * g.s;
  const double is = 1.0 / g.step;
  const double rho = sqrt((double)R.Xf / (double)R.c1) * 1.001 + 2.0 * g.step;
  // sub-pixel column c sits at ox + step (c + 1/2); clamp in FP64 before the
  // conversion to int, so that a far-away centre cannot overflow it
  auto lo = [&](double c, double o, int m) {
    return (int)fmin(fmax(ceil((c - rho - o) * is - 0.5), 0.0), (double)m);
  };
  auto hi = [&](double c, double o, int m) {
    return (int)fmin(fmax(floor((c + rho - o) * is - 0.5), -1.0), (double)(m - 1));
  };
  const int cx0 = lo(R.x, g.ox, W), cx1 = hi(R.x, g.ox, W);
  const int cy0 = lo(R.y, g.oy, H), cy1 = hi(R.y, g.oy, H);
  const int bw = cx1 - cx0 + 1, bh = cy1 - cy0 + 1;
  const int cells = bw > 0 && bh > 0 ? bw * bh : 0;
  const float4* __restrict__ r = rec + (size_t)b * rec_stride;
  const float c1x2 = 2.0f * R.c1;
  float px = 0.f, py = 0.f, pa = 0.f;
  for (int i = lane; i < cells; i += 64) {
    const int iy = i / bw;
    const int cy = cy0 + iy, cx = cx0 + (i - iy * bw);
    const int row = cy / g.s, col = cx / g.s;
    const int si = (cy - row * g.s) * g.s + (cx - col * g.s);
    const float4 rr = r[((size_t)row * g.nx + col) * g.s2 + si];
    const float dx = rr.x - R.x, dy = rr.y - R.y;
    const float X2 = fmaf(dy, dy, dx * dx) * R.c1;
    if (X2 < R.Xf) {
      float h, dh;
      tnfw_h_dh_near(X2, R, h, dh);
      const float GD = fmaf(rr.z, dx, rr.w * dy);
      const float e = c1x2 * dh * GD;
      px = fmaf(e, dx, fmaf(h, rr.z, px));
      py = fmaf(e, dy, fmaf(h, rr.w, py));
      pa = fmaf(h, GD, pa);
    }
  }
  px = wave_sum(px);
  py = wave_sum(py);
  pa = wave_sum(pa);
  if (lane == 0) {
    const float ars = sub_ars[(size_t)b * n + k];
    float* o = gpart + (((size_t)kRecPartsTnfw * B + b) * n + k) * 3;
    o[0] = ars * px;
    o[1] = ars * py;
    o[2] = -pa;
  }
}

// Fixed-order final sums: macro partials over blocks (TwoSum), log L over
// residual blocks (FP64), subhalo quarters in order.
__global__ __launch_bounds__(256) void k_grad_finalize(int B, int P, int bpi, const float* __restrict__ part,
                                                      float* __restrict__ g_macro, int nres,
                                                      const float* __restrict__ lpart, double* __restrict__ logL,
                                                      int n, int parts, const float* __restrict__ gpart,
                                                      float* __restrict__ g_sub) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  const long nm = (long)B * P, nl = B, ns = (long)B * n * 3;
  if (i < nm) {
    const int b = (int)(i / P), p = (int)(i - (long)b * P);
    float hi = 0.f, lo = 0.f;
    for (int j = 0; j < bpi; ++j) two_sum_acc(hi, lo, part[((size_t)b * bpi + j) * P + p]);
    g_macro[i] = hi + lo;
  } else if (i < nm + nl) {
    const int b = (int)(i - nm);
    double acc = 0.0;
    for (int j = 0; j < nres; ++j) acc += (double)lpart[(size_t)b * nres + j];
    if (logL) logL[b] = acc;
  } else if (i < nm + nl + ns && g_sub) {
    const long e = i - nm - nl;
    float hi = 0.f, lo = 0.f;
    for (int q = 0; q < parts; ++q) two_sum_acc(hi, lo, gpart[(size_t)q * ns + e]);
    g_sub[e] = hi + lo;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_residual(int B, int npix, const float* model, const float* data, const float* w, float* resid,
                           float* part, int* nblocks, hipStream_t st) {
  const int nb = (npix + 255) / 256;
  *nblocks = nb;
  hipLaunchKernelGGL(k_residual, dim3(nb, B), dim3(256), 0, st, npix, model, data, w, resid, part);
  return hipGetLastError();
}

hipError_t launch_grad_pixel(int split, bool kept, bool tnfw, bool epl, int B, int bpi, const ImageDesc* descs,
                             const float* lamU, float4* rec, int rec_stride, float* part, int P, hipStream_t st) {
  const dim3 grid((unsigned)((long)B * bpi));
#define JT_GP(S, K, Q, E) hipLaunchKernelGGL((k_grad_pixel<S, K, Q, E>), grid, dim3(split_threads(S)), 0, st, descs, \
                                             bpi, lamU, rec, rec_stride, part, P)
#define JT_GP_S(K, Q, E) \
  if (split == 1) JT_GP(1, K, Q, E); else if (split == 2) JT_GP(2, K, Q, E); \
  else if (split == 4) JT_GP(4, K, Q, E); else JT_GP(8, K, Q, E)
  if (kept) {
    // the positions come from the forward launch: no pair kernel is run
    if (epl) { JT_GP_S(true, NfwPairs, true); } else { JT_GP_S(true, NfwPairs, false); }
  } else if (tnfw) {
    if (epl) { JT_GP_S(false, TnfwPairs, true); } else { JT_GP_S(false, TnfwPairs, false); }
  } else {
    if (epl) { JT_GP_S(false, NfwPairs, true); } else { JT_GP_S(false, NfwPairs, false); }
  }
#undef JT_GP_S
#undef JT_GP
  if (epl) {
#define JT_GE(S) hipLaunchKernelGGL((k_grad_epl<S>), grid, dim3(split_lanes(S)), 0, st, descs, bpi, rec, rec_stride, \
                                    part, P)
    if (split == 1) JT_GE(1); else if (split == 2) JT_GE(2); else if (split == 4) JT_GE(4); else JT_GE(8);
#undef JT_GE
  }
  return hipGetLastError();
}

hipError_t launch_grad_subhalo(int B, int n, const float* x, const float* y, const float* rs, const float* ars,
                               const float4* rec, int rec_stride, int nrec_loop, float* gpart, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_subhalo, dim3((n + kSubhaloBlock - 1) / kSubhaloBlock, B, kRecParts), dim3(kSubhaloBlock),
                     0, st, x, y, rs, ars, rec,
                     rec_stride, nrec_loop, n, gpart);
  return hipGetLastError();
}

hipError_t launch_grad_subhalo_tnfw(int B, int n, const TRec* utab, int records, const float* ars,
                                    const float4* rec, int rec_stride, int nrec_loop, const GridC& g, float* gpart,
                                    hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_subhalo_tnfw, dim3((n + kSubhaloBlock - 1) / kSubhaloBlock, B, kRecPartsTnfw),
                     dim3(kSubhaloBlock), 0, st, utab, records, ars, rec, rec_stride, nrec_loop, n, gpart);
  hipLaunchKernelGGL(k_grad_subhalo_tnfw_near, dim3(n, B), dim3(64), 0, st, utab, records, ars, rec, rec_stride, g,
                     n, gpart);
  return hipGetLastError();
}

hipError_t launch_grad_finalize(int B, int P, int bpi, const float* part, float* g_macro, int nres,
                                const float* lpart, double* logL, int n, int parts, const float* gpart, float* g_sub,
                                hipStream_t st) {
  const long total = (long)B * P + B + (long)B * n * 3;
  hipLaunchKernelGGL(k_grad_finalize, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, B, P, bpi, part,
                     g_macro, nres, lpart, logL, n, parts, gpart, g_sub);
  return hipGetLastError();
}

int grad_max_params() { return kGradMaxP; }

}  // namespace jt
