/*
 * jt.h -- C ABI of libjt, an MI355X (gfx950) lensed-image simulator.
 *
 * The library computes the paper's three-step image simulation (JAXtronomy,
 * section "Improvements over lenstronomy in image simulation"):
 *   1. every image-plane angle theta is mapped to the source plane,
 *      beta = theta - sum of the deflections of all deflectors at theta;
 *   2. the source light is evaluated at beta (lens light at theta);
 *   3. the image is blurred by the point spread function.
 * The deflectors are those of the paper's deflector table that the path uses:
 * SIE (NIE with zero core; SIS as q = 1), external SHEAR and NFW (the subhalo
 * profile), plus a point mass used only by tests.  The light profile is the
 * elliptical Sersic of the flux table (SERSIC_ELLIPSE_Q_PHI parameterisation).
 *
 * Conventions shared by every call
 *  - Angles are arcsec, position angles radians (counter-clockwise from +x to
 *    the major axis).  Images are row-major float32 [ny][nx]; row i runs along
 *    +y, column j along +x, and the grid is centred on (x0, y0).
 *  - Sub-pixel (a, b) of pixel (i, j), a, b in [0, s):
 *      x = x0 + (j - (nx-1)/2) d + ((b + 1/2)/s - 1/2) d,  y likewise with (i, a).
 *    A pixel value is d^2 times the mean sub-pixel surface brightness.
 *  - All device pointers are caller-owned; the library never frees them and
 *    never keeps them after the call returns (except through explicit handles).
 *    Host pointers are read during the call only.
 *  - Calls are asynchronous on the given HIP stream (0 = the null stream).
 *    Argument errors return synchronously and launch nothing.  A device
 *    fault surfaces as JT_EDEVICE from jt_sync or a later call.
 *  - Arithmetic on the device is FP32; host parameter preparation is FP64.
 *  - Every call returning jt_status sets a thread-local message readable with
 *    jt_last_error() when it returns anything but JT_OK.
 */
#ifndef JT_H
#define JT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  JT_OK = 0,
  JT_EINVAL = 1,         /* bad argument (null pointer, size, parameter range) */
  JT_ENOMEM = 2,         /* device allocation failed, or a request can never fit */
  JT_EDEVICE = 3,        /* HIP runtime or kernel error */
  JT_EUNSUPPORTED = 4,   /* valid but not implemented (e.g. too many components) */
  JT_EBUSY = 5,          /* resource still in use */
  JT_ECANCELLED = 6      /* serving ticket cancelled */
} jt_status;

/* Limits (compile-time; exceeded -> JT_EUNSUPPORTED). */
#define JT_MAX_SERSIC 8        /* per light list (source or lens light)       */
#define JT_MAX_POINT_MASS 16   /* point masses per lens                       */
#define JT_MAX_PSF 255         /* largest odd PSF side for the direct path    */
#define JT_NOALLOC_SCRATCH_BYTES (8u << 20) /* static scratch of jt_simulate_image_noalloc, per device */

typedef struct jt_ctx jt_ctx;  /* one per device: workspace, resident tables, profiling */

/* Create a context on HIP device `device` (it becomes current on the calling
 * thread).  *out receives the context.  JT_EINVAL for a bad device index. */
jt_status jt_create(int device, jt_ctx** out);
/* Destroy a context: waits for its work, frees its workspace and handles. */
void jt_destroy(jt_ctx* ctx);
/* Thread-local description of the last non-OK status on this thread. */
const char* jt_last_error(void);
/* Library version string. */
const char* jt_version(void);
/* Wait for all work on `stream`; JT_EDEVICE if the device reported an error. */
jt_status jt_sync(jt_ctx* ctx, hipStream_t stream);

/* ----------------------------------------------------------------------
 * Parameters (plain host structs, read during the call)
 * -------------------------------------------------------------------- */
typedef struct {
  int nx, ny;            /* pixels, >= 1 */
  int supersample;       /* s >= 1 sub-pixels per axis */
  double pixel_scale;    /* d > 0, arcsec per pixel */
  double x0, y0;         /* grid centre */
} jt_grid;

/* SIE (Kormann et al. 1994; Keeton 2001): kappa = theta_E / (2 sqrt(q x'^2 + y'^2/q)).
 * theta_E > 0, q in (0, 1], centre (cx, cy). */
typedef struct { double theta_E, q, phi, cx, cy; } jt_sie;

/* EPL, elliptical power-law main deflector (Tessore & Metcalf 2015; in the
 * paper's deflector table):
 * kappa = (3 - gamma)/2 (theta_E / sqrt(q x'^2 + y'^2/q))^(gamma - 1), gamma the
 * slope of the 3-D density (gamma = 2 is the SIE above).  theta_E >= 0,
 * gamma in (1, 3), q in [0.05, 1], position angle phi, centre (cx, cy).  The
 * deflection is the hypergeometric closed form, summed as its power series in
 * FP64 to full double precision (more terms as q falls: about 30 at q = 0.6,
 * 400 at q = 0.05). */
typedef struct { double theta_E, gamma, q, phi, cx, cy; } jt_epl;

/* External shear about the origin: alpha = (g1 x + g2 y, g2 x - g1 y). */
typedef struct { double gamma1, gamma2; } jt_shear;

/* NFW subhalos as device float32 structure-of-arrays of length n (arcsec):
 * centre (x, y), scale radius Rs > 0 and alpha_Rs = |alpha| at r = Rs.
 * alpha_k = alpha_Rs/(1 - ln 2) * g(r/Rs)/(r/Rs) * (dx, dy)/r with
 * g(x) = ln(x/2) + F(x) (Bartelmann 1996; Golse & Kneib 2002).
 * r_trunc != NULL (device float32[n], each > 0): truncated NFW (TNFW, in the
 * paper's deflector table) in the form of Baltz, Marshall & Oguri (2009) with
 * truncation exponent 1, density rho_NFW tau^2/(tau^2 + (r/Rs)^2),
 * tau = r_trunc/Rs, and the same rho_0 as the NFW of this alpha_Rs, so that
 * alpha_k = alpha_Rs/(1 - ln 2) * G(r/Rs, tau)/(r/Rs) * (dx, dy)/r with G the
 * projected mass in the units of g.  Device arrays are not validated. */
typedef struct { int n; const float *x, *y, *Rs, *alpha_Rs, *r_trunc; } jt_nfw;

/* Point masses (test profile), host float64 arrays of length n <= 16:
 * alpha = theta_E^2 (dx, dy) / r^2. */
typedef struct { int n; const double *x, *y, *theta_E; } jt_point_masses;

typedef struct {
  int has_sie, has_shear;
  jt_sie sie;
  jt_shear shear;
  jt_nfw nfw;                /* n = 0: no subhalos */
  uint64_t subhalo_handle;   /* nonzero: a table from jt_upload_subhalos or jt_upload_tnfw, `nfw` ignored */
  jt_point_masses pm;        /* n = 0: none */
  int has_epl;               /* adds an EPL (with or without the SIE) */
  jt_epl epl;
} jt_lens;

/* Elliptical Sersic: I = amp exp(-b_n [(R/R_sersic)^(1/n) - 1]),
 * R = sqrt(q x'^2 + y'^2/q); amp = I(R_sersic); R_sersic > 0, n in [0.2, 10],
 * q in (0, 1]. */
typedef struct { double amp, R_sersic, n_sersic, q, phi, cx, cy; } jt_sersic;

/* Elliptical Gaussian light (the paper's flux table: GAUSSIAN, GAUSSIAN_ELLIPSE,
 * MULTI_GAUSSIAN as several of them): I = amp/(2 pi sigma^2) exp(-R^2/(2 sigma^2)),
 * R^2 = q x'^2 + y'^2/q, so amp is the total flux.  sigma > 0, q in (0, 1]. */
typedef struct { double amp, sigma, q, phi, cx, cy; } jt_gaussian;

/* Core-Sersic light (CORE_SERSIC; Graham et al. 2003, Trujillo et al. 2004):
 * I = amp (1 + (R_b/R)^alpha)^(gamma/alpha)
 *         exp(-b_n [((R^alpha + R_b^alpha)/R_sersic^alpha)^(1/(n alpha)) - 1]),
 * R as the Sersic's, floored at 1e-6 R_b; R_b -> 0 gives the Sersic.
 * R_sersic, R_b > 0, n in [0.2, 10], gamma in [0, 2), alpha in (0, 20]. */
typedef struct { double amp, R_sersic, R_b, n_sersic, gamma, alpha, q, phi, cx, cy; } jt_core_sersic;

/* Cartesian shapelets (SHAPELETS; Refregier 2003): I = sum over
 * n1 + n2 <= n_max of coeff c_{n1 n2} beta^-1 phi_n1((x-cx)/beta) phi_n2((y-cy)/beta),
 * phi_n(u) = (2^n sqrt(pi) n!)^(-1/2) H_n(u) exp(-u^2/2).  coeff: host double
 * [(n_max+1)(n_max+2)/2], ordered by n = n1 + n2, then n2 = 0..n.
 * n_max in [0, 10], beta > 0. */
typedef struct { int n_max; double beta, cx, cy; const double* coeff; } jt_shapelets;

/* A light list: Sersic components (host array c[n], n <= JT_MAX_SERSIC) and
 * optionally up to 8 Gaussians, 2 core-Sersic components and one shapelet
 * set (host arrays, read during the call).
 * bn_exact = 0: b_n = 1.9992 n - 0.3271 (Capaccioli 1989);
 * bn_exact = 1: b_n solves P(2n, b_n) = 1/2 (R_sersic is the half-light radius).
 * The batched draws, the adjoint and the linear amplitude solver take Sersic
 * components only. */
typedef struct {
  int n; const jt_sersic* c; int bn_exact;
  int n_gauss; const jt_gaussian* gauss;
  int n_core; const jt_core_sersic* core;
  const jt_shapelets* shapelets;     /* NULL: none */
} jt_light;

/* b_n of the Sersic profile as the library uses it (host FP64): the
 * Capaccioli fit 1.9992 n - 0.3271, or (exact != 0) the root of
 * P(2n, b) = 1/2 by Newton iteration on the regularised incomplete gamma.
 * Returns NaN for n outside [0.2, 10]. */
double jt_sersic_bn(double n, int exact);

/* ----------------------------------------------------------------------
 * Step 1: ray shooting (deflection angles at each deflector)
 * -------------------------------------------------------------------- */
/* beta = theta - sum of the deflections of `lens` at the n points
 * (x[i], y[i]) (device float32).  Outputs bx, by: device float32[n],
 * overlapping neither the inputs nor each other (JT_EINVAL).  n = 0 is a
 * no-op. */
jt_status jt_ray_shoot(jt_ctx* ctx, int n, const float* x, const float* y,
                       const jt_lens* lens, float* bx, float* by, hipStream_t stream);

/* The total deflection alpha(theta) itself (same kernel as jt_ray_shoot). */
jt_status jt_deflection(jt_ctx* ctx, int n, const float* x, const float* y,
                        const jt_lens* lens, float* ax, float* ay, hipStream_t stream);

/* ----------------------------------------------------------------------
 * Step 2: surface brightness on the traced grid
 * -------------------------------------------------------------------- */
/* sb[i] = sum_src I(bx[i], by[i]) + sum_lens_light I(x[i], y[i]).
 * Device float32 arrays of length n.  `src` or `lens_light` may be NULL
 * (no component); x, y may be NULL when lens_light is empty, bx, by when src
 * is.  sb may be one of the inputs itself (in place) but must not otherwise
 * overlap them (JT_EINVAL). */
jt_status jt_source_sb(jt_ctx* ctx, int n, const float* x, const float* y,
                       const float* bx, const float* by, const jt_light* src,
                       const jt_light* lens_light, float* sb, hipStream_t stream);

/* ----------------------------------------------------------------------
 * Step 3: PSF convolution
 * -------------------------------------------------------------------- */
/* out[i][j] = sum_{a,b} psf[a][b] img[i - a + c][j - b + c], c = (k-1)/2,
 * zero outside the image, same size (a true convolution).  img, out: device
 * float32 [ny][nx], out overlapping neither img nor psf (JT_EINVAL); psf:
 * device float32 [k][k], k odd.
 * method: 0 = auto (direct below the measured crossover), 1 = direct
 * (FP32 matrix-core products of LDS-staged tiles, k <= JT_MAX_PSF), 2 = FFT
 * (FP64 transform). */
jt_status jt_convolve(jt_ctx* ctx, const float* img, int nx, int ny, const float* psf,
                      int k, int method, float* out, hipStream_t stream);

/* The method (1 direct, 2 FFT) that method 0 selects for an nx x ny image
 * and a k x k PSF; 0 when neither path takes the shape.  Host only. */
int jt_convolve_auto_method(int nx, int ny, int k);

/* ----------------------------------------------------------------------
 * Fused simulation: steps 1-2 and the supersample average in one kernel,
 * then step 3.
 * -------------------------------------------------------------------- */
/* out: device float32 [ny][nx], not overlapping psf (JT_EINVAL).  psf: device
 * float32 [k][k] (odd k), or NULL with k = 0 to return the unconvolved image.
 * Uses ctx workspace for the unconvolved image when a PSF is given. */
jt_status jt_simulate_image(jt_ctx* ctx, const jt_grid* grid, const jt_lens* lens,
                            const jt_light* src, const jt_light* lens_light,
                            const float* psf, int k, float* out, hipStream_t stream);

/* jt_simulate_image for callers that cannot allocate device memory (code
 * under HIP stream capture, serving loops that must not allocate, harnesses
 * that forbid it).  Same arguments, kernels and results as jt_simulate_image
 * whenever that call convolves directly (bit for bit); this one always
 * convolves directly, so a PSF larger than JT_MAX_PSF is JT_EUNSUPPORTED.
 * It calls no hipMalloc, hipFree or other allocating routine: the packed
 * subhalo table (16 B per NFW subhalo, 80 B per TNFW subhalo, rounded up to
 * a multiple of 4 plus 4 padding records, 256-byte aligned; none with a
 * resident subhalo handle) and the unconvolved image (4 B per pixel, 256-byte
 * aligned; none without a PSF) live in one static device array of
 * JT_NOALLOC_SCRATCH_BYTES per device, looked up by jt_create.  A call needing
 * more than that returns JT_EUNSUPPORTED and launches nothing (e.g. a
 * 1000 x 1000 image with 50 000 NFW subhalos needs 4.8 MB and fits).
 * Every call on a device shares its array: calls that overlap on one device
 * (different streams, or threads without ordering between them) race and
 * corrupt each other's results; calls on one stream are safe. */
jt_status jt_simulate_image_noalloc(jt_ctx* ctx, const jt_grid* grid, const jt_lens* lens,
                                    const jt_light* src, const jt_light* lens_light,
                                    const float* psf, int k, float* out, hipStream_t stream);

/* ----------------------------------------------------------------------
 * Batches of parameter draws: forward images, the chi^2 log-likelihood and
 * its gradient.  The paper names automatic differentiation as what makes
 * gradient-based fitting possible (section "Improvements over lenstronomy in
 * lens modelling", L-BFGS); here the gradient is a hand-written adjoint.
 * -------------------------------------------------------------------- */
/* B draws on one grid, each with a main deflector (an SIE, or an EPL when
 * `epl` is given), an external shear, n_sub NFW subhalos (truncated NFWs when
 * `sub_r_trunc` is given) and n_src source + n_ll lens-light Sersic components
 * (b_n from the Capaccioli fit).  Host arrays are read during the call; the
 * subhalo SoA is device float32 [B][n_sub] (draw b at offset b * n_sub). */
typedef struct {
  int B;
  const jt_sie* sie;                /* host [B] (ignored, may be NULL, when epl is given) */
  const jt_shear* shear;            /* host [B] */
  int n_sub;                        /* >= 0 */
  const float *sub_x, *sub_y, *sub_Rs, *sub_alpha_Rs;   /* device [B][n_sub] */
  int n_src, n_ll;                  /* n_src + n_ll <= 3 for jt_chi2_grad */
  const jt_sersic* src;             /* host [B][n_src] */
  const jt_sersic* ll;              /* host [B][n_ll] (NULL when n_ll = 0) */
  const jt_epl* epl;                /* host [B], or NULL: the main deflector is the SIE */
  const float* sub_r_trunc;         /* device [B][n_sub] (each > 0, not validated), or NULL */
} jt_draws;

/* Forward images of every draw: out device float32 [B][ny][nx], not
 * overlapping psf (JT_EINVAL).  psf device [k][k] (odd k) or NULL with k = 0
 * (no convolution). */
jt_status jt_simulate_batch(jt_ctx* ctx, const jt_grid* grid, const jt_draws* draws,
                            const float* psf, int k, float* out, hipStream_t stream);

/* log L_b = -1/2 sum_i w_i (m_b,i - d_i)^2 for every draw.  data, inv_var:
 * device float32 [ny][nx] (inv_var = w = 1/sigma^2).  logL: device double [B]. */
jt_status jt_chi2(jt_ctx* ctx, const jt_grid* grid, const jt_draws* draws, const float* psf, int k,
                  const float* data, const float* inv_var, double* logL, hipStream_t stream);

/* log L and its gradient for every draw, by a hand-written adjoint.  The backward
 * pass recomputes each sub-pixel's traced position from the lens parameters
 * instead of storing it in the forward launch, so its workspace does not
 * grow with the supersampled grid.
 * g_macro: device float32 [B][P], P = 7 + 7 (n_src + n_ll), in the order
 *   (theta_E, q, phi, cx, cy) of the SIE, (gamma1, gamma2), then
 *   (amp, R_sersic, n_sersic, q, phi, cx, cy) per source, then per lens-light
 *   component; with an EPL main deflector P = 8 + 7 (n_src + n_ll) and the
 *   row starts (theta_E, gamma, q, phi, cx, cy) of the EPL (its partials by
 *   forward-mode differentiation of the deflection's series; 0 when
 *   theta_E = 0).
 * g_sub: device float32 [B][n_sub][3] = d log L / d(x, y, alpha_Rs) per
 *   subhalo, NFW or truncated (Rs and r_trunc held fixed; may be NULL when
 *   n_sub = 0).
 * logL: device double [B] (may be NULL).  Deterministic: fixed summation order,
 * so a call repeated gives the same bits.  A draw's gradient depends on the
 * rest of the batch only through the wave split picked from the batch's total
 * sub-pixel count, which regroups the sums (FP32 rounding, ~1e-6 relative).
 * JT_EUNSUPPORTED when n_src + n_ll > 3. */
jt_status jt_chi2_grad(jt_ctx* ctx, const jt_grid* grid, const jt_draws* draws, const float* psf, int k,
                       const float* data, const float* inv_var, double* logL, float* g_macro,
                       float* g_sub, hipStream_t stream);

/* Same results as jt_chi2_grad, bit for bit, but the forward launch keeps
 * every sub-pixel's traced position (8 bytes per sub-pixel per draw of extra
 * workspace, allocated from the context) and the backward pass reads it back
 * instead of summing the subhalos a second time: faster when the subhalo sum
 * dominates and the workspace fits.  Same arguments and errors. */
jt_status jt_chi2_grad_kept(jt_ctx* ctx, const jt_grid* grid, const jt_draws* draws, const float* psf, int k,
                            const float* data, const float* inv_var, double* logL, float* g_macro,
                            float* g_sub, hipStream_t stream);

/* ----------------------------------------------------------------------
 * Linear amplitude solver
 * -------------------------------------------------------------------- */
/* The image is linear in each Sersic component's amplitude (the paper keeps
 * lenstronomy's linear amplitude solver, section "Why JAXtronomy?").  With
 * basis images B_j = PSF * (image of component j alone at unit amplitude),
 * components ordered as src then lens_light (their amp fields are ignored),
 * this solves
 *     a = argmin_a sum_i w_i (d_i - sum_j a_j B_j,i)^2
 * by the normal equations summed in FP64 in a fixed order and a Cholesky
 * factorisation on the device (scaled to unit diagonal).  1 <= n_src + n_ll
 * <= 8.  data d and inv_var w: device float32 [ny][nx].  Outputs (device,
 * written on `stream`): amps double[n_src + n_ll]; model float32 [ny][nx]
 * (may be NULL) = sum_j a_j B_j rounded once; logL double[1] (may be NULL)
 * = -1/2 sum_i w_i (d_i - model_i)^2.  A normal matrix that is not positive
 * definite (a component that adds nothing to the image, or two that
 * coincide) gives NaN amplitudes (and a NaN model and logL).  Grid, lens and
 * psf/k as in jt_simulate_image. */
jt_status jt_linear_amplitudes(jt_ctx* ctx, const jt_grid* grid, const jt_lens* lens, const jt_light* src,
                               const jt_light* lens_light, const float* psf, int k, const float* data,
                               const float* inv_var, double* amps, float* model, double* logL,
                               hipStream_t stream);

/* ----------------------------------------------------------------------
 * Fitting loops (section "Improvements over lenstronomy in lens modelling":
 * the particle swarm kept from lenstronomy, and L-BFGS on gradients)
 * -------------------------------------------------------------------- */
/* The parameter vector is a jt_draws macro row: (theta_E, q, phi, cx, cy) of
 * the SIE, (gamma1, gamma2), then (amp, R_sersic, n_sersic, q, phi, cx, cy)
 * per source and per lens-light component; P = 7 + 7 (n_src + n_ll).  Every
 * evaluation shares the fixed subhalos, the PSF and the data. */
typedef struct {
  int n_src, n_ll;                  /* n_src + n_ll >= 1 (<= 3 for jt_lbfgs) */
  const double *lower, *upper;      /* host [P]: the search box, inside each parameter's domain */
  int n_sub;                        /* fixed NFW subhalos, device float32 [n_sub] each */
  const float *sub_x, *sub_y, *sub_Rs, *sub_alpha_Rs;
  const float* psf;                 /* device [k][k] (odd k), or NULL with k = 0 */
  int k;
  const float *data, *inv_var;      /* device float32 [ny][nx] */
} jt_fit_problem;

/* Particle swarm (Kennedy & Eberhart 1995, inertia weight of Shi & Eberhart
 * 1998) maximising log L: starts uniform in the box (v = 0), then
 * v <- w v + c1 r0 (pbest - x) + c2 r1 (gbest - x), x <- x + v, a coordinate
 * leaving the box is set on it with zero velocity.  Random numbers r are
 * jt_uniform(seed, i) at fixed counters (jt_pso_move), so a run is
 * reproducible.  Each step's N particles are one batched jt_chi2 launch. */
typedef struct {
  int n_particles, n_iterations;    /* >= 1, >= 0 */
  double inertia, c_cognitive, c_social;   /* w, c1, c2 (e.g. 0.7298, 1.49618, 1.49618) */
  uint64_t seed;
} jt_pso_cfg;
/* Host outputs: best [P], best_logL, history [n_iterations] (swarm best after
 * each step; may be NULL).  Synchronises `stream` once per step. */
jt_status jt_pso(jt_ctx* ctx, const jt_grid* grid, const jt_fit_problem* prob, const jt_pso_cfg* cfg,
                 double* best, double* best_logL, double* history, hipStream_t stream);
/* The update jt_pso applies at step t >= 1 to the host arrays x, v [N][P]
 * (pbest [N][P], gbest [P]), with r0, r1 = jt_uniform(seed, 2 ((t N + p) P + d) + 0, 1). */
jt_status jt_pso_move(int N, int P, int t, uint64_t seed, double w, double c1, double c2, const double* lower,
                      const double* upper, double* x, double* v, const double* pbest, const double* gbest);
/* Counter-based uniform in [0, 1): the (i+1)-th output of SplitMix64 (Steele,
 * Lea & Flood 2014) seeded with `seed`, shifted right by 11, times 2^-53. */
double jt_uniform(uint64_t seed, uint64_t i);

/* L-BFGS (Nocedal 1980; Liu & Nocedal 1989) minimising -log L from `starts`
 * points at once.  A coordinate on a bound whose gradient points out of the
 * box (so every coordinate with lower = upper) is held; on the free ones the
 * direction is the two-loop recursion over the last `memory` pairs with
 * H0 = (s.y / y.y) I (unit steepest descent without pairs or when the
 * direction does not descend); steps from 1, halved until the box-projected
 * trial satisfies the Armijo condition with constant 1e-4 (41 trials, then
 * the chain stops); stops after max_iter accepted steps, a relative change
 * of -log L at most ftol, or a projected gradient at most gtol.  The trial
 * points of all running chains are one batched jt_chi2_grad launch per round.
 * x0, x: host [starts][P]; logL host [starts]; iterations host [starts] (may
 * be NULL).  The gradient is the FP32 adjoint's, so chains stop once its
 * round-off hides further descent. */
typedef struct {
  int starts, memory, max_iter;     /* >= 1, >= 1, >= 0 */
  double ftol, gtol;
} jt_lbfgs_cfg;
jt_status jt_lbfgs(jt_ctx* ctx, const jt_grid* grid, const jt_fit_problem* prob, const jt_lbfgs_cfg* cfg,
                   const double* x0, double* x, double* logL, int* iterations, hipStream_t stream);

/* ----------------------------------------------------------------------
 * Resident tables
 * -------------------------------------------------------------------- */
/* Copy n subhalos (host float32 SoA) into a device-resident, pre-derived
 * table owned by ctx (n = 0 allowed).  *handle != 0 on success. */
jt_status jt_upload_subhalos(jt_ctx* ctx, int n, const float* x, const float* y,
                             const float* Rs, const float* alpha_Rs, uint64_t* handle);
/* The same for truncated subhalos (r_trunc, host float32[n], each > 0; see
 * jt_nfw).  Every call that takes a subhalo handle takes such tables too;
 * the continuous-batching server keeps each launch to one profile (a TNFW
 * request and an NFW one never share a batch). */
jt_status jt_upload_tnfw(jt_ctx* ctx, int n, const float* x, const float* y, const float* Rs,
                         const float* alpha_Rs, const float* r_trunc, uint64_t* handle);
/* Copy a host float32 [k][k] PSF (odd k) into device memory owned by ctx. */
jt_status jt_upload_psf(jt_ctx* ctx, const float* psf, int k, uint64_t* handle);
/* Device pointer of a resident PSF (valid until released). */
jt_status jt_psf_pointer(jt_ctx* ctx, uint64_t handle, const float** dev_psf, int* k);
/* Release a handle (waits for the device). JT_EINVAL if unknown. */
jt_status jt_release(jt_ctx* ctx, uint64_t handle);

/* ----------------------------------------------------------------------
 * Serving: continuous batching of heterogeneous simulation requests.
 * The paper notes that the pipeline's run time varies strongly with the
 * deflector and light models, the grid and the PSF size (image-simulation
 * section), and that per-call overhead can dominate simple profiles; the
 * server therefore packs whatever requests are waiting into one launch of the
 * fused kernel over a (request, pixel block) tile list, keeps subhalo tables
 * and PSFs resident, admits requests by device-memory footprint, and keeps
 * several batches in flight on separate streams.
 * -------------------------------------------------------------------- */
typedef struct jt_server jt_server;

typedef struct {
  size_t hbm_budget_bytes;   /* device arena for in-flight request buffers (> 0) */
  int max_batch_images;      /* requests per batch (>= 1) */
  double max_batch_pairs;    /* work cap per batch in (sub-pixel, subhalo) pairs (> 0;
                                a truncated-NFW pair counts as 1.55, its measured cost);
                                a larger request runs in chunks of its pixel blocks of
                                at most this much work, one such request at a time,
                                while later requests are batched beside it */
  int max_inflight_batches;  /* batches on the device at once (>= 1) */
  int n_streams;             /* streams the batches rotate over (>= 1) */
} jt_server_cfg;

/* One image to simulate.  Lens and light parameters are copied at submit;
 * the resident subhalo table and PSF must outlive the ticket. */
typedef struct {
  jt_grid grid;
  int has_sie, has_shear;
  jt_sie sie;
  jt_shear shear;
  uint64_t subhalo_handle;   /* from jt_upload_subhalos or jt_upload_tnfw; 0 = none */
  jt_light src, lens_light;  /* host arrays, read during jt_server_submit */
  uint64_t psf_handle;       /* from jt_upload_psf; 0 = no convolution */
  float* out;                /* device float32 [ny][nx], written when the ticket completes */
  int has_epl;               /* EPL main deflector, as in jt_lens */
  jt_epl epl;
} jt_request;

typedef enum { JT_TICKET_QUEUED = 0, JT_TICKET_RUNNING = 1, JT_TICKET_DONE = 2, JT_TICKET_CANCELLED = 3,
               JT_TICKET_FAILED = 4 } jt_ticket_state;

typedef struct {
  uint64_t submitted, completed, cancelled, failed, batches;
  uint64_t arena_bytes, arena_in_use, arena_peak;
  double device_seconds;     /* simulated executor: modelled device time */
  double wait_seconds;       /* sum over finished requests of submission -> launch */
  double run_seconds;        /* sum over finished requests of launch -> completion */
  double max_wait_seconds;   /* longest submission -> launch */
} jt_server_stats;

/* Server on the device of ctx; starts its scheduling thread. */
jt_status jt_server_create(jt_ctx* ctx, const jt_server_cfg* cfg, jt_server** out);
/* Server with a simulated device (no GPU): a batch "runs" for
 * (sum of its pairs) / pairs_per_second seconds.  Requests then read
 * subhalo_handle as the subhalo count and psf_handle as the PSF side; `out` is
 * never touched.  For tests of the scheduler. */
jt_status jt_server_create_simulated(const jt_server_cfg* cfg, double pairs_per_second, jt_server** out);
/* Simulated server only (JT_EINVAL otherwise): the batch launched as number
 * `batch` (1-based count of launches; 0 = none) fails when it completes, as
 * a device error would.  For tests of the failure path. */
jt_status jt_server_simulate_failure(jt_server* srv, uint64_t batch);
/* Queue a request: JT_EINVAL (bad request), JT_ENOMEM (can never fit the
 * arena), JT_EDEVICE (the server has seen a device failure), JT_OK (*ticket
 * set).  A batch that fails on the device fails every ticket in flight and
 * queued (JT_TICKET_FAILED), and the server refuses all later submissions:
 * create a new one (on a fresh context if the device itself failed). */
jt_status jt_server_submit(jt_server* srv, const jt_request* req, uint64_t* ticket);
/* Current state (jt_ticket_state) of a ticket. */
jt_status jt_server_poll(jt_server* srv, uint64_t ticket, int* state);
/* Wait until the ticket leaves the queue and the device (timeout_s < 0: no
 * limit).  JT_OK when done (latency_s = completion - submission, may be NULL),
 * JT_ECANCELLED, JT_EDEVICE (failed), JT_EBUSY (timed out).  Once it has
 * returned a final state the ticket is forgotten (later calls: JT_EINVAL). */
jt_status jt_server_wait(jt_server* srv, uint64_t ticket, double timeout_s, double* latency_s);
/* Cancel a queued ticket (JT_EBUSY once it runs). */
jt_status jt_server_cancel(jt_server* srv, uint64_t ticket);
jt_status jt_server_get_stats(jt_server* srv, jt_server_stats* stats);
/* Stop scheduling, cancel queued tickets, wait for running batches, free.
 * A chunked request in progress launches no further chunk and ends
 * CANCELLED once its launched chunks have finished (a request whose
 * convolution is already running completes normally).  Threads already in
 * jt_server_wait return (every ticket reaches a final state) before the
 * server is freed; no call on the server may start once this has begun. */
void jt_server_destroy(jt_server* srv);

/* ----------------------------------------------------------------------
 * Kernel timing (HIP events recorded on the launch stream)
 * -------------------------------------------------------------------- */
typedef enum {
  JT_K_PREP = 0,        /* subhalo table derivation */
  JT_K_RAY = 1,         /* ray shooting (jt_ray_shoot / jt_deflection) */
  JT_K_SB = 2,          /* surface brightness */
  JT_K_SIM = 3,         /* fused simulate kernel */
  JT_K_CONV = 4,        /* convolution */
  JT_K_GRAD = 5,        /* adjoint: residual, per-sub-pixel and subhalo passes */
  JT_K_COUNT = 6
} jt_kernel_id;
/* Measurement: FP32 issue-rate calibration (not part of the simulation).
 * Launches `blocks` blocks of 256 threads; every lane runs `iters` rounds over
 * eight independent FP32 chains of one instruction class:
 *   kind 0: 8 FMA per round (register operands)   kind 3: 16 multiplies
 *   kind 1: 8 v_rsq_f32                           kind 4: 8 FMA with a literal
 *   kind 2: 16 FMA + 2 v_rsq_f32                  kind 5: 8 v_log_f32 + 8 adds
 *   kind 6: 8 accumulating FMA, SGPR operand       kind 7: 8 FMA on three VGPRs
 * out: device float32[blocks * 256] (chain sums, written so nothing is
 * optimised away).  Timing is the caller's (events on `stream`), so that the
 * rates the roofline figures use are measured by committed code.
 * JT_EINVAL for a kind outside 0..7 or non-positive sizes. */
jt_status jt_calibrate_valu(int kind, int blocks, int iters, float* out, hipStream_t stream);

/* Enable (1) or disable (0) event timing of every launch; resets the totals. */
jt_status jt_profile_enable(jt_ctx* ctx, int on);
/* Total milliseconds and launch count of kernel `id` since enabling (waits for
 * the recorded events). */
jt_status jt_profile_read(jt_ctx* ctx, int id, double* total_ms, int* launches);

#ifdef __cplusplus
}
#endif
#endif /* JT_H */
