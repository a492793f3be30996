// Host-callable launchers of the HIP kernels (internal to libjt).
#pragma once

#include <hip/hip_runtime.h>

#include "jt_device.hpp"

namespace jt {

// Records of a packed subhalo table for n subhalos: n rounded up to a multiple
// of 4, plus 4 records that the prefetch of the last group reads.  Records past
// n are padding {1e18, 1e18, 1, 0}: far field with c2 = 0, an exact zero term.
inline int subhalo_loop_count(int n) { return (n + 3) & ~3; }
inline int subhalo_table_records(int n) { return subhalo_loop_count(n) + 4; }

// Writes all subhalo_table_records(n) records (padding included).
hipError_t launch_prep_subhalos(int n, const float* x, const float* y, const float* rs,
                                const float* ars, SubRec* out, hipStream_t st);
// The same for truncated subhalos (TRec records; padding has c2 = 0).
hipError_t launch_prep_tnfw(int n, const float* x, const float* y, const float* rs, const float* ars,
                            const float* rt, TRec* out, hipStream_t st);
// `sub` holds SubRec records, or TRec records when tnfw is set.
hipError_t launch_ray_shoot(bool alpha, bool tnfw, int n, const float* x, const float* y, const MacroC& mc,
                            const void* sub, int nloop, float* ox, float* oy, hipStream_t st);
hipError_t launch_source_sb(int n, const float* x, const float* y, const float* bx, const float* by,
                            const LightC& src, const LightC& ll, float* sb, hipStream_t st);
// g.ppb is set by the launcher from the chosen split.
hipError_t launch_simulate(GridC g, const MacroC& mc, bool tnfw, const void* sub, int nloop, const LightC& src,
                           const LightC& ll, float* img, hipStream_t st);
// Unit-amplitude image of every light component (sources, then lens light)
// into basis [src.n + ll.n][ny][nx]; src.n + ll.n <= kMaxBasis.
hipError_t launch_simulate_basis(GridC g, const MacroC& mc, bool tnfw, const void* sub, int nloop,
                                 const LightC& src, const LightC& ll, float* basis, hipStream_t st);
// Linear amplitude solver over n <= kMaxBasis basis images of npix pixels:
// FP64 normal-equation partials of kLinBlocks blocks (kLinTerms each), the
// Cholesky solve on the device (NaN amplitudes when the matrix is not
// positive definite), then the model and the log-likelihood.
constexpr int kLinTerms = kMaxBasis * (kMaxBasis + 1) / 2 + kMaxBasis;
constexpr int kLinBlocks = 256;
hipError_t launch_linear_solve(int npix, int n, const float* basis, const float* data, const float* w,
                               double* part, double* amps, float* model, double* logL, hipStream_t st);
// Wave-groups per block for `points` sub-pixels in whole units of `unit`.
int pick_split(long points, int unit, int nloop);
// Direct convolution on the matrix cores (k_conv_mfma).  The launch shape of
// an nx x ny image with a k x k kernel: column groups of 16 outputs per block
// (nc), waves splitting each column group's input rows (s) and input rows per
// LDS-staged chunk (t).  It depends on (nx, ny, k) alone and fixes the order
// of every sum, so an image convolved alone, in a batch of draws or in a
// served batch gives the same bits.
struct ConvShape {
  int nc, s, t;
};
ConvShape conv_shape(int nx, int ny, int k);
int conv_shape_kind(const ConvShape& sh);      // 0: (4, 1), 1: (2, 2), 2: (1, 8)
size_t conv_lds_bytes(int k, const ConvShape& sh);
int conv_tiles_x(int nx, const ConvShape& sh);  // 16 nc output columns per tile
int conv_tiles_y(int ny);                       // 16 output rows per tile
// `batch` images at img + z * in_stride -> out + z * out_stride; flip = the
// adjoint (correlation with the kernel).
hipError_t launch_conv_direct_batched(bool flip, int batch, const float* img, long in_stride, int nx, int ny,
                                      const float* psf, int k, float* out, long out_stride, hipStream_t st);
// Heterogeneous convolutions of one shape kind: tiles (desc, tile_x, tile_y,
// -), each descriptor with its own k and rows per chunk; `lds` bytes cover the
// largest conv_lds_bytes of the launch's descriptors.
hipError_t launch_conv_desc(int kind, const ConvDesc* descs, const int4* tiles, int ntiles, size_t lds,
                            hipStream_t st);
// Batched fused simulation over image descriptors (see k_simulate_desc).
// tnfw: every descriptor's table holds TRec records (not with keep_beta).
hipError_t launch_simulate_desc(int split, bool tnfw, bool extra, bool keep_beta, const ImageDesc* descs,
                                const int2* tiles, int nblocks, int blocks_per_image, hipStream_t st);
// Per-draw subhalo tables from [B][n] SoA into B tables of
// subhalo_table_records(n) records.
hipError_t launch_prep_subhalos_batched(int B, int n, const float* x, const float* y, const float* rs,
                                        const float* ars, SubRec* out, hipStream_t st);
// Truncated tables of B draws, out [B][subhalo_table_records(n)]; unit: every
// record built for alpha_Rs = 1 (the adjoint's per-lane constants).
hipError_t launch_prep_tnfw_batched(int B, int n, const float* x, const float* y, const float* rs, const float* ars,
                                    const float* rt, bool unit, TRec* out, hipStream_t st);

// ---- FFT convolution (fft.hip) ----
// Cost model of the direct/FFT choice (method 0), fitted to kernel times on
// MI355X (images 100^2..1000^2, k = 21..101):
//   direct: kConvDirectFixedS + E / min(kConvMfmaMacPerS, waves * kConvMfmaMacPerWaveS),
//           E = nx ny (16 + k - 1) kp multiply-adds issued (the banded operand's
//           zeros included), waves = tiles * nc * s of conv_shape
//   FFT:    kConvFftFixedS + Nx Ny / kConvFftPointsPerS (padded 2-3-5 sizes)
constexpr double kConvDirectFixedS = 6e-6;
constexpr double kConvMfmaMacPerS = 4.9e13;
constexpr double kConvMfmaMacPerWaveS = 1.35e10;
constexpr double kConvFftFixedS = 30e-6;
constexpr double kConvFftPointsPerS = 1.45e10;
bool conv_prefers_fft(int nx, int ny, int k);
constexpr int kFftMinN = 16, kFftMaxN = 2048;
// Padded FFT length (the smallest 2^a 3^b 5^c that avoids wrap-around) for an
// image side n and kernel side k.
int fft_size_for(int n, int k);
size_t fft_workspace_bytes(int nx, int ny, int k);
// tw_x, tw_y: tables exp(-2 pi i t / N), t < N, for N = fft_size_for(nx, k)
// and fft_size_for(ny, k); ws: fft_workspace_bytes.
hipError_t launch_fft_convolve(const float* img, int nx, int ny, const float* psf, int k, float* out, void* ws,
                               const double2* tw_x, const double2* tw_y, hipStream_t st);

// ---- adjoint (adjoint.hip) ----
constexpr int kRecPartsHost = 4;  // parts of the adjoint's subhalo-major pass
// The truncated profile's far pass takes 16 parts, and its near pass adds one
// more (part 16 of gpart).
constexpr int kRecPartsTnfwHost = 16;
hipError_t launch_residual(int B, int npix, const float* model, const float* data, const float* w, float* resid,
                           float* part, int* nblocks, hipStream_t st);
// tnfw: the draws' subhalos are truncated (the recomputed deflection uses the
// TNFW tables); epl: their main deflector is an EPL (macro row [EPL 6, shear 2,
// Sersic ...]).
hipError_t launch_grad_pixel(int split, bool kept, bool tnfw, bool epl, int B, int bpi, const ImageDesc* descs,
                             const float* lamU, float4* rec, int rec_stride, float* part, int P, hipStream_t st);
// Subhalo-major pass for truncated subhalos: far pairs in kRecPartsTnfwHost
// parts, then the near pairs (the general form, a wave per subhalo and draw
// over its box of the grid g) as one more part; gpart holds
// kRecPartsTnfwHost + 1 parts.  utab [B][records]: each draw's table built for
// alpha_Rs = 1 (launch_prep_tnfw_batched with unit set).
hipError_t launch_grad_subhalo_tnfw(int B, int n, const TRec* utab, int records, const float* ars,
                                    const float4* rec, int rec_stride, int nrec_loop, const GridC& g, float* gpart,
                                    hipStream_t st);
// draws' subhalo SoA x, y, rs, ars: device [B][n]
hipError_t launch_grad_subhalo(int B, int n, const float* x, const float* y, const float* rs, const float* ars,
                               const float4* rec, int rec_stride, int nrec_loop, float* gpart, hipStream_t st);
hipError_t launch_grad_finalize(int B, int P, int bpi, const float* part, float* g_macro, int nres,
                                const float* lpart, double* logL, int n, int parts, const float* gpart, float* g_sub,
                                hipStream_t st);
int grad_max_params();
hipError_t launch_conv_direct(const float* img, int nx, int ny, const float* psf, int k, float* out,
                              hipStream_t st);

}  // namespace jt
