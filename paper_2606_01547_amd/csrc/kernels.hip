// HIP kernels of the lensed-image simulation for gfx950.
//
//  k_prep_subhalos  device SoA (x, y, Rs, alpha_Rs) -> packed SubRec table
//  k_prep_tnfw      device SoA (x, y, Rs, alpha_Rs, r_trunc) -> packed TRec table
//  k_ray_shoot      step 1 at explicit points: beta = theta - alpha (or alpha)
//  k_source_sb      step 2 at explicit points
//  k_simulate       steps 1-2 plus the supersample average, fused
//  k_conv_mfma      step 3, direct convolution on the matrix cores
//
// Subhalo records are read with wave-uniform indices from a read-only table, so
// the 16-byte NFW records arrive through scalar loads into SGPRs and feed the
// VALU as scalar operands (they enter only subtractions and multiplies, which
// issue at full rate with one); the 80-byte truncated-NFW records, whose
// polynomial coefficients are FMA operands, are staged through LDS per wave
// instead.  Every lane runs the same subhalo at its own sub-pixel.  The
// per-sub-pixel subhalo sum is formed tile by tile: a tile of kSubTile pairs is
// summed in plain FP32 and the tile partial enters a TwoSum-compensated
// accumulator.  The summation order is fixed, so results are bitwise
// reproducible and independent of launch batching.
#include "jt_device.hpp"
#include "jt_kernels.hpp"
#include "jt_sum.hpp"

namespace jt {

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prep_subhalos(int n, int padded, const float* __restrict__ x,
                                                      const float* __restrict__ y,
                                                      const float* __restrict__ rs,
                                                      const float* __restrict__ ars,
                                                      SubRec* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) {
    if (i < padded) out[i] = kSubRecPad;
    return;
  }
  out[i] = make_subrec(x[i], y[i], rs[i], ars[i]);
}

__global__ __launch_bounds__(256) void k_prep_tnfw(int n, int padded, const float* __restrict__ x,
                                                  const float* __restrict__ y, const float* __restrict__ rs,
                                                  const float* __restrict__ ars, const float* __restrict__ rt,
                                                  TRec* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) {
    if (i < padded) out[i] = trec_pad();
    return;
  }
  out[i] = make_trec(x[i], y[i], rs[i], ars[i], rt[i]);
}

// ---------------------------------------------------------------------------
// Step 1 at explicit points.  Block = kSplit wave-groups x split_lanes(kSplit)
// points; all groups see the same points.
template <bool kAlpha, int kSplit, class P>
__global__ __launch_bounds__(split_threads(kSplit)) void k_ray_shoot(int n, const float* __restrict__ x,
                                                                    const float* __restrict__ y, MacroC mc,
                                                                    const void* __restrict__ sub, int nloop,
                                                                    float* __restrict__ ox, float* __restrict__ oy) {
  __shared__ RangeScratch<kSplit> scratch;
  constexpr int kW = split_lanes(kSplit);
  // kW is a multiple of the wave size, so the group index is wave-uniform;
  // readfirstlane lets the compiler keep the subhalo loop on scalar loads.
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x / kW);
  const int slot = threadIdx.x - g * kW;
  const int i = blockIdx.x * kW + slot;
  const bool valid = i < n;
  const float tx = valid ? x[i] : 0.f;
  const float ty = valid ? y[i] : 0.f;
  double sx = 0.0, sy = 0.0;
  subhalo_ranges<kSplit, P>(tx, ty, sub, nloop, g, slot, scratch, sx, sy);
  __syncthreads();
  if (g == 0 && valid) {
    double ax, ay;
    total_deflection64<kSplit>(mc, tx, ty, scratch, slot, sx, sy, ax, ay);
    ox[i] = (float)(kAlpha ? ax : (double)tx - ax);
    oy[i] = (float)(kAlpha ? ay : (double)ty - ay);
  }
}

// Step 2 at explicit points: sb = sources at beta + lens light at theta.  A
// list without components reads none of its coordinates.  With kVec every
// thread below n/4 takes four consecutive points through 16-byte loads and
// stores (all arrays 16-byte aligned), and the last n mod 4 points take one
// thread each; otherwise one point per thread.
template <bool kExtra>
__device__ __forceinline__ float sb_at(const LightC& src, const LightC& ll, bool hs, bool hl, const float* x,
                                       const float* y, const float* bx, const float* by, int i) {
  float v = hs ? light_sum<kExtra>(src, bx[i], by[i]) : 0.f;
  if (hl) v += light_sum<kExtra>(ll, x[i], y[i]);
  return v;
}

template <bool kExtra, bool kVec>
__global__ __launch_bounds__(256) void k_source_sb(int n, const float* __restrict__ x,
                                                  const float* __restrict__ y,
                                                  const float* __restrict__ bx,
                                                  const float* __restrict__ by, LightC src,
                                                  LightC ll, float* __restrict__ sb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool hs = light_any(src), hl = light_any(ll);
  if (!kVec) {
    if (i < n) sb[i] = sb_at<kExtra>(src, ll, hs, hl, x, y, bx, by, i);
    return;
  }
  const int n4 = n >> 2;
  if (i >= n4) {
    const int j = 4 * n4 + (i - n4);
    if (j < n) sb[j] = sb_at<kExtra>(src, ll, hs, hl, x, y, bx, by, j);
    return;
  }
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (hs) {
    const float4 u = reinterpret_cast<const float4*>(bx)[i], w = reinterpret_cast<const float4*>(by)[i];
    v.x = light_sum<kExtra>(src, u.x, w.x);
    v.y = light_sum<kExtra>(src, u.y, w.y);
    v.z = light_sum<kExtra>(src, u.z, w.z);
    v.w = light_sum<kExtra>(src, u.w, w.w);
  }
  if (hl) {
    const float4 u = reinterpret_cast<const float4*>(x)[i], w = reinterpret_cast<const float4*>(y)[i];
    v.x += light_sum<kExtra>(ll, u.x, w.x);
    v.y += light_sum<kExtra>(ll, u.y, w.y);
    v.z += light_sum<kExtra>(ll, u.z, w.z);
    v.w += light_sum<kExtra>(ll, u.w, w.w);
  }
  reinterpret_cast<float4*>(sb)[i] = v;
}

// Sub-pixel slot of a simulate block: slot t of wave-group 0..kSplit-1 holds
// sub-pixel (t mod s^2) of local pixel (t / s^2) of the block's g.ppb pixels.
struct SubPixel {
  int pixel;             // global pixel index (0 when invalid)
  int sub;               // sub-pixel index in the pixel, a * s + b
  bool valid;
  double dx, dy;         // sub-pixel centre (FP64)
  float tx, ty;          // its correctly rounded FP32 value (pair loop, lens light)
};

__device__ __forceinline__ SubPixel subpixel_of(const GridC& g, int block, int t) {
  SubPixel sp;
  const int lp = t / g.s2;
  const int si = t - lp * g.s2;
  const int npix = g.nx * g.ny;
  const int p = block * g.ppb + lp;
  sp.valid = (lp < g.ppb) && (p < npix);
  sp.pixel = sp.valid ? p : 0;
  sp.sub = si;
  const int row = sp.pixel / g.nx;
  const int col = sp.pixel - row * g.nx;
  const int a = si / g.s;
  const int b = si - a * g.s;
  sp.dx = g.ox + g.step * ((double)(col * g.s + b) + 0.5);
  sp.dy = g.oy + g.step * ((double)(row * g.s + a) + 0.5);
  sp.tx = (float)sp.dx;
  sp.ty = (float)sp.dy;
  return sp;
}

// Steps 1-2 and the supersample average for pixel block `block` of one
// image.  The kSplit wave-groups share the subhalo quarters of the same
// slots; group 0 combines them, evaluates the light, and the pixel values are
// reduced through LDS in a fixed order.
template <int kSplit, class P = NfwPairs, bool kExtra = false, bool kKeepBeta = false>
__device__ __forceinline__ void simulate_block(const GridC& g, const MacroC& mc, const void* __restrict__ sub,
                                               int nloop, const LightC& src, const LightC& ll,
                                               float* __restrict__ img, int block,
                                               RangeScratch<kSplit>& scratch, float* red,
                                               float2* __restrict__ beta = nullptr) {
  constexpr int kW = split_lanes(kSplit);
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / kW);  // wave-uniform (kW % 64 == 0)
  const int t = threadIdx.x - grp * kW;
  const SubPixel sp = subpixel_of(g, block, t);
  double sx = 0.0, sy = 0.0;
  subhalo_ranges<kSplit, P>(sp.tx, sp.ty, sub, nloop, grp, t, scratch, sx, sy);
  __syncthreads();
  if (grp == 0) {
    double ax, ay;
    total_deflection64<kSplit>(mc, sp.dx, sp.dy, scratch, t, sx, sy, ax, ay);
    const float bx = (float)(sp.dx - ax), by = (float)(sp.dy - ay);
    // the traced position, kept for the adjoint: [pixel][sub-pixel]
    if (kKeepBeta && sp.valid) beta[(long)sp.pixel * g.s2 + sp.sub] = make_float2(bx, by);
    float v = light_sum<kExtra>(src, bx, by);
    if (light_any(ll)) v += light_sum<kExtra>(ll, sp.tx, sp.ty);
    red[t] = v;
  }
  __syncthreads();
  if (threadIdx.x < g.ppb) {
    const int q = block * g.ppb + threadIdx.x;
    if (q < g.nx * g.ny) {
      float acc = 0.f;
      const float* r = red + threadIdx.x * g.s2;
      for (int k = 0; k < g.s2; ++k) acc += r[k];
      img[q] = acc * g.area_over_s2;
    }
  }
}

template <int kSplit, class P, bool kExtra>
__global__ __launch_bounds__(split_threads(kSplit)) void k_simulate(GridC g, MacroC mc, const void* __restrict__ sub,
                                                                   int nloop, LightC src, LightC ll,
                                                                   float* __restrict__ img) {
  __shared__ RangeScratch<kSplit> scratch;
  __shared__ float red[split_lanes(kSplit)];
  simulate_block<kSplit, P, kExtra>(g, mc, sub, nloop, src, ll, img, blockIdx.x, scratch, red);
}

// Basis images of the linear amplitude solver: the deflection of each
// sub-pixel once, then every light component at unit amplitude (sources at
// beta, lens light at theta, sources first), each averaged over its pixel in
// the same order as k_simulate.  basis: [src.n + ll.n][ny][nx].
template <int kSplit, class P>
__global__ __launch_bounds__(split_threads(kSplit)) void k_simulate_basis(GridC g, MacroC mc,
                                                                         const void* __restrict__ sub, int nloop,
                                                                         LightC src, LightC ll,
                                                                         float* __restrict__ basis) {
  __shared__ RangeScratch<kSplit> scratch;
  __shared__ float red[kMaxBasis][split_lanes(kSplit)];
  constexpr int kW = split_lanes(kSplit);
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / kW);
  const int t = threadIdx.x - grp * kW;
  const SubPixel sp = subpixel_of(g, blockIdx.x, t);
  double sx = 0.0, sy = 0.0;
  subhalo_ranges<kSplit, P>(sp.tx, sp.ty, sub, nloop, grp, t, scratch, sx, sy);
  __syncthreads();
  if (grp == 0) {
    double ax, ay;
    total_deflection64<kSplit>(mc, sp.dx, sp.dy, scratch, t, sx, sy, ax, ay);
    const float bx = (float)(sp.dx - ax), by = (float)(sp.dy - ay);
    for (int j = 0; j < src.n; ++j) red[j][t] = sersic_unit(src.c[j], bx, by);
    for (int j = 0; j < ll.n; ++j) red[src.n + j][t] = sersic_unit(ll.c[j], sp.tx, sp.ty);
  }
  __syncthreads();
  const int n = src.n + ll.n;
  const long npix = (long)g.nx * g.ny;
  for (int idx = threadIdx.x; idx < g.ppb * n; idx += blockDim.x) {
    const int j = idx / g.ppb;
    const int lp = idx - j * g.ppb;
    const long q = (long)blockIdx.x * g.ppb + lp;
    if (q < npix) {
      float acc = 0.f;
      const float* r = red[j] + lp * g.s2;
      for (int k = 0; k < g.s2; ++k) acc += r[k];
      basis[j * npix + q] = acc * g.area_over_s2;
    }
  }
}

// Batched images: block b works on image descs[b / blocks_per_image] when
// every image has the same grid (tiles == nullptr), otherwise on the
// (image, pixel block) pair tiles[b].
template <int kSplit, class P, bool kExtra, bool kKeepBeta>
__global__ __launch_bounds__(split_threads(kSplit)) void k_simulate_desc(const ImageDesc* __restrict__ descs,
                                                                        const int2* __restrict__ tiles,
                                                                        int blocks_per_image) {
  __shared__ RangeScratch<kSplit> scratch;
  __shared__ float red[split_lanes(kSplit)];
  int di, blk;
  if (tiles) {
    const int2 tl = tiles[blockIdx.x];
    di = tl.x;
    blk = tl.y;
  } else {
    di = blockIdx.x / blocks_per_image;
    blk = blockIdx.x - di * blocks_per_image;
  }
  const ImageDesc& d = descs[di];
  simulate_block<kSplit, P, kExtra, kKeepBeta>(d.g, d.mc, d.sub, d.nloop, d.src, d.ll, d.img, blk, scratch, red,
                                               d.beta);
}

// ---------------------------------------------------------------------------
// Direct convolution on the matrix cores.  The "same" convolution is a dense
// contraction: for a 16-row output block, out[i][j] = sum over input rows t
// and taps b of K[i + 2c - t][b] X[t][j - b + c] (rows t of the block's input
// window, K zero outside its k x k support), i.e. C = A B with A[i][(t, b)] =
// K[i + 2c - t][b] (a banded Toeplitz matrix of the kernel) and B[(t, b)][j] =
// X[t][j - b + c] (a Hankel matrix of the image rows).  Each wave forms a
// 16 x 16 output tile with v_mfma_f32_16x16x4f32 (FP32 products and sums),
// four taps per instruction, both operands read from LDS: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds C[4 (l / 16) + v][l % 16].
// A block of NC x S waves covers 16 rows x 16 NC columns; the S waves of a
// column group split the input rows of each staged chunk and their partial
// tiles are added in wave order, so that small images still give the chip
// enough waves.  The input window is staged T rows at a time (T from the LDS
// budget) with the kernel rows those rows meet; the order of every sum is
// fixed by (k, NC, S, T), which depend on the image size and k only, so
// results are reproducible and independent of batching.
typedef float jt_floatx4 __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int conv_mfma_kp(int k) { return (k + 3) & ~3; }

// The launch shape of an nx x ny image with a k x k kernel: 16 x 64 tiles
// (4 waves, one per column group) when they alone give at least 512 blocks,
// else 16 x 32 tiles with 2 waves per column group, else 16 x 16 tiles with 8
// waves splitting the rows; it depends on (nx, ny, k) alone.
ConvShape conv_shape(int nx, int ny, int k) {
  ConvShape sh;
  const long ty = (ny + 15) / 16;
  if ((long)((nx + 63) / 64) * ty >= 512) {
    sh.nc = 4;
    sh.s = 1;
  } else if ((long)((nx + 31) / 32) * ty >= 512) {
    sh.nc = 2;
    sh.s = 2;
  } else {
    sh.nc = 1;
    sh.s = 8;
  }
  // rows per chunk: all 16 + k - 1 window rows if they fit the LDS budget
  // (32 KB for the 4-wave large-image blocks, so that several stay resident;
  // 64 KB otherwise), never fewer than 8
  const int kp = conv_mfma_kp(k), xw = 16 * sh.nc + kp - 1, kw = kp + 1;
  const long budget = (sh.nc == 4 ? 32768 : 65536) / (long)sizeof(float) - (sh.s > 1 ? 256L * sh.nc * sh.s : 0);
  long t = (budget - 15L * kw) / (xw + kw);
  const int nrows = 16 + k - 1;
  if (t > nrows) t = nrows;
  if (t < 8) t = 8;
  sh.t = (int)t;
  return sh;
}

size_t conv_lds_bytes(int k, const ConvShape& sh) {
  const int kp = conv_mfma_kp(k);
  const size_t xs = (size_t)sh.t * (16 * sh.nc + kp - 1);
  const size_t ks = (size_t)(sh.t + 15) * (kp + 1);
  const size_t part = sh.s > 1 ? (size_t)256 * sh.nc * sh.s : 0;
  return sizeof(float) * (xs + ks + part);
}

template <bool kFlip, int NC, int S>
__device__ __forceinline__ void conv_tile_mfma(const float* __restrict__ img, int nx, int ny,
                                               const float* __restrict__ psf, int k, int T,
                                               float* __restrict__ out, int tile_x, int tile_y, float* lds) {
  constexpr int kThreads = 64 * NC * S;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int wc = w % NC, ws = w / NC;
  const int c = (k - 1) / 2, kp = conv_mfma_kp(k);
  const int XW = 16 * NC + kp - 1, KW = kp + 1;
  float* xs = lds;                          // [T][XW]       input rows of the chunk
  float* ks = lds + T * XW;                 // [T + 15][KW]  kernel rows they meet
  float* part = ks + (T + 15) * KW;         // [NC S][256]   partial tiles (S > 1)
  const int i0 = tile_y * 16, j0 = tile_x * 16 * NC;
  const int colmin = j0 - (kp - 1) + c;
  const int nrows = 16 + k - 1;
  const int rows_per_wave = (T + S - 1) / S;
  const int il = lane & 15, bb = lane >> 4;
  jt_floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  for (int t0 = 0; t0 < nrows; t0 += T) {
    const int tn = min(T, nrows - t0);
    const int amin = 2 * c - t0 - (T - 1);
    __syncthreads();
    // wave w stages rows w, w + NC S, ...; its lanes the columns
    for (int tt = w; tt < T; tt += NC * S) {
      const int gi = i0 - c + t0 + tt;
      const bool row_in = tt < tn && gi >= 0 && gi < ny;
      for (int cc = lane; cc < XW; cc += 64) {
        const int gj = colmin + cc;
        xs[tt * XW + cc] = (row_in && gj >= 0 && gj < nx) ? img[(long)gi * nx + gj] : 0.f;
      }
    }
    for (int rr = w; rr < T + 15; rr += NC * S) {
      const int a = amin + rr;
      const bool row_in = a >= 0 && a < k;
      const float* prow = kFlip ? psf + (k - 1 - a) * k + (k - 1) : psf + a * k;
      for (int b = lane; b < KW; b += 64)
        ks[rr * KW + b] = (row_in && b < k) ? (kFlip ? prow[-b] : prow[b]) : 0.f;
    }
    __syncthreads();
    const int tb = ws * rows_per_wave, te = min(tb + rows_per_wave, tn);
    for (int tt = tb; tt < te; ++tt) {
      // A[i][bb] = K[i + 2c - t][b0 + bb]: ks row i - tt + T - 1
      const float* arow = ks + (il - tt + T - 1) * KW + bb;
      // B[bb][j] = X[t][j - (b0 + bb) + c]: xs row tt, column 16 wc + j - b0 - bb + kp - 1
      const float* brow = xs + tt * XW + 16 * wc + il - bb + kp - 1;
      int b0 = 0;
      for (; b0 + 8 <= kp; b0 += 8) {
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[b0], brow[-b0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[b0 + 4], brow[-(b0 + 4)], acc1, 0, 0, 0);
      }
      if (b0 < kp) acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[b0], brow[-b0], acc0, 0, 0, 0);
    }
  }
  jt_floatx4 acc = acc0 + acc1;
  if (S > 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) part[w * 256 + v * 64 + lane] = acc[v];
    __syncthreads();
    if (ws != 0) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float sum = part[wc * 256 + v * 64 + lane];
      for (int u = 1; u < S; ++u) sum += part[(u * NC + wc) * 256 + v * 64 + lane];
      acc[v] = sum;
    }
  }
  const int j = j0 + 16 * wc + il;
  if (j < nx) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 4 * bb + v;
      if (i < ny) out[(long)i * nx + j] = acc[v];
    }
  }
}


// blockIdx.z selects an image of a batch (strided images, one PSF).
template <bool kFlip, int NC, int S>
__global__ __launch_bounds__(64 * NC * S) void k_conv_mfma(const float* __restrict__ img, long in_stride, int nx,
                                                           int ny, const float* __restrict__ psf, int k, int T,
                                                           float* __restrict__ out, long out_stride) {
  extern __shared__ float lds[];
  conv_tile_mfma<kFlip, NC, S>(img + blockIdx.z * in_stride, nx, ny, psf, k, T, out + blockIdx.z * out_stride,
                               blockIdx.x, blockIdx.y, lds);
}

// Heterogeneous batch: block b convolves tile (tiles[b].y, tiles[b].z) of
// image descs[tiles[b].x]; every descriptor of the launch has this shape's
// (NC, S), its own k and rows per chunk, and the dynamic LDS fits the largest.
template <int NC, int S>
__global__ __launch_bounds__(64 * NC * S) void k_conv_desc(const ConvDesc* __restrict__ descs,
                                                           const int4* __restrict__ tiles) {
  extern __shared__ float lds[];
  const int4 tl = tiles[blockIdx.x];
  const ConvDesc& d = descs[tl.x];
  conv_tile_mfma<false, NC, S>(d.img, d.nx, d.ny, d.psf, d.k, d.t, d.out, tl.y, tl.z, lds);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Wave-groups sharing one sub-pixel's subhalo ranges: enough waves to give
// every SIMD of the 256 CUs about 32 over the launch (four rounds of wave
// slots, so the last, partly filled round costs little), while keeping whole
// pixels (`unit` sub-pixel slots each) in a wave-group.
int pick_split(long points, int unit, int nloop) {
  if (nloop < 64) return 1;
  const long target = 32L * 1024 * 64;
  for (int split = 1; split < 8; split *= 2) {
    const long w = split_lanes(split);
    const long used = (w / unit) * unit;          // slots holding whole pixels
    const long lanes = (points + used - 1) / used * split_threads(split);
    if (lanes >= target) return split;
    if (split_lanes(split * 2) / unit < 1) return split;  // a pixel no longer fits a group
  }
  return 8;
}

hipError_t launch_prep_subhalos(int n, const float* x, const float* y, const float* rs,
                                const float* ars, SubRec* out, hipStream_t st) {
  const int padded = subhalo_table_records(n);
  hipLaunchKernelGGL(k_prep_subhalos, dim3((padded + 255) / 256), dim3(256), 0, st, n, padded, x, y, rs,
                     ars, out);
  return hipGetLastError();
}

hipError_t launch_prep_tnfw(int n, const float* x, const float* y, const float* rs, const float* ars,
                            const float* rt, TRec* out, hipStream_t st) {
  const int padded = subhalo_table_records(n);
  hipLaunchKernelGGL(k_prep_tnfw, dim3((padded + 255) / 256), dim3(256), 0, st, n, padded, x, y, rs, ars, rt, out);
  return hipGetLastError();
}

namespace {
template <class P>
void ray_shoot_on(bool alpha, int split, dim3 grid, int n, const float* x, const float* y, const MacroC& mc,
                  const void* sub, int nloop, float* ox, float* oy, hipStream_t st) {
#define JT_RAY(A, S) hipLaunchKernelGGL((k_ray_shoot<A, S, P>), grid, dim3(split_threads(S)), 0, st, n, x, y, mc, \
                                        sub, nloop, ox, oy)
  if (alpha) {
    if (split == 1) JT_RAY(true, 1); else if (split == 2) JT_RAY(true, 2); else if (split == 4) JT_RAY(true, 4);
    else JT_RAY(true, 8);
  } else {
    if (split == 1) JT_RAY(false, 1); else if (split == 2) JT_RAY(false, 2); else if (split == 4) JT_RAY(false, 4);
    else JT_RAY(false, 8);
  }
#undef JT_RAY
}

template <class P, bool kExtra>
void simulate_on(int split, unsigned blocks, const GridC& g, const MacroC& mc, const void* sub, int nloop,
                 const LightC& src, const LightC& ll, float* img, hipStream_t st) {
#define JT_SIM(S) hipLaunchKernelGGL((k_simulate<S, P, kExtra>), dim3(blocks), dim3(split_threads(S)), 0, st, g, mc, \
                                     sub, nloop, src, ll, img)
  if (split == 1) JT_SIM(1); else if (split == 2) JT_SIM(2); else if (split == 4) JT_SIM(4); else JT_SIM(8);
#undef JT_SIM
}
}  // namespace

hipError_t launch_ray_shoot(bool alpha, bool tnfw, int n, const float* x, const float* y, const MacroC& mc,
                            const void* sub, int nloop, float* ox, float* oy, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int split = pick_split(n, 1, nloop);
  const int w = split_lanes(split);
  const dim3 grid((n + w - 1) / w);
  if (tnfw)
    ray_shoot_on<TnfwPairs>(alpha, split, grid, n, x, y, mc, sub, nloop, ox, oy, st);
  else
    ray_shoot_on<NfwPairs>(alpha, split, grid, n, x, y, mc, sub, nloop, ox, oy, st);
  return hipGetLastError();
}

hipError_t launch_source_sb(int n, const float* x, const float* y, const float* bx, const float* by,
                            const LightC& src, const LightC& ll, float* sb, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const bool hs = light_any(src), hl = light_any(ll);
  const auto a16 = [](const float* p) { return ((uintptr_t)p & 15) == 0; };
  const bool extra = light_has_extra(src) || light_has_extra(ll);
  // The extra profiles take one point per thread: four inlined copies of their
  // code (shapelets above all) left the four-point variant with 97 VGPRs and
  // 2 KB of per-lane scratch, four times slower than the plain Sersic list.
  const bool vec = !extra && a16(sb) && (!hs || (a16(bx) && a16(by))) && (!hl || (a16(x) && a16(y)));
  const int threads = vec ? (n >> 2) + (n & 3) : n;
  const dim3 grid((threads + 255) / 256), block(256);
  if (vec)
    hipLaunchKernelGGL((k_source_sb<false, true>), grid, block, 0, st, n, x, y, bx, by, src, ll, sb);
  else if (extra)
    hipLaunchKernelGGL((k_source_sb<true, false>), grid, block, 0, st, n, x, y, bx, by, src, ll, sb);
  else
    hipLaunchKernelGGL((k_source_sb<false, false>), grid, block, 0, st, n, x, y, bx, by, src, ll, sb);
  return hipGetLastError();
}

hipError_t launch_simulate(GridC g, const MacroC& mc, bool tnfw, const void* sub, int nloop, const LightC& src,
                           const LightC& ll, float* img, hipStream_t st) {
  const long npix = (long)g.nx * g.ny;
  const int split = pick_split(npix * g.s2, g.s2, nloop);
  g.ppb = split_lanes(split) / g.s2;
  const long blocks = (npix + g.ppb - 1) / g.ppb;
  const bool extra = light_has_extra(src) || light_has_extra(ll);
  if (tnfw && extra)
    simulate_on<TnfwPairs, true>(split, (unsigned)blocks, g, mc, sub, nloop, src, ll, img, st);
  else if (tnfw)
    simulate_on<TnfwPairs, false>(split, (unsigned)blocks, g, mc, sub, nloop, src, ll, img, st);
  else if (extra)
    simulate_on<NfwPairs, true>(split, (unsigned)blocks, g, mc, sub, nloop, src, ll, img, st);
  else
    simulate_on<NfwPairs, false>(split, (unsigned)blocks, g, mc, sub, nloop, src, ll, img, st);
  return hipGetLastError();
}


namespace {
template <class P>
void basis_on(int split, unsigned blocks, const GridC& g, const MacroC& mc, const void* sub, int nloop,
              const LightC& src, const LightC& ll, float* basis, hipStream_t st) {
#define JT_BAS(S) hipLaunchKernelGGL((k_simulate_basis<S, P>), dim3(blocks), dim3(split_threads(S)), 0, st, g, mc, \
                                     sub, nloop, src, ll, basis)
  if (split == 1) JT_BAS(1); else if (split == 2) JT_BAS(2); else if (split == 4) JT_BAS(4); else JT_BAS(8);
#undef JT_BAS
}
}  // namespace

hipError_t launch_simulate_basis(GridC g, const MacroC& mc, bool tnfw, const void* sub, int nloop,
                                 const LightC& src, const LightC& ll, float* basis, hipStream_t st) {
  const long npix = (long)g.nx * g.ny;
  const int split = pick_split(npix * g.s2, g.s2, nloop);
  g.ppb = split_lanes(split) / g.s2;
  const long blocks = (npix + g.ppb - 1) / g.ppb;
  if (tnfw)
    basis_on<TnfwPairs>(split, (unsigned)blocks, g, mc, sub, nloop, src, ll, basis, st);
  else
    basis_on<NfwPairs>(split, (unsigned)blocks, g, mc, sub, nloop, src, ll, basis, st);
  return hipGetLastError();
}

hipError_t launch_conv_direct(const float* img, int nx, int ny, const float* psf, int k, float* out,
                              hipStream_t st) {
  return launch_conv_direct_batched(false, 1, img, 0, nx, ny, psf, k, out, 0, st);
}

int conv_shape_kind(const ConvShape& sh) { return sh.nc == 4 ? 0 : sh.nc == 2 ? 1 : 2; }
int conv_tiles_x(int nx, const ConvShape& sh) { return (nx + 16 * sh.nc - 1) / (16 * sh.nc); }
int conv_tiles_y(int ny) { return (ny + 15) / 16; }

hipError_t launch_conv_direct_batched(bool flip, int batch, const float* img, long in_stride, int nx, int ny,
                                      const float* psf, int k, float* out, long out_stride, hipStream_t st) {
  const ConvShape sh = conv_shape(nx, ny, k);
  const dim3 grid(conv_tiles_x(nx, sh), conv_tiles_y(ny), batch);
  const size_t lds = conv_lds_bytes(k, sh);
#define JT_CM(F, N, S) hipLaunchKernelGGL((k_conv_mfma<F, N, S>), grid, dim3(64 * N * S), lds, st, img, in_stride, \
                                          nx, ny, psf, k, sh.t, out, out_stride)
  if (flip) {
    if (sh.nc == 4) JT_CM(true, 4, 1); else if (sh.nc == 2) JT_CM(true, 2, 2); else JT_CM(true, 1, 8);
  } else {
    if (sh.nc == 4) JT_CM(false, 4, 1); else if (sh.nc == 2) JT_CM(false, 2, 2); else JT_CM(false, 1, 8);
  }
#undef JT_CM
  return hipGetLastError();
}

hipError_t launch_conv_desc(int kind, const ConvDesc* descs, const int4* tiles, int ntiles, size_t lds,
                            hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)ntiles);
  if (kind == 0)
    hipLaunchKernelGGL((k_conv_desc<4, 1>), grid, dim3(256), lds, st, descs, tiles);
  else if (kind == 1)
    hipLaunchKernelGGL((k_conv_desc<2, 2>), grid, dim3(256), lds, st, descs, tiles);
  else
    hipLaunchKernelGGL((k_conv_desc<1, 8>), grid, dim3(512), lds, st, descs, tiles);
  return hipGetLastError();
}


hipError_t launch_simulate_desc(int split, bool tnfw, bool extra, bool keep_beta, const ImageDesc* descs,
                                const int2* tiles, int nblocks, int blocks_per_image, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;

#define JT_SIMD(S, P, E, K) hipLaunchKernelGGL((k_simulate_desc<S, P, E, K>), dim3((unsigned)nblocks), \
                                               dim3(split_threads(S)), 0, st, descs, tiles, blocks_per_image)
#define JT_SIMD_S(P, E, K) \
  if (split == 1) JT_SIMD(1, P, E, K); else if (split == 2) JT_SIMD(2, P, E, K); \
  else if (split == 4) JT_SIMD(4, P, E, K); else JT_SIMD(8, P, E, K)
  if (keep_beta && tnfw) {
    JT_SIMD_S(TnfwPairs, false, true);
  } else if (keep_beta) {
    JT_SIMD_S(NfwPairs, false, true);
  } else if (tnfw && extra) {
    JT_SIMD_S(TnfwPairs, true, false);
  } else if (tnfw) {
    JT_SIMD_S(TnfwPairs, false, false);
  } else if (extra) {
    JT_SIMD_S(NfwPairs, true, false);
  } else {
    JT_SIMD_S(NfwPairs, false, false);
  }
#undef JT_SIMD_S
#undef JT_SIMD
  return hipGetLastError();
}

// grid (ceil(records / 256), B): draw b's SoA [b][n] -> table b of `records`.
__global__ __launch_bounds__(256) void k_prep_subhalos_batched(int n, int records, const float* __restrict__ x,
                                                              const float* __restrict__ y,
                                                              const float* __restrict__ rs,
                                                              const float* __restrict__ ars,
                                                              SubRec* __restrict__ out) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= records) return;
  SubRec* o = out + (size_t)b * records;
  if (i >= n) {
    o[i] = kSubRecPad;
    return;
  }
  const size_t j = (size_t)b * n + i;
  o[i] = make_subrec(x[j], y[j], rs[j], ars[j]);
}

__global__ __launch_bounds__(256) void k_prep_tnfw_batched(int n, int records, const float* __restrict__ x,
                                                          const float* __restrict__ y, const float* __restrict__ rs,
                                                          const float* __restrict__ ars,
                                                          const float* __restrict__ rt, int unit,
                                                          TRec* __restrict__ out) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= records) return;
  TRec* o = out + (size_t)b * records;
  if (i >= n) {
    o[i] = trec_pad();
    return;
  }
  const size_t j = (size_t)b * n + i;
  o[i] = make_trec(x[j], y[j], rs[j], unit ? 1.0f : ars[j], rt[j]);
}

hipError_t launch_prep_tnfw_batched(int B, int n, const float* x, const float* y, const float* rs, const float* ars,
                                    const float* rt, bool unit, TRec* out, hipStream_t st) {
  const int records = subhalo_table_records(n);
  hipLaunchKernelGGL(k_prep_tnfw_batched, dim3((records + 255) / 256, B), dim3(256), 0, st, n, records, x, y, rs,
                     ars, rt, unit ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_prep_subhalos_batched(int B, int n, const float* x, const float* y, const float* rs,
                                        const float* ars, SubRec* out, hipStream_t st) {
  const int records = subhalo_table_records(n);
  hipLaunchKernelGGL(k_prep_subhalos_batched, dim3((records + 255) / 256, B), dim3(256), 0, st, n, records, x, y, rs,
                     ars, out);
  return hipGetLastError();
}

}  // namespace jt
