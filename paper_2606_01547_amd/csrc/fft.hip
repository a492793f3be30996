// FFT convolution (the paper's FFT-convolution section): FP64 complex
// transforms of zero-padded rows and columns, a pointwise product with the
// kernel spectrum, the inverse transforms and a crop to the same-size output.
//
// Each row transform runs in LDS as a mixed-radix Stockham autosort FFT
// (radices 4, 2, 3 and 5; the radix-2 formulation of Govindaraju et al. 2008
// generalised to radix p): a pass of radix p over sub-transforms of length Ns
// takes, for j < N/p with k = j mod Ns, the p values src[j + t N/p],
// multiplies value t by exp(-+2 pi i t k / (Ns p)), applies the p-point DFT and
// writes its outputs to dst[(j - k) p + k + t Ns]; after the passes (radix 4
// while N has a factor 4, then 2, 3, 5) the result is in natural order.
// Columns are transformed as rows of a transposed array.
//
// Sizes: Nx >= max(nx + c, k) and Ny >= max(ny + c, k) (c = (k-1)/2), the
// smallest such products 2^a 3^b 5^c up to kFftMaxN (a 1000-pixel side with a
// 101-pixel kernel pads to 1080, not 2048); with that padding the circular
// convolution equals the linear one on every output of the "same" region (the
// wrapped indices of the image land in zero padding, and the kernel itself is
// not wrapped).  FP64 keeps the round-off ~1e-15 of the image maximum, far
// inside the per-pixel error bar of faint pixels.
#include "jt_device.hpp"
#include "jt_kernels.hpp"

namespace jt {

constexpr int kFftThreads = 256;

// p-point DFT of v[0..p) in place: y_m = sum_n v_n exp(-+2 pi i m n / p).
template <int P>
__device__ __forceinline__ void dft_small(double2* v, bool inverse) {
  const double sg = inverse ? -1.0 : 1.0;   // the sign of the sine terms
  if (P == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = make_double2(a.x + b.x, a.y + b.y);
    v[1] = make_double2(a.x - b.x, a.y - b.y);
  } else if (P == 4) {
    // y1 = (a - c) - i (b - d), y3 = (a - c) + i (b - d) for the forward sign
    const double2 a = v[0], b = v[1], c = v[2], d = v[3];
    const double2 s0 = make_double2(a.x + c.x, a.y + c.y), d0 = make_double2(a.x - c.x, a.y - c.y);
    const double2 s1 = make_double2(b.x + d.x, b.y + d.y), d1 = make_double2(b.x - d.x, b.y - d.y);
    v[0] = make_double2(s0.x + s1.x, s0.y + s1.y);
    v[2] = make_double2(s0.x - s1.x, s0.y - s1.y);
    v[1] = make_double2(d0.x + sg * d1.y, d0.y - sg * d1.x);
    v[3] = make_double2(d0.x - sg * d1.y, d0.y + sg * d1.x);
  } else {
    // direct sums with exp(-2 pi i q / P), q < P
    constexpr double kC3[3] = {1.0, -0.5, -0.5};
    constexpr double kS3[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
    constexpr double kC5[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410, -0.80901699437494742410,
                               0.30901699437494742410};
    constexpr double kS5[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917, -0.58778525229247312917,
                               -0.95105651629515357212};
    const double* C = P == 3 ? kC3 : kC5;
    const double* S = P == 3 ? kS3 : kS5;
    double2 x[P];
#pragma unroll
    for (int n = 0; n < P; ++n) x[n] = v[n];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int n = 0; n < P; ++n) {
        const int q = (m * n) % P;
        const double c = C[q], sn = -sg * S[q];   // exp(-+i theta) = cos -+ i sin
        re += x[n].x * c - x[n].y * sn;
        im += x[n].x * sn + x[n].y * c;
      }
      v[m] = make_double2(re, im);
    }
  }
}

// One Stockham pass of radix P from src to dst (N points, sub-transforms of
// length Ns so far); tw[t] = exp(-2 pi i t / N), t < N.
template <int P>
__device__ __forceinline__ void fft_pass(const double2* __restrict__ src, double2* __restrict__ dst, int N, int Ns,
                                         const double2* __restrict__ tw, bool inverse) {
  const int m = N / P;
  const int step = N / (Ns * P);
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const int k = j % Ns;
    double2 v[P];
#pragma unroll
    for (int t = 0; t < P; ++t) v[t] = src[j + t * m];
#pragma unroll
    for (int t = 1; t < P; ++t) {
      const double2 w = tw[t * k * step];
      const double wi = inverse ? -w.y : w.y;
      v[t] = make_double2(v[t].x * w.x - v[t].y * wi, v[t].x * wi + v[t].y * w.x);
    }
    dft_small<P>(v, inverse);
    const int d = (j - k) * P + k;
#pragma unroll
    for (int t = 0; t < P; ++t) dst[d + t * Ns] = v[t];
  }
}

// In-LDS FFT of length N (a product of 2, 3 and 5) over buffers a (input) and
// b; returns the buffer holding the result.  tw[t] = exp(-2 pi i t / N), t < N.
__device__ __forceinline__ double2* fft_lds(double2* a, double2* b, int N, const double2* __restrict__ tw, bool inverse) {
  double2* src = a;
  double2* dst = b;
  int Ns = 1, rem = N;
  while (rem > 1) {
    const int p = (rem & 3) == 0 ? 4 : (rem & 1) == 0 ? 2 : rem % 3 == 0 ? 3 : 5;
    if (p == 4) fft_pass<4>(src, dst, N, Ns, tw, inverse);
    else if (p == 2) fft_pass<2>(src, dst, N, Ns, tw, inverse);
    else if (p == 3) fft_pass<3>(src, dst, N, Ns, tw, inverse);
    else fft_pass<5>(src, dst, N, Ns, tw, inverse);
    __syncthreads();
    double2* t = src;
    src = dst;
    dst = t;
    rem /= p;
    Ns *= p;
  }
  return src;
}

// Forward FFT of each padded real row: A[r][0..Nx) = FFT(img row r, zeros),
// rows r >= ny are zero.  grid = Ny blocks.
__global__ __launch_bounds__(kFftThreads) void k_fft_rows_real(const float* __restrict__ img, int nx, int ny, int Nx,
                                                              double2* __restrict__ A, const double2* __restrict__ tw) {
  extern __shared__ double2 sh[];
  double2* a = sh;
  double2* b = sh + Nx;
  const int r = blockIdx.x;
  double2* row = A + (size_t)r * Nx;
  if (r >= ny) {
    for (int j = threadIdx.x; j < Nx; j += blockDim.x) row[j] = make_double2(0.0, 0.0);
    return;
  }
  for (int j = threadIdx.x; j < Nx; j += blockDim.x)
    a[j] = make_double2(j < nx ? (double)img[(size_t)r * nx + j] : 0.0, 0.0);
  __syncthreads();
  const double2* res = fft_lds(a, b, Nx, tw, false);
  for (int j = threadIdx.x; j < Nx; j += blockDim.x) row[j] = res[j];
}

// B[c][r] = A[r][c] for A [rows][cols]; 32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose_c(const double2* __restrict__ A, int rows, int cols,
                                                    double2* __restrict__ B) {
  __shared__ double2 t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int i = ty; i < 32; i += 8) {
    const int r = by + i, c = bx + tx;
    if (r < rows && c < cols) t[i][tx] = A[(size_t)r * cols + c];
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int c = bx + i, r = by + tx;
    if (r < rows && c < cols) B[(size_t)c * rows + r] = t[tx][i];
  }
}

// In place on each row of B [rows][N]: forward FFT, then (spec != null)
// multiply by spec's row and inverse FFT.  grid = rows blocks.
__global__ __launch_bounds__(kFftThreads) void k_fft_rows_mul(double2* __restrict__ B, int N,
                                                             const double2* __restrict__ spec,
                                                             const double2* __restrict__ tw) {
  extern __shared__ double2 sh[];
  double2* a = sh;
  double2* b = sh + N;
  double2* row = B + (size_t)blockIdx.x * N;
  for (int j = threadIdx.x; j < N; j += blockDim.x) a[j] = row[j];
  __syncthreads();
  double2* res = fft_lds(a, b, N, tw, false);
  if (spec) {
    const double2* srow = spec + (size_t)blockIdx.x * N;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      const double2 x = res[j], y = srow[j];
      res[j] = make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
    }
    __syncthreads();
    double2* other = (res == a) ? b : a;
    res = fft_lds(res, other, N, tw, true);
  }
  for (int j = threadIdx.x; j < N; j += blockDim.x) row[j] = res[j];
}

// Inverse FFT of rows c .. c+ny-1 of A [Ny][Nx] and the crop
// out[i][j] = Re(row_{i+c}[j + c]) * scale.  grid = ny blocks.
__global__ __launch_bounds__(kFftThreads) void k_fft_rows_crop(const double2* __restrict__ A, int Nx, int nx, int c,
                                                              double scale, float* __restrict__ out,
                                                              const double2* __restrict__ tw) {
  extern __shared__ double2 sh[];
  double2* a = sh;
  double2* b = sh + Nx;
  const int i = blockIdx.x;
  const double2* row = A + (size_t)(i + c) * Nx;
  for (int j = threadIdx.x; j < Nx; j += blockDim.x) a[j] = row[j];
  __syncthreads();
  const double2* res = fft_lds(a, b, Nx, tw, true);
  for (int j = threadIdx.x; j < nx; j += blockDim.x) out[(size_t)i * nx + j] = (float)(res[j + c].x * scale);
}

// ---------------------------------------------------------------------------
// Smallest 2^a 3^b 5^c >= max(n + (k-1)/2, k, kFftMinN).
int fft_size_for(int n, int k) {
  int N = n + (k - 1) / 2 > k ? n + (k - 1) / 2 : k;
  if (N < kFftMinN) N = kFftMinN;
  for (;; ++N) {
    int r = N;
    for (int p : {2, 3, 5})
      while (r % p == 0) r /= p;
    if (r == 1) return N;
  }
}

size_t fft_workspace_bytes(int nx, int ny, int k) {
  const size_t Nx = (size_t)fft_size_for(nx, k), Ny = (size_t)fft_size_for(ny, k);
  return 3 * Nx * Ny * sizeof(double2);
}

hipError_t launch_fft_convolve(const float* img, int nx, int ny, const float* psf, int k, float* out, void* ws,
                               const double2* tw_x, const double2* tw_y, hipStream_t st) {
  const int c = (k - 1) / 2;
  const int Nx = fft_size_for(nx, k), Ny = fft_size_for(ny, k);
  double2* A = (double2*)ws;
  double2* B = A + (size_t)Nx * Ny;
  double2* Kf = B + (size_t)Nx * Ny;
  const dim3 tb(256);
  const size_t shx = 2 * sizeof(double2) * Nx, shy = 2 * sizeof(double2) * Ny;
  // kernel spectrum, transposed layout [Nx][Ny]
  hipLaunchKernelGGL(k_fft_rows_real, dim3(Ny), dim3(kFftThreads), shx, st, psf, k, k, Nx, A, tw_x);
  hipLaunchKernelGGL(k_transpose_c, dim3((Nx + 31) / 32, (Ny + 31) / 32), tb, 0, st, A, Ny, Nx, Kf);
  hipLaunchKernelGGL(k_fft_rows_mul, dim3(Nx), dim3(kFftThreads), shy, st, Kf, Ny, nullptr, tw_y);
  // image
  hipLaunchKernelGGL(k_fft_rows_real, dim3(Ny), dim3(kFftThreads), shx, st, img, nx, ny, Nx, A, tw_x);
  hipLaunchKernelGGL(k_transpose_c, dim3((Nx + 31) / 32, (Ny + 31) / 32), tb, 0, st, A, Ny, Nx, B);
  hipLaunchKernelGGL(k_fft_rows_mul, dim3(Nx), dim3(kFftThreads), shy, st, B, Ny, Kf, tw_y);
  hipLaunchKernelGGL(k_transpose_c, dim3((Ny + 31) / 32, (Nx + 31) / 32), tb, 0, st, B, Nx, Ny, A);
  hipLaunchKernelGGL(k_fft_rows_crop, dim3(ny), dim3(kFftThreads), shx, st, A, Nx, nx, c,
                     1.0 / ((double)Nx * (double)Ny), out, tw_x);
  return hipGetLastError();
}

}  // namespace jt
