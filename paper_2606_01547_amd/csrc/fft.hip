// FFT convolution (the paper's FFT-convolution section): FP64 complex
// transforms of zero-padded rows and columns, a pointwise product with the
// kernel spectrum, the inverse transforms and a crop to the same-size output.
//
// Each row transform runs in LDS as a radix-2 Stockham autosort FFT
// (Stockham; formulation of Govindaraju et al. 2008): log2 N stages, stage
// with half-span L reads src[j] and src[j + N/2], multiplies the second by
// exp(-+2 pi i (j mod L) / (2L)) and writes the sum and difference to
// dst[2L floor(j/L) + (j mod L)] and that index + L.  Columns are transformed
// as rows of a transposed array.
//
// Sizes: Nx >= max(nx + c, k) and Ny >= max(ny + c, k) (c = (k-1)/2), powers
// of two up to kFftMaxN; with that padding the circular convolution equals the
// linear one on every output of the "same" region (the wrapped indices of the
// image land in zero padding, and the kernel itself is not wrapped).  FP64 keeps the round-off ~1e-15 of
// the image maximum, far inside the per-pixel error bar of faint pixels.
#include "jt_device.hpp"
#include "jt_kernels.hpp"

namespace jt {

constexpr int kFftThreads = 256;

// In-LDS FFT of length N = 2^logN over buffers a (input) and b; returns the
// buffer holding the result.  tw[t] = exp(-2 pi i t / N), t < N/2.
__device__ __forceinline__ double2* fft_lds(double2* a, double2* b, int N, const double2* __restrict__ tw, bool inverse) {
  const int half = N >> 1;
  double2* src = a;
  double2* dst = b;
  for (int L = 1; L < N; L <<= 1) {
    const int stride = N / (2 * L);   // twiddle index step
    for (int j = threadIdx.x; j < half; j += blockDim.x) {
      const int k = j & (L - 1);
      const double2 w0 = tw[k * stride];
      const double wr = w0.x, wi = inverse ? -w0.y : w0.y;
      const double2 u = src[j];
      const double2 v = src[j + half];
      const double vr = v.x * wr - v.y * wi;
      const double vi = v.x * wi + v.y * wr;
      const int d = 2 * (j - k) + k;
      dst[d] = make_double2(u.x + vr, u.y + vi);
      dst[d + L] = make_double2(u.x - vr, u.y - vi);
    }
    __syncthreads();
    double2* t = src;
    src = dst;
    dst = t;
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
int fft_size_for(int n, int k) {
  const int need = n + (k - 1) / 2 > k ? n + (k - 1) / 2 : k;
  int N = kFftMinN;
  while (N < need) N <<= 1;
  return N;
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
