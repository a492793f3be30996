// Linear amplitude solver kernels for gfx950: the weighted normal equations
// of the unit-amplitude basis images (FP64 partial sums in a fixed order), a
// one-thread Cholesky solve, then the model image and its log-likelihood.
//
//  k_normal_partials  per block: sum_i w B_j B_l (l <= j) and sum_i w B_j d
//  k_solve_amplitudes block sums in order; Jacobi-scaled Cholesky in LDS
//  k_model_partials   model = sum_j a_j B_j (FP64, rounded once); -1/2 w r^2
//  k_sum_logl         the block partials in order
#include "jt_device.hpp"
#include "jt_kernels.hpp"

namespace jt {

namespace {
constexpr int kPairTerms = kMaxBasis * (kMaxBasis + 1) / 2;

// Deterministic block sum of one double per thread (256 threads).
__device__ __forceinline__ double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}
}  // namespace

__global__ __launch_bounds__(256) void k_normal_partials(int npix, int n, const float* __restrict__ B,
                                                        const float* __restrict__ d, const float* __restrict__ w,
                                                        double* __restrict__ part) {
  __shared__ double red[256];
  double acc[kLinTerms];
#pragma unroll
  for (int t = 0; t < kLinTerms; ++t) acc[t] = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < npix; i += (long)gridDim.x * 256) {
    double b[kMaxBasis];
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j) b[j] = j < n ? (double)B[(long)j * npix + i] : 0.0;
    const double wi = w[i];
    const double wd = wi * (double)d[i];
    int t = 0;
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j) {
      const double wb = wi * b[j];
#pragma unroll
      for (int l = 0; l <= j; ++l) acc[t++] += wb * b[l];
    }
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j) acc[kPairTerms + j] += wd * b[j];
  }
#pragma unroll
  for (int t = 0; t < kLinTerms; ++t) {
    const double s = block_sum256(acc[t], red);
    if (threadIdx.x == 0) part[(long)blockIdx.x * kLinTerms + t] = s;
  }
}

// One block of 64 threads.  Packed terms: (j, l <= j) row by row, then the
// right-hand side.  The matrix is scaled to unit diagonal before the
// factorisation; a pivot below 1e-12 (a component that adds nothing, or
// two that coincide) marks the system singular and every amplitude NaN.
__global__ __launch_bounds__(64) void k_solve_amplitudes(int n, int nblocks, const double* __restrict__ part,
                                                         double* __restrict__ amps) {
  __shared__ double M[kLinTerms];
  __shared__ double A[kMaxBasis][kMaxBasis];
  __shared__ double v[kMaxBasis], D[kMaxBasis];
  const int t = threadIdx.x;
  if (t < kLinTerms) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(long)b * kLinTerms + t];
    M[t] = s;
  }
  __syncthreads();
  if (t != 0) return;
  int idx = 0;
  for (int j = 0; j < kMaxBasis; ++j)
    for (int l = 0; l <= j; ++l, ++idx) {
      A[j][l] = M[idx];
      A[l][j] = M[idx];
    }
  bool ok = true;
  for (int j = 0; j < n; ++j) {
    v[j] = M[kPairTerms + j];
    if (!(A[j][j] > 0.0)) ok = false;
    D[j] = ok ? 1.0 / sqrt(A[j][j]) : 0.0;
  }
  if (ok) {
    for (int j = 0; j < n; ++j) {
      for (int l = 0; l < n; ++l) A[j][l] *= D[j] * D[l];
      v[j] *= D[j];
    }
    // A = L L^T in the lower triangle
    for (int j = 0; j < n && ok; ++j) {
      double s = A[j][j];
      for (int k = 0; k < j; ++k) s -= A[j][k] * A[j][k];
      if (!(s > 1e-12)) {
        ok = false;
        break;
      }
      const double ljj = sqrt(s);
      A[j][j] = ljj;
      for (int i = j + 1; i < n; ++i) {
        double r = A[i][j];
        for (int k = 0; k < j; ++k) r -= A[i][k] * A[j][k];
        A[i][j] = r / ljj;
      }
    }
  }
  if (!ok) {
    for (int j = 0; j < n; ++j) amps[j] = __longlong_as_double(0x7ff8000000000000LL);
    return;
  }
  for (int j = 0; j < n; ++j) {          // L y = v
    double r = v[j];
    for (int k = 0; k < j; ++k) r -= A[j][k] * v[k];
    v[j] = r / A[j][j];
  }
  for (int j = n - 1; j >= 0; --j) {     // L^T x = y
    double r = v[j];
    for (int k = j + 1; k < n; ++k) r -= A[k][j] * v[k];
    v[j] = r / A[j][j];
  }
  for (int j = 0; j < n; ++j) amps[j] = v[j] * D[j];
}

__global__ __launch_bounds__(256) void k_model_partials(int npix, int n, const float* __restrict__ B,
                                                       const double* __restrict__ amps,
                                                       const float* __restrict__ d, const float* __restrict__ w,
                                                       float* __restrict__ model, double* __restrict__ part) {
  __shared__ double red[256];
  __shared__ double a[kMaxBasis];
  if (threadIdx.x < kMaxBasis) a[threadIdx.x] = threadIdx.x < n ? amps[threadIdx.x] : 0.0;
  __syncthreads();
  double acc = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < npix; i += (long)gridDim.x * 256) {
    double m = 0.0;
    for (int j = 0; j < n; ++j) m += a[j] * (double)B[(long)j * npix + i];
    const float mf = (float)m;
    if (model) model[i] = mf;
    const double r = (double)d[i] - (double)mf;
    acc += -0.5 * (double)w[i] * r * r;
  }
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(64) void k_sum_logl(int nblocks, const double* __restrict__ part,
                                                 double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[b];
  *out = s;
}

// part: kLinBlocks * (kLinTerms + 1) doubles of workspace.
hipError_t launch_linear_solve(int npix, int n, const float* basis, const float* data, const float* w,
                               double* part, double* amps, float* model, double* logL, hipStream_t st) {
  double* part2 = part + (long)kLinBlocks * kLinTerms;
  hipLaunchKernelGGL(k_normal_partials, dim3(kLinBlocks), dim3(256), 0, st, npix, n, basis, data, w, part);
  hipLaunchKernelGGL(k_solve_amplitudes, dim3(1), dim3(64), 0, st, n, kLinBlocks, part, amps);
  if (model || logL)
    hipLaunchKernelGGL(k_model_partials, dim3(kLinBlocks), dim3(256), 0, st, npix, n, basis, amps, data, w, model,
                       part2);
  if (logL) hipLaunchKernelGGL(k_sum_logl, dim3(1), dim3(64), 0, st, kLinBlocks, part2, logL);
  return hipGetLastError();
}

}  // namespace jt
