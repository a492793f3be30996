// Issue-rate calibration kernels for the measurement side of the library:
// they fix the per-clock FP32 rates that the roofline figures are stated
// against and check the units of the instruction counters (each counted
// VALU instruction is one wave64 instruction, 64 lane-operations).
//
// Every lane runs `iters` rounds over eight independent chains (b and c
// arrive as kernel arguments, so kinds 0 and 2 compile to FMAs on register
// operands), so the
// issue rate, not the dependency latency, bounds the time when enough waves
// are resident.  The chains converge to 1 (fixed point of a <- 0.999 a + 1e-3
// and of a <- a^(-1/2)), so no value over- or underflows.
//   kind 0: 8 FMA per round                       (FMA rate)
//   kind 1: 8 reciprocal square roots per round   (transcendental rate)
//   kind 2: 16 FMA + 2 reciprocal square roots    (the pair loop's mix)
//   kind 3: 8 multiplies per round                (non-FMA rate)
//   kind 4: 8 FMA with literal constants per round (VOP2 forms carrying a
//           32-bit literal, as polynomial evaluations compile to)
//   kind 5: 8 base-2 logarithms per round         (the other transcendental)
//   kind 6: 8 accumulating FMA a += x b, one SGPR operand (VOP2 v_fmac_f32)
//   kind 7: 8 FMA on three VGPR operands        (VOP3 v_fma_f32, no SGPR)
// The sums of the chains are written to out[blocks * 256] so that nothing is
// optimised away.
#include <hip/hip_runtime.h>

#include "../../include/jt.h"

namespace jt {

constexpr int kCalibThreads = 256;

template <int KIND>
__global__ __launch_bounds__(kCalibThreads) void k_valu_calib(int iters, float b, float c, float* __restrict__ out) {
  float a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = 1.0f + 1e-3f * (float)((threadIdx.x + 31 * i) & 63);
  // per-lane copies of the constants (vector registers) for kinds 6 and 7
  const float lane = (float)(threadIdx.x & 1);
  const float xv = 1e-7f * (1.0f + lane), bv = b + 1e-9f * lane, cv = c - 1e-9f * lane;
#pragma unroll 4
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (KIND == 0) {
        a[i] = fmaf(a[i], b, c);
      } else if (KIND == 1) {
        a[i] = __builtin_amdgcn_rsqf(a[i]);
      } else if (KIND == 2) {
        a[i] = fmaf(a[i], b, c);
        a[i] = fmaf(a[i], b, c);
        if (i < 2) a[i] = __builtin_amdgcn_rsqf(a[i]);
      } else if (KIND == 3) {
        a[i] = a[i] * b;
        a[i] = a[i] * (1.0f / b);
      } else if (KIND == 4) {
        a[i] = fmaf(a[i], 0.999f - 1e-4f * (float)i, 1e-3f + 1e-7f * (float)i);
      } else if (KIND == 5) {
        a[i] = __builtin_amdgcn_logf(a[i]) + 2.0f;
      } else if (KIND == 6) {
        a[i] = fmaf(xv, b, a[i]);
      } else {
        a[i] = fmaf(a[i], bv, cv);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i];
  out[(size_t)blockIdx.x * kCalibThreads + threadIdx.x] = s;
}

}  // namespace jt

extern "C" jt_status jt_calibrate_valu(int kind, int blocks, int iters, float* out, hipStream_t stream) {
  if (kind < 0 || kind > 7 || blocks < 1 || iters < 1 || !out) return JT_EINVAL;
  switch (kind) {
    case 0: hipLaunchKernelGGL(jt::k_valu_calib<0>, dim3(blocks), dim3(jt::kCalibThreads), 0, stream, iters, 0.999f, 1e-3f, out); break;
    case 1: hipLaunchKernelGGL(jt::k_valu_calib<1>, dim3(blocks), dim3(jt::kCalibThreads), 0, stream, iters, 0.999f, 1e-3f, out); break;
    case 2: hipLaunchKernelGGL(jt::k_valu_calib<2>, dim3(blocks), dim3(jt::kCalibThreads), 0, stream, iters, 0.999f, 1e-3f, out); break;
    case 3: hipLaunchKernelGGL(jt::k_valu_calib<3>, dim3(blocks), dim3(jt::kCalibThreads), 0, stream, iters, 0.999f, 1e-3f, out); break;
    case 4: hipLaunchKernelGGL(jt::k_valu_calib<4>, dim3(blocks), dim3(jt::kCalibThreads), 0, stream, iters, 0.999f, 1e-3f, out); break;
    case 5: hipLaunchKernelGGL(jt::k_valu_calib<5>, dim3(blocks), dim3(jt::kCalibThreads), 0, stream, iters, 0.999f, 1e-3f, out); break;
    case 6: hipLaunchKernelGGL(jt::k_valu_calib<6>, dim3(blocks), dim3(jt::kCalibThreads), 0, stream, iters, 0.999f, 1e-3f, out); break;
    default: hipLaunchKernelGGL(jt::k_valu_calib<7>, dim3(blocks), dim3(jt::kCalibThreads), 0, stream, iters, 0.999f, 1e-3f, out); break;
  }
  return hipGetLastError() == hipSuccess ? JT_OK : JT_EDEVICE;
}
