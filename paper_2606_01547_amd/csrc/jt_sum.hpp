// The canonical subhalo summation order shared by the forward and adjoint
// kernels (gfx950).
#pragma once

#include "jt_device.hpp"

namespace jt {

constexpr int kSubTile = 64;

// The subhalo table viewed through the constant address space: it is never
// written while a kernel reads it, and this lets wave-uniform reads become
// scalar loads even when the table pointer itself was read from memory.
typedef const __attribute__((address_space(4))) float* SubTable;

__device__ __forceinline__ SubRec load_rec(SubTable t, int k) {
  return SubRec{t[4 * k], t[4 * k + 1], t[4 * k + 2], t[4 * k + 3]};
}

// ---------------------------------------------------------------------------
// Canonical subhalo summation order.  The nloop records (a multiple of 4) are
// cut into kQuarters contiguous ranges with boundaries that are multiples of
// 4; each range is summed in tiles of kSubTile pairs (plain FP32 inside a
// tile, TwoSum across tiles), and the ranges are combined in index order.  A
// launch may hand the ranges of one sub-pixel to 1, 2 or 4 waves (kSplit);
// the arithmetic and its order do not change, so every launch shape gives
// bitwise the same deflection.
// ---------------------------------------------------------------------------
constexpr int kQuarters = 4;

__host__ __device__ __forceinline__ int quarter_bound(int nloop, int q) {
  const int step = ((nloop + 15) / 16) * 4;  // ceil(nloop / 4) rounded up to a multiple of 4
  return min(q * step, nloop);
}

// Sum of the pair terms over records [kb, ke) as (hi, lo) per component.  The
// table holds 4 readable records past every range end (the next range, or
// the padding at the end), so the next group is always prefetched.
__device__ __forceinline__ float4 subhalo_range_sum(float tx, float ty, const SubRec* table, int kb, int ke) {
  const SubTable sub = (SubTable)(const float*)table;
  float hx = 0.f, lx = 0.f, hy = 0.f, ly = 0.f;
  SubRec n0 = load_rec(sub, kb), n1 = load_rec(sub, kb + 1), n2 = load_rec(sub, kb + 2), n3 = load_rec(sub, kb + 3);
  for (int k0 = kb; k0 < ke; k0 += kSubTile) {
    const int kend = min(k0 + kSubTile, ke);
    float px = 0.f, py = 0.f;
    for (int k = k0; k < kend; k += 4) {
      const SubRec s0 = n0, s1 = n1, s2 = n2, s3 = n3;
      n0 = load_rec(sub, k + 4);
      n1 = load_rec(sub, k + 5);
      n2 = load_rec(sub, k + 6);
      n3 = load_rec(sub, k + 7);
      nfw_pairs4(tx, ty, s0, s1, s2, s3, px, py);
    }
    two_sum_acc(hx, lx, px);
    two_sum_acc(hy, ly, py);
  }
  return make_float4(hx, lx, hy, ly);
}

// Total deflection in FP64 at the sub-pixel (tx, ty): the macro lens plus the
// (hi, lo) quarter partials of the subhalo sum, added in quarter order.
__device__ __forceinline__ void total_deflection64(const MacroC& mc, double tx, double ty, const float4* q,
                                                   int stride, double& ax, double& ay) {
  macro_deflection64(mc, tx, ty, ax, ay);
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int i = 0; i < kQuarters; ++i) {
    const float4 v = q[i * stride];
    sx += (double)v.x + (double)v.y;
    sy += (double)v.z + (double)v.w;
  }
  ax += sx;
  ay += sy;
}

// Per-block quarter partials: [quarter][slot], slot < 256 / kSplit.
template <int kSplit>
struct QuarterScratch {
  float4 q[kQuarters][256 / kSplit];
};

// The quarters handled by wave-group g of kSplit, for the sub-pixel (tx, ty),
// written to scratch.q[*][slot].
template <int kSplit>
__device__ __forceinline__ void subhalo_quarters(float tx, float ty, const SubRec* __restrict__ sub, int nloop,
                                                 int g, int slot, QuarterScratch<kSplit>& scratch) {
  constexpr int kPer = kQuarters / kSplit;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int q = g * kPer + i;
    scratch.q[q][slot] = subhalo_range_sum(tx, ty, sub, quarter_bound(nloop, q), quarter_bound(nloop, q + 1));
  }
}

}  // namespace jt
