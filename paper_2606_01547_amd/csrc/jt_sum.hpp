// The canonical subhalo summation order shared by the forward and adjoint
// kernels (gfx950).
#pragma once

#include <cstddef>
#include <type_traits>

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
// cut into kRanges contiguous ranges with boundaries that are multiples of 4;
// each range is summed in tiles of kSubTile pairs (plain FP32 inside a tile,
// TwoSum across tiles) into (hi, lo), and the ranges are added in FP64 in
// index order, hi + lo of one range at a time.  A launch hands the ranges of
// one sub-pixel to 1, 2, 4 or 8 wave-groups (kSplit) that leave them in LDS
// for group 0 (one group adds them as it goes); the arithmetic and its order
// do not change, so every launch shape gives bitwise the same deflection.
// ---------------------------------------------------------------------------
constexpr int kRanges = 8;

__host__ __device__ __forceinline__ int range_bound(int nloop, int e) {
  const int step = ((nloop + 4 * kRanges - 1) / (4 * kRanges)) * 4;  // ceil(nloop / kRanges), multiple of 4
  return min(e * step, nloop);
}

// Boundaries of `parts` contiguous parts of n records, multiples of 4 (the
// adjoint's sums over sub-pixel records).
__host__ __device__ __forceinline__ int part_bound(int n, int parts, int q) {
  const int step = ((n + 4 * parts - 1) / (4 * parts)) * 4;
  return min(q * step, n);
}

// The pair kernels of the subhalo profiles: the record type, how a record is
// read from the table, and the contribution of four records at one point.
struct NfwPairs {
  using Rec = SubRec;
  static __device__ __forceinline__ Rec load(SubTable t, int k) { return load_rec(t, k); }
  static __device__ __forceinline__ void run4(float tx, float ty, const Rec& a, const Rec& b, const Rec& c,
                                              const Rec& d, float& px, float& py) {
    nfw_pairs4(tx, ty, a, b, c, d, px, py);
  }
};

// The truncated profile: its records are staged through LDS (tnfw_range_sum),
// so the type only names the record.
struct TnfwPairs {
  using Rec = TRec;
};

// Sum of the pair terms over records [kb, ke) as (hi, lo) per component.  The
// table holds 4 readable records past every range end (the next range, or
// the padding at the end), so the next group is always prefetched.
template <class P>
__device__ __forceinline__ float4 subhalo_range_sum(float tx, float ty, const void* table, int kb, int ke) {
  using Rec = typename P::Rec;
  const SubTable sub = (SubTable)(const float*)table;
  float hx = 0.f, lx = 0.f, hy = 0.f, ly = 0.f;
  Rec n0 = P::load(sub, kb), n1 = P::load(sub, kb + 1), n2 = P::load(sub, kb + 2), n3 = P::load(sub, kb + 3);
  for (int k0 = kb; k0 < ke; k0 += kSubTile) {
    const int kend = min(k0 + kSubTile, ke);
    float px = 0.f, py = 0.f;
    for (int k = k0; k < kend; k += 4) {
      const Rec s0 = n0, s1 = n1, s2 = n2, s3 = n3;
      n0 = P::load(sub, k + 4);
      n1 = P::load(sub, k + 5);
      n2 = P::load(sub, k + 6);
      n3 = P::load(sub, k + 7);
      P::run4(tx, ty, s0, s1, s2, s3, px, py);
    }
    two_sum_acc(hx, lx, px);
    two_sum_acc(hy, ly, py);
  }
  return make_float4(hx, lx, hy, ly);
}

// The truncated profile's 80-byte records: the first 48 bytes (centre, c1, Xf,
// c2, the general form's tau constants, k1 and the far field's three lowest
// coefficients) through scalar loads; the last 32 (the other eight
// coefficients) through LDS.  An FMA reading a scalar register issues at half
// rate on gfx950, but the broadcast LDS reads of a wave (1 KB per 16-byte read)
// share the CU's LDS bandwidth with the other waves, and with three 16-byte
// reads per record they, not the FMAs, set the loop's pace; with two the four
// half-rate FMAs cost less than the read saved.  Each wave copies kStage
// records' 32-byte tails at a time into its own LDS stage (coalesced 16-byte
// loads) and every lane then reads the current tails at one address (a
// broadcast) into vector registers.  Records go two per step (tnfw_pair2), the
// next step's heads loaded while this one computes.  Same pairs, same order,
// same arithmetic as one record at a time from scalar registers, so the same
// sums.  Must be called by whole waves (every lane active; the copy is shared
// out by lane), at most kWaves waves per block.
constexpr int kTnfwHeadF = 12;  // floats of a record's scalar head
constexpr int kTnfwHeadQ = kTnfwHeadF / 4;
constexpr int kTnfwTailQ = 2;   // float4s of a record's LDS tail
static_assert(kTnfwFarDeg == 10 && sizeof(TRec) == (kTnfwHeadQ + kTnfwTailQ) * sizeof(float4) &&
                  offsetof(TRec, a) + 3 * sizeof(float) == kTnfwHeadF * sizeof(float),
              "TRec layout");

__device__ __forceinline__ TRec tnfw_rec(const float (&h)[kTnfwHeadF], const float4* q) {
  const float4 q0 = q[0], q1 = q[1];
  TRec r;
  r.x = h[0];
  r.y = h[1];
  r.c1 = h[2];
  r.Xf = h[3];
  r.tau = h[4];
  r.t2 = h[5];
  r.itau = h[6];
  r.c2 = h[7];
  r.k1 = h[8];
  r.a[0] = h[9];
  r.a[1] = h[10];
  r.a[2] = h[11];
  r.a[3] = q0.x;
  r.a[4] = q0.y;
  r.a[5] = q0.z;
  r.a[6] = q0.w;
  r.a[7] = q1.x;
  r.a[8] = q1.y;
  r.a[9] = q1.z;
  r.a[10] = q1.w;
  return r;
}

// Waits for a step's LDS tail reads before the next step's heads are
// requested: LDS reads and scalar loads count on one counter and scalar loads
// may return out of order, so with the loads issued first the wait for the
// tails would cover the loads as well and the prefetch would gain nothing.
// lgkmcnt(0) with the vector-memory and export counts left open, then a
// scheduling barrier so that the loads are not moved above the wait.
__device__ __forceinline__ void tail_wait() {
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_sched_barrier(0);
}

template <int kWaves, int kStage>
__device__ __forceinline__ float4 tnfw_range_sum(float tx, float ty, const void* table, int kb, int ke) {
  __shared__ float4 stage[kWaves][kStage * kTnfwTailQ];
  float4* st = stage[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63;
  const float4* __restrict__ g4 = (const float4*)table;
  const SubTable sub = (SubTable)(const float*)table;
  constexpr int kF = (int)(sizeof(TRec) / sizeof(float));   // floats per record
  auto head = [&](int k, float (&h)[kTnfwHeadF]) {
#pragma unroll
    for (int i = 0; i < kTnfwHeadF; ++i) h[i] = sub[kF * k + i];
  };
  float hx = 0.f, lx = 0.f, hy = 0.f, ly = 0.f;
  // heads of the next two records, loaded a step ahead (the table has readable
  // records past every range end)
  float ha[kTnfwHeadF], hb[kTnfwHeadF];
  head(kb, ha);
  head(kb + 1, hb);
  for (int k0 = kb; k0 < ke; k0 += kSubTile) {
    const int kend = min(k0 + kSubTile, ke);
    float px = 0.f, py = 0.f;
    for (int s0 = k0; s0 < kend; s0 += kStage) {
      const int m = min(kStage, kend - s0);
      // the previous stage's reads come before these writes, and these writes
      // before the reads below (one wave's LDS operations execute in order)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int e = lane; e < m * kTnfwTailQ; e += 64) {
        const int rk = e / kTnfwTailQ;
        st[e] = g4[(size_t)(s0 + rk) * (kTnfwHeadQ + kTnfwTailQ) + kTnfwHeadQ + (e - rk * kTnfwTailQ)];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // two records per step (m is a multiple of 4: range bounds, tiles and
      // stages all are)
      for (int k = 0; k < m; k += 4) {
        float hc[kTnfwHeadF], hd[kTnfwHeadF];
        {
          const TRec ra = tnfw_rec(ha, st + kTnfwTailQ * k), rb = tnfw_rec(hb, st + kTnfwTailQ * (k + 1));
          tail_wait();
          head(s0 + k + 2, hc);
          head(s0 + k + 3, hd);
          tnfw_pair2(tx, ty, ra, rb, px, py);
        }
        {
          const TRec rc = tnfw_rec(hc, st + kTnfwTailQ * (k + 2)), rd = tnfw_rec(hd, st + kTnfwTailQ * (k + 3));
          tail_wait();
          head(s0 + k + 4, ha);
          head(s0 + k + 5, hb);
          tnfw_pair2(tx, ty, rc, rd, px, py);
        }
      }
    }
    two_sum_acc(hx, lx, px);
    two_sum_acc(hy, ly, py);
  }
  return make_float4(hx, lx, hy, ly);
}

// Range partials of a block's sub-pixels, [range][slot], slot <
// split_lanes(kSplit).  With one group the ranges are added as they are
// computed and nothing is stored.
template <int kSplit>
struct RangeScratch {
  float4 r[kSplit == 1 ? 1 : kRanges][split_lanes(kSplit)];
};

// The ranges of wave-group g for the sub-pixel (tx, ty).  With one group they
// are added to (sx, sy) in FP64 as they are computed; otherwise each group
// stores its ranges for group 0, which adds them after the block's barrier.
template <int kSplit, class P = NfwPairs>
__device__ __forceinline__ void subhalo_ranges(float tx, float ty, const void* __restrict__ sub, int nloop, int g,
                                               int slot, RangeScratch<kSplit>& scratch, double& sx, double& sy) {
  constexpr int kOwn = kRanges / kSplit;
  // LDS stage of the truncated profile: about 20 KB per block with the range
  // partials (40 KB for 8-wave blocks), so that 8 waves per SIMD stay resident
  constexpr int kWaves = split_threads(kSplit) / 64;
  constexpr int kBudget = (kWaves == 8 ? 40960 : 20480) - (int)sizeof(RangeScratch<kSplit>) - 1024;
  constexpr int kRecB = kTnfwTailQ * 16;   // LDS bytes per staged record
  constexpr int kStage = kBudget / (kWaves * kRecB) >= 32 ? 32 : kBudget / (kWaves * kRecB) >= 16 ? 16 : 8;
#pragma unroll 1
  for (int i = 0; i < kOwn; ++i) {
    const int e = g * kOwn + i;
    float4 v;
    if constexpr (std::is_same<P, TnfwPairs>::value)
      v = tnfw_range_sum<kWaves, kStage>(tx, ty, sub, range_bound(nloop, e), range_bound(nloop, e + 1));
    else
      v = subhalo_range_sum<P>(tx, ty, sub, range_bound(nloop, e), range_bound(nloop, e + 1));
    if (kSplit == 1) {
      sx += (double)v.x + (double)v.y;
      sy += (double)v.z + (double)v.w;
    } else {
      scratch.r[e][slot] = v;
    }
  }
}

// Group 0, after the block's barrier: the stored ranges in order, then the
// total deflection in FP64 at the sub-pixel (tx, ty) = macro lens + subhalos.
template <int kSplit>
__device__ __forceinline__ void total_deflection64(const MacroC& mc, double tx, double ty,
                                                   const RangeScratch<kSplit>& scratch, int slot, double sx, double sy,
                                                   double& ax, double& ay) {
  if (kSplit > 1) {
    // one range at a time: this epilogue must not raise the kernel's
    // register count above the pair loop's
#pragma unroll 1
    for (int e = 0; e < kRanges; ++e) {
      const float4 v = scratch.r[e][slot];
      sx += (double)v.x + (double)v.y;
      sy += (double)v.z + (double)v.w;
    }
  }
  macro_deflection64(mc, tx, ty, ax, ay);
  ax += sx;
  ay += sy;
}

}  // namespace jt
