// Fixed-order reduction of per-tile partial rows (kNP FP64 slots each), shared
// by the standalone reduction kernel and the reduction workgroups that ride
// along in the Poisson z pass.  Sums, maxima (signal speed) and bitwise ors
// (error bits) are combined in one fixed order, so results never depend on
// scheduling.
#pragma once

#include "common.hpp"

namespace gp {

constexpr int kRedThreads = 256;
constexpr int kLanesPerSlot = kRedThreads / kNP;  // lanes per partial slot (the rest idle)

__device__ __forceinline__ double combine(int slot, double a, double b) {
  const int s = slot % kNS;
  if (s == S_SPEED) return fmax(a, b);
  if (s == S_ERR) return (double)((uint32_t)a | (uint32_t)b);
  return a + b;
}

// Rows [r0, r1) of a [row][kNP] table -> one kNP row `out`, by a workgroup of
// kRedThreads threads; `red` is kRedThreads doubles of LDS.  Lane l of slot s
// combines rows r0 + l, r0 + l + kLanesPerSlot, ... in that order (their loads
// issued four at a time), then thread s combines the lanes in order.
__device__ inline void reduce_rows(const double* __restrict__ in, int r0, int r1, double* __restrict__ out,
                                   double* red) {
  constexpr int L = kLanesPerSlot;
  const int slot = threadIdx.x % kNP, lane = threadIdx.x / kNP;
  double v = 0.0;
  if (lane < L) {
    int r = r0 + lane;
    for (; r + 3 * L < r1; r += 4 * L) {
      double x[4];
#pragma unroll
      for (int q = 0; q < 4; q++) x[q] = in[(size_t)(r + q * L) * kNP + slot];
#pragma unroll
      for (int q = 0; q < 4; q++) v = combine(slot, v, x[q]);
    }
    for (; r < r1; r += L) v = combine(slot, v, in[(size_t)r * kNP + slot]);
  }
  red[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < kNP) {
    double a = red[threadIdx.x];
    for (int l = 1; l < L; l++) a = combine(threadIdx.x, a, red[l * kNP + threadIdx.x]);
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

}  // namespace gp
