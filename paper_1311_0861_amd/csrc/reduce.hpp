// End-of-step reductions of one GPUPEGAS step, shared by the standalone
// reduction kernels and the workgroups that ride along in the Poisson passes
// (the first level in the z pass, the finalize in the last inverse pass):
//   - partial rows (kNP FP64 slots per tile) -> per-run scratch rows;
//   - per run: scratch rows and the spectral potential-energy partials ->
//     the CFL step, the time advance and one diagnostics record.
// Sums, maxima (signal speed) and bitwise ors (error bits) are combined in one
// fixed order by the first kRedThreads threads of a workgroup, whatever its
// size, so results never depend on scheduling or on which kernel carries them.
//
// The paper gives no CFL rule; the step is C h / (max over cells and axes of
// the fastest signal speed of either component: |v_d| + sqrt(gamma p / rho) for
// the gas, |u_d| + sqrt(3 Pi_dd / n) for the stars -- the largest eigenvalues of
// the Eulerian systems of Sec. 2.1 and 2.2 shifted by the advection speed).
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace gp {

constexpr int kRedThreads = 256;
constexpr int kLanesPerSlot = kRedThreads / kNP;  // lanes per partial slot (the rest idle)
// LDS (doubles) of finalize_run: the lane table, the run's totals and the
// potential-energy sum of each wave
constexpr int kFinLds = kRedThreads + kNP + kRedThreads / 64;

__device__ __forceinline__ double combine(int slot, double a, double b) {
  const int s = slot % kNS;
  if (s == S_SPEED) return fmax(a, b);
  if (s == S_ERR) return (double)((uint32_t)a | (uint32_t)b);
  return a + b;
}

// Rows [r0, r1) of a [row][kNP] table -> one kNP row `out`; `red` is
// kRedThreads doubles of LDS.  Every thread of the workgroup must call it.
// Lane l of slot s combines rows r0 + l, r0 + l + kLanesPerSlot, ... in that
// order (their loads issued four at a time), then thread s combines the lanes
// in order.
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
  if (threadIdx.x < kRedThreads) red[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < kNP) {
    double a = red[threadIdx.x];
    for (int l = 1; l < L; l++) a = combine(threadIdx.x, a, red[l * kNP + threadIdx.x]);
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

// Finishes run r of a finalize job; `lds` is kFinLds doubles.  Every thread of
// the workgroup (at least kRedThreads) must call it.
__device__ inline void finalize_run(const FinJob& job, int r, double* lds) {
  double* red = lds;
  double* tot = lds + kRedThreads;
  double* ered = tot + kNP;
  const FinDesc F = job.fin[r];
  // the potential-energy partials are summed first (strided per thread, four
  // loads in flight, then across each wave and the waves in order), so that
  // their loads overlap the reduction of the scratch rows
  double e = 0.0;
  if (threadIdx.x < kRedThreads) {
    unsigned b = threadIdx.x;
    for (; b + 3 * kRedThreads < F.nep; b += 4 * kRedThreads) {
      double x[4];
#pragma unroll
      for (int q = 0; q < 4; q++) x[q] = job.epot[F.eoff + b + q * kRedThreads];
#pragma unroll
      for (int q = 0; q < 4; q++) e += x[q];
    }
    for (; b < F.nep; b += kRedThreads) e += job.epot[F.eoff + b];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if ((threadIdx.x & 63) == 0 && threadIdx.x < kRedThreads) ered[threadIdx.x >> 6] = e;
  reduce_rows(job.scratch, (int)F.soff, (int)(F.soff + F.nscr), tot, red);  // its barriers also order ered[]
  if (threadIdx.x != 0) return;
  double epot_sum = ered[0];
  for (int w = 1; w < kRedThreads / 64; w++) epot_sum += ered[w];
  DevScalars* sc = F.sc;
  const Grid& g = F.g;
  const Phys& ph = F.ph;
  const int advanced = job.advanced;

  const double h = g.h, h3 = h * h * h;
  constexpr int G = kGasSlots, B = kBmeSlots;
  const double speed = fmax(tot[G + S_SPEED], tot[B + S_SPEED]);
  if (advanced) {
    sc->outflow_gas += sc->dt * h * h * tot[G + S_OUTFLOW];
    sc->outflow_bme += sc->dt * h * h * tot[B + S_OUTFLOW];
    sc->t += sc->dt;
    sc->step += 1;
  }
  uint32_t err = (uint32_t)tot[G + S_ERR] | (uint32_t)tot[B + S_ERR];
  double dt;
  if (ph.fixed_dt > 0.0) {
    dt = ph.fixed_dt;
  } else if (speed > 0.0) {
    dt = ph.cfl * h / speed;
  } else {
    dt = 0.0;
    err |= ERR_NOSPEED;
  }
  if (ph.t_end > 0.0) dt = fmin(dt, fmax(ph.t_end - sc->t, 0.0));
  sc->dt = dt;
  sc->err |= err;

  gp_diag d;
  d.step = sc->step;
  d.t = sc->t;
  d.dt = dt;
  d.mass_gas = h3 * tot[G + S_MASS];
  d.mass_bme = h3 * tot[B + S_MASS];
  for (int a = 0; a < 3; a++) d.mom[a] = h3 * (tot[G + S_MOMX + a] + tot[B + S_MOMX + a]);
  d.e_gas = h3 * tot[G + S_ENERGY];
  d.e_bme = h3 * tot[B + S_ENERGY];
  d.e_pot = 0.5 * h3 * F.epot_scale * epot_sum;
  d.kappa_gas = h3 * tot[G + S_KAPPA];
  d.kappa_bme = h3 * tot[B + S_KAPPA];
  d.outflow_gas = sc->outflow_gas;
  d.outflow_bme = sc->outflow_bme;
  d.n_sync_gas = advanced ? tot[G + S_NSYNC] : 0.0;
  d.n_sync_bme = advanced ? tot[B + S_NSYNC] : 0.0;
  d.err = sc->err;
  d.pad = 0u;
  F.ring[sc->ndiag % kDiagCap] = d;
  sc->ndiag += 1;
}

}  // namespace gp
