// End-of-step reductions of one GPUPEGAS step: the CFL step and the
// diagnostics record, from the per-block FP64 partials of the cell kernels and
// the spectral potential-energy partials of the Poisson z pass.
//
// The paper gives no CFL rule; the step is C h / (max over cells and axes of
// the fastest signal speed of either component: |v_d| + sqrt(gamma p / rho) for
// the gas, |u_d| + sqrt(3 Pi_dd / n) for the stars -- the largest eigenvalues of
// the Eulerian systems of Sec. 2.1 and 2.2 shifted by the advection speed).
// Reductions run in a fixed order (strided per-thread sums, then a fixed tree),
// so results do not depend on scheduling.
#include "common.hpp"
#include "kernels.hpp"
#include "reduce.hpp"

namespace gp {

// First level, when no Poisson z pass carries it: workgroup b reduces partial
// rows [src_begin, src_end) into scratch row b.
__global__ void __launch_bounds__(kRedThreads) k_reduce_rows(const double* __restrict__ in,
                                                             const RedItem* __restrict__ items,
                                                             double* __restrict__ out) {
  __shared__ double red[kRedThreads];
  const RedItem it = items[blockIdx.x];
  reduce_rows(in, (int)it.src_begin, (int)it.src_end, out + (size_t)blockIdx.x * kNP, red);
}

// Second level: workgroup r finishes run r.
__global__ void __launch_bounds__(kRedThreads) k_finalize(const double* __restrict__ rows,
                                                          const double* __restrict__ epot,
                                                          const FinDesc* __restrict__ fin, int advanced) {
  __shared__ double tot[kNP];
  __shared__ double red[kRedThreads];
  __shared__ double ered[kRedThreads / 64];
  const FinDesc F = fin[blockIdx.x];
  // the potential-energy partials are summed first (strided per thread, then
  // across each wave and the waves in order), so that their loads overlap
  // the reduction of the scratch rows
  double e = 0.0;
  {
    unsigned b = threadIdx.x;
    for (; b + 3 * kRedThreads < F.nep; b += 4 * kRedThreads) {
      double x[4];
#pragma unroll
      for (int q = 0; q < 4; q++) x[q] = epot[F.eoff + b + q * kRedThreads];
#pragma unroll
      for (int q = 0; q < 4; q++) e += x[q];
    }
    for (; b < F.nep; b += kRedThreads) e += epot[F.eoff + b];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if ((threadIdx.x & 63) == 0) ered[threadIdx.x >> 6] = e;
  reduce_rows(rows, (int)F.soff, (int)(F.soff + F.nscr), tot, red);  // its barriers also order ered[]
  if (threadIdx.x != 0) return;
  double epot_sum = ered[0];
  for (int w = 1; w < kRedThreads / 64; w++) epot_sum += ered[w];
  DevScalars* sc = F.sc;
  const Grid& g = F.g;
  const Phys& ph = F.ph;

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

void launch_reduce(const RedJob& red, hipStream_t st) {
  k_reduce_rows<<<red.n, kRedThreads, 0, st>>>(red.partials, red.items, red.scratch);
}

void launch_finalize(const double* scratch, const double* epot_partials, const FinDesc* fin, int nruns,
                     int advanced, hipStream_t st) {
  k_finalize<<<nruns, kRedThreads, 0, st>>>(scratch, epot_partials, fin, advanced);
}

template <typename D, typename S>
__global__ void k_convert(D* __restrict__ dst, const S* __restrict__ src, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (D)src[i];
}

template <typename D, typename S>
void launch_convert(D* dst, const S* src, size_t n, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  k_convert<D, S><<<(unsigned)blocks, 256, 0, st>>>(dst, src, n);
}

template <typename D, typename T>
__global__ void k_density_times(D* __restrict__ dst, const double* __restrict__ dens, const T* __restrict__ vel,
                                size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (D)((T)dens[i] * vel[i]);
}

template <typename D, typename T>
void launch_density_times(D* dst, const double* dens, const T* vel, size_t n, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  k_density_times<D, T><<<(unsigned)blocks, 256, 0, st>>>(dst, dens, vel, n);
}

template void launch_density_times<double, double>(double*, const double*, const double*, size_t, hipStream_t);
template void launch_density_times<float, double>(float*, const double*, const double*, size_t, hipStream_t);
template void launch_density_times<double, float>(double*, const double*, const float*, size_t, hipStream_t);
template void launch_density_times<float, float>(float*, const double*, const float*, size_t, hipStream_t);

template void launch_convert<double, double>(double*, const double*, size_t, hipStream_t);
template void launch_convert<double, float>(double*, const float*, size_t, hipStream_t);
template void launch_convert<float, double>(float*, const double*, size_t, hipStream_t);
template void launch_convert<float, float>(float*, const float*, size_t, hipStream_t);

}  // namespace gp
