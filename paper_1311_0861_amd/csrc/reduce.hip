// Standalone reduction kernels of one GPUPEGAS step (the arithmetic is in
// reduce.hpp): the first level when no run has gravity (else the Poisson z
// pass carries it), and the finalize for the stage-by-stage path and runs
// without gravity (else the last inverse Poisson pass carries it).
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
__global__ void __launch_bounds__(kRedThreads) k_finalize(FinJob job) {
  __shared__ double lds[kFinLds];
  finalize_run(job, (int)blockIdx.x, lds);
}

void launch_reduce(const RedJob& red, hipStream_t st) {
  k_reduce_rows<<<red.n, kRedThreads, 0, st>>>(red.partials, red.items, red.scratch);
}

void launch_finalize(const FinJob& job, hipStream_t st) { k_finalize<<<job.n, kRedThreads, 0, st>>>(job); }

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
