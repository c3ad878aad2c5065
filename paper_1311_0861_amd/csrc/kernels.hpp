// Host-side launch entry points of the GPUPEGAS kernels (one per stage).
#pragma once

#include "common.hpp"

namespace gp {

// ---- Eulerian stage --------------------------------------------------------
template <typename T>
void launch_eulerian(const Fields<T>& in, const Fields<T>& out, const T* phi, const Grid& g,
                     const Phys& ph, const DevScalars* sc, hipStream_t st);

// ---- Lagrangian stage + energy balance + diagnostics partials -------------
// Corner velocities (6 components, (nx+1)(ny+1)(nz+1) vertices each, component
// stride vstride) from the post-Eulerian velocities.
template <typename T>
void launch_vertex(const Fields<T>& eul, T* vtx, size_t vstride, const Grid& g, hipStream_t st);
// cur: rho, n at t^n; eul: post-Eulerian fields (velocities in the momentum
// slots); out: new state (its rho/n pointers must differ from cur's).  Writes
// s = rho + n and one kNP-slot partial row per block.
template <typename T>
void launch_lagrangian(const Fields<T>& cur, const Fields<T>& eul, const Fields<T>& out, const T* vtx,
                       size_t vstride, T* s, const Grid& g, const Phys& ph, const DevScalars* sc,
                       double* partials, hipStream_t st);

// Partials and s = rho + n of a state that has not been advanced (prologue).
template <typename T>
void launch_init_partials(const Fields<T>& cur, T* s, const Grid& g, const Phys& ph,
                          double* partials, hipStream_t st);

// ---- FFT Poisson ---------------------------------------------------------
template <typename T>
struct cplx {
  T x, y;
};

struct FftAxis {
  int L;         // complex transform length on this axis
  int nst;       // number of radix stages
  int rad[16];   // radices, applied first to last
};

template <typename T>
struct FftTables {
  const cplx<T>* tw_x;    // exp(-2 pi i k / Mx), k < Mx = nx / 2
  const cplx<T>* wn_x;    // exp(-2 pi i k / nx), k <= nx / 2 (real-to-complex split)
  const cplx<T>* tw_y;    // exp(-2 pi i k / ny)
  const cplx<T>* tw_z;    // exp(-2 pi i k / nz)
  const double* dx;       // D(k) = 1 - (2/3) sin^2(pi k / n) per axis
  const double* dy;
  const double* dz;
};

struct FftGeom {
  int nx, ny, nz, px;     // px = nx / 2 + 1 (half-spectrum row length)
  FftAxis ax, ay, az;     // ax.L = nx / 2
  int rows_per_block;     // x passes
  int cols_y, cols_z;     // columns per block in the y / z passes
  double green_scale;     // -4 pi G h^2 / 6
  double norm;            // 2 / (nx ny nz)
};

int fft_blocks_z(const FftGeom& f);

template <typename T>
void launch_fft_x_fwd(const T* s, cplx<T>* spec, const FftGeom& f, const FftTables<T>& t, hipStream_t st);
template <typename T>
void launch_fft_y(cplx<T>* spec, const FftGeom& f, const FftTables<T>& t, bool inverse, hipStream_t st);
template <typename T>
void launch_fft_z_green(cplx<T>* spec, const FftGeom& f, const FftTables<T>& t, double* epot_partials,
                        hipStream_t st);
template <typename T>
void launch_fft_x_inv(const cplx<T>* spec, T* phi, const FftGeom& f, const FftTables<T>& t, hipStream_t st);

// ---- reductions / finalize ---------------------------------------------
// Two-level fixed-order reduction of the per-block partials, then the CFL
// step, time advance and diagnostics record.  advanced = 0 for the prologue.
void launch_finalize(const double* partials, int nrows, double* scratch, int nscratch,
                     const double* epot_partials, int nepot, const Grid& g, const Phys& ph,
                     double epot_scale, int advanced, DevScalars* sc, gp_diag* ring, hipStream_t st);

// ---- conversions ---------------------------------------------------------
template <typename D, typename S>
void launch_convert(D* dst, const S* src, size_t n, hipStream_t st);
// dst = density * velocity (post-Eulerian momentum for inspection)
template <typename D, typename T>
void launch_density_times(D* dst, const double* dens, const T* vel, size_t n, hipStream_t st);

}  // namespace gp
