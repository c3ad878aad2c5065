// Host-side launch entry points of the GPUPEGAS kernels (one per stage).
#pragma once

#include "common.hpp"

namespace gp {

// All per-cell stages are persistent launches of `nblocks` workgroups over a
// (run, tile column) work list made for tile shape `shape` (0: 64 x 4,
// 1: 32 x 8; see TileShape); runs[] are the device descriptors of the batch.

// ---- Eulerian stage (comp = COMP_GAS or COMP_BME) --------------------------
template <typename T>
void launch_eulerian(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity, int comp,
                     bool cool, int shape, unsigned nblocks, hipStream_t st);

// ---- Lagrangian stage + energy balance + diagnostics partials -------------
// New state of component comp into cur / dens[parity ^ 1], and that
// component's kNS slots of the partial row of each tile (row R.row0 + tile).
template <typename T>
void launch_lagrangian(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity, double* partials,
                       int comp, int shape, unsigned nblocks, hipStream_t st);
// One component's partial rows of a state that has not been advanced
// (prologue), over that component's Lagrangian work list.
template <typename T>
void launch_init_partials(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity,
                          double* partials, int comp, int shape, unsigned nblocks, hipStream_t st);

// ---- FFT Poisson ---------------------------------------------------------
// Aligned to its size, so that a value moves in one 16-byte (FP64) or 8-byte
// (FP32) access: with lanes on neighbouring LDS lines of odd pitch that keeps
// every access free of bank conflicts, where two 8-byte halves would not be.
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
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
  const cplx<T>* tw_yh;   // exp(-2 pi i k / (ny / 2)) (half-length y transforms of the plane passes)
  const cplx<T>* tw_z;    // exp(-2 pi i k / nz)
  const double* dx;       // D(k) = 1 - (2/3) sin^2(pi k / n) per axis
  const double* dy;
  const double* dz;
};

struct FftGeom {
  int nx, ny, nz, px;     // px = nx / 2 + 1 (half-spectrum row length)
  int nruns;              // runs of this size stored back to back
  FftAxis ax, ay, az;     // ax.L = nx / 2
  int plane;              // 1: x and y transforms per half z plane in LDS
  FftAxis ayh;            // ayh.L = ny / 2 (plane passes)
  int hp;                 // row pitch of a half plane in LDS (complex values, odd, >= nx/2 + 1)
  int rows_per_block;     // x passes
  int cols_y, cols_z;     // columns per block in the y / z passes
  double green_scale;     // -4 pi G h^2 / 6
  double norm;            // 2 / (nx ny nz)
};

// Radix plan (8s, then 4, 2, 3) of a complex transform of length L = 2^a 3^b.
FftAxis make_axis(int L);
// Geometry of the periodic solve for nruns runs of nx*ny*nz in precision prec
// (GP_FP64 / GP_FP32): line and column blocking, and the per-half-plane x and
// y transforms where planes is set and two such workgroups fit on a CU (this
// also raises the plane kernels' dynamic-LDS limit).  green_scale is left 0.
FftGeom make_fft_geom(int nx, int ny, int nz, int nruns, int prec, bool planes);

// Potential-energy partials the z pass writes: one per (spectrum row, column
// chunk), contiguous per run.
int fft_blocks_z(const FftGeom& f);

// LDS a workgroup of the plane passes may take (gfx950).
constexpr int kPlaneLdsMax = 160 * 1024;
size_t plane_lds_bytes(const FftGeom& f, size_t csz);
// Raises the dynamic-LDS limit of the plane kernels to `bytes`.
template <typename T>
hipError_t fft_plane_prepare(int bytes);

// First level of the reduction of the per-tile partial rows (kNP FP64 slots
// each): workgroup b reduces partial rows items[b] into scratch row b.  It
// rides along in the first Poisson z pass of a step, or runs on its own when
// no run has gravity.
struct RedItem {
  unsigned src_begin, src_end;  // partial rows reduced into one scratch row
};
struct RedJob {
  const double* partials;
  const RedItem* items;
  double* scratch;
  int n;  // workgroups; 0 = none
};
// Second level and the end of the step: workgroup r finishes run r -- the
// CFL step, time advance and diagnostics record (advanced = 1 after a step,
// 0 for the initial state).  It rides along in the last inverse Poisson pass
// of a step, or runs on its own.
struct FinDesc {
  Grid g;
  Phys ph;
  unsigned soff, nscr;  // scratch rows of the run
  unsigned eoff, nep;   // potential-energy partials of the run
  double epot_scale;    // 1 / (nx ny nz)
  DevScalars* sc;
  gp_diag* ring;
};
struct FinJob {
  const double* scratch;
  const double* epot;
  const FinDesc* fin;
  int n;  // runs (workgroups); 0 = none
  int advanced;
};

// Poisson source of each run of a size class: s = rho + n, formed in FP64
// from the current densities (slot = run position in the class).
struct SrcSlot {
  const double* rho[2];  // by buffer parity
  const double* nb[2];
};
template <typename T>
void launch_fft_x_fwd(const SrcSlot* src, int parity, cplx<T>* spec, const FftGeom& f, const FftTables<T>& t,
                      hipStream_t st);
template <typename T>
void launch_fft_y(cplx<T>* spec, const FftGeom& f, const FftTables<T>& t, bool inverse, hipStream_t st);
// ky_major: the spectrum is stored C[run][ky][z][kx] (as the plane passes
// write it) rather than C[run][z][ky][kx].  The first red.n workgroups of the
// launch run the reduction job instead.
template <typename T>
void launch_fft_z_green(cplx<T>* spec, const FftGeom& f, const FftTables<T>& t, double* epot_partials,
                        bool ky_major, const RedJob& red, hipStream_t st);
template <typename T>
void launch_fft_xy_fwd(const SrcSlot* src, int parity, cplx<T>* spec, const FftGeom& f, const FftTables<T>& t,
                       hipStream_t st);
template <typename T>
void launch_fft_xy_inv(const cplx<T>* spec, T* phi, const FftGeom& f, const FftTables<T>& t, const FinJob& fin,
                       hipStream_t st);
template <typename T>
void launch_fft_x_inv(const cplx<T>* spec, T* phi, const FftGeom& f, const FftTables<T>& t, const FinJob& fin,
                      hipStream_t st);

// ---- isolated-boundary Poisson (zero padding to 2n on each axis) ----------
// Geometry of one size class: the source occupies the first nx, ny, nz cells
// of each padded axis; the spectrum of a run is C[z][y][kx], rows of px bins,
// py rows per plane, nz + 2 planes (the z pass keeps nz + 2 of its 2nz
// outputs, the y inverse ny + 2 of its 2ny).
struct IsoGeom {
  int nx, ny, nz;       // grid
  int px;               // nx + 1: bins of a padded row (real length 2 nx)
  int py, pz;           // 2 ny, 2 nz
  int nruns;            // runs of this size stored back to back
  FftAxis ax, ay, az;   // complex lengths nx (packed pairs of a padded row), 2 ny, 2 nz
  int rows_per_block;   // x passes
  int cols_y, cols_z;   // columns per workgroup of the column passes
  size_t run_stride;    // spectrum values per run
  size_t ext_cells;     // (nx + 2)(ny + 2)(nz + 2): potential on the grid and its ring
  double norm;          // 2 / (8 nx ny nz): inverse normalisation of the packed real transforms
};
template <typename T>
struct IsoTables {
  const cplx<T>* tw_x;  // exp(-2 pi i k / nx), k < nx
  const cplx<T>* wn_x;  // exp(-2 pi i k / (2 nx)), k <= nx
  const cplx<T>* tw_y;  // exp(-2 pi i k / (2 ny))
  const cplx<T>* tw_z;  // exp(-2 pi i k / (2 nz))
  const double* green;  // DFT of the sampled Green function at kx <= nx, ky <= ny,
                        // kz <= nz: (nz + 1)(ny + 1) rows of px values
};
// Potential-energy partials of the isolated z pass (one per ky line and
// column chunk), contiguous per run.
int iso_blocks_z(const IsoGeom& f);
// One step's passes.  x and y forward: s = rho + n of every run of the class
// -> its zero-padded spectrum.  z: forward, times the Green spectrum, inverse,
// potential-energy partials (the first red.n workgroups run the reduction job
// instead).  y and x inverse: -> the potential on the grid and its one-cell
// ring, (nx + 2)(ny + 2)(nz + 2) values per run, cell i at index i + 1 on each
// axis (the first fin.n workgroups of the x pass finish the step instead).
template <typename T>
void launch_iso_fwd(const SrcSlot* src, int parity, cplx<T>* spec, const IsoGeom& f, const IsoTables<T>& t,
                    hipStream_t st);
template <typename T>
void launch_iso_z(cplx<T>* spec, const IsoGeom& f, const IsoTables<T>& t, double* epot_partials, const RedJob& red,
                  hipStream_t st);
template <typename T>
void launch_iso_inv(cplx<T>* spec, T* phi_ext, const IsoGeom& f, const IsoTables<T>& t, const FinJob& fin,
                    hipStream_t st);
// The Green spectrum of a class (FP64): samples g on the padded lattice into
// `work` (pz planes of py rows of px values), transforms it along x, y and z,
// and keeps the real part at kx <= nx, ky <= ny, kz <= nz in t.green.  f is
// the class geometry laid out for FP64 with nruns = 1.
void launch_iso_green(cplx<double>* work, const IsoGeom& f, const IsoTables<double>& t, double* green, double h,
                      double G, hipStream_t st);
// dst = the grid part of a potential stored with its ring (nx ny nz values)
template <typename D, typename S>
void launch_phi_interior(D* dst, const S* ext, int nx, int ny, int nz, hipStream_t st);

// ---- reductions / finalize ---------------------------------------------
void launch_reduce(const RedJob& red, hipStream_t st);
void launch_finalize(const FinJob& job, hipStream_t st);

// ---- conversions ---------------------------------------------------------
template <typename D, typename S>
void launch_convert(D* dst, const S* src, size_t n, hipStream_t st);
// dst = density * velocity (post-Eulerian momentum for inspection)
template <typename D, typename T>
void launch_density_times(D* dst, const double* dens, const T* vel, size_t n, hipStream_t st);

}  // namespace gp
