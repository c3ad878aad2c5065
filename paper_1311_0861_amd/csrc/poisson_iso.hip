// Poisson solve with isolated boundaries: the free-space potential of the
// cell masses by zero padding (the method of Hockney and Eastwood, which
// Sec. 1 of Kulikov, arXiv:1311.0861, cites among the Poisson solvers of other
// codes), in place of the periodic 27-point solve of Sec. 2.3:
//   Phi(x_i) = sum_j g(x_i - x_j) s_j,  s = rho + n,
//   g(d) = -G h^2 / |d|  for a displacement of d != 0 cells,
//   g(0) = -G h^2 c0,    c0 = 6 ln((1 + sqrt 3) / sqrt 2) - pi / 2,
// c0 h^2 being the integral of 1 / |x| over a cube of side h about its centre
// (a cell's own mass spread uniformly over the cell).  s is padded with zeros
// to (2nx, 2ny, 2nz) and g is sampled on that lattice at the minimum-image
// displacement (|d_a| <= n_a on each axis).  The cyclic convolution of the
// two, a product of their DFTs, then equals the free-space sum at every cell
// whose displacement to every source cell is at most n_a on each axis: the
// grid and its one-cell ring (cells -1 .. n_a), which the gravity of the
// outermost cells reads.
//
// g is even on each axis, so its DFT is real and even: it is computed once per
// size class on the GPU in FP64 (the passes below, run on the sampled g) and
// stored for kx <= nx, ky <= ny, kz <= nz.  Each step runs
//   x forward : rows y < ny, z < nz of s padded to length 2nx, as nx packed
//               (even, odd) pairs of which the last nx/2 are zero -> a
//               half-length complex FFT and the split to nx + 1 bins;
//   y forward : columns of length 2ny whose lines y >= ny are zero (not read);
//   z         : columns of length 2nz whose lines z >= nz are zero: forward,
//               times the Green spectrum and the inverse normalisation (the
//               potential energy sum G^ |s^|^2 on the way), inverse; only the
//               outputs at z = 0 .. nz and 2nz - 1 (that is, -1) are stored;
//   y inverse : those nz + 2 planes; outputs at y = 0 .. ny and -1;
//   x inverse : those rows; the real outputs at x = -1, 0 .. nx, stored as the
//               potential on the grid and its ring.
// Every pass works in place on lines its own workgroup loaded whole.
#include <algorithm>
#include <cmath>

#include "fft_core.hpp"
#include "reduce.hpp"

namespace gp {

// Compile-time shape of a cubic N^3 grid (N = 0: every size from IsoGeom at
// run time).  With N > 0 the kernels below derive every index from constants;
// the host launches such an instance only for a geometry that matches it
// (iso_fixed), and the arithmetic is the same, hence the same bits.
template <typename T, int N>
struct IsoShape {
  static constexpr int M = N;                                            // packed pairs of a padded row
  static constexpr int RB = N ? std::max(1, max_points<T>() / (2 * N)) : 0;  // rows per x block
  static constexpr int L = 2 * N;                                        // padded column length
  static constexpr int CB = N ? 8 : 0;                                   // columns per column block
};

// ---- x forward -----------------------------------------------------------
// GREEN = false: rows y < ny, z < nz of s (run after run), the padded half of
// each row zero.  GREEN = true: every row of the padded lattice (py pz of one
// run), the sampled Green function g; gscale = -G h^2, g0 = g(0).
template <typename T, bool GREEN, int N = 0>
__global__ void __launch_bounds__(kFftThreads) k_iso_x_fwd(const SrcSlot* __restrict__ src, int parity,
                                                           cplx<T>* __restrict__ spec, IsoGeom f, IsoTables<T> t,
                                                           double gscale, double g0) {
  static_assert(N == 0 || !GREEN, "compile-time shapes are for the source rows");
  using S = IsoShape<T, N>;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  // grid and padded sizes: constants for a compile-time shape
  const int nx = N ? N : f.nx, ny = N ? N : f.ny, nz = N ? N : f.nz;
  const int px = N ? N + 1 : f.px, py = N ? 2 * N : f.py, pz = N ? 2 * N : f.pz;
  const int M = N ? S::M : f.ax.L, xp = M | 1;  // M = nx packed pairs per padded row; odd pitch
  const int nload = GREEN ? M : M / 2;          // pairs that carry data
  const int RB = N ? S::RB : f.rows_per_block;
  cplx<T>* tw = lds + RB * xp;
  cplx<T>* wn = tw + M;
  const int ry = GREEN ? py : ny;  // rows per plane
  const int rows_run = ry * (GREEN ? pz : nz);
  const int nrows = rows_run * f.nruns;
  const int row0 = blockIdx.x * RB;
  const int rows = min(RB, nrows - row0);
  load_twiddles<kFftThreads>(tw, t.tw_x, M);
  load_twiddles<kFftThreads>(wn, t.wn_x, M + 1);
  const CDiv<N ? S::M / 2 : 0> dl(nload);
  const CDiv<N ? S::M + 1 : 0> dm1(M + 1);
  staged_copy<kFftThreads, 4, cplx<T>>(
      rows * nload,
      [&](int q) {
        const int rq = (int)dl.div(q);
        const int row = row0 + rq, m = q - rq * nload;
        if constexpr (GREEN) {
          // one run: row = y + py z
          const int z = row / ry, y = row - z * ry;
          const double dy = y <= ny ? y : y - py, dz = z <= nz ? z : z - pz;
          double v[2];
#pragma unroll
          for (int u = 0; u < 2; u++) {
            const int x = 2 * m + u;
            const double dx = x <= nx ? x : x - 2 * nx;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            v[u] = r == 0.0 ? g0 : gscale / r;
          }
          return cplx<T>{(T)v[0], (T)v[1]};
        } else {
          const int slot = row / rows_run;  // may exceed the range of FastDiv
          const size_t c = (size_t)(row - slot * rows_run) * nx + 2 * m;
          const SrcSlot& S = src[slot];
          const dpair a = gload(reinterpret_cast<const dpair*>(S.rho[parity] + c));
          const dpair b = gload(reinterpret_cast<const dpair*>(S.nb[parity] + c));
          return cplx<T>{(T)(a.x + b.x), (T)(a.y + b.y)};
        }
      },
      [&](int q, cplx<T> v) {
        const int rq = (int)dl.div(q);
        lds[rq * xp + q - rq * nload] = v;
      });
  if constexpr (!GREEN) {
    // the padded half of each row
    for (int q = threadIdx.x; q < rows * nload; q += kFftThreads) {
      const int rq = (int)dl.div(q);
      lds[rq * xp + nload + q - rq * nload] = cplx<T>{T(0), T(0)};
    }
  }
  __syncthreads();
  x_rows_fft<T, S::M, S::RB, false>(lds, rows, xp, f.ax, tw);
  // even/odd split into nx + 1 bins; spectrum row y + py z of the run
  for (int q = threadIdx.x; q < rows * (M + 1); q += kFftThreads) {
    const int rq = (int)dm1.div(q), k = q - rq * (M + 1);
    const int row = row0 + rq;
    const int slot = row / rows_run, rr = row - slot * rows_run;
    const int z = rr / ry, y = rr - z * ry;
    const cplx<T> zk = lds[rq * xp + (k == M ? 0 : k)];
    const cplx<T> zc = lds[rq * xp + (k == 0 ? 0 : M - k)];
    spec[(size_t)slot * f.run_stride + ((size_t)z * py + y) * px + k] = split_fwd(zk, zc, wn[k]);
  }
}

// ---- column passes ---------------------------------------------------------
// A workgroup takes cb consecutive kx columns of one outer line (a z plane in
// the y passes, a ky row in the z pass) of one run; line j of column c lives
// at base + j * stride + c.  Lines j >= nin are zero and not read.  After the
// transform(s) lines 0 .. nout - 2 and L - 1 are stored at positions
// 0 .. nout - 1 (every line when nout == L), which keeps the outputs at
// 0 .. n and -1 of a padded axis.
// MODE 0: forward, 1: inverse, 2: forward * Green spectrum * inverse (z pass,
// whose first red.n workgroups reduce partial rows instead).
// Column transform of a column block: the compile-time one for N > 0.
template <typename T, int N, bool INV>
__device__ __forceinline__ void iso_col_fft(cplx<T>* lds, int cb, const FftAxis& ax, const cplx<T>* tw) {
  using S = IsoShape<T, N>;
  if constexpr (N > 0)
    cfft<T, S::L, S::CB, 1, S::CB, kFftThreads, INV>(lds, tw);
  else
    col_fft(lds, cb, ax, tw, INV);
}

template <typename T, int MODE, int N = 0>
__global__ void __launch_bounds__(kFftThreads) k_iso_col(cplx<T>* __restrict__ spec, IsoGeom f, IsoTables<T> t,
                                                         FftAxis ax, const cplx<T>* __restrict__ twg, int cb_rt,
                                                         size_t stride, size_t outer_stride, int outer_div, int nin,
                                                         int nout, double* __restrict__ epot_partials, RedJob red) {
  using S = IsoShape<T, N>;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  // grid and padded sizes: constants for a compile-time shape
  const int nx = N ? N : f.nx, ny = N ? N : f.ny, nz = N ? N : f.nz;
  const int px = N ? N + 1 : f.px, py = N ? 2 * N : f.py, pz = N ? 2 * N : f.pz;
  const int cb = N ? S::CB : cb_rt;
  int bid = (int)blockIdx.x, nblk = (int)gridDim.x;
  if constexpr (MODE == 2) {
    if (bid < red.n) {
      const RedItem it = red.items[bid];
      reduce_rows(red.partials, (int)it.src_begin, (int)it.src_end, red.scratch + (size_t)bid * kNP,
                  reinterpret_cast<double*>(smem_raw));
      return;
    }
    bid -= red.n;
    nblk -= red.n;
  }
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);  // L rows of cb columns
  const int L = N ? S::L : ax.L;
  cplx<T>* tw = lds + cb * L;
  const int nchunks = (px + cb - 1) / cb;
  const ColBlock cbk = col_block(bid, nchunks, nblk / nchunks);
  const int chunk = cbk.chunk, oline = cbk.oline;
  const int run = oline / outer_div, outer = oline - run * outer_div;
  const int kx0 = chunk * cb;
  const int ncols = min(cb, px - kx0);
  load_twiddles<kFftThreads>(tw, twg, L);
  const CDiv<S::CB> dcb(cb);
  cplx<T>* base = spec + (size_t)run * f.run_stride + (size_t)outer * outer_stride + kx0;
  staged_copy<kFftThreads, 4, cplx<T>>(
      cb * nin,
      [&](int q) {
        const int j = (int)dcb.div(q), c = q - j * cb;
        const cplx<T> v = gload(base + (size_t)j * stride + min(c, ncols - 1));
        return (c < ncols) ? v : cplx<T>{T(0), T(0)};
      },
      [&](int q, cplx<T> v) { lds[q] = v; });
  for (int q = cb * nin + (int)threadIdx.x; q < cb * L; q += kFftThreads) lds[q] = cplx<T>{T(0), T(0)};
  __syncthreads();
  iso_col_fft<T, N, MODE == 1>(lds, cb, ax, tw);
  if constexpr (MODE == 2) {
    // line position = kz, outer = ky; the Green spectrum is even in ky and kz
    __shared__ double red_ep[kFftThreads / 64];
    const int kyr = min(outer, py - outer);
    const double* grow = t.green + (size_t)kyr * px + kx0;
    const size_t gplane = (size_t)(ny + 1) * px;
    double ep = 0.0;
    for (int q = threadIdx.x; q < cb * L; q += kFftThreads) {
      const int kz = (int)dcb.div(q), c = q - kz * cb;
      if (c >= ncols) continue;
      const int kx = kx0 + c, kzr = min(kz, pz - kz);
      const double gk = gload(grow + (size_t)kzr * gplane + c);
      const double w = (kx == 0 || kx == nx) ? 1.0 : 2.0;  // Hermitian half spectrum of the padded x axis
      cplx<T>& v = lds[q];
      ep += w * gk * ((double)v.x * (double)v.x + (double)v.y * (double)v.y);
      const T gs = (T)(gk * f.norm);
      v.x *= gs;
      v.y *= gs;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ep += __shfl_xor(ep, off, 64);
    if ((threadIdx.x & 63) == 0) red_ep[threadIdx.x >> 6] = ep;
    __syncthreads();  // also orders the scaled values before the inverse transform
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < kFftThreads / 64; w++) s += red_ep[w];
      epot_partials[(size_t)oline * nchunks + chunk] = s;
    }
    iso_col_fft<T, N, true>(lds, cb, ax, tw);
  }
  for (int q = threadIdx.x; q < cb * nout; q += kFftThreads) {
    const int j = (int)dcb.div(q), c = q - j * cb;
    if (c >= ncols) continue;
    const int from = (nout == L || j < nout - 1) ? j : L - 1;
    base[(size_t)j * stride + c] = lds[from * cb + c];
  }
}

// ---- x inverse: rows of the kept planes -> potential with its ring ---------
// The first fin.n workgroups finish the step instead (one per run).
template <typename T, int N = 0>
__global__ void __launch_bounds__(kFftThreads) k_iso_x_inv(const cplx<T>* __restrict__ spec, T* __restrict__ phi,
                                                           IsoGeom f, IsoTables<T> t, FinJob fin) {
  using S = IsoShape<T, N>;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  if ((int)blockIdx.x < fin.n) {
    finalize_run(fin, (int)blockIdx.x, reinterpret_cast<double*>(smem_raw));
    return;
  }
  // grid and padded sizes: constants for a compile-time shape
  const int nx = N ? N : f.nx, ny = N ? N : f.ny, nz = N ? N : f.nz;
  const int px = N ? N + 1 : f.px, py = N ? 2 * N : f.py, pz = N ? 2 * N : f.pz;
  const int bid = (int)blockIdx.x - fin.n;
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int M = N ? S::M : f.ax.L, xp = M | 1;
  const int RB = N ? S::RB : f.rows_per_block;
  cplx<T>* xin = lds + RB * xp;  // RB rows of M + 1 bins
  cplx<T>* tw = xin + RB * (M + 1);
  cplx<T>* wn = tw + M;
  const int ex = nx + 2, ey = ny + 2, ez = nz + 2;
  const int rows_run = ey * ez;
  const int nrows = rows_run * f.nruns;
  const int row0 = bid * RB;
  const int rows = min(RB, nrows - row0);
  load_twiddles<kFftThreads>(tw, t.tw_x, M);
  load_twiddles<kFftThreads>(wn, t.wn_x, M + 1);
  const CDiv<S::M> dm(M);
  const CDiv<N ? S::M + 1 : 0> dm1(M + 1);
  const CDiv<N ? N + 2 : 0> dex(ex);
  // kept row yo of kept plane zo sits at spectrum row yo + py zo
  staged_copy<kFftThreads, 4, cplx<T>>(
      rows * (M + 1),
      [&](int q) {
        const int rq = (int)dm1.div(q), k = q - rq * (M + 1);
        const int row = row0 + rq;
        const int slot = row / rows_run, rr = row - slot * rows_run;
        const int zo = rr / ey, yo = rr - zo * ey;
        return gload(spec + (size_t)slot * f.run_stride + ((size_t)zo * py + yo) * px + k);
      },
      [&](int q, cplx<T> v) { xin[q] = v; });
  __syncthreads();
  for (int q = threadIdx.x; q < rows * M; q += kFftThreads) {
    const int rr = (int)dm.div(q), k = q - rr * M;
    lds[rr * xp + k] = split_inv(xin[rr * (M + 1) + k], xin[rr * (M + 1) + M - k], wn[k]);
  }
  __syncthreads();
  x_rows_fft<T, S::M, S::RB, true>(lds, rows, xp, f.ax, tw);
  // real value at position p of the padded row is component p & 1 of pair
  // p / 2; ring position 0 holds p = 2nx - 1, positions 1 .. nx + 1 hold p = 0 .. nx
  for (int q = threadIdx.x; q < rows * ex; q += kFftThreads) {
    const int rq = (int)dex.div(q), xo = q - rq * ex;
    const int row = row0 + rq;
    const int slot = row / rows_run, rr = row - slot * rows_run;
    const int zo = rr / ey, yo = rr - zo * ey;
    const int p = xo == 0 ? 2 * nx - 1 : xo - 1;
    const cplx<T> v = lds[rq * xp + (p >> 1)];
    const int zi = zo == nz + 1 ? 0 : zo + 1, yi = yo == ny + 1 ? 0 : yo + 1;
    phi[(size_t)slot * f.ext_cells + ((size_t)zi * ey + yi) * ex + xo] = (p & 1) ? v.y : v.x;
  }
}

__global__ void k_iso_green_extract(const cplx<double>* __restrict__ work, double* __restrict__ green, IsoGeom f) {
  const size_t n = (size_t)f.px * (f.ny + 1) * (f.nz + 1);
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const size_t kx = q % f.px, r = q / f.px;
    const size_t ky = r % (f.ny + 1), kz = r / (f.ny + 1);
    green[q] = work[(kz * f.py + ky) * f.px + kx].x;
  }
}

template <typename D, typename S>
__global__ void k_phi_interior(D* __restrict__ dst, const S* __restrict__ ext, int nx, int ny, int nz) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const size_t i = q % nx, r = q / nx;
    const size_t j = r % ny, k = r / ny;
    dst[q] = (D)ext[((k + 1) * (ny + 2) + (j + 1)) * (nx + 2) + (i + 1)];
  }
}

// ---- host launchers -----------------------------------------------------------
namespace {

size_t x_lds(const IsoGeom& f, size_t csz, bool inv) {
  const size_t M = f.ax.L, RB = f.rows_per_block;
  return csz * (RB * (M | 1) + (inv ? RB * (M + 1) : 0) + M + M + 1);
}

size_t col_lds(int cb, int L, size_t csz) { return csz * ((size_t)cb * L + L); }

// Grid size N of the compile-time kernels f runs on (the 128^3 runs of the
// benchmark), or 0: cubic, blocks of 8 columns, full x blocks of the
// compile-time row count.
template <typename T>
int iso_fixed(const IsoGeom& f) {
  constexpr int N = 128;
  if (f.nx == N && f.ny == N && f.nz == N && f.cols_y == IsoShape<T, N>::CB && f.cols_z == IsoShape<T, N>::CB &&
      f.rows_per_block == IsoShape<T, N>::RB)
    return N;
  return 0;
}

// column pass over `nouter` outer lines per run
template <typename T, int MODE>
void col_pass(cplx<T>* spec, const IsoGeom& f, const IsoTables<T>& t, const FftAxis& ax, const cplx<T>* tw, int cb,
              size_t stride, size_t outer_stride, int nouter, int nruns, int nin, int nout, double* epot,
              const RedJob& red, hipStream_t st, int fixed) {
  const int nchunks = (f.px + cb - 1) / cb;
  const int nblk = nchunks * nouter * nruns + (MODE == 2 ? red.n : 0);
  size_t lds = col_lds(cb, ax.L, sizeof(cplx<T>));
  if (MODE == 2 && red.n > 0) lds = std::max(lds, sizeof(double) * kRedThreads);
  if (fixed == 128)
    k_iso_col<T, MODE, 128><<<nblk, kFftThreads, lds, st>>>(spec, f, t, ax, tw, cb, stride, outer_stride, nouter,
                                                            nin, nout, epot, red);
  else
    k_iso_col<T, MODE><<<nblk, kFftThreads, lds, st>>>(spec, f, t, ax, tw, cb, stride, outer_stride, nouter, nin,
                                                       nout, epot, red);
}

}  // namespace

int iso_blocks_z(const IsoGeom& f) { return ((f.px + f.cols_z - 1) / f.cols_z) * f.py * f.nruns; }

template <typename T>
void launch_iso_fwd(const SrcSlot* src, int parity, cplx<T>* spec, const IsoGeom& f, const IsoTables<T>& t,
                    hipStream_t st) {
  const int nrows = f.ny * f.nz * f.nruns;
  const int nblk = (nrows + f.rows_per_block - 1) / f.rows_per_block;
  const int fixed = iso_fixed<T>(f);
  const size_t xl = x_lds(f, sizeof(cplx<T>), false);
  if (fixed == 128)
    k_iso_x_fwd<T, false, 128><<<nblk, kFftThreads, xl, st>>>(src, parity, spec, f, t, 0.0, 0.0);
  else
    k_iso_x_fwd<T, false><<<nblk, kFftThreads, xl, st>>>(src, parity, spec, f, t, 0.0, 0.0);
  // y: planes z < nz, lines y < ny read, all 2ny stored
  const size_t row = f.px, plane = (size_t)f.px * f.py;
  col_pass<T, 0>(spec, f, t, f.ay, t.tw_y, f.cols_y, row, plane, f.nz, f.nruns, f.ny, f.py, nullptr, RedJob{}, st,
                 fixed);
}

template <typename T>
void launch_iso_z(cplx<T>* spec, const IsoGeom& f, const IsoTables<T>& t, double* epot_partials, const RedJob& red,
                  hipStream_t st) {
  // lines z < nz read; z = 0 .. nz and 2nz - 1 stored
  const size_t row = f.px, plane = (size_t)f.px * f.py;
  col_pass<T, 2>(spec, f, t, f.az, t.tw_z, f.cols_z, plane, row, f.py, f.nruns, f.nz, f.nz + 2, epot_partials, red,
                 st, iso_fixed<T>(f));
}

template <typename T>
void launch_iso_inv(cplx<T>* spec, T* phi_ext, const IsoGeom& f, const IsoTables<T>& t, const FinJob& fin,
                    hipStream_t st) {
  const size_t row = f.px, plane = (size_t)f.px * f.py;
  // y: the nz + 2 kept planes, all 2ny lines read, y = 0 .. ny and 2ny - 1 stored
  const int fixed = iso_fixed<T>(f);
  col_pass<T, 1>(spec, f, t, f.ay, t.tw_y, f.cols_y, row, plane, f.nz + 2, f.nruns, f.py, f.ny + 2, nullptr,
                 RedJob{}, st, fixed);
  const int nrows = (f.ny + 2) * (f.nz + 2) * f.nruns;
  const int nblk = (nrows + f.rows_per_block - 1) / f.rows_per_block + fin.n;
  size_t lds = x_lds(f, sizeof(cplx<T>), true);
  if (fin.n > 0) lds = std::max(lds, sizeof(double) * kFinLds);
  if (fixed == 128)
    k_iso_x_inv<T, 128><<<nblk, kFftThreads, lds, st>>>(spec, phi_ext, f, t, fin);
  else
    k_iso_x_inv<T><<<nblk, kFftThreads, lds, st>>>(spec, phi_ext, f, t, fin);
}

void launch_iso_green(cplx<double>* work, const IsoGeom& f, const IsoTables<double>& t, double* green, double h,
                      double G, hipStream_t st) {
  const double c0 = 6.0 * std::log((1.0 + std::sqrt(3.0)) / std::sqrt(2.0)) - M_PI / 2.0;
  const double gscale = -G * h * h;
  const int nrows = f.py * f.pz;
  const int nblk = (nrows + f.rows_per_block - 1) / f.rows_per_block;
  k_iso_x_fwd<double, true><<<nblk, kFftThreads, x_lds(f, sizeof(cplx<double>), false), st>>>(
      nullptr, 0, work, f, t, gscale, gscale * c0);
  const size_t row = f.px, plane = (size_t)f.px * f.py;
  col_pass<double, 0>(work, f, t, f.ay, t.tw_y, f.cols_y, row, plane, f.pz, 1, f.py, f.py, nullptr, RedJob{}, st, 0);
  col_pass<double, 0>(work, f, t, f.az, t.tw_z, f.cols_z, plane, row, f.py, 1, f.pz, f.pz, nullptr, RedJob{}, st, 0);
  k_iso_green_extract<<<1024, 256, 0, st>>>(work, green, f);
}

template <typename D, typename S>
void launch_phi_interior(D* dst, const S* ext, int nx, int ny, int nz, hipStream_t st) {
  const size_t n = (size_t)nx * ny * nz;
  const unsigned nblk = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
  k_phi_interior<D, S><<<nblk, 256, 0, st>>>(dst, ext, nx, ny, nz);
}

template void launch_iso_fwd<double>(const SrcSlot*, int, cplx<double>*, const IsoGeom&, const IsoTables<double>&,
                                     hipStream_t);
template void launch_iso_fwd<float>(const SrcSlot*, int, cplx<float>*, const IsoGeom&, const IsoTables<float>&,
                                    hipStream_t);
template void launch_iso_z<double>(cplx<double>*, const IsoGeom&, const IsoTables<double>&, double*, const RedJob&,
                                   hipStream_t);
template void launch_iso_z<float>(cplx<float>*, const IsoGeom&, const IsoTables<float>&, double*, const RedJob&,
                                  hipStream_t);
template void launch_iso_inv<double>(cplx<double>*, double*, const IsoGeom&, const IsoTables<double>&,
                                     const FinJob&, hipStream_t);
template void launch_iso_inv<float>(cplx<float>*, float*, const IsoGeom&, const IsoTables<float>&, const FinJob&,
                                    hipStream_t);
template void launch_phi_interior<double, double>(double*, const double*, int, int, int, hipStream_t);
template void launch_phi_interior<float, double>(float*, const double*, int, int, int, hipStream_t);
template void launch_phi_interior<double, float>(double*, const float*, int, int, int, hipStream_t);
template void launch_phi_interior<float, float>(float*, const float*, int, int, int, hipStream_t);

}  // namespace gp
