// FFT Poisson solve of one GPUPEGAS step (Kulikov, arXiv:1311.0861, Sec. 2.3):
//   Phi^(k) = -4 pi G h^2 s^(k) / (6 (1 - D_x D_y D_z)),  D_d = 1 - (2/3) sin^2(pi k_d / N_d),
//   Phi^(0) = 0  (periodic, zero-mean potential; the printed symbol lacks the
//   minus sign that Laplace(Phi) = 4 pi G s requires).
//
// Five passes over a half spectrum C[z][y][kx], kx in [0, nx/2] (row pitch px):
//   x forward  : the source s = rho + n - <rho + n> is formed in FP64 from the
//                densities (the constant leaves Phi unchanged, as its zero mode
//                is dropped, and keeping it out of an FP32 transform keeps the
//                other modes accurate); real rows of length nx -> complex FFT
//                of length nx/2 on packed (even, odd) pairs, then the even/odd
//                split to nx/2+1 bins;
//   y forward  : columns of C along y;
//   z fused    : forward along z, multiply by the symbol (and the inverse
//                normalisation), accumulate sum |s^|^2 G for the potential
//                energy, inverse along z -- one read and one write of C;
//   y inverse, x inverse (complex-to-real).
// Each workgroup stages whole lines in LDS and runs a Stockham autosort FFT
// (radices 8, 4, 3, 2; output in natural order) with all butterflies of a stage
// held in registers between two barriers, so the stages work in place.
// Twiddles come from tables computed on the host in FP64.
#include "common.hpp"
#include "kernels.hpp"

namespace gp {

constexpr int kFftThreads = 256;

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
// multiply by -i (forward) or +i (inverse)
template <typename T>
__device__ __forceinline__ cplx<T> rot(cplx<T> a, bool inv) {
  return inv ? cplx<T>{-a.y, a.x} : cplx<T>{a.y, -a.x};
}

template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T> v[R], bool inv) {
  if constexpr (R == 2) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    const T s = inv ? T(0.86602540378443864676) : T(-0.86602540378443864676);
    const cplx<T> t1 = cadd(v[1], v[2]);
    const cplx<T> t2 = {v[0].x - T(0.5) * t1.x, v[0].y - T(0.5) * t1.y};
    const cplx<T> d = {s * (v[1].x - v[2].x), s * (v[1].y - v[2].y)};  // times i below
    v[0] = cadd(v[0], t1);
    v[1] = {t2.x - d.y, t2.y + d.x};
    v[2] = {t2.x + d.y, t2.y - d.x};
  } else if constexpr (R == 4) {
    const cplx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const cplx<T> t2 = cadd(v[1], v[3]), t3 = rot(csub(v[1], v[3]), inv);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else {  // R == 8: two radix-4 halves and the W_8 combination
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft_small<T, 4>(e, inv);
    dft_small<T, 4>(o, inv);
    const T h = T(0.70710678118654752440);
    const T sg = inv ? T(1) : T(-1);
    const cplx<T> w1 = {h, sg * h}, w3 = {-h, sg * h};
    const cplx<T> o1 = cmul(o[1], w1), o2 = rot(o[2], inv), o3 = cmul(o[3], w3);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
}

// Largest number of complex points one workgroup stages (32 KiB of LDS).
template <typename T>
constexpr int max_points() {
  return 32768 / (int)sizeof(cplx<T>);
}

// One Stockham stage of radix R on `lines` lines of length L (line pitch lp),
// in place: reads to registers, barrier, writes, barrier.
template <typename T, int R>
__device__ void fft_stage(cplx<T>* buf, int lines, int L, int lp, int Ns, const cplx<T>* tw, bool inv) {
  constexpr int MAXB = (max_points<T>() / R + kFftThreads - 1) / kFftThreads;
  const int nb = L / R;
  const int total = lines * nb;
  const int tstep = L / (Ns * R);
  cplx<T> v[MAXB][R];
#pragma unroll
  for (int b = 0; b < MAXB; b++) {
    const int q = threadIdx.x + b * kFftThreads;
    if (q < total) {
      const int line = q / nb, jj = q - line * nb;
      const int kk = jj % Ns;
      const cplx<T>* base = buf + line * lp;
#pragma unroll
      for (int r = 0; r < R; r++) {
        cplx<T> x = base[jj + r * nb];
        if (r > 0) {
          cplx<T> w = tw[kk * r * tstep];
          if (inv) w.y = -w.y;
          x = cmul(x, w);
        }
        v[b][r] = x;
      }
      dft_small<T, R>(v[b], inv);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; b++) {
    const int q = threadIdx.x + b * kFftThreads;
    if (q < total) {
      const int line = q / nb, jj = q - line * nb;
      const int kk = jj % Ns;
      cplx<T>* base = buf + line * lp;
      const int d0 = (jj / Ns) * Ns * R + kk;
#pragma unroll
      for (int r = 0; r < R; r++) base[d0 + r * Ns] = v[b][r];
    }
  }
  __syncthreads();
}

template <typename T>
__device__ void lds_fft(cplx<T>* buf, int lines, int lp, const FftAxis& ax, const cplx<T>* tw, bool inv) {
  int Ns = 1;
  for (int s = 0; s < ax.nst; s++) {
    const int R = ax.rad[s];
    if (R == 8)
      fft_stage<T, 8>(buf, lines, ax.L, lp, Ns, tw, inv);
    else if (R == 4)
      fft_stage<T, 4>(buf, lines, ax.L, lp, Ns, tw, inv);
    else if (R == 3)
      fft_stage<T, 3>(buf, lines, ax.L, lp, Ns, tw, inv);
    else
      fft_stage<T, 2>(buf, lines, ax.L, lp, Ns, tw, inv);
    Ns *= R;
  }
}

template <typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* dst, const cplx<T>* src, int n) {
  for (int t = threadIdx.x; t < n; t += kFftThreads) dst[t] = src[t];
}

// ---- x forward: rows of s (length nx) -> C rows (nx/2 + 1 bins) -------------
template <typename T>
__global__ void __launch_bounds__(kFftThreads) k_fft_x_fwd(const SrcSlot* __restrict__ src, int parity,
                                                           cplx<T>* __restrict__ spec, FftGeom f, FftTables<T> t) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int M = f.ax.L;
  const int RB = f.rows_per_block;
  cplx<T>* tw = lds + RB * M;
  cplx<T>* wn = tw + M;
  const int rows_run = f.ny * f.nz;
  const int nrows = rows_run * f.nruns;
  const int row0 = blockIdx.x * RB;
  const int rows = min(RB, nrows - row0);
  load_twiddles(tw, t.tw_x, M);
  load_twiddles(wn, t.wn_x, M + 1);
  // packed (even, odd) pairs of each row of s
  for (int q = threadIdx.x; q < rows * M; q += kFftThreads) {
    const int row = row0 + q / M, m = q % M;
    const int slot = row / rows_run;
    const size_t c = (size_t)(row - slot * rows_run) * f.nx + 2 * m;
    const SrcSlot& S = src[slot];
    const double shift = S.sc->shift;
    const double* rho = S.rho[parity];
    const double* nb = S.nb[parity];
    lds[q] = {(T)(rho[c] + nb[c] - shift), (T)(rho[c + 1] + nb[c + 1] - shift)};
  }
  __syncthreads();
  lds_fft(lds, rows, M, f.ax, tw, false);
  // even/odd split: X[k] = E[k] + W_N^k O[k]
  for (int q = threadIdx.x; q < rows * (M + 1); q += kFftThreads) {
    const int rr = q / (M + 1), k = q - rr * (M + 1);
    const cplx<T> zk = lds[rr * M + (k == M ? 0 : k)];
    cplx<T> zc = lds[rr * M + (k == 0 ? 0 : M - k)];
    zc.y = -zc.y;
    const cplx<T> E = {T(0.5) * (zk.x + zc.x), T(0.5) * (zk.y + zc.y)};
    const cplx<T> O = {T(0.5) * (zk.y - zc.y), T(-0.5) * (zk.x - zc.x)};  // -i (zk - zc) / 2
    spec[(size_t)(row0 + rr) * f.px + k] = cadd(E, cmul(wn[k], O));
  }
}

// ---- x inverse: C rows -> real rows of phi ---------------------------------
template <typename T>
__global__ void __launch_bounds__(kFftThreads) k_fft_x_inv(const cplx<T>* __restrict__ spec, T* __restrict__ phi,
                                                           FftGeom f, FftTables<T> t) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int M = f.ax.L;
  const int RB = f.rows_per_block;
  cplx<T>* xin = lds + RB * M;          // RB rows of M + 1 bins
  cplx<T>* tw = xin + RB * (M + 1);
  cplx<T>* wn = tw + M;
  const int nrows = f.ny * f.nz * f.nruns;
  const int row0 = blockIdx.x * RB;
  const int rows = min(RB, nrows - row0);
  load_twiddles(tw, t.tw_x, M);
  load_twiddles(wn, t.wn_x, M + 1);
  for (int q = threadIdx.x; q < rows * (M + 1); q += kFftThreads) xin[q] = spec[(size_t)row0 * f.px + q];
  __syncthreads();
  // Z[k] = E[k] + i O[k],  E = (X_k + conj X_{M-k}) / 2,  O = (X_k - conj X_{M-k}) / 2 * W_N^{-k}
  for (int q = threadIdx.x; q < rows * M; q += kFftThreads) {
    const int rr = q / M, k = q - rr * M;
    const cplx<T> xk = xin[rr * (M + 1) + k];
    cplx<T> xc = xin[rr * (M + 1) + M - k];
    xc.y = -xc.y;
    const cplx<T> E = {T(0.5) * (xk.x + xc.x), T(0.5) * (xk.y + xc.y)};
    cplx<T> w = wn[k];
    w.y = -w.y;
    const cplx<T> O = cmul({T(0.5) * (xk.x - xc.x), T(0.5) * (xk.y - xc.y)}, w);
    lds[rr * M + k] = {E.x - O.y, E.y + O.x};
  }
  __syncthreads();
  lds_fft(lds, rows, M, f.ax, tw, true);
  cplx<T>* dst = reinterpret_cast<cplx<T>*>(phi) + (size_t)row0 * M;
  for (int q = threadIdx.x; q < rows * M; q += kFftThreads) dst[q] = lds[q];
}

// ---- column passes (y, and the fused z pass) -------------------------------
// A workgroup takes `cb` consecutive kx columns and one index of the other
// transverse axis of one run; line j of column c lives at base + j * stride + c
// with base = run * run_stride + o * outer_stride + kx0 for outer index
// run * outer_div + o.
template <typename T, int MODE>  // MODE 0: forward, 1: inverse, 2: forward * symbol * inverse
__global__ void __launch_bounds__(kFftThreads) k_fft_col(cplx<T>* __restrict__ spec, FftGeom f, FftTables<T> t,
                                                         FftAxis ax, const cplx<T>* __restrict__ twg, int cb,
                                                         size_t stride, size_t outer_stride, int outer_div,
                                                         size_t run_stride, double* __restrict__ epot_partials) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int L = ax.L;
  const int lp = L + 1;  // padded line pitch
  cplx<T>* tw = lds + cb * lp;
  const int nchunks = (f.px + cb - 1) / cb;
  const int chunk = blockIdx.x % nchunks;
  const int oline = blockIdx.x / nchunks;
  const int outer = oline % outer_div;
  const int kx0 = chunk * cb;
  const int ncols = min(cb, f.px - kx0);
  load_twiddles(tw, twg, L);
  cplx<T>* base = spec + (size_t)(oline / outer_div) * run_stride + (size_t)outer * outer_stride + kx0;
  for (int q = threadIdx.x; q < cb * L; q += kFftThreads) {
    const int c = q % cb, j = q / cb;
    lds[c * lp + j] = (c < ncols) ? base[(size_t)j * stride + c] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  lds_fft(lds, cb, lp, ax, tw, MODE == 1);
  if constexpr (MODE == 2) {
    // z pass: outer = ky, line position = kz, column = kx
    __shared__ double red[kFftThreads / 64];
    double ep = 0.0;
    const double dy = t.dy[outer];
    for (int q = threadIdx.x; q < cb * L; q += kFftThreads) {
      const int c = q / L, kz = q - c * L;
      if (c >= ncols) continue;
      const int kx = kx0 + c;
      cplx<T>& v = lds[c * lp + kz];
      double gk = 0.0;
      if (kx != 0 || outer != 0 || kz != 0) gk = f.green_scale / (1.0 - t.dx[kx] * dy * t.dz[kz]);
      const double w = (kx == 0 || 2 * kx == f.nx) ? 1.0 : 2.0;  // Hermitian half spectrum
      ep += w * gk * ((double)v.x * (double)v.x + (double)v.y * (double)v.y);
      const T gs = (T)(gk * f.norm);
      v.x *= gs;
      v.y *= gs;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ep += __shfl_xor(ep, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ep;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < kFftThreads / 64; w++) s += red[w];
      epot_partials[blockIdx.x] = s;
    }
    lds_fft(lds, cb, lp, ax, tw, true);
  }
  for (int q = threadIdx.x; q < cb * L; q += kFftThreads) {
    const int c = q % cb, j = q / cb;
    if (c < ncols) base[(size_t)j * stride + c] = lds[c * lp + j];
  }
}

static size_t x_lds_bytes(const FftGeom& f, size_t csz, bool inv) {
  const size_t M = f.ax.L, RB = f.rows_per_block;
  return csz * (RB * M + (inv ? RB * (M + 1) : 0) + M + M + 1);
}

int fft_blocks_z(const FftGeom& f) { return ((f.px + f.cols_z - 1) / f.cols_z) * f.ny * f.nruns; }

template <typename T>
void launch_fft_x_fwd(const SrcSlot* src, int parity, cplx<T>* spec, const FftGeom& f, const FftTables<T>& t,
                      hipStream_t st) {
  const int nrows = f.ny * f.nz * f.nruns;
  const int nblk = (nrows + f.rows_per_block - 1) / f.rows_per_block;
  k_fft_x_fwd<T><<<nblk, kFftThreads, x_lds_bytes(f, sizeof(cplx<T>), false), st>>>(src, parity, spec, f, t);
}

template <typename T>
void launch_fft_x_inv(const cplx<T>* spec, T* phi, const FftGeom& f, const FftTables<T>& t, hipStream_t st) {
  const int nrows = f.ny * f.nz * f.nruns;
  const int nblk = (nrows + f.rows_per_block - 1) / f.rows_per_block;
  k_fft_x_inv<T><<<nblk, kFftThreads, x_lds_bytes(f, sizeof(cplx<T>), true), st>>>(spec, phi, f, t);
}

template <typename T>
void launch_fft_y(cplx<T>* spec, const FftGeom& f, const FftTables<T>& t, bool inverse, hipStream_t st) {
  const int cb = f.cols_y;
  const int nblk = ((f.px + cb - 1) / cb) * f.nz * f.nruns;
  const size_t lds = sizeof(cplx<T>) * ((size_t)cb * (f.ay.L + 1) + f.ay.L);
  const size_t stride = f.px, outer = (size_t)f.px * f.ny, run = outer * f.nz;
  if (inverse)
    k_fft_col<T, 1><<<nblk, kFftThreads, lds, st>>>(spec, f, t, f.ay, t.tw_y, cb, stride, outer, f.nz, run, nullptr);
  else
    k_fft_col<T, 0><<<nblk, kFftThreads, lds, st>>>(spec, f, t, f.ay, t.tw_y, cb, stride, outer, f.nz, run, nullptr);
}

template <typename T>
void launch_fft_z_green(cplx<T>* spec, const FftGeom& f, const FftTables<T>& t, double* epot_partials,
                        hipStream_t st) {
  const int cb = f.cols_z;
  const int nblk = fft_blocks_z(f);
  const size_t lds = sizeof(cplx<T>) * ((size_t)cb * (f.az.L + 1) + f.az.L);
  const size_t stride = (size_t)f.px * f.ny, outer = f.px, run = stride * f.nz;
  k_fft_col<T, 2><<<nblk, kFftThreads, lds, st>>>(spec, f, t, f.az, t.tw_z, cb, stride, outer, f.ny, run,
                                                  epot_partials);
}

template void launch_fft_x_fwd<double>(const SrcSlot*, int, cplx<double>*, const FftGeom&,
                                       const FftTables<double>&, hipStream_t);
template void launch_fft_x_fwd<float>(const SrcSlot*, int, cplx<float>*, const FftGeom&, const FftTables<float>&,
                                      hipStream_t);
template void launch_fft_x_inv<double>(const cplx<double>*, double*, const FftGeom&, const FftTables<double>&,
                                       hipStream_t);
template void launch_fft_x_inv<float>(const cplx<float>*, float*, const FftGeom&, const FftTables<float>&,
                                      hipStream_t);
template void launch_fft_y<double>(cplx<double>*, const FftGeom&, const FftTables<double>&, bool, hipStream_t);
template void launch_fft_y<float>(cplx<float>*, const FftGeom&, const FftTables<float>&, bool, hipStream_t);
template void launch_fft_z_green<double>(cplx<double>*, const FftGeom&, const FftTables<double>&, double*,
                                         hipStream_t);
template void launch_fft_z_green<float>(cplx<float>*, const FftGeom&, const FftTables<float>&, double*,
                                        hipStream_t);

}  // namespace gp
