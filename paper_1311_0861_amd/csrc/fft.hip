// FFT Poisson solve of one GPUPEGAS step (Kulikov, arXiv:1311.0861, Sec. 2.3):
//   Phi^(k) = -4 pi G h^2 s^(k) / (6 (1 - D_x D_y D_z)),  D_d = 1 - (2/3) sin^2(pi k_d / N_d),
//   Phi^(0) = 0  (periodic, zero-mean potential; the printed symbol lacks the
//   minus sign that Laplace(Phi) = 4 pi G s requires).
//
// Passes over a half spectrum of rows of px = nx/2 + 1 values, kx in [0, nx/2],
// stored C[z][ky][kx] by the line passes and C[ky][z][kx] by the plane passes:
//   xy forward : the source s = rho + n is formed in FP64 from the densities
//                (its mean is the zero mode, which the symbol drops, so Phi
//                solves the equation for s - <s>); real rows of length nx ->
//                complex FFT of length nx/2 on packed (even, odd) pairs, the
//                even/odd split to nx/2+1 bins, then the columns along y;
//   z fused    : forward along z, multiply by the symbol (and the inverse
//                normalisation), accumulate sum |s^|^2 G for the potential
//                energy, inverse along z -- one read and one write of C;
//   xy inverse : columns along y, then the complex-to-real rows.
// Where two workgroups holding half a z plane fit on a CU, the plane passes
// split the y transform by row parity (see the plane passes below): one
// workgroup per (plane, row parity) does both transforms, and the z pass
// joins and splits the two halves (three passes over C in all); otherwise the
// x and y transforms are separate passes (five in all).
// Each workgroup stages whole lines in LDS and runs a Stockham autosort FFT
// (radices 8, 4, 3, 2; output in natural order) with all butterflies of a stage
// held in registers between two barriers, so the stages work in place.
// Twiddles come from tables computed on the host in FP64.
#include <algorithm>
#include <type_traits>

#include "fft_core.hpp"
#include "reduce.hpp"

namespace gp {


// ---- x forward: rows of s (length nx) -> C rows (nx/2 + 1 bins) -------------
// MC, RBC > 0: the half row length and the rows per block are compile-time
// constants (equal to f.ax.L and f.rows_per_block).
template <typename T, int MC = 0, int RBC = 0>
__global__ void __launch_bounds__(kFftThreads) k_fft_x_fwd(const SrcSlot* __restrict__ src, int parity,
                                                           cplx<T>* __restrict__ spec, FftGeom f, FftTables<T> t) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int M = MC ? MC : f.ax.L, xp = M | 1;  // odd row pitch
  const int RB = RBC ? RBC : f.rows_per_block;
  cplx<T>* tw = lds + RB * xp;
  cplx<T>* wn = tw + M;
  const int rows_run = f.ny * f.nz;
  const int nrows = rows_run * f.nruns;
  const int row0 = blockIdx.x * RB;
  const int rows = min(RB, nrows - row0);
  load_twiddles<kFftThreads>(tw, t.tw_x, M);
  load_twiddles<kFftThreads>(wn, t.wn_x, M + 1);
  const CDiv<MC> dm(M);
  const CDiv<MC ? MC + 1 : 0> dm1(M + 1);
  // packed (even, odd) pairs of each row of s
  staged_copy<kFftThreads, 4, cplx<T>>(
      rows * M,
      [&](int q) {
        const int rq = (int)dm.div(q);
        const int row = row0 + rq, m = q - rq * M;
        const int slot = row / rows_run;  // may exceed the range of FastDiv
        const size_t c = (size_t)(row - slot * rows_run) * f.nx + 2 * m;
        const SrcSlot& S = src[slot];
        const dpair a = gload(reinterpret_cast<const dpair*>(S.rho[parity] + c));
        const dpair b = gload(reinterpret_cast<const dpair*>(S.nb[parity] + c));
        return cplx<T>{(T)(a.x + b.x), (T)(a.y + b.y)};
      },
      [&](int q, cplx<T> v) {
        const int rq = (int)dm.div(q);
        lds[rq * xp + q - rq * M] = v;
      });
  __syncthreads();
  x_rows_fft<T, MC, RBC, false>(lds, rows, xp, f.ax, tw);
  // even/odd split: X[k] = E[k] + W_N^k O[k]
  for (int q = threadIdx.x; q < rows * (M + 1); q += kFftThreads) {
    const int rr = (int)dm1.div(q), k = q - rr * (M + 1);
    const cplx<T> zk = lds[rr * xp + (k == M ? 0 : k)];
    const cplx<T> zc = lds[rr * xp + (k == 0 ? 0 : M - k)];
    spec[(size_t)(row0 + rr) * f.px + k] = split_fwd(zk, zc, wn[k]);
  }
}

// ---- x inverse: C rows -> real rows of phi ---------------------------------
// The first fin.n workgroups finish the step instead (one per run).
template <typename T, int MC = 0, int RBC = 0>
__global__ void __launch_bounds__(kFftThreads) k_fft_x_inv(const cplx<T>* __restrict__ spec, T* __restrict__ phi,
                                                           FftGeom f, FftTables<T> t, FinJob fin) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  if ((int)blockIdx.x < fin.n) {
    finalize_run(fin, (int)blockIdx.x, reinterpret_cast<double*>(smem_raw));
    return;
  }
  const int bid = (int)blockIdx.x - fin.n;
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int M = MC ? MC : f.ax.L, xp = M | 1;  // odd row pitch
  const int RB = RBC ? RBC : f.rows_per_block;
  cplx<T>* xin = lds + RB * xp;         // RB rows of M + 1 bins
  cplx<T>* tw = xin + RB * (M + 1);
  cplx<T>* wn = tw + M;
  const int nrows = f.ny * f.nz * f.nruns;
  const int row0 = bid * RB;
  const int rows = min(RB, nrows - row0);
  load_twiddles<kFftThreads>(tw, t.tw_x, M);
  load_twiddles<kFftThreads>(wn, t.wn_x, M + 1);
  const CDiv<MC> dm(M);
  staged_copy<kFftThreads, 4, cplx<T>>(
      rows * (M + 1), [&](int q) { return gload(spec + (size_t)row0 * f.px + q); },
      [&](int q, cplx<T> v) { xin[q] = v; });
  __syncthreads();
  for (int q = threadIdx.x; q < rows * M; q += kFftThreads) {
    const int rr = (int)dm.div(q), k = q - rr * M;
    lds[rr * xp + k] = split_inv(xin[rr * (M + 1) + k], xin[rr * (M + 1) + M - k], wn[k]);
  }
  __syncthreads();
  x_rows_fft<T, MC, RBC, true>(lds, rows, xp, f.ax, tw);
  cplx<T>* dst = reinterpret_cast<cplx<T>*>(phi) + (size_t)row0 * M;
  for (int q = threadIdx.x; q < rows * M; q += kFftThreads) {
    const int rq = (int)dm.div(q);
    dst[q] = lds[rq * xp + q - rq * M];
  }
}

// ---- column passes (y, and the fused z pass; block layout: col_block) -----
// In the z pass the first red.n workgroups reduce partial rows instead (they
// need nothing from the transform, and the pass has room beside it).
// With pair set (the z pass after the plane passes) a workgroup takes the cb
// columns of two spectrum rows, line o and line o + pair_stride / outer_stride
// (ky and ky + ny/2), which hold E and O: it forms C[ky] = E + W^ky O and
// C[ky + ny/2] = E - W^ky O before the z transforms, and stores e = C[ky] +
// C[ky + ny/2] and o = (C[ky] - C[ky + ny/2]) W^-ky after them.
// LC, CBC, NRC > 0: the transform length, the columns per row and the rows
// per workgroup are compile-time constants (they must equal ax.L, cb and
// 1 + pair), so that every index is derived from constants.
template <typename T, int MODE, int LC = 0, int CBC = 0, int NRC = 0>  // MODE 0: forward, 1: inverse, 2: forward * symbol * inverse
__global__ void __launch_bounds__(kFftThreads) k_fft_col(cplx<T>* __restrict__ spec, FftGeom f, FftTables<T> t,
                                                         FftAxis ax, const cplx<T>* __restrict__ twg, int cb_rt,
                                                         size_t stride, size_t outer_stride, int outer_div,
                                                         size_t run_stride, double* __restrict__ epot_partials,
                                                         RedJob red, int pair, size_t pair_stride) {
  static_assert(LC == 0 || (CBC > 0 && (NRC == 1 || (MODE == 2 && NRC == 2))), "compile-time block shape");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
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
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int L = LC ? LC : ax.L;
  const int cb = CBC ? CBC : cb_rt;
  const int nr = NRC ? NRC : ((MODE == 2 && pair) ? 2 : 1);  // spectrum rows per workgroup
  const int cw = nr * cb;                                      // LDS columns: cb per row
  // LDS holds the block as L rows of cw columns: element j of column c at
  // j * cw + c, so that lanes on neighbouring columns touch neighbouring words
  cplx<T>* tw = lds + cw * L;
  // the transforms along the columns of the block
  auto transform = [&](bool inv) {
    if constexpr (LC > 0) {
      constexpr int CW = CBC * NRC;
      if (inv)
        cfft<T, LC, CW, 1, CW, kFftThreads, true>(lds, tw);
      else
        cfft<T, LC, CW, 1, CW, kFftThreads, false>(lds, tw);
    } else {
      col_fft(lds, cw, ax, tw, inv);
    }
  };
  const int nchunks = (f.px + cb - 1) / cb;
  const ColBlock cbk = col_block(bid, nchunks, nblk / nchunks);
  const int chunk = cbk.chunk, oline = cbk.oline;
  const int run = oline / outer_div, outer = oline - run * outer_div;
  const int kx0 = chunk * cb;
  const int ncols = min(cb, f.px - kx0);
  load_twiddles<kFftThreads>(tw, twg, L);
  const FastDiv dcw(cw), dcb(cb);
  // index split q -> (q / n, q % n) by a compile-time or a run-time divisor
  auto split_cb = [&](int q, int& j, int& c) {
    if constexpr (CBC > 0) {
      j = q / CBC;
      c = q % CBC;
    } else {
      j = (int)dcb.div(q);
      c = q - j * cb;
    }
  };
  auto split_cw = [&](int q, int& j, int& c) {
    if constexpr (CBC > 0) {
      j = q / (CBC * NRC);
      c = q % (CBC * NRC);
    } else {
      j = (int)dcw.div(q);
      c = q - j * cw;
    }
  };
  // z pass: the symbol's factors D(kz) and D(kx) D(ky) of this block
  double* gz = reinterpret_cast<double*>(tw + L);
  double* gxy = gz + L;
  if constexpr (MODE == 2) {
    for (int q = threadIdx.x; q < L + cw; q += kFftThreads) {
      if (q < L) {
        gz[q] = gload(t.dz + q);
      } else {
        const int c = q - L, h = c >= cb ? 1 : 0, cc = c - h * cb;
        gxy[c] = cc < ncols ? gload(t.dx + kx0 + cc) * gload(t.dy + outer + h * outer_div) : 0.0;
      }
    }
  }
  cplx<T>* base = spec + (size_t)run * run_stride + (size_t)outer * outer_stride + kx0;
  cplx<T> wk = {T(1), T(0)};  // W^ky of the row pair
  if (nr == 2) {
    // E and O of one (kz, kx) by one thread, combined on their way to LDS
    wk = gload(t.tw_y + outer);
    struct Pair {
      cplx<T> e, o;
    };
    staged_copy<kFftThreads, 2, Pair>(
        cb * L,
        [&](int q) {
          int j, cc;
          split_cb(q, j, cc);
          const cplx<T>* g = base + (size_t)j * stride + min(cc, ncols - 1);
          Pair v{gload(g), gload(g + pair_stride)};
          if (cc >= ncols) v = Pair{{T(0), T(0)}, {T(0), T(0)}};
          return v;
        },
        [&](int q, Pair v) {
          int j, cc;
          split_cb(q, j, cc);
          const cplx<T> o = cmul(v.o, wk);
          lds[j * cw + cc] = cadd(v.e, o);
          lds[j * cw + cb + cc] = csub(v.e, o);
        });
  } else {
    staged_copy<kFftThreads, 4, cplx<T>>(
        cw * L,
        [&](int q) {
          int j, c;
          split_cw(q, j, c);
          const cplx<T> v = gload(base + (size_t)j * stride + min(c, ncols - 1));
          return (c < ncols) ? v : cplx<T>{T(0), T(0)};
        },
        [&](int q, cplx<T> v) { lds[q] = v; });
  }
  __syncthreads();
  transform(MODE == 1);
  if constexpr (MODE == 2) {
    // z pass: line position = kz, column = (row h, kx); the potential-energy
    // partial of each row goes to slot (line, chunk), so that a run's
    // partials are contiguous whichever form ran
    __shared__ double red_ep[2][kFftThreads / 64];
    double ep[2] = {0.0, 0.0};
    for (int q = threadIdx.x; q < cw * L; q += kFftThreads) {
      int kz, c;
      split_cw(q, kz, c);
      const int h = c >= cb ? 1 : 0, cc = c - h * cb;
      if (cc >= ncols) continue;
      const int kx = kx0 + cc, ky = outer + h * outer_div;
      cplx<T>& v = lds[q];
      double gk = 0.0;
      if (kx != 0 || ky != 0 || kz != 0) gk = f.green_scale / (1.0 - gxy[c] * gz[kz]);
      const double w = (kx == 0 || 2 * kx == f.nx) ? 1.0 : 2.0;  // Hermitian half spectrum
      ep[h] += w * gk * ((double)v.x * (double)v.x + (double)v.y * (double)v.y);
      const T gs = (T)(gk * f.norm);
      v.x *= gs;
      v.y *= gs;
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) ep[h] += __shfl_xor(ep[h], off, 64);
      if ((threadIdx.x & 63) == 0) red_ep[h][threadIdx.x >> 6] = ep[h];
    }
    __syncthreads();
    if (threadIdx.x < nr) {
      const int h = threadIdx.x;
      double s = 0.0;
      for (int w = 0; w < kFftThreads / 64; w++) s += red_ep[h][w];
      const size_t line = (size_t)run * outer_div * nr + outer + h * outer_div;  // spectrum row of the run
      epot_partials[line * nchunks + chunk] = s;
    }
    transform(true);
    if (nr == 2) {
      // e and o of one (z, kx) by one thread, formed on their way out
      const cplx<T> wc = {wk.x, -wk.y};
      for (int q = threadIdx.x; q < cb * L; q += kFftThreads) {
        int j, cc;
        split_cb(q, j, cc);
        if (cc >= ncols) continue;
        const cplx<T> c0 = lds[j * cw + cc], c1 = lds[j * cw + cb + cc];
        cplx<T>* g = base + (size_t)j * stride + cc;
        g[0] = cadd(c0, c1);
        g[pair_stride] = cmul(csub(c0, c1), wc);
      }
      return;
    }
  }
  for (int q = threadIdx.x; q < cw * L; q += kFftThreads) {
    int j, c;
    split_cw(q, j, c);
    if (c < ncols) base[(size_t)j * stride + c] = lds[q];
  }
}

// ---- xy plane passes: the transverse transforms of half a z plane in LDS ---
// The y transform of length ny splits by row parity (decimation in time):
//   C[k] = E[k] + W^k O[k],  C[k + ny/2] = E[k] - W^k O[k],  k < ny/2,
// with E, O the length-ny/2 transforms of the even and the odd rows and
// W = exp(-2 pi i / ny).  Workgroup (plane, p) takes rows 2j + p: the x
// transform of each row (nx/2 + 1 bins, from the half-length complex FFT and
// the split) and the length-ny/2 transforms of the nx/2 + 1 columns, held as
// ny/2 rows of odd pitch hp; it stores E or O in spectrum rows p ny/2 + k.
// The z pass forms C from E and O before its transforms and returns the even
// and odd parts e = C[k] + C[k + ny/2], o = (C[k] - C[k + ny/2]) W^-k after
// them, so that the inverse plane pass again takes one row parity: row 2j + p
// of the inverse y transform is the length-ny/2 inverse transform of e or o.
// Two workgroups per plane, each with half the LDS of a whole plane.
// Transform of a half plane: compile-time form when L > 0, else run-time.
template <typename T, int L, int LINES, int LS, int ES, bool INV>
__device__ __forceinline__ void plane_fft(cplx<T>* buf, int lines, int ls, int es, const FftAxis& ax,
                                          const cplx<T>* tw) {
  if constexpr (L > 0)
    cfft<T, L, LINES, LS, ES, kPlaneThreads, INV>(buf, tw);
  else
    lds_fft<T, kPlaneThreads, plane_points<T>()>(buf, lines, ls, es, ax, tw, INV);
}

// Compile-time plane geometry of an NX x NY plane (all zero for run-time).
template <int NX, int NY>
struct PlaneShape {
  static constexpr int M = NX / 2, HY = NY / 2, HP = NX ? ((NX / 2 + 1) | 1) : 0;
  static constexpr int M1 = NX ? M + 1 : 0, H = NX ? M / 2 + 1 : 0;
};

template <typename T>
struct PlaneLds {
  cplx<T>* pl;   // ny/2 x hp half plane
  cplx<T>* twx;  // M
  cplx<T>* wn;   // M + 1
  cplx<T>* twy;  // ny / 2
};

template <typename T>
__device__ __forceinline__ PlaneLds<T> plane_lds(const FftGeom& f, const FftTables<T>& t) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  PlaneLds<T> s;
  const int M = f.ax.L;
  s.pl = reinterpret_cast<cplx<T>*>(smem_raw);
  s.twx = s.pl + (f.ny / 2) * f.hp;
  s.wn = s.twx + M;
  s.twy = s.wn + M + 1;
  load_twiddles<kPlaneThreads>(s.twx, t.tw_x, M);
  load_twiddles<kPlaneThreads>(s.wn, t.wn_x, M + 1);
  load_twiddles<kPlaneThreads>(s.twy, t.tw_yh, f.ny / 2);
  return s;
}

// NX, NY > 0: the plane size is a compile-time constant (it must equal
// f.nx, f.ny), so that every index is derived from constants.
template <typename T, int NX = 0, int NY = 0>
__global__ void __launch_bounds__(kPlaneThreads) k_fft_xy_fwd(const SrcSlot* __restrict__ src, int parity,
                                                             cplx<T>* __restrict__ spec, FftGeom f, FftTables<T> t) {
  constexpr int NT = kPlaneThreads;
  using PS = PlaneShape<NX, NY>;
  const PlaneLds<T> s = plane_lds(f, t);
  const int M = NX ? PS::M : f.ax.L, hy = NY ? PS::HY : f.ny / 2, hp = NX ? PS::HP : f.hp;
  const CDiv<PS::M> dm(M);
  const CDiv<PS::M1> dm1(M + 1);
  const CDiv<PS::H> dh(M / 2 + 1);
  const int plane = (int)blockIdx.x >> 1, p = (int)blockIdx.x & 1;  // run * nz + z, row parity
  const int slot = plane / f.nz, z = plane - slot * f.nz;
  const SrcSlot& S = src[slot];
  // rows 2j + p of the plane, M packed (even, odd) pairs each
  const size_t off = ((size_t)z * f.ny + p) * f.nx;
  const dpair* rho = reinterpret_cast<const dpair*>(S.rho[parity] + off);
  const dpair* nb = reinterpret_cast<const dpair*>(S.nb[parity] + off);
  auto source = [&](int q) {
    const int j = (int)dm.div(q);
    const size_t e = (size_t)q + (size_t)j * M;  // pair m of row 2j + p: 2 j M + m
    const dpair a = gload(rho + e), c = gload(nb + e);
    return cplx<T>{(T)(a.x + c.x), (T)(a.y + c.y)};
  };
  constexpr int HALF = PS::HY / 2 * PS::M;  // pairs in half the rows
  if constexpr (NX > 0 && HALF % NT == 0) {
    // Every load of the half plane goes out first; the first half of the
    // rows is staged and transformed while the second half is still
    // arriving, then the second half (the same row transforms, the same bits).
    constexpr int PER = HALF / NT;
    cplx<T> v[2][PER];
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
      for (int i = 0; i < PER; i++) v[h][i] = source(h * HALF + (int)threadIdx.x + i * NT);
#pragma unroll
    for (int h = 0; h < 2; h++) {
#pragma unroll
      for (int i = 0; i < PER; i++) {
        const int q = h * HALF + (int)threadIdx.x + i * NT;
        const int j = (int)dm.div(q), m = q - j * M;
        s.pl[j * hp + m] = v[h][i];
      }
      lds_barrier();
      plane_fft<T, PS::M, PS::HY / 2, PS::HP, 1, false>(s.pl + h * (PS::HY / 2) * PS::HP, hy / 2, hp, 1, f.ax,
                                                        s.twx);
    }
  } else {
    staged_copy<NT, 8, cplx<T>>(hy * M, source, [&](int q, cplx<T> v) {
      const int j = (int)dm.div(q), m = q - j * M;
      s.pl[j * hp + m] = v;
    });
    lds_barrier();
    plane_fft<T, PS::M, PS::HY, PS::HP, 1, false>(s.pl, hy, hp, 1, f.ax, s.twx);
  }
  // split of each row into its M + 1 bins, pairs (k, M - k) by one thread
  const int H = M / 2 + 1;
  for (int q = threadIdx.x; q < hy * H; q += NT) {
    const int j = (int)dh.div(q), k = q - j * H;
    cplx<T>* row = s.pl + j * hp;
    if (k == 0) {
      const cplx<T> z0 = row[0];
      row[0] = {z0.x + z0.y, T(0)};
      row[M] = {z0.x - z0.y, T(0)};
    } else {
      const cplx<T> a = row[k], b = row[M - k];
      row[k] = split_fwd(a, b, s.wn[k]);
      if (2 * k != M) row[M - k] = split_fwd(b, a, s.wn[M - k]);
    }
  }
  lds_barrier();
  plane_fft<T, PS::HY, PS::M1, 1, PS::HP, false>(s.pl, M + 1, 1, hp, f.ayh, s.twy);
  // E or O into spectrum rows p ny/2 + k, ky-major: C[run][ky][z][kx], so
  // that the z pass reads contiguous blocks
  cplx<T>* out = spec + (((size_t)slot * f.ny + (size_t)p * hy) * f.nz + z) * f.px;
  const size_t kys = (size_t)f.nz * f.px;
  for (int q = threadIdx.x; q < hy * (M + 1); q += NT) {
    const int ky = (int)dm1.div(q), kx = q - ky * (M + 1);
    out[ky * kys + kx] = s.pl[ky * hp + kx];
  }
}

// The first fin.n workgroups finish the step instead (one per run).
template <typename T, int NX = 0, int NY = 0>
__global__ void __launch_bounds__(kPlaneThreads) k_fft_xy_inv(const cplx<T>* __restrict__ spec, T* __restrict__ phi,
                                                             FftGeom f, FftTables<T> t, FinJob fin) {
  constexpr int NT = kPlaneThreads;
  using PS = PlaneShape<NX, NY>;
  if ((int)blockIdx.x < fin.n) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    finalize_run(fin, (int)blockIdx.x, reinterpret_cast<double*>(smem_raw));
    return;
  }
  const PlaneLds<T> s = plane_lds(f, t);
  const int M = NX ? PS::M : f.ax.L, hy = NY ? PS::HY : f.ny / 2, hp = NX ? PS::HP : f.hp;
  const CDiv<PS::M> dm(M);
  const CDiv<PS::M1> dm1(M + 1);
  const CDiv<PS::H> dh(M / 2 + 1);
  const int b = (int)blockIdx.x - fin.n;
  const int plane = b >> 1, p = b & 1;  // run * nz + z, row parity
  const int slot = plane / f.nz, z = plane - slot * f.nz;
  const cplx<T>* in = spec + (((size_t)slot * f.ny + (size_t)p * hy) * f.nz + z) * f.px;
  const size_t kys = (size_t)f.nz * f.px;
  // e or o (rows p ny/2 + k, left there by the z pass)
  staged_copy<NT, 8, cplx<T>>(
      hy * (M + 1),
      [&](int q) {
        const int ky = (int)dm1.div(q), kx = q - ky * (M + 1);
        return gload(in + ky * kys + kx);
      },
      [&](int q, cplx<T> v) {
        const int ky = (int)dm1.div(q), kx = q - ky * (M + 1);
        s.pl[ky * hp + kx] = v;
      });
  lds_barrier();
  plane_fft<T, PS::HY, PS::M1, 1, PS::HP, true>(s.pl, M + 1, 1, hp, f.ayh, s.twy);
  // complex-to-real split of each row: M + 1 bins -> M packed pairs
  const int H = M / 2 + 1;
  for (int q = threadIdx.x; q < hy * H; q += NT) {
    const int j = (int)dh.div(q), k = q - j * H;
    cplx<T>* row = s.pl + j * hp;
    if (k == 0) {
      const T x0 = row[0].x, xm = row[M].x;  // X[0] and X[M] of a real row are real
      row[0] = {T(0.5) * (x0 + xm), T(0.5) * (x0 - xm)};
    } else {
      const cplx<T> a = row[k], c = row[M - k];
      row[k] = split_inv(a, c, s.wn[k]);
      if (2 * k != M) row[M - k] = split_inv(c, a, s.wn[M - k]);
    }
  }
  lds_barrier();
  plane_fft<T, PS::M, PS::HY, PS::HP, 1, true>(s.pl, hy, hp, 1, f.ax, s.twx);
  // rows 2j + p of phi, M packed pairs each
  cplx<T>* dst = reinterpret_cast<cplx<T>*>(phi) + ((size_t)plane * f.ny + p) * M;
  for (int q = threadIdx.x; q < hy * M; q += NT) {
    const int j = (int)dm.div(q), m = q - j * M;
    dst[(size_t)q + (size_t)j * M] = s.pl[j * hp + m];
  }
}

FftAxis make_axis(int L) {
  FftAxis a{};
  a.L = L;
  int m = L;
  while (m % 8 == 0 && m > 1) { a.rad[a.nst++] = 8; m /= 8; }
  while (m % 4 == 0) { a.rad[a.nst++] = 4; m /= 4; }
  while (m % 2 == 0) { a.rad[a.nst++] = 2; m /= 2; }
  while (m % 3 == 0) { a.rad[a.nst++] = 3; m /= 3; }
  return a;
}

FftGeom make_fft_geom(int nx, int ny, int nz, int nruns, int prec, bool planes) {
  const size_t es = prec == GP_FP64 ? sizeof(double) : sizeof(float);
  const int maxpts = 32768 / (int)(2 * es);
  FftGeom f{};
  f.nx = nx;
  f.ny = ny;
  f.nz = nz;
  f.nruns = nruns;
  f.px = f.nx / 2 + 1;
  f.ax = make_axis(f.nx / 2);
  f.ay = make_axis(f.ny);
  f.az = make_axis(f.nz);
  f.rows_per_block = std::max(1, maxpts / (2 * f.ax.L));
  // columns per workgroup: at most 8 (and the LDS budget), spread evenly
  // over the px = nx/2 + 1 half-spectrum columns so no chunk is nearly empty
  // (8 measured faster than 16, 4 or 2 at 64^3 to 256^3)
  auto even_cols = [&](int L, int cap) {
    const int cmax = std::max(1, std::min({cap, f.px, maxpts / L}));
    const int nch = (f.px + cmax - 1) / cmax;
    return (f.px + nch - 1) / nch;
  };
  f.cols_y = even_cols(f.ay.L, 8);
  // x and y transforms of the even or the odd rows of a z plane per
  // workgroup where two such workgroups fit on a CU (with one per CU the
  // separate x and y passes are faster, e.g. 256^3 FP32)
  f.ayh = make_axis(f.ny / 2);
  f.hp = (f.ax.L + 1) | 1;  // odd row pitch: lanes on neighbouring rows hit other banks
  int dev = 0, lds_dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_dev, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    lds_dev = 0;
  const int lds_max = std::min(kPlaneLdsMax, lds_dev);
  f.plane = planes && 2 * plane_lds_bytes(f, 2 * es) <= (size_t)lds_max;
  if (f.plane) {
    // the plane kernels' dynamic-LDS limit (shared by every size class)
    const hipError_t e = prec == GP_FP64 ? fft_plane_prepare<double>(lds_max) : fft_plane_prepare<float>(lds_max);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      f.plane = 0;
    }
  }
  // the z pass after the plane passes holds the columns of two ky rows, 64
  // bytes of each row per z (4 FP64 or 8 FP32 columns)
  // (exactly 64 bytes where the LDS allows: the same number of blocks as an
  // even spread, since px = nx/2 + 1 is one above a multiple of it)
  f.cols_z = f.plane ? std::max(1, std::min({32 / (int)es, f.px, maxpts / (2 * f.az.L)})) : even_cols(f.az.L, 8);
  f.norm = 2.0 / ((double)f.nx * f.ny * f.nz);
  return f;
}

size_t plane_lds_bytes(const FftGeom& f, size_t csz) {
  const size_t M = f.ax.L;
  return csz * ((size_t)(f.ny / 2) * f.hp + M + M + 1 + f.ny / 2);
}

// The plane passes are instantiated with compile-time shapes for square
// planes of 64, 96 and 128 cells (the benchmarked grids); other sizes run the
// run-time form.
template <typename T, int NX>
static hipError_t plane_prepare_one(int bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy_fwd<T, NX, NX>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy_inv<T, NX, NX>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}

template <typename T>
hipError_t fft_plane_prepare(int bytes) {
  hipError_t e = plane_prepare_one<T, 0>(bytes);
  if (e == hipSuccess) e = plane_prepare_one<T, 64>(bytes);
  if (e == hipSuccess) e = plane_prepare_one<T, 96>(bytes);
  if (e == hipSuccess) e = plane_prepare_one<T, 128>(bytes);
  return e;
}

// Calls fn(std::integral_constant<int, N>) with N the plane size when the
// plane passes have a compile-time instance for f, else with N = 0.
template <typename Fn>
static void with_plane_shape(const FftGeom& f, Fn fn) {
  if (f.nx == f.ny) {
    if (f.nx == 64) return fn(std::integral_constant<int, 64>{});
    if (f.nx == 96) return fn(std::integral_constant<int, 96>{});
    if (f.nx == 128) return fn(std::integral_constant<int, 128>{});
  }
  fn(std::integral_constant<int, 0>{});
}

template <typename T>
void launch_fft_xy_fwd(const SrcSlot* src, int parity, cplx<T>* spec, const FftGeom& f, const FftTables<T>& t,
                       hipStream_t st) {
  with_plane_shape(f, [&](auto n) {
    constexpr int N = decltype(n)::value;
    k_fft_xy_fwd<T, N, N><<<2 * f.nz * f.nruns, kPlaneThreads, plane_lds_bytes(f, sizeof(cplx<T>)), st>>>(
        src, parity, spec, f, t);
  });
}

template <typename T>
void launch_fft_xy_inv(const cplx<T>* spec, T* phi, const FftGeom& f, const FftTables<T>& t, const FinJob& fin,
                       hipStream_t st) {
  size_t lds = plane_lds_bytes(f, sizeof(cplx<T>));
  if (fin.n > 0) lds = std::max(lds, sizeof(double) * kFinLds);
  with_plane_shape(f, [&](auto n) {
    constexpr int N = decltype(n)::value;
    k_fft_xy_inv<T, N, N><<<2 * f.nz * f.nruns + fin.n, kPlaneThreads, lds, st>>>(spec, phi, f, t, fin);
  });
}

static size_t x_lds_bytes(const FftGeom& f, size_t csz, bool inv) {
  const size_t M = f.ax.L, RB = f.rows_per_block;
  return csz * (RB * (M | 1) + (inv ? RB * (M + 1) : 0) + M + M + 1);
}

int fft_blocks_z(const FftGeom& f) { return ((f.px + f.cols_z - 1) / f.cols_z) * f.ny * f.nruns; }

// Calls fn(std::integral_constant<int, N>) with N = nx / 2 when the line
// passes have a compile-time instance for f (rows of 256 and 512 cells, the
// benchmarked line-form grids), else with N = 0.
template <typename T, typename Fn>
static void with_line_shape(const FftGeom& f, Fn fn) {
  constexpr int P = max_points<T>();
  if (f.ax.L == 128 && f.rows_per_block == std::max(1, P / 256)) return fn(std::integral_constant<int, 128>{});
  if (f.ax.L == 256 && f.rows_per_block == std::max(1, P / 512)) return fn(std::integral_constant<int, 256>{});
  fn(std::integral_constant<int, 0>{});
}

template <typename T>
void launch_fft_x_fwd(const SrcSlot* src, int parity, cplx<T>* spec, const FftGeom& f, const FftTables<T>& t,
                      hipStream_t st) {
  const int nrows = f.ny * f.nz * f.nruns;
  const int nblk = (nrows + f.rows_per_block - 1) / f.rows_per_block;
  with_line_shape<T>(f, [&](auto m) {
    constexpr int M = decltype(m)::value;
    constexpr int RB = M ? std::max(1, max_points<T>() / (2 * M)) : 0;
    k_fft_x_fwd<T, M, RB><<<nblk, kFftThreads, x_lds_bytes(f, sizeof(cplx<T>), false), st>>>(src, parity, spec, f,
                                                                                             t);
  });
}

template <typename T>
void launch_fft_x_inv(const cplx<T>* spec, T* phi, const FftGeom& f, const FftTables<T>& t, const FinJob& fin,
                      hipStream_t st) {
  const int nrows = f.ny * f.nz * f.nruns;
  const int nblk = (nrows + f.rows_per_block - 1) / f.rows_per_block + fin.n;
  size_t lds = x_lds_bytes(f, sizeof(cplx<T>), true);
  if (fin.n > 0) lds = std::max(lds, sizeof(double) * kFinLds);
  with_line_shape<T>(f, [&](auto m) {
    constexpr int M = decltype(m)::value;
    constexpr int RB = M ? std::max(1, max_points<T>() / (2 * M)) : 0;
    k_fft_x_inv<T, M, RB><<<nblk, kFftThreads, lds, st>>>(spec, phi, f, t, fin);
  });
}

template <typename T>
void launch_fft_y(cplx<T>* spec, const FftGeom& f, const FftTables<T>& t, bool inverse, hipStream_t st) {
  const int cb = f.cols_y;
  const int nblk = ((f.px + cb - 1) / cb) * f.nz * f.nruns;
  const size_t lds = sizeof(cplx<T>) * ((size_t)cb * f.ay.L + f.ay.L);
  const size_t stride = f.px, outer = (size_t)f.px * f.ny, run = outer * f.nz;
  auto go = [&](auto mode, auto len) {
    constexpr int MODE = decltype(mode)::value, L = decltype(len)::value;
    k_fft_col<T, MODE, L, L ? 8 : 0, L ? 1 : 0><<<nblk, kFftThreads, lds, st>>>(
        spec, f, t, f.ay, t.tw_y, cb, stride, outer, f.nz, run, nullptr, RedJob{}, 0, 0);
  };
  auto with_len = [&](auto mode) {
    if (cb == 8 && f.ay.L == 256) return go(mode, std::integral_constant<int, 256>{});
    if (cb == 8 && f.ay.L == 512) return go(mode, std::integral_constant<int, 512>{});
    go(mode, std::integral_constant<int, 0>{});
  };
  if (inverse)
    with_len(std::integral_constant<int, 1>{});
  else
    with_len(std::integral_constant<int, 0>{});
}

// The z pass with its length and block shape fixed at compile time, for the
// shapes the benchmarked grids use (64 bytes of each of two rows per z after
// the plane passes; 8 columns of one row after the line passes); false if the
// shape has no such instance (the run-time form then runs).
template <typename T, int L, int CB, int NR>
static void z_fixed(int nblk, size_t lds, hipStream_t st, cplx<T>* spec, const FftGeom& f, const FftTables<T>& t,
                    size_t stride, size_t outer, int lines, size_t run, double* ep, const RedJob& red, size_t ps) {
  k_fft_col<T, 2, L, CB, NR><<<nblk, kFftThreads, lds, st>>>(spec, f, t, f.az, t.tw_z, CB, stride, outer, lines,
                                                             run, ep, red, NR == 2, ps);
}

template <typename T>
static bool launch_z_fixed(int nblk, size_t lds, hipStream_t st, cplx<T>* spec, const FftGeom& f,
                           const FftTables<T>& t, int cb, size_t stride, size_t outer, int lines, size_t run,
                           double* ep, const RedJob& red, int nr, size_t ps) {
  constexpr int CP = 32 / (int)sizeof(T);  // columns of 64 bytes
#define GP_Z_FIXED(LL, CBB, NRR)                                                                 \
  if (f.az.L == LL && cb == CBB && nr == NRR) {                                                  \
    z_fixed<T, LL, CBB, NRR>(nblk, lds, st, spec, f, t, stride, outer, lines, run, ep, red, ps); \
    return true;                                                                                 \
  }
  GP_Z_FIXED(64, CP, 2)
  GP_Z_FIXED(96, CP, 2)
  GP_Z_FIXED(128, CP, 2)
  GP_Z_FIXED(256, 8, 1)
  GP_Z_FIXED(512, 8, 1)
#undef GP_Z_FIXED
  return false;
}

template <typename T>
void launch_fft_z_green(cplx<T>* spec, const FftGeom& f, const FftTables<T>& t, double* epot_partials,
                        bool ky_major, const RedJob& red, hipStream_t st) {
  const int cb = f.cols_z;
  // after the plane passes (ky-major) each workgroup pairs rows ky, ky + ny/2
  const int nr = ky_major ? 2 : 1;
  const int lines = f.ny / nr;
  const int nchunks = (f.px + cb - 1) / cb;
  const int nblk = nchunks * lines * f.nruns + red.n;
  const size_t cw = (size_t)nr * cb;
  size_t lds = sizeof(cplx<T>) * (cw * f.az.L + f.az.L) + sizeof(double) * (f.az.L + cw);
  if (red.n > 0) lds = std::max(lds, sizeof(double) * kRedThreads);
  const size_t run = (size_t)f.px * f.ny * f.nz;
  // C[run][z][ky][kx] (line passes) or C[run][ky][z][kx] (plane passes)
  const size_t stride = ky_major ? (size_t)f.px : (size_t)f.px * f.ny;
  const size_t outer = ky_major ? (size_t)f.px * f.nz : (size_t)f.px;
  const size_t ps = (size_t)lines * outer;
  if (!launch_z_fixed<T>(nblk, lds, st, spec, f, t, cb, stride, outer, lines, run, epot_partials, red, nr, ps))
    k_fft_col<T, 2><<<nblk, kFftThreads, lds, st>>>(spec, f, t, f.az, t.tw_z, cb, stride, outer, lines, run,
                                                    epot_partials, red, nr == 2, ps);
}

template void launch_fft_x_fwd<double>(const SrcSlot*, int, cplx<double>*, const FftGeom&,
                                       const FftTables<double>&, hipStream_t);
template void launch_fft_x_fwd<float>(const SrcSlot*, int, cplx<float>*, const FftGeom&, const FftTables<float>&,
                                      hipStream_t);
template void launch_fft_x_inv<double>(const cplx<double>*, double*, const FftGeom&, const FftTables<double>&,
                                       const FinJob&, hipStream_t);
template void launch_fft_x_inv<float>(const cplx<float>*, float*, const FftGeom&, const FftTables<float>&,
                                      const FinJob&, hipStream_t);
template void launch_fft_y<double>(cplx<double>*, const FftGeom&, const FftTables<double>&, bool, hipStream_t);
template void launch_fft_y<float>(cplx<float>*, const FftGeom&, const FftTables<float>&, bool, hipStream_t);
template void launch_fft_z_green<double>(cplx<double>*, const FftGeom&, const FftTables<double>&, double*, bool,
                                         const RedJob&, hipStream_t);
template void launch_fft_z_green<float>(cplx<float>*, const FftGeom&, const FftTables<float>&, double*, bool,
                                        const RedJob&, hipStream_t);

template void launch_fft_xy_fwd<double>(const SrcSlot*, int, cplx<double>*, const FftGeom&,
                                        const FftTables<double>&, hipStream_t);
template void launch_fft_xy_fwd<float>(const SrcSlot*, int, cplx<float>*, const FftGeom&, const FftTables<float>&,
                                       hipStream_t);
template void launch_fft_xy_inv<double>(const cplx<double>*, double*, const FftGeom&, const FftTables<double>&,
                                        const FinJob&, hipStream_t);
template void launch_fft_xy_inv<float>(const cplx<float>*, float*, const FftGeom&, const FftTables<float>&,
                                       const FinJob&, hipStream_t);
template hipError_t fft_plane_prepare<double>(int);
template hipError_t fft_plane_prepare<float>(int);

}  // namespace gp
