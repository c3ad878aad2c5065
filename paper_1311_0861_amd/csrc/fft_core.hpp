// LDS FFT building blocks shared by the Poisson passes (periodic and
// isolated): complex arithmetic, radix-2/3/4/8 butterflies written from the
// DFT definitions, one Stockham autosort stage in LDS, staged global loads,
// the real-to-complex split of a packed transform, and the XCD-aware block
// index of the column passes.
#pragma once

#include "column.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace gp {
constexpr int kFftThreads = 256;     // x passes and column passes
constexpr int kPlaneThreads = 1024;  // xy plane passes

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

// Largest number of complex points one workgroup of the line passes stages
// (32 KiB of LDS), and of the plane passes (the whole LDS of a workgroup).
template <typename T>
constexpr int max_points() {
  return 32768 / (int)sizeof(cplx<T>);
}
template <typename T>
constexpr int plane_points() {
  return kPlaneLdsMax / (int)sizeof(cplx<T>);
}

// Division by a workgroup-uniform d through a multiply-high, exact while
// q * d < 2^32 (the LDS indexes it divides stay below 2^15 and the divisors
// below 2^14): one instruction where the compiler's division by a run-time
// value takes about twenty.
struct FastDiv {
  uint32_t d, m;
  __device__ explicit FastDiv(uint32_t dv) : d(dv), m(dv == 1 ? 0u : 0xffffffffu / dv + 1u) {}
  __device__ __forceinline__ uint32_t div(uint32_t q) const { return d == 1 ? q : __umulhi(q, m); }
};

// One Stockham stage of radix R on `lines` lines of length L, in place: reads
// to registers, barrier, writes, barrier.  Element j of line l sits at
// buf[l * ls + j * es]; at most PMAX points (lines * L) per call.  The line
// index runs fastest across the threads, so neighbouring lanes work on
// neighbouring lines at the same element: one word apart when the lines are
// LDS columns (ls = 1), an odd pitch apart when they are rows (es = 1); either
// way they fall in different banks, and they share their twiddle factor.
template <typename T, int R, int NT, int PMAX>
__device__ void fft_stage(cplx<T>* buf, int lines, int L, int ls, int es, int Ns, const cplx<T>* tw, bool inv) {
  constexpr int MAXB = (PMAX / R + NT - 1) / NT;
  const int nb = L / R;
  const int total = lines * nb;
  const int tstep = L / (Ns * R);
  const FastDiv dline(lines), dns(Ns);
  cplx<T> v[MAXB][R];
  // the thread's indexes are the same in every stage of a radix; computed
  // here rather than hoisted out of the stage loop, where they would all stay
  // live for the whole transform
  const int tid = (int)fresh(threadIdx.x);
#pragma unroll
  for (int b = 0; b < MAXB; b++) {
    const int q = tid + b * NT;
    if (q < total) {
      const int jj = (int)dline.div(q);
      const int line = q - jj * lines;
      const int kk = jj - (int)dns.div(jj) * Ns;
      const cplx<T>* base = buf + line * ls;
#pragma unroll
      for (int r = 0; r < R; r++) {
        cplx<T> x = base[(jj + r * nb) * es];
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
  lds_barrier();
#pragma unroll
  for (int b = 0; b < MAXB; b++) {
    // recomputed rather than held over the barrier beside the butterflies
    const int q = (int)fresh(threadIdx.x) + b * NT;
    if (q < total) {
      const int jj = (int)dline.div(q);
      const int line = q - jj * lines;
      const int jn = (int)dns.div(jj);
      const int kk = jj - jn * Ns;
      cplx<T>* base = buf + line * ls;
      const int d0 = jn * Ns * R + kk;
#pragma unroll
      for (int r = 0; r < R; r++) base[(d0 + r * Ns) * es] = v[b][r];
    }
  }
  lds_barrier();
}

template <typename T, int NT, int PMAX>
__device__ void lds_fft(cplx<T>* buf, int lines, int ls, int es, const FftAxis& ax, const cplx<T>* tw, bool inv) {
  int Ns = 1;
  for (int s = 0; s < ax.nst; s++) {
    const int R = ax.rad[s];
    if (R == 8)
      fft_stage<T, 8, NT, PMAX>(buf, lines, ax.L, ls, es, Ns, tw, inv);
    else if (R == 4)
      fft_stage<T, 4, NT, PMAX>(buf, lines, ax.L, ls, es, Ns, tw, inv);
    else if (R == 3)
      fft_stage<T, 3, NT, PMAX>(buf, lines, ax.L, ls, es, Ns, tw, inv);
    else
      fft_stage<T, 2, NT, PMAX>(buf, lines, ax.L, ls, es, Ns, tw, inv);
    Ns *= R;
  }
}

// ---- transforms whose length and line count are known at compile time -----
// The same Stockham stages as fft_stage (same butterflies, twiddle indexes and
// order of operations, hence the same bits), with every index derived from
// compile-time constants: the run-time form spends most of its instructions
// on 32-bit multiplies and divides of the line count, stride and Ns.

// Radix plan of a length L in make_axis order (8s, then 4s, 2s, 3s).
struct RadPlan {
  int nst;
  int rad[16];
};
constexpr RadPlan rad_plan(int L) {
  RadPlan p{0, {}};
  int m = L;
  while (m % 8 == 0 && m > 1) {
    p.rad[p.nst++] = 8;
    m /= 8;
  }
  while (m % 4 == 0) {
    p.rad[p.nst++] = 4;
    m /= 4;
  }
  while (m % 2 == 0) {
    p.rad[p.nst++] = 2;
    m /= 2;
  }
  while (m % 3 == 0) {
    p.rad[p.nst++] = 3;
    m /= 3;
  }
  return p;
}
// Product of the radices before stage s.
constexpr int rad_ns(int L, int s) {
  const RadPlan p = rad_plan(L);
  int n = 1;
  for (int q = 0; q < s; q++) n *= p.rad[q];
  return n;
}

// One stage on LINES lines of length L, element j of line l at
// buf[l * LS + j * ES], in place.
template <typename T, int R, int NS, int L, int LINES, int LS, int ES, int NT, bool INV>
__device__ __forceinline__ void cstage(cplx<T>* buf, const cplx<T>* tw) {
  constexpr int nb = L / R;
  constexpr int total = LINES * nb;
  constexpr int tstep = L / (NS * R);
  constexpr int MAXB = (total + NT - 1) / NT;
  cplx<T> v[MAXB][R];
  const int tid = (int)threadIdx.x;
#pragma unroll
  for (int b = 0; b < MAXB; b++) {
    const int q = tid + b * NT;
    if (total % NT == 0 || q < total) {
      const int jj = q / LINES, line = q % LINES;
      const int kk = jj % NS;
      const cplx<T>* base = buf + line * LS;
#pragma unroll
      for (int r = 0; r < R; r++) {
        cplx<T> x = base[(jj + r * nb) * ES];
        if (r > 0) {
          cplx<T> w = tw[kk * r * tstep];
          if (INV) w.y = -w.y;
          x = cmul(x, w);
        }
        v[b][r] = x;
      }
      dft_small<T, R>(v[b], INV);
    }
  }
  lds_barrier();
#pragma unroll
  for (int b = 0; b < MAXB; b++) {
    const int q = tid + b * NT;
    if (total % NT == 0 || q < total) {
      const int jj = q / LINES, line = q % LINES;
      const int kk = jj % NS;
      cplx<T>* base = buf + line * LS;
      const int d0 = (jj / NS) * NS * R + kk;
#pragma unroll
      for (int r = 0; r < R; r++) base[(d0 + r * NS) * ES] = v[b][r];
    }
  }
  lds_barrier();
}

// Transform of length L along LINES lines (strides LS, ES): all stages.
template <typename T, int L, int LINES, int LS, int ES, int NT, bool INV, int S = 0>
__device__ __forceinline__ void cfft(cplx<T>* buf, const cplx<T>* tw) {
  constexpr RadPlan p = rad_plan(L);
  if constexpr (S < p.nst) {
    cstage<T, p.rad[S], rad_ns(L, S), L, LINES, LS, ES, NT, INV>(buf, tw);
    cfft<T, L, LINES, LS, ES, NT, INV, S + 1>(buf, tw);
  }
}

// rows (pitch lp, odd) of the line passes
template <typename T>
__device__ __forceinline__ void line_fft(cplx<T>* buf, int lines, int lp, const FftAxis& ax, const cplx<T>* tw,
                                         bool inv) {
  lds_fft<T, kFftThreads, max_points<T>()>(buf, lines, lp, 1, ax, tw, inv);
}

// columns of an LDS block of `cols` columns (row pitch cols)
template <typename T>
__device__ __forceinline__ void col_fft(cplx<T>* buf, int cols, const FftAxis& ax, const cplx<T>* tw, bool inv) {
  lds_fft<T, kFftThreads, max_points<T>()>(buf, cols, 1, cols, ax, tw, inv);
}

// Division by N, or by a run-time divisor (FastDiv) when N = 0.
template <int N>
struct CDiv {
  __device__ explicit CDiv(uint32_t) {}
  __device__ __forceinline__ uint32_t div(uint32_t q) const { return q / N; }
};
template <>
struct CDiv<0> : FastDiv {
  __device__ explicit CDiv(uint32_t d) : FastDiv(d) {}
};

// Rows of a line pass: the compile-time transform when MC, RBC > 0 (the row
// length and the rows per block, which must equal ax.L and the block's row
// count when it is full); a last block with fewer rows, or MC = 0, takes the
// run-time transform.
template <typename T, int MC, int RBC, bool INV>
__device__ __forceinline__ void x_rows_fft(cplx<T>* lds, int rows, int xp, const FftAxis& ax, const cplx<T>* tw) {
  if constexpr (MC > 0) {
    if (rows == RBC) {
      cfft<T, MC, RBC, MC | 1, 1, kFftThreads, INV>(lds, tw);
      return;
    }
  }
  line_fft(lds, rows, xp, ax, tw, INV);
}

template <int NT, typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* dst, const cplx<T>* src, int n) {
  for (int t = threadIdx.x; t < n; t += NT) dst[t] = src[t];
}

// Load through a global-address-space pointer (plain loads of pointers that
// were read from memory compile to flat loads, which also count against the
// LDS wait counter).
template <typename V>
__device__ __forceinline__ V gload(const V* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(1))) V*)p;
#else
  return *p;  // host pass: parsed, never run
#endif
}

// (even, odd) pair of FP64 values, 16-byte aligned (a clang vector type: the
// HIP double2 class copies through a generic-address-space reference)
typedef double dpair __attribute__((ext_vector_type(2)));

// Copies n values from global memory into LDS with up to KB loads in flight
// per thread: get(q) loads (and converts) value q, put(q, v) stores it.  get
// is called for every slot of a batch with q clamped to n - 1, so that the
// loads issue back to back without branches; only the stores are guarded.
template <int NT, int KB, typename V, typename Get, typename Put>
__device__ __forceinline__ void staged_copy(int n, Get get, Put put) {
  for (int q0 = threadIdx.x; q0 < n; q0 += KB * NT) {
    V v[KB];
#pragma unroll
    for (int u = 0; u < KB; u++) v[u] = get(min(q0 + u * NT, n - 1));
#pragma unroll
    for (int u = 0; u < KB; u++) {
      const int q = q0 + u * NT;
      if (q < n) put(q, v[u]);
    }
  }
}

// Real-to-complex split of a packed transform Z (pairs (even, odd) of a real
// row of length 2M): bin k from Z[k] and Z[M - k], with w = exp(-2 pi i k / 2M).
//   X[k] = E + w O,  E = (Z[k] + conj Z[M-k]) / 2,  O = -i (Z[k] - conj Z[M-k]) / 2
template <typename T>
__device__ __forceinline__ cplx<T> split_fwd(cplx<T> zk, cplx<T> zc, cplx<T> w) {
  zc.y = -zc.y;
  const cplx<T> E = {T(0.5) * (zk.x + zc.x), T(0.5) * (zk.y + zc.y)};
  const cplx<T> O = {T(0.5) * (zk.y - zc.y), T(-0.5) * (zk.x - zc.x)};
  return cadd(E, cmul(w, O));
}
// Its inverse: Z[k] = E + i O,  E = (X[k] + conj X[M-k]) / 2,
// O = (X[k] - conj X[M-k]) / 2 * conj(w).
template <typename T>
__device__ __forceinline__ cplx<T> split_inv(cplx<T> xk, cplx<T> xc, cplx<T> w) {
  xc.y = -xc.y;
  const cplx<T> E = {T(0.5) * (xk.x + xc.x), T(0.5) * (xk.y + xc.y)};
  w.y = -w.y;
  const cplx<T> O = cmul({T(0.5) * (xk.x - xc.x), T(0.5) * (xk.y - xc.y)}, w);
  return {E.x - O.y, E.y + O.x};
}

// ---- column passes (y, and the fused z pass) -------------------------------
// A workgroup takes `cb` consecutive kx columns and one index of the other
// transverse axis of one run; line j of column c lives at base + j * stride + c
// with base = run * run_stride + o * outer_stride + kx0 for outer index
// run * outer_div + o.  The chunks of one outer line read neighbouring words
// (rows of the spectrum are not cache-line aligned), so the block index puts
// all chunks of a line on one XCD: blocks go round-robin over the 8 XCDs, and
// in each group of 8 lines the chunk varies slowest.
struct ColBlock {
  int chunk, oline;
};
__device__ __forceinline__ ColBlock col_block(int b, int nchunks, int nolines) {
  const int gsz = 8 * nchunks;
  const int g = b / gsz, rem = b - g * gsz;
  const int r = min(8, nolines - g * 8);  // lines in this group
  const int chunk = rem / r;
  return {chunk, g * 8 + (rem - chunk * r)};
}

}  // namespace gp
