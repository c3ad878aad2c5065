// Lagrangian (FlIC) stage of one GPUPEGAS step (Kulikov, arXiv:1311.0861,
// Sec. 2.1, Fig. "lagrange"), with the end-of-step cell work fused in:
//   - every quantity f obeys (f^{n+1} - f^n)/tau + sum_d (F_{d+} - F_{d-})/h = 0,
//     F on a face = (1/4) sum over its 4 corners of v_d f^+, f^+ the upwind
//     cell value for that corner's velocity; a corner velocity is the mean of
//     the 8 cells sharing the vertex (post-Eulerian m/rho for the gas, q/n for
//     the stars), computed once per vertex by k_vertex; the flux is written per
//     cell as A+ f_c + A- f_{c+e_d};
//   - correctness integrals kappa (Sec. 2.4) measured on the advected state;
//   - energy balance: e := E - |m|^2/(2 rho) where that exceeds eta E, and
//     each diagonal stress Pi_dd := W_dd - q_d^2/n where that exceeds eta W_dd;
//   - per-tile FP64 partial sums for the CFL step and the diagnostics (the
//     Poisson source is formed from rho and n by the first FFT pass).
// rho and n are advected in FP64 with each face flux formed by the same
// operations from both sides, so mass telescopes to rounding in both
// precisions.  The gas and the stars / dark matter advect with their own
// corner velocities and share nothing else in this stage, so each has its own
// kernel (6 and 16 fields), which halves the live state of a joint one.
#include "common.hpp"
#include "kernels.hpp"

namespace gp {

// One component's per-thread partial sums (the kNS slots of its block).
struct Acc {
  double v[kNS];
  uint32_t err;
};

__device__ __forceinline__ void acc_init(Acc& a) {
#pragma unroll
  for (int s = 0; s < kNS; s++) a.v[s] = 0.0;
  a.err = 0u;
}

// Fixed-order block reduction of one component's accumulators into its kNS
// slots of a partial row.
__device__ __forceinline__ void block_reduce_store(Acc& a, gptr<double> slots) {
  __shared__ double red[kBlock / 64][kNS];
  const int tid = threadIdx.x + kTX * threadIdx.y;
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a.v[S_SPEED] = fmax(a.v[S_SPEED], __shfl_xor(a.v[S_SPEED], off, 64));
#pragma unroll
    for (int s = S_MASS; s < S_ERR; s++) a.v[s] += __shfl_xor(a.v[s], off, 64);
    a.err |= (uint32_t)__shfl_xor((int)a.err, off, 64);
  }
  a.v[S_ERR] = (double)a.err;
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < kNS; s++) red[wave][s] = a.v[s];
  }
  __syncthreads();
  if (tid < kNS) {
    constexpr int nw = kBlock / 64;
    double v = red[0][tid];
    if (tid == S_SPEED) {
      for (int w = 1; w < nw; w++) v = fmax(v, red[w][tid]);
    } else if (tid == S_ERR) {
      uint32_t e = (uint32_t)v;
      for (int w = 1; w < nw; w++) e |= (uint32_t)red[w][tid];
      v = (double)e;
    } else {
      for (int w = 1; w < nw; w++) v += red[w][tid];
    }
    slots[tid] = v;
  }
  __syncthreads();  // the next tile of a persistent workgroup reuses red[]
}

// ---- end-of-step cell terms -------------------------------------------------

// Gas: kappa integrand |E - e - |m|^2/(2 rho)| (Sec. 2.4) and kinetic energy.
template <typename T>
__device__ __forceinline__ T gas_kappa(double rho, const T m[3], T E, T e, T& ekin) {
  const T rr = T(rho);
  ekin = (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / (T(2) * rr);
  return fabs(E - e - ekin);
}

// Gas diagnostics of a finished cell: signal speed, sums, error bits.
template <typename T>
__device__ __forceinline__ void gas_terms(Acc& a, double rho, const T m[3], T E, T e, T gamma) {
  const T rr = T(rho);
  const T p = (gamma - T(1)) * e;
  const T cs = sqrt(fmax(gamma * p / rr, T(0)));
  T sp = T(0);
#pragma unroll
  for (int d = 0; d < 3; d++) sp = fmax(sp, fabs(m[d] / rr) + cs);
  a.v[S_SPEED] = fmax(a.v[S_SPEED], (double)sp);
  a.v[S_MASS] += rho;
#pragma unroll
  for (int d = 0; d < 3; d++) a.v[S_MOMX + d] += (double)m[d];
  a.v[S_ENERGY] += (double)E;
  bool fin = isfinite(rho) && isfinite(E) && isfinite(e);
#pragma unroll
  for (int d = 0; d < 3; d++) fin = fin && isfinite(m[d]);
  uint32_t err = 0u;
  if (!fin) err |= ERR_NONFINITE;
  if (!(rho > 0.0)) err |= ERR_DENSITY;
  if (!(p > T(0))) err |= ERR_PRESSURE;
  a.err |= err;
}

// Stars / dark matter: thermal tensor T = W - q q / n and the kappa integrand
// sum_ij |T_ij - Pi_ij| (Sec. 2.4).
template <typename T>
__device__ __forceinline__ T bme_kappa(double n, const T q[3], const T P[6], const T W[6], T Tt[6]) {
  const T rn = T(n);
  T kb = T(0);
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = a; b < 3; b++) {
      const int s = sym(a, b);
      Tt[s] = W[s] - q[a] * q[b] / rn;
      kb += fabs(Tt[s] - P[s]);
    }
  return kb;
}

template <typename T>
__device__ __forceinline__ void bme_terms(Acc& a, double n, const T q[3], const T P[6], const T W[6]) {
  const T rn = T(n);
  T sp = T(0);
#pragma unroll
  for (int d = 0; d < 3; d++) sp = fmax(sp, fabs(q[d] / rn) + sqrt(fmax(T(3) * P[sym(d, d)] / rn, T(0))));
  a.v[S_SPEED] = fmax(a.v[S_SPEED], (double)sp);
  a.v[S_MASS] += n;
#pragma unroll
  for (int d = 0; d < 3; d++) a.v[S_MOMX + d] += (double)q[d];
  a.v[S_ENERGY] += 0.5 * ((double)W[0] + (double)W[3] + (double)W[5]);
  bool fin = isfinite(n);
#pragma unroll
  for (int d = 0; d < 3; d++) fin = fin && isfinite(q[d]);
#pragma unroll
  for (int s = 0; s < 6; s++) fin = fin && isfinite(P[s]) && isfinite(W[s]);
  uint32_t err = 0u;
  if (!fin) err |= ERR_NONFINITE;
  if (!(n > 0.0)) err |= ERR_DENSITY;
  if (!(P[0] > T(0)) || !(P[3] > T(0)) || !(P[5] > T(0))) err |= ERR_STRESS;
  a.err |= err;
}

// Corner velocities: vertex (I, J, K), I in [0, nx], sits between cells I-1
// and I on x (likewise y, z); its velocity is the mean of the 8 cells sharing
// it, cells outside the grid taken by the hydrodynamic boundary rule.  The
// post-Eulerian momentum slots hold velocities already.
template <typename T>
__device__ __forceinline__ void vertex_point(const Fields<T>& eul, gptr<T> vtx, const Grid& g,
                                             size_t vstride, int I, int J, int K) {
  const size_t nx = g.nx, nxy = (size_t)g.nx * g.ny;
  const size_t xi[2] = {(size_t)bc_index(I - 1, g.nx, g.bc[0]), (size_t)bc_index(I, g.nx, g.bc[0])};
  const size_t yj[2] = {nx * bc_index(J - 1, g.ny, g.bc[1]), nx * bc_index(J, g.ny, g.bc[1])};
  const size_t zk[2] = {nxy * bc_index(K - 1, g.nz, g.bc[2]), nxy * bc_index(K, g.nz, g.bc[2])};
  T acc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int c3 = 0; c3 < 2; c3++)
#pragma unroll
    for (int b3 = 0; b3 < 2; b3++)
#pragma unroll
      for (int a3 = 0; a3 < 2; a3++) {
        const size_t cc = xi[a3] + yj[b3] + zk[c3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
          acc[d] += eul.o[oidx(GP_MX + d)][cc];
          acc[3 + d] += eul.o[oidx(GP_QX + d)][cc];
        }
      }
  const size_t w = I + (size_t)(g.nx + 1) * (J + (size_t)(g.ny + 1) * K);
#pragma unroll
  for (int v = 0; v < 6; v++) vtx[v * vstride + w] = acc[v] * T(0.125);
}

// Vertices are processed in flat index order, kBlock per work item, so every
// wave writes 64 consecutive vertices whatever the (nx+1) row length.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_vertex(const RunDev<T>* __restrict__ runs,
                                                   const WorkItem* __restrict__ work, unsigned nwork) {
  const WorkRange wr = xcd_range(nwork);
  const unsigned tid = threadIdx.x + kTX * threadIdx.y;
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const int run = uniform(work[w].run), tile = uniform(work[w].tile);
    const RunDev<T>& R = runs[run];
    const unsigned vx = R.g.nx + 1, vy = R.g.ny + 1;
    const size_t v = (size_t)tile * kBlock + tid;
    if (v < (size_t)vx * vy * (R.g.nz + 1)) {
      const unsigned I = (unsigned)(v % vx);
      const size_t JK = v / vx;
      const unsigned J = (unsigned)(JK % vy), K = (unsigned)(JK / vy);
      vertex_point<T>(fields_eul(R), as_global(R.vtx), R.g, R.vstride, (int)I, (int)J, (int)K);
    }
  }
}

// ---- Lagrangian cell update -------------------------------------------------

// Corners of cell (i, j, k): vertex planes k and k+1 (uniform) and the four
// in-plane vertices (i, j), (i+1, j), (i, j+1), (i+1, j+1).
struct VtxStencil {
  size_t z[2];
  uint32_t xy[4];
};

__device__ __forceinline__ VtxStencil make_vtx_stencil(const Grid& g, int i, int j, int k) {
  VtxStencil v;
  const uint32_t vx = (uint32_t)g.nx + 1;
  const size_t vxy = (size_t)vx * (size_t)(g.ny + 1);
  v.z[0] = vxy * (size_t)k;
  v.z[1] = vxy * (size_t)(k + 1);
  v.xy[0] = (uint32_t)i + vx * (uint32_t)j;
  v.xy[1] = v.xy[0] + 1u;
  v.xy[2] = v.xy[0] + vx;
  v.xy[3] = v.xy[2] + 1u;
  return v;
}

// A+ / A- of the six faces from the corner velocities of one component
// (components c0 .. c0+2 of the corner array): [axis][side], side 0 = minus
// face, 1 = plus face.  Corner s = sx + 2 sy + 4 sz is vertex (i + sx, j + sy,
// k + sz); a face normal to d on side `side` has the 4 corners with
// s_d = side, summed in increasing s -- the same order from both cells that
// share the face.
template <typename T>
__device__ __forceinline__ void face_coeffs(gptr<const T> vtx, size_t vstride, int c0, const VtxStencil& V,
                                            T ap[3][2], T am[3][2]) {
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const gptr<const T> comp = vtx + (size_t)(c0 + d) * vstride;
    T pos[2] = {T(0), T(0)}, neg[2] = {T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 8; s++) {
      const int sx = s & 1, sy = (s >> 1) & 1, sz = (s >> 2) & 1;
      const T v = ld_at(comp, V.z[sz], V.xy[sx + 2 * sy]);
      const int side = d == 0 ? sx : (d == 1 ? sy : sz);
      pos[side] += fmax(v, T(0));
      neg[side] += fmin(v, T(0));
    }
#pragma unroll
    for (int side = 0; side < 2; side++) {
      ap[d][side] = pos[side] * T(0.25);
      am[d][side] = neg[side] * T(0.25);
    }
  }
}

// Face flux of an FP64 density; both cells sharing the face evaluate exactly
// this expression with the same operands.
__device__ __forceinline__ double face_flux(double ap, double am, double fl, double fr) {
  return __fma_rn(ap, fl, __dmul_rn(am, fr));
}

// Advected FP64 density of the centre cell from its 7-point values dn[], and
// the flux leaving the grid through outflow faces (per unit area and time).
template <typename T>
__device__ __forceinline__ double advect_density(const double dn[7], const T ap[3][2], const T am[3][2], double rd,
                                                 const Grid& g, int i, int j, int k, double& out) {
  const int ci[3] = {i, j, k};
  const int nn[3] = {g.nx, g.ny, g.nz};
  double div = 0.0;
  out = 0.0;
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const double Fp = face_flux(ap[d][1], am[d][1], dn[0], dn[2 + 2 * d]);
    const double Fm = face_flux(ap[d][0], am[d][0], dn[1 + 2 * d], dn[0]);
    div += Fp - Fm;
    if (g.bc[d] == GP_BC_OUTFLOW) {
      if (ci[d] == nn[d] - 1) out += Fp;
      if (ci[d] == 0) out -= Fm;
    }
  }
  return dn[0] - rd * div;
}

// 7-point weights of the flux update of every field of a component.
template <typename T>
struct Weights {
  T c, p[3], m[3];
};
template <typename T>
__device__ __forceinline__ Weights<T> flux_weights(const T ap[3][2], const T am[3][2], T r) {
  Weights<T> w;
  w.c = T(1);
#pragma unroll
  for (int d = 0; d < 3; d++) {
    w.c -= r * (ap[d][1] - am[d][0]);
    w.p[d] = -r * am[d][1];
    w.m[d] = r * ap[d][0];
  }
  return w;
}

// Flux update of one field from its post-Eulerian 7-point values; a momentum
// slot holds a velocity and is multiplied by the density of the same point.
template <bool kMom, typename T>
__device__ __forceinline__ T advect(gptr<const T> f, const Stencil& s, const Weights<T>& w, const double dn[7]) {
  T x[7];
  x[0] = ld_pt<0>(f, s);
  x[1] = ld_pt<1>(f, s);
  x[2] = ld_pt<2>(f, s);
  x[3] = ld_pt<3>(f, s);
  x[4] = ld_pt<4>(f, s);
  x[5] = ld_pt<5>(f, s);
  x[6] = ld_pt<6>(f, s);
  if constexpr (kMom) {
#pragma unroll
    for (int p = 0; p < 7; p++) x[p] *= (T)dn[p];
  }
  T v = w.c * x[0];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    v += w.p[d] * x[2 + 2 * d];
    v += w.m[d] * x[1 + 2 * d];
  }
  return v;
}

__device__ __forceinline__ void load_density(double dn[7], gptr<const double> f, const Stencil& s) {
  dn[0] = ld_pt<0>(f, s);
  dn[1] = ld_pt<1>(f, s);
  dn[2] = ld_pt<2>(f, s);
  dn[3] = ld_pt<3>(f, s);
  dn[4] = ld_pt<4>(f, s);
  dn[5] = ld_pt<5>(f, s);
  dn[6] = ld_pt<6>(f, s);
}

// Gas: rho, m, E, e of cell (i, j, k).
template <typename T>
__device__ __forceinline__ void lag_gas_cell(Acc& acc, const RunDev<T>& R, int parity, double tau_d, int i, int j,
                                             int k) {
  const Grid& g = R.g;
  const double rd = tau_d / g.h;
  const Stencil s = make_stencil(g, i, j, k, false);
  T ap[3][2], am[3][2];
  face_coeffs(as_global((const T*)R.vtx), R.vstride, 0, make_vtx_stencil(g, i, j, k), ap, am);
  double dn[7];
  load_density(dn, as_global((const double*)R.dens[parity][0]), s);
  double outg;
  const double rho = advect_density(dn, ap, am, rd, g, i, j, k, outg);
  const Weights<T> w = flux_weights(ap, am, (T)rd);

  T m[3];
#pragma unroll
  for (int d = 0; d < 3; d++) m[d] = advect<true>(as_global((const T*)R.tmp[oidx(GP_MX + d)]), s, w, dn);
  const T E = advect<false>(as_global((const T*)R.tmp[oidx(GP_E)]), s, w, dn);
  T e = advect<false>(as_global((const T*)R.tmp[oidx(GP_EINT)]), s, w, dn);

  // correctness integral, then the energy balance
  T ekin;
  acc.v[S_KAPPA] += (double)gas_kappa(rho, m, E, e, ekin);
  if (R.ph.eta >= 0.0) {
    const T et = E - ekin;
    if (et > (T)R.ph.eta * E) {
      e = et;
      acc.v[S_NSYNC] += 1.0;
    }
  }
  acc.v[S_OUTFLOW] += outg;

  const size_t z = s.z[1];
  const uint32_t xy = s.xy[0];
  st_at(as_global(R.dens[parity ^ 1][0]), z, xy, rho);
#pragma unroll
  for (int d = 0; d < 3; d++) st_at(as_global(R.cur[oidx(GP_MX + d)]), z, xy, m[d]);
  st_at(as_global(R.cur[oidx(GP_E)]), z, xy, E);
  st_at(as_global(R.cur[oidx(GP_EINT)]), z, xy, e);
  gas_terms(acc, rho, m, E, e, (T)R.ph.gamma);
}

// Stars / dark matter: n, q, Pi, W of cell (i, j, k).
template <typename T>
__device__ __forceinline__ void lag_bme_cell(Acc& acc, const RunDev<T>& R, int parity, double tau_d, int i, int j,
                                             int k) {
  const Grid& g = R.g;
  const double rd = tau_d / g.h;
  const Stencil s = make_stencil(g, i, j, k, false);
  T ap[3][2], am[3][2];
  face_coeffs(as_global((const T*)R.vtx), R.vstride, 3, make_vtx_stencil(g, i, j, k), ap, am);
  double dn[7];
  load_density(dn, as_global((const double*)R.dens[parity][1]), s);
  double outb;
  const double n = advect_density(dn, ap, am, rd, g, i, j, k, outb);
  const Weights<T> w = flux_weights(ap, am, (T)rd);

  T q[3], P[6], W[6];
#pragma unroll
  for (int d = 0; d < 3; d++) q[d] = advect<true>(as_global((const T*)R.tmp[oidx(GP_QX + d)]), s, w, dn);
#pragma unroll
  for (int m = 0; m < 6; m++) {
    P[m] = advect<false>(as_global((const T*)R.tmp[oidx(GP_PXX + m)]), s, w, dn);
    W[m] = advect<false>(as_global((const T*)R.tmp[oidx(GP_WXX + m)]), s, w, dn);
  }

  // correctness integral, then the energy balance of each diagonal stress
  T Tt[6];
  acc.v[S_KAPPA] += (double)bme_kappa(n, q, P, W, Tt);
  if (R.ph.eta >= 0.0) {
    const T eta = (T)R.ph.eta;
    bool any = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int m = sym(d, d);
      if (Tt[m] > eta * W[m]) {
        P[m] = Tt[m];
        any = true;
      }
    }
    if (any) acc.v[S_NSYNC] += 1.0;
  }
  acc.v[S_OUTFLOW] += outb;

  const size_t z = s.z[1];
  const uint32_t xy = s.xy[0];
  st_at(as_global(R.dens[parity ^ 1][1]), z, xy, n);
#pragma unroll
  for (int d = 0; d < 3; d++) st_at(as_global(R.cur[oidx(GP_QX + d)]), z, xy, q[d]);
#pragma unroll
  for (int m = 0; m < 6; m++) {
    st_at(as_global(R.cur[oidx(GP_PXX + m)]), z, xy, P[m]);
    st_at(as_global(R.cur[oidx(GP_WXX + m)]), z, xy, W[m]);
  }
  bme_terms(acc, n, q, P, W);
}

template <int C, typename T>
__global__ void __launch_bounds__(kBlock) k_lagrangian(const RunDev<T>* __restrict__ runs,
                                                       const WorkItem* __restrict__ work, unsigned nwork,
                                                       int parity, double* __restrict__ partials) {
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const int run = uniform(work[w].run), tile = uniform(work[w].tile);
    const RunDev<T>& R = runs[run];
    const TileCell c = tile_cell(R, tile);
    Acc acc;
    acc_init(acc);
    if (c.inside) {
      if constexpr (C == COMP_GAS)
        lag_gas_cell<T>(acc, R, parity, R.sc->dt, c.i, c.j, c.k);
      else
        lag_bme_cell<T>(acc, R, parity, R.sc->dt, c.i, c.j, c.k);
    }
    block_reduce_store(acc, as_global(partials) + ((size_t)R.row0 + tile) * kNP + C * kNS);
  }
}

// Diagnostics terms of one cell of a state that has not been advanced.
template <typename T>
__device__ __forceinline__ void init_cell(Acc& ga, Acc& ba, const RunDev<T>& R, int parity, int i, int j, int k) {
  const Stencil s = make_stencil(R.g, i, j, k, false);
  const size_t z = s.z[1];
  const uint32_t xy = s.xy[0];
  auto f = [&](int field) { return ld_at(as_global((const T*)R.cur[oidx(field)]), z, xy); };
  const double rho = ld_at(as_global((const double*)R.dens[parity][0]), z, xy);
  const double n = ld_at(as_global((const double*)R.dens[parity][1]), z, xy);
  T m[3], q[3], P[6], W[6];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    m[d] = f(GP_MX + d);
    q[d] = f(GP_QX + d);
  }
#pragma unroll
  for (int a = 0; a < 6; a++) {
    P[a] = f(GP_PXX + a);
    W[a] = f(GP_WXX + a);
  }
  const T E = f(GP_E), e = f(GP_EINT);
  T ekin, Tt[6];
  ga.v[S_KAPPA] += (double)gas_kappa(rho, m, E, e, ekin);
  ba.v[S_KAPPA] += (double)bme_kappa(n, q, P, W, Tt);
  gas_terms(ga, rho, m, E, e, (T)R.ph.gamma);
  bme_terms(ba, n, q, P, W);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_partials(const RunDev<T>* __restrict__ runs,
                                                          const WorkItem* __restrict__ work, unsigned nwork,
                                                          int parity, double* __restrict__ partials) {
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const int run = uniform(work[w].run), tile = uniform(work[w].tile);
    const RunDev<T>& R = runs[run];
    const TileCell c = tile_cell(R, tile);
    Acc ga, ba;
    acc_init(ga);
    acc_init(ba);
    if (c.inside) init_cell<T>(ga, ba, R, parity, c.i, c.j, c.k);
    const gptr<double> row = as_global(partials) + ((size_t)R.row0 + tile) * kNP;
    block_reduce_store(ga, row + kGasSlots);
    block_reduce_store(ba, row + kBmeSlots);
  }
}

template <typename T>
void launch_vertex(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, unsigned nblocks, hipStream_t st) {
  k_vertex<T><<<nblocks, dim3(kTX, kTY, 1), 0, st>>>(runs, work, nwork);
}
template <typename T>
void launch_lagrangian(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity, double* partials,
                       int comp, unsigned nblocks, hipStream_t st) {
  if (comp == COMP_GAS)
    k_lagrangian<COMP_GAS, T><<<nblocks, dim3(kTX, kTY, 1), 0, st>>>(runs, work, nwork, parity, partials);
  else
    k_lagrangian<COMP_BME, T><<<nblocks, dim3(kTX, kTY, 1), 0, st>>>(runs, work, nwork, parity, partials);
}
template <typename T>
void launch_init_partials(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity,
                          double* partials, unsigned nblocks, hipStream_t st) {
  k_init_partials<T><<<nblocks, dim3(kTX, kTY, 1), 0, st>>>(runs, work, nwork, parity, partials);
}
#define GP_INSTANTIATE(T)                                                                                  \
  template void launch_vertex<T>(const RunDev<T>*, const WorkItem*, unsigned, unsigned, hipStream_t);       \
  template void launch_lagrangian<T>(const RunDev<T>*, const WorkItem*, unsigned, int, double*, int,        \
                                     unsigned, hipStream_t);                                                \
  template void launch_init_partials<T>(const RunDev<T>*, const WorkItem*, unsigned, int, double*, unsigned, \
                                        hipStream_t);
GP_INSTANTIATE(double)
GP_INSTANTIATE(float)
#undef GP_INSTANTIATE

}  // namespace gp
