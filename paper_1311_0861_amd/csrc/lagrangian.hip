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
// precisions.
#include "common.hpp"
#include "kernels.hpp"

namespace gp {

struct CellAcc {
  double v[kNP];
  uint32_t err;
};

__device__ __forceinline__ void acc_init(CellAcc& a) {
#pragma unroll
  for (int s = 0; s < kNP; s++) a.v[s] = 0.0;
  a.err = 0u;
}

// Diagnostics terms of one cell of a finished state.
template <typename T>
__device__ __forceinline__ void cell_terms(CellAcc& a, double rho, double n, const T m[3], T E, T e,
                                           const T q[3], const T P[6], const T W[6], T gamma) {
  const T rr = T(rho), rn = T(n);
  const T p = (gamma - T(1)) * e;
  const T cs = sqrt(fmax(gamma * p / rr, T(0)));
  T sp = T(0);
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const T cg = fabs(m[d] / rr) + cs;
    const T cb = fabs(q[d] / rn) + sqrt(fmax(T(3) * P[sym(d, d)] / rn, T(0)));
    sp = fmax(sp, fmax(cg, cb));
  }
  a.v[P_SPEED] = fmax(a.v[P_SPEED], (double)sp);
  a.v[P_MGAS] += rho;
  a.v[P_MBME] += n;
#pragma unroll
  for (int d = 0; d < 3; d++) a.v[P_MOMX + d] += (double)m[d] + (double)q[d];
  a.v[P_EGAS] += (double)E;
  a.v[P_EBME] += 0.5 * ((double)W[0] + (double)W[3] + (double)W[5]);

  uint32_t err = 0u;
  bool fin = isfinite(rho) && isfinite(n) && isfinite(E) && isfinite(e);
#pragma unroll
  for (int d = 0; d < 3; d++) fin = fin && isfinite(m[d]) && isfinite(q[d]);
#pragma unroll
  for (int s = 0; s < 6; s++) fin = fin && isfinite(P[s]) && isfinite(W[s]);
  if (!fin) err |= ERR_NONFINITE;
  if (!(rho > 0.0) || !(n > 0.0)) err |= ERR_DENSITY;
  if (!(p > T(0))) err |= ERR_PRESSURE;
  if (!(P[0] > T(0)) || !(P[3] > T(0)) || !(P[5] > T(0))) err |= ERR_STRESS;
  a.err |= err;
}

// Correctness integrands of Sec. 2.4 and the thermal tensor T = W - q q / n.
template <typename T>
__device__ __forceinline__ void kappa_terms(double rho, double n, const T m[3], T E, T e, const T q[3],
                                            const T P[6], const T W[6], T& ekin, T Tt[6], T& kg,
                                            T& kb) {
  const T rr = T(rho), rn = T(n);
  ekin = (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / (T(2) * rr);
  kg = fabs(E - e - ekin);
  kb = T(0);
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = a; b < 3; b++) {
      const int s = sym(a, b);
      Tt[s] = W[s] - q[a] * q[b] / rn;
      kb += fabs(Tt[s] - P[s]);
    }
}

// Fixed-order block reduction of the cell accumulators into one partial row.
__device__ __forceinline__ void block_reduce_store(CellAcc& a, gptr<double> row) {
  __shared__ double red[(kTX * kTY) / 64][kNP];
  const int tid = threadIdx.x + kTX * threadIdx.y;
  const int lane = tid & 63, wave = tid >> 6;
  a.v[P_ERR] = (double)a.err;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a.v[P_SPEED] = fmax(a.v[P_SPEED], __shfl_xor(a.v[P_SPEED], off, 64));
#pragma unroll
    for (int s = P_MGAS; s < P_ERR; s++) a.v[s] += __shfl_xor(a.v[s], off, 64);
    a.err |= (uint32_t)__shfl_xor((int)a.err, off, 64);
  }
  a.v[P_ERR] = (double)a.err;
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < kNP; s++) red[wave][s] = a.v[s];
  }
  __syncthreads();
  if (tid < kNP) {
    constexpr int nw = (kTX * kTY) / 64;
    double v = red[0][tid];
    if (tid == P_SPEED) {
      for (int w = 1; w < nw; w++) v = fmax(v, red[w][tid]);
    } else if (tid == P_ERR) {
      uint32_t e = (uint32_t)v;
      for (int w = 1; w < nw; w++) e |= (uint32_t)red[w][tid];
      v = (double)e;
    } else {
      for (int w = 1; w < nw; w++) v += red[w][tid];
    }
    row[tid] = v;
  }
  __syncthreads();  // the next tile of a persistent workgroup reuses red[]
}

// Face flux of an FP64 density; both cells sharing the face evaluate exactly
// this expression with the same operands.
__device__ __forceinline__ double face_flux(double ap, double am, double fl, double fr) {
  return __fma_rn(ap, fl, __dmul_rn(am, fr));
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

// One cell of the Lagrangian stage and its end-of-step work.
template <typename T>
__device__ __forceinline__ void lagrangian_cell(CellAcc& acc, const Fields<T>& cur, const Fields<T>& eul,
                                                const Fields<T>& out, gptr<const T> vtx, size_t vstride,
                                                const Grid& g, const Phys& ph, double tau_d, int i, int j,
                                                int k) {
  const size_t nx = g.nx, nxy = (size_t)g.nx * g.ny;
  const double rd = tau_d / g.h;
  const T r = (T)rd;
  const T gamma = (T)ph.gamma;
  const size_t xi[3] = {(size_t)bc_index(i - 1, g.nx, g.bc[0]), (size_t)i,
                        (size_t)bc_index(i + 1, g.nx, g.bc[0])};
  const size_t yj[3] = {nx * bc_index(j - 1, g.ny, g.bc[1]), nx * j,
                        nx * bc_index(j + 1, g.ny, g.bc[1])};
  const size_t zk[3] = {nxy * bc_index(k - 1, g.nz, g.bc[2]), nxy * k,
                        nxy * bc_index(k + 1, g.nz, g.bc[2])};
  const size_t c = xi[1] + yj[1] + zk[1];

  // A+ / A- on the six faces: [axis][side], side 0 = minus face, 1 = plus face.
  // Corner s = sx + 2 sy + 4 sz is vertex (i + sx, j + sy, k + sz); a face
  // normal to d on side `side` has the 4 corners with s_d = side.
  const size_t vx = g.nx + 1, vxy = (size_t)(g.nx + 1) * (g.ny + 1);
  const size_t w0 = i + vx * j + vxy * k;
  T apg[3][2], amg[3][2], apb[3][2], amb[3][2];
#pragma unroll
  for (int d = 0; d < 3; d++)
#pragma unroll
    for (int side = 0; side < 2; side++) {
      T pg = T(0), ng = T(0), pb = T(0), nb = T(0);
#pragma unroll
      for (int s = 0; s < 8; s++) {
        if (((s >> d) & 1) != side) continue;
        const size_t w = w0 + (s & 1) + vx * ((s >> 1) & 1) + vxy * ((s >> 2) & 1);
        const T vgd = vtx[d * vstride + w], vbd = vtx[(3 + d) * vstride + w];
        pg += fmax(vgd, T(0));
        ng += fmin(vgd, T(0));
        pb += fmax(vbd, T(0));
        nb += fmin(vbd, T(0));
      }
      apg[d][side] = pg * T(0.25);
      amg[d][side] = ng * T(0.25);
      apb[d][side] = pb * T(0.25);
      amb[d][side] = nb * T(0.25);
    }

  // neighbour indices along each axis
  const size_t cmn[3] = {xi[0] + yj[1] + zk[1], xi[1] + yj[0] + zk[1], xi[1] + yj[1] + zk[0]};
  const size_t cpl[3] = {xi[2] + yj[1] + zk[1], xi[1] + yj[2] + zk[1], xi[1] + yj[1] + zk[2]};
  const int ci[3] = {i, j, k};
  const int nn[3] = {g.nx, g.ny, g.nz};

  // densities at the 7 points: centre, then minus / plus neighbour per axis
  double rh[7], nd[7];
  rh[0] = cur.rho[c];
  nd[0] = cur.nb[c];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    rh[1 + 2 * d] = cur.rho[cmn[d]];
    rh[2 + 2 * d] = cur.rho[cpl[d]];
    nd[1 + 2 * d] = cur.nb[cmn[d]];
    nd[2 + 2 * d] = cur.nb[cpl[d]];
  }
  // explicit FP64 face fluxes of rho and n, and the boundary outflow
  double divr = 0.0, divn = 0.0, outg = 0.0, outb = 0.0;
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const double Fp = face_flux(apg[d][1], amg[d][1], rh[0], rh[2 + 2 * d]);
    const double Fm = face_flux(apg[d][0], amg[d][0], rh[1 + 2 * d], rh[0]);
    const double Gp = face_flux(apb[d][1], amb[d][1], nd[0], nd[2 + 2 * d]);
    const double Gm = face_flux(apb[d][0], amb[d][0], nd[1 + 2 * d], nd[0]);
    divr += Fp - Fm;
    divn += Gp - Gm;
    if (g.bc[d] == GP_BC_OUTFLOW) {
      if (ci[d] == nn[d] - 1) { outg += Fp; outb += Gp; }
      if (ci[d] == 0) { outg -= Fm; outb -= Gm; }
    }
  }
  const double rho = rh[0] - rd * divr;
  const double n = nd[0] - rd * divn;

  // other fields: 7-point stencil with the same face coefficients; the
  // momenta are rebuilt as density times post-Eulerian velocity
  T wcg = T(1), wcb = T(1), wpg[3], wmg[3], wpb[3], wmb[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    wcg -= r * (apg[d][1] - amg[d][0]);
    wcb -= r * (apb[d][1] - amb[d][0]);
    wpg[d] = -r * amg[d][1];
    wmg[d] = r * apg[d][0];
    wpb[d] = -r * amb[d][1];
    wmb[d] = r * apb[d][0];
  }
  T nv[kNO];
#pragma unroll
  for (int f = 0; f < kNO; f++) {
    const auto src = eul.o[f];
    const bool gas = f < oidx(GP_N + 1);  // mx my mz E e
    const bool gmom = f <= oidx(GP_MZ);
    const bool bmom = f >= oidx(GP_QX) && f <= oidx(GP_QZ);
    auto val = [&](int p, size_t idx) -> T {
      const T x = src[idx];
      return gmom ? (T)rh[p] * x : (bmom ? (T)nd[p] * x : x);
    };
    const T wc = gas ? wcg : wcb;
    T v = wc * val(0, c);
#pragma unroll
    for (int d = 0; d < 3; d++) {
      v += (gas ? wpg[d] : wpb[d]) * val(2 + 2 * d, cpl[d]);
      v += (gas ? wmg[d] : wmb[d]) * val(1 + 2 * d, cmn[d]);
    }
    nv[f] = v;
  }

  // energy balance and correctness integrals
  T m[3] = {nv[oidx(GP_MX)], nv[oidx(GP_MY)], nv[oidx(GP_MZ)]};
  T q[3] = {nv[oidx(GP_QX)], nv[oidx(GP_QY)], nv[oidx(GP_QZ)]};
  T E = nv[oidx(GP_E)], e = nv[oidx(GP_EINT)];
  T P[6], W[6];
#pragma unroll
  for (int s = 0; s < 6; s++) {
    P[s] = nv[oidx(GP_PXX + s)];
    W[s] = nv[oidx(GP_WXX + s)];
  }
  T ekin, Tt[6], kg, kb;
  kappa_terms(rho, n, m, E, e, q, P, W, ekin, Tt, kg, kb);
  acc.v[P_KGAS] += (double)kg;
  acc.v[P_KBME] += (double)kb;
  if (ph.eta >= 0.0) {
    const T eta = (T)ph.eta;
    const T et = E - ekin;
    if (et > eta * E) {
      e = et;
      acc.v[P_SYNCG] += 1.0;
    }
    bool any = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int s = sym(d, d);
      if (Tt[s] > eta * W[s]) {
        P[s] = Tt[s];
        any = true;
      }
    }
    if (any) acc.v[P_SYNCB] += 1.0;
  }
  acc.v[P_OUTG] += outg;
  acc.v[P_OUTB] += outb;

  out.rho[c] = rho;
  out.nb[c] = n;
#pragma unroll
  for (int d = 0; d < 3; d++) {
    out.o[oidx(GP_MX + d)][c] = m[d];
    out.o[oidx(GP_QX + d)][c] = q[d];
  }
  out.o[oidx(GP_E)][c] = E;
  out.o[oidx(GP_EINT)][c] = e;
#pragma unroll
  for (int s = 0; s < 6; s++) {
    out.o[oidx(GP_PXX + s)][c] = P[s];
    out.o[oidx(GP_WXX + s)][c] = W[s];
  }
  cell_terms(acc, rho, n, m, E, e, q, P, W, gamma);
}

template <typename T>
__global__ void __launch_bounds__(kBlock, 3) k_lagrangian(const RunDev<T>* __restrict__ runs,
                                                       const WorkItem* __restrict__ work, unsigned nwork,
                                                       int parity, double* __restrict__ partials) {
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const int run = uniform(work[w].run), tile = uniform(work[w].tile);
    const RunDev<T>& R = runs[run];
    const int ntx = R.ntx, nty = R.nty;
    const int i = (tile % ntx) * kTX + threadIdx.x;
    const int j = ((tile / ntx) % nty) * kTY + threadIdx.y;
    const int k = tile / (ntx * nty);
    CellAcc acc;
    acc_init(acc);
    if (i < R.g.nx && j < R.g.ny)
      lagrangian_cell<T>(acc, fields_state(R, parity), fields_eul(R), fields_next(R, parity), as_global((const T*)R.vtx), R.vstride,
                         R.g, R.ph, R.sc->dt, i, j, k);
    block_reduce_store(acc, as_global(partials) + ((size_t)R.row0 + tile) * kNP);
  }
}

// Diagnostics terms of one cell of a state that has not been advanced.
template <typename T>
__device__ __forceinline__ void init_cell(CellAcc& acc, const Fields<T>& cur, const Grid& g, const Phys& ph,
                                          int i, int j, int k) {
  const size_t c = i + (size_t)g.nx * (j + (size_t)g.ny * k);
  const double rho = cur.rho[c], n = cur.nb[c];
  T m[3], q[3], P[6], W[6];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    m[d] = cur.o[oidx(GP_MX + d)][c];
    q[d] = cur.o[oidx(GP_QX + d)][c];
  }
#pragma unroll
  for (int s = 0; s < 6; s++) {
    P[s] = cur.o[oidx(GP_PXX + s)][c];
    W[s] = cur.o[oidx(GP_WXX + s)][c];
  }
  const T E = cur.o[oidx(GP_E)][c], e = cur.o[oidx(GP_EINT)][c];
  T ekin, Tt[6], kg, kb;
  kappa_terms(rho, n, m, E, e, q, P, W, ekin, Tt, kg, kb);
  acc.v[P_KGAS] += (double)kg;
  acc.v[P_KBME] += (double)kb;
  cell_terms(acc, rho, n, m, E, e, q, P, W, (T)ph.gamma);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_partials(const RunDev<T>* __restrict__ runs,
                                                          const WorkItem* __restrict__ work, unsigned nwork,
                                                          int parity, double* __restrict__ partials) {
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const int run = uniform(work[w].run), tile = uniform(work[w].tile);
    const RunDev<T>& R = runs[run];
    const int ntx = R.ntx, nty = R.nty;
    const int i = (tile % ntx) * kTX + threadIdx.x;
    const int j = ((tile / ntx) % nty) * kTY + threadIdx.y;
    const int k = tile / (ntx * nty);
    CellAcc acc;
    acc_init(acc);
    if (i < R.g.nx && j < R.g.ny) init_cell<T>(acc, fields_state(R, parity), R.g, R.ph, i, j, k);
    block_reduce_store(acc, as_global(partials) + ((size_t)R.row0 + tile) * kNP);
  }
}

template <typename T>
void launch_vertex(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, unsigned nblocks, hipStream_t st) {
  k_vertex<T><<<nblocks, dim3(kTX, kTY, 1), 0, st>>>(runs, work, nwork);
}
template <typename T>
void launch_lagrangian(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity, double* partials,
                       unsigned nblocks, hipStream_t st) {
  k_lagrangian<T><<<nblocks, dim3(kTX, kTY, 1), 0, st>>>(runs, work, nwork, parity, partials);
}
template <typename T>
void launch_init_partials(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity,
                          double* partials, unsigned nblocks, hipStream_t st) {
  k_init_partials<T><<<nblocks, dim3(kTX, kTY, 1), 0, st>>>(runs, work, nwork, parity, partials);
}
#define GP_INSTANTIATE(T)                                                                                  \
  template void launch_vertex<T>(const RunDev<T>*, const WorkItem*, unsigned, unsigned, hipStream_t);       \
  template void launch_lagrangian<T>(const RunDev<T>*, const WorkItem*, unsigned, int, double*, unsigned,   \
                                     hipStream_t);                                                          \
  template void launch_init_partials<T>(const RunDev<T>*, const WorkItem*, unsigned, int, double*, unsigned, \
                                        hipStream_t);
GP_INSTANTIATE(double)
GP_INSTANTIATE(float)
#undef GP_INSTANTIATE

}  // namespace gp
