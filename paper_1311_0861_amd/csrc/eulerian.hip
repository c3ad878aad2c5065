// Eulerian stage of one GPUPEGAS step (Kulikov, arXiv:1311.0861, Sec. 2.1-2.2).
//
// With the fluid frozen, every equation of Sec. 2 keeps its non-advective
// right-hand side; divergences take the closed-form interface states of the
// linearised Riemann problems, gravity is -grad Phi by central difference:
//   m_i  -= tau/h d_i P + tau rho g_i
//   E    -= tau/h sum_d d_d(P V) + tau m.g
//   e    -= tau/h (gamma-1) e sum_d d_d V
//   q_i  -= tau/h sum_d d_d Pi*_{id} + tau n g_i
//   W_ij -= tau/h sum_d d_d(Pi*_{jd} u*_i + Pi*_{id} u*_j) + tau (q_i g_j + q_j g_i)
//   Pi_ij-= tau/h sum_d (Pi_jd d_d u*_i + Pi_id d_d u*_j)
// (d_d X = X at face c+1/2 e_d minus X at face c-1/2 e_d).  rho and n are
// not touched by this stage.  The momentum slots of the output hold the
// post-Eulerian velocities v' = m'/rho and u' = q'/n, which is what the
// Lagrangian stage advects with (it rebuilds m' = rho v' where it needs it).
//
// The two components only share the potential, so each has its own kernel:
// the gas kernel touches 5 + 1 arrays per stencil point, the stars / dark
// matter kernel 10 + 1, and each holds half the live state of a joint one,
// which buys occupancy for these latency-bound stencils.
#include "common.hpp"
#include "kernels.hpp"

namespace gp {

// Gravity acceleration -grad Phi at a cell (zero when G = 0): central
// differences of the periodic potential.
template <typename T>
__device__ __forceinline__ void gravity(gptr<const T> phi, const Grid& g, double G, int i, int j, int k,
                                        T grad[3]) {
  grad[0] = grad[1] = grad[2] = T(0);
  if (G == 0.0) return;
  const Stencil w = make_stencil(g, i, j, k, true);
  const T r2h = (T)(0.5 / g.h);
  grad[0] = (ld_pt<2>(phi, w) - ld_pt<1>(phi, w)) * r2h;
  grad[1] = (ld_pt<4>(phi, w) - ld_pt<3>(phi, w)) * r2h;
  grad[2] = (ld_pt<6>(phi, w) - ld_pt<5>(phi, w)) * r2h;
}

// ---------------------------------------------------------------- gas ----

template <typename T>
struct GasPrim {
  T rho, v[3], p;
};

template <typename T>
struct GasIn {
  gptr<const double> rho;
  gptr<const T> m[3], E, e;
};

template <int P, typename T>
__device__ __forceinline__ GasPrim<T> load_gas(const GasIn<T>& in, const Stencil& s, T gm1) {
  GasPrim<T> q;
  q.rho = (T)ld_pt<P>(in.rho, s);
  const T ir = rcp(q.rho);
#pragma unroll
  for (int d = 0; d < 3; d++) q.v[d] = ld_pt<P>(in.m[d], s) * ir;
  q.p = gm1 * ld_pt<P>(in.e, s);
  return q;
}

// Sec. 2.1: V and P at a face between left and right states; z is the
// acoustic impedance sqrt(gamma (pL + pR) rhoL rhoR / (rhoL + rhoR)).
template <typename T>
__device__ __forceinline__ void gas_face(const GasPrim<T>& L, const GasPrim<T>& R, int d, T gamma, T& V, T& P) {
  const T pl = L.p, pr = R.p;
  const T z = sqrt(gamma * (pl + pr) * L.rho * R.rho * rcp(L.rho + R.rho));
  const T rz = rcp(z);
  V = T(0.5) * (L.v[d] + R.v[d]) + T(0.5) * (pl - pr) * rz;
  P = T(0.5) * (pl + pr) + T(0.5) * (L.v[d] - R.v[d]) * z;
}

template <int D, typename T>
__device__ __forceinline__ void gas_axis(const GasIn<T>& in, const Stencil& s, const GasPrim<T>& C, T gamma,
                                         T gm1, T& dP, T& dPV, T& dV) {
  T Vm, Pm, Vp, Pp;
  const GasPrim<T> L = load_gas<1 + 2 * D>(in, s, gm1);
  const GasPrim<T> R = load_gas<2 + 2 * D>(in, s, gm1);
  gas_face(L, C, D, gamma, Vm, Pm);
  gas_face(C, R, D, gamma, Vp, Pp);
  dP = Pp - Pm;
  dPV += Pp * Vp - Pm * Vm;
  dV += Vp - Vm;
}

template <typename T>
__device__ __forceinline__ void eul_gas_cell(const RunDev<T>& R, int parity, double tau_d, int i, int j, int k) {
  const Grid& g = R.g;
  const T tau = (T)tau_d, r = (T)(tau_d / g.h);
  const T gamma = (T)R.ph.gamma, gm1 = gamma - T(1);
  const Stencil s = make_stencil(g, i, j, k, false);
  GasIn<T> in;
  in.rho = as_global((const double*)R.dens[parity][0]);
#pragma unroll
  for (int d = 0; d < 3; d++) in.m[d] = as_global((const T*)R.cur[oidx(GP_MX + d)]);
  in.E = as_global((const T*)R.cur[oidx(GP_E)]);
  in.e = as_global((const T*)R.cur[oidx(GP_EINT)]);

  T grad[3];
  gravity<T>(as_global((const T*)R.phi), g, R.ph.G, i, j, k, grad);
  const GasPrim<T> C = load_gas<0>(in, s, gm1);
  T dP[3], dPV = T(0), dV = T(0);
  gas_axis<0>(in, s, C, gamma, gm1, dP[0], dPV, dV);
  gas_axis<1>(in, s, C, gamma, gm1, dP[1], dPV, dV);
  gas_axis<2>(in, s, C, gamma, gm1, dP[2], dPV, dV);

  // momentum slots receive v' = m' / rho
  T m[3];
#pragma unroll
  for (int d = 0; d < 3; d++) m[d] = ld_pt<0>(in.m[d], s);
  const T irho = rcp(C.rho);
  const size_t z = s.z[1];
  const uint32_t xy = s.xy[0];
#pragma unroll
  for (int d = 0; d < 3; d++)
    st_at(as_global((T*)R.tmp[oidx(GP_MX + d)]), z, xy, (m[d] - r * dP[d] - tau * C.rho * grad[d]) * irho);
  st_at(as_global((T*)R.tmp[oidx(GP_E)]), z, xy,
        ld_pt<0>(in.E, s) - r * dPV - tau * (m[0] * grad[0] + m[1] * grad[1] + m[2] * grad[2]));
  const T e = ld_pt<0>(in.e, s);
  st_at(as_global((T*)R.tmp[oidx(GP_EINT)]), z, xy, e - r * gm1 * e * dV);
}

// ------------------------------------------------- stars / dark matter ----

template <typename T>
struct BmePrim {
  T n, u[3], P[6];
};

template <typename T>
struct BmeIn {
  gptr<const double> n;
  gptr<const T> q[3], P[6], W[6];
};

template <int Pt, typename T>
__device__ __forceinline__ BmePrim<T> load_bme(const BmeIn<T>& in, const Stencil& s) {
  BmePrim<T> q;
  q.n = (T)ld_pt<Pt>(in.n, s);
  const T in_ = rcp(q.n);
#pragma unroll
  for (int d = 0; d < 3; d++) q.u[d] = ld_pt<Pt>(in.q[d], s) * in_;
#pragma unroll
  for (int m = 0; m < 6; m++) q.P[m] = ld_pt<Pt>(in.P[m], s);
  return q;
}

// Sec. 2.2: interface state of the BME Eulerian system for normal axis D
// (the printed x-normal formulas with the transverse axes a, b in place of
// y, z).  Bracketed coefficients use the arithmetic means of n, Pi_DD, Pi_Da,
// Pi_Db.  us[i] = u*_i, ps[i] = Pi*_{D i} in lab components.
template <typename T, int D>
__device__ __forceinline__ void bme_face(const BmePrim<T>& L, const BmePrim<T>& R, T us[3], T ps[3]) {
  constexpr int A_ = (D + 1) % 3, B_ = (D + 2) % 3;
  constexpr int sDD = sym(D, D), sDA = sym(D, A_), sDB = sym(D, B_);
  const T sqrt3 = T(1.7320508075688772935);
  const T nbar = T(0.5) * (L.n + R.n);
  const T A = T(0.5) * (L.P[sDD] + R.P[sDD]);
  const T B = T(0.5) * (L.P[sDA] + R.P[sDA]);
  const T C = T(0.5) * (L.P[sDB] + R.P[sDB]);
  const T Z1 = sqrt(T(3) * nbar * A);  // sqrt(3 n Pi_DD): fast wave impedance
  const T rZ1 = rcp(Z1);
  const T Z2 = Z1 * T(0.57735026918962576451);   // sqrt(n Pi_DD): slow (shear) impedance
  const T rZ2 = rZ1 * T(1.7320508075688772935);
  const T rA = rcp(A);
  const T dpdd = T(0.5) * (L.P[sDD] - R.P[sDD]);
  const T dpda = T(0.5) * (L.P[sDA] - R.P[sDA]);
  const T dpdb = T(0.5) * (L.P[sDB] - R.P[sDB]);
  const T dud = T(0.5) * (L.u[D] - R.u[D]);
  const T dua = T(0.5) * (L.u[A_] - R.u[A_]);
  const T dub = T(0.5) * (L.u[B_] - R.u[B_]);
  const T cross_u = dpdd * (T(1) - sqrt3) * rA * rZ1;  // coupling of the fast wave into u_a, u_b
  const T cross_p = dud * nbar * (sqrt3 - T(1)) * rZ2;  // and into Pi_Da, Pi_Db
  us[D] = T(0.5) * (L.u[D] + R.u[D]) + dpdd * rZ1;
  us[A_] = T(0.5) * (L.u[A_] + R.u[A_]) + dpda * rZ2 + B * cross_u;
  us[B_] = T(0.5) * (L.u[B_] + R.u[B_]) + dpdb * rZ2 + C * cross_u;
  ps[D] = A + dud * Z1;
  ps[A_] = B + dua * Z2 + B * cross_p;
  ps[B_] = C + dub * Z2 + C * cross_p;
}

// Contributions of the two faces normal to axis D of the centre cell.
template <int D, typename T>
__device__ __forceinline__ void bme_axis(const BmeIn<T>& in, const Stencil& s, const BmePrim<T>& C, T dq[3],
                                         T dW[6], T dPi[6]) {
  T usm[3], psm[3], usp[3], psp[3];
  {
    const BmePrim<T> L = load_bme<1 + 2 * D>(in, s);
    bme_face<T, D>(L, C, usm, psm);
  }
  {
    const BmePrim<T> R = load_bme<2 + 2 * D>(in, s);
    bme_face<T, D>(C, R, usp, psp);
  }
#pragma unroll
  for (int i = 0; i < 3; i++) dq[i] += psp[i] - psm[i];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      const int m = sym(i, j);
      dW[m] += (psp[j] * usp[i] + psp[i] * usp[j]) - (psm[j] * usm[i] + psm[i] * usm[j]);
      dPi[m] += C.P[sym(j, D)] * (usp[i] - usm[i]) + C.P[sym(i, D)] * (usp[j] - usm[j]);
    }
}

template <typename T>
__device__ __forceinline__ void eul_bme_cell(const RunDev<T>& R, int parity, double tau_d, int i, int j, int k) {
  const Grid& g = R.g;
  const T tau = (T)tau_d, r = (T)(tau_d / g.h);
  const Stencil s = make_stencil(g, i, j, k, false);
  BmeIn<T> in;
  in.n = as_global((const double*)R.dens[parity][1]);
#pragma unroll
  for (int d = 0; d < 3; d++) in.q[d] = as_global((const T*)R.cur[oidx(GP_QX + d)]);
#pragma unroll
  for (int m = 0; m < 6; m++) {
    in.P[m] = as_global((const T*)R.cur[oidx(GP_PXX + m)]);
    in.W[m] = as_global((const T*)R.cur[oidx(GP_WXX + m)]);
  }

  T grad[3];
  gravity<T>(as_global((const T*)R.phi), g, R.ph.G, i, j, k, grad);
  const BmePrim<T> C = load_bme<0>(in, s);
  T dq[3] = {T(0), T(0), T(0)};
  T dW[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  T dPi[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  bme_axis<0>(in, s, C, dq, dW, dPi);
  bme_axis<1>(in, s, C, dq, dW, dPi);
  bme_axis<2>(in, s, C, dq, dW, dPi);

  // momentum slots receive u' = q' / n
  T q[3];
#pragma unroll
  for (int d = 0; d < 3; d++) q[d] = ld_pt<0>(in.q[d], s);
  const T inb = rcp(C.n);
  const size_t z = s.z[1];
  const uint32_t xy = s.xy[0];
#pragma unroll
  for (int d = 0; d < 3; d++)
    st_at(as_global((T*)R.tmp[oidx(GP_QX + d)]), z, xy, (q[d] - r * dq[d] - tau * C.n * grad[d]) * inb);
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = a; b < 3; b++) {
      const int m = sym(a, b);
      st_at(as_global((T*)R.tmp[oidx(GP_WXX + m)]), z, xy,
            ld_pt<0>(in.W[m], s) - r * dW[m] - tau * (q[a] * grad[b] + q[b] * grad[a]));
      st_at(as_global((T*)R.tmp[oidx(GP_PXX + m)]), z, xy, C.P[m] - r * dPi[m]);
    }
}

// ------------------------------------------------------------ launches ----

// Persistent launches over the (run, tile) work list of a batch.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_eul_gas(const RunDev<T>* __restrict__ runs,
                                                    const WorkItem* __restrict__ work, unsigned nwork, int parity) {
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const int run = uniform(work[w].run), tile = uniform(work[w].tile);
    const RunDev<T>& R = runs[run];
    const TileCell c = tile_cell(R, tile);
    if (c.inside) eul_gas_cell<T>(R, parity, R.sc->dt, c.i, c.j, c.k);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_eul_bme(const RunDev<T>* __restrict__ runs,
                                                    const WorkItem* __restrict__ work, unsigned nwork, int parity) {
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const int run = uniform(work[w].run), tile = uniform(work[w].tile);
    const RunDev<T>& R = runs[run];
    const TileCell c = tile_cell(R, tile);
    if (c.inside) eul_bme_cell<T>(R, parity, R.sc->dt, c.i, c.j, c.k);
  }
}

template <typename T>
void launch_eulerian(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity, int comp,
                     unsigned nblocks, hipStream_t st) {
  if (comp == COMP_GAS)
    k_eul_gas<T><<<nblocks, dim3(kTX, kTY, 1), 0, st>>>(runs, work, nwork, parity);
  else
    k_eul_bme<T><<<nblocks, dim3(kTX, kTY, 1), 0, st>>>(runs, work, nwork, parity);
}

template void launch_eulerian<double>(const RunDev<double>*, const WorkItem*, unsigned, int, int, unsigned,
                                      hipStream_t);
template void launch_eulerian<float>(const RunDev<float>*, const WorkItem*, unsigned, int, int, unsigned,
                                     hipStream_t);

}  // namespace gp
