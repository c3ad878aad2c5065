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
  T rho, vd, p;  // density, velocity normal to the face, pressure
};

template <typename T>
struct GasIn {
  gptr<const double> rho;
  gptr<const T> m[3], E, e;
};

// Raw loads of one stencil point for faces normal to D: rho, m_D, e.
template <typename T>
struct GasRaw {
  double rho;
  T md, e;
};

template <int P, int D, typename T>
__device__ __forceinline__ GasRaw<T> load_gas(const GasIn<T>& in, const Stencil& s) {
  GasRaw<T> r;
  r.rho = ld_pt<P>(in.rho, s);
  r.md = ld_pt<P>(in.m[D], s);
  r.e = ld_pt<P>(in.e, s);
  return r;
}

template <typename T>
__device__ __forceinline__ GasPrim<T> prim_of(const GasRaw<T>& r, T gm1) {
  GasPrim<T> q;
  q.rho = (T)r.rho;
  q.vd = r.md * rcp(q.rho);
  q.p = gm1 * r.e;
  return q;
}

// Sec. 2.1: V and P at a face between left and right states; z is the
// acoustic impedance sqrt(gamma (pL + pR) rhoL rhoR / (rhoL + rhoR)).
template <typename T>
__device__ __forceinline__ void gas_face(const GasPrim<T>& L, const GasPrim<T>& R, T gamma, T& V, T& P) {
  const T pl = L.p, pr = R.p;
  const T z = sqrt(gamma * (pl + pr) * L.rho * R.rho * rcp(L.rho + R.rho));
  const T rz = rcp(z);
  V = T(0.5) * (L.vd + R.vd) + T(0.5) * (pl - pr) * rz;
  P = T(0.5) * (pl + pr) + T(0.5) * (L.vd - R.vd) * z;
}

template <typename T>
__device__ __forceinline__ void gas_axis(const GasRaw<T>& lo, const GasRaw<T>& hi, const GasPrim<T>& C, T gamma,
                                         T gm1, T& dP, T& dPV, T& dV) {
  T Vm, Pm, Vp, Pp;
  gas_face(prim_of(lo, gm1), C, gamma, Vm, Pm);
  gas_face(C, prim_of(hi, gm1), gamma, Vp, Pp);
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

  // every load of the cell first (3 per neighbour), then the faces
  const double rho_c = ld_pt<0>(in.rho, s);
  T m[3];
#pragma unroll
  for (int d = 0; d < 3; d++) m[d] = ld_pt<0>(in.m[d], s);
  const T e = ld_pt<0>(in.e, s), E = ld_pt<0>(in.E, s);
  const GasRaw<T> xl = load_gas<1, 0>(in, s), xh = load_gas<2, 0>(in, s);
  const GasRaw<T> yl = load_gas<3, 1>(in, s), yh = load_gas<4, 1>(in, s);
  const GasRaw<T> zl = load_gas<5, 2>(in, s), zh = load_gas<6, 2>(in, s);
  T grad[3];
  gravity<T>(as_global((const T*)R.phi), g, R.ph.G, i, j, k, grad);

  GasPrim<T> C;
  C.rho = (T)rho_c;
  const T irho = rcp(C.rho);
  C.p = gm1 * e;
  T dP[3], dPV = T(0), dV = T(0);
  C.vd = m[0] * irho;
  gas_axis(xl, xh, C, gamma, gm1, dP[0], dPV, dV);
  C.vd = m[1] * irho;
  gas_axis(yl, yh, C, gamma, gm1, dP[1], dPV, dV);
  C.vd = m[2] * irho;
  gas_axis(zl, zh, C, gamma, gm1, dP[2], dPV, dV);

  // momentum slots receive v' = m' / rho
  const size_t z = s.z[1];
  const uint32_t xy = s.xy[0];
#pragma unroll
  for (int d = 0; d < 3; d++)
    st_at(as_global((T*)R.tmp[oidx(GP_MX + d)]), z, xy, (m[d] - r * dP[d] - tau * C.rho * grad[d]) * irho);
  st_at(as_global((T*)R.tmp[oidx(GP_E)]), z, xy, E - r * dPV - tau * (m[0] * grad[0] + m[1] * grad[1] + m[2] * grad[2]));
  st_at(as_global((T*)R.tmp[oidx(GP_EINT)]), z, xy, e - r * gm1 * e * dV);
}

// ------------------------------------------------- stars / dark matter ----

template <typename T>
struct BmeIn {
  gptr<const double> n;
  gptr<const T> q[3], P[6], W[6];
};

// One side of a face normal to axis D: density, velocity and row D of Pi
// (components DD, DA, DB with A = D+1, B = D+2 mod 3).
template <typename T>
struct BmeSide {
  T n, u[3], pdd, pda, pdb;
};

// Raw loads of a neighbour across a face normal to D (converted only when
// the face is solved, so the loads stay in flight meanwhile).
template <typename T>
struct BmeRaw {
  double n;
  T q[3], p[3];
};

template <int Pt, int D, typename T>
__device__ __forceinline__ BmeRaw<T> load_raw(const BmeIn<T>& in, const Stencil& s) {
  constexpr int A_ = (D + 1) % 3, B_ = (D + 2) % 3;
  BmeRaw<T> r;
  r.n = ld_pt<Pt>(in.n, s);
#pragma unroll
  for (int d = 0; d < 3; d++) r.q[d] = ld_pt<Pt>(in.q[d], s);
  r.p[0] = ld_pt<Pt>(in.P[sym(D, D)], s);
  r.p[1] = ld_pt<Pt>(in.P[sym(D, A_)], s);
  r.p[2] = ld_pt<Pt>(in.P[sym(D, B_)], s);
  return r;
}

template <typename T>
__device__ __forceinline__ BmeSide<T> side_of(const BmeRaw<T>& r) {
  BmeSide<T> o;
  o.n = (T)r.n;
  const T in_ = rcp(o.n);
#pragma unroll
  for (int d = 0; d < 3; d++) o.u[d] = r.q[d] * in_;
  o.pdd = r.p[0];
  o.pda = r.p[1];
  o.pdb = r.p[2];
  return o;
}

// Centre cell: n, u and the full Pi.
template <typename T>
struct BmeCentre {
  T n, u[3], P[6];
};

template <int D, typename T>
__device__ __forceinline__ BmeSide<T> centre_side(const BmeCentre<T>& C) {
  BmeSide<T> o;
  o.n = C.n;
#pragma unroll
  for (int d = 0; d < 3; d++) o.u[d] = C.u[d];
  o.pdd = C.P[sym(D, D)];
  o.pda = C.P[sym(D, (D + 1) % 3)];
  o.pdb = C.P[sym(D, (D + 2) % 3)];
  return o;
}

// Sec. 2.2: interface state of the BME Eulerian system for normal axis D
// (the printed x-normal formulas with the transverse axes a, b in place of
// y, z).  Bracketed coefficients use the arithmetic means of n, Pi_DD, Pi_Da,
// Pi_Db.  us[i] = u*_i, ps[i] = Pi*_{D i} in lab components.
template <typename T, int D>
__device__ __forceinline__ void bme_face(const BmeSide<T>& L, const BmeSide<T>& R, T us[3], T ps[3]) {
  constexpr int A_ = (D + 1) % 3, B_ = (D + 2) % 3;
  const T sqrt3 = T(1.7320508075688772935);
  const T nbar = T(0.5) * (L.n + R.n);
  const T A = T(0.5) * (L.pdd + R.pdd);
  const T B = T(0.5) * (L.pda + R.pda);
  const T C = T(0.5) * (L.pdb + R.pdb);
  const T Z1 = sqrt(T(3) * nbar * A);  // sqrt(3 n Pi_DD): fast wave impedance
  const T rZ1 = rcp(Z1);
  const T Z2 = Z1 * T(0.57735026918962576451);   // sqrt(n Pi_DD): slow (shear) impedance
  const T rZ2 = rZ1 * T(1.7320508075688772935);
  const T rA = rcp(A);
  const T dpdd = T(0.5) * (L.pdd - R.pdd);
  const T dpda = T(0.5) * (L.pda - R.pda);
  const T dpdb = T(0.5) * (L.pdb - R.pdb);
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

// Adds the contribution of one face normal to axis D, with sign sg (+1 for
// the plus face, -1 for the minus face), to the divergences of the centre
// cell: d_D of Pi*_{iD}, of Pi*_{jD} u*_i + Pi*_{iD} u*_j, and the Pi_{jD} u*_i
// + Pi_{iD} u*_j terms.  Faces are folded in one at a time, so only one face
// state is live.
template <int D, typename T>
__device__ __forceinline__ void bme_face_add(const T us[3], const T ps[3], T sg, const BmeCentre<T>& C, T dq[3],
                                             T dW[6], T dPi[6]) {
#pragma unroll
  for (int i = 0; i < 3; i++) dq[i] += sg * ps[i];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      const int m = sym(i, j);
      dW[m] += sg * (ps[j] * us[i] + ps[i] * us[j]);
      dPi[m] += sg * (C.P[sym(j, D)] * us[i] + C.P[sym(i, D)] * us[j]);
    }
}

// Solves the face on side `plus` of axis D against the neighbour's raw loads
// and folds it in.
template <int D, bool kPlus, typename T>
__device__ __forceinline__ void bme_face_step(const BmeRaw<T>& nb, const BmeCentre<T>& C, T dq[3], T dW[6],
                                              T dPi[6]) {
  T us[3], ps[3];
  if constexpr (kPlus)
    bme_face<T, D>(centre_side<D>(C), side_of(nb), us, ps);
  else
    bme_face<T, D>(side_of(nb), centre_side<D>(C), us, ps);
  bme_face_add<D>(us, ps, kPlus ? T(1) : T(-1), C, dq, dW, dPi);
}

// Ends a face phase: the accumulators must hold this face's contribution
// here (an empty asm that reads and rewrites them), so the face is solved
// while the loads issued for later faces are still in flight, instead of
// being deferred until every load has returned.
template <typename T>
__device__ __forceinline__ void phase_fence(T dq[3], T dW[6], T dPi[6]) {
#pragma unroll
  for (int a = 0; a < 3; a++) asm volatile("" : "+v"(dq[a]));
#pragma unroll
  for (int a = 0; a < 6; a++) asm volatile("" : "+v"(dW[a]), "+v"(dPi[a]));
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

  // centre, then the six neighbours two faces ahead of the face being solved
  T qc[3];
  BmeCentre<T> C;
  C.n = (T)ld_pt<0>(in.n, s);
#pragma unroll
  for (int d = 0; d < 3; d++) qc[d] = ld_pt<0>(in.q[d], s);
#pragma unroll
  for (int m = 0; m < 6; m++) C.P[m] = ld_pt<0>(in.P[m], s);
  BmeRaw<T> a = load_raw<1, 0>(in, s);
  BmeRaw<T> b = load_raw<2, 0>(in, s);
  {
    const T inb = rcp(C.n);
#pragma unroll
    for (int d = 0; d < 3; d++) C.u[d] = qc[d] * inb;
  }
  T dq[3] = {T(0), T(0), T(0)};
  T dW[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  T dPi[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  bme_face_step<0, false>(a, C, dq, dW, dPi);
  BmeRaw<T> c = load_raw<3, 1>(in, s);
  phase_fence(dq, dW, dPi);
  bme_face_step<0, true>(b, C, dq, dW, dPi);
  BmeRaw<T> d = load_raw<4, 1>(in, s);
  phase_fence(dq, dW, dPi);
  bme_face_step<1, false>(c, C, dq, dW, dPi);
  BmeRaw<T> e = load_raw<5, 2>(in, s);
  phase_fence(dq, dW, dPi);
  bme_face_step<1, true>(d, C, dq, dW, dPi);
  BmeRaw<T> f = load_raw<6, 2>(in, s);
  T W[6];
#pragma unroll
  for (int m = 0; m < 6; m++) W[m] = ld_pt<0>(in.W[m], s);
  T grad[3];
  gravity<T>(as_global((const T*)R.phi), g, R.ph.G, i, j, k, grad);
  phase_fence(dq, dW, dPi);
  bme_face_step<2, false>(e, C, dq, dW, dPi);
  phase_fence(dq, dW, dPi);
  bme_face_step<2, true>(f, C, dq, dW, dPi);

  // momentum slots receive u' = q' / n
  const T inb = rcp(C.n);
  const size_t z = s.z[1];
  const uint32_t xy = s.xy[0];
#pragma unroll
  for (int dd = 0; dd < 3; dd++)
    st_at(as_global((T*)R.tmp[oidx(GP_QX + dd)]), z, xy, (qc[dd] - r * dq[dd] - tau * C.n * grad[dd]) * inb);
#pragma unroll
  for (int aa = 0; aa < 3; aa++)
#pragma unroll
    for (int bb = aa; bb < 3; bb++) {
      const int m = sym(aa, bb);
      st_at(as_global((T*)R.tmp[oidx(GP_WXX + m)]), z, xy,
            W[m] - r * dW[m] - tau * (qc[aa] * grad[bb] + qc[bb] * grad[aa]));
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
