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
#include "common.hpp"
#include "kernels.hpp"

namespace gp {

template <typename T>
struct Prim {
  T rho, v[3], p;
  T n, u[3], P[6];
};

template <typename T>
__device__ __forceinline__ void load_prim(const Fields<T>& s, size_t c, T gm1, Prim<T>& q) {
  q.rho = (T)s.rho[c];
  q.n = (T)s.nb[c];
  const T ir = rcp(q.rho), in = rcp(q.n);
#pragma unroll
  for (int d = 0; d < 3; d++) {
    q.v[d] = s.o[oidx(GP_MX + d)][c] * ir;
    q.u[d] = s.o[oidx(GP_QX + d)][c] * in;
  }
  q.p = gm1 * s.o[oidx(GP_EINT)][c];
#pragma unroll
  for (int m = 0; m < 6; m++) q.P[m] = s.o[oidx(GP_PXX + m)][c];
}

// Sec. 2.1: V and P at a face between left and right states; z is the
// acoustic impedance sqrt(gamma (pL + pR) rhoL rhoR / (rhoL + rhoR)).
template <typename T>
__device__ __forceinline__ void gas_face(const Prim<T>& L, const Prim<T>& R, int d, T gamma, T& V,
                                         T& P) {
  const T pl = L.p, pr = R.p;
  const T z = sqrt(gamma * (pl + pr) * L.rho * R.rho * rcp(L.rho + R.rho));
  const T rz = rcp(z);
  V = T(0.5) * (L.v[d] + R.v[d]) + T(0.5) * (pl - pr) * rz;
  P = T(0.5) * (pl + pr) + T(0.5) * (L.v[d] - R.v[d]) * z;
}

// Sec. 2.2: interface state of the BME Eulerian system for normal axis D
// (the printed x-normal formulas with the transverse axes a, b in place of
// y, z).  Bracketed coefficients use the arithmetic means of n, Pi_DD, Pi_Da,
// Pi_Db.  us[i] = u*_i, ps[i] = Pi*_{D i} in lab components.
template <typename T, int D>
__device__ __forceinline__ void bme_face(const Prim<T>& L, const Prim<T>& R, T us[3], T ps[3]) {
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
template <typename T, int D>
__device__ __forceinline__ void axis_terms(const Fields<T>& in, size_t cm, size_t cp, const Prim<T>& C,
                                           T gamma, T gm1, T& dP, T& dPV, T& dV, T dq[3], T dW[6],
                                           T dPi[6]) {
  Prim<T> N;
  T Vm, Pm, Vp, Pp, usm[3], psm[3], usp[3], psp[3];
  load_prim(in, cm, gm1, N);
  gas_face(N, C, D, gamma, Vm, Pm);
  bme_face<T, D>(N, C, usm, psm);
  load_prim(in, cp, gm1, N);
  gas_face(C, N, D, gamma, Vp, Pp);
  bme_face<T, D>(C, N, usp, psp);
  dP = Pp - Pm;
  dPV += Pp * Vp - Pm * Vm;
  dV += Vp - Vm;
#pragma unroll
  for (int i = 0; i < 3; i++) dq[i] += psp[i] - psm[i];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      const int s = sym(i, j);
      dW[s] += (psp[j] * usp[i] + psp[i] * usp[j]) - (psm[j] * usm[i] + psm[i] * usm[j]);
      dPi[s] += C.P[sym(j, D)] * (usp[i] - usm[i]) + C.P[sym(i, D)] * (usp[j] - usm[j]);
    }
}

// One cell of the Eulerian stage; tau_d is the step, (i, j, k) the cell.
template <typename T>
__device__ __forceinline__ void eulerian_cell(const Fields<T>& in, const Fields<T>& out,
                                              gptr<const T> phi, const Grid& g, const Phys& ph,
                                              double tau_d, int i, int j, int k) {
  const size_t nx = g.nx, nxy = (size_t)g.nx * g.ny;
  const size_t c = i + nx * j + nxy * k;
  const T tau = (T)tau_d, r = (T)(tau_d / g.h);
  const T gamma = (T)ph.gamma, gm1 = gamma - T(1);

  // neighbour cells under the hydrodynamic boundary rule
  const size_t im = bc_index(i - 1, g.nx, g.bc[0]), ip = bc_index(i + 1, g.nx, g.bc[0]);
  const size_t jm = bc_index(j - 1, g.ny, g.bc[1]), jp = bc_index(j + 1, g.ny, g.bc[1]);
  const size_t km = bc_index(k - 1, g.nz, g.bc[2]), kp = bc_index(k + 1, g.nz, g.bc[2]);
  const size_t row = nx * j + nxy * k;

  // gravity: central difference of the periodic potential
  T grad[3] = {T(0), T(0), T(0)};
  if (ph.G != 0.0) {
    const T r2h = (T)(0.5 / g.h);
    const size_t wim = wrap_index(i - 1, g.nx), wip = wrap_index(i + 1, g.nx);
    const size_t wjm = wrap_index(j - 1, g.ny), wjp = wrap_index(j + 1, g.ny);
    const size_t wkm = wrap_index(k - 1, g.nz), wkp = wrap_index(k + 1, g.nz);
    grad[0] = (phi[row + wip] - phi[row + wim]) * r2h;
    grad[1] = (phi[i + nx * wjp + nxy * k] - phi[i + nx * wjm + nxy * k]) * r2h;
    grad[2] = (phi[i + nx * j + nxy * wkp] - phi[i + nx * j + nxy * wkm]) * r2h;
  }

  Prim<T> C;
  load_prim(in, c, gm1, C);
  T dP[3], dPV = T(0), dV = T(0);
  T dq[3] = {T(0), T(0), T(0)};
  T dW[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  T dPi[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  axis_terms<T, 0>(in, row + im, row + ip, C, gamma, gm1, dP[0], dPV, dV, dq, dW, dPi);
  axis_terms<T, 1>(in, i + nx * jm + nxy * k, i + nx * jp + nxy * k, C, gamma, gm1, dP[1], dPV, dV,
                   dq, dW, dPi);
  axis_terms<T, 2>(in, i + nx * j + nxy * km, i + nx * j + nxy * kp, C, gamma, gm1, dP[2], dPV, dV,
                   dq, dW, dPi);

  // gas (momentum slots receive v' = m' / rho)
  T m[3];
#pragma unroll
  for (int d = 0; d < 3; d++) m[d] = in.o[oidx(GP_MX + d)][c];
  const T irho = rcp(C.rho), inb = rcp(C.n);
#pragma unroll
  for (int d = 0; d < 3; d++) out.o[oidx(GP_MX + d)][c] = (m[d] - r * dP[d] - tau * C.rho * grad[d]) * irho;
  out.o[oidx(GP_E)][c] =
      in.o[oidx(GP_E)][c] - r * dPV - tau * (m[0] * grad[0] + m[1] * grad[1] + m[2] * grad[2]);
  const T e = in.o[oidx(GP_EINT)][c];
  out.o[oidx(GP_EINT)][c] = e - r * gm1 * e * dV;

  // stars / dark matter (momentum slots receive u' = q' / n)
  T q[3];
#pragma unroll
  for (int d = 0; d < 3; d++) q[d] = in.o[oidx(GP_QX + d)][c];
#pragma unroll
  for (int d = 0; d < 3; d++) out.o[oidx(GP_QX + d)][c] = (q[d] - r * dq[d] - tau * C.n * grad[d]) * inb;
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = a; b < 3; b++) {
      const int s = sym(a, b);
      out.o[oidx(GP_WXX + s)][c] =
          in.o[oidx(GP_WXX + s)][c] - r * dW[s] - tau * (q[a] * grad[b] + q[b] * grad[a]);
      out.o[oidx(GP_PXX + s)][c] = C.P[s] - r * dPi[s];
    }
}

// Persistent launch over the (run, tile) work list of a batch.
template <typename T>
__global__ void __launch_bounds__(kBlock, 3) k_eulerian(const RunDev<T>* __restrict__ runs,
                                                     const WorkItem* __restrict__ work, unsigned nwork,
                                                     int parity) {
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const int run = uniform(work[w].run), tile = uniform(work[w].tile);
    const RunDev<T>& R = runs[run];
    const int ntx = R.ntx, nty = R.nty;
    const int i = (tile % ntx) * kTX + threadIdx.x;
    const int j = ((tile / ntx) % nty) * kTY + threadIdx.y;
    const int k = tile / (ntx * nty);
    if (i < R.g.nx && j < R.g.ny)
      eulerian_cell<T>(fields_state(R, parity), fields_eul(R), as_global((const T*)R.phi), R.g, R.ph, R.sc->dt, i, j, k);
  }
}

template <typename T>
void launch_eulerian(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity, unsigned nblocks,
                     hipStream_t st) {
  k_eulerian<T><<<nblocks, dim3(kTX, kTY, 1), 0, st>>>(runs, work, nwork, parity);
}

template void launch_eulerian<double>(const RunDev<double>*, const WorkItem*, unsigned, int, unsigned, hipStream_t);
template void launch_eulerian<float>(const RunDev<float>*, const WorkItem*, unsigned, int, unsigned, hipStream_t);

}  // namespace gp
