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
// the gas kernel needs 5 primitives + the potential per stencil point, the
// stars / dark matter kernel 10 + 1, and each holds half the live state of a
// joint one, which buys occupancy for these latency-bound stencils.
#include "column.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace gp {

// ---------------------------------------------------------------- gas ----

template <typename T>
struct GasPrim {
  T rho, vd, p;  // density, velocity normal to the face, pressure
};

// Sec. 2.1: V and P at a face between left and right states; z is the
// acoustic impedance sqrt(gamma (pL + pR) rhoL rhoR / (rhoL + rhoR)).
// The face solvers fuse multiply-adds only where written (fma): a face is
// solved in more than one place (a chunk's first z face in the column
// prologue, every other one in the plane loop and carried to the next
// plane), and fusing left to the compiler is decided per inlined copy, which
// would give those copies different bits, so results would depend on where
// the tiling puts chunk boundaries.
template <typename T>
__device__ __forceinline__ void gas_face(const GasPrim<T>& L, const GasPrim<T>& R, T gamma, T& V, T& P) {
#pragma clang fp contract(off)
  const T pl = L.p, pr = R.p;
  const T zz = gamma * (pl + pr) * L.rho * R.rho * rcp(L.rho + R.rho);
  const T rz = rsqrt_nr(zz);
  const T z = zz * rz;
  V = fma(T(0.5) * (pl - pr), rz, T(0.5) * (L.vd + R.vd));
  P = fma(T(0.5) * (L.vd - R.vd), z, T(0.5) * (pl + pr));
}

// ------------------------------------------------- stars / dark matter ----

// One side of a face normal to axis D: density, velocity and row D of Pi
// (components DD, DA, DB with A = D+1, B = D+2 mod 3).
template <typename T>
struct BmeSide {
  T n, u[3], pdd, pda, pdb;
};

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
// (Multiply-adds fused only where written, as in gas_face.)
template <typename T, int D>
__device__ __forceinline__ void bme_face(const BmeSide<T>& L, const BmeSide<T>& R, T us[3], T ps[3]) {
#pragma clang fp contract(off)
  constexpr int A_ = (D + 1) % 3, B_ = (D + 2) % 3;
  const T sqrt3 = T(1.7320508075688772935);
  const T nbar = T(0.5) * (L.n + R.n);
  const T A = T(0.5) * (L.pdd + R.pdd);
  const T B = T(0.5) * (L.pda + R.pda);
  const T C = T(0.5) * (L.pdb + R.pdb);
  const T Z1sq = T(3) * nbar * A;
  const T rZ1 = rsqrt_nr(Z1sq);
  const T Z1 = Z1sq * rZ1;  // sqrt(3 n Pi_DD): fast wave impedance
  const T Z2 = Z1 * T(0.57735026918962576451);   // sqrt(n Pi_DD): slow (shear) impedance
  const T rZ2 = rZ1 * T(1.7320508075688772935);
  const T rA = T(3) * nbar * (rZ1 * rZ1);  // 1 / A, as rZ1^2 = 1 / (3 n A)
  const T dpdd = T(0.5) * (L.pdd - R.pdd);
  const T dpda = T(0.5) * (L.pda - R.pda);
  const T dpdb = T(0.5) * (L.pdb - R.pdb);
  const T dud = T(0.5) * (L.u[D] - R.u[D]);
  const T dua = T(0.5) * (L.u[A_] - R.u[A_]);
  const T dub = T(0.5) * (L.u[B_] - R.u[B_]);
  const T cross_u = dpdd * (T(1) - sqrt3) * rA * rZ1;  // coupling of the fast wave into u_a, u_b
  const T cross_p = dud * nbar * (sqrt3 - T(1)) * rZ2;  // and into Pi_Da, Pi_Db
  us[D] = fma(dpdd, rZ1, T(0.5) * (L.u[D] + R.u[D]));
  us[A_] = fma(B, cross_u, fma(dpda, rZ2, T(0.5) * (L.u[A_] + R.u[A_])));
  us[B_] = fma(C, cross_u, fma(dpdb, rZ2, T(0.5) * (L.u[B_] + R.u[B_])));
  ps[D] = fma(dud, Z1, A);
  ps[A_] = fma(B, cross_p, fma(dua, Z2, B));
  ps[B_] = fma(C, cross_p, fma(dub, Z2, C));
}

// Adds the contributions of the two faces normal to axis D (interface states
// usm, psm of the minus face and usp, psp of the plus face) to the
// divergences of the centre cell: d_D of Pi*_{iD}, of Pi*_{jD} u*_i +
// Pi*_{iD} u*_j, and the Pi_{jD} u*_i + Pi_{iD} u*_j terms.  The last take
// the centre's own Pi, so the two faces combine into Pi_{jD} (u*+_i - u*-_i)
// + Pi_{iD} (u*+_j - u*-_j).
template <int D, typename T>
__device__ __forceinline__ void bme_face_pair(const T usm[3], const T psm[3], const T usp[3], const T psp[3],
                                              const BmeCentre<T>& C, T dq[3], T dW[6], T dPi[6]) {
  T du[3];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    dq[i] += psp[i] - psm[i];
    du[i] = usp[i] - usm[i];
  }
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      const int m = sym(i, j);
      dW[m] += (psp[j] * usp[i] + psp[i] * usp[j]) - (psm[j] * usm[i] + psm[i] * usm[j]);
      dPi[m] += C.P[sym(j, D)] * du[i] + C.P[sym(i, D)] * du[j];
    }
}

// ------------------------------------------------------------ columns ----
//
// Both kernels walk tile columns (see column.hpp).  For plane k the
// primitives of every cell of the tile and its ring sit in LDS, formed once
// per cell as they are staged (u = q / n, v = m / rho, p = (gamma - 1) e);
// the next plane's primitives come into registers a plane ahead and the
// previous plane's are read back from the LDS centres.  The potential has
// its own tile with a periodic ring.

// Gas tile slots: rho, v_x, v_y, v_z, p.  Stars / DM: n, u_x, u_y, u_z, Pi (6).
constexpr int kGasPrims = 5;
constexpr int kBmePrims = 10;

template <int D, typename T, int LY, int LX>
__device__ __forceinline__ GasPrim<T> gas_at(const T (&t)[kGasPrims][LY][LX], int r, int c) {
  return GasPrim<T>{t[0][r][c], t[1 + D][r][c], t[4][r][c]};
}
template <int D, typename T>
__device__ __forceinline__ GasPrim<T> gas_of(const T (&a)[kGasPrims]) {
  return GasPrim<T>{a[0], a[1 + D], a[4]};
}
template <int D, typename T, int LY, int LX>
__device__ __forceinline__ BmeSide<T> bme_at(const T (&t)[kBmePrims][LY][LX], int r, int c) {
  BmeSide<T> o;
  o.n = t[0][r][c];
#pragma unroll
  for (int d = 0; d < 3; d++) o.u[d] = t[1 + d][r][c];
  o.pdd = t[4 + sym(D, D)][r][c];
  o.pda = t[4 + sym(D, (D + 1) % 3)][r][c];
  o.pdb = t[4 + sym(D, (D + 2) % 3)][r][c];
  return o;
}
template <int D, typename T>
__device__ __forceinline__ BmeSide<T> bme_of(const T (&a)[kBmePrims]) {
  BmeSide<T> o;
  o.n = a[0];
#pragma unroll
  for (int d = 0; d < 3; d++) o.u[d] = a[1 + d];
  o.pdd = a[4 + sym(D, D)];
  o.pda = a[4 + sym(D, (D + 1) % 3)];
  o.pdb = a[4 + sym(D, (D + 2) % 3)];
  return o;
}

// Potential at plane offset z and in-plane offset xy (phi_plane and
// make_phi_column give both for either boundary of the potential), zero
// without gravity.
template <typename T>
__device__ __forceinline__ T phi_at(gptr<const T> phi, bool grav, size_t z, uint32_t xy) {
  return grav ? ld_at(phi, z, xy) : T(0);
}

// Cooling rate of the energy equations (Sec. 2: the -q that Sec. 2.1 puts in
// the Eulerian stage).  The paper tabulates q; the stand-in is the power law
// q = lambda rho^2 theta^alpha of theta = p / rho above theta_min (0 below).
template <typename T>
__device__ __forceinline__ T cooling_rate(const Phys& ph, T rho, T theta) {
  if (!(theta > (T)ph.cool_theta_min)) return T(0);
  return (T)ph.cool_lambda * rho * rho * pow(theta, (T)ph.cool_alpha);
}

// COOL: the cooling source is compiled in (launched when a run of the batch
// cools; runs with lambda = 0 skip it).
template <typename T, bool COOL, class S>
__global__ void __launch_bounds__(kBlock) k_eul_gas(const RunDev<T>* __restrict__ runs,
                                                    const WorkItem* __restrict__ work, unsigned nwork, int parity) {
  __shared__ T s_g[kGasPrims][S::LY][S::LX];
  __shared__ T s_phi[S::LY][S::LX];
  const int lx = threadIdx.x, ly = threadIdx.y;
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const WorkItem it = load_item(work, w);
    const int run = it.run;
    const RunDev<T>& R = runs[run];
    const Grid& g = R.g;
    const Column col = make_column<S>(g, it, false);
    const Column pc = make_phi_column<S>(g, it);
    const bool grav = R.ph.G != 0.0;
    const T gext[3] = {(T)R.ph.gext[0], (T)R.ph.gext[1], (T)R.ph.gext[2]};
    const bool cool = COOL && R.ph.cool_lambda != 0.0;
    const size_t nxy = (size_t)g.nx * g.ny;
    const double tau_d = R.sc->dt;
    const T tau = (T)tau_d, r = (T)(tau_d / g.h), r2h = (T)(0.5 / g.h);
    const T gamma = (T)R.ph.gamma, gm1 = gamma - T(1);
    const gptr<const double> rho_in = as_global((const double*)R.dens[parity][0]);
    gptr<const T> m_in[3];
#pragma unroll
    for (int d = 0; d < 3; d++) m_in[d] = as_global((const T*)R.cur[oidx(GP_MX + d)]);
    const gptr<const T> E_in = as_global((const T*)R.cur[oidx(GP_E)]);
    const gptr<const T> e_in = as_global((const T*)R.cur[oidx(GP_EINT)]);
    const gptr<const T> phi = as_global((const T*)R.phi);
    // raw loads of a cell, then its primitives
    auto load = [&](size_t z, uint32_t xy, double& rho, T m[3], T& e) {
      rho = ld_at(rho_in, z, xy);
#pragma unroll
      for (int d = 0; d < 3; d++) m[d] = ld_at(m_in[d], z, xy);
      e = ld_at(e_in, z, xy);
    };
    auto prims = [&](double rho, const T m[3], T e, T (&a)[kGasPrims]) {
      a[0] = (T)rho;
      const T ir = rcp(a[0]);
#pragma unroll
      for (int d = 0; d < 3; d++) a[1 + d] = m[d] * ir;
      a[4] = gm1 * e;
    };

    // prologue: plane k0 into registers, the potential of plane k0 - 1 into
    // the LDS centre, and the z- face of plane k0; from then on each plane's
    // z- face is the previous plane's z+ face (same inputs, same bits)
    T pc_[kGasPrims], mc[3], ec, phc;
    T Vz, Pz;  // z+ face of the previous plane
    {
      const size_t zm = plane_at(g, col.k0 - 1, g.bc[2]), z0 = nxy * (size_t)col.k0;
      double rho, rho0;
      T m[3], e, pm[kGasPrims];
      load(zm, col.xy_c, rho, m, e);
      load(z0, col.xy_c, rho0, mc, ec);
      const T phm = phi_at(phi, grav, phi_plane(g, col.k0 - 1), pc.xy_c);
      phc = phi_at(phi, grav, phi_plane(g, col.k0), pc.xy_c);
      prims(rho, m, e, pm);
      prims(rho0, mc, ec, pc_);
      gas_face(gas_of<2>(pm), gas_of<2>(pc_), gamma, Vz, Pz);
      s_phi[ly + 1][lx + 1] = phm;
    }
    // the ring of each plane is fetched a plane ahead, so staging it never
    // waits on memory (every lane has a valid ring address)
    double rho_h;
    T m_h[3], e_h, phh;
    auto load_ring = [&](int kr) {
      const size_t zr = nxy * (size_t)kr;
      load(zr, col.xy_h, rho_h, m_h, e_h);
      phh = phi_at(phi, grav, phi_plane(g, kr), pc.xy_h);
    };
    load_ring(col.k0);
    for (int k = col.k0; k < col.k1; k++) {
      const size_t zk = nxy * (size_t)k, zp = plane_at(g, k + 1, g.bc[2]);
      const uint32_t xy_c = col.xy_c, pxy_c = pc.xy_c;
      const T phm = s_phi[ly + 1][lx + 1];
      lds_barrier();  // every thread is done with the previous plane's tiles
      if (col.ring) {
        T a[kGasPrims];
        prims(rho_h, m_h, e_h, a);
#pragma unroll
        for (int f = 0; f < kGasPrims; f++) s_g[f][col.hr][col.hc] = a[f];
        s_phi[col.hr][col.hc] = phh;
      }
#pragma unroll
      for (int f = 0; f < kGasPrims; f++) s_g[f][ly + 1][lx + 1] = pc_[f];
      s_phi[ly + 1][lx + 1] = phc;
      // the next plane's centres (needed by the z+ face, formed last), the
      // next ring, then this plane's E (needed by the store)
      double rho_n;
      T m_n[3], e_n;
      load(zp, xy_c, rho_n, m_n, e_n);
      const T php = phi_at(phi, grav, phi_plane(g, k + 1), pxy_c);
      if (k + 1 < col.k1) load_ring(k + 1);
      const T E = ld_at(E_in, zk, xy_c);
      lds_barrier();

      if (col.active) {
        // faces: x / y neighbours from the tile, z from registers
        T Vm, Pm, Vp, Pp, dP[3], dPV = T(0), dV = T(0);
        gas_face(gas_at<0>(s_g, ly + 1, lx), gas_of<0>(pc_), gamma, Vm, Pm);
        gas_face(gas_of<0>(pc_), gas_at<0>(s_g, ly + 1, lx + 2), gamma, Vp, Pp);
        dP[0] = Pp - Pm;
        dPV += Pp * Vp - Pm * Vm;
        dV += Vp - Vm;
        gas_face(gas_at<1>(s_g, ly, lx + 1), gas_of<1>(pc_), gamma, Vm, Pm);
        gas_face(gas_of<1>(pc_), gas_at<1>(s_g, ly + 2, lx + 1), gamma, Vp, Pp);
        dP[1] = Pp - Pm;
        dPV += Pp * Vp - Pm * Vm;
        dV += Vp - Vm;
        Vm = Vz;
        Pm = Pz;
        T pn[kGasPrims];
        prims(rho_n, m_n, e_n, pn);
        gas_face(gas_of<2>(pc_), gas_of<2>(pn), gamma, Vp, Pp);
        Vz = Vp;
        Pz = Pp;
        dP[2] = Pp - Pm;
        dPV += Pp * Vp - Pm * Vm;
        dV += Vp - Vm;
        T grad[3] = {T(0), T(0), T(0)};
        if (grav) {
          grad[0] = (s_phi[ly + 1][lx + 2] - s_phi[ly + 1][lx]) * r2h;
          grad[1] = (s_phi[ly + 2][lx + 1] - s_phi[ly][lx + 1]) * r2h;
          grad[2] = (php - phm) * r2h;
        }
        // a uniform external field adds to the self-gravity (exact when 0)
#pragma unroll
        for (int d = 0; d < 3; d++) grad[d] -= gext[d];
        // momentum slots receive v' = m' / rho
        const T irho = rcp(pc_[0]);
        const uint32_t xy = xy_c;
#pragma unroll
        for (int d = 0; d < 3; d++)
          st_at(as_global((T*)R.tmp[oidx(GP_MX + d)]), zk, xy, (mc[d] - r * dP[d] - tau * pc_[0] * grad[d]) * irho);
        T Enew = E - r * dPV - tau * (mc[0] * grad[0] + mc[1] * grad[1] + mc[2] * grad[2]);
        T enew = ec - r * gm1 * ec * dV;
        if (cool) {
          const T qc = cooling_rate<T>(R.ph, pc_[0], pc_[4] * irho);  // theta = p / rho
          Enew -= tau * qc;
          enew -= tau * qc;
        }
        st_at(as_global((T*)R.tmp[oidx(GP_E)]), zk, xy, Enew);
        st_at(as_global((T*)R.tmp[oidx(GP_EINT)]), zk, xy, enew);
      }
      prims(rho_n, m_n, e_n, pc_);
#pragma unroll
      for (int d = 0; d < 3; d++) mc[d] = m_n[d];
      ec = e_n;
      phc = php;
    }
    lds_barrier();  // the next item restages the tiles
  }
}

template <typename T, class S>
__global__ void __launch_bounds__(kBlock, 2) k_eul_bme(const RunDev<T>* __restrict__ runs,
                                                    const WorkItem* __restrict__ work, unsigned nwork, int parity) {
  __shared__ T s_p[kBmePrims][S::LY][S::LX];
  __shared__ T s_phi[S::LY][S::LX];
  const int lx = threadIdx.x, ly = threadIdx.y;
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const WorkItem it = load_item(work, w);
    const int run = it.run;
    const RunDev<T>& R = runs[run];
    const Grid& g = R.g;
    const Column col = make_column<S>(g, it, false);
    const Column pc = make_phi_column<S>(g, it);
    const bool grav = R.ph.G != 0.0;
    const T gext[3] = {(T)R.ph.gext[0], (T)R.ph.gext[1], (T)R.ph.gext[2]};
    const size_t nxy = (size_t)g.nx * g.ny;
    const double tau_d = R.sc->dt;
    const T tau = (T)tau_d, r = (T)(tau_d / g.h), r2h = (T)(0.5 / g.h);
    const gptr<const double> n_in = as_global((const double*)R.dens[parity][1]);
    gptr<const T> q_in[3], P_in[6];
#pragma unroll
    for (int d = 0; d < 3; d++) q_in[d] = as_global((const T*)R.cur[oidx(GP_QX + d)]);
#pragma unroll
    for (int m = 0; m < 6; m++) P_in[m] = as_global((const T*)R.cur[oidx(GP_PXX + m)]);
    const gptr<const T> phi = as_global((const T*)R.phi);
    auto load = [&](size_t z, uint32_t xy, double& n, T q[3], T P[6]) {
      n = ld_at(n_in, z, xy);
#pragma unroll
      for (int d = 0; d < 3; d++) q[d] = ld_at(q_in[d], z, xy);
#pragma unroll
      for (int m = 0; m < 6; m++) P[m] = ld_at(P_in[m], z, xy);
    };
    auto prims = [&](double n, const T q[3], const T P[6], T (&a)[kBmePrims]) {
      a[0] = (T)n;
      const T in_ = rcp(a[0]);
#pragma unroll
      for (int d = 0; d < 3; d++) a[1 + d] = q[d] * in_;
#pragma unroll
      for (int m = 0; m < 6; m++) a[4 + m] = P[m];
    };

    // prologue: plane k0 into registers, the potential of plane k0 - 1 into
    // the LDS centre, and the z- face of plane k0; from then on each plane's
    // z- face is the previous plane's z+ face (same inputs, same bits)
    T pc_[kBmePrims], qc[3], phc;
    T usz[3], psz[3];  // z+ face of the previous plane
    {
      const size_t zm = plane_at(g, col.k0 - 1, g.bc[2]), z0 = nxy * (size_t)col.k0;
      double n, n0;
      T q[3], P[6], P0[6], pm[kBmePrims];
      load(zm, col.xy_c, n, q, P);
      load(z0, col.xy_c, n0, qc, P0);
      const T phm = phi_at(phi, grav, phi_plane(g, col.k0 - 1), pc.xy_c);
      phc = phi_at(phi, grav, phi_plane(g, col.k0), pc.xy_c);
      prims(n, q, P, pm);
      prims(n0, qc, P0, pc_);
      bme_face<T, 2>(bme_of<2>(pm), bme_of<2>(pc_), usz, psz);
      s_phi[ly + 1][lx + 1] = phm;
    }
    // the ring of each plane is fetched a plane ahead, so staging it never
    // waits on memory (every lane has a valid ring address)
    double n_h;
    T q_h[3], P_h[6], phh;
    auto load_ring = [&](int kr) {
      const size_t zr = nxy * (size_t)kr;
      load(zr, fresh(col.xy_h), n_h, q_h, P_h);
      phh = phi_at(phi, grav, phi_plane(g, kr), fresh(pc.xy_h));
    };
    load_ring(col.k0);
    for (int k = col.k0; k < col.k1; k++) {
      const size_t zk = nxy * (size_t)k, zp = plane_at(g, k + 1, g.bc[2]);
      const uint32_t xy_c = fresh(col.xy_c);
      const uint32_t pxy_c = fresh(pc.xy_c);
      const T phm = s_phi[ly + 1][lx + 1];
      lds_barrier();  // every thread is done with the previous plane's tiles
      if (col.ring) {
        T a[kBmePrims];
        prims(n_h, q_h, P_h, a);
#pragma unroll
        for (int f = 0; f < kBmePrims; f++) s_p[f][col.hr][col.hc] = a[f];
        s_phi[col.hr][col.hc] = phh;
      }
#pragma unroll
      for (int f = 0; f < kBmePrims; f++) s_p[f][ly + 1][lx + 1] = pc_[f];
      s_phi[ly + 1][lx + 1] = phc;
      // the next plane's centres (needed by the z+ face, formed last), the
      // next ring, then this plane's W (needed by the store)
      double n_n;
      T q_n[3], P_n[6], W[6];
      load(zp, xy_c, n_n, q_n, P_n);
      const T php = phi_at(phi, grav, phi_plane(g, k + 1), pxy_c);
      if (k + 1 < col.k1) load_ring(k + 1);
#pragma unroll
      for (int m = 0; m < 6; m++) W[m] = ld_at(as_global((const T*)R.cur[oidx(GP_WXX + m)]), zk, xy_c);
      lds_barrier();

      if (col.active) {
        BmeCentre<T> C;
        C.n = pc_[0];
#pragma unroll
        for (int d = 0; d < 3; d++) C.u[d] = pc_[1 + d];
#pragma unroll
        for (int m = 0; m < 6; m++) C.P[m] = pc_[4 + m];
        T dq[3] = {T(0), T(0), T(0)};
        T dW[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        T dPi[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        T usm[3], psm[3], usp[3], psp[3];
        bme_face<T, 0>(bme_at<0>(s_p, ly + 1, lx), centre_side<0>(C), usm, psm);
        bme_face<T, 0>(centre_side<0>(C), bme_at<0>(s_p, ly + 1, lx + 2), usp, psp);
        bme_face_pair<0>(usm, psm, usp, psp, C, dq, dW, dPi);
        bme_face<T, 1>(bme_at<1>(s_p, ly, lx + 1), centre_side<1>(C), usm, psm);
        bme_face<T, 1>(centre_side<1>(C), bme_at<1>(s_p, ly + 2, lx + 1), usp, psp);
        bme_face_pair<1>(usm, psm, usp, psp, C, dq, dW, dPi);
        T pn[kBmePrims];
        prims(n_n, q_n, P_n, pn);
        bme_face<T, 2>(centre_side<2>(C), bme_of<2>(pn), usp, psp);
        bme_face_pair<2>(usz, psz, usp, psp, C, dq, dW, dPi);
#pragma unroll
        for (int i = 0; i < 3; i++) {
          usz[i] = usp[i];
          psz[i] = psp[i];
        }
        T grad[3] = {T(0), T(0), T(0)};
        if (grav) {
          grad[0] = (s_phi[ly + 1][lx + 2] - s_phi[ly + 1][lx]) * r2h;
          grad[1] = (s_phi[ly + 2][lx + 1] - s_phi[ly][lx + 1]) * r2h;
          grad[2] = (php - phm) * r2h;
        }
        // a uniform external field adds to the self-gravity (exact when 0)
#pragma unroll
        for (int d = 0; d < 3; d++) grad[d] -= gext[d];
        // momentum slots receive u' = q' / n
        const T inb = rcp(C.n);
        const uint32_t xy = xy_c;
#pragma unroll
        for (int d = 0; d < 3; d++)
          st_at(as_global((T*)R.tmp[oidx(GP_QX + d)]), zk, xy, (qc[d] - r * dq[d] - tau * C.n * grad[d]) * inb);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = a; b < 3; b++) {
            const int m = sym(a, b);
            st_at(as_global((T*)R.tmp[oidx(GP_WXX + m)]), zk, xy,
                  W[m] - r * dW[m] - tau * (qc[a] * grad[b] + qc[b] * grad[a]));
            st_at(as_global((T*)R.tmp[oidx(GP_PXX + m)]), zk, xy, C.P[m] - r * dPi[m]);
          }
      }
      prims(n_n, q_n, P_n, pc_);
#pragma unroll
      for (int d = 0; d < 3; d++) qc[d] = q_n[d];
      phc = php;
    }
    lds_barrier();  // the next item restages the tiles
  }
}

template <typename T, class S>
void launch_eulerian_shape(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity, int comp,
                           bool cool, unsigned nblocks, hipStream_t st) {
  const dim3 blk(S::TX, S::TY, 1);
  if (comp == COMP_GAS && cool)
    k_eul_gas<T, true, S><<<nblocks, blk, 0, st>>>(runs, work, nwork, parity);
  else if (comp == COMP_GAS)
    k_eul_gas<T, false, S><<<nblocks, blk, 0, st>>>(runs, work, nwork, parity);
  else
    k_eul_bme<T, S><<<nblocks, blk, 0, st>>>(runs, work, nwork, parity);
}

template <typename T>
void launch_eulerian(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity, int comp,
                     bool cool, int shape, unsigned nblocks, hipStream_t st) {
  if (shape == 1)
    launch_eulerian_shape<T, Shape1>(runs, work, nwork, parity, comp, cool, nblocks, st);
  else
    launch_eulerian_shape<T, Shape0>(runs, work, nwork, parity, comp, cool, nblocks, st);
}

template void launch_eulerian<double>(const RunDev<double>*, const WorkItem*, unsigned, int, int, bool, int,
                                      unsigned, hipStream_t);
template void launch_eulerian<float>(const RunDev<float>*, const WorkItem*, unsigned, int, int, bool, int, unsigned,
                                     hipStream_t);

}  // namespace gp
