// Lagrangian (FlIC) stage of one GPUPEGAS step (Kulikov, arXiv:1311.0861,
// Sec. 2.1, Fig. "lagrange"), with the end-of-step cell work fused in:
//   - every quantity f obeys (f^{n+1} - f^n)/tau + sum_d (F_{d+} - F_{d-})/h = 0,
//     F on a face = (1/4) sum over its 4 corners of v_d f^+, f^+ the upwind
//     cell value for that corner's velocity; a corner velocity is the mean of
//     the 8 cells sharing the vertex (post-Eulerian m/rho for the gas, q/n for
//     the stars), formed on chip from the velocity tiles by one fixed
//     expression, so every cell sharing a vertex sees the same bits; the flux
//     is written per cell as A+ f_c + A- f_{c+e_d};
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
#include <limits>

#include "column.hpp"
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
// slots of a partial row (tid = the thread's index in the workgroup).
__device__ __forceinline__ void block_reduce_store(Acc& a, gptr<double> slots, int tid) {
  __shared__ double red[kBlock / 64][kNS];
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

// sqrt(max(x, 0)) for the signal speeds, from the Newton-refined reciprocal
// square root, without a branch: 0 where x is not positive (NaN included, as
// fmax gives); a subnormal x gives x / sqrt(smallest normal), as negligible
// beside the velocity it is added to as its square root would be.
template <typename T>
__device__ __forceinline__ T sqrt_pos(T x) {
  const T y = x * rsqrt_nr(fmax(x, std::numeric_limits<T>::min()));
  return x > T(0) ? y : T(0);
}

// Gas: kappa integrand |E - e - |m|^2/(2 rho)| (Sec. 2.4) and kinetic energy
// (ir = 1 / rho: every division of a cell's end-of-step terms is by its
// density, so one reciprocal serves them all).
template <typename T>
__device__ __forceinline__ T gas_kappa(T ir, const T m[3], T E, T e, T& ekin) {
  ekin = T(0.5) * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * ir;
  return fabs(E - e - ekin);
}

// Gas diagnostics of a finished cell: signal speed, sums, error bits.
template <typename T>
__device__ __forceinline__ void gas_terms(Acc& a, double rho, T ir, const T m[3], T E, T e, T gamma) {
  const T p = (gamma - T(1)) * e;
  const T cs = sqrt_pos(gamma * p * ir);
  T sp = T(0);
#pragma unroll
  for (int d = 0; d < 3; d++) sp = fmax(sp, fabs(m[d]) * ir + cs);
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
__device__ __forceinline__ T bme_kappa(T iv, const T q[3], const T P[6], const T W[6], T Tt[6]) {
  T kb = T(0);
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = a; b < 3; b++) {
      const int s = sym(a, b);
      Tt[s] = W[s] - q[a] * q[b] * iv;
      kb += fabs(Tt[s] - P[s]);
    }
  return kb;
}

template <typename T>
__device__ __forceinline__ void bme_terms(Acc& a, double n, T iv, const T q[3], const T P[6], const T W[6]) {
  T sp = T(0);
#pragma unroll
  for (int d = 0; d < 3; d++) sp = fmax(sp, fabs(q[d]) * iv + sqrt_pos(T(3) * P[sym(d, d)] * iv));
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

// ---- Lagrangian flux update -------------------------------------------------

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

// Flux update of one field from its 7 post-Eulerian point values x[] (point
// order: centre, minus / plus x, y, z).
template <typename T>
__device__ __forceinline__ T advect7(const T x[7], const Weights<T>& w) {
  T v = w.c * x[0];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    v += w.p[d] * x[2 + 2 * d];
    v += w.m[d] * x[1 + 2 * d];
  }
  return v;
}

// ---- column kernels ---------------------------------------------------------
//
// A workgroup owns a 64 x 4 tile of cells and walks a chunk of z planes.  For
// plane k the tile of every advected field, with a one-cell ring of x / y
// neighbours, sits in LDS; the z+ neighbours come into registers one plane
// ahead and the z- ones are read back from the LDS centres of the previous
// plane.  The velocity tiles of planes k and k+1 (with rings) are both held,
// which is what the corner velocities of vertex plane k+1 need; the corners
// of vertex planes k and k+1 sit in a double-buffered LDS tile.  Each plane
// of a field is thus read from memory once per tile plus its ring, in
// coalesced rows, instead of 7 times through the cache hierarchy, and the
// corner velocities never go to memory.

// vertex tile of a cell tile of shape S: corner values staged per vertex
// plane, and per thread
template <class S>
struct Vertex {
  static constexpr int VX = S::TX + 1, VY = S::TY + 1;
  static constexpr int TILE = 3 * VX * VY;
  static constexpr int PER = (TILE + kBlock - 1) / kBlock;
};

// Advected fields of a component (after the density), its corner velocity
// components and density slot.
template <int C>
struct Comp;
template <>
struct Comp<COMP_GAS> {
  static constexpr int kNF = 5;  // m_x m_y m_z E e
  static constexpr int kFirst = GP_MX;
  static constexpr int kVel = 0;
  static constexpr int kDens = 0;
};
template <>
struct Comp<COMP_BME> {
  static constexpr int kNF = 15;  // q_x q_y q_z, Pi (6), W (6)
  static constexpr int kFirst = GP_QX;
  static constexpr int kVel = 3;
  static constexpr int kDens = 1;
};

// Gas epilogue: kappa, energy balance, stores and diagnostics of a cell.
template <typename T>
__device__ __forceinline__ void gas_finish(Acc& acc, const RunDev<T>& R, int parity, size_t z, uint32_t xy,
                                           double rho, const T nv[5], double out) {
  T m[3] = {nv[0], nv[1], nv[2]};
  const T E = nv[3];
  T e = nv[4];
  T ekin;
  const T ir = rcp(T(rho));
  acc.v[S_KAPPA] += (double)gas_kappa(ir, m, E, e, ekin);
  if (R.ph.eta >= 0.0) {
    const T et = E - ekin;
    if (et > (T)R.ph.eta * E) {
      e = et;
      acc.v[S_NSYNC] += 1.0;
    }
  }
  acc.v[S_OUTFLOW] += out;
  st_at(as_global(R.dens[parity ^ 1][0]), z, xy, rho);
#pragma unroll
  for (int d = 0; d < 3; d++) st_at(as_global(R.cur[oidx(GP_MX + d)]), z, xy, m[d]);
  st_at(as_global(R.cur[oidx(GP_E)]), z, xy, E);
  st_at(as_global(R.cur[oidx(GP_EINT)]), z, xy, e);
  gas_terms(acc, rho, ir, m, E, e, (T)R.ph.gamma);
}

// Stars / dark matter epilogue, streamed over the six stress / energy pairs
// (next(m, P_m, W_m) forms pair m): kappa, the energy balance of each
// diagonal stress, stores and diagnostics of a cell.
template <typename T, typename Next>
__device__ __forceinline__ void bme_stream(Acc& acc, const RunDev<T>& R, int parity, size_t z, uint32_t xy,
                                           double n, const T q[3], double out, Next next) {
  const T iv = rcp(T(n));
  const T eta = (T)R.ph.eta;
  const bool balance = R.ph.eta >= 0.0;
  T kb = T(0), sp = T(0), wtr = T(0);
  bool any = false, fin = isfinite(n), stress_ok = true;
#pragma unroll
  for (int d = 0; d < 3; d++) fin = fin && isfinite(q[d]);
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = a; b < 3; b++) {
      const int m = sym(a, b);
      T P, W;
      next(m, P, W);
      const T Tt = W - q[a] * q[b] * iv;
      kb += fabs(Tt - P);
      if (a == b) {
        if (balance && Tt > eta * W) {
          P = Tt;
          any = true;
        }
        sp = fmax(sp, fabs(q[a]) * iv + sqrt_pos(T(3) * P * iv));
        stress_ok = stress_ok && (P > T(0));
        wtr += W;
      }
      fin = fin && isfinite(P) && isfinite(W);
      st_at(as_global(R.cur[oidx(GP_PXX + m)]), z, xy, P);
      st_at(as_global(R.cur[oidx(GP_WXX + m)]), z, xy, W);
    }
  acc.v[S_KAPPA] += (double)kb;
  if (any) acc.v[S_NSYNC] += 1.0;
  acc.v[S_OUTFLOW] += out;
  st_at(as_global(R.dens[parity ^ 1][1]), z, xy, n);
#pragma unroll
  for (int d = 0; d < 3; d++) st_at(as_global(R.cur[oidx(GP_QX + d)]), z, xy, q[d]);
  acc.v[S_SPEED] = fmax(acc.v[S_SPEED], (double)sp);
  acc.v[S_MASS] += n;
#pragma unroll
  for (int d = 0; d < 3; d++) acc.v[S_MOMX + d] += (double)q[d];
  acc.v[S_ENERGY] += 0.5 * (double)wtr;
  uint32_t err = 0u;
  if (!fin) err |= ERR_NONFINITE;
  if (!(n > 0.0)) err |= ERR_DENSITY;
  if (!stress_ok) err |= ERR_STRESS;
  acc.err |= err;
}

// Per-cell inputs of the flux update: the face coefficients, weights and the
// 7-point density of the centre cell.
template <typename T>
struct CellFlux {
  T ap[3][2], am[3][2];
  Weights<T> w;
  double dn[7];
};

// Flux update of the field in tile slot t from its 7 post-Eulerian values
// (x / y ring and centre from the LDS tile, z neighbours from registers).
template <typename T, int NT, int LY, int LX>
__device__ __forceinline__ T field_update(const T (&tile)[NT][LY][LX], int t, int lx, int ly, T zm, T zp,
                                          const CellFlux<T>& cf) {
  T x[7];
  x[0] = tile[t][ly + 1][lx + 1];
  x[1] = tile[t][ly + 1][lx];
  x[2] = tile[t][ly + 1][lx + 2];
  x[3] = tile[t][ly][lx + 1];
  x[4] = tile[t][ly + 2][lx + 1];
  x[5] = zm;
  x[6] = zp;
  return advect7(x, cf.w);
}

// Waves per SIMD the register budget aims at (the stars / DM tiles take
// 67-76 KB of LDS per workgroup in FP64, which allows two workgroups per CU;
// in FP32 half that, and three fit).
template <int C, typename T>
constexpr int lag_waves() {
  return C == COMP_GAS ? 3 : (sizeof(T) == 8 ? 2 : 3);
}

template <int C, typename T, class S>
__global__ void __launch_bounds__(kBlock, (lag_waves<C, T>())) k_lagrangian(const RunDev<T>* __restrict__ runs,
                                                                        const WorkItem* __restrict__ work,
                                                                        unsigned nwork, int parity,
                                                                        double* __restrict__ partials) {
  using K = Comp<C>;
  constexpr int NF = K::kNF;
  constexpr int O0 = K::kFirst < GP_N ? K::kFirst - 1 : K::kFirst - 2;  // first "other" slot
  constexpr int kLX = S::LX, kLY = S::LY;
  constexpr int kVX = Vertex<S>::VX, kVY = Vertex<S>::VY, kVTile = Vertex<S>::TILE, kVPer = Vertex<S>::PER;
  __shared__ double s_dn[kLY][kLX];
  __shared__ T s_f[NF - 3][kLY][kLX];  // plane k of the fields after the velocities
  __shared__ T s_u[2][3][kLY][kLX];    // velocity tiles of planes k and k+1, alternating
  __shared__ T s_v[2][kVTile];        // corner velocities of vertex planes k and k+1
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + S::TX * ly;
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const WorkItem it = load_item(work, w);
    const RunDev<T>& R = runs[it.run];
    const Grid& g = R.g;
    const Column col = make_column<S>(g, it, false);
    const int k0 = col.k0, k1 = col.k1, i = col.i, j = col.j;
    const bool active = col.active, ring = col.ring;
    const int hr = col.hr, hc = col.hc;
    const size_t nxy = (size_t)g.nx * g.ny;
    const gptr<const double> din = as_global((const double*)R.dens[parity][K::kDens]);
    auto fin = [&](int f) { return as_global((const T*)R.tmp[O0 + f]); };
    auto plane = [&](int k) -> size_t { return plane_at(g, k, g.bc[2]); };

    // Corner velocities.  Vertex (I, J, K) is the mean of the 8 cells I-1..I,
    // J-1..J, K-1..K (boundary rule outside the grid); the cells come from
    // the velocity tiles (with their rings) of planes K-1 and K.  Entry e of
    // the vertex tile (component e / (kVX kVY), vertex row and column within
    // it) is formed by thread e mod kBlock; vo[] is the tile offset of its
    // lower-left cell.
    int vo[kVPer];
#pragma unroll
    for (int q = 0; q < kVPer; q++) {
      const int e = min(tid + q * kBlock, kVTile - 1);
      const int d = e / (kVX * kVY), rem = e % (kVX * kVY);
      vo[q] = (d * kLY + rem / kVX) * kLX + rem % kVX;
    }
    // The 8-cell sum is the plane K-1 sum plus the plane K sum of the 2 x 2
    // cells, each summed y-major then x.  The plane K sums stay in registers
    // as the plane K-1 sums of the next vertex plane (half the LDS reads of
    // summing all eight cells per vertex plane).
    T hs[kVPer];
    auto xy_sum = [&](const T (&u)[3][kLY][kLX], int q) {
      const T* a = &u[0][0][0];
      const int o = vo[q];
      T v = a[o];
      v += a[o + 1];
      v += a[o + kLX];
      v += a[o + kLX + 1];
      return v;
    };
    auto corner_plane = [&](const T (&hi)[3][kLY][kLX], T* dst) {
#pragma unroll
      for (int q = 0; q < kVPer; q++) {
        const T h = xy_sum(hi, q);
        if (tid + q * kBlock < kVTile) dst[tid + q * kBlock] = (hs[q] + h) * T(0.125);
        hs[q] = h;
      }
    };
    // centre and ring of plane z of the three velocities into tile u
    auto stage_velocity = [&](size_t z, uint32_t xy_h, T (&u)[3][kLY][kLX], const T ctr[3]) {
#pragma unroll
      for (int d = 0; d < 3; d++) u[d][ly + 1][lx + 1] = ctr[d];
      if (ring) {
#pragma unroll
        for (int d = 0; d < 3; d++) u[d][hr][hc] = ld_at(fin(d), z, xy_h);
      }
    };

    const uint32_t xy_c = col.xy_c, xy_h = col.xy_h;
    // Every line of a plane is fetched by its owner (as centres) and by the
    // neighbouring tiles (as their ring).  Both fetches are issued in the
    // same plane step of the sweep, so whichever comes second finds the line
    // in the XCD's L2.  In the step of plane k the loop fetches
    //   - the density and the fields after the velocities of plane k + 1,
    //     centres and ring: the centres are this step's z+ neighbours and
    //     next step's centres, the ring is staged next step;
    //   - the velocities of plane k + 2, centres and ring: staged next step
    //     as the velocity tile the corners of vertex plane k + 2 need.
    // The z- neighbours are read back from the LDS centres of the previous
    // plane and the z+ velocities from the velocity tile of plane k + 1.
    // prologue: plane k0 - 1 goes to the LDS centre slots and to the
    // velocity tile s_u[(k0 + 1) & 1], the velocities of plane k0 to
    // s_u[k0 & 1] (the two give the corners of vertex plane k0); the rest of
    // plane k0 (centres and ring) and the velocities of plane k0 + 1 come
    // into registers.
    double dc, rdn, dn1;
    T fc[NF], rf[NF], uc[3], ur[3];  // fc, rf: slots 3..NF-1
    {
      const size_t zm = plane(k0 - 1), z0 = nxy * (size_t)k0, z1 = plane(k0 + 1);
      T um[3], u0[3];
      s_dn[ly + 1][lx + 1] = ld_at(din, zm, xy_c);
#pragma unroll
      for (int f = 0; f < 3; f++) um[f] = ld_at(fin(f), zm, xy_c);
#pragma unroll
      for (int f = 3; f < NF; f++) s_f[f - 3][ly + 1][lx + 1] = ld_at(fin(f), zm, xy_c);
      stage_velocity(zm, xy_h, s_u[(k0 + 1) & 1], um);
      dc = ld_at(din, z0, xy_c);
#pragma unroll
      for (int f = 0; f < 3; f++) u0[f] = ld_at(fin(f), z0, xy_c);
#pragma unroll
      for (int f = 3; f < NF; f++) fc[f] = ld_at(fin(f), z0, xy_c);
      stage_velocity(z0, xy_h, s_u[k0 & 1], u0);
      rdn = ld_at(din, z0, xy_h);
#pragma unroll
      for (int f = 3; f < NF; f++) rf[f] = ld_at(fin(f), z0, xy_h);
#pragma unroll
      for (int d = 0; d < 3; d++) {
        uc[d] = ld_at(fin(d), z1, xy_c);
        ur[d] = ld_at(fin(d), z1, xy_h);
      }
      dn1 = ld_at(din, z1, xy_c);
      lds_barrier();
#pragma unroll
      for (int q = 0; q < kVPer; q++) hs[q] = xy_sum(s_u[(k0 + 1) & 1], q);
      corner_plane(s_u[k0 & 1], s_v[k0 & 1]);
    }

    Acc acc;
    acc_init(acc);
    T apz = T(0), amz = T(0);  // A+ / A- of the z+ face of the previous plane
    const double rd = R.sc->dt / g.h;
    const T r = (T)rd;
    for (int k = k0; k < k1; k++) {
      const size_t zk = nxy * (size_t)k, zp = plane(k + 1), zpp = plane(k + 2);
      const int cu = k & 1, nu = cu ^ 1;  // velocity tiles of planes k and k+1
      const uint32_t xy_c = fresh(col.xy_c), xy_h = fresh(col.xy_h);
      // the previous centres become the z- neighbours (each thread reads back
      // its own slot; the velocities from the tile of plane k - 1)
      const double dm = s_dn[ly + 1][lx + 1];
      T fm[NF];
#pragma unroll
      for (int f = 0; f < 3; f++) fm[f] = s_u[nu][f][ly + 1][lx + 1];
#pragma unroll
      for (int f = 3; f < NF; f++) fm[f] = s_f[f - 3][ly + 1][lx + 1];
      lds_barrier();  // every thread is done with the previous plane's tiles
      // plane k (ring and centres) and the velocity tile of plane k + 1
      // (every lane has a valid ring address; only ring lanes store)
      if (ring) {
        s_dn[hr][hc] = rdn;
#pragma unroll
        for (int f = 3; f < NF; f++) s_f[f - 3][hr][hc] = rf[f];
#pragma unroll
        for (int d = 0; d < 3; d++) s_u[nu][d][hr][hc] = ur[d];
      }
      s_dn[ly + 1][lx + 1] = dc;
#pragma unroll
      for (int f = 3; f < NF; f++) s_f[f - 3][ly + 1][lx + 1] = fc[f];
#pragma unroll
      for (int d = 0; d < 3; d++) s_u[nu][d][ly + 1][lx + 1] = uc[d];
      // this step's fetches (the z+ centres first: they are needed first;
      // the z+ density, needed before them, was fetched a step earlier)
      const double dp = dn1;
      T fp[NF];
#pragma unroll
      for (int f = 3; f < NF; f++) fp[f] = ld_at(fin(f), zp, xy_c);
      if (k + 1 < k1) {
        issue_order();
        dn1 = ld_at(din, zpp, xy_c);
        rdn = ld_at(din, zp, xy_h);
#pragma unroll
        for (int f = 3; f < NF; f++) rf[f] = ld_at(fin(f), zp, xy_h);
#pragma unroll
        for (int d = 0; d < 3; d++) {
          uc[d] = ld_at(fin(d), zpp, xy_c);
          ur[d] = ld_at(fin(d), zpp, xy_h);
        }
      }
      lds_barrier();
      corner_plane(s_u[nu], s_v[(k + 1) & 1]);
      lds_barrier();

      if (active) {
        CellFlux<T> cf;
        // A+ / A- of the six faces from the corners in vertex planes k, k+1:
        // a quarter of the sums of max(v, 0) and of min(v, 0) over a face's
        // four corners, formed as (S + |S|') / 8 and (S - |S|') / 8 from the
        // sum S of the corner values and the sum |S|' of their magnitudes
        // (exactly 0 where all four corners share a sign); both cells of a
        // face sum its corners in the same order.
#pragma unroll
        for (int d = 0; d < 2; d++) {
          T sum[2] = {T(0), T(0)}, mag[2] = {T(0), T(0)};
#pragma unroll
          for (int s = 0; s < 8; s++) {
            const int sx = s & 1, sy = (s >> 1) & 1, sz = (s >> 2) & 1;
            const T v = s_v[(k + sz) & 1][d * kVX * kVY + (ly + sy) * kVX + lx + sx];
            const int side = d == 0 ? sx : sy;
            sum[side] += v;
            mag[side] += fabs(v);
          }
#pragma unroll
          for (int side = 0; side < 2; side++) {
            cf.ap[d][side] = (sum[side] + mag[side]) * T(0.125);
            cf.am[d][side] = (sum[side] - mag[side]) * T(0.125);
          }
        }
        // z faces: the four corners of vertex plane K in the same order.  In
        // the gas kernel the z- face of plane k is the z+ face of plane k - 1
        // (same bits), carried in registers after the first plane of the
        // item; the stars / DM kernel, at its register limit, recomputes it
        // (carrying measured 1% slower there, 2% faster for the gas).
        auto z_side = [&](int kv, T& ap, T& am) {
          T sum = T(0), mag = T(0);
#pragma unroll
          for (int s = 0; s < 4; s++) {
            const T v = s_v[kv & 1][2 * kVX * kVY + (ly + (s >> 1)) * kVX + lx + (s & 1)];
            sum += v;
            mag += fabs(v);
          }
          ap = (sum + mag) * T(0.125);
          am = (sum - mag) * T(0.125);
        };
        if (C != COMP_GAS || k == k0) z_side(k, apz, amz);
        cf.ap[2][0] = apz;
        cf.am[2][0] = amz;
        z_side(k + 1, apz, amz);
        cf.ap[2][1] = apz;
        cf.am[2][1] = amz;
        cf.dn[0] = dc;
        cf.dn[1] = s_dn[ly + 1][lx];
        cf.dn[2] = s_dn[ly + 1][lx + 2];
        cf.dn[3] = s_dn[ly][lx + 1];
        cf.dn[4] = s_dn[ly + 2][lx + 1];
        cf.dn[5] = dm;
        cf.dn[6] = dp;
        double out;
        const double dnew = advect_density(cf.dn, cf.ap, cf.am, rd, g, i, j, k, out);
        cf.w = flux_weights(cf.ap, cf.am, r);
        const uint32_t xy = xy_c;  // i + nx j for a cell inside the grid
        // velocities: x / y neighbours from the velocity tile of plane k
        auto vel_update = [&](int d) -> T {
          T x[7];
          x[0] = s_u[cu][d][ly + 1][lx + 1];
          x[1] = s_u[cu][d][ly + 1][lx];
          x[2] = s_u[cu][d][ly + 1][lx + 2];
          x[3] = s_u[cu][d][ly][lx + 1];
          x[4] = s_u[cu][d][ly + 2][lx + 1];
          x[5] = fm[d];
          x[6] = s_u[nu][d][ly + 1][lx + 1];
#pragma unroll
          for (int p = 0; p < 7; p++) x[p] *= (T)cf.dn[p];
          return advect7(x, cf.w);
        };
        if constexpr (C == COMP_GAS) {
          T nv[NF];
#pragma unroll
          for (int d = 0; d < 3; d++) nv[d] = vel_update(d);
#pragma unroll
          for (int f = 3; f < NF; f++) nv[f] = field_update<T, NF - 3>(s_f, f - 3, lx, ly, fm[f], fp[f], cf);
          gas_finish(acc, R, parity, zk, xy, dnew, nv, out);
        } else {
          // momenta first (the thermal tensor needs them), then each stress /
          // energy pair is finished and stored before the next is formed
          T q[3];
#pragma unroll
          for (int d = 0; d < 3; d++) q[d] = vel_update(d);
          bme_stream(acc, R, parity, zk, xy, dnew, q, out, [&](int m, T& P, T& W) {
            P = field_update<T, NF - 3>(s_f, m, lx, ly, fm[3 + m], fp[3 + m], cf);
            W = field_update<T, NF - 3>(s_f, 6 + m, lx, ly, fm[9 + m], fp[9 + m], cf);
          });
        }
      }
      dc = dp;
#pragma unroll
      for (int f = 3; f < NF; f++) fc[f] = fp[f];
    }
    block_reduce_store(acc, as_global(partials) + ((size_t)R.row0 + it.row) * kNP + C * kNS, tid);
  }
}

// Diagnostics terms of one component of a cell of a state that has not been
// advanced.
template <int C, typename T>
__device__ __forceinline__ void init_cell(Acc& acc, const RunDev<T>& R, int parity, size_t z, uint32_t xy) {
  auto f = [&](int field) { return ld_at(as_global((const T*)R.cur[oidx(field)]), z, xy); };
  if constexpr (C == COMP_GAS) {
    const double rho = ld_at(as_global((const double*)R.dens[parity][0]), z, xy);
    T m[3];
#pragma unroll
    for (int d = 0; d < 3; d++) m[d] = f(GP_MX + d);
    const T E = f(GP_E), e = f(GP_EINT);
    T ekin;
    const T ir = rcp(T(rho));
    acc.v[S_KAPPA] += (double)gas_kappa(ir, m, E, e, ekin);
    gas_terms(acc, rho, ir, m, E, e, (T)R.ph.gamma);
  } else {
    const double n = ld_at(as_global((const double*)R.dens[parity][1]), z, xy);
    T q[3], P[6], W[6], Tt[6];
#pragma unroll
    for (int d = 0; d < 3; d++) q[d] = f(GP_QX + d);
#pragma unroll
    for (int a = 0; a < 6; a++) {
      P[a] = f(GP_PXX + a);
      W[a] = f(GP_WXX + a);
    }
    const T iv = rcp(T(n));
    acc.v[S_KAPPA] += (double)bme_kappa(iv, q, P, W, Tt);
    bme_terms(acc, n, iv, q, P, W);
  }
}

// Partial rows of one component of a state that has not been advanced, over
// the same items (and rows) as that component's Lagrangian kernel.
template <int C, typename T, class S>
__global__ void __launch_bounds__(kBlock) k_init_partials(const RunDev<T>* __restrict__ runs,
                                                          const WorkItem* __restrict__ work, unsigned nwork,
                                                          int parity, double* __restrict__ partials) {
  const WorkRange wr = xcd_range(nwork);
  for (unsigned w = wr.first; w < wr.end; w += wr.stride) {
    const WorkItem it = load_item(work, w);
    const RunDev<T>& R = runs[it.run];
    const Grid& g = R.g;
    const Column col = make_column<S>(g, it, false);
    Acc acc;
    acc_init(acc);
    if (col.active)
      for (int k = col.k0; k < col.k1; k++) init_cell<C, T>(acc, R, parity, (size_t)g.nx * g.ny * k, col.xy_c);
    block_reduce_store(acc, as_global(partials) + ((size_t)R.row0 + it.row) * kNP + C * kNS,
                       (int)threadIdx.x + S::TX * (int)threadIdx.y);
  }
}

template <typename T, class S>
void launch_lagrangian_shape(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity,
                             double* partials, int comp, bool init, unsigned nblocks, hipStream_t st) {
  const dim3 blk(S::TX, S::TY, 1);
  if (init && comp == COMP_GAS)
    k_init_partials<COMP_GAS, T, S><<<nblocks, blk, 0, st>>>(runs, work, nwork, parity, partials);
  else if (init)
    k_init_partials<COMP_BME, T, S><<<nblocks, blk, 0, st>>>(runs, work, nwork, parity, partials);
  else if (comp == COMP_GAS)
    k_lagrangian<COMP_GAS, T, S><<<nblocks, blk, 0, st>>>(runs, work, nwork, parity, partials);
  else
    k_lagrangian<COMP_BME, T, S><<<nblocks, blk, 0, st>>>(runs, work, nwork, parity, partials);
}

template <typename T>
void launch_lagrangian(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity, double* partials,
                       int comp, int shape, unsigned nblocks, hipStream_t st) {
  if (shape == 1)
    launch_lagrangian_shape<T, Shape1>(runs, work, nwork, parity, partials, comp, false, nblocks, st);
  else
    launch_lagrangian_shape<T, Shape0>(runs, work, nwork, parity, partials, comp, false, nblocks, st);
}
template <typename T>
void launch_init_partials(const RunDev<T>* runs, const WorkItem* work, unsigned nwork, int parity,
                          double* partials, int comp, int shape, unsigned nblocks, hipStream_t st) {
  if (shape == 1)
    launch_lagrangian_shape<T, Shape1>(runs, work, nwork, parity, partials, comp, true, nblocks, st);
  else
    launch_lagrangian_shape<T, Shape0>(runs, work, nwork, parity, partials, comp, true, nblocks, st);
}
#define GP_INSTANTIATE(T)                                                                                  \
  template void launch_lagrangian<T>(const RunDev<T>*, const WorkItem*, unsigned, int, double*, int, int,   \
                                     unsigned, hipStream_t);                                                \
  template void launch_init_partials<T>(const RunDev<T>*, const WorkItem*, unsigned, int, double*, int, int, \
                                        unsigned, hipStream_t);
GP_INSTANTIATE(double)
GP_INSTANTIATE(float)
#undef GP_INSTANTIATE

}  // namespace gp
