// Internal definitions shared by the GPUPEGAS HIP kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "gpupegas.h"

namespace gp {

constexpr int kNF = 22;    // state fields
constexpr int kNO = 20;    // fields other than rho and n (stored in the working precision)
constexpr int kDiagCap = 4096;

// Per-tile partial sums: one block of kNS slots per component (gas first,
// then stars / dark matter), each written by that component's Lagrangian
// kernel and combined by the fixed-order reductions.
enum : int {
  S_SPEED = 0,  // max signal speed (max, not sum)
  S_MASS, S_MOMX, S_MOMY, S_MOMZ, S_ENERGY, S_KAPPA, S_OUTFLOW, S_NSYNC,
  S_ERR,        // error bits (or, not sum)
  kNS
};
constexpr int kGasSlots = 0;
constexpr int kBmeSlots = kNS;
constexpr int kNP = 2 * kNS;  // slots per partial row
enum Component : int { COMP_GAS = 0, COMP_BME = 1 };

// Latched device error bits (also reported per diagnostics record).
enum : uint32_t {
  ERR_NONFINITE = 1u, ERR_DENSITY = 2u, ERR_PRESSURE = 4u, ERR_STRESS = 8u, ERR_NOSPEED = 16u
};

// Index of a field other than rho / n inside the "other" array.
__host__ __device__ constexpr int oidx(int field) { return field < GP_N ? field - 1 : field - 2; }

// State pointer table.  rho and n are always FP64 (exact telescoping of the
// mass flux in both precisions); the other 20 fields use the working type T.
template <typename T>
struct Fields {
  __attribute__((address_space(1))) double* rho;
  __attribute__((address_space(1))) double* nb;
  __attribute__((address_space(1))) T* o[kNO];  // mx my mz E e | qx qy qz | Pxx..Pzz | Wxx..Wzz
};

struct Grid {
  int nx, ny, nz;
  int bc[3];    // GP_BC_OUTFLOW / GP_BC_PERIODIC
  int phi_iso;  // 1: the potential has isolated boundaries and is stored with a one-cell ring
  double h;
  size_t ncell;
};

struct Phys {
  double gamma, G, cfl, eta, fixed_dt, t_end;
  double cool_lambda, cool_alpha, cool_theta_min;  // cooling q = lambda rho^2 theta^alpha (theta = p / rho)
  double gext[3];                                  // uniform external gravitational acceleration
};

// Scalars the step reads and writes on the device (no host round trip).
struct DevScalars {
  double t;              // time of the current state
  double dt;             // step the next update uses
  double outflow_gas;    // cumulative outflow
  double outflow_bme;
  int64_t step;
  uint32_t err;          // latched error bits
  uint32_t ndiag;        // diagnostics records written so far
};

// Symmetric-tensor slot of (i, j) in xx xy xz yy yz zz order.
__host__ __device__ constexpr int sym(int i, int j) {
  return (i == j) ? (i == 0 ? 0 : (i == 1 ? 3 : 5)) : ((i + j == 1) ? 1 : ((i + j == 2) ? 2 : 4));
}

// Hydrodynamic boundary rule: outflow clamps (zero gradient), periodic wraps.
__device__ __forceinline__ int bc_index(int i, int n, int bc) {
  if (bc == GP_BC_PERIODIC) return i < 0 ? i + n : (i >= n ? i - n : i);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}
__device__ __forceinline__ int wrap_index(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Per-cell kernels work on 64 x 4 tiles of an x-y plane (one thread per cell,
// a wave covers 64 consecutive x cells); a tile index runs x fastest, then y,
// then z.
constexpr int kTX = 64;
constexpr int kTY = 4;
constexpr int kBlock = kTX * kTY;

// Device descriptor of one run of a batch (a single simulation is a batch of
// one).  rho and n alternate between dens[0] and dens[1] each step; "cur"
// holds the state, "tmp" the post-Eulerian fields.
template <typename T>
struct RunDev {
  Grid g;
  Phys ph;
  double* dens[2][2];  // [parity][rho, n]
  T* cur[kNO];
  T* tmp[kNO];
  T* phi;
  DevScalars* sc;
  unsigned row0;       // first row of this run in the partial-sum table
  int ntx, nty;        // cell tiles along x and y
};

// One work item of a per-cell kernel: a 64 x 4 tile column (col = tx + ntx
// ty) of one run over planes [k0, k1), whose partial sums go to partial row
// row0 + row of that run.
struct WorkItem {
  int run, col, k0, k1, row;
  int pad[3];
};

// The item of list slot w, with every field in scalar registers.
__device__ __forceinline__ WorkItem load_item(const WorkItem* work, unsigned w) {
  WorkItem it;
  it.run = __builtin_amdgcn_readfirstlane(work[w].run);
  it.col = __builtin_amdgcn_readfirstlane(work[w].col);
  it.k0 = __builtin_amdgcn_readfirstlane(work[w].k0);
  it.k1 = __builtin_amdgcn_readfirstlane(work[w].k1);
  it.row = __builtin_amdgcn_readfirstlane(work[w].row);
  return it;
}

// The hardware hands consecutive workgroups to the 8 XCDs in turn, and each
// XCD has its own L2.  A persistent launch gives XCD x one contiguous range of
// work items (a block of tiles that share halos, in the order the host lists
// them); its workgroups stride through that range together, so tiles sharing
// halos run on the same XCD close in time.  Which workgroup takes a tile never
// changes a result.  A grid of fewer than kNumXcd workgroups leaves some XCDs
// without a workgroup, so it walks the whole list with a plain grid stride.
constexpr unsigned kNumXcd = 8;
struct WorkRange {
  unsigned first, end, stride;
};
__device__ __forceinline__ WorkRange xcd_range(unsigned nwork) {
  const unsigned G = gridDim.x, b = blockIdx.x;
  if (G < kNumXcd) return WorkRange{b, nwork, G};
  const unsigned x = b % kNumXcd, slot = b / kNumXcd;
  const unsigned nb_x = (G - x + kNumXcd - 1) / kNumXcd;  // workgroups on XCD x
  const unsigned q = nwork / kNumXcd, rem = nwork % kNumXcd;
  const unsigned start = x * q + min(x, rem);
  const unsigned count = q + (x < rem ? 1u : 0u);
  WorkRange r;
  r.first = start + slot;
  r.end = start + count;
  r.stride = nb_x;
  return r;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Pointers read from a descriptor in memory are generic to the compiler;
// typing them as global-address-space pointers lets it emit global (not flat)
// memory instructions for every access through them.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

// Reciprocal by Newton's iteration r <- r + r (1 - x r) from the hardware
// estimate: two steps in FP64 and one in FP32 reach the working precision to
// within an ulp or so, at about half the cost of an IEEE divide.  Used for
// the strictly positive densities, pressures and impedances of the stencils.
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  const float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}

// Addresses of a cell's 7-point stencil.  A tile lies in one z plane, so the
// planes it touches (k-1, k, k+1 under a boundary rule) are the same for the
// whole wave; each lane keeps 32-bit in-plane element offsets.  A load is a
// wave-uniform plane base (scalar registers) plus a 32-bit lane byte offset,
// i.e. one global load with a scalar base and no 64-bit address arithmetic in
// vector registers.  Point p: 0 centre, 1 / 2 minus / plus x, 3 / 4 minus /
// plus y, 5 / 6 minus / plus z.
struct Stencil {
  size_t z[3];     // element offsets of planes k-1, k, k+1
  uint32_t xy[5];  // in-plane offsets of the centre, x-1, x+1, y-1, y+1
};

// wrap = true applies the periodic rule on every axis (the potential),
// otherwise each axis follows its hydrodynamic boundary condition.
__device__ __forceinline__ Stencil make_stencil(const Grid& g, int i, int j, int k, bool wrap) {
  Stencil s;
  const size_t nxy = (size_t)g.nx * g.ny;
  const uint32_t nx = (uint32_t)g.nx;
  const int im = wrap ? wrap_index(i - 1, g.nx) : bc_index(i - 1, g.nx, g.bc[0]);
  const int ip = wrap ? wrap_index(i + 1, g.nx) : bc_index(i + 1, g.nx, g.bc[0]);
  const int jm = wrap ? wrap_index(j - 1, g.ny) : bc_index(j - 1, g.ny, g.bc[1]);
  const int jp = wrap ? wrap_index(j + 1, g.ny) : bc_index(j + 1, g.ny, g.bc[1]);
  const int km = wrap ? wrap_index(k - 1, g.nz) : bc_index(k - 1, g.nz, g.bc[2]);
  const int kp = wrap ? wrap_index(k + 1, g.nz) : bc_index(k + 1, g.nz, g.bc[2]);
  s.z[0] = nxy * (size_t)km;
  s.z[1] = nxy * (size_t)k;
  s.z[2] = nxy * (size_t)kp;
  s.xy[0] = (uint32_t)i + nx * (uint32_t)j;
  s.xy[1] = (uint32_t)im + nx * (uint32_t)j;
  s.xy[2] = (uint32_t)ip + nx * (uint32_t)j;
  s.xy[3] = (uint32_t)i + nx * (uint32_t)jm;
  s.xy[4] = (uint32_t)i + nx * (uint32_t)jp;
  return s;
}

// Element at plane offset z (uniform) and in-plane offset xy (per lane).
template <typename E>
__device__ __forceinline__ E ld_at(gptr<const E> base, size_t z, uint32_t xy) {
  const gptr<const char> plane = (gptr<const char>)(base + z);
  return *(gptr<const E>)(plane + xy * (uint32_t)sizeof(E));
}
// Streaming store: the stage's outputs are read again only by the next stage,
// so they should not displace the halo lines that neighbouring tiles still
// read from L2.
template <typename E>
__device__ __forceinline__ void st_at(gptr<E> base, size_t z, uint32_t xy, E v) {
  const gptr<char> plane = (gptr<char>)(base + z);
  __builtin_nontemporal_store(v, (gptr<E>)(plane + xy * (uint32_t)sizeof(E)));
}
// Stencil point P (compile-time) of an array.
template <int P, typename E>
__device__ __forceinline__ E ld_pt(gptr<const E> base, const Stencil& s) {
  if constexpr (P == 0) return ld_at(base, s.z[1], s.xy[0]);
  if constexpr (P >= 1 && P <= 4) return ld_at(base, s.z[1], s.xy[P]);
  if constexpr (P == 5) return ld_at(base, s.z[0], s.xy[0]);
  return ld_at(base, s.z[2], s.xy[0]);
}

// Tile coordinates of a cell work item: lane (threadIdx.x, threadIdx.y) of
// tile t covers cell (i, j) of plane k.
struct TileCell {
  int i, j, k;
  bool inside;
};
template <typename R>
__device__ __forceinline__ TileCell tile_cell(const R& run, int tile) {
  TileCell c;
  const int ntx = run.ntx, nty = run.nty;
  c.i = (tile % ntx) * kTX + (int)threadIdx.x;
  c.j = ((tile / ntx) % nty) * kTY + (int)threadIdx.y;
  c.k = tile / (ntx * nty);
  c.inside = c.i < run.g.nx && c.j < run.g.ny;
  return c;
}

template <typename T>
__device__ __forceinline__ Fields<T> fields_state(const RunDev<T>& R, int parity) {
  Fields<T> f;
  f.rho = as_global(R.dens[parity][0]);
  f.nb = as_global(R.dens[parity][1]);
#pragma unroll
  for (int o = 0; o < kNO; o++) f.o[o] = as_global(R.cur[o]);
  return f;
}
template <typename T>
__device__ __forceinline__ Fields<T> fields_eul(const RunDev<T>& R) {
  Fields<T> f;
  f.rho = nullptr;
  f.nb = nullptr;
#pragma unroll
  for (int o = 0; o < kNO; o++) f.o[o] = as_global(R.tmp[o]);
  return f;
}
template <typename T>
__device__ __forceinline__ Fields<T> fields_next(const RunDev<T>& R, int parity) {
  Fields<T> f;
  f.rho = as_global(R.dens[parity ^ 1][0]);
  f.nb = as_global(R.dens[parity ^ 1][1]);
#pragma unroll
  for (int o = 0; o < kNO; o++) f.o[o] = as_global(R.cur[o]);
  return f;
}

}  // namespace gp
