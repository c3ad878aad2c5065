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

// Per-cell kernels work on TX x TY tiles of an x-y plane, one thread per
// cell (kBlock threads; a wave covers 64 / TX rows of TX consecutive x
// cells).  The shape is a template parameter of each per-cell kernel, picked
// per kernel by the engine's autotuner among kNumShapes candidates.
constexpr int kBlock = 256;
template <int TX_, int TY_>
struct TileShape {
  static constexpr int TX = TX_, TY = TY_;
  static constexpr int LX = TX + 2, LY = TY + 2;  // the tile with its one-cell ring
  static constexpr int RING = 2 * LX + 2 * TY;    // ring cells of a plane tile
  static_assert(TX * TY == kBlock && RING <= kBlock, "one thread per cell; one ring cell per thread at most");
};
constexpr int kNumShapes = 2;
constexpr int kShapeTX[kNumShapes] = {64, 32};
constexpr int kShapeTY[kNumShapes] = {4, 8};
using Shape0 = TileShape<64, 4>;
using Shape1 = TileShape<32, 8>;

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
};

// One work item of a per-cell kernel: the tile column with origin (i0, j0)
// of one run over planes [k0, k1), whose partial sums go to partial row
// row0 + row of that run.
struct WorkItem {
  int run, i0, j0, k0, k1, row;
  int pad[2];
};

// The item of list slot w, with every field in scalar registers.
__device__ __forceinline__ WorkItem load_item(const WorkItem* work, unsigned w) {
  WorkItem it;
  it.run = __builtin_amdgcn_readfirstlane(work[w].run);
  it.i0 = __builtin_amdgcn_readfirstlane(work[w].i0);
  it.j0 = __builtin_amdgcn_readfirstlane(work[w].j0);
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
// Reciprocal square root by Newton's iteration y <- y + (y / 2)(1 - x y^2)
// from the hardware estimate (two steps in FP64, one in FP32), for positive
// x: an impedance sqrt(x) and its reciprocal then cost one estimate, its
// refinement and a product x y instead of an IEEE square root and a
// reciprocal of it.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = __builtin_fma(-x * y, y, 1.0);
  y = __builtin_fma(0.5 * y, e, y);
  e = __builtin_fma(-x * y, y, 1.0);
  return __builtin_fma(0.5 * y, e, y);
}
__device__ __forceinline__ float rsqrt_nr(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  const float e = __builtin_fmaf(-x * y, y, 1.0f);
  return __builtin_fmaf(0.5f * y, e, y);
}
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
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

}  // namespace gp
