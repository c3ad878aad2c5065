// Internal definitions shared by the GPUPEGAS HIP kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "gpupegas.h"

namespace gp {

constexpr int kNF = 22;    // state fields
constexpr int kNO = 20;    // fields other than rho and n (stored in the working precision)
constexpr int kNP = 16;    // per-block partial-sum slots
constexpr int kDiagCap = 4096;

// Partial-sum slots written by the per-cell epilogues and read by the finalize.
enum : int {
  P_SPEED = 0,  // max signal speed (max, not sum)
  P_MGAS, P_MBME, P_MOMX, P_MOMY, P_MOMZ, P_EGAS, P_EBME,
  P_KGAS, P_KBME, P_OUTG, P_OUTB, P_SYNCG, P_SYNCB, P_ERR,
  P_PAD
};

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
  double* rho;
  double* nb;
  T* o[kNO];  // mx my mz E e | qx qy qz | Pxx Pxy Pxz Pyy Pyz Pzz | Wxx Wxy Wxz Wyy Wyz Wzz
};

struct Grid {
  int nx, ny, nz;
  int bc[3];  // GP_BC_OUTFLOW / GP_BC_PERIODIC
  double h;
  size_t ncell;
};

struct Phys {
  double gamma, G, cfl, eta, fixed_dt, t_end;
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

// Launch shape of the per-cell kernels: 64 x 4 threads cover a 64 x 4 tile
// of an x-y plane; blockIdx.z walks the z planes.
constexpr int kTX = 64;
constexpr int kTY = 4;

inline unsigned cell_blocks(const Grid& g) {
  return ((g.nx + kTX - 1) / kTX) * ((g.ny + kTY - 1) / kTY) * g.nz;
}

// The hardware hands consecutive workgroups of a 1D grid to the 8 XCDs in
// turn, and each XCD has its own L2.  Remap the dispatch index so that XCD x
// gets one contiguous range of tiles (a slab of z planes, swept in order):
// tiles that share y/z halos then run on the same XCD close in time.
constexpr int kNumXcd = 8;
struct TileId {
  int tx, ty, tz;   // tile coordinates, x fastest
  unsigned lin;     // linear tile index (row of the partial-sum table)
};
__device__ __forceinline__ TileId xcd_tile(int ntx, int nty) {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned q = nb / kNumXcd, rem = nb % kNumXcd;
  const unsigned x = b % kNumXcd, idx = b / kNumXcd;
  const unsigned v = x * q + min(x, rem) + idx;
  TileId t;
  t.lin = v;
  t.tx = v % ntx;
  t.ty = (v / ntx) % nty;
  t.tz = v / (ntx * nty);
  return t;
}

}  // namespace gp
