// Tile-column geometry shared by the Eulerian and Lagrangian kernels.
//
// A column work item is a TX x TY tile of cells (a TileShape) and a chunk of
// z planes; the workgroup walks the planes in order.  For plane k it keeps
// the tile of each field it needs, with a one-cell ring of x / y neighbours,
// in LDS (LY x LX values, the tile at rows / columns 1..TY / 1..TX); z
// neighbours are held in registers.  Each lane owns the cell of its
// (threadIdx.x, threadIdx.y); the first RING lanes of the workgroup also
// fetch one ring cell each.
#pragma once

#include "common.hpp"

namespace gp {

// Source cell of tile position x under a boundary rule: the rule itself on
// the one-cell ring outside the grid (x = -1 or x = n); positions further out
// (ragged edge tiles) are never read and take any valid cell.
__device__ __forceinline__ int ring_src(int x, int n, int bc) {
  if (x < 0 || x == n) return bc_index(x, n, bc);
  return x < n ? x : n - 1;
}

struct Column {
  int i0, j0, k0, k1;  // tile origin and plane range [k0, k1)
  int i, j;            // this lane's cell
  bool active;         // the cell is inside the grid
  uint32_t xy_c;       // in-plane offset the lane stages for its own slot
  bool ring;           // the lane also stages ring cell (hr, hc)
  int hr, hc;          // LDS row / column of that ring cell
  uint32_t xy_h;       // its in-plane offset
};

// Geometry of a work item for tile shape S.  periodic = true takes the
// periodic rule on x and y (the potential) instead of the hydrodynamic one.
template <class S>
__device__ __forceinline__ Column make_column(const Grid& g, const WorkItem& it, bool periodic) {
  Column c;
  c.i0 = it.i0;
  c.j0 = it.j0;
  c.k0 = it.k0;
  c.k1 = it.k1;
  c.i = c.i0 + (int)threadIdx.x;
  c.j = c.j0 + (int)threadIdx.y;
  c.active = c.i < g.nx && c.j < g.ny;
  const int bx = periodic ? GP_BC_PERIODIC : g.bc[0], by = periodic ? GP_BC_PERIODIC : g.bc[1];
  const uint32_t nx = (uint32_t)g.nx;
  c.xy_c = (uint32_t)ring_src(c.i, g.nx, bx) + nx * (uint32_t)ring_src(c.j, g.ny, by);
  // ring cells: rows -1 and TY (LX each), then columns -1 and TX
  const int tid = (int)threadIdx.x + S::TX * (int)threadIdx.y;
  c.ring = tid < S::RING;
  if (tid < S::LX) {
    c.hr = 0;
    c.hc = tid;
  } else if (tid < 2 * S::LX) {
    c.hr = S::LY - 1;
    c.hc = tid - S::LX;
  } else if (tid < 2 * S::LX + S::TY) {
    c.hr = 1 + tid - 2 * S::LX;
    c.hc = 0;
  } else {
    c.hr = 1 + min(tid - 2 * S::LX - S::TY, S::TY - 1);
    c.hc = S::LX - 1;
  }
  c.xy_h = (uint32_t)ring_src(c.i0 + c.hc - 1, g.nx, bx) + nx * (uint32_t)ring_src(c.j0 + c.hr - 1, g.ny, by);
  return c;
}

// The potential's geometry.  Periodic: nx ny nz values, wrapped on every
// axis.  Isolated: the grid and its one-cell ring, (nx+2)(ny+2)(nz+2) values
// with cell i at index i + 1 on each axis; tile positions beyond the ring
// (ragged edge tiles) are never read and take the ring's last cell.
template <class S>
__device__ __forceinline__ Column make_phi_column(const Grid& g, const WorkItem& it) {
  Column c = make_column<S>(g, it, true);
  if (g.phi_iso) {
    const uint32_t ex = (uint32_t)g.nx + 2;
    c.xy_c = (uint32_t)(min(c.i, g.nx) + 1) + ex * (uint32_t)(min(c.j, g.ny) + 1);
    c.xy_h = (uint32_t)(min(c.i0 + c.hc - 1, g.nx) + 1) + ex * (uint32_t)(min(c.j0 + c.hr - 1, g.ny) + 1);
  }
  return c;
}

// Re-issues a lane offset inside a plane loop.  Without it the compiler
// hoists "array base + lane offset" out of the loop as one 64-bit vector
// pointer per array and adds the plane offset to each of them every
// iteration; with the offset opaque, each access is a scalar plane base plus
// a 32-bit lane offset (one global load with a scalar base).
__device__ __forceinline__ uint32_t fresh(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// fences global memory, which makes every wave wait for all its outstanding
// global loads first, including loads fetched ahead for later planes.  In
// the column kernels threads share data through LDS alone (the global arrays
// a kernel writes are not read by it), so an LDS fence is enough.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Compiler-only ordering point for memory accesses (no instruction, no
// wait): loads written before it are issued before loads written after it.
// The column kernels issue a plane's ring loads first and the loads fetched
// ahead for later planes after them, so waiting for the ring does not wait
// for the fetch-ahead.
__device__ __forceinline__ void issue_order() { asm volatile("" ::: "memory"); }

// Element offset of plane k under the z boundary rule.
__device__ __forceinline__ size_t plane_at(const Grid& g, int k, int bc) {
  return (size_t)g.nx * (size_t)g.ny * (size_t)bc_index(k, g.nz, bc);
}

// Element offset of plane k (-1 .. nz) of the potential (see make_phi_column).
__device__ __forceinline__ size_t phi_plane(const Grid& g, int k) {
  if (g.phi_iso) return (size_t)(g.nx + 2) * (size_t)(g.ny + 2) * (size_t)(k + 1);
  return plane_at(g, k, GP_BC_PERIODIC);
}

}  // namespace gp
