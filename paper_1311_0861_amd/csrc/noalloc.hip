// gp_potential_noalloc: the periodic potential of gp_get_potential (the FFT
// solve of the 27-point Poisson equation, Kulikov arXiv:1311.0861 Sec. 2.3)
// for densities the caller holds on the device, with no device allocation:
// the half spectrum, the twiddle and symbol tables, the source descriptor and
// the potential-energy partials live in one fixed file-scope device array.
// It runs the same Poisson kernels as a step; only its tables are formed on
// the device (a kernel, so that the whole call is kernel launches and can be
// captured in a HIP graph) instead of on the host.
//
// Each GPU holds its own copy of the array, whose address is looked up once
// per device with hipGetSymbolAddress; kernels receive that address, never
// the array's host-side name.  Every call on a GPU shares its array and
// leaves the last call's contents there; nothing in it must start at zero
// (every pass overwrites what a later pass reads).  Calls that overlap on one
// GPU (other streams or host threads) race on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

using namespace gp;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
gp_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GP_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return GP_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GP_OK;
}

bool len_ok(int n) {
  if (n < 4 || n > 1024 || n % 2 != 0) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

// Offsets (bytes, 256-aligned) of the workspace parts.
struct Layout {
  size_t spec, tw_x, wn_x, tw_y, tw_yh, tw_z, dx, dy, dz, slot, epot, total;
};
Layout layout(const FftGeom& f, size_t es) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~size_t(255);
    return at;
  };
  const size_t cs = 2 * es;
  L.spec = take((size_t)f.px * f.ny * f.nz * cs);
  L.tw_x = take((size_t)f.ax.L * cs);
  L.wn_x = take((size_t)(f.ax.L + 1) * cs);
  L.tw_y = take((size_t)f.ay.L * cs);
  L.tw_yh = take((size_t)f.ayh.L * cs);
  L.tw_z = take((size_t)f.az.L * cs);
  L.dx = take((size_t)f.px * sizeof(double));
  L.dy = take((size_t)f.ny * sizeof(double));
  L.dz = take((size_t)f.nz * sizeof(double));
  L.slot = take(sizeof(SrcSlot));
  L.epot = take((size_t)fft_blocks_z(f) * sizeof(double));
  L.total = off;
  return L;
}

template <typename T>
struct TableOut {
  cplx<T>* tw[5];  // x, x split, y, half y, z
  int n[5];        // entries
  int len[5];      // transform lengths (exp(-2 pi i k / len))
  double* d[3];    // D(k) = 1 - (2/3) sin^2(pi k / N) per axis
  int dn[3], dN[3];
};

// Twiddle and symbol tables and the source descriptor, formed on the device
// in FP64 (sincospi, then rounded to T).
template <typename T>
__global__ void k_noalloc_tables(TableOut<T> o, SrcSlot* slot, const double* rho, const double* nb) {
  const int tid = (int)(blockIdx.x * blockDim.x + threadIdx.x), nth = (int)(gridDim.x * blockDim.x);
  if (tid == 0) *slot = SrcSlot{{rho, rho}, {nb, nb}};
  for (int a = 0; a < 5; a++)
    for (int k = tid; k < o.n[a]; k += nth) {
      double s, c;
      sincospi(2.0 * (double)k / (double)o.len[a], &s, &c);
      o.tw[a][k] = cplx<T>{(T)c, (T)(-s)};
    }
  for (int a = 0; a < 3; a++)
    for (int k = tid; k < o.dn[a]; k += nth) {
      const double s = sinpi((double)k / (double)o.dN[a]);
      o.d[a][k] = 1.0 - 2.0 / 3.0 * s * s;
    }
}

template <typename T>
gp_status run(const FftGeom& f, const Layout& L, unsigned char* base, const double* rho, const double* nb, T* phi,
              hipStream_t st) {
  TableOut<T> o{};
  const int lens[5] = {f.ax.L, f.nx, f.ay.L, f.ayh.L, f.az.L};
  const int ns[5] = {f.ax.L, f.ax.L + 1, f.ay.L, f.ayh.L, f.az.L};
  const size_t offs[5] = {L.tw_x, L.wn_x, L.tw_y, L.tw_yh, L.tw_z};
  for (int a = 0; a < 5; a++) {
    o.tw[a] = reinterpret_cast<cplx<T>*>(base + offs[a]);
    o.n[a] = ns[a];
    o.len[a] = lens[a];
  }
  const size_t doffs[3] = {L.dx, L.dy, L.dz};
  const int dn[3] = {f.px, f.ny, f.nz}, dN[3] = {f.nx, f.ny, f.nz};
  for (int a = 0; a < 3; a++) {
    o.d[a] = reinterpret_cast<double*>(base + doffs[a]);
    o.dn[a] = dn[a];
    o.dN[a] = dN[a];
  }
  auto* slot = reinterpret_cast<SrcSlot*>(base + L.slot);
  k_noalloc_tables<T><<<8, 256, 0, st>>>(o, slot, rho, nb);

  FftTables<T> t{};
  t.tw_x = o.tw[0];
  t.wn_x = o.tw[1];
  t.tw_y = o.tw[2];
  t.tw_yh = o.tw[3];
  t.tw_z = o.tw[4];
  t.dx = o.d[0];
  t.dy = o.d[1];
  t.dz = o.d[2];
  auto* spec = reinterpret_cast<cplx<T>*>(base + L.spec);
  auto* epot = reinterpret_cast<double*>(base + L.epot);
  // the passes of a step's Poisson solve, with no reduction or finalize riding along
  if (f.plane) {
    launch_fft_xy_fwd<T>(slot, 0, spec, f, t, st);
  } else {
    launch_fft_x_fwd<T>(slot, 0, spec, f, t, st);
    launch_fft_y<T>(spec, f, t, false, st);
  }
  launch_fft_z_green<T>(spec, f, t, epot, f.plane != 0, RedJob{}, st);
  if (f.plane) {
    launch_fft_xy_inv<T>(spec, phi, f, t, FinJob{}, st);
  } else {
    launch_fft_y<T>(spec, f, t, true, st);
    launch_fft_x_inv<T>(spec, phi, f, t, FinJob{}, st);
  }
  return hipGetLastError() == hipSuccess ? GP_OK : GP_E_HIP;
}

}  // namespace

extern "C" gp_status gp_potential_noalloc(const gp_config* cfg, const double* rho, const double* nb, void* phi,
                                          void* hip_stream) {
  if (!cfg || !rho || !nb || !phi) return GP_E_INVALID;
  if (cfg->precision != GP_FP64 && cfg->precision != GP_FP32) return GP_E_INVALID;
  if (cfg->poisson != GP_POISSON_PERIODIC && cfg->poisson != GP_POISSON_ISOLATED) return GP_E_INVALID;
  if (cfg->G == 0.0) return GP_E_INVALID;
  for (int d = 0; d < 3; d++)
    if (!(cfg->hi[d] > cfg->lo[d]) || cfg->n[d] < 4) return GP_E_INVALID;
  const double h = (cfg->hi[0] - cfg->lo[0]) / cfg->n[0];
  for (int d = 1; d < 3; d++)
    if (std::fabs((cfg->hi[d] - cfg->lo[d]) / cfg->n[d] - h) > 1e-12 * h) return GP_E_INVALID;
  if (cfg->poisson != GP_POISSON_PERIODIC) return GP_E_UNSUPPORTED;
  for (int d = 0; d < 3; d++)
    if (!len_ok(cfg->n[d])) return GP_E_UNSUPPORTED;
  FftGeom f = make_fft_geom(cfg->n[0], cfg->n[1], cfg->n[2], 1, cfg->precision, true);
  f.green_scale = -4.0 * M_PI * cfg->G * h * h / 6.0;
  const size_t es = cfg->precision == GP_FP64 ? sizeof(double) : sizeof(float);
  const Layout L = layout(f, es);
  if (L.total > kNoAllocScratchBytes) return GP_E_UNSUPPORTED;  // beyond the fixed workspace
  void* base = nullptr;
  const gp_status s = scratch_address(&base);
  if (s != GP_OK) return s;
  auto* b = static_cast<unsigned char*>(base);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (cfg->precision == GP_FP64) return run<double>(f, L, b, rho, nb, static_cast<double*>(phi), st);
  return run<float>(f, L, b, rho, nb, static_cast<float*>(phi), st);
}
