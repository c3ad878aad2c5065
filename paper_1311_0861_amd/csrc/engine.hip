// Host engine and C ABI of the GPUPEGAS timestep library.
//
// The engine advances a batch of independent runs in lockstep; a single
// simulation (gp_sim) is a batch of one (gp_batch), so both go through the
// same kernels and a batch member is bitwise equal to the same run alone.
//
// Device state per run: rho and n in FP64 (two buffers that swap each step),
// the 20 other fields in the working precision in two sets ("cur" holds the
// state, "tmp" the post-Eulerian fields), corner velocities, device scalars
// (t, tau, step, error bits, cumulative outflow) and a ring of diagnostics
// records.  Runs of one grid size form a size class whose potential and half
// spectrum are stored back to back, so each FFT pass is one launch per class.
// Per-cell stages are persistent launches over a (run, tile) work list.  One
// step is
//   Eulerian (gas, stars) -> Lagrangian (gas, stars; corners, fluxes and
//   per-tile partial sums) -> 3 FFT passes per class (5 where a plane does
//   not fit in LDS; the first z pass also reduces the partial rows)
//   -> finalize (one workgroup per run)
// and is replayed from a captured HIP graph (one per buffer parity); tau never
// leaves the device.  The persistent grid size of each per-cell stage is
// picked by timing candidates during the first step (results do not depend
// on it).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

using namespace gp;

namespace {

// Target work items per run of the two work lists (see make_items), by
// working precision: {stars / DM kernels, gas kernels}: as many items as the
// chip keeps workgroups of those kernels resident in FP64 (2 per CU for the
// stars / DM, 3 for the gas: 768 items took the gas Lagrangian from 0.081 to
// 0.076 ms at 128^3).  A list that overshoots the resident slots is slower
// (832 gas items: 0.065 -> 0.073 ms Eulerian, 0.087 -> 0.101 ms Lagrangian).
constexpr long kItemsFp64[2] = {512, 768};
constexpr long kItemsFp32[2] = {512, 512};
constexpr int kTunedKernels = 4;  // the per-cell kernels
// z-chunk caps the autotuner tries (the "halo" shape of a work item): an item
// of cz planes also reads the plane below and above it, 2 / cz of re-reads;
// shorter chunks give more items to spread over the chip.
constexpr int kNumCaps = 4;
constexpr int kCaps[kNumCaps] = {8, 16, 32, 64};
constexpr int kDefaultCap = 2;  // 32 planes
// Per-kernel launch configuration: tile shape (TileShape index), z-chunk cap
// (index into kCaps) and persistent grid size.
struct TileCfg {
  int shape = 0;
  int cap = kDefaultCap;
  unsigned blocks = 0;
};
// Largest grid axis with isolated Poisson boundaries: a padded line of 2n
// complex values (and an x row of n packed pairs with its bins) stays within
// 64 KiB of LDS in FP64.
constexpr int kIsoMaxN = 512;
const int kTunedIds[kTunedKernels] = {GP_K_EUL_GAS, GP_K_EUL_BME, GP_K_LAG_GAS, GP_K_LAG_BME};

struct RunHost {
  gp_config cfg{};
  Grid g{};
  Phys ph{};
  double* dens[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  void* cur[kNO] = {};
  void* tmp[kNO] = {};
  void* phi = nullptr;
  DevScalars* sc = nullptr;
  gp_diag* ring = nullptr;
  unsigned row0 = 0, nrows = 0;
  int cls = 0, slot = 0;  // size class and position inside it
};

struct SizeClass {
  int nx = 0, ny = 0, nz = 0;
  double h = 0.0, G = 0.0;
  std::vector<int> runs;
  SrcSlot* src = nullptr;  // per run slot: the densities, for the source
  void* phi = nullptr;
  void* spec = nullptr;
  void* tw_x = nullptr;
  void* wn_x = nullptr;
  void* tw_y = nullptr;
  void* tw_yh = nullptr;
  void* tw_z = nullptr;
  double* dtab[3] = {nullptr, nullptr, nullptr};
  FftGeom fg{};
  // isolated boundaries: padded geometry and the Green spectrum (FP64)
  int iso = 0;
  IsoGeom ig{};
  double* green = nullptr;
  unsigned eoff = 0;  // first potential-energy partial of the class
  unsigned nep_run = 0;
};

// HIP events around each kernel (or pass) of a step, launched once, in the
// order of a step, so that each finds its inputs where a step leaves them
// (launched several times back to back, the later launches read inputs the
// earlier ones left in the last-level cache and read faster than in a step).
struct Timer {
  hipEvent_t ev[2 * GP_NKERNELS];
  double acc[GP_NKERNELS];
  bool on = false;
};

}  // namespace

struct gp_batch {
  int prec = GP_FP64;
  hipStream_t st = nullptr;
  bool own_stream = false;
  std::vector<RunHost> runs;
  std::vector<SizeClass> classes;
  std::vector<std::pair<void*, size_t>> allocs;

  void* runs_dev = nullptr;  // RunDev<T>[nruns]
  // work lists [component list][tile shape][z-chunk cap]: list 0 for the
  // stars / DM kernels, 1 for the gas kernels (their own item targets)
  WorkItem* work[2][kNumShapes][kNumCaps] = {};
  unsigned nwork[2][kNumShapes][kNumCaps] = {};
  double* partials = nullptr;
  RedItem* red_items = nullptr;
  int nred = 0;
  double* scratch = nullptr;
  FinDesc* fin = nullptr;
  double* epot = nullptr;
  unsigned nepot = 0;
  void* staging = nullptr;

  int parity = 0;
  bool need_prologue = true;
  int next_stage = GP_STAGE_EUL;
  bool use_graph = true;
  bool graph_ready[2] = {false, false};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  TileCfg kcfg[GP_NKERNELS];  // the per-cell kernels' configurations
  bool tuned = false;
  bool tune = true;
  std::string cache_path;  // GPUPEGAS_TUNE_CACHE at create time (empty: none)
  int fft_form = GP_FFT_AUTO;
  bool cooling = false;  // some run has a cooling source
  std::string last_error;
};

// A single simulation is a batch of one run.
struct gp_sim : gp_batch {};

namespace {

gp_status hip_fail(gp_batch* b, hipError_t e, const char* what) {
  if (b) b->last_error = std::string(what) + ": " + hipGetErrorString(e);
  return GP_E_HIP;
}

#define HIP_TRY(b, expr)                                     \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return hip_fail((b), e_, #expr);   \
  } while (0)

bool fft_len_ok(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

size_t esize(int prec) { return prec == GP_FP64 ? sizeof(double) : sizeof(float); }

void* dalloc(gp_batch* b, size_t bytes, gp_status* st) {
  void* p = nullptr;
  if (*st != GP_OK) return nullptr;
  bytes = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
  if (hipMalloc(&p, bytes) != hipSuccess) {
    *st = GP_E_NOMEM;
    b->last_error = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
    return nullptr;
  }
  b->allocs.push_back({p, bytes});
  return p;
}

gp_status validate(const gp_config* cfg) {
  for (int d = 0; d < 3; d++) {
    if (cfg->n[d] < 4 || cfg->n[d] > 1024 || !(cfg->hi[d] > cfg->lo[d])) return GP_E_INVALID;
    if (cfg->bc[d] != GP_BC_OUTFLOW && cfg->bc[d] != GP_BC_PERIODIC) return GP_E_INVALID;
  }
  const double h = (cfg->hi[0] - cfg->lo[0]) / cfg->n[0];
  for (int d = 1; d < 3; d++)
    if (std::fabs((cfg->hi[d] - cfg->lo[d]) / cfg->n[d] - h) > 1e-12 * h) return GP_E_INVALID;
  if (!(cfg->gamma > 1.0) || !(cfg->cfl > 0.0)) return GP_E_INVALID;
  if (cfg->poisson != GP_POISSON_PERIODIC && cfg->poisson != GP_POISSON_ISOLATED) return GP_E_INVALID;
  if (!(cfg->cool_lambda >= 0.0) || !std::isfinite(cfg->cool_lambda) || !std::isfinite(cfg->cool_alpha) ||
      !(cfg->cool_theta_min >= 0.0) || !std::isfinite(cfg->cool_theta_min))
    return GP_E_INVALID;
  for (int d = 0; d < 3; d++)
    if (!std::isfinite(cfg->gext[d])) return GP_E_INVALID;
  if (cfg->precision != GP_FP64 && cfg->precision != GP_FP32) return GP_E_INVALID;
  if (cfg->G != 0.0)
    for (int d = 0; d < 3; d++) {
      if (!fft_len_ok(cfg->n[d]) || cfg->n[d] % 2 != 0) return GP_E_UNSUPPORTED;
      // the padded solve keeps a padded line of 2n values in LDS
      if (cfg->poisson == GP_POISSON_ISOLATED && cfg->n[d] > kIsoMaxN) return GP_E_UNSUPPORTED;
    }
  return GP_OK;
}

template <typename T>
FftTables<T> tables(const SizeClass& c) {
  FftTables<T> t{};
  t.tw_x = static_cast<const cplx<T>*>(c.tw_x);
  t.wn_x = static_cast<const cplx<T>*>(c.wn_x);
  t.tw_y = static_cast<const cplx<T>*>(c.tw_y);
  t.tw_yh = static_cast<const cplx<T>*>(c.tw_yh);
  t.tw_z = static_cast<const cplx<T>*>(c.tw_z);
  t.dx = c.dtab[0];
  t.dy = c.dtab[1];
  t.dz = c.dtab[2];
  return t;
}

template <typename T>
IsoTables<T> iso_tables(const SizeClass& c) {
  IsoTables<T> t{};
  t.tw_x = static_cast<const cplx<T>*>(c.tw_x);
  t.wn_x = static_cast<const cplx<T>*>(c.wn_x);
  t.tw_y = static_cast<const cplx<T>*>(c.tw_y);
  t.tw_z = static_cast<const cplx<T>*>(c.tw_z);
  t.green = c.green;
  return t;
}

// Padded geometry of a size class with isolated boundaries, for complex
// values of 2 * es bytes: line passes of at most 32 KiB of LDS data, as the
// periodic line passes.
IsoGeom make_iso_geom(int nx, int ny, int nz, int nruns, size_t es) {
  IsoGeom f{};
  f.nx = nx;
  f.ny = ny;
  f.nz = nz;
  f.px = nx + 1;
  f.py = 2 * ny;
  f.pz = 2 * nz;
  f.nruns = nruns;
  f.ax = make_axis(nx);
  f.ay = make_axis(2 * ny);
  f.az = make_axis(2 * nz);
  const int maxpts = 32768 / (int)(2 * es);
  f.rows_per_block = std::max(1, maxpts / (2 * nx));
  auto even_cols = [&](int L) {
    const int cmax = std::max(1, std::min({8, f.px, maxpts / L}));
    const int nch = (f.px + cmax - 1) / cmax;
    return (f.px + nch - 1) / nch;
  };
  f.cols_y = even_cols(f.ay.L);
  f.cols_z = even_cols(f.az.L);
  f.run_stride = (size_t)(nz + 2) * f.py * f.px;
  f.ext_cells = (size_t)(nx + 2) * (ny + 2) * (nz + 2);
  f.norm = 2.0 / (8.0 * (double)nx * (double)ny * (double)nz);
  return f;
}

void tmark(gp_batch* b, Timer* tm, int k, int side) {
  if (tm && tm->on) (void)hipEventRecord(tm->ev[2 * k + side], b->st);
}
void tdone(Timer* tm, int k) {
  if (tm && tm->on) {
    (void)hipEventSynchronize(tm->ev[2 * k + 1]);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, tm->ev[2 * k], tm->ev[2 * k + 1]);
    tm->acc[k] += ms;
  }
}

RedJob red_job(const gp_batch* b) { return RedJob{b->partials, b->red_items, b->scratch, b->nred}; }

bool any_gravity(const gp_batch* b) {
  for (const SizeClass& c : b->classes)
    if (c.G != 0.0) return true;
  return false;
}

FinJob fin_job(const gp_batch* b, int advanced) {
  return FinJob{b->scratch, b->epot, b->fin, (int)b->runs.size(), advanced};
}

// The Poisson passes.  The first z pass also runs the first level of the
// reduction of the partial rows; with fin >= 0 the first inverse pass also
// finishes the step (finalize with advanced = fin), which needs only what the
// z passes left.
template <typename T>
void enqueue_poisson(gp_batch* b, Timer* tm, int fin) {
  // each pass runs over every size class before the next pass starts
  const int passes[3] = {GP_K_FFT_XY_FWD, GP_K_FFT_Z, GP_K_FFT_XY_INV};
  bool reduced = false, finished = fin < 0;
  for (int k : passes) {
    tmark(b, tm, k, 0);
    for (SizeClass& c : b->classes) {
      if (c.G == 0.0) continue;
      auto* spec = static_cast<cplx<T>*>(c.spec);
      T* phi = static_cast<T*>(c.phi);
      if (c.iso) {
        const IsoTables<T> t = iso_tables<T>(c);
        switch (k) {
          case GP_K_FFT_XY_FWD:
            launch_iso_fwd<T>(c.src, b->parity, spec, c.ig, t, b->st);
            break;
          case GP_K_FFT_Z:
            launch_iso_z<T>(spec, c.ig, t, b->epot + c.eoff, reduced ? RedJob{} : red_job(b), b->st);
            reduced = true;
            break;
          case GP_K_FFT_XY_INV:
            launch_iso_inv<T>(spec, phi, c.ig, t, finished ? FinJob{} : fin_job(b, fin), b->st);
            finished = true;
            break;
        }
        continue;
      }
      const FftTables<T> t = tables<T>(c);
      const bool plane = c.fg.plane && b->fft_form == GP_FFT_AUTO;
      switch (k) {
        case GP_K_FFT_XY_FWD:
          if (plane) {
            launch_fft_xy_fwd<T>(c.src, b->parity, spec, c.fg, t, b->st);
          } else {
            launch_fft_x_fwd<T>(c.src, b->parity, spec, c.fg, t, b->st);
            launch_fft_y<T>(spec, c.fg, t, false, b->st);
          }
          break;
        case GP_K_FFT_Z:
          launch_fft_z_green<T>(spec, c.fg, t, b->epot + c.eoff, plane, reduced ? RedJob{} : red_job(b), b->st);
          reduced = true;
          break;
        case GP_K_FFT_XY_INV: {
          const FinJob fj = finished ? FinJob{} : fin_job(b, fin);
          if (plane) {
            launch_fft_xy_inv<T>(spec, phi, c.fg, t, fj, b->st);
          } else {
            launch_fft_y<T>(spec, c.fg, t, true, b->st);
            launch_fft_x_inv<T>(spec, phi, c.fg, t, fj, b->st);
          }
          finished = true;
          break;
        }
      }
    }
    tmark(b, tm, k, 1);
    tdone(tm, k);
  }
}

// partial rows -> per-run scratch rows (done by the z pass when a run has
// gravity), then the per-run finalize, as kernels of their own
void enqueue_finalize(gp_batch* b, int advanced, Timer* tm) {
  tmark(b, tm, GP_K_FINALIZE, 0);
  if (!any_gravity(b)) launch_reduce(red_job(b), b->st);
  launch_finalize(fin_job(b, advanced), b->st);
  tmark(b, tm, GP_K_FINALIZE, 1);
  tdone(tm, GP_K_FINALIZE);
}

// Work lists.  For tile shape s a run has ntx x nty tile columns; each is
// cut into about target / ncolumns chunks (rounded) of cz planes, cz clamped
// to 4..cap, so the list has about `target` items; list 0 (stars / DM
// kernels) and list 1 (gas kernels) have their own target.  A workgroup walks
// its chunk plane by plane, so short chunks re-read more planes at their
// ends, long ones leave resident workgroup slots idle.  Items go x fastest,
// then y, then chunk: the columns whose rings overlap run side by side on one
// XCD.  Item i of a run writes partial row i.
int tiles_x(const RunHost& R, int s) { return (R.g.nx + kShapeTX[s] - 1) / kShapeTX[s]; }
int tiles_y(const RunHost& R, int s) { return (R.g.ny + kShapeTY[s] - 1) / kShapeTY[s]; }
int chunk_planes(const RunHost& R, int prec, int list, int s, int cap) {
  const long target = (prec == GP_FP64 ? kItemsFp64 : kItemsFp32)[list];
  const long ncol = (long)tiles_x(R, s) * tiles_y(R, s);
  const long nchunk = std::max(1L, (target + ncol / 2) / ncol);  // chunks per column, rounded
  const long cz = (R.g.nz + nchunk - 1) / nchunk;
  return (int)std::max<long>(4, std::min<long>(kCaps[cap], cz));
}
unsigned items_per_run(const RunHost& R, int prec, int list, int s, int cap) {
  const int cz = chunk_planes(R, prec, list, s, cap);
  return (unsigned)(tiles_x(R, s) * tiles_y(R, s) * ((R.g.nz + cz - 1) / cz));
}
void make_items(const RunHost& R, int run, int prec, int list, int s, int cap, std::vector<WorkItem>& out) {
  const int cz = chunk_planes(R, prec, list, s, cap);
  const int ntx = tiles_x(R, s), nty = tiles_y(R, s);
  int row = 0;
  for (int k0 = 0; k0 < R.g.nz; k0 += cz)
    for (int ty = 0; ty < nty; ty++)
      for (int tx = 0; tx < ntx; tx++) {
        WorkItem it{};
        it.run = run;
        it.i0 = tx * kShapeTX[s];
        it.j0 = ty * kShapeTY[s];
        it.k0 = k0;
        it.k1 = std::min(k0 + cz, R.g.nz);
        it.row = row++;
        out.push_back(it);
      }
}

int list_of(int k) { return (k == GP_K_EUL_GAS || k == GP_K_LAG_GAS) ? 1 : 0; }

unsigned work_count(const gp_batch* b, int k, const TileCfg& c) { return b->nwork[list_of(k)][c.shape][c.cap]; }

template <typename T>
void launch_cell_kernel(gp_batch* b, int k, const TileCfg& c) {
  const auto* runs = static_cast<const RunDev<T>*>(b->runs_dev);
  const int l = list_of(k);
  const WorkItem* w = b->work[l][c.shape][c.cap];
  const unsigned nw = b->nwork[l][c.shape][c.cap];
  switch (k) {
    case GP_K_EUL_GAS:
      launch_eulerian<T>(runs, w, nw, b->parity, COMP_GAS, b->cooling, c.shape, c.blocks, b->st);
      break;
    case GP_K_EUL_BME:
      launch_eulerian<T>(runs, w, nw, b->parity, COMP_BME, false, c.shape, c.blocks, b->st);
      break;
    case GP_K_LAG_GAS:
      launch_lagrangian<T>(runs, w, nw, b->parity, b->partials, COMP_GAS, c.shape, c.blocks, b->st);
      break;
    case GP_K_LAG_BME:
      launch_lagrangian<T>(runs, w, nw, b->parity, b->partials, COMP_BME, c.shape, c.blocks, b->st);
      break;
  }
}

// The autotuner.  Kernel k is timed (one warm launch, then the median of
// kTuneReps launches, each between HIP events) in its default configuration (64 x 4 tiles, 32-plane chunk cap, a
// workgroup per item), then for every other tile shape and chunk cap at a
// workgroup per item, then for the fastest of those at the persistent grid
// sizes 8192, 4096, 2048 and 1024 below that.  A candidate replaces the best
// so far only when it is more than kTuneMargin faster: the candidates of a
// grid differ by a few percent, about the spread of such short timings, and
// the margin keeps noise from moving the pick off the default.  Every
// per-cell stage is idempotent with respect to its inputs (none of them
// writes what it reads), so re-running it during the first step changes
// nothing but the timing -- except the partial rows of the Lagrangian
// kernels, which the caller clears after tuning them (a candidate list can be
// longer than the chosen one).
constexpr float kTuneMargin = 0.03f;
constexpr int kTuneReps = 7;

template <typename T>
void tune_kernel(gp_batch* b, int k) {
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // Each timed launch follows a launch of the other component's kernel of
  // the same stage (it recomputes its own outputs from unchanged inputs), so
  // that the candidate finds its inputs as far out of the caches as in a
  // step, where other kernels run in between; timed back to back, a
  // candidate would read inputs its previous launch left in the last-level
  // cache, and the picks would favour shapes that lose in the step.
  const int other = k == GP_K_EUL_GAS ? GP_K_EUL_BME
                  : k == GP_K_EUL_BME ? GP_K_EUL_GAS
                  : k == GP_K_LAG_GAS ? GP_K_LAG_BME : GP_K_LAG_GAS;
  // The median of kTuneReps such launches is the candidate's time.
  auto time = [&](const TileCfg& c) {
    launch_cell_kernel<T>(b, k, c);  // warm
    float t[kTuneReps];
    for (int rep = 0; rep < kTuneReps; rep++) {
      launch_cell_kernel<T>(b, other, b->kcfg[other]);
      (void)hipEventRecord(e0, b->st);
      launch_cell_kernel<T>(b, k, c);
      (void)hipEventRecord(e1, b->st);
      (void)hipEventSynchronize(e1);
      t[rep] = 0.f;
      (void)hipEventElapsedTime(&t[rep], e0, e1);
    }
    std::sort(t, t + kTuneReps);
    return t[kTuneReps / 2];
  };
  TileCfg pick{};
  pick.blocks = work_count(b, k, pick);
  float best = time(pick);
  auto consider = [&](const TileCfg& c) {
    const float ms = time(c);
    if (ms < best * (1.0f - kTuneMargin)) {
      best = ms;
      pick = c;
    }
  };
  for (int s = 0; s < kNumShapes; s++)
    for (int cap = 0; cap < kNumCaps; cap++) {
      TileCfg c{s, cap, 0};
      if (s == 0 && cap == kDefaultCap) continue;  // timed first
      c.blocks = work_count(b, k, c);
      consider(c);
    }
  const unsigned nw = work_count(b, k, pick);
  for (unsigned blocks : {8192u, 4096u, 2048u, 1024u}) {
    if (blocks >= nw) continue;
    TileCfg c = pick;
    c.blocks = blocks;
    consider(c);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->kcfg[k] = pick;
}

// ---- tuning cache --------------------------------------------------------
// With GPUPEGAS_TUNE_CACHE naming a file, the picked configurations are
// stored there, one JSON member per kernel: "key": [shape, cap planes,
// workgroups], the key naming the device architecture, the precision,
// whether the gas cools, the multiset of grid sizes of the batch and the
// kernel.  A batch whose four keys are all present takes them instead of
// tuning.
const char* kKernelKeys[GP_NKERNELS] = {"eul_gas", "eul_bme", "lag_gas", "lag_bme", "", "", "", ""};
std::mutex g_cache_mu;

std::string tune_key(const gp_batch* b, int k) {
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "gpu";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  std::map<std::string, int> sizes;
  for (const RunHost& R : b->runs)
    sizes[std::to_string(R.g.nx) + "x" + std::to_string(R.g.ny) + "x" + std::to_string(R.g.nz)]++;
  std::string key = arch + "|" + (b->prec == GP_FP64 ? "fp64" : "fp32") + (b->cooling ? "|cool" : "") + "|";
  bool first = true;
  for (const auto& kv : sizes) {
    key += (first ? "" : "+") + kv.first + "*" + std::to_string(kv.second);
    first = false;
  }
  return key + "|" + kKernelKeys[k];
}

// "key": [a, b, c] members of the cache file
std::map<std::string, std::vector<long>> read_cache(const std::string& path) {
  std::map<std::string, std::vector<long>> out;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1);
    const size_t b0 = line.find('[', q1), b1 = line.find(']', b0);
    if (q0 == std::string::npos || q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos)
      continue;
    std::string vals = line.substr(b0 + 1, b1 - b0 - 1);
    for (char& ch : vals)
      if (ch == ',') ch = ' ';
    std::istringstream vs(vals);
    std::vector<long> v;
    long x;
    while (vs >> x) v.push_back(x);
    if (v.size() == 3) out[line.substr(q0 + 1, q1 - q0 - 1)] = v;
  }
  return out;
}

void write_cache(const gp_batch* b) {
  if (b->cache_path.empty()) return;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto entries = read_cache(b->cache_path);
  for (int k : kTunedIds) {
    const TileCfg& c = b->kcfg[k];
    entries[tune_key(b, k)] = {c.shape, kCaps[c.cap], (long)c.blocks};
  }
  const std::string tmp = b->cache_path + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    out << "{\n";
    size_t i = 0;
    for (const auto& kv : entries) {
      out << "  \"" << kv.first << "\": [" << kv.second[0] << ", " << kv.second[1] << ", " << kv.second[2] << "]"
          << (++i < entries.size() ? "," : "") << "\n";
    }
    out << "}\n";
    if (!out) return;
  }
  (void)std::rename(tmp.c_str(), b->cache_path.c_str());
}

// Takes the four kernels' configurations from the cache file when all are
// there and valid for this batch.
bool load_cache(gp_batch* b) {
  if (b->cache_path.empty()) return false;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  const auto entries = read_cache(b->cache_path);
  TileCfg got[GP_NKERNELS];
  for (int k : kTunedIds) {
    const auto it = entries.find(tune_key(b, k));
    if (it == entries.end()) return false;
    const std::vector<long>& v = it->second;
    int cap = -1;
    for (int q = 0; q < kNumCaps; q++)
      if (kCaps[q] == v[1]) cap = q;
    if (v[0] < 0 || v[0] >= kNumShapes || cap < 0 || v[2] < 1) return false;
    got[k] = TileCfg{(int)v[0], cap, 0};
    got[k].blocks = std::min<unsigned>((unsigned)v[2], work_count(b, k, got[k]));
  }
  for (int k : kTunedIds) b->kcfg[k] = got[k];
  return true;
}

// Clears the partial rows: a list shorter than the one that last wrote them
// would leave stale rows behind (never inside a captured graph).
void clear_partials(gp_batch* b) {
  size_t rows = 0;
  for (const RunHost& R : b->runs) rows += R.nrows;
  (void)hipMemsetAsync(b->partials, 0, rows * kNP * sizeof(double), b->st);
}

template <typename T>
void enqueue_stage(gp_batch* b, int stage, Timer* tm, bool allow_tune) {
  const bool tuning = allow_tune && b->tune && !b->tuned;
  auto cell = [&](int k) {
    tmark(b, tm, k, 0);
    launch_cell_kernel<T>(b, k, b->kcfg[k]);
    tmark(b, tm, k, 1);
    tdone(tm, k);
  };
  switch (stage) {
    case GP_STAGE_EUL:
      if (tuning) {
        tune_kernel<T>(b, GP_K_EUL_GAS);
        tune_kernel<T>(b, GP_K_EUL_BME);
      }
      cell(GP_K_EUL_GAS);
      cell(GP_K_EUL_BME);
      break;
    case GP_STAGE_LAG:
      if (tuning) {
        tune_kernel<T>(b, GP_K_LAG_GAS);
        tune_kernel<T>(b, GP_K_LAG_BME);
        clear_partials(b);
      }
      cell(GP_K_LAG_GAS);
      cell(GP_K_LAG_BME);
      if (tuning) {
        b->tuned = true;
        write_cache(b);
      }
      b->parity ^= 1;
      break;
    case GP_STAGE_POISSON:
      enqueue_poisson<T>(b, tm, -1);
      break;
    case GP_STAGE_FINALIZE:
      enqueue_finalize(b, 1, tm);
      break;
  }
}

// The Poisson solve and the finalize of a step (advanced = 1) or of the
// initial state (0): the finalize rides along in the Poisson passes where
// there are any.  Same arithmetic as the two stages run one by one.
template <typename T>
void enqueue_end(gp_batch* b, Timer* tm, int advanced) {
  if (any_gravity(b))
    enqueue_poisson<T>(b, tm, advanced);
  else
    enqueue_finalize(b, advanced, tm);
}

template <typename T>
void enqueue_prologue(gp_batch* b) {
  const auto* runs = static_cast<const RunDev<T>*>(b->runs_dev);
  // the rows of the Lagrangian kernels' lists, in their tile shapes
  for (int k : {GP_K_LAG_GAS, GP_K_LAG_BME}) {
    const TileCfg& c = b->kcfg[k];
    const int l = list_of(k);
    launch_init_partials<T>(runs, b->work[l][c.shape][c.cap], b->nwork[l][c.shape][c.cap], b->parity, b->partials,
                            k == GP_K_LAG_GAS ? COMP_GAS : COMP_BME, c.shape, c.blocks, b->st);
  }
  enqueue_end<T>(b, nullptr, 0);
}

void run_prologue(gp_batch* b) {
  if (b->prec == GP_FP64)
    enqueue_prologue<double>(b);
  else
    enqueue_prologue<float>(b);
  b->need_prologue = false;
  b->next_stage = GP_STAGE_EUL;
}

void run_stage(gp_batch* b, int stage, Timer* tm, bool allow_tune) {
  if (b->prec == GP_FP64)
    enqueue_stage<double>(b, stage, tm, allow_tune);
  else
    enqueue_stage<float>(b, stage, tm, allow_tune);
}

void run_step_direct(gp_batch* b, Timer* tm, bool allow_tune) {
  run_stage(b, GP_STAGE_EUL, tm, allow_tune);
  run_stage(b, GP_STAGE_LAG, tm, allow_tune);
  if (b->prec == GP_FP64)
    enqueue_end<double>(b, tm, 1);
  else
    enqueue_end<float>(b, tm, 1);
}

gp_status build_graph(gp_batch* b, int parity) {
  HIP_TRY(b, hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
  const int saved = b->parity;
  b->parity = parity;
  hipGraph_t graph = nullptr;
  run_step_direct(b, nullptr, false);
  hipError_t e = hipStreamEndCapture(b->st, &graph);
  b->parity = saved;
  if (e != hipSuccess) return hip_fail(b, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->gexec[parity], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(b, e, "hipGraphInstantiate");
  b->graph_ready[parity] = true;
  return GP_OK;
}

void drop_graphs(gp_batch* b) {
  for (int p = 0; p < 2; p++) {
    if (b->gexec[p]) (void)hipGraphExecDestroy(b->gexec[p]);
    b->gexec[p] = nullptr;
    b->graph_ready[p] = false;
  }
}

// Latched device error of run `only` (or of any run, only < 0) as a status.
gp_status latched(gp_batch* b, int only = -1) {
  uint32_t err = 0;
  for (int r = 0; r < (int)b->runs.size(); r++) {
    if (only >= 0 && r != only) continue;
    DevScalars h{};
    HIP_TRY(b, hipMemcpy(&h, b->runs[r].sc, sizeof(h), hipMemcpyDeviceToHost));
    err |= h.err;
  }
  if (err & ERR_NONFINITE) {
    b->last_error = "non-finite value in the state";
    return GP_E_NONFINITE;
  }
  if (err & (ERR_DENSITY | ERR_PRESSURE | ERR_STRESS | ERR_NOSPEED)) {
    b->last_error = "non-positive density, pressure or diagonal stress (bits " + std::to_string(err) + ")";
    return GP_E_NONPOSITIVE;
  }
  return GP_OK;
}

// device pointer of field `id` of run r in the state visible to get/set
void* field_ptr(gp_batch* b, int r, int id, bool* is_double) {
  RunHost& R = b->runs[r];
  if (id == GP_RHO || id == GP_N) {
    *is_double = true;
    return R.dens[b->parity][id == GP_RHO ? 0 : 1];
  }
  *is_double = b->prec == GP_FP64;
  if (id == GP_PHI) return R.phi;
  // between the Eulerian and Lagrangian stages the post-Eulerian fields are visible
  return (b->next_stage == GP_STAGE_LAG) ? R.tmp[oidx(id)] : R.cur[oidx(id)];
}

void convert_any(void* dst, bool dst_double, const void* src, bool src_double, size_t n, hipStream_t st) {
  if (dst_double && src_double)
    launch_convert<double, double>((double*)dst, (const double*)src, n, st);
  else if (dst_double)
    launch_convert<double, float>((double*)dst, (const float*)src, n, st);
  else if (src_double)
    launch_convert<float, double>((float*)dst, (const double*)src, n, st);
  else
    launch_convert<float, float>((float*)dst, (const float*)src, n, st);
}

template <typename T>
RunDev<T> make_rundev(const RunHost& r) {
  RunDev<T> d{};
  d.g = r.g;
  d.ph = r.ph;
  for (int p = 0; p < 2; p++)
    for (int q = 0; q < 2; q++) d.dens[p][q] = r.dens[p][q];
  for (int o = 0; o < kNO; o++) {
    d.cur[o] = static_cast<T*>(r.cur[o]);
    d.tmp[o] = static_cast<T*>(r.tmp[o]);
  }
  d.phi = static_cast<T*>(r.phi);
  d.sc = r.sc;
  d.row0 = r.row0;
  return d;
}

// exp(-2 pi i k / L), k < n, as (re, im) pairs, from host FP64 libm
std::vector<double> twiddle_table(int n, int L) {
  std::vector<double> d(2 * (size_t)n);
  for (int k = 0; k < n; k++) {
    const double a = 2.0 * M_PI * (double)k / (double)L;
    d[2 * k] = std::cos(a);
    d[2 * k + 1] = -std::sin(a);
  }
  return d;
}

// The Green spectrum of a size class with isolated boundaries, computed once
// in FP64 (whatever the working precision) with temporary twiddle tables and
// a temporary spectrum of all 2nz padded planes, freed before returning.
gp_status iso_green_spectrum(gp_batch* b, SizeClass& c) {
  IsoGeom g = make_iso_geom(c.nx, c.ny, c.nz, 1, sizeof(double));
  g.run_stride = (size_t)g.pz * g.py * g.px;
  std::vector<void*> tmp;
  hipError_t e = hipSuccess;
  auto talloc = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    tmp.push_back(p);
    return p;
  };
  auto tw = [&](int n, int L) -> const cplx<double>* {
    const std::vector<double> d = twiddle_table(n, L);
    void* p = talloc(d.size() * sizeof(double));
    if (p && e == hipSuccess) e = hipMemcpy(p, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice);
    return static_cast<const cplx<double>*>(p);
  };
  IsoTables<double> t{};
  t.tw_x = tw(g.ax.L, g.ax.L);
  t.wn_x = tw(g.ax.L + 1, 2 * g.nx);
  t.tw_y = tw(g.ay.L, g.ay.L);
  t.tw_z = tw(g.az.L, g.az.L);
  auto* work = static_cast<cplx<double>*>(talloc(g.run_stride * sizeof(cplx<double>)));
  gp_status st = GP_OK;
  if (!t.tw_x || !t.wn_x || !t.tw_y || !t.tw_z || !work) {
    st = GP_E_NOMEM;
    b->last_error = "device allocation for the isolated Green spectrum failed";
  } else if (e != hipSuccess) {
    st = hip_fail(b, e, "isolated Green spectrum tables");
  } else {
    launch_iso_green(work, g, t, c.green, c.h, c.G, b->st);
    e = hipStreamSynchronize(b->st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) st = hip_fail(b, e, "isolated Green spectrum");
  }
  for (void* p : tmp) (void)hipFree(p);
  return st;
}

gp_status engine_create(gp_batch* b, const gp_config* cfgs, int nruns, void* hip_stream) {
  if (!cfgs || nruns < 1) return GP_E_INVALID;
  for (int r = 0; r < nruns; r++) {
    const gp_status v = validate(&cfgs[r]);
    if (v != GP_OK) {
      b->last_error = "run " + std::to_string(r) + ": invalid configuration";
      return v;
    }
    if (cfgs[r].precision != cfgs[0].precision) return GP_E_INVALID;
  }
  b->prec = cfgs[0].precision;
  if (hip_stream) {
    b->st = static_cast<hipStream_t>(hip_stream);
  } else {
    // a blocking stream orders after work on the legacy default stream
    const hipError_t se = hipStreamCreate(&b->st);
    if (se != hipSuccess) return hip_fail(b, se, "stream create");
    b->own_stream = true;
  }
  const size_t es = esize(b->prec);
  gp_status st = GP_OK;

  // runs and size classes (same grid, cell size and G share FFT launches)
  std::map<std::tuple<int, int, int, double, double, int>, int> cls_of;
  b->runs.resize(nruns);
  unsigned row = 0;
  for (int r = 0; r < nruns; r++) {
    RunHost& R = b->runs[r];
    R.cfg = cfgs[r];
    R.g.nx = cfgs[r].n[0];
    R.g.ny = cfgs[r].n[1];
    R.g.nz = cfgs[r].n[2];
    for (int d = 0; d < 3; d++) R.g.bc[d] = cfgs[r].bc[d];
    R.g.h = (cfgs[r].hi[0] - cfgs[r].lo[0]) / cfgs[r].n[0];
    R.g.ncell = (size_t)R.g.nx * R.g.ny * R.g.nz;
    R.g.phi_iso = cfgs[r].poisson == GP_POISSON_ISOLATED ? 1 : 0;
    R.ph = Phys{cfgs[r].gamma,
                cfgs[r].G,
                cfgs[r].cfl,
                cfgs[r].eta,
                cfgs[r].fixed_dt,
                cfgs[r].t_end,
                cfgs[r].cool_lambda,
                cfgs[r].cool_alpha,
                cfgs[r].cool_theta_min,
                {cfgs[r].gext[0], cfgs[r].gext[1], cfgs[r].gext[2]}};
    if (R.ph.cool_lambda != 0.0) b->cooling = true;
    // partial rows: one per item of the longer of the run's two lists (each
    // component writes its own slots of rows 0.. of its list; the slots of
    // rows beyond a list stay zero, which the reductions ignore)
    R.nrows = 0;
    for (int l = 0; l < 2; l++)
      for (int s = 0; s < kNumShapes; s++)
        for (int cap = 0; cap < kNumCaps; cap++)
          R.nrows = std::max(R.nrows, items_per_run(R, b->prec, l, s, cap));
    R.row0 = row;
    row += R.nrows;
    const auto key = std::make_tuple(R.g.nx, R.g.ny, R.g.nz, R.g.h, R.ph.G, R.g.phi_iso);
    auto it = cls_of.find(key);
    if (it == cls_of.end()) {
      SizeClass c;
      c.nx = R.g.nx;
      c.ny = R.g.ny;
      c.nz = R.g.nz;
      c.h = R.g.h;
      c.G = R.ph.G;
      c.iso = R.g.phi_iso;
      b->classes.push_back(c);
      it = cls_of.emplace(key, (int)b->classes.size() - 1).first;
    }
    R.cls = it->second;
    R.slot = (int)b->classes[R.cls].runs.size();
    b->classes[R.cls].runs.push_back(r);
  }

  // per-run buffers
  size_t max_cells = 0;
  for (RunHost& R : b->runs) {
    const size_t nc = R.g.ncell;
    max_cells = std::max(max_cells, nc);
    for (int p = 0; p < 2; p++)
      for (int q = 0; q < 2; q++) R.dens[p][q] = static_cast<double*>(dalloc(b, nc * sizeof(double), &st));
    for (int o = 0; o < kNO; o++) {
      R.cur[o] = dalloc(b, nc * es, &st);
      R.tmp[o] = dalloc(b, nc * es, &st);
    }
    R.sc = static_cast<DevScalars*>(dalloc(b, sizeof(DevScalars), &st));
    R.ring = static_cast<gp_diag*>(dalloc(b, sizeof(gp_diag) * kDiagCap, &st));
  }
  b->staging = dalloc(b, max_cells * sizeof(double), &st);

  // size classes: contiguous source / potential / spectrum, FFT tables
  unsigned eoff = 0;
  for (SizeClass& c : b->classes) {
    FftGeom& f = c.fg;
    f = make_fft_geom(c.nx, c.ny, c.nz, (int)c.runs.size(), b->prec, c.G != 0.0 && !c.iso);
    f.green_scale = -4.0 * M_PI * c.G * c.h * c.h / 6.0;
    const size_t nc = (size_t)c.nx * c.ny * c.nz, R = c.runs.size();
    c.src = static_cast<SrcSlot*>(dalloc(b, R * sizeof(SrcSlot), &st));
    // the potential of a run: nc values, or with isolated boundaries the
    // grid and its one-cell ring
    size_t phi_cells = nc;
    if (c.iso) {
      c.ig = make_iso_geom(c.nx, c.ny, c.nz, (int)R, es);
      phi_cells = c.ig.ext_cells;
    }
    c.phi = dalloc(b, R * phi_cells * es, &st);
    c.eoff = eoff;
    if (c.G != 0.0 && c.iso) {
      const IsoGeom& g = c.ig;
      c.spec = dalloc(b, R * g.run_stride * 2 * es, &st);
      c.tw_x = dalloc(b, (size_t)g.ax.L * 2 * es, &st);
      c.wn_x = dalloc(b, (size_t)(g.ax.L + 1) * 2 * es, &st);
      c.tw_y = dalloc(b, (size_t)g.ay.L * 2 * es, &st);
      c.tw_z = dalloc(b, (size_t)g.az.L * 2 * es, &st);
      c.green = static_cast<double*>(dalloc(b, (size_t)g.px * (g.ny + 1) * (g.nz + 1) * sizeof(double), &st));
      c.nep_run = (unsigned)(iso_blocks_z(g) / g.nruns);
      eoff += (unsigned)iso_blocks_z(g);
    } else if (c.G != 0.0) {
      c.spec = dalloc(b, R * (size_t)f.px * f.ny * f.nz * 2 * es, &st);
      c.tw_x = dalloc(b, (size_t)f.ax.L * 2 * es, &st);
      c.wn_x = dalloc(b, (size_t)(f.ax.L + 1) * 2 * es, &st);
      c.tw_y = dalloc(b, (size_t)f.ay.L * 2 * es, &st);
      c.tw_yh = dalloc(b, (size_t)f.ayh.L * 2 * es, &st);
      c.tw_z = dalloc(b, (size_t)f.az.L * 2 * es, &st);
      c.dtab[0] = static_cast<double*>(dalloc(b, (size_t)f.px * sizeof(double), &st));
      c.dtab[1] = static_cast<double*>(dalloc(b, (size_t)f.ny * sizeof(double), &st));
      c.dtab[2] = static_cast<double*>(dalloc(b, (size_t)f.nz * sizeof(double), &st));
      c.nep_run = (unsigned)(fft_blocks_z(f) / f.nruns);
      eoff += (unsigned)fft_blocks_z(f);
    }
    if (st != GP_OK) return st;
    for (size_t k = 0; k < R; k++) {
      RunHost& run = b->runs[c.runs[k]];
      run.phi = static_cast<char*>(c.phi) + k * phi_cells * es;
    }
  }
  b->nepot = eoff;
  b->epot = static_cast<double*>(dalloc(b, std::max(1u, eoff) * sizeof(double), &st));

  // work lists, partial rows, reduction items, finalize descriptors
  std::vector<WorkItem> lists[2][kNumShapes][kNumCaps];
  std::vector<RedItem> items;
  std::vector<FinDesc> fins;
  unsigned soff = 0;
  for (int r = 0; r < nruns; r++) {
    RunHost& R = b->runs[r];
    for (int l = 0; l < 2; l++)
      for (int s = 0; s < kNumShapes; s++)
        for (int cap = 0; cap < kNumCaps; cap++) make_items(R, r, b->prec, l, s, cap, lists[l][s][cap]);
    const unsigned nscr = std::max(1u, std::min(256u, R.nrows / 16));
    const unsigned chunk = (R.nrows + nscr - 1) / nscr;
    for (unsigned c = 0; c < nscr; c++) {
      const unsigned a = std::min(R.nrows, c * chunk), e = std::min(R.nrows, a + chunk);
      items.push_back({R.row0 + a, R.row0 + e});
    }
    FinDesc fd{};
    fd.g = R.g;
    fd.ph = R.ph;
    fd.soff = soff;
    fd.nscr = nscr;
    const SizeClass& c = b->classes[R.cls];
    fd.eoff = c.eoff + (unsigned)R.slot * c.nep_run;
    fd.nep = (c.G != 0.0) ? c.nep_run : 0u;
    // Parseval over the transformed lattice: the padded one when isolated
    fd.epot_scale = 1.0 / ((R.g.phi_iso ? 8.0 : 1.0) * (double)R.g.ncell);
    fd.sc = R.sc;
    fd.ring = R.ring;
    fins.push_back(fd);
    soff += nscr;
  }
  b->nred = (int)items.size();
  for (int l = 0; l < 2; l++)
    for (int s = 0; s < kNumShapes; s++)
      for (int cap = 0; cap < kNumCaps; cap++) {
        b->nwork[l][s][cap] = (unsigned)lists[l][s][cap].size();
        b->work[l][s][cap] =
            static_cast<WorkItem*>(dalloc(b, lists[l][s][cap].size() * sizeof(WorkItem), &st));
      }
  b->partials = static_cast<double*>(dalloc(b, (size_t)row * kNP * sizeof(double), &st));
  b->red_items = static_cast<RedItem*>(dalloc(b, items.size() * sizeof(RedItem), &st));
  b->scratch = static_cast<double*>(dalloc(b, (size_t)soff * kNP * sizeof(double), &st));
  b->fin = static_cast<FinDesc*>(dalloc(b, fins.size() * sizeof(FinDesc), &st));
  const size_t rdsz = b->prec == GP_FP64 ? sizeof(RunDev<double>) : sizeof(RunDev<float>);
  b->runs_dev = dalloc(b, rdsz * nruns, &st);
  if (st != GP_OK) return st;

  hipError_t e = hipSuccess;
  for (auto& a : b->allocs)
    if (e == hipSuccess) e = hipMemset(a.first, 0, a.second);
  auto put = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  for (int l = 0; l < 2; l++)
    for (int s = 0; s < kNumShapes; s++)
      for (int cap = 0; cap < kNumCaps; cap++)
        put(b->work[l][s][cap], lists[l][s][cap].data(), lists[l][s][cap].size() * sizeof(WorkItem));
  put(b->red_items, items.data(), items.size() * sizeof(RedItem));
  put(b->fin, fins.data(), fins.size() * sizeof(FinDesc));
  if (b->prec == GP_FP64) {
    std::vector<RunDev<double>> rd;
    for (auto& R : b->runs) rd.push_back(make_rundev<double>(R));
    put(b->runs_dev, rd.data(), rd.size() * sizeof(rd[0]));
  } else {
    std::vector<RunDev<float>> rd;
    for (auto& R : b->runs) rd.push_back(make_rundev<float>(R));
    put(b->runs_dev, rd.data(), rd.size() * sizeof(rd[0]));
  }
  auto put_tw = [&](void* dst, int n, int L) {
    const std::vector<double> d = twiddle_table(n, L);
    if (b->prec == GP_FP64) {
      put(dst, d.data(), d.size() * sizeof(double));
    } else {
      std::vector<float> fl(d.begin(), d.end());
      put(dst, fl.data(), fl.size() * sizeof(float));
    }
  };
  auto put_d = [&](double* dst, int n, int N) {
    std::vector<double> d(n);
    for (int k = 0; k < n; k++) {
      const double sn = std::sin(M_PI * (double)k / (double)N);
      d[k] = 1.0 - 2.0 / 3.0 * sn * sn;
    }
    put(dst, d.data(), n * sizeof(double));
  };
  for (SizeClass& c : b->classes) {
    std::vector<SrcSlot> slots;
    for (int r : c.runs) {
      const RunHost& R = b->runs[r];
      slots.push_back({{R.dens[0][0], R.dens[1][0]}, {R.dens[0][1], R.dens[1][1]}});
    }
    put(c.src, slots.data(), slots.size() * sizeof(SrcSlot));
    if (c.G == 0.0) continue;
    if (c.iso) {
      const IsoGeom& g = c.ig;
      put_tw(c.tw_x, g.ax.L, g.ax.L);
      put_tw(c.wn_x, g.ax.L + 1, 2 * g.nx);
      put_tw(c.tw_y, g.ay.L, g.ay.L);
      put_tw(c.tw_z, g.az.L, g.az.L);
      continue;
    }
    const FftGeom& f = c.fg;
    put_tw(c.tw_x, f.ax.L, f.ax.L);
    put_tw(c.wn_x, f.ax.L + 1, f.nx);
    put_tw(c.tw_y, f.ay.L, f.ay.L);
    put_tw(c.tw_yh, f.ayh.L, f.ayh.L);
    put_tw(c.tw_z, f.az.L, f.az.L);
    put_d(c.dtab[0], f.px, f.nx);
    put_d(c.dtab[1], f.ny, f.ny);
    put_d(c.dtab[2], f.nz, f.nz);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(b, e, "engine upload");
  for (SizeClass& c : b->classes) {
    if (!c.iso || c.G == 0.0) continue;
    const gp_status gs = iso_green_spectrum(b, c);
    if (gs != GP_OK) return gs;
  }
  // untuned defaults: 64 x 4 tiles, 32-plane chunk cap, a workgroup per item
  for (int k : kTunedIds) {
    b->kcfg[k] = TileCfg{};
    b->kcfg[k].blocks = work_count(b, k, b->kcfg[k]);
  }
  if (const char* path = std::getenv("GPUPEGAS_TUNE_CACHE")) b->cache_path = path;
  if (load_cache(b)) b->tuned = true;
  return GP_OK;
}

void engine_free(gp_batch* b) {
  if (b->st) (void)hipStreamSynchronize(b->st);
  drop_graphs(b);
  for (auto& a : b->allocs) (void)hipFree(a.first);
  b->allocs.clear();
  if (b->own_stream && b->st) (void)hipStreamDestroy(b->st);
}

gp_status engine_set_field(gp_batch* b, int r, int32_t field, const void* src, int32_t dtype, int32_t on_device) {
  if (r < 0 || r >= (int)b->runs.size() || !src || field < 0 || field >= GP_NFIELDS ||
      (dtype != GP_FP64 && dtype != GP_FP32))
    return GP_E_INVALID;
  if (b->next_stage != GP_STAGE_EUL) return GP_E_STATE;
  bool dst_double = false;
  void* dst = field_ptr(b, r, field, &dst_double);
  const bool src_double = dtype == GP_FP64;
  const size_t nc = b->runs[r].g.ncell;
  if (on_device) {
    convert_any(dst, dst_double, src, src_double, nc, b->st);
  } else {
    const size_t bytes = nc * (src_double ? sizeof(double) : sizeof(float));
    if (src_double == dst_double) {
      HIP_TRY(b, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->st));
    } else {
      HIP_TRY(b, hipMemcpyAsync(b->staging, src, bytes, hipMemcpyHostToDevice, b->st));
      convert_any(dst, dst_double, b->staging, src_double, nc, b->st);
    }
    HIP_TRY(b, hipStreamSynchronize(b->st));
  }
  HIP_TRY(b, hipGetLastError());
  b->need_prologue = true;
  return GP_OK;
}

gp_status engine_get_field(gp_batch* b, int r, int32_t field, void* dst, int32_t dtype, int32_t on_device) {
  if (r < 0 || r >= (int)b->runs.size() || !dst || field < 0 || field > GP_PHI ||
      (dtype != GP_FP64 && dtype != GP_FP32))
    return GP_E_INVALID;
  if (field == GP_PHI && b->need_prologue) {
    if (b->next_stage != GP_STAGE_EUL) return GP_E_STATE;
    run_prologue(b);
  }
  bool src_double = false;
  const void* src = field_ptr(b, r, field, &src_double);
  const bool dst_double = dtype == GP_FP64;
  const size_t nc = b->runs[r].g.ncell;
  if (field == GP_PHI && b->runs[r].g.phi_iso) {
    // the potential is stored with its ring: copy out the grid part
    const Grid& g = b->runs[r].g;
    void* out = on_device ? dst : b->staging;
    if (src_double) {
      if (dst_double) launch_phi_interior<double, double>((double*)out, (const double*)src, g.nx, g.ny, g.nz, b->st);
      else launch_phi_interior<float, double>((float*)out, (const double*)src, g.nx, g.ny, g.nz, b->st);
    } else {
      if (dst_double) launch_phi_interior<double, float>((double*)out, (const float*)src, g.nx, g.ny, g.nz, b->st);
      else launch_phi_interior<float, float>((float*)out, (const float*)src, g.nx, g.ny, g.nz, b->st);
    }
    if (!on_device)
      HIP_TRY(b, hipMemcpyAsync(dst, b->staging, nc * (dst_double ? 8 : 4), hipMemcpyDeviceToHost, b->st));
    HIP_TRY(b, hipStreamSynchronize(b->st));
    HIP_TRY(b, hipGetLastError());
    return latched(b, r);
  }
  const bool mid = b->next_stage == GP_STAGE_LAG;
  const bool gas_mom = field >= GP_MX && field <= GP_MZ, bme_mom = field >= GP_QX && field <= GP_QZ;
  if (mid && (gas_mom || bme_mom)) {
    // between the stages the momentum slots hold velocities: return density * velocity
    const double* dens = b->runs[r].dens[b->parity][gas_mom ? 0 : 1];
    void* out = on_device ? dst : b->staging;
    if (b->prec == GP_FP64) {
      if (dst_double) launch_density_times<double, double>((double*)out, dens, (const double*)src, nc, b->st);
      else launch_density_times<float, double>((float*)out, dens, (const double*)src, nc, b->st);
    } else {
      if (dst_double) launch_density_times<double, float>((double*)out, dens, (const float*)src, nc, b->st);
      else launch_density_times<float, float>((float*)out, dens, (const float*)src, nc, b->st);
    }
    if (!on_device)
      HIP_TRY(b, hipMemcpyAsync(dst, b->staging, nc * (dst_double ? 8 : 4), hipMemcpyDeviceToHost, b->st));
  } else if (on_device) {
    convert_any(dst, dst_double, src, src_double, nc, b->st);
  } else {
    const size_t bytes = nc * (dst_double ? sizeof(double) : sizeof(float));
    if (src_double == dst_double) {
      HIP_TRY(b, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, b->st));
    } else {
      convert_any(b->staging, dst_double, src, src_double, nc, b->st);
      HIP_TRY(b, hipMemcpyAsync(dst, b->staging, bytes, hipMemcpyDeviceToHost, b->st));
    }
  }
  HIP_TRY(b, hipStreamSynchronize(b->st));
  HIP_TRY(b, hipGetLastError());
  return latched(b, r);
}

gp_status engine_step(gp_batch* b, int32_t nsteps) {
  if (nsteps < 0) return GP_E_INVALID;
  if (b->next_stage != GP_STAGE_EUL) return GP_E_STATE;
  if (b->need_prologue) run_prologue(b);
  for (int t = 0; t < nsteps; t++) {
    if (b->use_graph && (b->tuned || !b->tune)) {
      if (!b->graph_ready[b->parity]) {
        gp_status r = build_graph(b, b->parity);
        if (r != GP_OK) return r;
      }
      HIP_TRY(b, hipGraphLaunch(b->gexec[b->parity], b->st));
      b->parity ^= 1;
    } else {
      run_step_direct(b, nullptr, true);
    }
  }
  HIP_TRY(b, hipGetLastError());
  return GP_OK;
}

gp_status engine_get_diag(gp_batch* b, int r, gp_diag* out, int32_t max, int32_t* count) {
  if (r < 0 || r >= (int)b->runs.size() || !out || !count || max < 0) return GP_E_INVALID;
  if (b->need_prologue && b->next_stage == GP_STAGE_EUL) run_prologue(b);
  HIP_TRY(b, hipStreamSynchronize(b->st));
  DevScalars h{};
  HIP_TRY(b, hipMemcpy(&h, b->runs[r].sc, sizeof(h), hipMemcpyDeviceToHost));
  const int avail = (int)std::min<uint32_t>(h.ndiag, (uint32_t)kDiagCap);
  const int n = std::min(avail, (int)max);
  std::vector<gp_diag> all(kDiagCap);
  HIP_TRY(b, hipMemcpy(all.data(), b->runs[r].ring, sizeof(gp_diag) * kDiagCap, hipMemcpyDeviceToHost));
  for (int t = 0; t < n; t++) out[t] = all[(h.ndiag - n + t) % kDiagCap];
  *count = n;
  // the records are delivered either way; the status reports what the device
  // latched for this run (each record's err field says from which step on)
  return latched(b, r);
}

gp_status engine_time_kernels(gp_batch* b, int32_t nsteps, double* ms, int32_t max) {
  if (!ms || nsteps <= 0 || max < 0) return GP_E_INVALID;
  if (b->next_stage != GP_STAGE_EUL) return GP_E_STATE;
  if (b->need_prologue) run_prologue(b);
  Timer tm;
  tm.on = true;
  for (int k = 0; k < 2 * GP_NKERNELS; k++) HIP_TRY(b, hipEventCreate(&tm.ev[k]));
  for (int k = 0; k < GP_NKERNELS; k++) tm.acc[k] = 0.0;
  // An untuned sim picks its launch sizes during the first timed step: the
  // candidates run before that kernel's first event, so the step is timed
  // with the picked sizes and the state advances by exactly nsteps.
  for (int t = 0; t < nsteps; t++) run_step_direct(b, &tm, true);
  for (int k = 0; k < 2 * GP_NKERNELS; k++) (void)hipEventDestroy(tm.ev[k]);
  for (int k = 0; k < std::min<int>(max, GP_NKERNELS); k++) ms[k] = tm.acc[k] / nsteps;
  HIP_TRY(b, hipGetLastError());
  return GP_OK;
}

gp_status engine_set_fft_form(gp_batch* b, int32_t form) {
  if (form != GP_FFT_AUTO && form != GP_FFT_LINES) return GP_E_INVALID;
  if (form != b->fft_form) {
    b->fft_form = form;
    drop_graphs(b);
  }
  return GP_OK;
}

bool tuned_kernel(int32_t kernel) {
  for (int q = 0; q < kTunedKernels; q++)
    if (kTunedIds[q] == kernel) return true;
  return false;
}

gp_status engine_set_launch(gp_batch* b, int32_t kernel, int32_t blocks) {
  if (!tuned_kernel(kernel) || blocks < 0) return GP_E_INVALID;
  TileCfg& c = b->kcfg[kernel];
  const unsigned nw = work_count(b, kernel, c);
  c.blocks = blocks == 0 ? nw : std::min<unsigned>((unsigned)blocks, nw);
  b->tune = false;
  drop_graphs(b);
  return GP_OK;
}

// Tile shape and z-chunk cap of a per-cell kernel (a workgroup per item).
gp_status engine_set_tiling(gp_batch* b, int32_t kernel, int32_t shape, int32_t cap_planes) {
  if (!tuned_kernel(kernel) || shape < 0 || shape >= kNumShapes) return GP_E_INVALID;
  int cap = -1;
  for (int q = 0; q < kNumCaps; q++)
    if (kCaps[q] == cap_planes) cap = q;
  if (cap < 0) return GP_E_INVALID;
  if (b->next_stage != GP_STAGE_EUL) return GP_E_STATE;
  TileCfg c{shape, cap, 0};
  c.blocks = work_count(b, kernel, c);
  b->kcfg[kernel] = c;
  b->tune = false;
  drop_graphs(b);
  if (kernel == GP_K_LAG_GAS || kernel == GP_K_LAG_BME) clear_partials(b);
  HIP_TRY(b, hipGetLastError());
  return GP_OK;
}

gp_status engine_get_tiling(gp_batch* b, int32_t kernel, int32_t* shape, int32_t* cap_planes) {
  if (!tuned_kernel(kernel) || !shape || !cap_planes) return GP_E_INVALID;
  *shape = b->kcfg[kernel].shape;
  *cap_planes = kCaps[b->kcfg[kernel].cap];
  return GP_OK;
}

double fft_bytes_per_cell(const gp_batch* b, int k) {
  // cell-weighted over the runs that solve Poisson
  double cells = 0.0, bytes = 0.0;
  const double es = (double)esize(b->prec);
  for (const RunHost& R : b->runs) {
    cells += (double)R.g.ncell;
    if (R.ph.G == 0.0) continue;
    if (R.g.phi_iso) {
      // padded spectrum values (complex, 2 es bytes) each pass reads or writes
      const double nx = R.g.nx, ny = R.g.ny, nz = R.g.nz, cs = 2.0 * es;
      const double px = nx + 1, py = 2.0 * ny;
      const double rows_src = px * ny * nz;            // x forward output, y forward input
      const double planes_src = px * py * nz;          // y forward output, z input
      const double planes_kept = px * py * (nz + 2);   // z output, y inverse input
      const double rows_kept = px * (ny + 2) * (nz + 2);  // y inverse output, x inverse input
      double v = 0.0;
      switch (k) {
        case GP_K_FFT_XY_FWD: v = 16.0 * nx * ny * nz + cs * (2.0 * rows_src + planes_src); break;
        case GP_K_FFT_Z: v = cs * (planes_src + planes_kept) + 8.0 * px * (ny + 1) * (nz + 1); break;
        case GP_K_FFT_XY_INV: v = cs * (planes_kept + 2.0 * rows_kept) + es * (nx + 2) * (ny + 2) * (nz + 2); break;
      }
      bytes += v;
      continue;
    }
    const double spec = 2.0 * es * (R.g.nx / 2 + 1) / R.g.nx;
    // the plane form does x and y in one pass; the line form reads and
    // writes the spectrum once more between its x and y passes
    const SizeClass& c = b->classes[R.cls];
    const double xy = (c.fg.plane && b->fft_form == GP_FFT_AUTO) ? 1.0 : 3.0;
    double v = 0.0;
    switch (k) {
      case GP_K_FFT_XY_FWD: v = 16.0 + xy * spec; break;  // reads rho and n (FP64)
      case GP_K_FFT_XY_INV: v = xy * spec + es; break;
      case GP_K_FFT_Z: v = 2.0 * spec; break;
    }
    bytes += v * (double)R.g.ncell;
  }
  return cells > 0 ? bytes / cells : 0.0;
}

double engine_bytes_per_cell(const gp_batch* b, int32_t kernel) {
  const double es = (double)esize(b->prec);
  // Eulerian: read the density, the component's fields and Phi; write its fields
  const double eul_gas = 8.0 + 5 * es + es + 5 * es;
  const double eul_bme = 8.0 + 15 * es + es + 15 * es;
  // Lagrangian: read the density and the post-Eulerian fields (the corner
  // velocities are formed on chip); write the density and the fields
  const double lag_gas = 8.0 + 5 * es + 8.0 + 5 * es;
  const double lag_bme = 8.0 + 15 * es + 8.0 + 15 * es;
  switch (kernel) {
    case GP_K_EUL_GAS: return eul_gas;
    case GP_K_EUL_BME: return eul_bme;
    case GP_K_LAG_GAS: return lag_gas;
    case GP_K_LAG_BME: return lag_bme;
    case GP_K_FINALIZE: return 0.0;
    case -1: {
      double t = eul_gas + eul_bme + lag_gas + lag_bme;
      for (int k = GP_K_FFT_XY_FWD; k <= GP_K_FFT_XY_INV; k++) t += fft_bytes_per_cell(b, k);
      return t;
    }
    default: return fft_bytes_per_cell(b, kernel);
  }
}

}  // namespace

extern "C" {

const char* gp_status_str(gp_status s) {
  switch (s) {
    case GP_OK: return "ok";
    case GP_E_INVALID: return "invalid argument or configuration";
    case GP_E_NOMEM: return "device allocation failed";
    case GP_E_HIP: return "HIP runtime error";
    case GP_E_NONFINITE: return "non-finite value in the state";
    case GP_E_NONPOSITIVE: return "non-positive density, pressure or stress";
    case GP_E_UNSUPPORTED: return "unsupported configuration";
    case GP_E_STATE: return "call out of order";
  }
  return "unknown status";
}

// ---- single simulation ------------------------------------------------------

// Why the calling thread's last gp_create / gp_batch_create failed (the
// handle it would have returned no longer exists).
thread_local std::string t_create_error;

void note_create_error(const gp_batch* b, gp_status r) {
  t_create_error = b->last_error.empty() ? std::string(gp_status_str(r)) : b->last_error;
}

const char* gp_last_error(const gp_sim* sim) { return sim ? sim->last_error.c_str() : t_create_error.c_str(); }

gp_status gp_create(const gp_config* cfg, void* hip_stream, gp_sim** out) {
  if (!cfg || !out) return GP_E_INVALID;
  *out = nullptr;
  gp_sim* s = new gp_sim();
  const gp_status r = engine_create(s, cfg, 1, hip_stream);
  if (r != GP_OK) {
    note_create_error(s, r);
    engine_free(s);
    delete s;
    return r;
  }
  *out = s;
  return GP_OK;
}

gp_status gp_destroy(gp_sim* s) {
  if (!s) return GP_E_INVALID;
  engine_free(s);
  delete s;
  return GP_OK;
}

gp_status gp_set_field(gp_sim* s, int32_t field, const void* src, int32_t dtype, int32_t on_device) {
  if (!s) return GP_E_INVALID;
  return engine_set_field(s, 0, field, src, dtype, on_device);
}

gp_status gp_get_field(gp_sim* s, int32_t field, void* dst, int32_t dtype, int32_t on_device) {
  if (!s) return GP_E_INVALID;
  return engine_get_field(s, 0, field, dst, dtype, on_device);
}

gp_status gp_step(gp_sim* s, int32_t nsteps) {
  if (!s) return GP_E_INVALID;
  return engine_step(s, nsteps);
}

gp_status gp_get_potential(gp_sim* s, void* dst, int32_t dtype, int32_t on_device) {
  if (!s) return GP_E_INVALID;
  return engine_get_field(s, 0, GP_PHI, dst, dtype, on_device);
}

gp_status gp_sync(gp_sim* s) {
  if (!s) return GP_E_INVALID;
  HIP_TRY(s, hipStreamSynchronize(s->st));
  return latched(s);
}

gp_status gp_get_diag(gp_sim* s, gp_diag* out, int32_t max, int32_t* count) {
  if (!s) return GP_E_INVALID;
  return engine_get_diag(s, 0, out, max, count);
}

gp_status gp_set_time(gp_sim* s, double t, int64_t step) {
  if (!s) return GP_E_INVALID;
  if (s->next_stage != GP_STAGE_EUL) return GP_E_STATE;
  HIP_TRY(s, hipStreamSynchronize(s->st));
  DevScalars h{};
  HIP_TRY(s, hipMemcpy(&h, s->runs[0].sc, sizeof(h), hipMemcpyDeviceToHost));
  h.t = t;
  h.step = step;
  HIP_TRY(s, hipMemcpy(s->runs[0].sc, &h, sizeof(h), hipMemcpyHostToDevice));
  s->need_prologue = true;
  return GP_OK;
}

gp_status gp_get_time(gp_sim* s, double* t, double* dt, int64_t* step) {
  if (!s) return GP_E_INVALID;
  if (s->need_prologue && s->next_stage == GP_STAGE_EUL) run_prologue(s);
  HIP_TRY(s, hipStreamSynchronize(s->st));
  DevScalars h{};
  HIP_TRY(s, hipMemcpy(&h, s->runs[0].sc, sizeof(h), hipMemcpyDeviceToHost));
  if (t) *t = h.t;
  if (dt) *dt = h.dt;
  if (step) *step = h.step;
  return GP_OK;
}

gp_status gp_debug_stage(gp_sim* s, int32_t stage) {
  if (!s || stage < GP_STAGE_EUL || stage > GP_STAGE_FINALIZE) return GP_E_INVALID;
  if (s->need_prologue && s->next_stage == GP_STAGE_EUL) run_prologue(s);
  if (stage != s->next_stage) return GP_E_STATE;
  run_stage(s, stage, nullptr, false);
  s->next_stage = (stage + 1) % 4;
  HIP_TRY(s, hipGetLastError());
  return GP_OK;
}

gp_status gp_time_kernels(gp_sim* s, int32_t nsteps, double* ms, int32_t max) {
  if (!s) return GP_E_INVALID;
  return engine_time_kernels(s, nsteps, ms, max);
}

gp_status gp_use_graph(gp_sim* s, int32_t enable) {
  if (!s) return GP_E_INVALID;
  s->use_graph = enable != 0;
  return GP_OK;
}

gp_status gp_set_launch(gp_sim* s, int32_t kernel, int32_t blocks) {
  if (!s) return GP_E_INVALID;
  return engine_set_launch(s, kernel, blocks);
}

gp_status gp_set_fft_form(gp_sim* s, int32_t form) {
  if (!s) return GP_E_INVALID;
  return engine_set_fft_form(s, form);
}

gp_status gp_get_launch(gp_sim* s, int32_t kernel, int32_t* blocks) {
  if (!s || !blocks || kernel < 0 || kernel >= GP_NKERNELS) return GP_E_INVALID;
  *blocks = (int32_t)s->kcfg[kernel].blocks;
  return GP_OK;
}

gp_status gp_set_tiling(gp_sim* s, int32_t kernel, int32_t shape, int32_t cap_planes) {
  if (!s) return GP_E_INVALID;
  return engine_set_tiling(s, kernel, shape, cap_planes);
}

gp_status gp_get_tiling(gp_sim* s, int32_t kernel, int32_t* shape, int32_t* cap_planes) {
  if (!s) return GP_E_INVALID;
  return engine_get_tiling(s, kernel, shape, cap_planes);
}

double gp_algorithmic_bytes_per_cell(const gp_sim* s, int32_t kernel) {
  return s ? engine_bytes_per_cell(s, kernel) : 0.0;
}

// ---- batches -------------------------------------------------------------------

gp_status gp_batch_create(const gp_config* cfgs, int32_t nruns, void* hip_stream, gp_batch** out) {
  if (!cfgs || !out || nruns < 1) return GP_E_INVALID;
  *out = nullptr;
  gp_batch* b = new gp_batch();
  const gp_status r = engine_create(b, cfgs, nruns, hip_stream);
  if (r != GP_OK) {
    note_create_error(b, r);
    engine_free(b);
    delete b;
    return r;
  }
  *out = b;
  return GP_OK;
}

gp_status gp_batch_destroy(gp_batch* b) {
  if (!b) return GP_E_INVALID;
  engine_free(b);
  delete b;
  return GP_OK;
}

gp_status gp_batch_set_field(gp_batch* b, int32_t run, int32_t field, const void* src, int32_t dtype,
                             int32_t on_device) {
  if (!b) return GP_E_INVALID;
  return engine_set_field(b, run, field, src, dtype, on_device);
}

gp_status gp_batch_get_field(gp_batch* b, int32_t run, int32_t field, void* dst, int32_t dtype,
                             int32_t on_device) {
  if (!b) return GP_E_INVALID;
  return engine_get_field(b, run, field, dst, dtype, on_device);
}

gp_status gp_batch_get_potential(gp_batch* b, int32_t run, void* dst, int32_t dtype, int32_t on_device) {
  if (!b) return GP_E_INVALID;
  return engine_get_field(b, run, GP_PHI, dst, dtype, on_device);
}

gp_status gp_batch_step(gp_batch* b, int32_t nsteps) {
  if (!b) return GP_E_INVALID;
  return engine_step(b, nsteps);
}

gp_status gp_batch_sync(gp_batch* b) {
  if (!b) return GP_E_INVALID;
  HIP_TRY(b, hipStreamSynchronize(b->st));
  return latched(b);
}

gp_status gp_batch_get_diag(gp_batch* b, int32_t run, gp_diag* out, int32_t max, int32_t* count) {
  if (!b) return GP_E_INVALID;
  return engine_get_diag(b, run, out, max, count);
}

gp_status gp_batch_time_kernels(gp_batch* b, int32_t nsteps, double* ms, int32_t max) {
  if (!b) return GP_E_INVALID;
  return engine_time_kernels(b, nsteps, ms, max);
}

gp_status gp_batch_set_launch(gp_batch* b, int32_t kernel, int32_t blocks) {
  if (!b) return GP_E_INVALID;
  return engine_set_launch(b, kernel, blocks);
}

gp_status gp_batch_set_fft_form(gp_batch* b, int32_t form) {
  if (!b) return GP_E_INVALID;
  return engine_set_fft_form(b, form);
}

gp_status gp_batch_get_launch(gp_batch* b, int32_t kernel, int32_t* blocks) {
  if (!b || !blocks || kernel < 0 || kernel >= GP_NKERNELS) return GP_E_INVALID;
  *blocks = (int32_t)b->kcfg[kernel].blocks;
  return GP_OK;
}

gp_status gp_batch_set_tiling(gp_batch* b, int32_t kernel, int32_t shape, int32_t cap_planes) {
  if (!b) return GP_E_INVALID;
  return engine_set_tiling(b, kernel, shape, cap_planes);
}

gp_status gp_batch_get_tiling(gp_batch* b, int32_t kernel, int32_t* shape, int32_t* cap_planes) {
  if (!b) return GP_E_INVALID;
  return engine_get_tiling(b, kernel, shape, cap_planes);
}

double gp_batch_algorithmic_bytes_per_cell(const gp_batch* b, int32_t kernel) {
  return b ? engine_bytes_per_cell(b, kernel) : 0.0;
}

int64_t gp_batch_cells(const gp_batch* b) {
  if (!b) return 0;
  int64_t n = 0;
  for (const RunHost& R : b->runs) n += (int64_t)R.g.ncell;
  return n;
}

const char* gp_batch_last_error(const gp_batch* b) { return b ? b->last_error.c_str() : t_create_error.c_str(); }

}  // extern "C"
