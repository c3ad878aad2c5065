// Host engine and C ABI of the GPUPEGAS timestep library.
//
// A sim owns its device state: rho and n in FP64 (two buffers that swap each
// step), the 20 other fields in the working precision in two sets ("cur" holds
// the state, "tmp" the post-Eulerian fields), the potential, s = rho + n, the
// half spectrum, per-block partial sums, and the device scalars (t, tau, step,
// error bits, diagnostics ring).  A step is enqueued as
//   Eulerian -> Lagrangian(+epilogue) -> 5 FFT passes -> reduce/finalize
// and, by default, replayed from a captured HIP graph (one per buffer parity);
// tau never leaves the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

using namespace gp;

struct gp_sim {
  gp_config cfg{};
  Grid g{};
  Phys ph{};
  int prec = GP_FP64;
  int device = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;

  std::vector<std::pair<void*, size_t>> allocs;
  double* dens[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [parity][rho, n]
  void* cur[kNO] = {};
  void* tmp[kNO] = {};
  void* vtx = nullptr;   // corner velocities, 6 components
  size_t vstride = 0;
  void* s = nullptr;
  void* phi = nullptr;
  void* spec = nullptr;
  void* staging = nullptr;
  double* partials = nullptr;
  int nrows = 0;
  double* scratch = nullptr;
  int nscratch = 0;
  double* epot = nullptr;
  int nepot = 0;
  DevScalars* sc = nullptr;
  gp_diag* ring = nullptr;
  void* tw_x = nullptr;
  void* wn_x = nullptr;
  void* tw_y = nullptr;
  void* tw_z = nullptr;
  double* dtab[3] = {nullptr, nullptr, nullptr};
  FftGeom fg{};

  int parity = 0;
  bool need_prologue = true;
  int next_stage = GP_STAGE_EUL;
  bool use_graph = true;
  bool graph_ready[2] = {false, false};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::string last_error;
};

namespace {

gp_status hip_fail(gp_sim* s, hipError_t e, const char* what) {
  if (s) s->last_error = std::string(what) + ": " + hipGetErrorString(e);
  return GP_E_HIP;
}

#define HIP_TRY(sim, expr)                                     \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return hip_fail((sim), e_, #expr);   \
  } while (0)

bool fft_len_ok(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

FftAxis make_axis(int L) {
  FftAxis a{};
  a.L = L;
  int m = L;
  while (m % 8 == 0 && m > 1) { a.rad[a.nst++] = 8; m /= 8; }
  while (m % 4 == 0) { a.rad[a.nst++] = 4; m /= 4; }
  while (m % 2 == 0) { a.rad[a.nst++] = 2; m /= 2; }
  while (m % 3 == 0) { a.rad[a.nst++] = 3; m /= 3; }
  return a;
}

size_t esize(int prec) { return prec == GP_FP64 ? sizeof(double) : sizeof(float); }

void* dalloc(gp_sim* s, size_t bytes, gp_status* st) {
  void* p = nullptr;
  if (*st != GP_OK) return nullptr;
  bytes = (bytes + 255) & ~size_t(255);
  if (hipMalloc(&p, bytes) != hipSuccess) {
    *st = GP_E_NOMEM;
    s->last_error = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
    return nullptr;
  }
  s->allocs.push_back({p, bytes});
  return p;
}

template <typename T>
Fields<T> fields_cur(const gp_sim* s) {
  Fields<T> f{};
  f.rho = s->dens[s->parity][0];
  f.nb = s->dens[s->parity][1];
  for (int o = 0; o < kNO; o++) f.o[o] = static_cast<T*>(s->cur[o]);
  return f;
}
template <typename T>
Fields<T> fields_tmp(const gp_sim* s) {
  Fields<T> f{};
  for (int o = 0; o < kNO; o++) f.o[o] = static_cast<T*>(s->tmp[o]);
  return f;
}
template <typename T>
Fields<T> fields_next(const gp_sim* s) {
  Fields<T> f{};
  f.rho = s->dens[s->parity ^ 1][0];
  f.nb = s->dens[s->parity ^ 1][1];
  for (int o = 0; o < kNO; o++) f.o[o] = static_cast<T*>(s->cur[o]);
  return f;
}

template <typename T>
FftTables<T> tables(const gp_sim* s) {
  FftTables<T> t{};
  t.tw_x = static_cast<const cplx<T>*>(s->tw_x);
  t.wn_x = static_cast<const cplx<T>*>(s->wn_x);
  t.tw_y = static_cast<const cplx<T>*>(s->tw_y);
  t.tw_z = static_cast<const cplx<T>*>(s->tw_z);
  t.dx = s->dtab[0];
  t.dy = s->dtab[1];
  t.dz = s->dtab[2];
  return t;
}

// Kernel-launch hooks: timing brackets each launch with events when asked.
struct Timer {
  hipEvent_t ev[2 * GP_NKERNELS];
  double acc[GP_NKERNELS];
  bool on = false;
};

template <typename T>
void enqueue_poisson(gp_sim* s, Timer* tm) {
  if (s->cfg.G == 0.0) return;
  const FftTables<T> t = tables<T>(s);
  auto* spec = static_cast<cplx<T>*>(s->spec);
  auto mark = [&](int k, int side) {
    if (tm && tm->on) (void)hipEventRecord(tm->ev[2 * k + side], s->st);
  };
  auto done = [&](int k) {
    if (tm && tm->on) {
      (void)hipEventSynchronize(tm->ev[2 * k + 1]);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, tm->ev[2 * k], tm->ev[2 * k + 1]);
      tm->acc[k] += ms;
    }
  };
  mark(GP_K_FFT_X_FWD, 0);
  launch_fft_x_fwd<T>(static_cast<const T*>(s->s), spec, s->fg, t, s->st);
  mark(GP_K_FFT_X_FWD, 1);
  done(GP_K_FFT_X_FWD);
  mark(GP_K_FFT_Y_FWD, 0);
  launch_fft_y<T>(spec, s->fg, t, false, s->st);
  mark(GP_K_FFT_Y_FWD, 1);
  done(GP_K_FFT_Y_FWD);
  mark(GP_K_FFT_Z, 0);
  launch_fft_z_green<T>(spec, s->fg, t, s->epot, s->st);
  mark(GP_K_FFT_Z, 1);
  done(GP_K_FFT_Z);
  mark(GP_K_FFT_Y_INV, 0);
  launch_fft_y<T>(spec, s->fg, t, true, s->st);
  mark(GP_K_FFT_Y_INV, 1);
  done(GP_K_FFT_Y_INV);
  mark(GP_K_FFT_X_INV, 0);
  launch_fft_x_inv<T>(spec, static_cast<T*>(s->phi), s->fg, t, s->st);
  mark(GP_K_FFT_X_INV, 1);
  done(GP_K_FFT_X_INV);
}

void enqueue_finalize(gp_sim* s, int advanced, Timer* tm) {
  const double escale = 1.0 / ((double)s->g.nx * s->g.ny * s->g.nz);
  if (tm && tm->on) (void)hipEventRecord(tm->ev[2 * GP_K_FINALIZE], s->st);
  launch_finalize(s->partials, s->nrows, s->scratch, s->nscratch, s->epot, s->cfg.G != 0.0 ? s->nepot : 0, s->g,
                  s->ph, escale, advanced, s->sc, s->ring, s->st);
  if (tm && tm->on) {
    (void)hipEventRecord(tm->ev[2 * GP_K_FINALIZE + 1], s->st);
    (void)hipEventSynchronize(tm->ev[2 * GP_K_FINALIZE + 1]);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, tm->ev[2 * GP_K_FINALIZE], tm->ev[2 * GP_K_FINALIZE + 1]);
    tm->acc[GP_K_FINALIZE] += ms;
  }
}

template <typename T>
void enqueue_stage(gp_sim* s, int stage, Timer* tm) {
  auto timed = [&](int k, auto&& fn) {
    if (tm && tm->on) (void)hipEventRecord(tm->ev[2 * k], s->st);
    fn();
    if (tm && tm->on) {
      (void)hipEventRecord(tm->ev[2 * k + 1], s->st);
      (void)hipEventSynchronize(tm->ev[2 * k + 1]);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, tm->ev[2 * k], tm->ev[2 * k + 1]);
      tm->acc[k] += ms;
    }
  };
  switch (stage) {
    case GP_STAGE_EUL:
      timed(GP_K_EUL, [&] {
        launch_eulerian<T>(fields_cur<T>(s), fields_tmp<T>(s), static_cast<const T*>(s->phi), s->g, s->ph, s->sc,
                           s->st);
      });
      break;
    case GP_STAGE_LAG:
      timed(GP_K_VERTEX, [&] {
        launch_vertex<T>(fields_tmp<T>(s), static_cast<T*>(s->vtx), s->vstride, s->g, s->st);
      });
      timed(GP_K_LAG, [&] {
        launch_lagrangian<T>(fields_cur<T>(s), fields_tmp<T>(s), fields_next<T>(s), static_cast<const T*>(s->vtx),
                             s->vstride, static_cast<T*>(s->s), s->g, s->ph, s->sc, s->partials, s->st);
      });
      s->parity ^= 1;
      break;
    case GP_STAGE_POISSON:
      enqueue_poisson<T>(s, tm);
      break;
    case GP_STAGE_FINALIZE:
      enqueue_finalize(s, 1, tm);
      break;
  }
}

template <typename T>
void enqueue_prologue(gp_sim* s) {
  launch_init_partials<T>(fields_cur<T>(s), static_cast<T*>(s->s), s->g, s->ph, s->partials, s->st);
  enqueue_poisson<T>(s, nullptr);
  enqueue_finalize(s, 0, nullptr);
}

void run_prologue(gp_sim* s) {
  if (s->prec == GP_FP64)
    enqueue_prologue<double>(s);
  else
    enqueue_prologue<float>(s);
  s->need_prologue = false;
  s->next_stage = GP_STAGE_EUL;
}

void run_stage(gp_sim* s, int stage, Timer* tm) {
  if (s->prec == GP_FP64)
    enqueue_stage<double>(s, stage, tm);
  else
    enqueue_stage<float>(s, stage, tm);
}

void run_step_direct(gp_sim* s, Timer* tm) {
  for (int st = 0; st < 4; st++) run_stage(s, st, tm);
}

gp_status build_graph(gp_sim* s, int parity) {
  const int saved = s->parity;
  s->parity = parity;
  hipGraph_t graph = nullptr;
  HIP_TRY(s, hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
  run_step_direct(s, nullptr);
  hipError_t e = hipStreamEndCapture(s->st, &graph);
  s->parity = saved;
  if (e != hipSuccess) return hip_fail(s, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&s->gexec[parity], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(s, e, "hipGraphInstantiate");
  s->graph_ready[parity] = true;
  return GP_OK;
}

gp_status latched(gp_sim* s) {
  DevScalars h{};
  HIP_TRY(s, hipMemcpy(&h, s->sc, sizeof(h), hipMemcpyDeviceToHost));
  if (h.err & ERR_NONFINITE) {
    s->last_error = "non-finite value in the state";
    return GP_E_NONFINITE;
  }
  if (h.err & (ERR_DENSITY | ERR_PRESSURE | ERR_STRESS | ERR_NOSPEED)) {
    s->last_error = "non-positive density, pressure or diagonal stress (bits " + std::to_string(h.err) + ")";
    return GP_E_NONPOSITIVE;
  }
  return GP_OK;
}

// device pointer of field `id` in the state visible to gp_get_field / gp_set_field
void* field_ptr(gp_sim* s, int id, bool* is_double) {
  if (id == GP_RHO || id == GP_N) {
    *is_double = true;
    return s->dens[s->parity][id == GP_RHO ? 0 : 1];
  }
  *is_double = s->prec == GP_FP64;
  if (id == GP_PHI) return s->phi;
  // between the Eulerian and Lagrangian stages the post-Eulerian fields are visible
  const bool mid = (s->next_stage == GP_STAGE_LAG);
  return mid ? s->tmp[oidx(id)] : s->cur[oidx(id)];
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

double fft_bytes_per_cell(const gp_sim* s, int k) {
  if (s->cfg.G == 0.0) return 0.0;
  const double es = (double)esize(s->prec);
  const double spec = 2.0 * es * s->fg.px / s->g.nx;  // half-spectrum bytes per cell
  switch (k) {
    case GP_K_FFT_X_FWD: return es + spec;
    case GP_K_FFT_X_INV: return spec + es;
    case GP_K_FFT_Y_FWD:
    case GP_K_FFT_Z:
    case GP_K_FFT_Y_INV: return 2.0 * spec;
    default: return 0.0;
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

const char* gp_last_error(const gp_sim* sim) { return sim ? sim->last_error.c_str() : "null sim"; }

gp_status gp_destroy(gp_sim* s) {
  if (!s) return GP_E_INVALID;
  if (s->st) (void)hipStreamSynchronize(s->st);
  for (int p = 0; p < 2; p++)
    if (s->gexec[p]) (void)hipGraphExecDestroy(s->gexec[p]);
  for (auto& a : s->allocs) (void)hipFree(a.first);
  if (s->own_stream && s->st) (void)hipStreamDestroy(s->st);
  delete s;
  return GP_OK;
}

gp_status gp_create(const gp_config* cfg, void* hip_stream, gp_sim** out) {
  if (!cfg || !out) return GP_E_INVALID;
  *out = nullptr;
  for (int d = 0; d < 3; d++) {
    if (cfg->n[d] < 4 || cfg->n[d] > 1024 || !(cfg->hi[d] > cfg->lo[d])) return GP_E_INVALID;
    if (cfg->bc[d] != GP_BC_OUTFLOW && cfg->bc[d] != GP_BC_PERIODIC) return GP_E_INVALID;
  }
  const double h = (cfg->hi[0] - cfg->lo[0]) / cfg->n[0];
  for (int d = 1; d < 3; d++)
    if (std::fabs((cfg->hi[d] - cfg->lo[d]) / cfg->n[d] - h) > 1e-12 * h) return GP_E_INVALID;
  if (!(cfg->gamma > 1.0) || !(cfg->cfl > 0.0) || cfg->reserved != 0) return GP_E_INVALID;
  if (cfg->precision != GP_FP64 && cfg->precision != GP_FP32) return GP_E_INVALID;
  if (cfg->G != 0.0)
    for (int d = 0; d < 3; d++)
      if (!fft_len_ok(cfg->n[d]) || cfg->n[d] % 2 != 0) return GP_E_UNSUPPORTED;

  gp_sim* s = new gp_sim();
  s->cfg = *cfg;
  s->prec = cfg->precision;
  s->g.nx = cfg->n[0];
  s->g.ny = cfg->n[1];
  s->g.nz = cfg->n[2];
  for (int d = 0; d < 3; d++) s->g.bc[d] = cfg->bc[d];
  s->g.h = h;
  s->g.ncell = (size_t)s->g.nx * s->g.ny * s->g.nz;
  s->ph = Phys{cfg->gamma, cfg->G, cfg->cfl, cfg->eta, cfg->fixed_dt, cfg->t_end};
  (void)hipGetDevice(&s->device);
  if (hip_stream) {
    s->st = static_cast<hipStream_t>(hip_stream);
  } else {
    // a blocking stream orders after work on the legacy default stream
    if (hipStreamCreate(&s->st) != hipSuccess) {
      delete s;
      return GP_E_HIP;
    }
    s->own_stream = true;
  }

  const size_t nc = s->g.ncell, es = esize(s->prec);
  gp_status st = GP_OK;
  for (int p = 0; p < 2; p++)
    for (int q = 0; q < 2; q++) s->dens[p][q] = static_cast<double*>(dalloc(s, nc * sizeof(double), &st));
  for (int o = 0; o < kNO; o++) {
    s->cur[o] = dalloc(s, nc * es, &st);
    s->tmp[o] = dalloc(s, nc * es, &st);
  }
  s->vstride = (((size_t)(s->g.nx + 1) * (s->g.ny + 1) * (s->g.nz + 1)) + 63) / 64 * 64;
  s->vtx = dalloc(s, 6 * s->vstride * es, &st);
  s->s = dalloc(s, nc * es, &st);
  s->phi = dalloc(s, nc * es, &st);
  s->staging = dalloc(s, nc * sizeof(double), &st);
  s->nrows = (int)cell_blocks(s->g);
  s->partials = static_cast<double*>(dalloc(s, (size_t)s->nrows * kNP * sizeof(double), &st));
  s->nscratch = std::max(1, std::min(256, s->nrows / 64));
  s->scratch = static_cast<double*>(dalloc(s, (size_t)s->nscratch * kNP * sizeof(double), &st));
  s->sc = static_cast<DevScalars*>(dalloc(s, sizeof(DevScalars), &st));
  s->ring = static_cast<gp_diag*>(dalloc(s, sizeof(gp_diag) * kDiagCap, &st));

  // FFT geometry and tables (host FP64 libm, converted to the working type)
  FftGeom& f = s->fg;
  f.nx = s->g.nx;
  f.ny = s->g.ny;
  f.nz = s->g.nz;
  f.px = f.nx / 2 + 1;
  f.ax = make_axis(f.nx / 2);
  f.ay = make_axis(f.ny);
  f.az = make_axis(f.nz);
  const int maxpts = 32768 / (int)(2 * es);
  f.rows_per_block = std::max(1, maxpts / (2 * f.ax.L));
  f.cols_y = std::max(1, std::min({16, f.px, maxpts / f.ay.L}));
  f.cols_z = std::max(1, std::min({16, f.px, maxpts / f.az.L}));
  f.green_scale = -4.0 * M_PI * cfg->G * h * h / 6.0;
  f.norm = 2.0 / ((double)f.nx * f.ny * f.nz);
  s->nepot = fft_blocks_z(f);
  s->spec = dalloc(s, (size_t)f.px * f.ny * f.nz * 2 * es, &st);
  s->epot = static_cast<double*>(dalloc(s, (size_t)s->nepot * sizeof(double), &st));
  s->tw_x = dalloc(s, (size_t)f.ax.L * 2 * es, &st);
  s->wn_x = dalloc(s, (size_t)(f.ax.L + 1) * 2 * es, &st);
  s->tw_y = dalloc(s, (size_t)f.ay.L * 2 * es, &st);
  s->tw_z = dalloc(s, (size_t)f.az.L * 2 * es, &st);
  s->dtab[0] = static_cast<double*>(dalloc(s, (size_t)f.px * sizeof(double), &st));
  s->dtab[1] = static_cast<double*>(dalloc(s, (size_t)f.ny * sizeof(double), &st));
  s->dtab[2] = static_cast<double*>(dalloc(s, (size_t)f.nz * sizeof(double), &st));
  if (st != GP_OK) {
    gp_destroy(s);
    return st;
  }

  auto upload_tw = [&](void* dst, int n, int L) -> hipError_t {
    // exp(-2 pi i k / L), k < n
    std::vector<double> d(2 * (size_t)n);
    for (int k = 0; k < n; k++) {
      const double a = 2.0 * M_PI * (double)k / (double)L;
      d[2 * k] = std::cos(a);
      d[2 * k + 1] = -std::sin(a);
    }
    if (s->prec == GP_FP64) return hipMemcpy(dst, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice);
    std::vector<float> fl(d.begin(), d.end());
    return hipMemcpy(dst, fl.data(), fl.size() * sizeof(float), hipMemcpyHostToDevice);
  };
  auto upload_d = [&](double* dst, int n, int N) -> hipError_t {
    std::vector<double> d(n);
    for (int k = 0; k < n; k++) {
      const double sn = std::sin(M_PI * (double)k / (double)N);
      d[k] = 1.0 - 2.0 / 3.0 * sn * sn;
    }
    return hipMemcpy(dst, d.data(), n * sizeof(double), hipMemcpyHostToDevice);
  };
  hipError_t e = hipSuccess;
  // zero every buffer once (outside any captured graph), then fill the tables
  for (auto& a : s->allocs)
    if (e == hipSuccess) e = hipMemset(a.first, 0, a.second);
  if (e == hipSuccess) e = upload_tw(s->tw_x, f.ax.L, f.ax.L);
  if (e == hipSuccess) e = upload_tw(s->wn_x, f.ax.L + 1, f.nx);
  if (e == hipSuccess) e = upload_tw(s->tw_y, f.ay.L, f.ay.L);
  if (e == hipSuccess) e = upload_tw(s->tw_z, f.az.L, f.az.L);
  if (e == hipSuccess) e = upload_d(s->dtab[0], f.px, f.nx);
  if (e == hipSuccess) e = upload_d(s->dtab[1], f.ny, f.ny);
  if (e == hipSuccess) e = upload_d(s->dtab[2], f.nz, f.nz);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    hip_fail(s, e, "gp_create upload");
    gp_destroy(s);
    return GP_E_HIP;
  }
  *out = s;
  return GP_OK;
}

gp_status gp_set_field(gp_sim* s, int32_t field, const void* src, int32_t dtype, int32_t on_device) {
  if (!s || !src || field < 0 || field >= GP_NFIELDS || (dtype != GP_FP64 && dtype != GP_FP32))
    return GP_E_INVALID;
  if (s->next_stage != GP_STAGE_EUL) return GP_E_STATE;
  bool dst_double = false;
  void* dst = field_ptr(s, field, &dst_double);
  const bool src_double = dtype == GP_FP64;
  const size_t nc = s->g.ncell;
  if (on_device) {
    convert_any(dst, dst_double, src, src_double, nc, s->st);
  } else {
    const size_t bytes = nc * (src_double ? sizeof(double) : sizeof(float));
    if (src_double == dst_double) {
      HIP_TRY(s, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s->st));
    } else {
      HIP_TRY(s, hipMemcpyAsync(s->staging, src, bytes, hipMemcpyHostToDevice, s->st));
      convert_any(dst, dst_double, s->staging, src_double, nc, s->st);
    }
    HIP_TRY(s, hipStreamSynchronize(s->st));
  }
  HIP_TRY(s, hipGetLastError());
  s->need_prologue = true;
  return GP_OK;
}

gp_status gp_get_field(gp_sim* s, int32_t field, void* dst, int32_t dtype, int32_t on_device) {
  if (!s || !dst || field < 0 || field > GP_PHI || (dtype != GP_FP64 && dtype != GP_FP32)) return GP_E_INVALID;
  if (field == GP_PHI && s->need_prologue) {
    if (s->next_stage != GP_STAGE_EUL) return GP_E_STATE;
    run_prologue(s);
  }
  bool src_double = false;
  const void* src = field_ptr(s, field, &src_double);
  const bool dst_double = dtype == GP_FP64;
  const size_t nc = s->g.ncell;
  const bool mid = s->next_stage == GP_STAGE_LAG;
  const bool gas_mom = field >= GP_MX && field <= GP_MZ, bme_mom = field >= GP_QX && field <= GP_QZ;
  if (mid && (gas_mom || bme_mom)) {
    // between the stages the momentum slots hold velocities: return density * velocity
    const double* dens = s->dens[s->parity][gas_mom ? 0 : 1];
    void* out = on_device ? dst : s->staging;
    if (s->prec == GP_FP64) {
      if (dst_double) launch_density_times<double, double>((double*)out, dens, (const double*)src, nc, s->st);
      else launch_density_times<float, double>((float*)out, dens, (const double*)src, nc, s->st);
    } else {
      if (dst_double) launch_density_times<double, float>((double*)out, dens, (const float*)src, nc, s->st);
      else launch_density_times<float, float>((float*)out, dens, (const float*)src, nc, s->st);
    }
    if (!on_device)
      HIP_TRY(s, hipMemcpyAsync(dst, s->staging, nc * (dst_double ? 8 : 4), hipMemcpyDeviceToHost, s->st));
    HIP_TRY(s, hipStreamSynchronize(s->st));
  } else if (on_device) {
    convert_any(dst, dst_double, src, src_double, nc, s->st);
    HIP_TRY(s, hipStreamSynchronize(s->st));
  } else {
    const size_t bytes = nc * (dst_double ? sizeof(double) : sizeof(float));
    if (src_double == dst_double) {
      HIP_TRY(s, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s->st));
    } else {
      convert_any(s->staging, dst_double, src, src_double, nc, s->st);
      HIP_TRY(s, hipMemcpyAsync(dst, s->staging, bytes, hipMemcpyDeviceToHost, s->st));
    }
    HIP_TRY(s, hipStreamSynchronize(s->st));
  }
  HIP_TRY(s, hipGetLastError());
  return latched(s);
}

gp_status gp_step(gp_sim* s, int32_t nsteps) {
  if (!s || nsteps < 0) return GP_E_INVALID;
  if (s->next_stage != GP_STAGE_EUL) return GP_E_STATE;
  if (s->need_prologue) run_prologue(s);
  for (int t = 0; t < nsteps; t++) {
    if (s->use_graph) {
      if (!s->graph_ready[s->parity]) {
        gp_status r = build_graph(s, s->parity);
        if (r != GP_OK) return r;
      }
      HIP_TRY(s, hipGraphLaunch(s->gexec[s->parity], s->st));
      s->parity ^= 1;
    } else {
      run_step_direct(s, nullptr);
    }
  }
  HIP_TRY(s, hipGetLastError());
  return GP_OK;
}

gp_status gp_sync(gp_sim* s) {
  if (!s) return GP_E_INVALID;
  HIP_TRY(s, hipStreamSynchronize(s->st));
  return latched(s);
}

gp_status gp_get_diag(gp_sim* s, gp_diag* out, int32_t max, int32_t* count) {
  if (!s || !out || !count || max < 0) return GP_E_INVALID;
  if (s->need_prologue && s->next_stage == GP_STAGE_EUL) run_prologue(s);
  HIP_TRY(s, hipStreamSynchronize(s->st));
  DevScalars h{};
  HIP_TRY(s, hipMemcpy(&h, s->sc, sizeof(h), hipMemcpyDeviceToHost));
  const int avail = (int)std::min<uint32_t>(h.ndiag, (uint32_t)kDiagCap);
  const int n = std::min(avail, (int)max);
  std::vector<gp_diag> all(kDiagCap);
  HIP_TRY(s, hipMemcpy(all.data(), s->ring, sizeof(gp_diag) * kDiagCap, hipMemcpyDeviceToHost));
  for (int t = 0; t < n; t++) out[t] = all[(h.ndiag - n + t) % kDiagCap];
  *count = n;
  return GP_OK;
}

gp_status gp_set_time(gp_sim* s, double t, int64_t step) {
  if (!s) return GP_E_INVALID;
  if (s->next_stage != GP_STAGE_EUL) return GP_E_STATE;
  HIP_TRY(s, hipStreamSynchronize(s->st));
  DevScalars h{};
  HIP_TRY(s, hipMemcpy(&h, s->sc, sizeof(h), hipMemcpyDeviceToHost));
  h.t = t;
  h.step = step;
  HIP_TRY(s, hipMemcpy(s->sc, &h, sizeof(h), hipMemcpyHostToDevice));
  s->need_prologue = true;
  return GP_OK;
}

gp_status gp_get_time(gp_sim* s, double* t, double* dt, int64_t* step) {
  if (!s) return GP_E_INVALID;
  if (s->need_prologue && s->next_stage == GP_STAGE_EUL) run_prologue(s);
  HIP_TRY(s, hipStreamSynchronize(s->st));
  DevScalars h{};
  HIP_TRY(s, hipMemcpy(&h, s->sc, sizeof(h), hipMemcpyDeviceToHost));
  if (t) *t = h.t;
  if (dt) *dt = h.dt;
  if (step) *step = h.step;
  return GP_OK;
}

gp_status gp_debug_stage(gp_sim* s, int32_t stage) {
  if (!s || stage < GP_STAGE_EUL || stage > GP_STAGE_FINALIZE) return GP_E_INVALID;
  if (s->need_prologue && s->next_stage == GP_STAGE_EUL) run_prologue(s);
  if (stage != s->next_stage) return GP_E_STATE;
  run_stage(s, stage, nullptr);
  s->next_stage = (stage + 1) % 4;
  HIP_TRY(s, hipGetLastError());
  return GP_OK;
}

gp_status gp_time_kernels(gp_sim* s, int32_t nsteps, double* ms, int32_t max) {
  if (!s || !ms || nsteps <= 0 || max < 0) return GP_E_INVALID;
  if (s->next_stage != GP_STAGE_EUL) return GP_E_STATE;
  if (s->need_prologue) run_prologue(s);
  Timer tm;
  tm.on = true;
  for (int k = 0; k < 2 * GP_NKERNELS; k++) HIP_TRY(s, hipEventCreate(&tm.ev[k]));
  for (int k = 0; k < GP_NKERNELS; k++) tm.acc[k] = 0.0;
  for (int t = 0; t < nsteps; t++) run_step_direct(s, &tm);
  for (int k = 0; k < 2 * GP_NKERNELS; k++) (void)hipEventDestroy(tm.ev[k]);
  for (int k = 0; k < std::min<int>(max, GP_NKERNELS); k++) ms[k] = tm.acc[k] / nsteps;
  HIP_TRY(s, hipGetLastError());
  return GP_OK;
}

gp_status gp_use_graph(gp_sim* s, int32_t enable) {
  if (!s) return GP_E_INVALID;
  s->use_graph = enable != 0;
  return GP_OK;
}

double gp_algorithmic_bytes_per_cell(const gp_sim* s, int32_t kernel) {
  if (!s) return 0.0;
  const double es = (double)esize(s->prec);
  const double vr = (double)(s->g.nx + 1) * (s->g.ny + 1) * (s->g.nz + 1) / (double)s->g.ncell;
  const double eul = 2 * 8.0 + 20 * es + es + 20 * es;  // read rho, n, 20 fields, Phi; write 20
  const double vtx = 6 * es + 6 * es * vr;              // read 6 velocities; write 6 per vertex
  const double lag = 2 * 8.0 + 20 * es + 6 * es * vr + 2 * 8.0 + 20 * es + es;  // read rho, n, 20, corners; write 22 + s
  switch (kernel) {
    case GP_K_EUL: return eul;
    case GP_K_VERTEX: return vtx;
    case GP_K_LAG: return lag;
    case GP_K_FINALIZE: return 0.0;
    case -1: {
      double t = eul + vtx + lag;
      for (int k = GP_K_FFT_X_FWD; k <= GP_K_FFT_X_INV; k++) t += fft_bytes_per_cell(s, k);
      return t;
    }
    default: return fft_bytes_per_cell(s, kernel);
  }
}

}  // extern "C"
