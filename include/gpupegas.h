/*
 * gpupegas.h -- C ABI of the MI355X GPUPEGAS timestep library (libgpupegas.so).
 *
 * One simulation ("sim") advances a two-component self-gravitating system on
 * a uniform periodic-or-outflow 3D grid of cubic cells, following
 * I. Kulikov, "GPUPEGAS: a new GPU-accelerated hydrodynamical code for
 * numerical simulation of interacting galaxies" (arXiv:1311.0861):
 *   - gas: density rho, momentum rho v, total energy rho E, internal energy
 *     rho eps, with p = (gamma - 1) rho eps (Sec. 2, gas system and EOS);
 *   - stars/dark matter as Boltzmann moment equations: density n, momentum
 *     n u, symmetric stress Pi_ij and energy tensor n E_ij = Pi_ij + n u_i u_j
 *     (Sec. 2, moment system);
 *   - gravity from Laplace(Phi) = 4 pi G (rho + n) (Sec. 2.3).
 * One step = Eulerian stage (Sec. 2.1, 2.2: closed-form interface states,
 * gravity sources) -> Lagrangian FlIC flux stage (Sec. 2.1) -> energy balance
 * and correctness integrals (Sec. 2.4) -> FFT Poisson with the 27-point symbol
 * (Sec. 2.3) -> CFL step and diagnostics, all on the GPU; the host only
 * enqueues work.
 *
 * Conventions
 *   - Every call returns a gp_status; GP_OK is 0, errors are negative.
 *   - Arrays are dense nx*ny*nz, cell (i,j,k) at index i + nx*(j + ny*k)
 *     (x fastest).  Cell centres are lo + (i + 1/2) h; h must be equal on the
 *     three axes (the Poisson symbol has one h).
 *   - Host pointers (on_device = 0) are copied synchronously.  Device pointers
 *     (on_device = 1, e.g. a torch tensor's data_ptr()) are read/written in
 *     stream order on the sim's stream; the library never keeps a caller
 *     pointer after the call returns.
 *   - The library owns all device memory of a sim.  A sim is not thread-safe;
 *     different sims are independent.
 *   - Device-side failures (non-finite values, rho or n <= 0, p <= 0 or a
 *     diagonal stress <= 0) are latched on the device and returned by the next
 *     synchronising call (gp_sync, gp_get_*), never by gp_step itself.
 */
#ifndef GPUPEGAS_H
#define GPUPEGAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GP_OK = 0,
  GP_E_INVALID = -1,     /* bad argument or configuration                  */
  GP_E_NOMEM = -2,       /* device allocation failed                       */
  GP_E_HIP = -3,         /* HIP runtime error (see gp_last_error)          */
  GP_E_NONFINITE = -4,   /* NaN/Inf appeared in the state                  */
  GP_E_NONPOSITIVE = -5, /* rho, n, p or a diagonal stress became <= 0     */
  GP_E_UNSUPPORTED = -6, /* valid request this build does not implement    */
  GP_E_STATE = -7        /* call out of order (e.g. stages out of sequence) */
} gp_status;

enum { GP_BC_OUTFLOW = 0, GP_BC_PERIODIC = 1 };
/* Boundary of the potential.  Periodic: the FFT solve of the 27-point
 * Poisson equation with its printed Fourier symbol (Sec. 2.3), zero-mean
 * potential.  Isolated: the free-space potential of the cell masses, sum over
 * cells of -G m / r with the cell's own term taken as a uniform cube, by zero
 * padding to twice the grid on each axis (Hockney and Eastwood's method,
 * which Sec. 1 cites among the Poisson solvers of other codes); the gravity
 * of the outermost cells then reads the potential on a one-cell ring outside
 * the grid, which the solve also delivers. */
enum { GP_POISSON_PERIODIC = 0, GP_POISSON_ISOLATED = 1 };
enum { GP_FP64 = 0, GP_FP32 = 1 };

/* State fields, in this order.  GP_PHI (the potential) is read-only. */
enum {
  GP_RHO = 0, GP_MX, GP_MY, GP_MZ, GP_E, GP_EINT,
  GP_N, GP_QX, GP_QY, GP_QZ,
  GP_PXX, GP_PXY, GP_PXZ, GP_PYY, GP_PYZ, GP_PZZ,
  GP_WXX, GP_WXY, GP_WXZ, GP_WYY, GP_WYZ, GP_WZZ,
  GP_NFIELDS = 22,
  GP_PHI = 22
};

/* Stages of one step, for gp_debug_stage, in the order they must run. */
enum { GP_STAGE_EUL = 0, GP_STAGE_LAG = 1, GP_STAGE_POISSON = 2, GP_STAGE_FINALIZE = 3 };

/* Kernels timed by gp_time_kernels.  The Eulerian and Lagrangian stages run
 * one kernel per component: the gas (rho, m, E, e) and the stars / dark
 * matter (n, q, Pi, W), which those stages never couple.  The Poisson solve
 * is three passes over the half spectrum: the x and y transforms (one kernel
 * over the even and odd rows of each z plane where two such half planes fit
 * in a CU's LDS, else an x and a y kernel, timed together), the z transforms
 * with the symbol (whose launch also reduces the
 * per-tile partial sums of the step), and the inverse x and y (whose launch
 * also finishes the step: CFL step, time advance, diagnostics record).
 * GP_K_FINALIZE times the finalize where it runs on its own: without
 * gravity, and stage by stage (gp_debug_stage). */
enum {
  GP_K_EUL_GAS = 0, GP_K_EUL_BME, GP_K_LAG_GAS, GP_K_LAG_BME, GP_K_FFT_XY_FWD,
  GP_K_FFT_Z, GP_K_FFT_XY_INV, GP_K_FINALIZE, GP_NKERNELS
};

typedef struct {
  int32_t n[3];      /* cells per axis; >= 4.  With G != 0 each must be even and
                        of the form 2^a 3^b (FFT lengths)                    */
  int32_t bc[3];     /* GP_BC_OUTFLOW (clamped, zero-gradient) or GP_BC_PERIODIC
                        for the hydrodynamics; the potential has its own     */
  double lo[3], hi[3];
  double gamma;      /* adiabatic index, > 1                                 */
  double G;          /* gravitational constant; 0 switches gravity off       */
  double cfl;        /* Courant number C: tau = C h / max signal speed       */
  double eta;        /* energy-balance threshold; < 0 switches it off        */
  double fixed_dt;   /* > 0: constant step instead of the CFL step           */
  double t_end;      /* > 0: the step is clipped so that t never exceeds it  */
  int32_t precision; /* GP_FP64, or GP_FP32 (rho and n stay FP64; CFL, sums
                        and the Poisson zero mode stay FP64)                  */
  int32_t poisson;   /* GP_POISSON_PERIODIC (0) or GP_POISSON_ISOLATED        */
  /* Cooling q of the gas energy equations (Sec. 2; applied in the Eulerian
   * stage, Sec. 2.1, to rho E and rho eps alike, from the state at t^n).  The
   * paper tabulates q (Sutherland and Dopita); this library takes the
   * power-law stand-in q = cool_lambda rho^2 theta^cool_alpha for
   * theta = p / rho > cool_theta_min, and q = 0 at or below it.
   * cool_lambda = 0 switches cooling off.  The step is not limited by the
   * cooling time: a tau q above rho eps latches GP_E_NONPOSITIVE. */
  double cool_lambda;    /* >= 0                                               */
  double cool_alpha;     /* any finite exponent                                */
  double cool_theta_min; /* >= 0                                               */
  /* Uniform external gravitational acceleration, added to the self-gravity
   * -grad Phi in the Eulerian sources of both components (the free fall g of
   * the Rayleigh-Taylor test of Sec. 4.4); zeros for none. */
  double gext[3];
} gp_config;

/* One diagnostics record per step (and one for the initial state).  Sums are
 * h^3-weighted over the grid, accumulated in FP64 in a fixed order. */
typedef struct {
  int64_t step;
  double t;
  double dt;          /* the step the next update will use                   */
  double mass_gas, mass_bme;
  double mom[3];      /* total momentum, gas + stars                          */
  double e_gas;       /* sum of rho E                                         */
  double e_bme;       /* sum of tr(n E_ij) / 2                                */
  double e_pot;       /* (1/2) sum (rho + n) Phi                              */
  double kappa_gas;   /* Sec. 2.4 integral, measured before energy balance    */
  double kappa_bme;
  double outflow_gas; /* cumulative mass that left through outflow faces      */
  double outflow_bme;
  double n_sync_gas;  /* cells whose internal energy was re-synchronised      */
  double n_sync_bme;  /* cells with at least one re-synchronised stress       */
  uint32_t err;       /* latched device error bits up to this record          */
  uint32_t pad;
} gp_diag;

typedef struct gp_sim gp_sim;

/* Create a sim on the uniform grid of Sec. 2 (x_i = i h per axis; here cell
 * centres lo + (i + 1/2) h) with the parameters gamma (gas EOS, Sec. 2) and G
 * (Poisson equation, Sec. 2 and 2.3).  hip_stream: a hipStream_t to run on,
 * or NULL for a stream the sim creates and owns.  On success *out receives
 * the handle, which the caller releases with gp_destroy; on failure *out is
 * NULL and nothing is allocated.  Returns GP_E_INVALID for a bad config
 * (h not equal on all axes, n < 4, gamma <= 1, cfl <= 0, poisson not one
 * of GP_POISSON_*), GP_E_UNSUPPORTED for FFT lengths the kernels do not
 * handle (with G != 0 every n must be even and 2^a 3^b), GP_E_NOMEM, GP_E_HIP.
 * With isolated boundaries and G != 0 the sim also computes the DFT of the
 * sampled Green function of its padded grid here (once, on the GPU). */
gp_status gp_create(const gp_config *cfg, void *hip_stream, gp_sim **out);
/* Wait for the sim's stream, free its device memory (and its stream if it
 * created it).  GP_E_INVALID for NULL. */
gp_status gp_destroy(gp_sim *sim);

/* Copy one state field in (set) or out (get): the conserved variables of the
 * gas system (rho, rho v, rho E, rho eps; Sec. 2) and of the moment system
 * (n, n u, Pi_ij, n E_ij; Sec. 2), ids GP_RHO .. GP_WZZ.  src / dst hold
 * nx*ny*nz values of the caller's type dtype (GP_FP64 or GP_FP32), x fastest;
 * values convert to the sim's storage type.  The library reads or writes the
 * caller's buffer only during the call (device buffers: in stream order on
 * the sim's stream) and never keeps the pointer.  Setting any field
 * invalidates Phi and tau; they are recomputed from the state by the next
 * gp_step, gp_debug_stage, gp_get_potential or gp_get_field(GP_PHI).
 * gp_get_field also takes GP_PHI (as gp_get_potential).  GP_E_INVALID for a
 * bad id, dtype or NULL pointer; GP_E_STATE for a set between the stages of
 * gp_debug_stage; gp_get_field returns the latched device status as
 * gp_sync does, after the copy. */
gp_status gp_set_field(gp_sim *sim, int32_t field, const void *src, int32_t dtype,
                       int32_t on_device);
gp_status gp_get_field(gp_sim *sim, int32_t field, void *dst, int32_t dtype,
                       int32_t on_device);

/* Potential Phi of the current state, nx*ny*nz values of type dtype into dst
 * (host or device as on_device says): with GP_POISSON_PERIODIC the solution
 * of Laplace(Phi) = 4 pi G (rho + n) on the 27-point stencil by FFT on the
 * periodic grid with the zero mode removed (Sec. 2.3); with
 * GP_POISSON_ISOLATED the free-space potential of the cell masses (see
 * GP_POISSON_ISOLATED; the ring outside the grid is not returned).  Computed first if the state was set since the
 * last step.  Returns the latched device status after the copy, as
 * gp_get_field. */
gp_status gp_get_potential(gp_sim *sim, void *dst, int32_t dtype, int32_t on_device);

/* Enqueue nsteps full steps (asynchronous): each step is the Eulerian stage
 * (Sec. 2.1 gas, Sec. 2.2 stars / dark matter), the Lagrangian FlIC stage
 * (Sec. 2.1), the energy balance and correctness integrals (Sec. 2.4), the
 * FFT Poisson solve (Sec. 2.3), and the CFL step (not in the paper: tau =
 * C h / max signal speed) with the diagnostics record.  Argument errors
 * (nsteps < 0: GP_E_INVALID; mid-way through gp_debug_stage: GP_E_STATE)
 * return at once; device errors are latched for the next synchronising
 * call. */
gp_status gp_step(gp_sim *sim, int32_t nsteps);

/* Wait for the sim's stream; returns the latched device error, if any. */
gp_status gp_sync(gp_sim *sim);

/* Copy the most recent min(max, available) diagnostics records (the
 * conservation sums and the Sec. 2.4 correctness integrals kappa of each
 * step), oldest first, into out[0 .. *count - 1].  The device keeps the last
 * 4096 records.  Synchronises, and returns the latched device status as
 * gp_sync does: the records are delivered either way, and each record's err
 * bits say from which step on an error was latched. */
gp_status gp_get_diag(gp_sim *sim, gp_diag *out, int32_t max, int32_t *count);

/* Set (t, step) of the current state, e.g. when resuming from saved fields;
 * tau is recomputed from the state.  gp_get_time returns the time, the step
 * the next update will use and the step count (NULL outputs are skipped). */
gp_status gp_set_time(gp_sim *sim, double t, int64_t step);
gp_status gp_get_time(gp_sim *sim, double *t, double *dt, int64_t *step);

/* Run one stage of a step (GP_STAGE_*: Eulerian, Sec. 2.1 and 2.2;
 * Lagrangian with the Sec. 2.4 balance; Poisson, Sec. 2.3; finalize: CFL step
 * and diagnostics), in order, for per-stage checks.  Between GP_STAGE_EUL and
 * GP_STAGE_LAG, gp_get_field returns the post-Eulerian fields.  GP_E_STATE if
 * called out of order. */
gp_status gp_debug_stage(gp_sim *sim, int32_t stage);

/* Run nsteps steps kernel by kernel with HIP events around every launch and
 * return the mean duration in milliseconds of each GP_K_* kernel in ms[0..]
 * (max entries).  Every kernel runs once, in the order of a step, so that it
 * finds its inputs where a step leaves them; the host waits for each event,
 * so the kernels do not overlap.  The state advances as with gp_step. */
gp_status gp_time_kernels(gp_sim *sim, int32_t nsteps, double *ms, int32_t max);

/* Use a captured HIP graph per step (default on).  Results are identical. */
gp_status gp_use_graph(gp_sim *sim, int32_t enable);

/* Launch configuration of a per-cell kernel (GP_K_EUL_GAS, GP_K_EUL_BME,
 * GP_K_LAG_GAS or GP_K_LAG_BME): the work is a list of (run, tile column,
 * chunk of z planes) items walked by a persistent grid of workgroups.  The
 * autotuner picks, during the first step, the tile shape (0: 64 x 4 cells,
 * 1: 32 x 8), the z-chunk cap (8, 16, 32 or 64 planes; an item reads the plane
 * below and above its chunk as its z halo) and the grid size (one workgroup
 * per item, or 8192 / 4096 / 2048 / 1024), each kernel by its own timing.
 * With the environment variable GPUPEGAS_TUNE_CACHE naming a file when the
 * sim is created, the picks are read from it (keyed by device architecture,
 * precision, cooling and the grid sizes of the batch) instead of tuning, and
 * written to it after tuning.  gp_set_launch fixes the grid size of the
 * current tiling (0 = one workgroup per item), gp_set_tiling the tile shape
 * and chunk cap (GP_E_INVALID for other values; GP_E_STATE between the
 * stages of gp_debug_stage); either disables the tuning.  The state, the
 * potential and the step never depend on them; the diagnostics sums are
 * summed over the items, so they match to rounding across tilings. */
gp_status gp_set_launch(gp_sim *sim, int32_t kernel, int32_t blocks);
gp_status gp_get_launch(gp_sim *sim, int32_t kernel, int32_t *blocks);
gp_status gp_set_tiling(gp_sim *sim, int32_t kernel, int32_t shape, int32_t cap_planes);
gp_status gp_get_tiling(gp_sim *sim, int32_t kernel, int32_t *shape, int32_t *cap_planes);

/* Form of the x and y transforms of the Poisson solve: GP_FFT_AUTO (one
 * workgroup per z plane and row parity wherever two such half planes of the
 * half spectrum fit in a CU's LDS, the z pass joining the two halves of the
 * y transform; else separate x and y passes) or GP_FFT_LINES (always the
 * separate passes).  Both compute the same transform, equal to rounding. */
enum { GP_FFT_AUTO = 0, GP_FFT_LINES = 1 };
gp_status gp_set_fft_form(gp_sim *sim, int32_t form);

const char *gp_status_str(gp_status s);
/* Text of the last error a sim recorded (HIP call and message, or the run
 * whose configuration was refused).  With sim = NULL: why the calling
 * thread's last failed gp_create or gp_batch_create failed.  The string is
 * owned by the library and valid until the next call on the same sim (or,
 * for NULL, the thread's next failed create). */
const char *gp_last_error(const gp_sim *sim);

/* ---- Ensembles --------------------------------------------------------------
 * A batch advances nruns independent runs (grids of any supported sizes, one
 * shared precision) in lockstep: each stage is one launch over all runs (the
 * Poisson passes one launch per distinct grid size), and each step is one
 * graph replay.  Every run keeps its own tau, time, diagnostics and error bits,
 * and evolves exactly as it would in its own gp_sim.  Fields, diagnostics and
 * errors are addressed by run index 0..nruns-1; other conventions are those of
 * the single-run calls above.  gp_batch_sync returns an error latched by any
 * run; gp_batch_get_field, gp_batch_get_potential and gp_batch_get_diag
 * return the one latched by that run. */
typedef struct gp_batch gp_batch;

gp_status gp_batch_create(const gp_config *cfgs, int32_t nruns, void *hip_stream, gp_batch **out);
gp_status gp_batch_destroy(gp_batch *b);
gp_status gp_batch_set_field(gp_batch *b, int32_t run, int32_t field, const void *src, int32_t dtype,
                             int32_t on_device);
gp_status gp_batch_get_field(gp_batch *b, int32_t run, int32_t field, void *dst, int32_t dtype,
                             int32_t on_device);
gp_status gp_batch_get_potential(gp_batch *b, int32_t run, void *dst, int32_t dtype, int32_t on_device);
gp_status gp_batch_step(gp_batch *b, int32_t nsteps);
gp_status gp_batch_sync(gp_batch *b);
gp_status gp_batch_get_diag(gp_batch *b, int32_t run, gp_diag *out, int32_t max, int32_t *count);
gp_status gp_batch_time_kernels(gp_batch *b, int32_t nsteps, double *ms, int32_t max);
gp_status gp_batch_set_launch(gp_batch *b, int32_t kernel, int32_t blocks);
gp_status gp_batch_get_launch(gp_batch *b, int32_t kernel, int32_t *blocks);
gp_status gp_batch_set_tiling(gp_batch *b, int32_t kernel, int32_t shape, int32_t cap_planes);
gp_status gp_batch_get_tiling(gp_batch *b, int32_t kernel, int32_t *shape, int32_t *cap_planes);
gp_status gp_batch_set_fft_form(gp_batch *b, int32_t form);
double gp_batch_algorithmic_bytes_per_cell(const gp_batch *b, int32_t kernel);
int64_t gp_batch_cells(const gp_batch *b);  /* total cells over all runs */
const char *gp_batch_last_error(const gp_batch *b);  /* b = NULL: as gp_last_error(NULL) */

/* Bytes the kernels move per cell per step by design (reads + writes of the
 * state, potential and spectrum), for the roofline; see the source for the
 * per-kernel split.  kernel = GP_K_* or -1 for the whole step. */
double gp_algorithmic_bytes_per_cell(const gp_sim *sim, int32_t kernel);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * periodic potential gp_get_potential returns (the same Poisson kernels), of
 * densities the caller holds, with no device allocation and no sim.
 *   cfg      grid (n, lo, hi; cubic cells), G != 0, precision (the type of
 *            phi: double for GP_FP64, float for GP_FP32), poisson must be
 *            GP_POISSON_PERIODIC; the other fields are not used.
 *   rho, n   device pointers, nx*ny*nz FP64 values each, x fastest (read).
 *   phi      device pointer, nx*ny*nz values of the working type (written).
 *   hip_stream  a hipStream_t, or NULL for the null stream; the call only
 *            enqueues kernels there (no copy, memset or host wait), so it can
 *            be captured.  The caller owns every buffer.
 * The spectrum, tables and partial sums live in a fixed workspace of 64 MiB
 * per GPU (a static device array, held until the process ends): grids whose
 * workspace exceeds it -- about px ny nz complex values plus small tables,
 * px = nx/2 + 1: cubic grids up to 192^3 in FP64 or 216^3 in FP32 -- return
 * GP_E_UNSUPPORTED before anything is enqueued, as do isolated boundaries
 * and FFT lengths other than even 2^a 3^b.  GP_E_INVALID for NULL pointers
 * or a bad config; GP_E_HIP for a launch failure.  All calls on one GPU share
 * its workspace: calls that overlap there (other streams or host threads)
 * race; calls ordered on one stream do not. */
gp_status gp_potential_noalloc(const gp_config *cfg, const double *rho, const double *n, void *phi,
                               void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GPUPEGAS_H */
