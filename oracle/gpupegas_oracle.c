/*
 * gpupegas_oracle.c -- plain, slow, FP64 CPU oracle of one GPUPEGAS timestep.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the GPU smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no source,
 * header, table or helper with the GPU path, and the GPU path never calls it.
 *
 * Method: I. Kulikov, "GPUPEGAS: a new GPU-accelerated hydrodynamical code for
 * numerical simulation of interacting galaxies", arXiv:1311.0861.
 *   gas dynamics with gravity ................. Sec. 2 (gas system, EOS)
 *   Boltzmann moment equations (BME) .......... Sec. 2 (moment system)
 *   uniform grid .............................. Sec. 2 (grid definition)
 *   Eulerian stage, gas face state (V, P) ..... Sec. 2.1 (closed-form solution)
 *   Lagrangian (FlIC) stage flux .............. Sec. 2.1 (flux F_{i+1/2,kl}, Fig. "lagrange")
 *   Eulerian stage, BME face state ............ Sec. 2.2 (closed-form solution)
 *   Poisson by FFT, 27-point symbol ........... Sec. 2.3
 *   isolated Poisson boundaries ............... zero-padded convolution with
 *       the sampled point-mass potential (Hockney and Eastwood, whose method
 *       Sec. 1 cites among the Poisson solvers of other codes)
 *   correctness integrals kappa ............... Sec. 2.4
 *
 * Where the paper is silent the oracle takes these readings (each is also
 * noted at the function that uses it):
 *   - cell-centred cubic cells, x_i = lo + (i + 1/2) h, h equal on all axes;
 *   - piecewise-constant face states (first-order Godunov), unsplit: all three
 *     axes are updated from the same state; all Eulerian right-hand sides use
 *     U^n and Phi^n;
 *   - Eulerian update = non-advective right-hand side of each equation of
 *     Sec. 2 with face values in the divergences, gravity g = central
 *     difference of Phi (periodic wrap);
 *   - Lagrangian corner velocities = mean of the 8 cells sharing the vertex,
 *     advecting velocity = post-Eulerian m'/rho (gas), q'/n (BME);
 *   - Poisson symbol carries a minus sign and the factor G; the k = 0 mode
 *     is zero (periodic, zero-mean potential);
 *   - energy balance: dual-energy synchronisation with threshold eta, applied
 *     after kappa is measured; CFL step C h / max signal speed.
 *   - hydrodynamic boundaries: outflow = clamped (zero-gradient) index,
 *     periodic = wrapped index.  A periodic Phi wraps; an isolated Phi is
 *     evaluated on a one-cell ring outside the grid as well, and the gravity
 *     of the outermost cells takes its values there.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NF 22           /* state fields */
#define ID_PHI 22       /* read-only potential */
#define DIAG_LEN 18

enum {
  RHO = 0, MX, MY, MZ, EN, EI,        /* gas: rho, rho v, rho E, rho eps      */
  NB, QX, QY, QZ,                     /* BME: n, n u                          */
  PXX, PXY, PXZ, PYY, PYZ, PZZ,       /* BME: Pi_ij (symmetric)               */
  WXX, WXY, WXZ, WYY, WYZ, WZZ        /* BME: n E_ij = Pi_ij + n u_i u_j      */
};

enum { ST_EUL = 0, ST_LAG = 1, ST_POISSON = 2, ST_FINALIZE = 3 };

enum {
  ERR_NONFINITE = 1u, ERR_DENSITY = 2u, ERR_PRESSURE = 4u, ERR_STRESS = 8u,
  ERR_NOSPEED = 16u
};

/* position of Pi_ij / W_ij inside the 6-slot symmetric storage xx,xy,xz,yy,yz,zz */
static const int SYM[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

typedef struct {
  int32_t n[3];       /* cells per axis                                      */
  int32_t bc[3];      /* 0 = outflow, 1 = periodic                            */
  double lo[3], hi[3];
  double gamma;       /* adiabatic index                                     */
  double G;           /* gravitational constant (0 disables gravity)         */
  double cfl;         /* Courant number                                      */
  double eta;         /* energy-balance threshold (negative disables)        */
  double fixed_dt;    /* > 0: use this step instead of the CFL step          */
  double t_end;       /* > 0: never step past this time                      */
  int32_t poisson;    /* 0 = periodic (Sec. 2.3), 1 = isolated               */
  double cool_lambda; /* cooling q = lambda rho^2 theta^alpha, theta = p/rho   */
  double cool_alpha;  /*   (0 switches cooling off)                           */
  double cool_theta_min; /* no cooling at or below this theta                 */
  double gext[3];     /* uniform external gravitational acceleration          */
} orc_config;

typedef struct {
  orc_config c;
  int nx, ny, nz;
  size_t ncell;
  double h;
  double *f[NF];       /* current state                                      */
  double *old[NF];     /* state at the start of the running stage            */
  double *vel[6];      /* cell velocities v'(3), u'(3) for the FlIC stage    */
  double *vtx[6];      /* corner velocities, (nx+1)(ny+1)(nz+1) each         */
  double *phi, *s;
  double *phi_ext;     /* isolated: Phi on the grid and a one-cell ring       */
  double *ghat;        /* isolated: spectrum of the padded Green function      */
  double t, dt;
  int64_t step;
  int need_prologue;
  int next_stage;
  uint32_t err;
  double outflow_gas, outflow_bme;              /* cumulative                */
  double kappa_gas, kappa_bme, nsync_gas, nsync_bme;   /* from the last FlIC stage */
  double *diag;
  size_t ndiag, cap;
} orc_sim;

/* ------------------------------------------------------------------------- */
/* indexing and boundary rule                                                */

static inline size_t cidx(const orc_sim *s, int i, int j, int k) {
  return (size_t)i + (size_t)s->nx * ((size_t)j + (size_t)s->ny * (size_t)k);
}

static inline int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

/* hydrodynamic boundary rule: outflow clamps (zero gradient), periodic wraps */
static inline int bcix(int i, int n, int bc) {
  if (bc == 1) return wrap(i, n);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

static size_t nbr(const orc_sim *s, int i, int j, int k, int d, int o) {
  int c[3] = {i, j, k};
  const int n[3] = {s->nx, s->ny, s->nz};
  c[d] = bcix(c[d] + o, n[d], s->c.bc[d]);
  return cidx(s, c[0], c[1], c[2]);
}

/* cell (i, j, k) + o e_d of the isolated potential's extended grid, which
 * holds the cells -1 .. n on each axis */
static size_t ext_nbr(const orc_sim *s, int i, int j, int k, int d, int o) {
  int c[3] = {i + 1, j + 1, k + 1};
  c[d] += o;
  return (size_t)c[0] + (size_t)(s->nx + 2) * ((size_t)c[1] + (size_t)(s->ny + 2) * (size_t)c[2]);
}

static size_t nbr_wrap(const orc_sim *s, int i, int j, int k, int d, int o) {
  int c[3] = {i, j, k};
  const int n[3] = {s->nx, s->ny, s->nz};
  c[d] = wrap(c[d] + o, n[d]);
  return cidx(s, c[0], c[1], c[2]);
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.1: interface velocity V and pressure P, the exact solution of the
 * linearised Eulerian-stage gas system for left/right states (rho, v, p),
 * v being the velocity component normal to the face. */
void orc_riemann_gas(double rl, double vl, double pl, double rr, double vr,
                     double pr, double gamma, double *V, double *P) {
  *V = 0.5 * (vl + vr) +
       0.5 * (pl - pr) * sqrt((rl + rr) / (rl * rr * gamma * (pl + pr)));
  *P = 0.5 * (pl + pr) +
       0.5 * (vl - vr) * sqrt(rl * rr * gamma * (pl + pr) / (rl + rr));
}

/* Sec. 2.2: interface state of the linearised Eulerian-stage BME system for a
 * face with normal axis d.  The paper prints the x-normal case; for normal d
 * the transverse axes a, b take the roles of y, z.  Bracketed coefficients use
 * the arithmetic mean of the left and right n, Pi_dd, Pi_da, Pi_db.
 * Inputs are n, u (3 lab components), Pi (6 symmetric slots) on each side.
 * Outputs: ustar[i] = u*_i and pstar[i] = Pi*_{d i} in lab components. */
void orc_riemann_bme(double nl, const double *ul, const double *pil, double nr,
                     const double *ur, const double *pir, int d, double *ustar,
                     double *pstar) {
  const int a = (d + 1) % 3, b = (d + 2) % 3;
  const double s3 = sqrt(3.0);
  const double nbar = 0.5 * (nl + nr);
  const double A = 0.5 * (pil[SYM[d][d]] + pir[SYM[d][d]]);
  const double B = 0.5 * (pil[SYM[d][a]] + pir[SYM[d][a]]);
  const double C = 0.5 * (pil[SYM[d][b]] + pir[SYM[d][b]]);
  const double dpdd = 0.5 * (pil[SYM[d][d]] - pir[SYM[d][d]]);
  const double dpda = 0.5 * (pil[SYM[d][a]] - pir[SYM[d][a]]);
  const double dpdb = 0.5 * (pil[SYM[d][b]] - pir[SYM[d][b]]);
  const double dud = 0.5 * (ul[d] - ur[d]);
  const double dua = 0.5 * (ul[a] - ur[a]);
  const double dub = 0.5 * (ul[b] - ur[b]);

  ustar[d] = 0.5 * (ul[d] + ur[d]) + dpdd * (1.0 / sqrt(3.0 * nbar * A));
  ustar[a] = 0.5 * (ul[a] + ur[a]) + dpda * (1.0 / sqrt(nbar * A)) +
             dpdd * (B * (1.0 - s3) / (A * sqrt(3.0 * nbar * A)));
  ustar[b] = 0.5 * (ul[b] + ur[b]) + dpdb * (1.0 / sqrt(nbar * A)) +
             dpdd * (C * (1.0 - s3) / (A * sqrt(3.0 * nbar * A)));
  pstar[d] = A + dud * sqrt(3.0 * nbar * A);
  pstar[a] = B + dua * sqrt(nbar * A) + dud * (B * nbar * (s3 - 1.0) / sqrt(nbar * A));
  pstar[b] = C + dub * sqrt(nbar * A) + dud * (C * nbar * (s3 - 1.0) / sqrt(nbar * A));
}

/* gas face between cells L and R (normal axis d), from the stage-start state */
static void gas_face(const orc_sim *s, size_t L, size_t R, int d, double *V,
                     double *P) {
  const double g = s->c.gamma;
  double rl = s->old[RHO][L], rr = s->old[RHO][R];
  double vl = s->old[MX + d][L] / rl, vr = s->old[MX + d][R] / rr;
  double pl = (g - 1.0) * s->old[EI][L], pr = (g - 1.0) * s->old[EI][R];
  orc_riemann_gas(rl, vl, pl, rr, vr, pr, g, V, P);
}

static void bme_face(const orc_sim *s, size_t L, size_t R, int d, double *us,
                     double *ps) {
  double nl = s->old[NB][L], nr = s->old[NB][R];
  double ul[3], ur[3], pl[6], pr[6];
  for (int i = 0; i < 3; i++) {
    ul[i] = s->old[QX + i][L] / nl;
    ur[i] = s->old[QX + i][R] / nr;
  }
  for (int m = 0; m < 6; m++) {
    pl[m] = s->old[PXX + m][L];
    pr[m] = s->old[PXX + m][R];
  }
  orc_riemann_bme(nl, ul, pl, nr, ur, pr, d, us, ps);
}

/* ------------------------------------------------------------------------- */
/* Eulerian stage (Sec. 2, 2.1, 2.2).  With the fluid frozen, each equation of
 * Sec. 2 keeps its non-advective right-hand side, with the divergence taken
 * from the face states of the Riemann solutions:
 *   gas:  m_i'  = m_i - tau/h d_i P - tau rho g_i
 *         E'    = E   - tau/h sum_d d_d(P V) - tau sum_d m_d g_d
 *         e'    = e   - tau/h (gamma-1) e sum_d d_d V
 *   BME:  q_i'  = q_i - tau/h sum_d d_d Pi*_{id} - tau n g_i
 *         W_ij' = W_ij - tau/h sum_d d_d(Pi*_{jd} u*_i + Pi*_{id} u*_j)
 *                      - tau (q_i g_j + q_j g_i)
 *         Pi_ij'= Pi_ij - tau/h sum_d (Pi_jd d_d u*_i + Pi_id d_d u*_j)
 * where d_d X = X(face c+1/2 e_d) - X(face c-1/2 e_d), g = grad Phi by central
 * difference; rho and n are unchanged.  The gas energy equations of Sec. 2
 * also lose the cooling function q, which Sec. 2.1 assigns to this stage:
 * E' and e' each take - tau q.  The paper's q is tabulated (Sutherland and
 * Dopita); the tables are not at hand, so q is a stand-in power law of the
 * density and theta = p / rho (proportional to the temperature):
 *   q = lambda rho^2 theta^alpha  for theta > theta_min,  0 otherwise,
 * evaluated from U^n like the other sources; lambda = 0 switches it off.
 * A uniform external gravitational acceleration gext (the free fall of the
 * Rayleigh-Taylor test of Sec. 4.4) adds to the self-gravity: the sources
 * above take g_d = d_d Phi - gext_d. */
static void stage_eulerian(orc_sim *s) {
  for (int q = 0; q < NF; q++) memcpy(s->old[q], s->f[q], s->ncell * sizeof(double));
  const double tau = s->dt, h = s->h, gam = s->c.gamma, r = tau / h;
  const int nx = s->nx, ny = s->ny, nz = s->nz;

#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        const size_t c = cidx(s, i, j, k);
        double grad[3];
        for (int d = 0; d < 3; d++)
          grad[d] = (s->c.poisson == 1
                         ? (s->phi_ext[ext_nbr(s, i, j, k, d, +1)] - s->phi_ext[ext_nbr(s, i, j, k, d, -1)]) / (2.0 * h)
                         : (s->phi[nbr_wrap(s, i, j, k, d, +1)] - s->phi[nbr_wrap(s, i, j, k, d, -1)]) / (2.0 * h)) -
                    s->c.gext[d];

        /* gas */
        double dP[3], dPV = 0.0, dV = 0.0;
        double usp[3][3], usm[3][3], psp[3][3], psm[3][3];
        for (int d = 0; d < 3; d++) {
          const size_t cm = nbr(s, i, j, k, d, -1), cp = nbr(s, i, j, k, d, +1);
          double Vm, Pm, Vp, Pp;
          gas_face(s, cm, c, d, &Vm, &Pm);
          gas_face(s, c, cp, d, &Vp, &Pp);
          dP[d] = Pp - Pm;
          dPV += Pp * Vp - Pm * Vm;
          dV += Vp - Vm;
          bme_face(s, cm, c, d, usm[d], psm[d]);
          bme_face(s, c, cp, d, usp[d], psp[d]);
        }
        const double rho = s->old[RHO][c];
        const double m[3] = {s->old[MX][c], s->old[MY][c], s->old[MZ][c]};
        for (int d = 0; d < 3; d++)
          s->f[MX + d][c] = m[d] - r * dP[d] - tau * rho * grad[d];
        double qc = 0.0;
        if (s->c.cool_lambda != 0.0) {
          const double theta = (gam - 1.0) * s->old[EI][c] / rho;
          if (theta > s->c.cool_theta_min) qc = s->c.cool_lambda * rho * rho * pow(theta, s->c.cool_alpha);
        }
        s->f[EN][c] = s->old[EN][c] - r * dPV -
                      tau * (m[0] * grad[0] + m[1] * grad[1] + m[2] * grad[2]) - tau * qc;
        s->f[EI][c] = s->old[EI][c] - r * (gam - 1.0) * s->old[EI][c] * dV - tau * qc;

        /* BME */
        const double n = s->old[NB][c];
        const double q[3] = {s->old[QX][c], s->old[QY][c], s->old[QZ][c]};
        for (int ii = 0; ii < 3; ii++) {
          double dq = 0.0;
          for (int d = 0; d < 3; d++) dq += psp[d][ii] - psm[d][ii];
          s->f[QX + ii][c] = q[ii] - r * dq - tau * n * grad[ii];
        }
        for (int ii = 0; ii < 3; ii++)
          for (int jj = ii; jj < 3; jj++) {
            const int m6 = SYM[ii][jj];
            double dW = 0.0, dPi = 0.0;
            for (int d = 0; d < 3; d++) {
              dW += (psp[d][jj] * usp[d][ii] + psp[d][ii] * usp[d][jj]) -
                    (psm[d][jj] * usm[d][ii] + psm[d][ii] * usm[d][jj]);
              dPi += s->old[PXX + SYM[jj][d]][c] * (usp[d][ii] - usm[d][ii]) +
                     s->old[PXX + SYM[ii][d]][c] * (usp[d][jj] - usm[d][jj]);
            }
            s->f[WXX + m6][c] = s->old[WXX + m6][c] - r * dW -
                                tau * (q[ii] * grad[jj] + q[jj] * grad[ii]);
            s->f[PXX + m6][c] = s->old[PXX + m6][c] - r * dPi;
          }
      }
}

/* ------------------------------------------------------------------------- */
/* Lagrangian (FlIC) stage, Sec. 2.1: every quantity f obeys
 *   (f^{n+1} - f^n)/tau + (F_{i+1/2} - F_{i-1/2})/h = 0   (summed over axes)
 * with the face flux F = (1/4) sum over the 4 face corners of v f^+, f^+ the
 * upwind cell value for that corner's velocity (rule of total deformation of
 * the cell).  Reading: a corner velocity is the mean of the 8 cells sharing the
 * vertex; the gas is advected by v' = m'/rho, the BME by u' = q'/n.  After the
 * update: the correctness integrals kappa (Sec. 2.4), the energy balance
 * (dual-energy synchronisation), the boundary outflow and s = rho + n. */
static size_t vidx(const orc_sim *s, int I, int J, int K) {
  return (size_t)I + (size_t)(s->nx + 1) * ((size_t)J + (size_t)(s->ny + 1) * (size_t)K);
}

static void stage_lagrangian(orc_sim *s) {
  for (int q = 0; q < NF; q++) memcpy(s->old[q], s->f[q], s->ncell * sizeof(double));
  const int nx = s->nx, ny = s->ny, nz = s->nz;
  const double tau = s->dt, h = s->h, r = tau / h;
  const double eta = s->c.eta;

  /* cell velocities after the Eulerian stage */
#pragma omp parallel for schedule(static)
  for (long c = 0; c < (long)s->ncell; c++) {
    for (int d = 0; d < 3; d++) {
      s->vel[d][c] = s->old[MX + d][c] / s->old[RHO][c];
      s->vel[3 + d][c] = s->old[QX + d][c] / s->old[NB][c];
    }
  }
  /* corner velocities: vertex (I,J,K) sits between cells I-1 and I on x, etc. */
#pragma omp parallel for schedule(static)
  for (int K = 0; K <= nz; K++)
    for (int J = 0; J <= ny; J++)
      for (int I = 0; I <= nx; I++) {
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int c3 = 0; c3 < 2; c3++)
          for (int b3 = 0; b3 < 2; b3++)
            for (int a3 = 0; a3 < 2; a3++) {
              const size_t cc = cidx(s, bcix(I - 1 + a3, nx, s->c.bc[0]),
                                     bcix(J - 1 + b3, ny, s->c.bc[1]),
                                     bcix(K - 1 + c3, nz, s->c.bc[2]));
              for (int v = 0; v < 6; v++) acc[v] += s->vel[v][cc];
            }
        const size_t w = vidx(s, I, J, K);
        for (int v = 0; v < 6; v++) s->vtx[v][w] = acc[v] / 8.0;
      }

  double *kg = calloc((size_t)nz, sizeof(double)), *kb = calloc((size_t)nz, sizeof(double));
  double *sg = calloc((size_t)nz, sizeof(double)), *sb = calloc((size_t)nz, sizeof(double));
  double *og = calloc((size_t)nz, sizeof(double)), *ob = calloc((size_t)nz, sizeof(double));

#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        const size_t c = cidx(s, i, j, k);
        const int ci[3] = {i, j, k};
        const int nn[3] = {nx, ny, nz};
        /* A+ and A- on the six faces for gas (comp 0) and BME (comp 1) */
        double Ap[2][3][2], Am[2][3][2]; /* [comp][axis][0: minus face, 1: plus face] */
        for (int d = 0; d < 3; d++) {
          const int a = (d + 1) % 3, b = (d + 2) % 3;
          for (int side = 0; side < 2; side++) {
            int V[3];
            V[d] = ci[d] + side; /* vertex index of the face plane */
            for (int comp = 0; comp < 2; comp++) {
              double pos = 0.0, neg = 0.0;
              for (int eb = 0; eb < 2; eb++)
                for (int ea = 0; ea < 2; ea++) {
                  V[a] = ci[a] + ea;
                  V[b] = ci[b] + eb;
                  const double vv = s->vtx[3 * comp + d][vidx(s, V[0], V[1], V[2])];
                  pos += vv > 0.0 ? vv : 0.0;
                  neg += vv < 0.0 ? vv : 0.0;
                }
              Ap[comp][d][side] = pos / 4.0;
              Am[comp][d][side] = neg / 4.0;
            }
          }
        }
        double outg = 0.0, outb = 0.0;
        for (int q = 0; q < NF; q++) {
          const int comp = q < NB ? 0 : 1;
          double div = 0.0;
          for (int d = 0; d < 3; d++) {
            const size_t cm = nbr(s, i, j, k, d, -1), cp = nbr(s, i, j, k, d, +1);
            const double Fp = Ap[comp][d][1] * s->old[q][c] + Am[comp][d][1] * s->old[q][cp];
            const double Fm = Ap[comp][d][0] * s->old[q][cm] + Am[comp][d][0] * s->old[q][c];
            div += Fp - Fm;
            if (q == RHO || q == NB) {
              double out = 0.0;
              if (s->c.bc[d] == 0 && ci[d] == nn[d] - 1) out += Fp;
              if (s->c.bc[d] == 0 && ci[d] == 0) out -= Fm;
              if (q == RHO) outg += out; else outb += out;
            }
          }
          s->f[q][c] = s->old[q][c] - r * div;
        }
        og[k] += outg;
        ob[k] += outb;

        /* Sec. 2.4 correctness integrals on the advected state */
        const double rho = s->f[RHO][c], n = s->f[NB][c];
        const double m[3] = {s->f[MX][c], s->f[MY][c], s->f[MZ][c]};
        const double q3[3] = {s->f[QX][c], s->f[QY][c], s->f[QZ][c]};
        const double ekin = (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / (2.0 * rho);
        kg[k] += fabs(s->f[EN][c] - s->f[EI][c] - ekin);
        double T[6];
        for (int ii = 0; ii < 3; ii++)
          for (int jj = ii; jj < 3; jj++) {
            const int m6 = SYM[ii][jj];
            T[m6] = s->f[WXX + m6][c] - q3[ii] * q3[jj] / n;
            kb[k] += fabs(T[m6] - s->f[PXX + m6][c]);
          }
        /* energy balance: dual-energy synchronisation */
        if (eta >= 0.0) {
          const double et = s->f[EN][c] - ekin;
          if (et > eta * s->f[EN][c]) {
            s->f[EI][c] = et;
            sg[k] += 1.0;
          }
          /* BME: the energy tr W / 2 lives on the diagonal, so each diagonal
             stress is synchronised on its own; off-diagonal stresses keep
             their evolution equation */
          int synced = 0;
          for (int d = 0; d < 3; d++) {
            const int m6 = SYM[d][d];
            if (T[m6] > eta * s->f[WXX + m6][c]) {
              s->f[PXX + m6][c] = T[m6];
              synced = 1;
            }
          }
          sb[k] += synced ? 1.0 : 0.0;
        }
        s->s[c] = s->f[RHO][c] + s->f[NB][c];
      }
  double Kg = 0, Kb = 0, Sg = 0, Sb = 0, Og = 0, Ob = 0;
  for (int k = 0; k < nz; k++) {
    Kg += kg[k]; Kb += kb[k]; Sg += sg[k]; Sb += sb[k]; Og += og[k]; Ob += ob[k];
  }
  const double h3 = h * h * h;
  s->kappa_gas = h3 * Kg;
  s->kappa_bme = h3 * Kb;
  s->nsync_gas = Sg;
  s->nsync_bme = Sb;
  s->outflow_gas += tau * h * h * Og;
  s->outflow_bme += tau * h * h * Ob;
  free(kg); free(kb); free(sg); free(sb); free(og); free(ob);
}

/* ------------------------------------------------------------------------- */
/* FFT: recursive mixed-radix (2, 3) decimation in time,
 *   X[k] = sum_m x[m] exp(sign 2 pi i m k / n).
 * tw holds exp(sign 2 pi i e / n0) for e in [0, n0); a sub-problem of length n
 * reads it with stride n0/n. */
static int fft_len_ok(int n) {
  if (n < 1) return 0;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

static void fft_rec(int n, const double *xr, const double *xi, int stride,
                    double *yr, double *yi, const double *twr, const double *twi,
                    int tstride) {
  if (n == 1) {
    yr[0] = xr[0];
    yi[0] = xi[0];
    return;
  }
  const int r = (n % 2 == 0) ? 2 : 3;
  const int m = n / r;
  for (int q = 0; q < r; q++)
    fft_rec(m, xr + (size_t)q * stride, xi + (size_t)q * stride, stride * r,
            yr + (size_t)q * m, yi + (size_t)q * m, twr, twi, tstride * r);
  for (int k = 0; k < m; k++) {
    double ar[3], ai[3];
    for (int q = 0; q < r; q++) {
      ar[q] = yr[(size_t)q * m + k];
      ai[q] = yi[(size_t)q * m + k];
    }
    for (int p = 0; p < r; p++) {
      double sr = 0.0, si = 0.0;
      for (int q = 0; q < r; q++) {
        const int e = (int)(((long)q * (k + (long)p * m)) % n);
        const double wr = twr[(size_t)e * tstride], wi = twi[(size_t)e * tstride];
        sr += ar[q] * wr - ai[q] * wi;
        si += ar[q] * wi + ai[q] * wr;
      }
      yr[k + (size_t)p * m] = sr;
      yi[k + (size_t)p * m] = si;
    }
  }
}

/* in-place 3D DFT of (re, im), x fastest; sign -1 forward, +1 inverse
 * (unnormalised).  Returns 0 on success, -1 for an unsupported length. */
int orc_dft3(int nx, int ny, int nz, double *re, double *im, int sign) {
  const int nn[3] = {nx, ny, nz};
  for (int d = 0; d < 3; d++)
    if (!fft_len_ok(nn[d])) return -1;
  const size_t sx = 1, sy = (size_t)nx, sz = (size_t)nx * ny;
  const size_t strides[3] = {sx, sy, sz};
  for (int d = 0; d < 3; d++) {
    const int n = nn[d];
    double *twr = malloc(sizeof(double) * (size_t)n), *twi = malloc(sizeof(double) * (size_t)n);
    for (int e = 0; e < n; e++) {
      const double ang = 2.0 * M_PI * (double)e / (double)n;
      twr[e] = cos(ang);
      twi[e] = (double)sign * sin(ang);
    }
    const int a = (d + 1) % 3, b = (d + 2) % 3;
    const long nlines = (long)nn[a] * nn[b];
#pragma omp parallel
    {
      double *buf = malloc(sizeof(double) * 4 * (size_t)n);
      double *xr = buf, *xi = buf + n, *yr = buf + 2 * n, *yi = buf + 3 * n;
#pragma omp for schedule(static)
      for (long L = 0; L < nlines; L++) {
        const int ia = (int)(L % nn[a]), ib = (int)(L / nn[a]);
        const size_t base = (size_t)ia * strides[a] + (size_t)ib * strides[b];
        for (int t = 0; t < n; t++) {
          xr[t] = re[base + (size_t)t * strides[d]];
          xi[t] = im[base + (size_t)t * strides[d]];
        }
        fft_rec(n, xr, xi, 1, yr, yi, twr, twi, 1);
        for (int t = 0; t < n; t++) {
          re[base + (size_t)t * strides[d]] = yr[t];
          im[base + (size_t)t * strides[d]] = yi[t];
        }
      }
      free(buf);
    }
    free(twr);
    free(twi);
  }
  return 0;
}

/* Sec. 2.3: Laplace(Phi) = 4 pi G (rho + n) on the 27-point stencil, solved in
 * Fourier space:
 *   Phi^(k) = -4 pi G h^2 s^(k) / (6 (1 - D_x D_y D_z)),
 *   D_d = 1 - (2/3) sin^2(pi k_d / N_d),  Phi^(0) = 0.
 * The printed symbol has no minus sign; the minus follows from the equation
 * itself (the operator's symbol is negative), and G multiplies 4 pi. */
int orc_poisson(int nx, int ny, int nz, double h, double G, const double *src,
                double *phi) {
  const size_t nc = (size_t)nx * ny * nz;
  if (G == 0.0) {
    memset(phi, 0, nc * sizeof(double));
    return 0;
  }
  double *re = malloc(nc * sizeof(double)), *im = calloc(nc, sizeof(double));
  memcpy(re, src, nc * sizeof(double));
  if (orc_dft3(nx, ny, nz, re, im, -1) != 0) {
    free(re); free(im);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int kz = 0; kz < nz; kz++)
    for (int ky = 0; ky < ny; ky++)
      for (int kx = 0; kx < nx; kx++) {
        const size_t c = (size_t)kx + (size_t)nx * ((size_t)ky + (size_t)ny * kz);
        if (kx == 0 && ky == 0 && kz == 0) {
          re[c] = 0.0;
          im[c] = 0.0;
          continue;
        }
        const double sx = sin(M_PI * kx / nx), sy = sin(M_PI * ky / ny), sz = sin(M_PI * kz / nz);
        const double Dx = 1.0 - 2.0 / 3.0 * sx * sx;
        const double Dy = 1.0 - 2.0 / 3.0 * sy * sy;
        const double Dz = 1.0 - 2.0 / 3.0 * sz * sz;
        const double Gk = -4.0 * M_PI * G * h * h / (6.0 * (1.0 - Dx * Dy * Dz));
        re[c] *= Gk;
        im[c] *= Gk;
      }
  orc_dft3(nx, ny, nz, re, im, +1);
  for (size_t c = 0; c < nc; c++) phi[c] = re[c] / (double)nc;
  free(re);
  free(im);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Isolated boundaries: Phi(x_i) = sum_j g(x_i - x_j) s_j, the free-space
 * potential of the cell masses, with the sampled point-mass potential
 *   g(d) = -G h^3 / (h |d|)  for a displacement of d != 0 cells,
 *   g(0) = -G h^2 c0,  c0 = 6 ln((1 + sqrt 3) / sqrt 2) - pi / 2,
 * c0 h^2 being the integral of 1/|x| over a cube of side h about its centre
 * (reading: a cell's own mass is spread uniformly over the cell).  Following
 * Hockney and Eastwood, the source is zero-padded to (2nx, 2ny, 2nz) and g is
 * sampled on that lattice at the minimum-image displacement (|d_a| <= n_a on
 * each axis); the cyclic convolution of the two then equals the free-space
 * sum at every output whose displacement to every source is at most n_a on
 * each axis, which covers the grid and its one-cell ring (cells -1 .. n).
 * Phi_ext holds those (nx+2)(ny+2)(nz+2) values, cell i at index i + 1. */
static double cube_centre_integral(void) {
  return 6.0 * log((1.0 + sqrt(3.0)) / sqrt(2.0)) - M_PI / 2.0;
}

/* the DFT of the padded Green function, which is real (g is even) */
static int iso_green_spectrum(int nx, int ny, int nz, double h, double G, double *ghat) {
  const int P[3] = {2 * nx, 2 * ny, 2 * nz};
  const size_t np = (size_t)P[0] * P[1] * P[2];
  double *re = malloc(np * sizeof(double)), *im = calloc(np, sizeof(double));
  const double c0 = cube_centre_integral();
#pragma omp parallel for schedule(static)
  for (int mz = 0; mz < P[2]; mz++)
    for (int my = 0; my < P[1]; my++)
      for (int mx = 0; mx < P[0]; mx++) {
        const double dx = mx <= nx ? mx : mx - P[0];
        const double dy = my <= ny ? my : my - P[1];
        const double dz = mz <= nz ? mz : mz - P[2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        re[(size_t)mx + (size_t)P[0] * ((size_t)my + (size_t)P[1] * mz)] =
            r == 0.0 ? -G * h * h * c0 : -G * h * h / r;
      }
  const int rc = orc_dft3(P[0], P[1], P[2], re, im, -1);
  if (rc == 0) memcpy(ghat, re, np * sizeof(double));
  free(re);
  free(im);
  return rc;
}

static int iso_convolve(int nx, int ny, int nz, const double *ghat, const double *src, double *phi_ext) {
  const int P[3] = {2 * nx, 2 * ny, 2 * nz};
  const size_t np = (size_t)P[0] * P[1] * P[2];
  double *re = calloc(np, sizeof(double)), *im = calloc(np, sizeof(double));
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++)
        re[(size_t)i + (size_t)P[0] * ((size_t)j + (size_t)P[1] * k)] =
            src[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)];
  int rc = orc_dft3(P[0], P[1], P[2], re, im, -1);
  if (rc == 0) {
    for (size_t c = 0; c < np; c++) {
      re[c] *= ghat[c];
      im[c] *= ghat[c];
    }
    orc_dft3(P[0], P[1], P[2], re, im, +1);
    for (int k = -1; k <= nz; k++)
      for (int j = -1; j <= ny; j++)
        for (int i = -1; i <= nx; i++) {
          const size_t q = (size_t)wrap(i, P[0]) + (size_t)P[0] * ((size_t)wrap(j, P[1]) + (size_t)P[1] * wrap(k, P[2]));
          phi_ext[(size_t)(i + 1) + (size_t)(nx + 2) * ((size_t)(j + 1) + (size_t)(ny + 2) * (k + 1))] =
              re[q] / (double)np;
        }
  }
  free(re);
  free(im);
  return rc;
}

/* Isolated potential of src on the grid and its one-cell ring, phi_ext of
 * (nx+2)(ny+2)(nz+2) values.  Returns 0, or -1 for an unsupported length. */
int orc_poisson_isolated(int nx, int ny, int nz, double h, double G, const double *src, double *phi_ext) {
  const size_t ne = (size_t)(nx + 2) * (ny + 2) * (nz + 2);
  if (G == 0.0) {
    memset(phi_ext, 0, ne * sizeof(double));
    return 0;
  }
  double *ghat = malloc((size_t)8 * nx * ny * nz * sizeof(double));
  int rc = iso_green_spectrum(nx, ny, nz, h, G, ghat);
  if (rc == 0) rc = iso_convolve(nx, ny, nz, ghat, src, phi_ext);
  free(ghat);
  return rc;
}

static void stage_poisson(orc_sim *s) {
  if (s->c.poisson != 1) {
    orc_poisson(s->nx, s->ny, s->nz, s->h, s->c.G, s->s, s->phi);
    return;
  }
  const int nx = s->nx, ny = s->ny, nz = s->nz;
  if (s->c.G == 0.0) {
    memset(s->phi_ext, 0, (size_t)(nx + 2) * (ny + 2) * (nz + 2) * sizeof(double));
  } else {
    if (!s->ghat) {
      s->ghat = malloc((size_t)8 * s->ncell * sizeof(double));
      iso_green_spectrum(nx, ny, nz, s->h, s->c.G, s->ghat);
    }
    iso_convolve(nx, ny, nz, s->ghat, s->s, s->phi_ext);
  }
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) s->phi[cidx(s, i, j, k)] = s->phi_ext[ext_nbr(s, i, j, k, 0, 0)];
}

/* ------------------------------------------------------------------------- */
/* CFL step and diagnostics of the current state.  The paper gives no CFL rule;
 * the step is C h / max over cells and axes of the fastest signal speed of
 * either component (gas: |v_d| + sqrt(gamma p / rho); BME: |u_d| + sqrt(3
 * Pi_dd / n), the eigenvalues of Sec. 2.1 and 2.2 shifted by the advection). */
static void finalize_state(orc_sim *s, int advanced) {
  const int nz = s->nz;
  const size_t plane = (size_t)s->nx * s->ny;
  const double gam = s->c.gamma, h = s->h, h3 = h * h * h;
  double *acc = calloc((size_t)nz * 12, sizeof(double));
  unsigned *errk = calloc((size_t)nz, sizeof(unsigned));

#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; k++) {
    double *a = acc + (size_t)k * 12;
    unsigned e = 0;
    for (size_t t = 0; t < plane; t++) {
      const size_t c = (size_t)k * plane + t;
      const double rho = s->f[RHO][c], n = s->f[NB][c];
      const double p = (gam - 1.0) * s->f[EI][c];
      for (int q = 0; q < NF; q++)
        if (!isfinite(s->f[q][c])) e |= ERR_NONFINITE;
      if (!(rho > 0.0) || !(n > 0.0)) e |= ERR_DENSITY;
      if (!(p > 0.0)) e |= ERR_PRESSURE;
      for (int d = 0; d < 3; d++) {
        const double pdd = s->f[PXX + SYM[d][d]][c];
        if (!(pdd > 0.0)) e |= ERR_STRESS;
        const double cg = fabs(s->f[MX + d][c] / rho) + sqrt(fmax(gam * p / rho, 0.0));
        const double cb = fabs(s->f[QX + d][c] / n) + sqrt(fmax(3.0 * pdd / n, 0.0));
        const double sp = cg > cb ? cg : cb;
        if (sp > a[0]) a[0] = sp;
      }
      a[1] += rho;
      a[2] += n;
      for (int d = 0; d < 3; d++) a[3 + d] += s->f[MX + d][c] + s->f[QX + d][c];
      a[6] += s->f[EN][c];
      a[7] += 0.5 * (s->f[WXX][c] + s->f[WYY][c] + s->f[WZZ][c]);
      a[8] += s->s[c] * s->phi[c];
      if (!advanced) {
        /* kappa of a state that has not been through the FlIC stage */
        const double ekin = (s->f[MX][c] * s->f[MX][c] + s->f[MY][c] * s->f[MY][c] +
                             s->f[MZ][c] * s->f[MZ][c]) / (2.0 * rho);
        a[9] += fabs(s->f[EN][c] - s->f[EI][c] - ekin);
        for (int ii = 0; ii < 3; ii++)
          for (int jj = ii; jj < 3; jj++) {
            const int m6 = SYM[ii][jj];
            a[10] += fabs(s->f[WXX + m6][c] - s->f[PXX + m6][c] -
                          s->f[QX + ii][c] * s->f[QX + jj][c] / n);
          }
      }
    }
    errk[k] = e;
  }
  double tot[12] = {0};
  unsigned err = 0;
  for (int k = 0; k < nz; k++) {
    const double *a = acc + (size_t)k * 12;
    if (a[0] > tot[0]) tot[0] = a[0];
    for (int v = 1; v < 12; v++) tot[v] += a[v];
    err |= errk[k];
  }
  free(acc);
  free(errk);

  double dt;
  if (s->c.fixed_dt > 0.0) {
    dt = s->c.fixed_dt;
  } else if (tot[0] > 0.0) {
    dt = s->c.cfl * h / tot[0];
  } else {
    dt = 0.0;
    err |= ERR_NOSPEED;
  }
  if (s->c.t_end > 0.0) {
    const double rem = s->c.t_end - s->t;
    dt = fmin(dt, rem > 0.0 ? rem : 0.0);
  }
  s->dt = dt;
  s->err |= err;

  if (s->ndiag == s->cap) {
    s->cap = s->cap ? 2 * s->cap : 64;
    s->diag = realloc(s->diag, s->cap * DIAG_LEN * sizeof(double));
  }
  double *rec = s->diag + s->ndiag * DIAG_LEN;
  s->ndiag++;
  rec[0] = (double)s->step;
  rec[1] = s->t;
  rec[2] = s->dt;
  rec[3] = h3 * tot[1];
  rec[4] = h3 * tot[2];
  rec[5] = h3 * tot[3];
  rec[6] = h3 * tot[4];
  rec[7] = h3 * tot[5];
  rec[8] = h3 * tot[6];
  rec[9] = h3 * tot[7];
  rec[10] = 0.5 * h3 * tot[8];
  rec[11] = advanced ? s->kappa_gas : h3 * tot[9];
  rec[12] = advanced ? s->kappa_bme : h3 * tot[10];
  rec[13] = s->outflow_gas;
  rec[14] = s->outflow_bme;
  rec[15] = advanced ? s->nsync_gas : 0.0;
  rec[16] = advanced ? s->nsync_bme : 0.0;
  rec[17] = (double)err;
}

/* state at t^n -> Phi^n, tau^n and the diagnostics record of step n */
static void prologue(orc_sim *s) {
  for (size_t c = 0; c < s->ncell; c++) s->s[c] = s->f[RHO][c] + s->f[NB][c];
  stage_poisson(s);
  finalize_state(s, 0);
  s->need_prologue = 0;
  s->next_stage = ST_EUL;
}

static void stage_finalize(orc_sim *s) {
  s->t += s->dt;
  s->step += 1;
  finalize_state(s, 1);
}

/* ------------------------------------------------------------------------- */
/* C entry points used by the tests (prefix orc_)                             */

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

orc_sim *orc_create(const orc_config *cfg) {
  for (int d = 0; d < 3; d++)
    if (cfg->n[d] < 1 || !(cfg->hi[d] > cfg->lo[d])) return NULL;
  const double h = (cfg->hi[0] - cfg->lo[0]) / cfg->n[0];
  for (int d = 1; d < 3; d++) {
    const double hd = (cfg->hi[d] - cfg->lo[d]) / cfg->n[d];
    if (fabs(hd - h) > 1e-12 * h) return NULL; /* one h in the symbol: cubic cells */
  }
  if (cfg->G != 0.0)
    for (int d = 0; d < 3; d++)
      if (!fft_len_ok(cfg->n[d])) return NULL;
  if (cfg->poisson != 0 && cfg->poisson != 1) return NULL;
  orc_sim *s = calloc(1, sizeof(orc_sim));
  s->c = *cfg;
  s->nx = cfg->n[0];
  s->ny = cfg->n[1];
  s->nz = cfg->n[2];
  s->ncell = (size_t)s->nx * s->ny * s->nz;
  s->h = h;
  const size_t nv = (size_t)(s->nx + 1) * (s->ny + 1) * (s->nz + 1);
  for (int q = 0; q < NF; q++) {
    s->f[q] = calloc(s->ncell, sizeof(double));
    s->old[q] = calloc(s->ncell, sizeof(double));
  }
  for (int v = 0; v < 6; v++) {
    s->vel[v] = calloc(s->ncell, sizeof(double));
    s->vtx[v] = calloc(nv, sizeof(double));
  }
  s->phi = calloc(s->ncell, sizeof(double));
  s->s = calloc(s->ncell, sizeof(double));
  if (cfg->poisson == 1) s->phi_ext = calloc((size_t)(s->nx + 2) * (s->ny + 2) * (s->nz + 2), sizeof(double));
  s->need_prologue = 1;
  s->next_stage = ST_EUL;
  return s;
}

void orc_destroy(orc_sim *s) {
  if (!s) return;
  for (int q = 0; q < NF; q++) {
    free(s->f[q]);
    free(s->old[q]);
  }
  for (int v = 0; v < 6; v++) {
    free(s->vel[v]);
    free(s->vtx[v]);
  }
  free(s->phi);
  free(s->s);
  free(s->phi_ext);
  free(s->ghat);
  free(s->diag);
  free(s);
}

int orc_set_field(orc_sim *s, int id, const double *src) {
  if (id < 0 || id >= NF) return -1;
  memcpy(s->f[id], src, s->ncell * sizeof(double));
  s->need_prologue = 1;
  s->next_stage = ST_EUL;
  return 0;
}

int orc_get_field(orc_sim *s, int id, double *dst) {
  if (id == ID_PHI) {
    if (s->need_prologue) prologue(s);
    memcpy(dst, s->phi, s->ncell * sizeof(double));
    return 0;
  }
  if (id < 0 || id >= NF) return -1;
  memcpy(dst, s->f[id], s->ncell * sizeof(double));
  return 0;
}

/* isolated potential on the grid and its one-cell ring ((nx+2)(ny+2)(nz+2)) */
int orc_get_phi_ext(orc_sim *s, double *dst) {
  if (s->c.poisson != 1) return -1;
  if (s->need_prologue) prologue(s);
  memcpy(dst, s->phi_ext, (size_t)(s->nx + 2) * (s->ny + 2) * (s->nz + 2) * sizeof(double));
  return 0;
}

void orc_set_time(orc_sim *s, double t, int64_t step) {
  s->t = t;
  s->step = step;
  s->need_prologue = 1;
  s->next_stage = ST_EUL;
}

double orc_get_dt(orc_sim *s) {
  if (s->need_prologue) prologue(s);
  return s->dt;
}

/* one stage of the step, in order EUL, LAG, POISSON, FINALIZE */
int orc_stage(orc_sim *s, int stage) {
  if (s->need_prologue) prologue(s);
  if (stage != s->next_stage) return -1;
  switch (stage) {
    case ST_EUL: stage_eulerian(s); break;
    case ST_LAG: stage_lagrangian(s); break;
    case ST_POISSON: stage_poisson(s); break;
    case ST_FINALIZE: stage_finalize(s); break;
    default: return -1;
  }
  s->next_stage = (stage + 1) % 4;
  return 0;
}

/* advance n full steps; returns the latched error bits (0 = clean) */
int orc_step(orc_sim *s, int nsteps) {
  if (s->need_prologue) prologue(s);
  if (s->next_stage != ST_EUL) return -1;
  for (int t = 0; t < nsteps; t++) {
    stage_eulerian(s);
    stage_lagrangian(s);
    stage_poisson(s);
    stage_finalize(s);
  }
  return (int)s->err;
}

int orc_diag_len(void) { return DIAG_LEN; }

int orc_diag_count(orc_sim *s) {
  if (s->need_prologue) prologue(s);
  return (int)s->ndiag;
}

int orc_get_diag(orc_sim *s, double *out, int max, int *count) {
  if (s->need_prologue) prologue(s);
  const int n = (int)s->ndiag < max ? (int)s->ndiag : max;
  const size_t first = s->ndiag - (size_t)n; /* the most recent n records */
  memcpy(out, s->diag + first * DIAG_LEN, (size_t)n * DIAG_LEN * sizeof(double));
  *count = n;
  return 0;
}
