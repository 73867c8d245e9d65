/*
 * fld_oracle.c -- plain, slow FP64 CPU reference for one implicit grey
 * flux-limited-diffusion (FLD) radiation step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP solver is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library, and the GPU library never calls it.
 *
 * What it computes (Norman et al., "Fully-Coupled Simulation of Cosmic
 * Reionization. I", Sec. 3.3 and Sec. 2):
 *
 *   PDE (eq. "fld"):      dE/dt = div(D grad E) - (adot/a) E - c kappa E + eta
 *   limiter (Sec. 2):     D = min{ c (9 kbar^2 + R^2)^(-1/2), D_max },
 *                         R = max{ |dE/dn| / Ebar, R_min }
 *                         with Ebar the arithmetic and kbar the harmonic mean
 *                         of the two cells that share the face.
 *   space (Sec. 3.3):     cell-centred finite volumes on a uniform periodic
 *                         Cartesian mesh -> 7-point operator L.
 *   time (Sec. 3.3):      theta-method with D lagged at E^n, so the step is
 *                         linear:  (I - theta dt L) dE = dt (L E^n + eta),
 *                         posed for the change dE = E^{n+1} - E^n
 *                         (residual-correction form).
 *   subcycling (Sec. 3.4): on a failed solve the radiation step is cut by 10x
 *                         and subcycled up to the requested step.
 *
 * The exact per-step result is the solution dE* of one symmetric positive
 * definite linear system.  The oracle therefore does not use multigrid: it
 * solves that system with Jacobi-preconditioned conjugate gradients to a
 * tight tolerance, which reaches dE* up to rounding.
 *
 * Readings where the paper is silent or ambiguous (each one is listed in the
 * design notes):
 *   - R uses the one-sided face-normal difference |E_q - E_p| / dx_d.
 *   - Ebar <= 0 (including E_p = E_q = 0) gives R = R_min.
 *   - kbar = 0 when either cell has kappa = 0 (the limit of the harmonic mean).
 *   - kappa, eta, a, adot are frozen over the step.
 *   - The mesh is comoving and eq. "fld" is taken as printed: Sec. 2 takes
 *     every spatial derivative with respect to the comoving position, so
 *     the limiter's R and the diffusion term use the comoving cell sizes,
 *     and a enters the step only through adot/a.
 *   - The time-step estimator the paper defers to prior work is replaced by
 *     rho = RMS(dE / max(|E^{n+1}|, e_floor)), dt_next = dt * clamp(tau/rho,
 *     0.1, 2).  This controller is PARITY UNPINNED (only its mechanism is
 *     tested).
 *
 * Layout: C order [nz][ny][nx], x fastest, periodic, no ghost cells.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The same source builds serially (liboracle.so, used for every parity check)
 * and with OpenMP over the cell loops (liboracle_omp.so, used only to time
 * the oracle on all host cores).  The parallel build sums its reductions in
 * another order, so its results agree with the serial ones to rounding only. */
#ifdef _OPENMP
#include <omp.h>
#define OR_FOR _Pragma("omp parallel for schedule(static)")
#define OR_FOR_SUM_S _Pragma("omp parallel for schedule(static) reduction(+:s)")
#else
#define OR_FOR
#define OR_FOR_SUM_S
#endif

/* Threads the cell loops run on (1 in the serial build); n > 0 sets it. */
int oracle_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* status codes returned by the oracle (its own numbering) */
#define OR_OK 0
#define OR_NOCONV 1
#define OR_NONFINITE 2
#define OR_BADARG 3

static int64_t wrap(int64_t i, int64_t n) { return ((i % n) + n) % n; }

static int64_t cell(int64_t i, int64_t j, int64_t k, int64_t nx, int64_t ny,
                    int64_t nz) {
  return (wrap(k, nz) * ny + wrap(j, ny)) * nx + wrap(i, nx);
}

/* Face value of the limiter between two neighbouring cells (Sec. 2, the
 * limiter D and its face-centred means). */
double oracle_face_limiter(double E1, double E2, double k1, double k2,
                           double dxd, double c, double d_max, double r_min) {
  double Ebar = 0.5 * (E1 + E2);
  double ksum = k1 + k2;
  double kbar = (ksum != 0.0) ? (2.0 * k1 * k2 / ksum) : 0.0;
  double R;
  if (Ebar > 0.0)
    R = fabs(E2 - E1) / (dxd * Ebar);
  else
    R = r_min;
  if (R < r_min) R = r_min;
  double D = c / sqrt(9.0 * kbar * kbar + R * R);
  if (D > d_max) D = d_max;
  return D;
}

/* Face limiters on the +x, +y, +z face of every cell. */
void oracle_faces(int nx, int ny, int nz, double dx, double dy, double dz,
                  const double *E, const double *kappa, double c, double d_max,
                  double r_min, double *Dx, double *Dy, double *Dz) {
  OR_FOR
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t p = cell(i, j, k, nx, ny, nz);
        int64_t qx = cell(i + 1, j, k, nx, ny, nz);
        int64_t qy = cell(i, j + 1, k, nx, ny, nz);
        int64_t qz = cell(i, j, k + 1, nx, ny, nz);
        Dx[p] = oracle_face_limiter(E[p], E[qx], kappa[p], kappa[qx], dx, c,
                                    d_max, r_min);
        Dy[p] = oracle_face_limiter(E[p], E[qy], kappa[p], kappa[qy], dy, c,
                                    d_max, r_min);
        Dz[p] = oracle_face_limiter(E[p], E[qz], kappa[p], kappa[qz], dz, c,
                                    d_max, r_min);
      }
}

/* (L u)_p: the finite-volume divergence of D grad u minus (adot/a + c kappa) u
 * (eq. "fld" right-hand side without eta). */
void oracle_apply_L(int nx, int ny, int nz, double dx, double dy, double dz,
                    const double *Dx, const double *Dy, const double *Dz,
                    const double *kappa, double c, double adot_over_a,
                    const double *u, double *out) {
  double ix2 = 1.0 / (dx * dx), iy2 = 1.0 / (dy * dy), iz2 = 1.0 / (dz * dz);
  OR_FOR
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t p = cell(i, j, k, nx, ny, nz);
        int64_t xp = cell(i + 1, j, k, nx, ny, nz), xm = cell(i - 1, j, k, nx, ny, nz);
        int64_t yp = cell(i, j + 1, k, nx, ny, nz), ym = cell(i, j - 1, k, nx, ny, nz);
        int64_t zp = cell(i, j, k + 1, nx, ny, nz), zm = cell(i, j, k - 1, nx, ny, nz);
        double div = (Dx[p] * (u[xp] - u[p]) - Dx[xm] * (u[p] - u[xm])) * ix2 +
                     (Dy[p] * (u[yp] - u[p]) - Dy[ym] * (u[p] - u[ym])) * iy2 +
                     (Dz[p] * (u[zp] - u[p]) - Dz[zm] * (u[p] - u[zm])) * iz2;
        out[p] = div - (adot_over_a + c * kappa[p]) * u[p];
      }
}

/* Everything the linear system of one theta-step needs. */
typedef struct {
  int nx, ny, nz;
  double dx, dy, dz, c, theta, dt, adot_over_a;
  const double *kappa;
  double *Dx, *Dy, *Dz; /* owned */
} or_system;

/* A u = u - theta dt L u  (Sec. 3.3, theta-method on the change dE) */
static void sys_apply_A(const or_system *s, const double *u, double *Lu,
                        double *out) {
  int64_t n = (int64_t)s->nx * s->ny * s->nz;
  oracle_apply_L(s->nx, s->ny, s->nz, s->dx, s->dy, s->dz, s->Dx, s->Dy, s->Dz,
                 s->kappa, s->c, s->adot_over_a, u, Lu);
  OR_FOR
  for (int64_t p = 0; p < n; ++p) out[p] = u[p] - s->theta * s->dt * Lu[p];
}

/* diagonal of A, for the Jacobi preconditioner */
static void sys_diag(const or_system *s, double *d) {
  double ix2 = 1.0 / (s->dx * s->dx), iy2 = 1.0 / (s->dy * s->dy),
         iz2 = 1.0 / (s->dz * s->dz);
  int nx = s->nx, ny = s->ny, nz = s->nz;
  OR_FOR
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t p = cell(i, j, k, nx, ny, nz);
        double faces = (s->Dx[p] + s->Dx[cell(i - 1, j, k, nx, ny, nz)]) * ix2 +
                       (s->Dy[p] + s->Dy[cell(i, j - 1, k, nx, ny, nz)]) * iy2 +
                       (s->Dz[p] + s->Dz[cell(i, j, k - 1, nx, ny, nz)]) * iz2;
        d[p] = 1.0 + s->theta * s->dt *
                         (s->adot_over_a + s->c * s->kappa[p] + faces);
      }
}

static double dot(const double *a, const double *b, int64_t n) {
  double s = 0.0;
  OR_FOR_SUM_S
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/*
 * Jacobi-preconditioned CG on A x = b from x = 0, stopping when
 * ||b - A x||_2 <= tol ||b||_2 (recursive residual; the caller may check the
 * true residual).  Returns OR_OK, OR_NOCONV or OR_NONFINITE.
 */
static int sys_pcg(const or_system *s, const double *b, double *x, double tol,
                   int max_iter, int *iters, double *relres) {
  int64_t n = (int64_t)s->nx * s->ny * s->nz;
  double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
  double *p = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double));
  double *Lw = malloc(n * sizeof(double)), *d = malloc(n * sizeof(double));
  int status = OR_NOCONV;
  sys_diag(s, d);
  OR_FOR
  for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
  double bb = dot(b, b, n);
  double rr = bb;
  *iters = 0;
  *relres = 0.0;
  if (!isfinite(bb)) { status = OR_NONFINITE; goto done; }
  if (bb == 0.0) { status = OR_OK; goto done; }
  double rz_old = 0.0;
  for (int it = 0; it < max_iter; ++it) {
    OR_FOR
    for (int64_t i = 0; i < n; ++i) z[i] = r[i] / d[i];
    double rz = dot(r, z, n);
    if (it == 0) {
      OR_FOR
      for (int64_t i = 0; i < n; ++i) p[i] = z[i];
    } else {
      double beta = rz / rz_old;
      OR_FOR
      for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    rz_old = rz;
    sys_apply_A(s, p, Lw, q);
    double alpha = rz / dot(p, q, n);
    OR_FOR
    for (int64_t i = 0; i < n; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    rr = dot(r, r, n);
    *iters = it + 1;
    if (!isfinite(rr)) { status = OR_NONFINITE; goto done; }
    if (rr <= tol * tol * bb) { status = OR_OK; break; }
  }
done:
  *relres = (bb > 0.0 && isfinite(rr)) ? sqrt(rr / bb) : 0.0;
  free(r); free(z); free(p); free(q); free(Lw); free(d);
  return status;
}

static int sys_init(or_system *s, int nx, int ny, int nz, double dx, double dy,
                    double dz, const double *E, const double *kappa, double c,
                    double d_max, double r_min, double theta, double dt,
                    double a, double adot) {
  int64_t n = (int64_t)nx * ny * nz;
  s->nx = nx; s->ny = ny; s->nz = nz;
  s->dx = dx; s->dy = dy; s->dz = dz;
  s->c = c; s->theta = theta; s->dt = dt; s->adot_over_a = adot / a;
  s->kappa = kappa;
  s->Dx = malloc(n * sizeof(double));
  s->Dy = malloc(n * sizeof(double));
  s->Dz = malloc(n * sizeof(double));
  oracle_faces(nx, ny, nz, dx, dy, dz, E, kappa, c, d_max, r_min, s->Dx, s->Dy,
               s->Dz);
  return OR_OK;
}

static void sys_free(or_system *s) { free(s->Dx); free(s->Dy); free(s->Dz); }

/* b = dt (L E^n + eta)  (right-hand side of the residual-correction form) */
static void sys_rhs(const or_system *s, const double *E, const double *eta,
                    double *b) {
  int64_t n = (int64_t)s->nx * s->ny * s->nz;
  oracle_apply_L(s->nx, s->ny, s->nz, s->dx, s->dy, s->dz, s->Dx, s->Dy, s->Dz,
                 s->kappa, s->c, s->adot_over_a, E, b);
  OR_FOR
  for (int64_t p = 0; p < n; ++p) b[p] = s->dt * (b[p] + eta[p]);
}

/* Matrix and right-hand side of one step, for inspection by tests:
 * diag = A_pp, Ax/Ay/Az = -A_{p,p+e_d} (positive numbers), b. */
void oracle_system(int nx, int ny, int nz, double dx, double dy, double dz,
                   const double *E, const double *kappa, const double *eta,
                   double c, double d_max, double r_min, double theta,
                   double dt, double a, double adot, double *diag, double *Ax,
                   double *Ay, double *Az, double *b) {
  or_system s;
  int64_t n = (int64_t)nx * ny * nz;
  sys_init(&s, nx, ny, nz, dx, dy, dz, E, kappa, c, d_max, r_min, theta, dt, a,
           adot);
  sys_diag(&s, diag);
  /* s.dx, s.dy, s.dz: the cell sizes the operator uses */
  for (int64_t p = 0; p < n; ++p) {
    Ax[p] = theta * dt * s.Dx[p] / (s.dx * s.dx);
    Ay[p] = theta * dt * s.Dy[p] / (s.dy * s.dy);
    Az[p] = theta * dt * s.Dz[p] / (s.dz * s.dz);
  }
  sys_rhs(&s, E, eta, b);
  sys_free(&s);
}

/* out = A u for the system defined by (E^n, kappa, dt, ...). */
void oracle_apply_A(int nx, int ny, int nz, double dx, double dy, double dz,
                    const double *E, const double *kappa, double c,
                    double d_max, double r_min, double theta, double dt,
                    double a, double adot, const double *u, double *out) {
  or_system s;
  int64_t n = (int64_t)nx * ny * nz;
  double *Lw = malloc(n * sizeof(double));
  sys_init(&s, nx, ny, nz, dx, dy, dz, E, kappa, c, d_max, r_min, theta, dt, a,
           adot);
  sys_apply_A(&s, u, Lw, out);
  free(Lw);
  sys_free(&s);
}

/*
 * Solve one step's system for dE (E^n, kappa, eta frozen).  Returns the
 * status; iters and relres report the CG run.
 */
int oracle_solve(int nx, int ny, int nz, double dx, double dy, double dz,
                 const double *E, const double *kappa, const double *eta,
                 double c, double d_max, double r_min, double theta, double dt,
                 double a, double adot, double tol, int max_iter, double *dE,
                 int *iters, double *relres) {
  if (nx < 1 || ny < 1 || nz < 1 || !(dt > 0.0) || !(a > 0.0))
    return OR_BADARG;
  or_system s;
  int64_t n = (int64_t)nx * ny * nz;
  double *b = malloc(n * sizeof(double));
  sys_init(&s, nx, ny, nz, dx, dy, dz, E, kappa, c, d_max, r_min, theta, dt, a,
           adot);
  sys_rhs(&s, E, eta, b);
  int st = sys_pcg(&s, b, dE, tol, max_iter, iters, relres);
  free(b);
  sys_free(&s);
  return st;
}

/*
 * Residual b - A x at a list of cells, each computed on its own from the
 * 13-cell neighbourhood it depends on (for spot checks on grids too large to
 * assemble whole).  cells[] holds linear indices.
 */
void oracle_residual_at(int nx, int ny, int nz, double dx, double dy, double dz,
                        const double *E, const double *kappa, const double *eta,
                        double c, double d_max, double r_min, double theta,
                        double dt, double a, double adot, const double *x,
                        const int64_t *cells, int64_t ncells, double *res,
                        double *rhs) {
  /* comoving cell sizes, as in sys_init */
  double hd[3] = {dx, dy, dz};
  double h2[3] = {hd[0] * hd[0], hd[1] * hd[1], hd[2] * hd[2]};
  double aa = adot / a;
  OR_FOR
  for (int64_t t = 0; t < ncells; ++t) {
    int64_t p = cells[t];
    int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((int64_t)nx * ny));
    double LE = 0.0, Lx = 0.0;
    for (int d = 0; d < 3; ++d) {
      int di = (d == 0), dj = (d == 1), dk = (d == 2);
      int64_t qp = cell(i + di, j + dj, k + dk, nx, ny, nz);
      int64_t qm = cell(i - di, j - dj, k - dk, nx, ny, nz);
      double Dp = oracle_face_limiter(E[p], E[qp], kappa[p], kappa[qp], hd[d],
                                      c, d_max, r_min);
      double Dm = oracle_face_limiter(E[qm], E[p], kappa[qm], kappa[p], hd[d],
                                      c, d_max, r_min);
      LE += (Dp * (E[qp] - E[p]) - Dm * (E[p] - E[qm])) / h2[d];
      Lx += (Dp * (x[qp] - x[p]) - Dm * (x[p] - x[qm])) / h2[d];
    }
    double mu = aa + c * kappa[p];
    LE -= mu * E[p];
    Lx -= mu * x[p];
    double b = dt * (LE + eta[p]);
    double Ax = x[p] - theta * dt * Lx;
    res[t] = b - Ax;
    if (rhs) rhs[t] = b;
  }
}

/*
 * One radiation step of length dt with subcycling (Sec. 3.4): try the whole
 * step; on a failed solve cut the radiation step by 10x and subcycle until the
 * requested time is reached, updating the step from the relative change.
 * E is updated in place only on success.  out_stats (nullable) receives
 * {substeps, cuts, total CG iterations, last relres, last rho, dt_next}.
 */
int oracle_step(int nx, int ny, int nz, double dx, double dy, double dz,
                double *E, const double *kappa, const double *eta, double c,
                double d_max, double r_min, double theta, double dt, double a,
                double adot, double tol, int max_iter, double tau_tol,
                double e_floor, int max_cuts, double *out_stats) {
  if (!(dt > 0.0)) return OR_BADARG;
  int64_t n = (int64_t)nx * ny * nz;
  double *Ework = malloc(n * sizeof(double));
  double *dE = malloc(n * sizeof(double));
  memcpy(Ework, E, n * sizeof(double));
  double t = 0.0, h = dt, rho = 0.0, relres = 0.0;
  int cuts = 0, substeps = 0, total_it = 0, st = OR_OK;
  while (dt - t > 1e-12 * dt) {
    if (h > dt - t) h = dt - t;
    int it = 0;
    st = oracle_solve(nx, ny, nz, dx, dy, dz, Ework, kappa, eta, c, d_max,
                      r_min, theta, h, a, adot, tol, max_iter, dE, &it,
                      &relres);
    total_it += it;
    if (st != OR_OK) {
      if (st == OR_BADARG) break;
      if (cuts >= max_cuts) break;
      h *= 0.1;
      ++cuts;
      continue;
    }
    double acc = 0.0;
    for (int64_t p = 0; p < n; ++p) {
      Ework[p] += dE[p];
      double w = fabs(Ework[p]);
      if (w < e_floor) w = e_floor;
      if (w > 0.0) acc += (dE[p] / w) * (dE[p] / w);
    }
    rho = sqrt(acc / (double)n);
    t += h;
    ++substeps;
    double f = (rho > 0.0) ? tau_tol / rho : 2.0;
    if (f < 0.1) f = 0.1;
    if (f > 2.0) f = 2.0;
    h *= f;
  }
  if (st == OR_OK) memcpy(E, Ework, n * sizeof(double));
  if (out_stats) {
    out_stats[0] = substeps;
    out_stats[1] = cuts;
    out_stats[2] = total_it;
    out_stats[3] = relres;
    out_stats[4] = rho;
    out_stats[5] = h;
  }
  free(Ework);
  free(dE);
  return st;
}

/* ---------------------------------------------------------------------------
 * Isothermal hydrogen chemistry: the loosely coupled chemistry solver of
 * Sec. 3.3 (one linearly implicit backward-Euler update per species and cell)
 * for the hydrogen-only, fixed-temperature gas of Test 1 (Sec. 4.1.1).
 *
 * Pure hydrogen leaves one independent species, the ionized fraction
 * x = n_HII / n_H, with n_HI = n_H (1 - x) and n_e = n_HII = n_H x.  The rate
 * equation of eq. "heat_chem" for it is
 *   dx/dt = Gamma (1 - x) - alpha_B n_H x^2,
 * with the photo-ionization rate of monochromatic radiation of energy
 * density E at the ionization threshold (Sec. 2: photon number density
 * E / (h nu), each photon ionizing at rate c sigma n_HI):
 *   Gamma = c sigma E / (h nu).
 * The linearly implicit update takes x at the new time wherever it enters
 * linearly and holds the electron density of the recombination term at the
 * old value:
 *   x+ - x = h [ Gamma (1 - x+) - alpha_B n_H x x+ ]
 *   =>  x+ = (x + h Gamma) / (1 + h (Gamma + alpha_B n_H x)).
 * E (and so Gamma) is the radiation field at the end of the radiation step,
 * frozen over the chemistry step (Sec. 3.4 processes the new E into the
 * rates first).  The step dt is taken in `substeps` equal pieces.  Finally
 * the opacity seen by the next radiation step is kappa = sigma n_HI.
 *
 * E and n_H are comoving densities (Sec. 2: comoving = proper a^3), so the
 * rates use the proper values E / a^3 and n_H / a^3, and kappa is the proper
 * opacity (per proper length) that the radiation step takes; a = 1 for a
 * static problem.
 * ------------------------------------------------------------------------- */
void oracle_chem_h(int64_t n, const double *E, const double *n_h, double *x,
                   double *kappa, double dt, int substeps, double c,
                   double sigma, double hnu, double alpha_b, double a) {
  double h = dt / (double)substeps;
  double inv_a3 = 1.0 / (a * a * a);
  for (int64_t p = 0; p < n; ++p) {
    double nh = n_h[p] * inv_a3;
    double gamma = c * sigma * (E[p] * inv_a3) / hnu;
    double xp = x[p];
    for (int s = 0; s < substeps; ++s)
      xp = (xp + h * gamma) / (1.0 + h * (gamma + alpha_b * nh * xp));
    x[p] = xp;
    kappa[p] = sigma * nh * (1.0 - xp);
  }
}
