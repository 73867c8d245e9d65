/*
 * fld.h -- C-ABI of the MI355X implicit grey flux-limited-diffusion (FLD)
 * radiation step (Norman et al., arXiv:1306.0645).
 *
 * The operation (Sec. 3.3, eq. "fld"): advance the comoving grey radiation
 * energy density E over one step dt of
 *
 *     dE/dt = div(D grad E) - (adot/a) E - c kappa E + eta
 *
 * on a uniform periodic Cartesian mesh, with the flux limiter (Sec. 2)
 *
 *     D = min{ c (9 kbar^2 + R^2)^(-1/2), D_max },  R = max{ |dE/dn| / Ebar, R_min },
 *
 * evaluated on each cell face from E^n (lagged), Ebar the arithmetic and kbar
 * the harmonic mean of the two cells that share the face.  Finite volumes give
 * a 7-point operator L; the theta-method (theta = 1 backward Euler, 1/2
 * trapezoidal) in residual-correction form gives one symmetric positive
 * definite system per step,
 *
 *     (I - theta dt L) dE = dt (L E^n + eta),     E^{n+1} = E^n + dE,
 *
 * solved by conjugate gradients preconditioned with a geometric multigrid
 * V-cycle with red/black Gauss-Seidel smoothing (Sec. 3.3, Table 1).  On a
 * failed solve fld_step cuts the radiation step by 10x and subcycles up to the
 * requested step (Sec. 3.4).
 *
 * Conventions for every entry point:
 *  - Field pointers are DEVICE pointers to FP64 arrays of nx*ny*nz cells in
 *    C order [nz][ny][nx] (x fastest), interior cells only; the periodic wrap
 *    is internal.  The caller owns all field memory and the workspace.
 *  - Units are the caller's, but must be consistent: c, dx, 1/kappa, dt, and
 *    D_max (length^2/time), R_min (1/length) in the same length/time units.
 *  - The mesh is comoving with expansion factor a: Sec. 2 takes every
 *    spatial derivative with respect to the comoving position, and E and eta
 *    are comoving densities, so eq. "fld" is posed on the comoving cell
 *    sizes dx, dy, dz as printed and a enters the step only through adot/a;
 *    kappa is the opacity the caller's chemistry gives (proper, per unit
 *    length); a = 1, adot = 0 for a static problem.
 *  - Work is enqueued on the hipStream_t given at create time (NULL = the
 *    default stream).  Calls that report convergence synchronise that stream.
 *  - No entry point allocates device memory: handles carve the caller's
 *    workspace.  Host-side metadata is malloc'd and freed by *_destroy.
 *  - Errors: FLD_EINVAL for bad arguments (checked before any launch),
 *    FLD_ENOMEM for a workspace or budget that is too small, FLD_ENOCONV when
 *    the solve reaches max_iter, FLD_ENONFINITE when a residual norm is NaN/Inf
 *    (NaN/Inf inputs), FLD_EDEVICE for a HIP runtime error, FLD_EBUSY for a
 *    pending served request.  No entry point writes E on error.
 *  - One handle per stream; handles are not thread-safe.
 */
#ifndef FLD_H_
#define FLD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fld_status {
  FLD_OK = 0,
  FLD_EINVAL = -1,
  FLD_ENOMEM = -2,
  FLD_ENOCONV = -3,
  FLD_ENONFINITE = -4,
  FLD_EDEVICE = -5,
  FLD_EBUSY = -6
} fld_status;

typedef enum fld_precision {
  FLD_PREC_FP64 = 0,  /* FP64 everywhere: PCG with a symmetric FP64 V-cycle */
  FLD_PREC_MIXED = 1  /* FP32 V-cycle (smoother, transfers, residuals)
                         whose output z is kept in FP32 at a per-problem
                         scale; x, r, q, the search direction p (unless
                         direction_fp64 = 0), the operator, the SpMV, the
                         outer residual, refinement and the coarsest solve in
                         FP64; flexible (Polak-Ribiere) PCG */
} fld_precision;

/* Multigrid smoother (Sec. 3.3 names red/black Gauss-Seidel sweeps). */
typedef enum fld_smoother {
  FLD_SMOOTH_RBGS = 0,   /* red/black Gauss-Seidel (default); with nu_pre =
                            nu_post = 1 the finest level runs fused passes */
  FLD_SMOOTH_JACOBI = 1  /* weighted Jacobi, weight 6/7 (the optimum for the
                            7-point Laplacian under full 2x coarsening); one
                            kernel per sweep and level, an extra iterate
                            buffer per level; tail_cells is ignored (only the
                            coarsest level goes to the tail kernel) */
} fld_smoother;

/* Periodic 3-D mesh.  Every extent must be even and >= 4 (red/black
 * colouring of a periodic grid needs even extents); nx*ny*nz < 2^31. */
typedef struct fld_grid {
  int32_t nx, ny, nz, reserved;
  double dx, dy, dz;  /* cell sizes, > 0 */
} fld_grid;

typedef struct fld_params {
  double c;            /* speed of light, > 0 */
  double theta;        /* time weight in [0.5, 1]; 1 = backward Euler (Sec. 3.3) */
  double d_max;        /* limiter cap D_max; paper: 0.006 c L_unit (Sec. 2) */
  double r_min;        /* limiter floor R_min; paper: 1e-20 / L_unit (Sec. 2) */
  double rtol;         /* stop when ||b - A dE||_2 <= rtol ||b||_2; paper 1e-8 (Table 1) */
  double tau_tol;      /* target RMS relative change per step; paper 1e-4 (Sec. 3.4) */
  double e_floor;      /* floor on |E| in that relative change, >= 0 */
  double coarse_scale; /* coarse-face scale: T_c = coarse_scale * (sum of the 4
                          fine faces); 0.5 rediscretises the operator (default) */
  int32_t max_iter;    /* PCG iteration cap; paper 50 (Table 1) */
  int32_t mg_levels;   /* multigrid levels incl. the finest; 0 = automatic */
  int32_t nu_pre;      /* smoothing sweeps before restriction (a red/black
                          sweep is both half-sweeps); paper 1 (Table 1) */
  int32_t nu_post;     /* sweeps after prolongation; paper 1 (Table 1) */
  int32_t precision;   /* fld_precision */
  int32_t max_dt_cuts; /* fld_step: at most this many 10x cuts (Sec. 3.4) */
  int32_t tile_z;      /* z-depth of one work tile; 0 = automatic */
  int32_t check_every; /* PCG iterations between host convergence reads; 0 = auto */
  int32_t use_graph;   /* 1 (default) = replay the PCG iteration from a captured
                          hipGraph; 0 = launch its kernels one by one */
  int32_t fused_tile_z;/* z-depth of the fused finest-level V-cycle tiles (even);
                          0 = automatic (64 planes where 2048 such tiles
                          remain, else 32 halved until 512 remain).  A grid
                          with 2048 fused finest tiles also runs the mixed
                          fused iteration's SpMV on them */
  int32_t cycle_switch;/* > 0 and nu_pre = nu_post = 1: when a solve needs
                          more PCG iterations than this, later solves of the
                          handle switch cycle, until one needs at most a
                          third of it and the handle switches back.  The
                          switched cycle is V(1,1) with trilinear correction
                          in mixed precision with prolongation = 2 when the
                          largest grid has at least 2^23 cells, else V(2,2);
                          an FP64 handle whose largest grid has at least 2^23
                          cells does not switch (its fused V(1,1) iteration
                          costs less than half a V(2,2) one).  0, or any
                          other configured cycle: the cycle stays as
                          configured.  Default 12 */
  int32_t prolongation;/* coarse-grid correction of the FP32 (mixed) cycle:
                          0 = piecewise constant, 1 = cell-centred trilinear,
                          2 = trilinear only while the handle is switched by
                          cycle_switch (default).  The FP64 cycle is always
                          piecewise constant with restriction = its
                          transpose, so it stays a symmetric preconditioner */
  int32_t warm_start;  /* fld_step / fld_batch_step (and each request of a
                          server): start each step's PCG from the handle's
                          previous successful dEs.  2 (default) = the
                          combination c1 dE(n) + c2 dE(n-1) that is closest
                          to the new solution in the new operator's A-norm
                          (Galerkin: (dE(i), A dE(j)) c_j = (dE(i), b)); 1 =
                          their extrapolation by the ratios of the step
                          sizes; 0 = start from dE = 0.  The residual
                          b - A dE0 is formed first, the guess is dropped if
                          it does not reduce ||b - A dE0|| below ||b||, and
                          the stopping rule is unchanged */
  int32_t tail_cells;  /* the coarsest level is solved (Jacobi-CG in FP64) by
                          one workgroup per problem; coarse levels of at most
                          this many cells above it join that kernel (same
                          sweeps, no per-level launches).  Default 512 (an 8^3
                          level: measured at 256^3, 2680 against 2652
                          Mcell-updates/s with 0 and 2658 with 4096) */
  int32_t smoother;    /* fld_smoother; default FLD_SMOOTH_RBGS */
  int32_t fused_levels;/* under V(1,1) red/black: the finest fused_levels
                          levels run the two fused passes (coarse ones with
                          4-plane tiles); 0 = automatic (the finest level, and
                          each coarser one that still holds at least 2^20
                          cells; decided per problem, so that a problem's
                          result does not depend on its batch) */
  int32_t coarse_op;   /* coarse face coefficients: 0 = coarse_scale times the
                          sum of the 4 fine faces the coarse face covers; 1 =
                          2 coarse_scale times the sum over the 4 fine rows
                          that cross it of the three fine faces between the
                          two coarse centres taken in series, 1 / (0.5/T_in +
                          1/T_face + 0.5/T_in'), which follows the flux
                          through a coarse cell that straddles an opacity
                          jump.  Both give coarse_scale times the fine sum
                          in a uniform medium and keep the coarse operator
                          7-point and symmetric */
  int32_t direction_fp64; /* mixed precision: 1 (default) = the PCG search
                          direction p in FP64, so only the V-cycle (whose
                          output z is FP32 at a per-problem scale) runs in
                          FP32; 0 = p rounded to FP32 at the scale of the z it
                          was formed from (8 B less per cell and iteration) */
  int32_t local_sweeps; /* mixed precision, fused V(1,1) cycle: after the
                          finest post-sweep, this many more red/black sweeps
                          (black, then red) restricted to the finest cells
                          whose coupling dominates their diagonal (sum of the
                          6 faces > local_coupling x diagonal, listed at each
                          assembly; the lists take 4 B per finest cell of the
                          workspace): in ionized bubbles, where absorption is
                          weak and D reaches D_max, one sweep leaves the error
                          that is smooth inside the bubble and the coarse
                          levels miss it.  0 = none.  Default 1 */
  double local_coupling; /* threshold of that mask, in [0, 1]; default 0.98 */
} fld_params;

typedef struct fld_stats {
  int32_t status;       /* fld_status of this call */
  int32_t iters;        /* PCG iterations (summed over substeps) */
  int32_t subcycles;    /* substeps taken by fld_step (1 if no cut) */
  int32_t dt_cuts;      /* 10x cuts taken by fld_step */
  int32_t levels;       /* multigrid levels used */
  int32_t restarts;     /* refinement restarts from the true FP64 residual */
  int32_t cycle_nu;     /* red/black sweeps per side of the V-cycle used last */
  int32_t trilinear;    /* 1: that cycle used the trilinear correction */
  double rel_resid;     /* true ||b - A dE||_2 / ||b||_2 of the last solve */
  double err_bound;     /* ||b - A dE||_2 / ||dE||_2: bounds the relative 2-norm
                           error of dE because ||A^-1||_2 <= 1 when adot >= 0 */
  double rel_change_rms;/* RMS of dE / max(|E^{n+1}|, e_floor), last substep */
  double dt_next;       /* suggested next step: dt * clamp(tau_tol/rho, 0.1, 2) */
  double bnorm;         /* ||b||_2 of the last solve */
  double dEnorm;        /* ||dE||_2 of the last solve */
} fld_stats;

typedef struct fld_handle fld_handle;
typedef struct fld_batch fld_batch;
typedef struct fld_server fld_server;

/* Paper defaults (Sec. 2, Sec. 3.4, Table 1) for a run whose length unit is
 * L_unit: d_max = 0.006 c L_unit, r_min = 1e-20 / L_unit, rtol = 1e-8,
 * max_iter = 50, nu_pre = nu_post = 1, theta = 1, tau_tol = 1e-4, FP64,
 * coarse_scale = 0.5, max_dt_cuts = 8, graph replay on, cycle_switch = 12,
 * prolongation = 2 (trilinear in the mixed cycle once it has switched to
 * V(2,2)), warm_start = 2, tail_cells = 512, smoother = FLD_SMOOTH_RBGS,
 * fused_levels = 0, coarse_op = 0, direction_fp64 = 1, local_sweeps = 1,
 * local_coupling = 0.98. */
void fld_default_params(fld_params *p, double c, double L_unit);

const char *fld_strerror(fld_status s);

/* Bytes of device workspace one handle needs for this grid and parameters
 * (fields, multigrid hierarchy, Krylov vectors, descriptor tables).  Returns
 * 0 for an invalid grid or parameter set. */
size_t fld_workspace_bytes(const fld_grid *g, const fld_params *p);

/* Create a solver handle for one grid.  workspace: device memory of at least
 * fld_workspace_bytes(g, p) bytes, 256-byte aligned, owned by the caller and
 * kept alive until fld_destroy.  hip_stream: hipStream_t or NULL.
 * Errors: FLD_EINVAL (grid/params), FLD_ENOMEM (workspace too small),
 * FLD_EDEVICE. */
fld_status fld_create(const fld_grid *g, const fld_params *p, void *hip_stream,
                      void *workspace, size_t workspace_bytes,
                      fld_handle **out);

/* Assemble one step's system (Sec. 2 limiter, Sec. 3.3 theta-method): face
 * coefficients from the limiter at E^n, the diagonal, b = dt (L E^n + eta),
 * and every coarse level of the multigrid hierarchy.  E_n, kappa, eta: device
 * FP64 [nz][ny][nx], read only, kappa >= 0.  dt > 0, a > 0; adot/a enters
 * the operator.  Enqueued; no synchronisation.
 * Errors: FLD_EINVAL, FLD_EDEVICE. */
fld_status fld_assemble(fld_handle *h, const double *E_n, const double *kappa,
                        const double *eta, double dt, double a, double adot);

/* Solve the assembled system for dE = E^{n+1} - E^n by multigrid-
 * preconditioned CG from dE = 0 (Sec. 3.3, Table 1) until the true FP64
 * residual satisfies ||b - A dE||_2 <= rtol ||b||_2.  dE: device FP64 output,
 * must not alias the inputs given to fld_assemble.  stats: host, nullable.
 * Synchronises the stream.  Errors: FLD_ENOCONV (max_iter reached; dE holds
 * the last iterate), FLD_ENONFINITE, FLD_EINVAL, FLD_EDEVICE. */
fld_status fld_solve(fld_handle *h, double *dE, fld_stats *stats);

/* One radiation step (Sec. 3.3-3.4): assemble at E, solve, E += dE.  If the
 * solve fails, the radiation step is cut by 10x and subcycled until dt is
 * covered, at most max_dt_cuts cuts.  E: device FP64, in E^n, out E^{n+1};
 * on any error E is left unchanged.  stats: host, nullable.  Synchronises.
 * Errors: FLD_ENOCONV (cuts exhausted), FLD_ENONFINITE, FLD_EINVAL,
 * FLD_EDEVICE. */
fld_status fld_step(fld_handle *h, double *E, const double *kappa,
                    const double *eta, double dt, double a, double adot,
                    fld_stats *stats);

/* Release the handle's host metadata (the workspace stays the caller's). */
fld_status fld_destroy(fld_handle *h);

/* Several steps with the step control on the device (Sec. 3.4, the
 * radiation subcycling loop): n_steps > 0 takes n_steps steps of dt, each
 * exactly as fld_step takes it (a failed solve cuts the substep by 10x and
 * the substeps then grow by the controller's factor until dt is covered);
 * n_steps = 0 takes steps of the controller's suggestion, the first of dt
 * and each next one of dt_next = h clamp(tau_tol / rho, 0.1, 2) (h the last
 * substep), clipped to end at t_end.  The assembly, PCG, verification, E
 * update and the controller run as captured graphs of `units` PCG iterations
 * (0 = 8); the host reads the per-problem state once per graph, not per
 * substep.  The cycle stays as configured (the adaptive switch of
 * cycle_switch does not act inside a run).  The results equal those of the
 * same steps through fld_step, bit for bit.  E: device FP64, in E^0, out E
 * after the last completed step (a failed step leaves E as the step before
 * it left it).  stats (host, nullable): iters, restarts, subcycles and
 * dt_cuts summed over the run, the rest of the last substep; steps_done
 * (host, nullable): steps completed.  Errors: those of fld_step, and
 * FLD_EINVAL for n_steps < 0, units < 0, or n_steps = 0 without t_end > 0. */
fld_status fld_advance(fld_handle *h, double *E, const double *kappa,
                       const double *eta, int32_t n_steps, double dt, double t_end,
                       double a, double adot, int32_t units, fld_stats *stats,
                       int32_t *steps_done);

/* --- One step without a caller workspace. --------------------------------
 * For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step as fld_create + fld_step + fld_destroy on the grid g, with kernels
 * launched one by one (use_graph is ignored), but its workspace is a device
 * array of FLD_STATIC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends.  It calls no hipMalloc or hipFree and no
 * routine that allocates device memory (host metadata is built and freed
 * within the call).  E (in E^n, out E^{n+1}), kappa, eta, dt, a, adot, stats
 * and the errors are those of fld_step; FLD_ENOMEM if
 * fld_workspace_bytes(g, p) exceeds FLD_STATIC_SCRATCH_BYTES (a 64^3 mixed or
 * an 80^3 FP64 grid fits).  Nothing carries over between calls.  Every call
 * on one device uses that device's single array: calls that overlap on one
 * device (two host threads, or two streams) race and must not be made. */
#define FLD_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
size_t fld_static_scratch_bytes(void);
fld_status fld_step_static(const fld_grid *g, const fld_params *p,
                           void *hip_stream, double *E, const double *kappa,
                           const double *eta, double dt, double a, double adot,
                           fld_stats *stats);

/* --- Components of the solve, exported for inspection and testing. ------ */

/* Copy the assembled finest-level system to caller device buffers (any may
 * be NULL): diag = A_pp, Tx/Ty/Tz = -A_{p,p+e_d} (the +x/+y/+z face of each
 * cell), b.  Synchronises.  Errors: FLD_EINVAL (nothing assembled), FLD_EDEVICE. */
fld_status fld_get_system(fld_handle *h, double *diag, double *Tx, double *Ty,
                          double *Tz, double *b);

/* out = A u with the assembled finest-level operator (7-point SpMV, Sec.
 * 3.3).  u, out: device FP64, distinct.  Synchronises. */
fld_status fld_apply(fld_handle *h, const double *u, double *out);

/* z = B r: one multigrid V-cycle (the PCG preconditioner, Table 1) applied to
 * r, in the handle's precision.  r, z: device FP64, distinct.  Synchronises. */
fld_status fld_precondition(fld_handle *h, const double *r, double *z);

/* --- Batched form: many independent problems of uneven sizes. ------------
 * All problems share the parameters; each has its own grid, fields, dt, a,
 * adot.  Every kernel of one multigrid level covers the tiles of all
 * problems in one launch; PCG scalars, convergence and the 10x cut rule are
 * per problem. */

/* Workspace bytes for n problems with the given grids (0 if invalid). */
size_t fld_batch_workspace_bytes(int32_t n, const fld_grid *grids,
                                 const fld_params *p);

fld_status fld_batch_create(int32_t n, const fld_grid *grids,
                            const fld_params *p, void *hip_stream,
                            void *workspace, size_t workspace_bytes,
                            fld_batch **out);

/* One step for every problem i: E[i] (in/out), kappa[i], eta[i] are device
 * pointers (the pointer arrays themselves are host arrays of length n);
 * dt, a, adot are host arrays of length n.  per_problem: host array of n
 * stats, nullable.  Returns FLD_OK if every problem succeeded, else the first
 * failing problem's status (each problem's own status is in its stats; a
 * failed problem's E is unchanged).  Synchronises. */
fld_status fld_batch_step(fld_batch *b, double *const *E,
                          const double *const *kappa,
                          const double *const *eta, const double *dt,
                          const double *a, const double *adot,
                          fld_stats *per_problem);

/* fld_advance for every problem of the batch (their own dt, a, adot; the
 * same n_steps or t_end); one unit covers all problems, each with its own
 * substeps.  per_problem and steps_done: host arrays of n, nullable.
 * Returns FLD_OK if every problem succeeded, else the first failing
 * problem's status. */
fld_status fld_batch_advance(fld_batch *b, double *const *E,
                             const double *const *kappa, const double *const *eta,
                             int32_t n_steps, const double *dt, double t_end,
                             const double *a, const double *adot, int32_t units,
                             fld_stats *per_problem, int32_t *steps_done);

fld_status fld_batch_destroy(fld_batch *b);

/* --- Served form: continuous batching of solve requests. ----------------
 * A server owns a device arena given by the caller.  Requests are admitted
 * in arrival order while their workspace fits the arena; admitted requests
 * keep their multigrid hierarchy resident and advance together, one PCG
 * iteration per scheduler tick for all of them, level by level.  Finished
 * requests free their arena space at tick boundaries and waiting requests
 * join there.  A background host thread runs the scheduler. */

typedef struct fld_request {
  fld_grid grid;
  int32_t n_steps;       /* steps of length dt to take, >= 1 */
  int32_t reserved;
  double dt, a, adot;
  const double *E;       /* device FP64 E^0; read at admission */
  const double *kappa;   /* device FP64; must stay valid until completion */
  const double *eta;     /* device FP64; must stay valid until completion */
  double *E_out;         /* device FP64 result E after n_steps */
} fld_request;

typedef struct fld_result {
  int32_t status;        /* fld_status of the request */
  int32_t steps_done;
  int32_t iters;         /* PCG iterations over all steps */
  int32_t dt_cuts;
  double queue_s;        /* submit -> admission, seconds */
  double latency_s;      /* submit -> result written, seconds */
  double rel_resid;      /* last solve's true relative residual */
  double err_bound;
} fld_result;

/* arena: device memory owned by the caller (the HBM budget for resident
 * hierarchies).  Errors: FLD_EINVAL, FLD_ENOMEM (arena below the minimum),
 * FLD_EDEVICE. */
fld_status fld_server_create(const fld_params *p, void *arena,
                             size_t arena_bytes, void *hip_stream,
                             fld_server **out);

/* Queue a request (copied; its pointers must stay valid until completion).
 * Errors: FLD_EINVAL (bad grid/fields), FLD_ENOMEM (can never fit). */
fld_status fld_server_submit(fld_server *s, const fld_request *r,
                             uint64_t *ticket);

/* FLD_OK with *res filled once the request is done (or its failure status in
 * res->status), FLD_EBUSY while pending, FLD_EINVAL for an unknown ticket. */
fld_status fld_server_poll(fld_server *s, uint64_t ticket, fld_result *res);

/* Block until every submitted request is done. */
fld_status fld_server_drain(fld_server *s);

/* Stop the scheduler thread (after draining) and free host metadata. */
fld_status fld_server_destroy(fld_server *s);

#ifdef __cplusplus
}
#endif

#endif /* FLD_H_ */
