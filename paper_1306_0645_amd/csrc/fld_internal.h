// Internal declarations of the FLD library: device-side descriptor tables
// shared by the HIP kernels and the host engine, and the kernel launchers.
//
// Every kernel works on a list of tiles.  A tile is a box of at most 256
// (x, y) columns and tz planes of one multigrid level of one problem, so the
// same kernel serves one large problem, a batch of uneven problems, and the
// changing set of a request server: the host only rebuilds the lists.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fld {

constexpr int kBlock = 256;          // threads per tile block (4 wave64)
constexpr int kFinBlock = 1024;      // threads of the per-problem finalize
constexpr int kTailBlock = 1024;     // threads of the V-cycle tail kernel
constexpr int kMaxLevels = 12;

// Status values (same numbers as the public fld_status).
enum : int {
  ST_OK = 0,
  ST_EINVAL = -1,
  ST_ENOMEM = -2,
  ST_ENOCONV = -3,
  ST_ENONFINITE = -4,
  ST_EDEVICE = -5,
  ST_EBUSY = -6
};

// Phase of one problem's PCG solve (Scal::phase).
enum : int {
  PH_ITER = 0,     // iterating
  PH_VERIFY = 1,   // recursive residual met the tolerance; true residual pending
  PH_DONE = 2      // final status decided
};

// One multigrid level of one problem.
struct LevelDev {
  int nx, ny, nz, n;
  double *Tx, *Ty, *Tz, *diag;       // FP64: -A_{p,p+e_d} on +faces; A_pp
  float *Tx32, *Ty32, *Tz32, *diag32;// FP32 copies (mixed precision)
  void *x;                           // V-cycle iterate (level precision);
                                     // finest level FP64 mode: aliases z
  void *f;                           // V-cycle right-hand side (levels >= 1)
  void *x2;                          // second iterate buffer (Jacobi smoother)
};

// One problem's finest-level Krylov state.
struct ProbDev {
  int nx, ny, nz, n;
  double *x, *r, *q, *b;
  double *z;             // FP64 form (null in the mixed form)
  double *p0, *p1;       // FP64 direction (FP64 form; mixed with direction_fp64)
  // mixed form: the V-cycle's FP32 output as it is, z = zscale * z32, and
  // the search direction either in FP32 at the scale of the z it was formed
  // from, p = pscale * pf0 (or pf1), or in FP64 in p0 / p1
  float *z32, *pf0, *pf1;
  double *r2;            // second residual buffer (fused V(1,1) iteration)
  // local smoothing (mixed fused cycle): the cells whose coupling to the
  // neighbours dominates the diagonal (sum of faces > local_coupling x
  // diagonal), listed per finest tile at the tile's own cells, and the
  // counts per tile and colour, lcnt[2 (t - t0) + colour] (k_lmask); kept
  // with the problem, since a server's tables are rebuilt between the
  // assembly and the sweeps that read them
  int *llist, *lcnt;
  double *cs;            // coarsest-level CG scratch: 4 * n_coarsest doubles
  int levels;            // number of multigrid levels
  int t0, t1;            // range of this problem's tiles in the finest list
  int f0, f1;            // range of its fused-cycle finest tiles
  int spf;               // the fused iteration's SpMV runs on the fused tiles
  int tail;              // first level of the single-workgroup V-cycle tail
  double *xb[3];         // the dE buffers (iterate and warm-start history)
  double *Ework;         // working copy of E while a step is subcycled
};

// Per-step inputs of one problem (uploaded by the host at each assembly).
struct StepDev {
  const double *E, *kappa, *eta;
  double *Eout;          // destination of E + dE (may equal E)
  double dt, adot_a;     // dt and adot/a
  double idx, idy, idz;  // 1 / dx, 1 / dy, 1 / dz (comoving cell sizes)
  // warm start: 0: x0 = 0; 1: x0 = w1 dE(n) + w2 dE(n-1) (extrapolation);
  // 2: x0 = c1 dE(n) + c2 dE(n-1) with c from the Galerkin condition in the
  // new operator, (dE(i), A dE(j)) c_j = (dE(i), b)
  double warm;
  double w1, w2;
  const double *h1, *h2; // dE(n), dE(n-1) (h2 null when w2 = 0); never P.x
};

// Per-problem PCG scalars (device resident, read back by the host).
struct Scal {
  double bb, rr, rho, rho_old, rzo, pq, alpha, beta;
  double s, inv_s;       // residual scale for the FP32 V-cycle
  double rr_true, tol2;  // true residual^2; rtol^2
  double change2;        // sum of (dE / max(|E|, floor))^2
  double dEdE;           // ||dE||^2
  double s_next;         // residual scale for the next V-cycle (snew set)
  double zscale;         // mixed form: z = zscale * z32 (the s its cycle ran at)
  double pscale;         // mixed form: newest p = pscale * pf (its z's zscale)
  double c1, c2;         // Galerkin warm guess x0 = c1 dE(n) + c2 dE(n-1)
  int iter, max_iter, phase, status;
  int active, restart, pbuf, restarts;
  int live;              // takes part in the current assembly / update
  int cold;              // the warm guess did not reduce ||r||: start from 0
  // fused iteration: the residual lives in r (rbuf = 0) or r2 (rbuf = 1);
  // has_dir: alpha, p and q of a previous iteration exist, so the down pass
  // forms r - alpha q; xlag: x still lacks alpha p (added by the next SpMV,
  // or by k_xfix when the iteration stops)
  int rbuf, has_dir, xlag, snew;
  int fresh;             // (re)started: the finest down pass is still due
  int committed;         // E += dE of this solve is done (FIN_STEP)
  // device-controlled stepping (fld_advance): ctl = 1 while the device runs
  // the substeps; stage 1: the next substep's assembly is due, 2: its warm
  // start is due, 0: neither (iterating, verifying, or done)
  int ctl, stage;
};

// Device-side step control of one problem (fld_advance): the requested run,
// its progress, and the warm-start history the host keeps otherwise.
struct CtlDev {
  double *E;             // the caller's E: E^0 in, E after the last step out
  double dt0, t_end;     // step size (adaptive: the first step's); end time
  int n_steps, adaptive; // fixed steps of dt0, or steps of the controller's
                         // dt_next until t_end
  int done, status;      // the run is over; its status
  double t, h, dt;       // time reached in the current step, the substep
                         // being taken, the current step's size
  double t_total;        // time covered by the completed steps
  int steps, substeps, cuts, cuts_total, iters, restarts;
  int in_work, target;   // E lives in Ework; the substep writes E (1) or Ework (2)
  int copy_due;          // the run's E is in Ework: copy it to E
  int prev_ok, xcur, xold, warm_now;
  double prev_h, prev_h2;
  double rho, dt_next, rel_resid, err_bound, bnorm, dEnorm;
};

// A tile: cells [x0, x0+tx) x [y0, y0+ty) x [z0, z0+tz) of one level of one
// problem.  Each thread owns cpt consecutive x cells of one row and walks the
// tile's planes.
struct Tile {
  int prob;
  int x0, y0, z0;
  int tx, ty, tz;
  int cpt;
};

// Launch context: the tables live in device memory.
// per-tile sums of the assembly: ||b||^2, ||b - A x0||^2 (extrapolated
// guess), and for the Galerkin guess (h_i, A h_j) and (h_i, b), h = dE(n),
// dE(n-1)
enum : int { AS_BB, AS_RR, AS_G11, AS_G12, AS_G22, AS_B1, AS_B2, kAsmSums };

struct Tables {
  LevelDev *lv;     // [kMaxLevels][nprob]
  ProbDev *pd;      // [nprob]
  StepDev *sd;      // [nprob]
  Scal *sc;         // [nprob]
  double *part;     // [n finest tiles][2] block partial sums
  double *lpart;    // [n finest tiles][2] the local sweeps' r.z changes
  CtlDev *ctl;      // [nprob] device-side step control
  double *gpart;    // [n finest tiles][kAsmSums] sums of the assembly
  int nprob;
};

// A launch covers a subset of the full tile table: ranges[2r] is the first
// block of range r, ranges[2r+1] the tile it maps to; ranges are sorted by
// block.  nblocks = total blocks of the launch.
struct TileList {
  const Tile *base;     // device: full tile table
  const int *ranges;    // device: 2 * nranges ints
  int nranges;
  int nblocks;
};

// ---- kernel ids of the timing hook (include/fld_profile.h) ----------------
enum : int {
  K_ASSEMBLE, K_COARSEN, K_FIN, K_PRE0_F, K_PRE0_C, K_HALF_F, K_HALF_C,
  K_HALF_OUT, K_RESTRICT_F, K_RESTRICT_C, K_PROLONG_F, K_PROLONG_C,
  K_COARSE_SOLVE, K_SPMV_P, K_UPDATE, K_TRUE_RESID, K_APPLY, K_SET_R,
  K_UPDATE_E, K_VDOWN_F, K_VDOWN_C, K_VUP_F, K_VUP_C, K_CHEM_H, K_ION_SUM,
  K_WARM_REVERT, K_JACOBI0_F, K_JACOBI_F, K_JACOBI_OUT,
  K_JACOBI_C, K_PROLONG_ADD_F, K_PROLONG_ADD_C, K_SPMV_PX, K_XFIX, K_WARM_X,
  K_LMASK, K_LOCAL, K_CONTROL, K_COPY_E, K_NUM
};

// Brackets one launch with hipEvents when its kernel id is selected.
struct ProfScope {
  ProfScope(int k, hipStream_t s);
  ~ProfScope();
  int k;
  hipStream_t s;
  hipEvent_t a;
};

#define FLD_LAUNCH(id, kern, grid, block, s, ...)                         \
  do {                                                                    \
    ::fld::ProfScope _ps((id), (s));                                      \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, __VA_ARGS__); \
  } while (0)

// ---- launchers (fld_kernels.hip, fld_fused.hip) ---------------------------
// prec: 0 = FP64 V-cycle, 1 = FP32 V-cycle.
void launch_assemble(const Tables &T, TileList L0, double c, double theta,
                     double dmax, double rmin, int mixed, hipStream_t s);
// op: 0 = coarse faces from the 4 fine faces they cover, 1 = from the fine
// rows through them, three faces in series (k_coarsen)
void launch_coarsen(const Tables &T, TileList coarse, int lc, double scale,
                    int mixed, int op, hipStream_t s);
// alt: FIN_RZ and FIN_RR2 read the partials of the fused finest tiles; FIN_PQ
// with alt marks the fused iteration's deferred updates
void launch_fin(const Tables &T, int which, int mixed, hipStream_t s,
                int alt = 0);
void launch_pre0(const Tables &T, TileList L, int l, int prec, hipStream_t s);
void launch_half(const Tables &T, TileList L, int l, int colour, int prec,
                 hipStream_t s);
void launch_half_out(const Tables &T, TileList L0, int prec, int flexible,
                     hipStream_t s);
void launch_resid_restrict(const Tables &T, TileList coarse, int lc, int prec,
                           hipStream_t s);
void launch_prolong_black(const Tables &T, TileList L, int l, int prec,
                          int trilinear, hipStream_t s);
void launch_vtail(const Tables &T, int prec, int nu_pre, int nu_post,
                  int trilinear, hipStream_t s);
// weighted Jacobi smoother: mode 0 = first sweep from x = 0, 1 = sweep,
// 2 = last finest-level sweep writing z and the r.z partials (in = x2);
// in_x2 selects the input buffer, the output is the other one
void launch_jacobi(const Tables &T, TileList L, int l, int prec, int mode,
                   int in_x2, int flexible, hipStream_t s);
// x (or x2) = x + P e: the coarse-grid correction of every cell
void launch_prolong_add(const Tables &T, TileList L, int l, int prec,
                        int trilinear, int to_x2, hipStream_t s);
// Krylov storage of the finest level (Engine::kmode): 0 = FP64 z and p,
// 1 = mixed form with FP32 z and p (each at a per-problem scale), 2 = mixed
// form with FP32 z and an FP64 search direction p
// lazy = 1 (fused iteration): also x += alpha p_old, the update deferred
// from the previous iteration (mixed forms only)
// the fused iteration's SpMV (x += alpha p_old, p = z + beta p_old, q = A p)
// on the finest fused tiles; its partials sum over the fused range
void launch_spmv_f(const Tables &T, TileList F0, int km, hipStream_t s);
void launch_spmv_p(const Tables &T, TileList L0, int lazy, int km, hipStream_t s);
// out = s * z32 right after a mixed-form V-cycle (the preconditioner alone)
void launch_z_out(const Tables &T, TileList L0, double *out, hipStream_t s);
// x += alpha p for problems that stopped iterating with the update pending
void launch_xfix(const Tables &T, TileList L0, int km, hipStream_t s);
void launch_update(const Tables &T, TileList L0, int km, hipStream_t s);
void launch_true_resid(const Tables &T, TileList L0, hipStream_t s);
void launch_warm_revert(const Tables &T, TileList L0, hipStream_t s);
// x0 = c1 dE(n) + c2 dE(n-1), r = b - A x0 (Galerkin warm guesses)
void launch_warm_x(const Tables &T, TileList L0, hipStream_t s);
// local smoothing of the mixed fused cycle: the list of strongly coupled
// finest cells (after the assembly), and one red/black sweep over them
// (colour 1 = black, then 0 = red) after the finest post-sweep, in z32,
// with the change of r.z per tile in lpart[2 t + colour]
void launch_lmask(const Tables &T, TileList L0, double coupling, hipStream_t s);
void launch_local(const Tables &T, TileList L0, int colour, hipStream_t s);
// device-controlled stepping (fld_control.hip): the controller after each
// unit's verification and commit (one block per problem), and the copy of a
// finished run's E from the working copy
struct CtlParams {
  double tau_tol;
  int max_dt_cuts;
  int warm_start;
};
void launch_control(const Tables &T, CtlParams cp, hipStream_t s);
void launch_copy_E(const Tables &T, TileList L0, hipStream_t s);
void launch_apply(const Tables &T, TileList L0, const double *u, double *out,
                  hipStream_t s);
void launch_set_r(const Tables &T, TileList L0, const double *r, int prec,
                  hipStream_t s);
// in_solve: right after a verification, for the problems it just decided
// (FIN_STEP then takes alt = 1)
void launch_update_E(const Tables &T, TileList L0, double floor, int copy_only,
                     hipStream_t s, int in_solve = 0);
// fused one-sweep V-cycle passes (fld_fused.hip)
// sel (finest level of the rotated fused iteration): VD_ALL every active
// problem, VD_FRESH those starting or restarting, VD_CONT the others
enum : int { VD_ALL = 0, VD_FRESH = 1, VD_CONT = 2 };
void launch_vdown(const Tables &T, TileList L, int l, int prec, int sel,
                  hipStream_t s);
void launch_vup(const Tables &T, TileList L, int l, int prec, int flexible,
                int trilinear, hipStream_t s);

// finalize kernels (launch_fin 'which')
enum : int {
  FIN_BB = 0,     // after assembly (its own kernel): ||b||^2 and the warm
                  // guess's sums, start the solve
  FIN_RZ = 1,     // after the V-cycle: rho = r.z, beta
  FIN_PQ = 2,     // after the SpMV: alpha = rho / p.q
  FIN_RR = 3,     // after the update: ||r||^2, convergence
  FIN_TRUE = 4,   // after the true residual: verify or restart
  FIN_STEP = 5,   // after E += dE: relative change and ||dE||^2
  FIN_SETR = 6,   // after loading an external r (preconditioner test)
  FIN_RR2 = 8,    // fused iteration, after the down pass formed r - alpha q:
                  // ||r||^2, convergence, switch the residual buffer
  FIN_XFIX = 9,   // after k_xfix: the deferred x update is done
  FIN_FRESH = 10, // after the prologue's down pass: the problems iterate on
  FIN_WARM = 11,  // after k_warm_x: keep the projected guess if it reduces
                  // the residual
  FIN_STAGE = 12  // device-controlled stepping: the substep's warm start is
                  // done, its PCG runs on
  // (FIN_RZ with alt = 2: the fused cycle's partials plus the local sweeps')
};

}  // namespace fld
