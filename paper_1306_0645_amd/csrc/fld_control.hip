// Device-side step control (Sec. 3.4): the radiation subcycling loop and the
// step-size controller run on the GPU, so that a run of many steps needs no
// host round trip per substep (fld_advance).
//
// The host captures a graph of `units`; each unit, for every problem whose
// state asks for it, does: the assembly of the next substep (and its warm
// start), one PCG iteration, the true-residual verification, E += dE on
// success, then this controller, then the copy of a finished run's E.  All
// kernels read the per-problem state from device memory and return at once
// where it does not apply, so a problem moves from substep to substep, and
// from step to step, inside the graph; the host reads the state once per
// graph.  The controller's arithmetic is the host driver's (Engine::run_steps
// and set_warm / note_success), operation for operation, so the device-run
// steps equal the host-run ones bit for bit.
#include "fld_device.h"

namespace fld {

// the next substep of problem p: its length, the E it starts from and the E
// it writes, and its warm-start guess (the buffers rotate as on the host)
__device__ void next_substep(const Tables &T, int p, CtlDev &c, const CtlParams &cp) {
#pragma clang fp contract(off)
  StepDev &S = T.sd[p];
  ProbDev &P = T.pd[p];
  c.h = fmin(c.h, c.dt - c.t);
  S.E = c.in_work ? P.Ework : c.E;
  S.dt = c.h;
  S.warm = 0.0;
  S.w1 = S.w2 = 0.0;
  S.h1 = S.h2 = nullptr;
  c.warm_now = 0;
  if (cp.warm_start && c.prev_ok >= 1 && c.prev_h > 0.0) {
    c.warm_now = 1;
    const double h1 = c.prev_h, r1 = c.h / h1;
    S.warm = cp.warm_start;
    S.w1 = r1;
    S.w2 = 0.0;
    const bool two = c.prev_ok >= 2 && c.prev_h2 > 0.0 && c.xold >= 0;
    if (two) {
      const double h0 = c.prev_h2;
      const double tau = (h1 + c.h) / (h0 + h1);
      S.w1 = r1 * (1.0 + tau);
      S.w2 = -(c.h / h0) * tau;
    }
    const int a = c.xcur, b = two ? c.xold : -1;
    int nxt = 0;
    while (nxt == a || nxt == b) ++nxt;
    S.h1 = P.xb[a];
    S.h2 = two ? P.xb[b] : nullptr;
    P.x = P.xb[nxt];
    c.xold = a;
    c.xcur = nxt;
  }
  const bool last = c.dt - (c.t + c.h) <= 1e-12 * c.dt;
  c.target = (!c.in_work && last) ? 1 : 2;
  S.Eout = c.target == 1 ? c.E : P.Ework;
  Scal &sc = T.sc[p];
  sc.stage = 1;
  sc.live = 1;
}

__device__ void finish_run(Scal &sc, CtlDev &c, int status) {
  c.done = 1;
  c.status = status;
  sc.live = 0;
  sc.stage = 0;
}

// One block per problem; thread 0 decides.  Acts once per decided substep:
// on success the substep is accounted (Sec. 3.4: t_rad += dt_rad, dt_rad
// from the relative change against tau_tol), on failure dt_rad is cut by
// 10x; then the next substep (or step) is set up, or the run ends.
__global__ __launch_bounds__(64) void k_control(Tables T, CtlParams cp) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0) return;
  const int p = blockIdx.x;
  Scal &sc = T.sc[p];
  CtlDev &c = T.ctl[p];
  if (!sc.ctl || c.done) return;
  c.copy_due = 0;
  if (sc.stage != 0 || sc.phase != PH_DONE) return;  // substep undecided
  c.iters += sc.iter;
  c.restarts += sc.restarts;
  if (sc.status == ST_OK) {
    c.prev_ok = c.warm_now ? 2 : 1;
    c.prev_h2 = c.prev_h;
    c.prev_h = c.h;
    const double n = (double)T.pd[p].n;
    c.substeps += 1;
    c.t += c.h;
    c.rho = sqrt(sc.change2 / n);
    double f = c.rho > 0.0 ? cp.tau_tol / c.rho : 2.0;
    f = fmin(2.0, fmax(0.1, f));
    c.bnorm = sqrt(sc.bb);
    c.dEnorm = sqrt(sc.dEdE);
    c.rel_resid = sc.bb > 0.0 ? sqrt(sc.rr_true / sc.bb) : 0.0;
    c.err_bound = c.dEnorm > 0.0 ? sqrt(sc.rr_true) / c.dEnorm : 0.0;
    if (c.target == 2) c.in_work = 1;
    c.h *= f;
    c.dt_next = c.h;
    if (c.dt - c.t <= 1e-12 * c.dt) {
      // the step is covered
      if (c.in_work) c.copy_due = 1;
      c.steps += 1;
      c.t_total += c.dt;
      const bool over = c.adaptive ? c.t_end - c.t_total <= 1e-12 * c.t_end
                                   : c.steps >= c.n_steps;
      if (over) {
        finish_run(sc, c, ST_OK);
        return;
      }
      c.dt = c.adaptive ? fmin(c.dt_next, c.t_end - c.t_total) : c.dt0;
      c.t = 0.0;
      c.h = c.dt;
      c.cuts = 0;
      c.in_work = 0;
    }
  } else if (c.cuts < cp.max_dt_cuts) {
    c.prev_ok = 0;
    c.h *= 0.1;
    c.cuts += 1;
    c.cuts_total += 1;
  } else {
    c.prev_ok = 0;
    finish_run(sc, c, sc.status != ST_OK ? sc.status : ST_ENOCONV);
    return;
  }
  next_substep(T, p, c, cp);
}

// E = Ework for a problem whose run (or step) ended in the working copy
__global__ __launch_bounds__(kBlock) void k_copy_E(Tables T, TileList TL) {
  const Tile t = get_tile(TL);
  const CtlDev &c = T.ctl[t.prob];
  if (!T.sc[t.prob].ctl || !c.copy_due) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const Col col = tile_col(t);
  if (!col.on) return;
  const int plane = L.nx * L.ny;
  int g = t.z0 * plane + col.j * L.nx + col.i;
  for (int k = 0; k < t.tz; ++k, g += plane) c.E[g] = P.Ework[g];
}

void launch_control(const Tables &T, CtlParams cp, hipStream_t s) {
  if (T.nprob) FLD_LAUNCH(K_CONTROL, k_control, T.nprob, 64, s, T, cp);
}

void launch_copy_E(const Tables &T, TileList L0, hipStream_t s) {
  if (L0.nblocks) FLD_LAUNCH(K_COPY_E, k_copy_E, L0.nblocks, kBlock, s, T, L0);
}

}  // namespace fld
