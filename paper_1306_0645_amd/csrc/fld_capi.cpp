// extern "C" entry points of the FLD library (declared in include/fld.h).
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fld.h"
#include "fld_engine.h"

using namespace fld;

struct fld_handle {
  Engine eng;
  size_t n = 0;  // finest cells
};

struct fld_batch {
  Engine eng;
};

namespace {

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  if (!a || !b) return false;
  const char *pa = (const char *)a, *pb = (const char *)b;
  return pa < pb + nb && pb < pa + na;
}

bool step_args_ok(double dt, double a, double adot) {
  return std::isfinite(dt) && dt > 0.0 && std::isfinite(a) && a > 0.0 &&
         std::isfinite(adot);
}

void fill_stats(fld_stats *s, const Job &j, int levels, int nu, int tri) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->cycle_nu = nu;
  s->trilinear = tri;
  s->status = j.status;
  s->iters = j.iters;
  s->subcycles = j.substeps;
  s->dt_cuts = j.cuts;
  s->levels = levels;
  s->restarts = j.restarts;
  s->rel_resid = j.rel_resid;
  s->err_bound = j.err_bound;
  s->rel_change_rms = j.rho;
  s->dt_next = j.dt_next;
  s->bnorm = j.bnorm;
  s->dEnorm = j.dEnorm;
}

}  // namespace

extern "C" {

void fld_default_params(fld_params *p, double c, double L_unit) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->c = c;
  p->theta = 1.0;
  p->d_max = 0.006 * c * L_unit;
  p->r_min = 1e-20 / L_unit;
  p->rtol = 1e-8;
  p->tau_tol = 1e-4;
  p->e_floor = 0.0;
  p->coarse_scale = 0.5;
  p->max_iter = 50;
  p->mg_levels = 0;
  p->nu_pre = 1;
  p->nu_post = 1;
  p->precision = FLD_PREC_FP64;
  p->max_dt_cuts = 8;
  p->tile_z = 0;
  p->check_every = 0;
  p->use_graph = 1;
  p->fused_tile_z = 0;
  p->cycle_switch = 12;
  p->prolongation = 2;
  p->warm_start = 2;
  p->tail_cells = 512;
  p->smoother = FLD_SMOOTH_RBGS;
  p->coarse_op = 0;
  p->direction_fp64 = 1;
  p->local_sweeps = 1;
  p->local_coupling = 0.98;
}

const char *fld_strerror(fld_status s) {
  switch (s) {
    case FLD_OK: return "success";
    case FLD_EINVAL: return "invalid argument";
    case FLD_ENOMEM: return "workspace or memory budget too small";
    case FLD_ENOCONV: return "linear solve did not converge";
    case FLD_ENONFINITE: return "non-finite residual (NaN/Inf in the inputs?)";
    case FLD_EDEVICE: return "HIP runtime error";
    case FLD_EBUSY: return "request still pending";
  }
  return "unknown status";
}

size_t fld_workspace_bytes(const fld_grid *g, const fld_params *p) {
  if (!g || !p || !grid_ok(*g) || !params_ok(*p)) return 0;
  std::vector<Hier> hs{make_hier(*g, *p)};
  return tables_bytes(hs) + problem_bytes(hs[0], *p);
}

fld_status fld_create(const fld_grid *g, const fld_params *p, void *hip_stream,
                      void *workspace, size_t workspace_bytes,
                      fld_handle **out) {
  if (!out) return FLD_EINVAL;
  *out = nullptr;
  if (!g || !p || !grid_ok(*g) || !params_ok(*p) || !workspace) return FLD_EINVAL;
  if (((uintptr_t)workspace) & 255) return FLD_EINVAL;
  const size_t need = fld_workspace_bytes(g, p);
  if (workspace_bytes < need) return FLD_ENOMEM;
  fld_handle *h = new (std::nothrow) fld_handle;
  if (!h) return FLD_ENOMEM;
  std::vector<fld_grid> gs{*g};
  std::vector<Hier> hs{make_hier(*g, *p)};
  Carver tbl;
  tbl.base = (char *)workspace;
  std::vector<Carver> pm(1);
  pm[0].base = (char *)workspace + tables_bytes(hs);
  const int st = h->eng.setup(*p, (hipStream_t)hip_stream, gs, tbl, pm);
  if (st) {
    delete h;
    return (fld_status)st;
  }
  h->n = (size_t)g->nx * g->ny * g->nz;
  *out = h;
  return FLD_OK;
}

fld_status fld_assemble(fld_handle *h, const double *E_n, const double *kappa,
                        const double *eta, double dt, double a, double adot) {
  if (!h || !E_n || !kappa || !eta || !step_args_ok(dt, a, adot)) return FLD_EINVAL;
  Engine &e = h->eng;
  e.fill_step(0, E_n, kappa, eta, dt, a, adot);
  e.prev_ok[0] = 0;  // a cold solve overwrites the warm-start guess
  int st = e.upload_sd_sc();
  if (st) return (fld_status)st;
  e.enqueue_assemble(e.all);
  if (hipGetLastError() != hipSuccess) return FLD_EDEVICE;
  e.assembled = true;
  return FLD_OK;
}

fld_status fld_solve(fld_handle *h, double *dE, fld_stats *stats) {
  if (!h || !dE) return FLD_EINVAL;
  Engine &e = h->eng;
  if (!e.assembled) return FLD_EINVAL;
  const StepDev &S = e.h_sd[0];
  const size_t nb = h->n * sizeof(double);
  if (overlaps(dE, nb, S.E, nb) || overlaps(dE, nb, S.kappa, nb) ||
      overlaps(dE, nb, S.eta, nb))
    return FLD_EINVAL;
  int st = e.run_solve();
  if (st) return (fld_status)st;
  const Scal sc = e.h_sc[0];
  e.h_sd[0].Eout = dE;
  e.h_sc[0].live = 1;
  st = e.upload_sd_sc();
  if (st) return (fld_status)st;
  launch_update_E(e.T, e.all.fine, 0.0, 1, e.stream);
  launch_fin(e.T, FIN_STEP, e.mixed, e.stream);
  st = e.download_sc();
  if (st) return (fld_status)st;
  Job j;
  j.status = sc.status;
  j.iters = sc.iter;
  j.restarts = sc.restarts;
  j.substeps = 1;
  j.bnorm = std::sqrt(sc.bb);
  j.dEnorm = std::sqrt(e.h_sc[0].dEdE);
  const double rr = sc.phase == PH_DONE && sc.status == ST_OK ? sc.rr_true : sc.rr;
  j.rel_resid = sc.bb > 0.0 ? std::sqrt(rr / sc.bb) : 0.0;
  j.err_bound = j.dEnorm > 0.0 ? std::sqrt(rr) / j.dEnorm : 0.0;
  fill_stats(stats, j, e.hier[0].levels, e.last_nu, e.last_tri);
  e.h_sc[0].live = 1;  // the assembled system stays available
  return (fld_status)sc.status;
}

fld_status fld_step(fld_handle *h, double *E, const double *kappa,
                    const double *eta, double dt, double a, double adot,
                    fld_stats *stats) {
  if (!h || !E || !kappa || !eta || !step_args_ok(dt, a, adot)) return FLD_EINVAL;
  Engine &e = h->eng;
  const size_t nb = h->n * sizeof(double);
  if (overlaps(E, nb, kappa, nb) || overlaps(E, nb, eta, nb)) return FLD_EINVAL;
  std::vector<Job> jobs(1);
  Job &j = jobs[0];
  j.E = E;
  j.kappa = kappa;
  j.eta = eta;
  j.dt = dt;
  j.a = a;
  j.adot = adot;
  j.h = dt;
  const int st = e.run_steps(jobs);
  if (st) return (fld_status)st;
  e.assembled = true;
  fill_stats(stats, j, e.hier[0].levels, e.last_nu, e.last_tri);
  return (fld_status)j.status;
}

fld_status fld_advance(fld_handle *h, double *E, const double *kappa,
                       const double *eta, int32_t n_steps, double dt, double t_end,
                       double a, double adot, int32_t units, fld_stats *stats,
                       int32_t *steps_done) {
  if (!h || !E || !kappa || !eta || !step_args_ok(dt, a, adot)) return FLD_EINVAL;
  if (n_steps < 0 || units < 0) return FLD_EINVAL;
  if (n_steps == 0 && !(std::isfinite(t_end) && t_end > 0.0)) return FLD_EINVAL;
  Engine &e = h->eng;
  const size_t nb = h->n * sizeof(double);
  if (overlaps(E, nb, kappa, nb) || overlaps(E, nb, eta, nb)) return FLD_EINVAL;
  std::vector<Job> jobs(1);
  Job &j = jobs[0];
  j.E = E;
  j.kappa = kappa;
  j.eta = eta;
  j.dt = dt;
  j.a = a;
  j.adot = adot;
  const int st = e.run_advance(jobs, n_steps, n_steps == 0, t_end, units ? units : 8);
  if (st) return (fld_status)st;
  e.assembled = true;
  fill_stats(stats, j, e.hier[0].levels, e.prm.nu_pre, e.trilinear());
  if (steps_done) *steps_done = j.steps;
  return (fld_status)j.status;
}

fld_status fld_destroy(fld_handle *h) {
  if (!h) return FLD_EINVAL;
  if (h->eng.stream) hipStreamSynchronize(h->eng.stream);
  else hipDeviceSynchronize();
  delete h;
  return FLD_OK;
}

fld_status fld_get_system(fld_handle *h, double *diag, double *Tx, double *Ty,
                          double *Tz, double *b) {
  if (!h || !h->eng.assembled) return FLD_EINVAL;
  Engine &e = h->eng;
  const size_t nb = h->n * sizeof(double);
  const LevelDev &L = e.mem[0].lv[0];
  const double *src[5] = {L.diag, L.Tx, L.Ty, L.Tz, e.mem[0].pd.b};
  double *dst[5] = {diag, Tx, Ty, Tz, b};
  for (int i = 0; i < 5; ++i)
    if (dst[i] && hipMemcpyAsync(dst[i], src[i], nb, hipMemcpyDeviceToDevice,
                                 e.stream) != hipSuccess)
      return FLD_EDEVICE;
  if (hipStreamSynchronize(e.stream) != hipSuccess) return FLD_EDEVICE;
  return FLD_OK;
}

fld_status fld_apply(fld_handle *h, const double *u, double *out) {
  if (!h || !u || !out || !h->eng.assembled) return FLD_EINVAL;
  const size_t nb = h->n * sizeof(double);
  if (overlaps(u, nb, out, nb)) return FLD_EINVAL;
  Engine &e = h->eng;
  launch_apply(e.T, e.all.fine, u, out, e.stream);
  if (hipGetLastError() != hipSuccess) return FLD_EDEVICE;
  if (hipStreamSynchronize(e.stream) != hipSuccess) return FLD_EDEVICE;
  return FLD_OK;
}

fld_status fld_precondition(fld_handle *h, const double *r, double *z) {
  if (!h || !r || !z || !h->eng.assembled) return FLD_EINVAL;
  const size_t nb = h->n * sizeof(double);
  if (overlaps(r, nb, z, nb)) return FLD_EINVAL;
  Engine &e = h->eng;
  launch_set_r(e.T, e.all.fine, r, e.mixed, e.stream);
  launch_fin(e.T, FIN_SETR, e.mixed, e.stream);
  e.enqueue_vcycle(e.all);
  const ProbDev &P = e.mem[0].pd;
  if (e.mixed) {
    launch_z_out(e.T, e.all.fine, z, e.stream);
    if (hipGetLastError() != hipSuccess) return FLD_EDEVICE;
  } else if (hipMemcpyAsync(z, P.z, nb, hipMemcpyDeviceToDevice, e.stream) != hipSuccess) {
    return FLD_EDEVICE;
  }
  int st = e.download_sc();  // also syncs
  if (st) return (fld_status)st;
  // the solve state was overwritten: a new fld_assemble is needed to solve
  e.h_sc[0].phase = PH_DONE;
  e.h_sc[0].active = 0;
  st = e.upload_sd_sc();
  if (st) return (fld_status)st;
  e.assembled = false;
  if (hipStreamSynchronize(e.stream) != hipSuccess) return FLD_EDEVICE;
  return FLD_OK;
}

// ---------------------------------------------------------------- batch ---

size_t fld_batch_workspace_bytes(int32_t n, const fld_grid *grids,
                                 const fld_params *p) {
  if (n < 1 || !grids || !p || !params_ok(*p)) return 0;
  std::vector<Hier> hs;
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    if (!grid_ok(grids[i])) return 0;
    hs.push_back(make_hier(grids[i], *p));
    total += problem_bytes(hs.back(), *p);
  }
  return tables_bytes(hs) + total;
}

fld_status fld_batch_create(int32_t n, const fld_grid *grids,
                            const fld_params *p, void *hip_stream,
                            void *workspace, size_t workspace_bytes,
                            fld_batch **out) {
  if (!out) return FLD_EINVAL;
  *out = nullptr;
  const size_t need = fld_batch_workspace_bytes(n, grids, p);
  if (!need || !workspace || (((uintptr_t)workspace) & 255)) return FLD_EINVAL;
  if (workspace_bytes < need) return FLD_ENOMEM;
  fld_batch *b = new (std::nothrow) fld_batch;
  if (!b) return FLD_ENOMEM;
  std::vector<fld_grid> gs(grids, grids + n);
  std::vector<Hier> hs;
  for (int i = 0; i < n; ++i) hs.push_back(make_hier(grids[i], *p));
  Carver tbl;
  tbl.base = (char *)workspace;
  std::vector<Carver> pm(n);
  size_t off = tables_bytes(hs);
  for (int i = 0; i < n; ++i) {
    pm[i].base = (char *)workspace + off;
    off += problem_bytes(hs[i], *p);
  }
  const int st = b->eng.setup(*p, (hipStream_t)hip_stream, gs, tbl, pm);
  if (st) {
    delete b;
    return (fld_status)st;
  }
  *out = b;
  return FLD_OK;
}

fld_status fld_batch_step(fld_batch *b, double *const *E,
                          const double *const *kappa, const double *const *eta,
                          const double *dt, const double *a, const double *adot,
                          fld_stats *per_problem) {
  if (!b || !E || !kappa || !eta || !dt || !a || !adot) return FLD_EINVAL;
  Engine &e = b->eng;
  const int n = (int)e.hier.size();
  std::vector<Job> jobs(n);
  for (int i = 0; i < n; ++i) {
    if (!E[i] || !kappa[i] || !eta[i] || !step_args_ok(dt[i], a[i], adot[i]))
      return FLD_EINVAL;
    const size_t nb = (size_t)e.hier[i].cells(0) * sizeof(double);
    if (overlaps(E[i], nb, kappa[i], nb) || overlaps(E[i], nb, eta[i], nb))
      return FLD_EINVAL;
    Job &j = jobs[i];
    j.E = E[i];
    j.kappa = kappa[i];
    j.eta = eta[i];
    j.dt = dt[i];
    j.a = a[i];
    j.adot = adot[i];
    j.h = dt[i];
  }
  const int st = e.run_steps(jobs);
  if (st) return (fld_status)st;
  e.assembled = true;
  int first = FLD_OK;
  for (int i = 0; i < n; ++i) {
    if (per_problem) fill_stats(&per_problem[i], jobs[i], e.hier[i].levels, e.last_nu, e.last_tri);
    if (jobs[i].status != FLD_OK && first == FLD_OK) first = jobs[i].status;
  }
  return (fld_status)first;
}

fld_status fld_batch_advance(fld_batch *b, double *const *E,
                             const double *const *kappa, const double *const *eta,
                             int32_t n_steps, const double *dt, double t_end,
                             const double *a, const double *adot, int32_t units,
                             fld_stats *per_problem, int32_t *steps_done) {
  if (!b || !E || !kappa || !eta || !dt || !a || !adot) return FLD_EINVAL;
  if (n_steps < 0 || units < 0) return FLD_EINVAL;
  if (n_steps == 0 && !(std::isfinite(t_end) && t_end > 0.0)) return FLD_EINVAL;
  Engine &e = b->eng;
  const int n = (int)e.hier.size();
  std::vector<Job> jobs(n);
  for (int i = 0; i < n; ++i) {
    if (!E[i] || !kappa[i] || !eta[i] || !step_args_ok(dt[i], a[i], adot[i]))
      return FLD_EINVAL;
    const size_t nb = (size_t)e.hier[i].cells(0) * sizeof(double);
    if (overlaps(E[i], nb, kappa[i], nb) || overlaps(E[i], nb, eta[i], nb))
      return FLD_EINVAL;
    Job &j = jobs[i];
    j.E = E[i];
    j.kappa = kappa[i];
    j.eta = eta[i];
    j.dt = dt[i];
    j.a = a[i];
    j.adot = adot[i];
  }
  const int st = e.run_advance(jobs, n_steps, n_steps == 0, t_end, units ? units : 8);
  if (st) return (fld_status)st;
  e.assembled = true;
  int first = FLD_OK;
  for (int i = 0; i < n; ++i) {
    if (per_problem)
      fill_stats(&per_problem[i], jobs[i], e.hier[i].levels, e.prm.nu_pre, e.trilinear());
    if (steps_done) steps_done[i] = jobs[i].steps;
    if (jobs[i].status != FLD_OK && first == FLD_OK) first = jobs[i].status;
  }
  return (fld_status)first;
}

fld_status fld_batch_destroy(fld_batch *b) {
  if (!b) return FLD_EINVAL;
  if (b->eng.stream) hipStreamSynchronize(b->eng.stream);
  else hipDeviceSynchronize();
  delete b;
  return FLD_OK;
}

}  // extern "C"
