// Served form: continuous batching of FLD step requests.
//
// A scheduler thread owns a device arena given by the caller.  Requests are
// admitted in arrival order while their workspace fits the free arena (a
// later, smaller request may pass one that does not fit, but a request that
// has been passed kMaxBypass times blocks further passing).  Admitted
// requests keep their multigrid hierarchy and their copy of E resident and
// advance together: every tick assembles the requests that start a substep,
// runs one PCG iteration for every request that is solving (one launch per
// kernel and multigrid level covers all of them), verifies converged ones
// with the true FP64 residual, and commits finished solves.  Requests that
// finish free their arena space at the tick boundary, where waiting requests
// join.  Per-problem arithmetic is independent of the other residents, so a
// request's result is the same alone and in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fld.h"
#include "fld_engine.h"

using namespace fld;

namespace {

constexpr int kMaxBypass = 4;
constexpr size_t kMinArena = 1 << 20;

double now_s() {
  return std::chrono::duration<double>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// first-fit allocator over [0, size) with coalescing, 256-byte granules
class ArenaAlloc {
 public:
  void init(size_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t n, size_t &off) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        off = it->first;
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto &kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<size_t, size_t> free_;
};

enum { RQ_QUEUED = 0, RQ_ASSEMBLE = 1, RQ_SOLVING = 2, RQ_DONE = 3 };

struct Req {
  uint64_t ticket = 0;
  fld_request r{};
  Hier hier;
  size_t bytes = 0, off = 0;
  int state = RQ_QUEUED;      // RQ_DONE is set under the server lock
  bool finished = false;      // outcome recorded by the worker
  int bypassed = 0;
  int step = 0;
  Job job;
  Scal sc{};
  // warm-start history across engine rebuilds (Engine::set_warm)
  char prev_ok = 0, warm_now = 0;
  double prev_h = 0, prev_h2 = 0;
  int xcur = 0, xold = -1;
  double t_submit = 0, t_admit = 0, t_done = 0;
  fld_result res{};
};

}  // namespace

struct fld_server {
  fld_params prm{};
  char *arena = nullptr;
  size_t arena_bytes = 0;
  hipStream_t stream = nullptr;
  ArenaAlloc alloc;
  size_t tables_off = 0, tables_sz = 0;
  bool have_tables = false;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> queue;             // waiting, arrival order
  std::vector<Req *> resident;         // admitted, in admission order
  std::unordered_map<uint64_t, Req *> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  int pending = 0;                     // submitted and not finished
  std::thread worker;
  Engine *eng = nullptr;

  void run();
  int tick();
  int rebuild();
  void finish(Req *q, int status);
};

// Record a request's outcome (worker thread); it is published to pollers
// under the lock at the end of the tick.
void fld_server::finish(Req *q, int status) {
  q->t_done = now_s();
  q->finished = true;
  q->res.status = status;
  q->res.steps_done = q->step;
  q->res.iters = q->job.iters;
  q->res.dt_cuts = q->job.cuts;
  q->res.queue_s = q->t_admit - q->t_submit;
  q->res.latency_s = q->t_done - q->t_submit;
  q->res.rel_resid = q->job.rel_resid;
  q->res.err_bound = q->job.err_bound;
}

// Rebuild the engine tables for the current resident set (tick boundary,
// stream idle).  Each request's device state stays where it is.  The new
// table block is allocated before the old one is released.
int fld_server::rebuild() {
  delete eng;
  eng = nullptr;
  size_t new_off = 0, new_sz = 0;
  std::vector<fld_grid> gs;
  std::vector<Hier> hs;
  for (Req *q : resident) {
    gs.push_back(q->r.grid);
    hs.push_back(q->hier);
  }
  if (!resident.empty()) {
    new_sz = tables_bytes(hs);
    if (!alloc.alloc(new_sz, new_off)) return ST_ENOMEM;
  }
  if (have_tables) alloc.release(tables_off, tables_sz);
  have_tables = !resident.empty();
  tables_off = new_off;
  tables_sz = new_sz;
  if (resident.empty()) return ST_OK;
  Carver tbl;
  tbl.base = arena + tables_off;
  std::vector<Carver> pm(resident.size());
  for (size_t i = 0; i < resident.size(); ++i) pm[i].base = arena + resident[i]->off;
  eng = new (std::nothrow) Engine;
  if (!eng) return ST_ENOMEM;
  int st = eng->setup(prm, stream, gs, tbl, pm);
  if (st) return st;
  for (size_t i = 0; i < resident.size(); ++i) {
    Req *q = resident[i];
    const Job &j = q->job;
    eng->fill_step((int)i, eng->mem[i].E_work, q->r.kappa, q->r.eta, j.h, j.a, j.adot);
    eng->h_sc[i] = q->sc;
    eng->h_sc[i].live = 0;
    // a request's dE buffers keep their place in its workspace
    eng->prev_ok[i] = q->prev_ok;
    eng->prev_h[i] = q->prev_h;
    eng->prev_h2[i] = q->prev_h2;
    eng->xcur[i] = q->xcur;
    eng->xold[i] = q->xold;
    eng->warm_now[i] = q->warm_now;
    eng->mem[i].pd.x = eng->h_pd[i].x = eng->mem[i].xb[q->xcur];
  }
  st = eng->upload_pd();
  if (st) return st;
  return eng->upload_sd_sc();
}

#define TRY(expr)             \
  do {                        \
    int _st = (expr);         \
    if (_st) return _st;      \
  } while (0)

// One scheduler tick over the resident set.
int fld_server::tick() {
  Engine &e = *eng;
  const int n = (int)resident.size();
  std::vector<char> mA(n, 0), mS(n, 0), mC(n, 0);
  bool anyA = false, anyS = false;
  // (1) assembly for requests starting a substep (warm-started from the
  // request's previous substeps, as fld_step does)
  bool anyW = false;
  for (int i = 0; i < n; ++i) {
    Req *q = resident[i];
    e.h_sc[i].live = 0;
    if (q->finished) continue;
    if (q->state == RQ_ASSEMBLE) {
      Job &j = q->job;
      j.h = std::min(j.h, j.dt - j.t);
      e.fill_step(i, e.mem[i].E_work, q->r.kappa, q->r.eta, j.h, j.a, j.adot);
      if (e.set_warm(i, j.h)) anyW = true;
      mA[i] = 1;
      anyA = true;
      q->state = RQ_SOLVING;
    }
    if (q->state == RQ_SOLVING) {
      mS[i] = 1;
      anyS = true;
    }
  }
  if (!anyS) return ST_OK;
  TRY(e.upload_sd_sc());
  if (anyW) TRY(e.upload_pd());
  ListSet lsA, lsS, lsC;
  if (anyA) {
    TRY(e.build_lists(mA, 1, lsA));
    e.enqueue_assemble(lsA);
    if (anyW) e.enqueue_warm(lsA);
  }
  // (2) one PCG iteration for every solving request (device flags decide)
  TRY(e.build_lists(mS, 2, lsS));
  e.enqueue_prologue(lsS);
  e.enqueue_iteration(lsS);
  TRY(e.download_sc());
  bool anyV = false, fix = false;
  for (int i = 0; i < n; ++i) {
    if (!mS[i]) continue;
    if (e.h_sc[i].phase == PH_VERIFY) anyV = true;
    if (e.h_sc[i].xlag && e.h_sc[i].phase != PH_ITER) fix = true;
  }
  if (fix) e.finish_x(lsS);
  if (anyV) {
    launch_true_resid(e.T, lsS.fine, stream);
    launch_fin(e.T, FIN_TRUE, e.mixed, stream);
    e.need_pro = true;
    TRY(e.download_sc());
  }
  // (3) commit finished solves; cut failed ones
  bool anyC = false;
  for (int i = 0; i < n; ++i) {
    e.h_sc[i].live = 0;
    if (!mS[i]) continue;
    Req *q = resident[i];
    const Scal &sc = e.h_sc[i];
    if (sc.phase != PH_DONE) continue;
    Job &j = q->job;
    j.iters += sc.iter;
    j.restarts += sc.restarts;
    if (sc.status == ST_OK) {
      e.note_success(i, j.h);
      mC[i] = 1;
      anyC = true;
      e.h_sd[i].E = e.mem[i].E_work;
      e.h_sd[i].Eout = e.mem[i].E_work;
      e.h_sc[i].live = 1;
    } else if (j.cuts < prm.max_dt_cuts) {
      e.prev_ok[i] = 0;
      j.h *= 0.1;
      j.cuts += 1;
      q->state = RQ_ASSEMBLE;
    } else {
      j.status = sc.status;
      finish(q, sc.status);
    }
  }
  if (anyC) {
    TRY(e.upload_sd_sc());
    TRY(e.build_lists(mC, 3, lsC));
    launch_update_E(e.T, lsC.fine, prm.e_floor, 0, stream);
    launch_fin(e.T, FIN_STEP, e.mixed, stream);
    TRY(e.download_sc());
    for (int i = 0; i < n; ++i) {
      if (!mC[i]) continue;
      Req *q = resident[i];
      Job &j = q->job;
      const Scal &sc = e.h_sc[i];
      const double cells = (double)q->hier.cells(0);
      j.substeps += 1;
      j.t += j.h;
      j.rho = std::sqrt(sc.change2 / cells);
      double f = j.rho > 0.0 ? prm.tau_tol / j.rho : 2.0;
      f = std::min(2.0, std::max(0.1, f));
      j.bnorm = std::sqrt(sc.bb);
      j.dEnorm = std::sqrt(sc.dEdE);
      j.rel_resid = sc.bb > 0.0 ? std::sqrt(sc.rr_true / sc.bb) : 0.0;
      j.err_bound = j.dEnorm > 0.0 ? std::sqrt(sc.rr_true) / j.dEnorm : 0.0;
      j.h *= f;
      j.dt_next = j.h;
      if (j.dt - j.t <= 1e-12 * j.dt) {
        q->step += 1;
        if (q->step >= q->r.n_steps) {
          const size_t nb = sizeof(double) * (size_t)q->hier.cells(0);
          if (hipMemcpyAsync(q->r.E_out, e.mem[i].E_work, nb,
                             hipMemcpyDeviceToDevice, stream) != hipSuccess)
            return ST_EDEVICE;
          if (hipStreamSynchronize(stream) != hipSuccess) return ST_EDEVICE;
          j.status = ST_OK;
          finish(q, ST_OK);
          continue;
        }
        j.t = 0.0;
        j.h = j.dt;
      }
      q->state = RQ_ASSEMBLE;
    }
    for (int i = 0; i < n; ++i) e.h_sc[i].live = 0;
  }
  for (int i = 0; i < n; ++i) {
    Req *q = resident[i];
    q->sc = e.h_sc[i];
    q->prev_ok = e.prev_ok[i];
    q->prev_h = e.prev_h[i];
    q->prev_h2 = e.prev_h2[i];
    q->xcur = e.xcur[i];
    q->xold = e.xold[i];
    q->warm_now = e.warm_now[i];
  }
  return ST_OK;
}

void fld_server::run() {
  for (;;) {
    bool changed = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      // publish and retire finished requests
      for (auto it = resident.begin(); it != resident.end();) {
        Req *q = *it;
        if (q->finished) {
          q->state = RQ_DONE;
          alloc.release(q->off, q->bytes);
          --pending;
          it = resident.erase(it);
          changed = true;
        } else {
          ++it;
        }
      }
      if (changed) cv_done.notify_all();
      while (!stop && queue.empty() && resident.empty()) cv_work.wait(lk);
      if (stop && queue.empty() && resident.empty()) break;
      // admit in arrival order with bounded bypass; the new tables must fit
      // beside the current ones
      std::vector<Hier> hs;
      for (Req *q : resident) hs.push_back(q->hier);
      for (auto it = queue.begin(); it != queue.end();) {
        Req *q = *it;
        std::vector<Hier> hs2 = hs;
        hs2.push_back(q->hier);
        size_t off = 0;
        const size_t tb = tables_bytes(hs2);
        bool ok = alloc.alloc(q->bytes, off);
        if (ok) {
          size_t toff = 0;
          if (!alloc.alloc(tb, toff)) {
            alloc.release(off, q->bytes);
            ok = false;
          } else {
            alloc.release(toff, tb);
          }
        }
        if (!ok) {
          if (q->bypassed >= kMaxBypass) break;
          q->bypassed += 1;
          ++it;
          continue;
        }
        q->off = off;
        q->t_admit = now_s();
        resident.push_back(q);
        hs.push_back(q->hier);
        it = queue.erase(it);
        changed = true;
        // E^0 -> resident copy; the job starts with a full step
        ProbMem m;
        Carver cv;
        cv.base = arena + off;
        carve_problem(cv, q->hier, prm, m);
        if (hipMemcpyAsync(m.E_work, q->r.E, sizeof(double) * (size_t)q->hier.cells(0),
                           hipMemcpyDeviceToDevice, stream) != hipSuccess)
          finish(q, ST_EDEVICE);
        q->job.dt = q->r.dt;
        q->job.a = q->r.a;
        q->job.adot = q->r.adot;
        q->job.h = q->r.dt;
        q->job.t = 0.0;
        q->state = RQ_ASSEMBLE;
        q->sc = Scal{};
        q->sc.phase = PH_DONE;
        q->sc.s = q->sc.inv_s = 1.0;
        q->sc.tol2 = prm.rtol * prm.rtol;
        q->sc.max_iter = prm.max_iter;
      }
    }
    int st = ST_OK;
    if (changed || !eng) st = rebuild();
    if (!st && eng) st = tick();
    if (st) {
      // device or memory failure: fail every resident request
      for (Req *q : resident)
        if (!q->finished) finish(q, st);
    }
  }
  delete eng;
  eng = nullptr;
}

extern "C" {

fld_status fld_server_create(const fld_params *p, void *arena,
                             size_t arena_bytes, void *hip_stream,
                             fld_server **out) {
  if (!out) return FLD_EINVAL;
  *out = nullptr;
  if (!p || !params_ok(*p) || !arena || (((uintptr_t)arena) & 255)) return FLD_EINVAL;
  if (arena_bytes < kMinArena) return FLD_ENOMEM;
  fld_server *s = new (std::nothrow) fld_server;
  if (!s) return FLD_ENOMEM;
  s->prm = *p;
  s->arena = (char *)arena;
  s->arena_bytes = arena_bytes;
  s->stream = (hipStream_t)hip_stream;
  s->alloc.init(arena_bytes);
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return FLD_OK;
}

fld_status fld_server_submit(fld_server *s, const fld_request *r,
                             uint64_t *ticket) {
  if (!s || !r || !ticket) return FLD_EINVAL;
  if (!grid_ok(r->grid) || r->n_steps < 1 || !r->E || !r->kappa || !r->eta ||
      !r->E_out)
    return FLD_EINVAL;
  if (!(std::isfinite(r->dt) && r->dt > 0.0 && std::isfinite(r->a) && r->a > 0.0 &&
        std::isfinite(r->adot)))
    return FLD_EINVAL;
  Req *q = new (std::nothrow) Req;
  if (!q) return FLD_ENOMEM;
  q->r = *r;
  q->hier = make_hier(r->grid, s->prm);
  q->bytes = problem_bytes(q->hier, s->prm);
  std::vector<Hier> one{q->hier};
  if (q->bytes + tables_bytes(one) + 1024 > s->arena_bytes) {
    delete q;
    return FLD_ENOMEM;
  }
  q->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    q->ticket = s->next_ticket++;
    s->all[q->ticket] = q;
    s->queue.push_back(q);
    s->pending += 1;
  }
  s->cv_work.notify_one();
  *ticket = q->ticket;
  return FLD_OK;
}

fld_status fld_server_poll(fld_server *s, uint64_t ticket, fld_result *res) {
  if (!s) return FLD_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return FLD_EINVAL;
  if (it->second->state != RQ_DONE) return FLD_EBUSY;
  if (res) *res = it->second->res;
  return FLD_OK;
}

fld_status fld_server_drain(fld_server *s) {
  if (!s) return FLD_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [s] { return s->pending == 0; });
  return FLD_OK;
}

fld_status fld_server_destroy(fld_server *s) {
  if (!s) return FLD_EINVAL;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [s] { return s->pending == 0; });
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto &kv : s->all) delete kv.second;
  delete s;
  return FLD_OK;
}

}  // extern "C"
