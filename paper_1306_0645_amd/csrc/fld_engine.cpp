// Host engine: hierarchy shapes, workspace layout, tile lists, and the PCG /
// step drivers of the implicit FLD solve.
#include "fld_engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace fld {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int hip_ok(hipError_t e) { return e == hipSuccess ? ST_OK : ST_EDEVICE; }

#define HIP_TRY(expr)                           \
  do {                                          \
    if ((expr) != hipSuccess) return ST_EDEVICE; \
  } while (0)

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

bool grid_ok(const fld_grid &g) {
  const int d[3] = {g.nx, g.ny, g.nz};
  for (int v : d)
    if (v < 4 || (v & 1)) return false;
  if ((long long)g.nx * g.ny * g.nz >= (1LL << 31)) return false;
  return finite_pos(g.dx) && finite_pos(g.dy) && finite_pos(g.dz);
}

bool params_ok(const fld_params &p) {
  if (!finite_pos(p.c)) return false;
  if (!(p.theta >= 0.5 && p.theta <= 1.0)) return false;
  if (!(p.d_max >= 0.0) || !(p.r_min >= 0.0)) return false;
  if (!(p.rtol >= 0.0) || !std::isfinite(p.rtol)) return false;
  if (!finite_pos(p.tau_tol) || !(p.e_floor >= 0.0)) return false;
  if (!finite_pos(p.coarse_scale)) return false;
  if (p.max_iter < 1 || p.mg_levels < 0 || p.mg_levels > kMaxLevels) return false;
  if (p.nu_pre < 1 || p.nu_pre > 8 || p.nu_post < 1 || p.nu_post > 8) return false;
  if (p.precision != FLD_PREC_FP64 && p.precision != FLD_PREC_MIXED) return false;
  if (p.max_dt_cuts < 0 || p.tile_z < 0 || p.tile_z > 64 || p.check_every < 0)
    return false;
  if (p.fused_tile_z < 0 || p.fused_tile_z > 256 || (p.fused_tile_z & 1)) return false;
  if (p.cycle_switch < 0) return false;
  if (p.warm_start < 0 || p.warm_start > 2) return false;
  if (p.tail_cells < 0) return false;
  if (p.prolongation < 0 || p.prolongation > 2) return false;
  if (p.smoother != FLD_SMOOTH_RBGS && p.smoother != FLD_SMOOTH_JACOBI) return false;
  if (p.fused_levels < 0 || p.fused_levels > kMaxLevels) return false;
  if (p.coarse_op < 0 || p.coarse_op > 1) return false;
  if (p.direction_fp64 < 0 || p.direction_fp64 > 1) return false;
  if (p.local_sweeps < 0 || p.local_sweeps > 8) return false;
  if (!(p.local_coupling >= 0.0 && p.local_coupling <= 1.0)) return false;
  return true;
}

// Full 2x coarsening while every extent stays even.  Automatic depth stops
// once an extent would drop below 4; an explicit depth allows extents >= 2.
Hier make_hier(const fld_grid &g, const fld_params &p) {
  Hier h;
  h.levels = 1;
  h.n[0][0] = g.nx;
  h.n[0][1] = g.ny;
  h.n[0][2] = g.nz;
  const int maxl = p.mg_levels > 0 ? p.mg_levels : kMaxLevels;
  while (h.levels < maxl) {
    const int *c = h.n[h.levels - 1];
    if ((c[0] | c[1] | c[2]) & 1) break;
    const int lim = p.mg_levels > 0 ? 4 : 8;
    if (c[0] < lim || c[1] < lim || c[2] < lim) break;
    for (int d = 0; d < 3; ++d) h.n[h.levels][d] = c[d] / 2;
    ++h.levels;
  }
  for (int l = 0; l < h.levels; ++l) {
    h.tiles[l] = count_tiles(p, h.n[l][0], h.n[l][1], h.n[l][2]);
    h.ftiles[l] = count_fused_tiles(p, l, h.n[l][0], h.n[l][1], h.n[l][2]);
  }
  // the tail: the coarsest level, and above it every level below the finest
  // with at most tail_cells cells
  h.tail = h.levels > 1 ? h.levels - 1 : 1;
  // (the single-workgroup tail smooths red/black: under the Jacobi smoother
  // it keeps to the coarsest level)
  const long long tc = p.smoother == FLD_SMOOTH_JACOBI ? 0 : p.tail_cells;
  while (h.tail > 1 && h.cells(h.tail - 1) <= tc) --h.tail;
  return h;
}

// Tiles of the fused one-sweep V-cycle kernels: 64 x 16 cells in x, y (their
// LDS buffers are sized for that) and fused_tile_z planes in z on the finest
// level.  Deeper tiles cut the z-halo but leave fewer tiles to hide latency:
// measured on gfx950 at 256^3 (Mcell-updates/s for 8, 16, 32, 64 planes: FP32
// cycle 2532, 2537, 2608, 2451; FP64 2203, 2268, 2308, 2217), 32 planes suit
// a grid that still gives 512 tiles with them; smaller grids halve the depth
// (down to 2 planes) until they do, since a handful of tiles marching 32
// planes each leaves the GPU idle (64^3: 8 tiles).  A grid that gives 2048
// tiles of 64 planes takes those (640^3, mixed, per PCG iteration: down pass
// 2.74 -> 2.68 ms, up pass 2.36 -> 2.33 ms, fused-tile SpMV 4.21 -> 4.15 ms).
// Coarse levels that run the fused passes are 8x smaller and use 4 planes
// where that is needed for a few tiles per CU (128^3 level of 256^3,
// Mcell-updates/s with 8 and 4 planes: FP32 cycle 2622, 2652; FP64 2367,
// 2383); a coarse level that still
// gives 512 tiles of 16 (or 8) planes takes those, for less z-halo (the
// 320^3 and 160^3 levels of 640^3, mixed, per PCG iteration: coarse up
// passes 0.38 -> 0.31 ms, down passes 0.32 -> 0.26 ms).
void fused_shape(const fld_params &p, int l, int nx, int ny, int nz, int &tx,
                 int &ty, int &tz) {
  tx = std::min(nx, 64);
  ty = std::min(ny, 16);
  if (l > 0) {
    const long long cxy = (long long)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
    tz = 16;
    while (tz > 4 && cxy * ((nz + tz - 1) / tz) < 512) tz >>= 1;
    tz = std::min(nz, tz);
    return;
  }
  if (p.fused_tile_z > 0) {
    tz = std::min(nz, p.fused_tile_z);
    return;
  }
  const long long xy = (long long)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
  tz = 32;
  if (xy * ((nz + 63) / 64) >= 2048) tz = 64;
  else while (tz > 2 && xy * ((nz + tz - 1) / tz) < 512) tz >>= 1;
  tz = std::min(tz, nz);
}

int count_fused_tiles(const fld_params &p, int l, int nx, int ny, int nz) {
  int tx, ty, tz;
  fused_shape(p, l, nx, ny, nz, tx, ty, tz);
  return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + tz - 1) / tz);
}

// The fused iteration's SpMV runs on the fused tiles (kSpRows rows per
// thread, 64 x 16 cells a tile) for a problem whose fused finest tiling still
// gives 2048 tiles; a smaller problem keeps the 64 x 4 tiles, whose one cell
// per thread and plane leaves more workgroups to hide latency.  A property of
// the problem alone, as the partial sums' order must be.
bool spmv_on_fused(const Hier &h) { return h.ftiles[0] >= 2048; }

bool fused_cycle(const fld_params &p) {
  return p.smoother == FLD_SMOOTH_RBGS && p.nu_pre == 1 && p.nu_post == 1;
}

// the PCG iteration with the residual update in the down pass (and its
// second residual buffer): fused cycle, mixed precision
bool lazy_iteration(const fld_params &p) {
  return fused_cycle(p) && p.precision == FLD_PREC_MIXED;
}

// Tiles are up to 64 cells wide in x (one wave per row, one cell per lane,
// so each load instruction covers consecutive addresses) and 4+ rows.
void tile_shape(const fld_params &p, int nx, int ny, int nz, int &tx, int &ty,
                int &tz) {
  tx = std::min(nx, 64);
  ty = std::max(1, std::min(ny, kBlock / tx));
  if (p.tile_z > 0) {
    tz = std::min(p.tile_z, nz);
  } else {
    // deepest power of two (<= 8) that still leaves >= 2048 tiles, so small
    // levels get enough workgroups to cover 256 CUs
    const long long xy = (long long)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
    tz = 8;
    while (tz > 1 && xy * ((nz + tz - 1) / tz) < 2048) tz >>= 1;
    tz = std::min(tz, nz);
  }
}

int count_tiles(const fld_params &p, int nx, int ny, int nz) {
  int tx, ty, tz;
  tile_shape(p, nx, ny, nz, tx, ty, tz);
  return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + tz - 1) / tz);
}

void carve_problem(Carver &cv, const Hier &h, const fld_params &p, ProbMem &m) {
  const bool mixed = p.precision == FLD_PREC_MIXED;
  const bool jacobi = p.smoother == FLD_SMOOTH_JACOBI;
  std::memset(&m, 0, sizeof(m));
  for (int l = 0; l < h.levels; ++l) {
    const size_t n = (size_t)h.cells(l);
    LevelDev &L = m.lv[l];
    L.nx = h.n[l][0];
    L.ny = h.n[l][1];
    L.nz = h.n[l][2];
    L.n = (int)n;
    L.Tx = cv.take<double>(n);
    L.Ty = cv.take<double>(n);
    L.Tz = cv.take<double>(n);
    L.diag = cv.take<double>(n);
    if (mixed) {
      L.Tx32 = cv.take<float>(n);
      L.Ty32 = cv.take<float>(n);
      L.Tz32 = cv.take<float>(n);
      L.diag32 = cv.take<float>(n);
    }
    if (l == 0) {
      ProbDev &P = m.pd;
      P.nx = L.nx;
      P.ny = L.ny;
      P.nz = L.nz;
      P.n = L.n;
      P.x = cv.take<double>(n);
      P.r = cv.take<double>(n);
      if (mixed) P.z32 = cv.take<float>(n);
      else P.z = cv.take<double>(n);
      if (mixed && !p.direction_fp64) {
        P.pf0 = cv.take<float>(n);
        P.pf1 = cv.take<float>(n);
      } else {
        P.p0 = cv.take<double>(n);
        P.p1 = cv.take<double>(n);
      }
      P.q = cv.take<double>(n);
      P.b = cv.take<double>(n);
      P.r2 = lazy_iteration(p) ? cv.take<double>(n) : nullptr;
      // (a dry run of the carve, base null, must take the same sizes: the
      // conditions name parameters, never carved pointers)
      const bool local = mixed && p.local_sweeps > 0;
      P.llist = local ? cv.take<int>(n) : nullptr;
      P.lcnt = local ? cv.take<int>(2 * (size_t)h.tiles[0]) : nullptr;
      L.x = mixed ? (void *)cv.take<float>(n) : (void *)P.z;
      L.f = nullptr;
      if (jacobi) L.x2 = mixed ? (void *)cv.take<float>(n) : (void *)cv.take<double>(n);
    } else {
      if (mixed) {
        L.x = cv.take<float>(n);
        L.f = cv.take<float>(n);
      } else {
        L.x = cv.take<double>(n);
        L.f = cv.take<double>(n);
      }
      if (jacobi) L.x2 = mixed ? (void *)cv.take<float>(n) : (void *)cv.take<double>(n);
    }
  }
  m.xb[0] = m.pd.x;
  m.xb[1] = cv.take<double>((size_t)h.cells(0));
  m.xb[2] = cv.take<double>((size_t)h.cells(0));
  m.pd.levels = h.levels;
  m.pd.tail = h.tail;
  m.pd.cs = cv.take<double>(4 * (size_t)h.cells(h.levels - 1));
  m.E_work = cv.take<double>((size_t)h.cells(0));
  for (int k = 0; k < 3; ++k) m.pd.xb[k] = m.xb[k];
  m.pd.Ework = m.E_work;
}

size_t problem_bytes(const Hier &h, const fld_params &p) {
  Carver cv;
  ProbMem m;
  carve_problem(cv, h, p, m);
  return align_up(cv.off);
}

static size_t tables_layout(Carver &cv, const std::vector<Hier> &hs,
                            Engine *e) {
  const int np = (int)hs.size();
  size_t ntiles = 0, nfine = 0, nranges = 0;
  for (const Hier &h : hs) {
    for (int l = 0; l < h.levels; ++l) ntiles += h.tiles[l] + h.ftiles[l];
    nfine += h.tiles[0] + h.ftiles[0];  // partial slots: both finest tilings
  }
  // fine, the two SpMV lists and kListsPerLevel lists per level: at most
  // one range per problem and list, 2 ints each, kListSlots sets
  nranges = (size_t)(kListsPerLevel * kMaxLevels + 3) * np * 2 * kListSlots;
  LevelDev *lv = cv.take<LevelDev>((size_t)kMaxLevels * np);
  ProbDev *pd = cv.take<ProbDev>(np);
  StepDev *sd = cv.take<StepDev>(np);
  Scal *sc = cv.take<Scal>(np);
  double *part = cv.take<double>(2 * std::max<size_t>(nfine, 1));
  double *lpart = cv.take<double>(2 * std::max<size_t>(nfine, 1));
  CtlDev *ctl = cv.take<CtlDev>(std::max(np, 1));
  double *gpart = cv.take<double>(kAsmSums * std::max<size_t>(nfine, 1));
  Tile *tiles = cv.take<Tile>(std::max<size_t>(ntiles, 1));
  int *ranges = cv.take<int>(nranges);
  if (e) {
    e->T.lv = lv;
    e->T.pd = pd;
    e->T.sd = sd;
    e->T.sc = sc;
    e->T.part = part;
    e->T.lpart = lpart;
    e->T.ctl = ctl;
    e->T.gpart = gpart;
    e->T.nprob = np;
    e->d_tiles = tiles;
    e->d_ranges = ranges;
    e->ranges_cap = nranges;
  }
  return align_up(cv.off);
}

size_t tables_bytes(const std::vector<Hier> &hs) {
  Carver cv;
  return tables_layout(cv, hs, nullptr);
}

Engine::~Engine() { release_graph(); }

int Engine::release_graph() {
  for (auto &g : graphs) {
    if (g.second.exec) hipGraphExecDestroy(g.second.exec);
    if (g.second.graph) hipGraphDestroy(g.second.graph);
  }
  graphs.clear();
  for (auto &g : unit_graphs) {
    if (g.second.exec) hipGraphExecDestroy(g.second.exec);
    if (g.second.graph) hipGraphDestroy(g.second.graph);
  }
  unit_graphs.clear();
  if (cap_stream) hipStreamDestroy(cap_stream);
  cap_stream = nullptr;
  return ST_OK;
}

int Engine::setup(const fld_params &p, hipStream_t s,
                  const std::vector<fld_grid> &g, Carver &tbl,
                  std::vector<Carver> &pm) {
  prm = p;
  stream = s;
  mixed = p.precision == FLD_PREC_MIXED;
  grids = g;
  const int np = (int)g.size();
  hier.resize(np);
  mem.resize(np);
  Lmax = 0;
  for (int i = 0; i < np; ++i) {
    hier[i] = make_hier(g[i], p);
    Lmax = std::max(Lmax, hier[i].levels);
  }
  tables_layout(tbl, hier, this);
  for (int i = 0; i < np; ++i) {
    // the caller sized each problem's block with the dry run (problem_bytes):
    // a carve that takes more would write past the block, so refuse it
    const size_t start = pm[i].off;
    carve_problem(pm[i], hier[i], p, mem[i]);
    if (align_up(pm[i].off) - start > problem_bytes(hier[i], p)) return ST_ENOMEM;
  }

  // full tile table, level-major; within a level the standard tiles of every
  // problem, then the fused-cycle tiles, so both finest tilings come first
  // (their indices are the partial-sum slots)
  fused = fused_cycle(p);
  lazy = lazy_iteration(p);
  // levels of each problem run by the fused passes: the finest, then each
  // coarser one of the problem that still holds 2^20 cells (or fused_levels
  // of them); a property of the problem alone, so that its result does not
  // depend on the company it is solved in
  ftop.assign(np, 1);
  for (int i = 0; i < np; ++i) {
    if (p.fused_levels > 0) {
      ftop[i] = std::min(p.fused_levels, hier[i].levels);
    } else {
      for (int l = 1; l < hier[i].levels && hier[i].cells(l) >= (1LL << 20); ++l)
        ftop[i] = l + 1;
    }
  }
  h_tiles.clear();
  tbeg.assign((size_t)np * kMaxLevels, 0);
  fbeg.assign((size_t)np * kMaxLevels, 0);
  auto emit = [&](int i, int nx, int ny, int nz, int tx, int ty, int tz) {
    for (int z0 = 0; z0 < nz; z0 += tz)
      for (int y0 = 0; y0 < ny; y0 += ty)
        for (int x0 = 0; x0 < nx; x0 += tx) {
          Tile t;
          t.prob = i;
          t.x0 = x0;
          t.y0 = y0;
          t.z0 = z0;
          t.tx = std::min(tx, nx - x0);
          t.ty = std::min(ty, ny - y0);
          t.tz = std::min(tz, nz - z0);
          t.cpt = 1;
          h_tiles.push_back(t);
        }
  };
  for (int l = 0; l < Lmax; ++l) {
    for (int i = 0; i < np; ++i) {
      if (l >= hier[i].levels) continue;
      tbeg[(size_t)i * kMaxLevels + l] = (int)h_tiles.size();
      const int nx = hier[i].n[l][0], ny = hier[i].n[l][1], nz = hier[i].n[l][2];
      int tx, ty, tz;
      tile_shape(prm, nx, ny, nz, tx, ty, tz);
      emit(i, nx, ny, nz, tx, ty, tz);
    }
    for (int i = 0; i < np; ++i) {
      if (l >= hier[i].levels) continue;
      fbeg[(size_t)i * kMaxLevels + l] = (int)h_tiles.size();
      const int nx = hier[i].n[l][0], ny = hier[i].n[l][1], nz = hier[i].n[l][2];
      int tx, ty, tz;
      fused_shape(prm, l, nx, ny, nz, tx, ty, tz);
      emit(i, nx, ny, nz, tx, ty, tz);
    }
  }
  h_lv.assign((size_t)kMaxLevels * np, LevelDev{});
  h_pd.resize(np);
  h_sd.assign(np, StepDev{});
  h_sc.assign(np, Scal{});
  prev_ok.assign(np, 0);
  prev_h.assign(np, 0.0);
  prev_h2.assign(np, 0.0);
  xcur.assign(np, 0);
  xold.assign(np, -1);
  warm_now.assign(np, 0);
  for (int i = 0; i < np; ++i) {
    for (int l = 0; l < hier[i].levels; ++l) h_lv[(size_t)l * np + i] = mem[i].lv[l];
    h_pd[i] = mem[i].pd;
    h_pd[i].t0 = tbeg[(size_t)i * kMaxLevels];
    h_pd[i].t1 = h_pd[i].t0 + hier[i].tiles[0];
    h_pd[i].f0 = fbeg[(size_t)i * kMaxLevels];
    h_pd[i].f1 = h_pd[i].f0 + hier[i].ftiles[0];
    h_pd[i].spf = spmv_on_fused(hier[i]) ? 1 : 0;
    h_sc[i].phase = PH_DONE;
    h_sc[i].tol2 = prm.rtol * prm.rtol;
    h_sc[i].max_iter = prm.max_iter;
    h_sc[i].s = 1.0;
    h_sc[i].inv_s = 1.0;
  }
  int st = upload_all();
  if (st) return st;
  std::vector<char> every(np, 1);
  st = build_lists(every, 0, all);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(stream));
  return ST_OK;
}

// Range lists of every launch kind for the problems flagged in member.
int Engine::build_lists(const std::vector<char> &member, int slot, ListSet &out) {
  const int np = (int)hier.size();
  const size_t per_slot = ranges_cap / kListSlots;
  int *slot_base = d_ranges + per_slot * slot;
  h_ranges.clear();
  auto make_any = [&](int level, bool fz, auto pred) {
    TileList L{};
    L.base = d_tiles;
    const int off = (int)h_ranges.size();
    int blocks = 0, nr = 0;
    for (int i = 0; i < np; ++i) {
      if (!member[i] || level >= hier[i].levels || !pred(i)) continue;
      h_ranges.push_back(blocks);
      h_ranges.push_back((fz ? fbeg : tbeg)[(size_t)i * kMaxLevels + level]);
      blocks += fz ? hier[i].ftiles[level] : hier[i].tiles[level];
      ++nr;
    }
    L.ranges = slot_base + off;
    L.nranges = nr;
    L.nblocks = blocks;
    return L;
  };
  auto make = [&](int level, auto pred) { return make_any(level, false, pred); };
  out.fine = make(0, [](int) { return true; });
  out.spf = make_any(0, true, [&](int i) { return spmv_on_fused(hier[i]); });
  out.spg = make(0, [&](int i) { return !spmv_on_fused(hier[i]); });
  for (int l = 0; l < kMaxLevels; ++l) {
    // per-level sweeps: every level above the tail (the single level of a
    // one-level hierarchy)
    auto smoothed = [&](int i) {
      return hier[i].levels == 1 ? l == 0 : l < hier[i].tail;
    };
    out.smooth[l] = make(l, smoothed);
    out.exist[l] = make(l, [&](int) { return l >= 1; });
    out.down[l] = make(l, [&](int i) { return l >= 1 && l <= hier[i].tail; });
    out.fsm[l] = make_any(l, true, [&](int i) { return smoothed(i) && l < ftop[i]; });
    // (a one-level problem runs the finest down pass too: in the fused PCG
    // iteration it forms the residual)
    out.fdn[l] = make_any(l, true, [&](int i) {
      return smoothed(i) && l < ftop[i] && (l < hier[i].levels - 1 || l == 0);
    });
    // the fused cycle's per-half-sweep levels, and the levels restricted into
    // from one of them
    out.gsm[l] = make(l, [&](int i) { return smoothed(i) && l >= ftop[i]; });
    out.gdn[l] = make(l, [&](int i) {
      return l >= 1 && l <= hier[i].tail && l - 1 >= ftop[i];
    });
  }
  if (h_ranges.size() > per_slot) return ST_EINVAL;
  if (!h_ranges.empty())
    HIP_TRY(hipMemcpyAsync(slot_base, h_ranges.data(), sizeof(int) * h_ranges.size(),
                           hipMemcpyHostToDevice, stream));
  return ST_OK;
}

int Engine::upload_all() {
  const int np = (int)hier.size();
  HIP_TRY(hipMemcpyAsync(T.lv, h_lv.data(), sizeof(LevelDev) * h_lv.size(),
                         hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(T.pd, h_pd.data(), sizeof(ProbDev) * np,
                         hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(d_tiles, h_tiles.data(), sizeof(Tile) * h_tiles.size(),
                         hipMemcpyHostToDevice, stream));
  int st = upload_sd_sc();
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(stream));
  return ST_OK;
}

int Engine::upload_sd_sc() {
  const int np = (int)hier.size();
  HIP_TRY(hipMemcpyAsync(T.sd, h_sd.data(), sizeof(StepDev) * np,
                         hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(T.sc, h_sc.data(), sizeof(Scal) * np,
                         hipMemcpyHostToDevice, stream));
  return ST_OK;
}

int Engine::download_sc() {
  const int np = (int)hier.size();
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h_sc.data(), T.sc, sizeof(Scal) * np,
                         hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return ST_OK;
}

// The switched cycle.  In mixed precision with automatic prolongation, on a
// problem of at least 2^23 cells, it is V(1,1) with trilinear correction: the
// fused passes make such a V(1,1) iteration less than half the cost of a
// per-half-sweep V(2,2) one (640^3 reionization share, mixed: 776
// Mcell-updates/s at 26.8 iterations per step against 564 at 17.1 with
// V(2,2)).  Smaller grids are launch-bound, so the iterations V(2,2) saves
// count for more (Test-1 and Test-2 octants of 32^3 to 128^3: V(2,2) 10-25 %
// faster).  Otherwise, and in FP64, V(2,2).
int Engine::set_switched(bool on) {
  if (on == switched) return ST_OK;
  switched = on;
  long long big = 0;
  for (const Hier &h : hier) big = std::max(big, h.cells(0));
  const bool tri_only = mixed && prm.prolongation == 2 && big >= (1LL << 23);
  const int nu = (on && !tri_only) ? 2 : 1;
  prm.nu_pre = prm.nu_post = nu;
  fused = fused_cycle(prm);
  lazy = lazy_iteration(prm);
  return release_graph();
}

// In FP64 the switched cycle is V(2,2), whose per-half-sweep kernels cost
// more than twice the fused V(1,1) passes on a grid that fills the GPU: on
// the 640^3 reionization share (FP64) V(1,1) took 34.6 iterations per step
// at 508 ms against 19.5 at 773 ms after switching.  So an FP64 handle whose
// largest grid has at least 2^23 cells keeps V(1,1).
bool Engine::switch_helps() const {
  if (mixed) return true;
  long long big = 0;
  for (const Hier &h : hier) big = std::max(big, h.cells(0));
  return big < (1LL << 23);
}

int Engine::trilinear() const {
  return (mixed && (prm.prolongation == 1 || (prm.prolongation == 2 && switched)))
             ? 1 : 0;
}

// Only a handle configured for V(1,1) adapts: to the switched cycle after a
// solve that needed more than cycle_switch iterations, and back once a
// switched solve needs at most a third of that.  Any other configured cycle
// is kept as is.
int Engine::adapt_cycle(int max_iters) {
  const int thr = prm.cycle_switch;
  if (thr <= 0 || !switch_helps()) return ST_OK;
  if (!switched && prm.nu_pre == 1 && prm.nu_post == 1 && max_iters > thr)
    return set_switched(true);
  if (switched && max_iters * 3 <= thr) return set_switched(false);
  return ST_OK;
}

void Engine::fill_step(int p, const double *E, const double *kappa,
                       const double *eta, double dt, double a, double adot) {
  StepDev &S = h_sd[p];
  S.E = E;
  S.kappa = kappa;
  S.eta = eta;
  S.Eout = nullptr;
  S.dt = dt;
  S.adot_a = adot / a;
  // comoving mesh, derivatives with respect to the comoving position (Sec.
  // 2): the comoving cell sizes; a enters only through adot / a
  S.idx = 1.0 / grids[p].dx;
  S.idy = 1.0 / grids[p].dy;
  S.idz = 1.0 / grids[p].dz;
  S.warm = 0.0;
  S.w1 = S.w2 = 0.0;
  S.h1 = S.h2 = nullptr;
  Scal &sc = h_sc[p];
  sc.live = 1;
  sc.tol2 = prm.rtol * prm.rtol;
  sc.max_iter = prm.max_iter;
}

void Engine::enqueue_assemble(const ListSet &ls) {
  launch_assemble(T, ls.fine, prm.c, prm.theta, prm.d_max, prm.r_min, mixed, stream);
  for (int l = 1; l < Lmax; ++l)
    launch_coarsen(T, ls.exist[l], l, prm.coarse_scale, mixed, prm.coarse_op, stream);
  if (mixed && prm.local_sweeps > 0)
    launch_lmask(T, ls.fine, prm.local_coupling, stream);
  launch_fin(T, FIN_BB, mixed, stream);
  need_pro = true;
}

// The fused V(1,1) cycle after its finest down pass: one sweep each way; the
// coarse levels with enough cells to fill the GPU run the two fused passes
// too (they never store the pre-smoothed x), the smaller, latency-bound ones
// the per-half-sweep kernels; last the finest up pass.
void Engine::enqueue_fused_rest(const ListSet &ls) {
  const int prec = mixed;
  const int tri = trilinear();
  for (int l = 1; l < Lmax; ++l) {
    launch_vdown(T, ls.fdn[l], l, prec, VD_ALL, stream);
    launch_pre0(T, ls.gsm[l], l, prec, stream);
    if (l + 1 < Lmax) launch_resid_restrict(T, ls.gdn[l + 1], l + 1, prec, stream);
  }
  if (Lmax > 1) launch_vtail(T, prec, 1, 1, tri, stream);
  for (int l = Lmax - 1; l >= 1; --l) {
    launch_vup(T, ls.fsm[l], l, prec, 0, tri, stream);
    launch_prolong_black(T, ls.gsm[l], l, prec, tri, stream);
    launch_half(T, ls.gsm[l], l, 0, prec, stream);
  }
  launch_vup(T, ls.fsm[0], 0, prec, mixed, tri, stream);
  if (local_on()) {
    for (int k = 0; k < prm.local_sweeps; ++k) {
      launch_local(T, ls.fine, 1, stream);
      launch_local(T, ls.fine, 0, stream);
    }
  }
}

// One V-cycle for every active problem.  Pre-smoothing: red then black
// (nu_pre sweeps); post-smoothing: black then red (nu_post sweeps), the
// adjoint order, so the FP64 cycle is a symmetric preconditioner.
void Engine::enqueue_vcycle(const ListSet &ls) {
  const int prec = mixed;
  const int tri = trilinear();
  if (fused) {
    launch_vdown(T, ls.fdn[0], 0, prec, VD_ALL, stream);
    enqueue_fused_rest(ls);
    return;
  }
  const TileList *smooth = ls.smooth, *down = ls.down;
  if (prm.smoother == FLD_SMOOTH_JACOBI) {
    // weighted Jacobi ping-pongs between x and x2.  Pre-smoothing ends in x
    // (restriction and the parent's prolongation read x); the correction
    // x + P e goes to the buffer that makes the last post-sweep read x2 and
    // write x, or z on the finest level.
    const int np = prm.nu_pre, nq = prm.nu_post;
    for (int l = 0; l < Lmax; ++l) {
      if (smooth[l].nblocks == 0) continue;
      int in2 = np & 1;  // first sweep writes x when nu_pre is odd
      launch_jacobi(T, smooth[l], l, prec, 0, in2, 0, stream);
      for (int s = 1; s < np; ++s) {
        in2 ^= 1;
        launch_jacobi(T, smooth[l], l, prec, 1, in2, 0, stream);
      }
      if (l + 1 < Lmax) launch_resid_restrict(T, down[l + 1], l + 1, prec, stream);
    }
    if (Lmax > 1) launch_vtail(T, prec, np, nq, tri, stream);
    for (int l = Lmax - 1; l >= 0; --l) {
      if (smooth[l].nblocks == 0) continue;
      int in2 = nq & 1;  // buffer the correction lands in
      launch_prolong_add(T, smooth[l], l, prec, tri, in2, stream);
      for (int s = 0; s < nq; ++s) {
        const int last = l == 0 && s == nq - 1;
        launch_jacobi(T, smooth[l], l, prec, last ? 2 : 1, in2, mixed, stream);
        in2 ^= 1;
      }
    }
    return;
  }
  for (int l = 0; l < Lmax; ++l) {
    if (smooth[l].nblocks == 0) continue;
    launch_pre0(T, smooth[l], l, prec, stream);
    for (int s = 1; s < prm.nu_pre; ++s) {
      launch_half(T, smooth[l], l, 0, prec, stream);
      launch_half(T, smooth[l], l, 1, prec, stream);
    }
    if (l + 1 < Lmax) launch_resid_restrict(T, down[l + 1], l + 1, prec, stream);
  }
  if (Lmax > 1) launch_vtail(T, prec, prm.nu_pre, prm.nu_post, tri, stream);
  for (int l = Lmax - 1; l >= 0; --l) {
    if (smooth[l].nblocks == 0) continue;
    launch_prolong_black(T, smooth[l], l, prec, tri, stream);
    for (int s = 0; s < prm.nu_post; ++s) {
      if (s > 0) launch_half(T, smooth[l], l, 1, prec, stream);
      if (l == 0 && s == prm.nu_post - 1) launch_half_out(T, smooth[0], prec, mixed, stream);
      else launch_half(T, smooth[l], l, 0, prec, stream);
    }
  }
}

// One PCG iteration.  Fused V(1,1) form in mixed precision: r -= alpha q
// happens in the next iteration's finest down pass (which reads r anyway),
// the convergence test right after it, and x += alpha p in the next SpMV
// (which reads p anyway), so the update needs no pass of its own.  (In FP64
// the extra loads push the down pass past its register budget: measured at
// 256^3, 2306 against 2375 Mcell-updates/s with the separate update.)  The
// unit enqueued here is rotated so that it ends with that test: it starts
// after the finest down pass, which the previous unit (or, for a problem
// starting or restarting, enqueue_prologue) has done, so the host sees a
// converged problem at the end of a batch instead of one unit later.  The
// other forms update x and r in a pass of their own.
void Engine::enqueue_iteration(const ListSet &ls) {
  if (lazy) {
    enqueue_fused_rest(ls);
    launch_fin(T, FIN_RZ, mixed, stream, local_on() ? 2 : 1);
    launch_spmv_f(T, ls.spf, kmode(), stream);
    launch_spmv_p(T, ls.spg, 1, kmode(), stream);
    launch_fin(T, FIN_PQ, mixed, stream, 1);
    launch_vdown(T, ls.fdn[0], 0, mixed, VD_CONT, stream);
    launch_fin(T, FIN_RR2, mixed, stream, 1);
    return;
  }
  enqueue_vcycle(ls);
  launch_fin(T, FIN_RZ, mixed, stream, fused ? 1 : 0);
  launch_spmv_p(T, ls.fine, 0, kmode(), stream);
  launch_fin(T, FIN_PQ, mixed, stream, 0);
  launch_update(T, ls.fine, kmode(), stream);
  launch_fin(T, FIN_RR, mixed, stream);
}

// The finest down pass for problems that start or restart their PCG (rotated
// fused iteration); a no-op otherwise.
void Engine::enqueue_prologue(const ListSet &ls) {
  if (!lazy || !need_pro) return;
  launch_vdown(T, ls.fdn[0], 0, mixed, VD_FRESH, stream);
  launch_fin(T, FIN_FRESH, mixed, stream);
  need_pro = false;
}

// x += alpha p for problems that stopped iterating with that update pending
// (fused form); keeps the host mirror in step
void Engine::finish_x(const ListSet &ls) {
  launch_xfix(T, ls.fine, kmode(), stream);
  launch_fin(T, FIN_XFIX, mixed, stream);
  for (Scal &sc : h_sc)
    if (sc.xlag && sc.phase != PH_ITER) sc.xlag = 0;
}

int Engine::check_every() const {
  if (prm.check_every > 0) return prm.check_every;
  long long cells = 0;
  for (const Hier &h : hier) cells += h.cells(0);
  // (the batch size of a handle's first solve, before run_solve has an
  // iteration count to go by) large grids: a host read every 2 iterations;
  // small grids, where reads cost more than iterations, every 4
  return cells >= (1LL << 22) ? 2 : 4;
}

// Iterate every problem in PH_ITER until each one is decided.  Problems whose
// recursive residual meets the tolerance are verified with the true FP64
// residual b - A x and restarted from it if it does not (refinement).
// predicted: the caller set the host mirror of every problem it just
// assembled to "iterating", so the first batch goes out without waiting to
// read the state back (a problem the assembly finished, b = 0, or failed,
// skips the batch's kernels on the device and shows up at the first read)
// commit: right after each verification, E += dE for the problems it
// decided (their Eout already set), so a converged step needs no further
// round trip.
int Engine::run_solve(bool predicted, bool commit) {
  last_nu = prm.nu_pre;
  last_tri = trilinear();
  int st = predicted ? ST_OK : download_sc();
  if (st) return st;
  first_batch = true;
  for (;;) {
    int nact = 0, nver = 0;
    bool fix = false;
    for (const Scal &sc : h_sc) {
      if (sc.phase == PH_ITER && sc.active) ++nact;
      else if (sc.phase == PH_VERIFY) ++nver;
      if (sc.xlag && sc.phase != PH_ITER) fix = true;
    }
    if (fix) finish_x(all);
    if (nver) {
      launch_true_resid(T, all.fine, stream);
      launch_fin(T, FIN_TRUE, mixed, stream);
      need_pro = true;
      if (commit) {
        launch_update_E(T, all.fine, prm.e_floor, 0, stream, 1);
        launch_fin(T, FIN_STEP, mixed, stream, 1);
      }
    } else if (nact) {
      enqueue_prologue(all);
      // iterations before the next host read: automatic mode sizes the
      // solve's first batch to one less than the last solve took and reads
      // after every iteration from there on, so a solve like the last costs
      // two reads and no iteration of a converged problem (one of
      // early-returning kernels, otherwise)
      int K = check_every();
      if (prm.check_every <= 0 && last_iters > 1)
        K = first_batch ? std::min(last_iters - 1, 16) : 1;
      first_batch = false;
      if (prm.use_graph) {
        Captured &g = graphs[K];
        if (!g.exec) {
          if (!cap_stream)
            HIP_TRY(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
          HIP_TRY(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
          hipStream_t saved = stream;
          stream = cap_stream;
          // one graph holds the K iterations between host checks
          for (int k = 0; k < K; ++k) enqueue_iteration(all);
          stream = saved;
          HIP_TRY(hipStreamEndCapture(cap_stream, &g.graph));
          HIP_TRY(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
        }
        HIP_TRY(hipGraphLaunch(g.exec, stream));
      } else {
        for (int k = 0; k < K; ++k) enqueue_iteration(all);
      }
    } else {
      break;
    }
    st = download_sc();
    if (st) return st;
  }
  int mx = 0;
  for (const Scal &sc : h_sc)
    if (sc.live) mx = std::max(mx, sc.iter);
  last_iters = mx;
  return ST_OK;
}

// Warm start of problem p's next solve over a step h, when its history
// allows: dE is about h times the mean rate over the step, so scale the last
// dE, or extrapolate the rate linearly from the last two (w1, w2; the
// Galerkin guess combines the same two with coefficients the device solves
// for).  The guess goes into the dE buffer that holds neither history entry,
// which becomes P.x (the caller uploads the problem table before the
// assembly).
bool Engine::set_warm(int p, double h) {
  warm_now[p] = 0;
  if (!prm.warm_start || prev_ok[p] < 1 || !(prev_h[p] > 0.0)) return false;
  warm_now[p] = 1;
  const double h1 = prev_h[p], r1 = h / h1;
  StepDev &S = h_sd[p];
  S.warm = prm.warm_start;
  S.w1 = r1;
  S.w2 = 0.0;
  const bool two = prev_ok[p] >= 2 && prev_h2[p] > 0.0 && xold[p] >= 0;
  if (two) {
    const double h0 = prev_h2[p];
    const double tau = (h1 + h) / (h0 + h1);
    S.w1 = r1 * (1.0 + tau);
    S.w2 = -(h / h0) * tau;
  }
  const int a = xcur[p], b = two ? xold[p] : -1;
  int nxt = 0;
  while (nxt == a || nxt == b) ++nxt;
  S.h1 = mem[p].xb[a];
  S.h2 = two ? mem[p].xb[b] : nullptr;
  mem[p].pd.x = h_pd[p].x = mem[p].xb[nxt];
  xold[p] = a;
  xcur[p] = nxt;
  return true;
}

// After the assembly of warm-started problems: the Galerkin guess and its
// residual (its coefficients come from FIN_BB), then x = 0, r = b wherever
// the guess was not kept (or b = 0).
void Engine::enqueue_warm(const ListSet &ls) {
  if (prm.warm_start > 1) {
    launch_warm_x(T, ls.fine, stream);
    launch_fin(T, FIN_WARM, mixed, stream);
  }
  launch_warm_revert(T, ls.fine, stream);
}

// dE of a successful substep of length h seeds the next one; after a warm
// start the one before stays in xb[xold]
void Engine::note_success(int p, double h) {
  prev_ok[p] = warm_now[p] ? 2 : 1;
  prev_h2[p] = prev_h[p];
  prev_h[p] = h;
}

int Engine::upload_pd() {
  HIP_TRY(hipMemcpyAsync(T.pd, h_pd.data(), sizeof(ProbDev) * h_pd.size(),
                         hipMemcpyHostToDevice, stream));
  return ST_OK;
}

// Steps for every job not done: assemble, solve, and on success E += dE;
// on failure cut the job's radiation step by 10x and subcycle (Sec. 3.4).
int Engine::run_steps(std::vector<Job> &jobs) {
  const int np = (int)jobs.size();
  std::vector<int> target(np, 0);  // 0: none, 1: caller E in place, 2: E_work
  bool warm = false;
  for (;;) {
    bool any = false;
    for (int p = 0; p < np; ++p) {
      Job &j = jobs[p];
      h_sc[p].live = 0;
      if (j.done) continue;
      any = true;
      j.h = std::min(j.h, j.dt - j.t);
      fill_step(p, j.in_work ? mem[p].E_work : j.E, j.kappa, j.eta, j.h, j.a, j.adot);
      if (set_warm(p, j.h)) warm = true;
      // where E + dE goes if this substep succeeds: the caller's E after
      // the last substep of a step that never left it, else the work copy
      const bool last = j.dt - (j.t + j.h) <= 1e-12 * j.dt;
      target[p] = (!j.in_work && last) ? 1 : 2;
      h_sd[p].Eout = target[p] == 1 ? j.E : mem[p].E_work;
    }
    if (!any) break;
    int st = upload_sd_sc();
    if (st) return st;
    if (warm) {
      st = upload_pd();
      if (st) return st;
    }
    // (an extrapolated guess's residual b - A x0 comes out of the assembly,
    // a Galerkin guess and its residual out of enqueue_warm; either is kept
    // only if it reduces the residual)
    enqueue_assemble(all);
    if (warm) {
      enqueue_warm(all);
      warm = false;
    }
    for (int p = 0; p < np; ++p) {
      if (jobs[p].done) continue;
      h_sc[p].phase = PH_ITER;
      h_sc[p].active = 1;
      h_sc[p].xlag = 0;
    }
    st = run_solve(true, true);
    if (st) return st;
    {
      int mx = 0;
      for (int p = 0; p < np; ++p)
        if (h_sc[p].live) mx = std::max(mx, h_sc[p].iter);
      st = adapt_cycle(mx);
      if (st) return st;
    }
    // problems the solve decided without a verification (b = 0) still need
    // their E update
    bool commit = false;
    std::vector<char> ok(np, 0);
    for (int p = 0; p < np; ++p) {
      Job &j = jobs[p];
      const bool live = h_sc[p].live;
      h_sc[p].live = 0;
      if (!live) {
        target[p] = 0;
        continue;
      }
      j.iters += h_sc[p].iter;
      j.restarts += h_sc[p].restarts;
      if (h_sc[p].phase == PH_DONE && h_sc[p].status == ST_OK) {
        note_success(p, j.h);
        ok[p] = 1;
        if (!h_sc[p].committed) {
          h_sc[p].live = 1;
          commit = true;
        }
      } else if (j.cuts < prm.max_dt_cuts) {
        prev_ok[p] = 0;
        j.h *= 0.1;
        j.cuts += 1;
      } else {
        prev_ok[p] = 0;
        j.done = true;
        j.status = h_sc[p].status != ST_OK ? h_sc[p].status : ST_ENOCONV;
      }
    }
    if (commit) {
      st = upload_sd_sc();
      if (st) return st;
      launch_update_E(T, all.fine, prm.e_floor, 0, stream);
      launch_fin(T, FIN_STEP, mixed, stream);
      st = download_sc();
      if (st) return st;
    }
    {
      for (int p = 0; p < np; ++p) {
        if (!ok[p]) continue;
        Job &j = jobs[p];
        const Scal &sc = h_sc[p];
        const double n = (double)hier[p].cells(0);
        j.substeps += 1;
        j.t += j.h;
        j.rho = std::sqrt(sc.change2 / n);
        double f = j.rho > 0.0 ? prm.tau_tol / j.rho : 2.0;
        f = std::min(2.0, std::max(0.1, f));
        j.bnorm = std::sqrt(sc.bb);
        j.dEnorm = std::sqrt(sc.dEdE);
        j.rel_resid = sc.bb > 0.0 ? std::sqrt(sc.rr_true / sc.bb) : 0.0;
        j.err_bound = j.dEnorm > 0.0 ? std::sqrt(sc.rr_true) / j.dEnorm : 0.0;
        if (target[p] == 2) j.in_work = true;
        j.h *= f;
        j.dt_next = j.h;
        if (j.dt - j.t <= 1e-12 * j.dt) {
          j.done = true;
          j.status = ST_OK;
          if (j.in_work)
            HIP_TRY(hipMemcpyAsync(j.E, mem[p].E_work,
                                   sizeof(double) * (size_t)hier[p].cells(0),
                                   hipMemcpyDeviceToDevice, stream));
        }
      }
      for (int p = 0; p < np; ++p) h_sc[p].live = 0;
    }
  }
  HIP_TRY(hipStreamSynchronize(stream));
  return ST_OK;
}

// One unit of device-controlled stepping: for every problem whose state
// asks for it, the next substep's assembly and warm start, the prologue of
// the fused iteration, one PCG iteration, the true-residual verification,
// E += dE, the controller and the copy of a finished run's E.
void Engine::enqueue_unit(const ListSet &ls, const CtlParams &cp) {
  launch_assemble(T, ls.fine, prm.c, prm.theta, prm.d_max, prm.r_min, mixed, stream);
  for (int l = 1; l < Lmax; ++l)
    launch_coarsen(T, ls.exist[l], l, prm.coarse_scale, mixed, prm.coarse_op, stream);
  if (mixed && prm.local_sweeps > 0)
    launch_lmask(T, ls.fine, prm.local_coupling, stream);
  launch_fin(T, FIN_BB, mixed, stream);
  if (prm.warm_start > 1) {
    launch_warm_x(T, ls.fine, stream);
    launch_fin(T, FIN_WARM, mixed, stream);
  }
  launch_warm_revert(T, ls.fine, stream);
  launch_fin(T, FIN_STAGE, mixed, stream);
  if (lazy) {
    launch_vdown(T, ls.fdn[0], 0, mixed, VD_FRESH, stream);
    launch_fin(T, FIN_FRESH, mixed, stream);
  }
  enqueue_iteration(ls);
  launch_xfix(T, ls.fine, kmode(), stream);
  launch_fin(T, FIN_XFIX, mixed, stream);
  launch_true_resid(T, ls.fine, stream);
  launch_fin(T, FIN_TRUE, mixed, stream);
  launch_update_E(T, ls.fine, prm.e_floor, 0, stream, 1);
  launch_fin(T, FIN_STEP, mixed, stream, 1);
  launch_control(T, cp, stream);
  launch_copy_E(T, ls.fine, stream);
}

// Steps of every job with the substep control on the device (Sec. 3.4, the
// radiation subcycling loop): n_steps steps of j.dt (or, adaptive, steps of
// the controller's dt_next from j.dt until t_end), each subcycled after a
// failed solve.  The host sets up the first substep as run_steps does, then
// replays a graph of `units` units and reads the state once per replay.  The
// cycle stays as configured (no adaptive switch inside a run).
int Engine::run_advance(std::vector<Job> &jobs, int n_steps, int adaptive,
                        double t_end, int units) {
  const int np = (int)jobs.size();
  std::vector<CtlDev> hc(np);
  for (int p = 0; p < np; ++p) {
    Job &j = jobs[p];
    const double h0 = adaptive ? std::min(j.dt, t_end) : j.dt;
    fill_step(p, j.E, j.kappa, j.eta, h0, j.a, j.adot);
    set_warm(p, h0);
    h_sd[p].Eout = j.E;  // the first substep covers its step: it writes E
    CtlDev &c = hc[p];
    std::memset(&c, 0, sizeof(c));
    c.E = j.E;
    c.dt0 = j.dt;
    c.t_end = t_end;
    c.n_steps = n_steps;
    c.adaptive = adaptive;
    c.dt = c.h = h0;
    c.target = 1;
    c.prev_ok = prev_ok[p];
    c.xcur = xcur[p];
    c.xold = xold[p];
    c.warm_now = warm_now[p];
    c.prev_h = prev_h[p];
    c.prev_h2 = prev_h2[p];
    Scal &sc = h_sc[p];
    sc.ctl = 1;
    sc.stage = 1;
    sc.live = 1;
    sc.phase = PH_DONE;
    sc.active = 0;
    sc.xlag = 0;
  }
  HIP_TRY(hipMemcpyAsync(T.ctl, hc.data(), sizeof(CtlDev) * np, hipMemcpyHostToDevice,
                         stream));
  int st = upload_pd();
  if (st) return st;
  st = upload_sd_sc();
  if (st) return st;
  const CtlParams cp{prm.tau_tol, prm.max_dt_cuts, prm.warm_start};
  Captured &g = unit_graphs[units];
  if (!g.exec) {
    if (!cap_stream)
      HIP_TRY(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
    hipStream_t saved = stream;
    stream = cap_stream;
    for (int u = 0; u < units; ++u) enqueue_unit(all, cp);
    stream = saved;
    HIP_TRY(hipStreamEndCapture(cap_stream, &g.graph));
    HIP_TRY(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
  }
  for (;;) {
    HIP_TRY(hipGraphLaunch(g.exec, stream));
    HIP_TRY(hipMemcpyAsync(hc.data(), T.ctl, sizeof(CtlDev) * np, hipMemcpyDeviceToHost,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));
    bool all_done = true;
    for (const CtlDev &c : hc) all_done = all_done && c.done;
    if (all_done) break;
  }
  // the host mirrors follow the device: tables, the iterate buffer in use,
  // the warm-start history, and the problems leave device control
  HIP_TRY(hipMemcpyAsync(h_pd.data(), T.pd, sizeof(ProbDev) * np, hipMemcpyDeviceToHost,
                         stream));
  HIP_TRY(hipMemcpyAsync(h_sd.data(), T.sd, sizeof(StepDev) * np, hipMemcpyDeviceToHost,
                         stream));
  st = download_sc();
  if (st) return st;
  for (int p = 0; p < np; ++p) {
    const CtlDev &c = hc[p];
    Job &j = jobs[p];
    mem[p].pd.x = h_pd[p].x;
    prev_ok[p] = (char)c.prev_ok;
    xcur[p] = c.xcur;
    xold[p] = c.xold;
    warm_now[p] = (char)c.warm_now;
    prev_h[p] = c.prev_h;
    prev_h2[p] = c.prev_h2;
    j.status = c.status;
    j.iters = c.iters;
    j.restarts = c.restarts;
    j.substeps = c.substeps;
    j.cuts = c.cuts_total;
    j.rho = c.rho;
    j.dt_next = c.dt_next;
    j.rel_resid = c.rel_resid;
    j.err_bound = c.err_bound;
    j.bnorm = c.bnorm;
    j.dEnorm = c.dEnorm;
    j.steps = c.steps;
    j.t = c.t_total;
    j.done = true;
    h_sc[p].ctl = 0;
    h_sc[p].stage = 0;
    h_sc[p].live = 0;
  }
  st = upload_sd_sc();
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(stream));
  return ST_OK;
}

}  // namespace fld
