// Host engine of the FLD library: owns a set of problems (one for a plain
// handle, many for a batch, a changing set for a server), their multigrid
// hierarchies carved from caller-provided device memory, the device tables
// and tile lists, and drives assembly, the PCG iteration and the step logic.
#pragma once

#include <map>
#include <vector>

#include "fld.h"
#include "fld_internal.h"

namespace fld {

size_t align_up(size_t v, size_t a = 256);

// bump allocator over caller memory (base == nullptr: size only)
struct Carver {
  char *base = nullptr;
  size_t off = 0;
  template <class T>
  T *take(size_t n) {
    off = align_up(off);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

// multigrid hierarchy shape of one grid
struct Hier {
  int levels = 0;
  int tail = 1;                 // first level of the single-workgroup tail
  int n[kMaxLevels][3] = {};
  int tiles[kMaxLevels] = {};   // tiles per level
  int ftiles[kMaxLevels] = {};  // fused-cycle tiles per level
  long long cells(int l) const { return (long long)n[l][0] * n[l][1] * n[l][2]; }
};

bool grid_ok(const fld_grid &g);
bool params_ok(const fld_params &p);
Hier make_hier(const fld_grid &g, const fld_params &p);
void tile_shape(const fld_params &p, int nx, int ny, int nz, int &tx, int &ty,
                int &tz);
int count_tiles(const fld_params &p, int nx, int ny, int nz);
void fused_shape(const fld_params &p, int l, int nx, int ny, int nz, int &tx,
                 int &ty, int &tz);
int count_fused_tiles(const fld_params &p, int l, int nx, int ny, int nz);
bool fused_cycle(const fld_params &p);
bool lazy_iteration(const fld_params &p);
bool spmv_on_fused(const Hier &h);
size_t problem_bytes(const Hier &h, const fld_params &p);
size_t tables_bytes(const std::vector<Hier> &hs);

// device memory of one problem
struct ProbMem {
  LevelDev lv[kMaxLevels];
  ProbDev pd;
  double *xb[3] = {};  // dE buffers: the iterate (pd.x) and two of history
  double *E_work = nullptr;
};
void carve_problem(Carver &cv, const Hier &h, const fld_params &p, ProbMem &m);

// one step request inside the engine
struct Job {
  double *E = nullptr;
  const double *kappa = nullptr, *eta = nullptr;
  double dt = 0, a = 1, adot = 0;
  double t = 0, h = 0;
  int cuts = 0, substeps = 0, iters = 0, restarts = 0, steps = 0;
  int status = ST_OK;
  bool done = false, in_work = false;
  double rho = 0, dt_next = 0, rel_resid = 0, err_bound = 0, bnorm = 0,
         dEnorm = 0;
};

// Launch lists of every kernel kind for one subset of the problems.
struct ListSet {
  TileList fine{}, smooth[kMaxLevels]{}, exist[kMaxLevels]{};
  TileList spf{}, spg{};        // fused-iteration SpMV: fused / standard tiles
  TileList fsm[kMaxLevels]{};   // fused tiles of smoothed levels
  TileList fdn[kMaxLevels]{};   // fused tiles of smoothed levels with a coarser one
  TileList down[kMaxLevels]{};  // levels restricted into from a per-level sweep
  TileList gsm[kMaxLevels]{};   // fused cycle: per-half-sweep smoothed levels
  TileList gdn[kMaxLevels]{};   // fused cycle: levels restricted into from one
};
constexpr int kListsPerLevel = 7;  // smooth, exist, down, fsm, fdn, gsm, gdn

constexpr int kListSlots = 4;  // independent range regions (server phases)

class Engine {
 public:
  fld_params prm{};
  hipStream_t stream = nullptr;
  int mixed = 0;
  std::vector<fld_grid> grids;
  std::vector<Hier> hier;
  std::vector<ProbMem> mem;
  int Lmax = 0;

  // host mirrors of the device tables
  std::vector<LevelDev> h_lv;
  std::vector<ProbDev> h_pd;
  std::vector<StepDev> h_sd;
  std::vector<Scal> h_sc;
  std::vector<Tile> h_tiles;
  std::vector<int> h_ranges;
  std::vector<int> tbeg;   // [p * kMaxLevels + l] first tile of (p, l)
  std::vector<int> fbeg;   // [p * kMaxLevels + l] first fused tile of (p, l)
  bool fused = false;      // one-sweep fused V-cycle kernels
  bool lazy = false;       // fused PCG iteration (residual update in the down pass)
  bool need_pro = false;   // some problem (re)starts: enqueue_prologue is due
  std::vector<int> ftop;   // per problem: levels 0 .. ftop - 1 run the fused passes
  int last_nu = 1;         // sweeps per side of the cycle used by the last solve
  int last_tri = 0;        // the last solve's cycle used trilinear correction
  bool switched = false;   // the adaptive switch changed the handle's cycle
  // per problem warm-start history: prev_ok = 0 none, 1 buffer xb[xcur]
  // (the iterate P.x) holds the dE of the last successful substep (length
  // prev_h), 2 also xb[xold] the one before it (length prev_h2).  A warm
  // step reads both and writes its guess into the third buffer, which
  // becomes P.x.
  std::vector<char> prev_ok;
  std::vector<double> prev_h, prev_h2;
  std::vector<int> xcur, xold;
  std::vector<char> warm_now;  // the current substep started from a warm guess

  Tables T{};
  Tile *d_tiles = nullptr;
  int *d_ranges = nullptr;
  size_t ranges_cap = 0;   // ints available at d_ranges (all slots)
  ListSet all;             // every problem (slot 0)

  // captured K-iteration batches, by K
  struct Captured {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::map<int, Captured> graphs;
  std::map<int, Captured> unit_graphs;  // device-controlled units, by count
  hipStream_t cap_stream = nullptr;
  int last_iters = 0;       // iterations of the last solve (its slowest problem)
  bool first_batch = true;  // the next batch is a solve's first
  bool assembled = false;
  int last_status = ST_OK;

  ~Engine();

  // lay out tables (in tbl) and problems (in pm[i]) and upload descriptors
  int setup(const fld_params &p, hipStream_t s, const std::vector<fld_grid> &g,
            Carver &tbl, std::vector<Carver> &pm);
  int upload_all();
  int upload_sd_sc();
  int download_sc();
  // lists for the problems flagged in member, in range slot 'slot'; uploads
  // the ranges (enqueued on the stream)
  int build_lists(const std::vector<char> &member, int slot, ListSet &out);
  int release_graph();

  // switch the V-cycle sweep counts (re-captures the graph next solve)
  int set_switched(bool on);
  bool set_warm(int p, double h);
  void note_success(int p, double h);
  int upload_pd();
  int trilinear() const;
  // finest-level Krylov storage (launch_spmv_p): 0 FP64, 1 mixed with an
  // FP32 direction, 2 mixed with an FP64 direction
  int kmode() const { return mixed ? (prm.direction_fp64 ? 2 : 1) : 0; }
  bool switch_helps() const;
  // extra red/black sweeps over the strongly coupled finest cells after the
  // fused cycle's post-sweep (mixed precision)
  bool local_on() const { return mixed && fused && prm.local_sweeps > 0; }
  // adaptive cycle choice after a solve that took max_iters iterations
  int adapt_cycle(int max_iters);

  void enqueue_assemble(const ListSet &ls);
  void enqueue_warm(const ListSet &ls);
  void enqueue_vcycle(const ListSet &ls);
  void enqueue_fused_rest(const ListSet &ls);
  void enqueue_iteration(const ListSet &ls);
  void enqueue_prologue(const ListSet &ls);
  void finish_x(const ListSet &ls);
  int run_solve(bool predicted = false, bool commit = false);
  int run_steps(std::vector<Job> &jobs);
  void enqueue_unit(const ListSet &ls, const CtlParams &cp);
  int run_advance(std::vector<Job> &jobs, int n_steps, int adaptive, double t_end,
                  int units);
  int check_every() const;
  void fill_step(int p, const double *E, const double *kappa, const double *eta,
                 double dt, double a, double adot);
};

int hip_ok(hipError_t e);

}  // namespace fld
