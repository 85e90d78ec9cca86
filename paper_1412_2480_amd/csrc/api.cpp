// C-ABI of the PIC hot-path library (declared in include/pic.h): planning,
// workspace carving, particle/field transfer, step sequencing, diagnostics
// and event timing. All device work is issued on the caller's stream; the
// device memory is the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pic.h"
#include "pic_dev.h"
#include "pic_launch.h"

namespace {

constexpr int kMaxCgBlocks = 4096;
constexpr int kDivBlocks = 512;
constexpr int kDivWords = 4;          // per-block words of the divergence diagnostics
constexpr int kTimingClasses = 9;
constexpr int kWgradBlocks = 256;     // work-groups of the weight-gradient partial sums
// message of the last failed pic_init on this thread (pic_last_error(NULL))
thread_local std::string g_init_err;
constexpr int kDefaultTrainCrop = 64;  // training window (cells per side) by default
constexpr int kMaxTrainCrop = 128;     // largest training window per side
constexpr int kDefaultLearnedMaxit = 30;
constexpr int kDefaultPrecondSlots = 16;
constexpr double kTuneTie = 0.02;     // autotuner: relative margin treated as a tie

struct Bump {
  uint8_t* base;
  size_t off = 0;
  explicit Bump(uint8_t* b) : base(b) {}
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

struct Tiling {
  int TX, TY, TXA, TYA;
  std::vector<int> ntx, nty, tile0;
  std::vector<long long> cell0;
  int n_tiles;
  long long n_cells, max_cells;
};

int tiles_along(int n, int T, int* widest) {
  if (n <= T) {
    *widest = n;
    return 1;
  }
  const int rem = n % T;
  if (rem == 0) {
    *widest = T;
    return n / T;
  }
  if (rem < 3) {
    *widest = T + rem;
    return n / T;
  }
  *widest = T;
  return n / T + 1;
}

}  // namespace

struct pic_ctx {
  std::vector<pic_run_desc> runs;
  pic_options opt{};
  pic_plan_info plan{};
  Tiling tl;
  hipStream_t stream = nullptr;
  uint8_t* ws = nullptr;
  size_t ws_bytes = 0;
  bool fast = false;
  bool split = true;
  bool ids = true;
  std::vector<DevRun> hruns;
  DevRun* d_runs = nullptr;
  int* d_tile_run = nullptr;
  DevState<float> sf{};
  DevState<double> sd{};
  FieldArgs fa{};
  double* d_stats = nullptr;
  // learned aid
  bool learned = false;      // storage carved (solver PIC_SOLVER_LEARNED_PCG)
  bool use_learned = false;  // field solves take the learned path
  bool collect = false;
  std::vector<NetTrain> nets;      // one per distinct operator
  std::vector<double*> net_pairs;  // pairs ring of each network
  NetWeights* d_nets = nullptr;
  std::vector<int> net_of_run, net_first_run;
  int pair_slots = 0;
  long long pairs_written = 0;
  long long train_cells = 0;       // cells of the training activations (largest first run)
  int adam_step = 0;
  double* d_history = nullptr;
  // injection staging (shock runs): particles sorted by tile + (tile, first, count) list
  long long inj_cap = 0;
  int* d_inj_cell = nullptr;
  void* d_inj_ox = nullptr;
  void* d_inj_oy = nullptr;
  void* d_inj_ux = nullptr;
  void* d_inj_uy = nullptr;
  void* d_inj_uz = nullptr;
  int* d_inj_id = nullptr;
  int* d_inj_list = nullptr;
  std::vector<std::array<long long, PIC_MAXS>> next_id;   // per run and species
  // inflow of shock runs generated on the device before every step
  InflowDev* d_inflow = nullptr;
  long long* d_inflow_step = nullptr;
  std::vector<InflowDev> inflow;   // host mirror of the table
  bool any_inflow = false;
  double* d_rho = nullptr;
  double* d_divpart = nullptr;
  int* d_err = nullptr;
  int phase = 0;
  long long step = 0;
  int parity = 0;                 // particle buffer swaps since init, mod 2
  int max_cg_blocks = 0;          // co-resident limit of the field-solve grid
  int cg_cap = 0;                 // requested work-groups of the field solve
  // graph mode: executable graphs of two steps per starting parity and
  // reordering pattern (index parity + 2 * pattern, see graph_two_steps)
  bool graph_ok = true;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec[8] = {};
  int gkey[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
  long long graph_replays = 0;
  long long diag_count = 0;
  int threads = 256;
  int device = 0;
  std::vector<double> h_stats;    // host copy of the solve statistics (sized at init)
  std::string err;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;  // (class, index of start event)
  double t_ms[kTimingClasses] = {};
  long long t_n[kTimingClasses] = {};
};

namespace {

int fail(pic_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                          \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ctx, PIC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int validate(const pic_run_desc* runs, int n_runs, const pic_options* o, std::string* msg) {
  if (!runs || n_runs < 1 || n_runs > PIC_MAX_RUNS) {
    *msg = "n_runs out of range";
    return PIC_E_INVAL;
  }
  if (!o) {
    *msg = "options missing";
    return PIC_E_INVAL;
  }
  if (o->precision != PIC_FP64 && o->precision != PIC_FP32_FAST) {
    *msg = "precision must be PIC_FP64 or PIC_FP32_FAST";
    return PIC_E_INVAL;
  }
  // a particle in the second tile column of a shock run must not reach behind
  // the wall (whose ghost columns only the first column's patches fold back),
  // and a one-cell tile loses every particle every step: two cells at least
  if ((o->tile_x > 0 && o->tile_x < 2) || (o->tile_y > 0 && o->tile_y < 2)) {
    *msg = "tiles need at least 2 cells along each axis";
    return PIC_E_INVAL;
  }
  if (o->solver != PIC_SOLVER_CG && o->solver != PIC_SOLVER_LEARNED_PCG) {
    *msg = "unknown solver";
    return PIC_E_INVAL;
  }
  if (o->sort_every < 0) {
    *msg = "sort_every must be >= 0";
    return PIC_E_INVAL;
  }
  if (o->gather != PIC_GATHER_NODAL && o->gather != PIC_GATHER_STAGGERED) {
    *msg = "gather must be PIC_GATHER_NODAL or PIC_GATHER_STAGGERED";
    return PIC_E_INVAL;
  }
  if (o->field_scheme != PIC_SCHEME_IMPLICIT && o->field_scheme != PIC_SCHEME_EXPLICIT) {
    *msg = "field_scheme must be PIC_SCHEME_IMPLICIT or PIC_SCHEME_EXPLICIT";
    return PIC_E_INVAL;
  }
  if (o->field_scheme == PIC_SCHEME_EXPLICIT && o->solver != PIC_SOLVER_CG) {
    *msg = "the explicit scheme has no field solve (solver must be PIC_SOLVER_CG)";
    return PIC_E_INVAL;
  }
  if (o->solver == PIC_SOLVER_LEARNED_PCG) {
    if (o->learned_form != PIC_NET_COLLAPSED && o->learned_form != PIC_NET_MFMA) {
      *msg = "learned_form must be PIC_NET_COLLAPSED or PIC_NET_MFMA";
      return PIC_E_INVAL;
    }
    if (o->learned_maxit < 0 || o->precond_slots < 0) {
      *msg = "learned_maxit and precond_slots must be >= 0";
      return PIC_E_INVAL;
    }
  }
  for (int r = 0; r < n_runs; ++r) {
    const pic_run_desc& d = runs[r];
    char buf[160];
    auto bad = [&](const char* what) {
      snprintf(buf, sizeof buf, "run %d: %s", r, what);
      *msg = buf;
      return PIC_E_INVAL;
    };
    if (d.nx < 8 || d.ny < 8 || d.nx > 32767 || d.ny > 32767) return bad("nx, ny must be in [8, 32767]");
    if (!(d.dx > 0) || !(d.dy > 0)) return bad("dx, dy must be positive");
    if (!(d.cfl > 0) || d.cfl > 1.0) return bad("cfl must be in (0, 1]");
    if (d.cfl * d.dx > d.dy * (1.0 + 1e-12)) return bad("dt must not exceed dy (one cell per step)");
    if (!(d.theta >= 0.5) || d.theta > 1.0) return bad("theta must be in [0.5, 1]");
    if (d.shape_order < 1 || d.shape_order > 3) return bad("shape_order must be 1, 2 or 3");
    if (d.bc != PIC_BC_PERIODIC && d.bc != PIC_BC_SHOCK)
      return bad("bc must be PIC_BC_PERIODIC or PIC_BC_SHOCK");
    if (d.bc == PIC_BC_SHOCK && d.nx < 16) return bad("a shock run needs nx >= 16");
    if (o->field_scheme == PIC_SCHEME_EXPLICIT) {
      if (d.bc != PIC_BC_PERIODIC) return bad("the explicit scheme is periodic only");
      const double r = d.dx / d.dy;
      if (d.cfl * d.cfl * (1.0 + r * r) > 1.0 + 1e-12)
        return bad("explicit scheme beyond the Courant limit: cfl^2 (1 + dx^2/dy^2) > 1");
    }
    if (d.n_species < 1 || d.n_species > PIC_MAX_SPECIES) return bad("n_species out of range");
    for (int s = 0; s < d.n_species; ++s)
      if (!(d.species[s].m > 0) || !std::isfinite(d.species[s].q) || !(d.species[s].ppc >= 0))
        return bad("species needs m > 0, finite q, ppc >= 0");
    if (!(d.cg_rtol > 0) || d.cg_maxit < 1) return bad("cg_rtol > 0 and cg_maxit >= 1 required");
  }
  return PIC_OK;
}

void make_tiling(const pic_run_desc* runs, int n_runs, const pic_options* o, Tiling* t) {
  t->TX = o->tile_x > 0 ? o->tile_x : 16;
  t->TY = o->tile_y > 0 ? o->tile_y : 16;
  t->TXA = t->TYA = 0;
  t->ntx.resize(n_runs);
  t->nty.resize(n_runs);
  t->tile0.resize(n_runs);
  t->cell0.resize(n_runs);
  int nt = 0;
  long long nc = 0, mc = 0;
  for (int r = 0; r < n_runs; ++r) {
    int wx, wy;
    t->ntx[r] = tiles_along(runs[r].nx, t->TX, &wx);
    t->nty[r] = tiles_along(runs[r].ny, t->TY, &wy);
    t->TXA = std::max(t->TXA, wx);
    t->TYA = std::max(t->TYA, wy);
    t->tile0[r] = nt;
    t->cell0[r] = nc;
    nt += t->ntx[r] * t->nty[r];
    const long long cells = (long long)runs[r].nx * runs[r].ny;
    nc += cells;
    mc = std::max(mc, cells);
  }
  t->n_tiles = nt;
  t->n_cells = nc;
  t->max_cells = mc;
}

// Runs that share the operator of Eq. (7) (dx, dy, cfl, theta) share one
// network of the learned solver; the first run of each group records its
// training pairs.
void group_nets(const pic_run_desc* runs, int n_runs, std::vector<int>* net_of,
                std::vector<int>* first) {
  net_of->assign(n_runs, -1);
  first->clear();
  for (int r = 0; r < n_runs; ++r) {
    for (size_t g = 0; g < first->size(); ++g) {
      const pic_run_desc& d = runs[(*first)[g]];
      if (d.dx == runs[r].dx && d.dy == runs[r].dy && d.cfl == runs[r].cfl &&
          d.theta == runs[r].theta) {
        (*net_of)[r] = (int)g;
        break;
      }
    }
    if ((*net_of)[r] < 0) {
      (*net_of)[r] = (int)first->size();
      first->push_back(r);
    }
  }
}

// Carve (or, with base == nullptr, size) the workspace.
template <typename R>
size_t carve(uint8_t* base, const Tiling& tl, const pic_plan_info& pl, int n_runs, bool fast,
             bool split, bool ids, int hist_cap, int pair_slots,
             const std::vector<long long>& net_cells, long long inj_cap, pic_ctx* c,
             DevState<R>* st) {
  Bump b(base);
  const int K = pl.tile_split;
  const long long nc = tl.n_cells;
  const size_t plane = (size_t)(tl.TXA + 5) * (tl.TYA + 5);
  DevRun* d_runs = b.take<DevRun>(n_runs);
  int* tile_run = b.take<int>(tl.n_tiles);
  double *E[3], *B[3], *J[3];
  for (int k = 0; k < 3; ++k) E[k] = b.take<double>(nc);
  for (int k = 0; k < 3; ++k) B[k] = b.take<double>(nc);
  for (int k = 0; k < 3; ++k) J[k] = b.take<double>(nc);
  float* Ef[6] = {};
  if (fast)
    for (int k = 0; k < 6; ++k) Ef[k] = b.take<float>(nc);
  double *x[3], *pp[3], *r0[3], *r1[3], *w0[3], *w1[3], *s0[3], *s1[3], *bsv[3];
  for (int k = 0; k < 3; ++k) {
    bsv[k] = b.take<double>(nc);
    x[k] = b.take<double>(nc);
    pp[k] = b.take<double>(nc);
    r0[k] = b.take<double>(nc);
    r1[k] = b.take<double>(nc);
    w0[k] = b.take<double>(nc);
    w1[k] = b.take<double>(nc);
    s0[k] = b.take<double>(nc);
    s1[k] = b.take<double>(nc);
  }
  double* part = b.take<double>((size_t)kMaxCgBlocks * 24);
  int* g_active = b.take<int>(4);
  unsigned* bar = b.take<unsigned>(kBarWords);
  double* stats = b.take<double>((size_t)n_runs * PIC_STAT_WORDS);
  // learned solver: per network the FP32 weights, their BF16 copy and
  // collapsed filter, Adam state and a ring of (b, dB) pairs; the training
  // activations are shared, sized for the largest network's first run
  const int n_nets = pair_slots > 0 ? (int)net_cells.size() : 0;
  std::vector<NetTrain> nets(n_nets);
  std::vector<double*> net_pairs(n_nets, nullptr);
  NetWeights* d_nets = nullptr;
  if (n_nets > 0) {
    d_nets = b.take<NetWeights>(n_nets);
    long long n1 = (long long)(kMaxTrainCrop + 6) * (kMaxTrainCrop + 6);
    for (long long v : net_cells) n1 = std::max(n1, v);
    NetTrain sh{};
    const size_t nC = (size_t)n1 * NET_C;
    sh.part = b.take<float>((size_t)kWgradBlocks * NET_C * NET_C * 9);
    sh.xin = b.take<float>(n1);
    sh.y = b.take<float>(n1);
    sh.gy = b.take<float>(n1);
    sh.tc = b.take<double>(n1);
    sh.h1 = b.take<float>(nC);
    sh.h2 = b.take<float>(nC);
    sh.gh1 = b.take<float>(nC);
    sh.gh2 = b.take<float>(nC);
    sh.dpart = b.take<double>(512);
    sh.scal = b.take<double>(4);
    sh.wg_blocks = kWgradBlocks;
    for (int g = 0; g < n_nets; ++g) {
      NetTrain nt = sh;
      nt.w = b.take<float>(NET_NW);
      nt.w2b = b.take<__bf16>(NET_C * NET_C * 9);
      nt.k49 = b.take<double>(64);
      nt.grad = b.take<float>(NET_NW);
      nt.m = b.take<float>(NET_NW);
      nt.v = b.take<float>(NET_NW);
      nets[g] = nt;
      net_pairs[g] = b.take<double>((size_t)pair_slots * 6 * net_cells[g]);
    }
  }
  double* history = b.take<double>((size_t)n_runs * hist_cap * PIC_REC_WORDS);
  int* err = b.take<int>(1);
  double* wk_part = b.take<double>((size_t)tl.n_tiles * K * PIC_MAXS * 2);
  double* rho = b.take<double>(tl.max_cells);
  int *inj_cell = nullptr, *inj_id = nullptr, *inj_list = nullptr;
  R *inj_ox = nullptr, *inj_oy = nullptr, *inj_ux = nullptr, *inj_uy = nullptr, *inj_uz = nullptr;
  if (inj_cap > 0) {
    inj_cell = b.take<int>(inj_cap);
    inj_ox = b.take<R>(inj_cap);
    inj_oy = b.take<R>(inj_cap);
    inj_ux = b.take<R>(inj_cap);
    inj_uy = b.take<R>(inj_cap);
    inj_uz = b.take<R>(inj_cap);
    inj_id = b.take<int>(inj_cap);
    inj_list = b.take<int>((size_t)3 * tl.n_tiles);
  }
  double* divpart = b.take<double>((size_t)kDivBlocks * kDivWords);
  InflowDev* inflow = b.take<InflowDev>(n_runs);
  long long* inflow_step = b.take<long long>(n_runs);
  double* patch[3];
  for (int k = 0; k < 3; ++k) patch[k] = b.take<double>((size_t)tl.n_tiles * K * plane);
  DevState<R> s{};
  for (int sp = 0; sp < PIC_MAXS; ++sp) {
    const size_t slots = (size_t)tl.n_tiles * pl.tile_slots[sp];
    if (pl.tile_slots[sp] == 0) continue;
    s.cell[sp] = b.take<int>(slots);
    s.ox[sp] = b.take<R>(slots);
    s.oy[sp] = b.take<R>(slots);
    s.ux[sp] = b.take<R>(slots);
    s.uy[sp] = b.take<R>(slots);
    s.uz[sp] = b.take<R>(slots);
    s.ncell[sp] = b.take<int>(slots);
    s.nox[sp] = b.take<R>(slots);
    s.noy[sp] = b.take<R>(slots);
    s.nux[sp] = b.take<R>(slots);
    s.nuy[sp] = b.take<R>(slots);
    s.nuz[sp] = b.take<R>(slots);
    if (ids) {
      s.id[sp] = b.take<int>(slots);
      s.nid[sp] = b.take<int>(slots);
    }
    s.cnt[sp] = b.take<int>(tl.n_tiles);
    s.stay_cnt[sp] = b.take<int>(tl.n_tiles);
    if (split) {
      s.old_cell[sp] = b.take<int>(slots);
      s.old_ox[sp] = b.take<R>(slots);
      s.old_oy[sp] = b.take<R>(slots);
    }
  }
  const size_t total = (b.off + 255) & ~size_t(255);
  if (!base) return total;

  s.n_runs = n_runs;
  s.n_tiles = tl.n_tiles;
  s.TX = tl.TX;
  s.TY = tl.TY;
  s.TXA = tl.TXA;
  s.TYA = tl.TYA;
  s.PW = tl.TXA + 5;
  s.PH = tl.TYA + 5;
  for (int sp = 0; sp < PIC_MAXS; ++sp) s.tile_slots[sp] = pl.tile_slots[sp];
  s.K = K;
  s.runs = d_runs;
  s.tile_run = tile_run;
  for (int k = 0; k < 3; ++k) {
    s.E[k] = E[k];
    s.B[k] = B[k];
    s.J[k] = J[k];
  }
  for (int k = 0; k < 6; ++k) s.Ef[k] = Ef[k];
  for (int k = 0; k < 3; ++k) s.patch[k] = patch[k];
  s.wk_part = wk_part;
  s.err = err;
  *st = s;

  FieldArgs& f = c->fa;
  f.n_runs = n_runs;
  f.runs = d_runs;
  for (int k = 0; k < 3; ++k) {
    f.E[k] = E[k];
    f.B[k] = B[k];
    f.J[k] = J[k];
    f.x[k] = x[k];
    f.p[k] = pp[k];
    f.r0[k] = r0[k];
    f.r1[k] = r1[k];
    f.w0[k] = w0[k];
    f.w1[k] = w1[k];
    f.s0[k] = s0[k];
    f.s1[k] = s1[k];
    f.bsv[k] = bsv[k];
  }
  for (int k = 0; k < 6; ++k) f.Ef[k] = Ef[k];
  f.part = part;
  f.g_active = g_active;
  f.bar = bar;
  f.err = err;
  f.stats = stats;
  f.wk_part = wk_part;
  f.K = K;
  f.history = history;
  f.hist_cap = hist_cap;
  f.nets = d_nets;
  c->nets = nets;
  c->net_pairs = net_pairs;
  c->d_nets = d_nets;
  c->d_runs = d_runs;
  c->d_tile_run = tile_run;
  c->d_stats = stats;
  c->d_history = history;
  c->d_rho = rho;
  c->d_inflow = inflow;
  c->d_inflow_step = inflow_step;
  c->inj_cap = inj_cap;
  c->d_inj_cell = inj_cell;
  c->d_inj_ox = inj_ox;
  c->d_inj_oy = inj_oy;
  c->d_inj_ux = inj_ux;
  c->d_inj_uy = inj_uy;
  c->d_inj_uz = inj_uz;
  c->d_inj_id = inj_id;
  c->d_inj_list = inj_list;
  c->d_divpart = divpart;
  c->d_err = err;
  return total;
}

// staged particles per injection call: four cell columns of every shock run
// at the largest ppc of its species
long long inject_cap_of(const pic_run_desc* runs, int n_runs) {
  long long cap = 0;
  for (int r = 0; r < n_runs; ++r) {
    if (runs[r].bc != PIC_BC_SHOCK) continue;
    double ppc = 0;
    for (int s = 0; s < runs[r].n_species; ++s) ppc = std::max(ppc, runs[r].species[s].ppc);
    cap += 4LL * runs[r].ny * (long long)std::ceil(ppc) + 64;
  }
  return cap;
}

int pair_slots_of(const pic_options* o) {
  if (o->solver != PIC_SOLVER_LEARNED_PCG) return 0;
  return o->precond_slots > 0 ? o->precond_slots : kDefaultPrecondSlots;
}

int plan_impl(const pic_run_desc* runs, int n_runs, const pic_options* o, pic_plan_info* out,
              Tiling* tl, std::string* msg) {
  int rc = validate(runs, n_runs, o, msg);
  if (rc) return rc;
  make_tiling(runs, n_runs, o, tl);
  const bool fast = o->precision == PIC_FP32_FAST;
  const size_t rsz = fast ? 4 : 8;
  const size_t plane = (size_t)(tl->TXA + 5) * (tl->TYA + 5);
  const size_t smem = plane * (6 * rsz + 3 * sizeof(double));
  if (smem > 64 * 1024) {
    *msg = "tile too large for LDS (fields + currents exceed 64 KiB)";
    return PIC_E_INVAL;
  }
  pic_plan_info p{};
  p.tile_x = tl->TX;
  p.tile_y = tl->TY;
  p.n_tiles = tl->n_tiles;
  p.n_cells = tl->n_cells;
  const double slack = o->slack > 0 ? o->slack : 0.25;
  int max_species = 0;
  for (int r = 0; r < n_runs; ++r) max_species = std::max(max_species, runs[r].n_species);
  for (int s = 0; s < PIC_MAX_SPECIES; ++s) {
    double ppc = 0;
    for (int r = 0; r < n_runs; ++r)
      if (s < runs[r].n_species) ppc = std::max(ppc, runs[r].species[s].ppc);
    if (s >= max_species) {
      p.tile_slots[s] = 0;
      continue;
    }
    double want = std::ceil(ppc * tl->TXA * tl->TYA * (1.0 + slack));
    long long slots = std::max(64LL, ((long long)want + 63) / 64 * 64);
    if (slots > (1LL << 30)) {
      *msg = "tile slots exceed 2^30";
      return PIC_E_INVAL;
    }
    p.tile_slots[s] = (int)slots;
    p.particle_slots[s] = slots * tl->n_tiles;
  }
  p.tile_split = o->tile_split > 0 ? std::min(o->tile_split, 64) : 4;
  // particles that change tile are written straight into the destination
  // tile's slots: there is no separate exchange buffer
  p.exchange_slots = 0;
  const int hist_cap = o->history_cap > 0 ? o->history_cap : 1;
  const bool split = true;
  const bool ids = o->track_ids != 0;
  const int slots = pair_slots_of(o);
  std::vector<long long> tc;
  if (slots > 0) {
    std::vector<int> net_of, first;
    group_nets(runs, n_runs, &net_of, &first);
    for (int r : first) tc.push_back((long long)runs[r].nx * runs[r].ny);
  }
  const long long ic = inject_cap_of(runs, n_runs);
  p.workspace_bytes = fast ? carve<float>(nullptr, *tl, p, n_runs, true, split, ids, hist_cap,
                                          slots, tc, ic, nullptr, (DevState<float>*)nullptr)
                           : carve<double>(nullptr, *tl, p, n_runs, false, split, ids, hist_cap,
                                           slots, tc, ic, nullptr, (DevState<double>*)nullptr);
  *out = p;
  return PIC_OK;
}

// ---------------------------------------------------------------- timing
void t_begin(pic_ctx* c, int cls) {
  if (!c->timing) return;
  if (c->ev_used + 2 > c->ev_pool.size()) {
    for (int k = 0; k < 256; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      c->ev_pool.push_back(e);
    }
  }
  (void)hipEventRecord(c->ev_pool[c->ev_used], c->stream);
  c->ev_marks.push_back({cls, c->ev_used});
  c->ev_used += 2;
}
void t_end(pic_ctx* c) {
  if (!c->timing || c->ev_marks.empty()) return;
  (void)hipEventRecord(c->ev_pool[c->ev_marks.back().second + 1], c->stream);
}
void t_resolve(pic_ctx* c) {
  if (c->ev_marks.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& m : c->ev_marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_pool[m.second], c->ev_pool[m.second + 1]) == hipSuccess) {
      c->t_ms[m.first] += ms;
      c->t_n[m.first] += 1;
    }
  }
  c->ev_marks.clear();
  c->ev_used = 0;
}

// ---------------------------------------------------------------- device steps
template <typename R>
DevState<R>& state(pic_ctx* c);
template <>
DevState<float>& state<float>(pic_ctx* c) { return c->sf; }
template <>
DevState<double>& state<double>(pic_ctx* c) { return c->sd; }

bool diag_step(pic_ctx* c) {
  return c->opt.diag_every > 0 && (c->step % c->opt.diag_every) == 0;
}

template <typename R>
int launch_particles(pic_ctx* c, int mode, int diag) {
  t_begin(c, mode == PIC_MODE_DEPOSIT ? 1 : 0);
  hipError_t e = pic_launch_particles<R>(state<R>(c), mode, diag, c->threads, c->stream);
  t_end(c);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("particle kernel: ") + hipGetErrorString(e));
  return PIC_OK;
}

// the next buffer (stayers + arrivals) becomes the current one
template <typename R>
void swap_buffers(DevState<R>& st) {
  for (int s = 0; s < PIC_MAXS; ++s) {
    std::swap(st.cell[s], st.ncell[s]);
    std::swap(st.ox[s], st.nox[s]);
    std::swap(st.oy[s], st.noy[s]);
    std::swap(st.ux[s], st.nux[s]);
    std::swap(st.uy[s], st.nuy[s]);
    std::swap(st.uz[s], st.nuz[s]);
    std::swap(st.id[s], st.nid[s]);
  }
}

template <typename R>
int launch_exchange(pic_ctx* c) {
  int ns = 0;
  for (auto& r : c->runs) ns = std::max(ns, r.n_species);
  t_begin(c, 2);
  hipError_t e = pic_launch_rebin<R>(state<R>(c), ns, c->stream);
  t_end(c);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("rebin: ") + hipGetErrorString(e));
  swap_buffers(state<R>(c));
  c->parity ^= 1;
  t_begin(c, 3);
  e = pic_launch_current_sum<R>(state<R>(c), c->tl.max_cells, c->stream);
  t_end(c);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("current sum: ") + hipGetErrorString(e));
  return PIC_OK;
}

int launch_field(pic_ctx* c, int diag, bool noalloc = false) {
  FieldArgs a = c->fa;
  if (noalloc) {
    const int r = pic_field_args_noalloc(a, c->device, c->tl.n_cells);
    if (r == -1) return fail(c, PIC_E_HIP, "the library's device scratch is not set up");
    if (r == -2)
      return fail(c, PIC_E_INVAL, "the allocation-free field solve holds at most 262144 cells "
                                  "(over all runs) and 4096 work-groups");
  }
  a.diag = diag;
  a.step = c->step;
  a.hist_slot = (int)(c->diag_count % std::max(1, c->opt.history_cap));
  a.learned = c->use_learned ? 1 : 0;
  a.collect = c->collect ? 1 : 0;
  a.pair_slot = c->pair_slots > 0 ? (int)(c->pairs_written % c->pair_slots) : 0;
  // (the allocation-free variant takes no event timing: events are created
  // on demand)
  if (!noalloc) t_begin(c, 5);
  hipError_t e = pic_launch_field_solve(a, c->stream);
  if (!noalloc) t_end(c);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("field solve: ") + hipGetErrorString(e));
  if (diag) c->diag_count += 1;
  if (c->collect) c->pairs_written += 1;
  return PIC_OK;
}

int read_stats(pic_ctx* c, pic_solve_stats* out) {
  const int n = (int)c->runs.size();
  std::vector<double>& h = c->h_stats;
  HIPCHK(c, hipMemcpyAsync(h.data(), c->d_stats, h.size() * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int rc = PIC_OK;
  for (int r = 0; r < n; ++r) {
    const double* st = h.data() + (size_t)r * PIC_STAT_WORDS;
    if (out) out[r].fallback = (int)st[12];
    for (int k = 0; k < 3; ++k) {
      const int it = (int)st[k];
      const double rel = st[3 + k], rec = st[16 + k];
      if (out) {
        out[r].iters[k] = it;
        out[r].relres[k] = rel;
        out[r].bnorm[k] = st[6 + k];
        out[r].learned_iters[k] = (int)st[9 + k];
        out[r].relres_recursive[k] = rec;
      }
      if (!std::isfinite(rel) || !std::isfinite(rec)) rc = PIC_E_NAN;
      else if (it >= c->runs[r].cg_maxit && rec > c->runs[r].cg_rtol && rc == PIC_OK)
        rc = PIC_E_NOCONV;
    }
  }
  if (rc == PIC_E_NOCONV) c->err = "field CG reached cg_maxit";
  if (rc == PIC_E_NAN) c->err = "non-finite CG residual";
  return rc;
}

int check_err(pic_ctx* c) {
  int h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, c->d_err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (h & PIC_ERRBIT_BARRIER)
    return fail(c, PIC_E_HIP, "field-solve grid barrier timed out (work-groups not co-resident)");
  if (h) {
    char buf[160];
    snprintf(buf, sizeof buf,
             "tile capacity exceeded (error bits 0x%x): a tile's particles outgrew its "
             "slots; raise slack", h);
    return fail(c, PIC_E_CAPACITY, buf);
  }
  return PIC_OK;
}

// device inflow of the shock runs that have one, before the particles move
template <typename R>
int launch_inflow(pic_ctx* c) {
  if (!c->any_inflow) return PIC_OK;
  int max_nty = 0, ns = 0;
  for (size_t r = 0; r < c->runs.size(); ++r) {
    max_nty = std::max(max_nty, c->tl.nty[r]);
    ns = std::max(ns, c->runs[r].n_species);
  }
  hipError_t e = pic_launch_inject_flow<R>(state<R>(c), c->d_inflow, c->d_inflow_step,
                                           (int)c->runs.size(), max_nty, ns, c->stream);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("inflow: ") + hipGetErrorString(e));
  return PIC_OK;
}

template <typename R>
int do_gather_push(pic_ctx* c) {
  int rc = launch_inflow<R>(c);
  if (rc) return rc;
  return launch_particles<R>(c, PIC_MODE_PUSH, diag_step(c) ? 1 : 0);
}
template <typename R>
int do_deposit(pic_ctx* c) {
  int rc = launch_particles<R>(c, PIC_MODE_DEPOSIT, 0);
  if (rc) return rc;
  return launch_exchange<R>(c);
}
// steps after whose re-binning the particles are reordered
bool sort_step(const pic_ctx* c, long long step) {
  const int k = c->opt.sort_every;
  return k > 0 && (step + 1) % k == 0;
}

template <typename R>
int launch_sort(pic_ctx* c) {
  int ns = 0;
  for (auto& r : c->runs) ns = std::max(ns, r.n_species);
  t_begin(c, 8);
  hipError_t e = pic_launch_sort<R>(state<R>(c), ns, c->tl.TXA * c->tl.TYA, c->stream);
  t_end(c);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("sort: ") + hipGetErrorString(e));
  swap_buffers(state<R>(c));
  c->parity ^= 1;
  return PIC_OK;
}

template <typename R>
int do_step(pic_ctx* c) {
  const int diag = diag_step(c) ? 1 : 0;
  int rc = launch_inflow<R>(c);
  if (rc) return rc;
  rc = launch_particles<R>(c, PIC_MODE_FUSED, diag);
  if (rc) return rc;
  rc = launch_exchange<R>(c);
  if (rc) return rc;
  if (sort_step(c, c->step)) {
    rc = launch_sort<R>(c);
    if (rc) return rc;
  }
  rc = launch_field(c, diag);
  if (rc) return rc;
  c->step += 1;
  return PIC_OK;
}

// Graph mode: two steps are captured once per starting buffer parity,
// reordering pattern and solver variant on an internal stream and replayed
// on the caller's stream. Everything a step reads that changes between steps
// lives in device memory (counts, fields, weights); what is baked into the
// graph (buffer pointers, which of the two steps end with a reordering, the
// solver variant, the diagnostics/collection switches) is the key.
bool graph_usable(pic_ctx* c) {
  if (!c->opt.graph || !c->graph_ok || c->timing || c->collect) return false;
  const int de = c->opt.diag_every;
  if (de > 0 && ((c->step % de) == 0 || ((c->step + 1) % de) == 0)) return false;
  return true;
}

template <typename R>
int graph_two_steps(pic_ctx* c) {
  // bit 0: the first step ends with a reordering, bit 1: the second
  const int pattern = (sort_step(c, c->step) ? 1 : 0) | (sort_step(c, c->step + 1) ? 2 : 0);
  const int slot = c->parity + 2 * pattern;
  const int key = c->use_learned ? 1 : 0;
  const bool cached = c->gexec[slot] && c->gkey[slot] == key;
  if (!cached) {
    if (c->gexec[slot]) {
      (void)hipGraphExecDestroy(c->gexec[slot]);
      c->gexec[slot] = nullptr;
    }
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      c->graph_ok = false;
      return PIC_E_HIP;
    }
    hipStream_t user = c->stream;
    const long long step0 = c->step, pairs0 = c->pairs_written, diag0 = c->diag_count;
    // the capture swaps the host's buffer pointers as the two steps do (twice
    // for the re-binnings, once per reordering): on success they stand where
    // the first replay leaves the device, on failure they are put back
    const int parity0 = c->parity;
    c->stream = c->cap_stream;
    c->fa.coop = 0;
    hipGraph_t g = nullptr;
    int rc = PIC_OK;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      rc = PIC_E_HIP;
    } else {
      rc = do_step<R>(c);
      if (rc == PIC_OK) rc = do_step<R>(c);
      if (hipStreamEndCapture(c->stream, &g) != hipSuccess) rc = PIC_E_HIP;
    }
    c->stream = user;
    c->fa.coop = 1;
    c->step = step0;
    c->pairs_written = pairs0;
    c->diag_count = diag0;
    hipGraphExec_t ex = nullptr;
    if (rc == PIC_OK && (!g || hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess))
      rc = PIC_E_HIP;
    if (g) (void)hipGraphDestroy(g);
    if (rc != PIC_OK) {
      // capture is not available: stay with plain launches from now on
      if (c->parity != parity0) {
        swap_buffers(state<R>(c));
        c->parity = parity0;
      }
      c->graph_ok = false;
      (void)hipGetLastError();
      return rc;
    }
    c->gexec[slot] = ex;
    c->gkey[slot] = key;
  }
  HIPCHK(c, hipGraphLaunch(c->gexec[slot], c->stream));
  if (cached && (pattern == 1 || pattern == 2)) {
    // a replay of a cached graph with one reordering: the device buffers end
    // swapped once against the start (a fresh capture has swapped already)
    swap_buffers(state<R>(c));
    c->parity ^= 1;
  }
  c->step += 2;
  c->graph_replays += 1;
  return PIC_OK;
}

// Parameters of the seeded drifting Maxwell-Juettner draw (the same recipe as
// the host generator): the boost and the rest-frame rejection envelope, a
// chi-3 piece below uc and a three-term Gamma mixture above.
PlasmaLoad plasma_load(uint64_t seed, int ppc, int x_cells, int ny, double gamma0, double T,
                       int direction) {
  PlasmaLoad L{};
  L.seed = seed;
  L.ppc = ppc;
  L.x_cells = x_cells;
  L.ny = ny;
  L.gamma0 = gamma0;
  L.beta = gamma0 > 1.0 ? (double)direction * std::sqrt(1.0 - 1.0 / (gamma0 * gamma0)) : 0.0;
  L.T = T;
  if (T > 0.0) {
    const double uc = 5.0 * std::sqrt(T);
    const double gc = std::sqrt(1.0 + uc * uc);
    const double s2 = 0.5 * (1.0 + gc) * T;
    const double sg = std::sqrt(s2);
    const double mass_a = std::pow(sg, 3.0) * std::sqrt(M_PI / 2.0);
    const double vc = uc / gc;
    const double lam = vc / T;
    const double c1 = uc * uc / lam, c2 = 2.0 * uc / std::pow(lam, 2.0),
                 c3 = 2.0 / std::pow(lam, 3.0);
    const double mass_b = std::exp(-(gc - 1.0) / T) * (c1 + c2 + c3);
    L.pa = mass_a / (mass_a + mass_b);
    L.s = sg;
    L.uc = uc;
    L.gc = gc;
    L.vc = vc;
    L.lam = lam;
    L.mix0 = c1 / (c1 + c2 + c3);
    L.mix1 = (c1 + c2) / (c1 + c2 + c3);
  }
  return L;
}

// In-cell offset in the particle precision. An FP64 offset just below 1 can
// round up to 1 in FP32; it is clamped to the largest value below 1 so that
// the particle keeps the cell (and hence the tile) it was binned into.
template <typename R>
R offset_below_one(double f) {
  const R r = (R)f;
  return r < R(1) ? r : std::nextafter(R(1), R(0));
}

template <typename R>
int load_impl(pic_ctx* c, int run, int s, int64_t n, const int32_t* ix, const int32_t* iy,
              const double* fx, const double* fy, const double* ux, const double* uy,
              const double* uz) {
  const pic_run_desc& d = c->runs[run];
  const Tiling& tl = c->tl;
  const int ntx = tl.ntx[run], nty = tl.nty[run], nt = ntx * nty;
  const int slots = c->plan.tile_slots[s];
  if (n > (int64_t)INT32_MAX) return fail(c, PIC_E_INVAL, "too many particles for int32 ids");
  std::vector<int> tile_of(n);
  std::vector<int> count(nt, 0);
  const int xmax = d.bc == PIC_BC_SHOCK ? d.nx - PIC_WALL_GAP : d.nx;
  for (int64_t k = 0; k < n; ++k) {
    if (ix[k] < 0 || ix[k] >= xmax || iy[k] < 0 || iy[k] >= d.ny || !(fx[k] >= 0.0) ||
        !(fx[k] < 1.0) || !(fy[k] >= 0.0) || !(fy[k] < 1.0) || !std::isfinite(ux[k]) ||
        !std::isfinite(uy[k]) || !std::isfinite(uz[k]))
      return fail(c, PIC_E_INVAL, "particle outside the grid, offset outside [0,1) or non-finite u");
    const int tx = std::min(ix[k] / tl.TX, ntx - 1);
    const int ty = std::min(iy[k] / tl.TY, nty - 1);
    tile_of[k] = ty * ntx + tx;
    if (++count[tile_of[k]] > slots)
      return fail(c, PIC_E_CAPACITY, "tile slots exceeded while loading; raise slack or ppc");
  }
  // Slot order inside a tile interleaves cells (the r-th particle of every
  // cell before the (r+1)-th of any), so the lanes of a wavefront deposit into
  // different cells instead of contending for the same LDS addresses.
  std::vector<int64_t> start(nt + 1, 0);
  for (int t = 0; t < nt; ++t) start[t + 1] = start[t] + count[t];
  std::vector<int64_t> order(n);
  std::vector<uint32_t> rank_in_cell(n);
  {
    std::vector<int> seen((size_t)d.nx * d.ny, 0);
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    for (int64_t k = 0; k < n; ++k) {
      rank_in_cell[k] = (uint32_t)seen[(size_t)iy[k] * d.nx + ix[k]]++;
      order[pos[tile_of[k]]++] = k;
    }
    const int cells_per_tile = tl.TXA * tl.TYA;
    for (int t = 0; t < nt; ++t) {
      auto key = [&](int64_t k) {
        const int tx = std::min(ix[k] / tl.TX, ntx - 1), ty = std::min(iy[k] / tl.TY, nty - 1);
        const int lc = (iy[k] - ty * tl.TY) * tl.TXA + (ix[k] - tx * tl.TX);
        return (uint64_t)rank_in_cell[k] * cells_per_tile + lc;
      };
      std::sort(order.begin() + start[t], order.begin() + start[t + 1],
                [&](int64_t a, int64_t b) { return key(a) < key(b); });
    }
  }
  const size_t tot = (size_t)nt * slots;
  std::vector<int> hcell(tot, -1), hid(tot, 0);
  std::vector<R> hox(tot, R(0)), hoy(tot, R(0)), hux(tot, R(0)), huy(tot, R(0)), huz(tot, R(0));
  std::vector<int> fill(nt, 0);
  for (int64_t kk = 0; kk < n; ++kk) {
    const int64_t k = order[kk];
    const int t = tile_of[k];
    const size_t o = (size_t)t * slots + fill[t]++;
    hcell[o] = (iy[k] << 16) | ix[k];
    hox[o] = offset_below_one<R>(fx[k]);
    hoy[o] = offset_below_one<R>(fy[k]);
    hux[o] = (R)ux[k];
    huy[o] = (R)uy[k];
    huz[o] = (R)uz[k];
    hid[o] = (int)k;
  }
  DevState<R>& st = state<R>(c);
  const size_t b0 = (size_t)tl.tile0[run] * slots;
  hipStream_t S = c->stream;
  HIPCHK(c, hipMemcpyAsync(st.cell[s] + b0, hcell.data(), tot * sizeof(int), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(st.ox[s] + b0, hox.data(), tot * sizeof(R), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(st.oy[s] + b0, hoy.data(), tot * sizeof(R), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(st.ux[s] + b0, hux.data(), tot * sizeof(R), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(st.uy[s] + b0, huy.data(), tot * sizeof(R), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(st.uz[s] + b0, huz.data(), tot * sizeof(R), hipMemcpyHostToDevice, S));
  if (st.id[s])
    HIPCHK(c, hipMemcpyAsync(st.id[s] + b0, hid.data(), tot * sizeof(int), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(st.cnt[s] + tl.tile0[run], count.data(), nt * sizeof(int),
                           hipMemcpyHostToDevice, S));
  HIPCHK(c, hipStreamSynchronize(S));
  c->next_id[run][s] = n;
  return PIC_OK;
}

// Append n particles to (run, species): staged sorted by tile, then one
// work-group per receiving tile copies them after the tile's particles.
template <typename R>
int inject_impl(pic_ctx* c, int run, int s, int64_t n, const int32_t* ix, const int32_t* iy,
                const double* fx, const double* fy, const double* ux, const double* uy,
                const double* uz) {
  const pic_run_desc& d = c->runs[run];
  const Tiling& tl = c->tl;
  const int ntx = tl.ntx[run], nty = tl.nty[run], nt = ntx * nty;
  const int slots = c->plan.tile_slots[s];
  if (n == 0) return PIC_OK;
  if (n > c->inj_cap)
    return fail(c, PIC_E_CAPACITY, "more particles than the injection staging holds "
                                   "(four cell columns of the run per call)");
  if (c->next_id[run][s] + n > (long long)INT32_MAX)
    return fail(c, PIC_E_INVAL, "particle ids exceed int32");
  const int xmax = d.bc == PIC_BC_SHOCK ? d.nx - PIC_WALL_GAP : d.nx;
  std::vector<int> tile_of(n), add(nt, 0);
  for (int64_t k = 0; k < n; ++k) {
    if (ix[k] < 0 || ix[k] >= xmax || iy[k] < 0 || iy[k] >= d.ny || !(fx[k] >= 0.0) ||
        !(fx[k] < 1.0) || !(fy[k] >= 0.0) || !(fy[k] < 1.0) || !std::isfinite(ux[k]) ||
        !std::isfinite(uy[k]) || !std::isfinite(uz[k]))
      return fail(c, PIC_E_INVAL, "injected particle outside the run, offset outside [0,1) "
                                  "or non-finite u");
    const int tx = std::min(ix[k] / tl.TX, ntx - 1);
    const int ty = std::min(iy[k] / tl.TY, nty - 1);
    tile_of[k] = ty * ntx + tx;
    add[tile_of[k]] += 1;
  }
  DevState<R>& st = state<R>(c);
  hipStream_t S = c->stream;
  std::vector<int> count(nt);
  HIPCHK(c, hipMemcpyAsync(count.data(), st.cnt[s] + tl.tile0[run], nt * sizeof(int),
                           hipMemcpyDeviceToHost, S));
  HIPCHK(c, hipStreamSynchronize(S));
  for (int t = 0; t < nt; ++t)
    if (count[t] + add[t] > slots)
      return fail(c, PIC_E_CAPACITY, "tile slots exceeded by injection; raise slack");
  std::vector<int> first(nt + 1, 0), list;
  for (int t = 0; t < nt; ++t) {
    first[t + 1] = first[t] + add[t];
    if (add[t]) {
      list.push_back(tl.tile0[run] + t);
      list.push_back(first[t]);
      list.push_back(add[t]);
    }
  }
  std::vector<int> hcell(n), hid(n), pos(first.begin(), first.end() - 1);
  std::vector<R> hox(n), hoy(n), hux(n), huy(n), huz(n);
  for (int64_t k = 0; k < n; ++k) {
    const int o = pos[tile_of[k]]++;
    hcell[o] = (iy[k] << 16) | ix[k];
    hox[o] = offset_below_one<R>(fx[k]);
    hoy[o] = offset_below_one<R>(fy[k]);
    hux[o] = (R)ux[k];
    huy[o] = (R)uy[k];
    huz[o] = (R)uz[k];
    hid[o] = (int)(c->next_id[run][s] + k);
  }
  HIPCHK(c, hipMemcpyAsync(c->d_inj_cell, hcell.data(), n * sizeof(int), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(c->d_inj_ox, hox.data(), n * sizeof(R), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(c->d_inj_oy, hoy.data(), n * sizeof(R), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(c->d_inj_ux, hux.data(), n * sizeof(R), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(c->d_inj_uy, huy.data(), n * sizeof(R), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(c->d_inj_uz, huz.data(), n * sizeof(R), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(c->d_inj_id, hid.data(), n * sizeof(int), hipMemcpyHostToDevice, S));
  HIPCHK(c, hipMemcpyAsync(c->d_inj_list, list.data(), list.size() * sizeof(int),
                           hipMemcpyHostToDevice, S));
  hipError_t e = pic_launch_inject<R>(st, s, (int)(list.size() / 3), c->d_inj_list, c->d_inj_cell,
                                      (const R*)c->d_inj_ox, (const R*)c->d_inj_oy,
                                      (const R*)c->d_inj_ux, (const R*)c->d_inj_uy,
                                      (const R*)c->d_inj_uz, c->d_inj_id, S);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("inject: ") + hipGetErrorString(e));
  HIPCHK(c, hipStreamSynchronize(S));
  c->next_id[run][s] += n;
  return PIC_OK;
}

template <typename R>
int read_impl(pic_ctx* c, int run, int s, int64_t cap, int32_t* ix, int32_t* iy, double* fx,
              double* fy, double* ux, double* uy, double* uz, int64_t* n_out) {
  const Tiling& tl = c->tl;
  const int nt = tl.ntx[run] * tl.nty[run];
  const int slots = c->plan.tile_slots[s];
  const size_t tot = (size_t)nt * slots;
  DevState<R>& st = state<R>(c);
  const size_t b0 = (size_t)tl.tile0[run] * slots;
  std::vector<int> hcell(tot), hid(tot), count(nt);
  std::vector<R> hox(tot), hoy(tot), hux(tot), huy(tot), huz(tot);
  hipStream_t S = c->stream;
  HIPCHK(c, hipMemcpyAsync(count.data(), st.cnt[s] + tl.tile0[run], nt * sizeof(int), hipMemcpyDeviceToHost, S));
  HIPCHK(c, hipMemcpyAsync(hcell.data(), st.cell[s] + b0, tot * sizeof(int), hipMemcpyDeviceToHost, S));
  HIPCHK(c, hipMemcpyAsync(hox.data(), st.ox[s] + b0, tot * sizeof(R), hipMemcpyDeviceToHost, S));
  HIPCHK(c, hipMemcpyAsync(hoy.data(), st.oy[s] + b0, tot * sizeof(R), hipMemcpyDeviceToHost, S));
  HIPCHK(c, hipMemcpyAsync(hux.data(), st.ux[s] + b0, tot * sizeof(R), hipMemcpyDeviceToHost, S));
  HIPCHK(c, hipMemcpyAsync(huy.data(), st.uy[s] + b0, tot * sizeof(R), hipMemcpyDeviceToHost, S));
  HIPCHK(c, hipMemcpyAsync(huz.data(), st.uz[s] + b0, tot * sizeof(R), hipMemcpyDeviceToHost, S));
  if (st.id[s])
    HIPCHK(c, hipMemcpyAsync(hid.data(), st.id[s] + b0, tot * sizeof(int), hipMemcpyDeviceToHost, S));
  HIPCHK(c, hipStreamSynchronize(S));
  int64_t n = 0;
  for (int t = 0; t < nt; ++t) n += count[t];
  *n_out = n;
  if (n > cap) return fail(c, PIC_E_INVAL, "output capacity smaller than the particle count");
  // storage positions in output order: ascending id (ids may have gaps once
  // a shock run has removed particles), or storage order without ids
  std::vector<std::pair<int, size_t>> order;
  order.reserve(n);
  int64_t seq = 0;
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < count[t]; ++k) {
      const size_t o = (size_t)t * slots + k;
      if (hcell[o] < 0) return fail(c, PIC_E_STATE, "particle store inconsistent (hole)");
      order.push_back({st.id[s] ? hid[o] : (int)seq++, o});
    }
  std::sort(order.begin(), order.end());
  for (size_t q = 1; q < order.size(); ++q)
    if (order[q].first == order[q - 1].first)
      return fail(c, PIC_E_STATE, "particle store inconsistent (duplicate id)");
  for (int64_t q = 0; q < n; ++q) {
    const size_t o = order[q].second;
    if (ix) ix[q] = hcell[o] & 0xffff;
    if (iy) iy[q] = hcell[o] >> 16;
    if (fx) fx[q] = (double)hox[o];
    if (fy) fy[q] = (double)hoy[o];
    if (ux) ux[q] = (double)hux[o];
    if (uy) uy[q] = (double)huy[o];
    if (uz) uz[q] = (double)huz[o];
  }
  return PIC_OK;
}

}  // namespace

namespace {

double* field_ptr(pic_ctx* c, int id) {
  const FieldArgs& f = c->fa;
  if (id >= PIC_EX && id <= PIC_EZ) return f.E[id - PIC_EX];
  if (id >= PIC_BX && id <= PIC_BZ) return f.B[id - PIC_BX];
  if (id >= PIC_JX && id <= PIC_JZ) return f.J[id - PIC_JX];
  return nullptr;
}

// charge density (species < 0) or one species' number density into d_rho
template <typename R>
int rho_impl(pic_ctx* c, int run, int species = -1) {
  hipError_t e = pic_launch_density<R>(state<R>(c), species, 256, c->stream);
  if (e == hipSuccess)
    e = pic_launch_charge_sum<R>(state<R>(c), run,
                                 (long long)c->runs[run].nx * c->runs[run].ny, c->d_rho, c->stream);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("charge: ") + hipGetErrorString(e));
  return PIC_OK;
}

// Work-groups of the persistent field solve: at most `cap` (and never more
// than can be co-resident), split over the runs in proportion to their cells,
// at least one each and no more than one per PIC_CG_THREADS cells.
void assign_cg_blocks(pic_ctx* c, int cap) {
  const int n_runs = (int)c->runs.size();
  int maxb = std::max(n_runs, std::min(c->max_cg_blocks, cap));
  long long want = 0;
  for (int r = 0; r < n_runs; ++r)
    want += ((long long)c->runs[r].nx * c->runs[r].ny + PIC_CG_THREADS - 1) / PIC_CG_THREADS;
  const int total = (int)std::min<long long>(maxb, std::max<long long>(want, n_runs));
  int blk = 0;
  for (int r = 0; r < n_runs; ++r) {
    const long long cells = (long long)c->runs[r].nx * c->runs[r].ny;
    long long nb = (long long)((double)total * cells / (double)c->tl.n_cells);
    const long long need = (cells + PIC_CG_THREADS - 1) / PIC_CG_THREADS;
    nb = std::max<long long>(1, std::min<long long>(nb, need));
    const int left = total - blk - (n_runs - 1 - r);
    nb = std::min<long long>(nb, left);
    if (r == n_runs - 1) nb = std::max<long long>(1, std::min<long long>(need, left));
    c->hruns[r].cg_blk_lo = blk;
    c->hruns[r].cg_blk_hi = blk + (int)nb;
    blk += (int)nb;
  }
  c->fa.n_blocks = blk;
  c->cg_cap = cap;
}

// Identity map plus small fixed noise (a splitmix64 sequence mapped to
// [-1, 1)), so that every channel receives gradient from the first update.
std::vector<float> initial_weights() {
  std::vector<float> w(NET_NW);
  uint64_t z = 0x2545F4914F6CDD1DULL;
  auto next = [&]() {
    z += 0x9E3779B97F4A7C15ULL;
    uint64_t x = z;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    x ^= x >> 31;
    return (double)(x >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  };
  const double amp = 0.01 * std::sqrt(3.0);   // standard deviation 0.01
  for (int k = 0; k < NET_C * 9; ++k) w[NET_W1 + k] = (float)(amp * next());
  for (int k = 0; k < NET_C * NET_C * 9; ++k)
    w[NET_W2 + k] = (float)(amp * next() / std::sqrt((double)NET_C));
  for (int k = 0; k < NET_C * 9; ++k) w[NET_W3 + k] = (float)(amp * next() / std::sqrt((double)NET_C));
  w[NET_W1 + 4] += 1.f;   // W1[0][1][1]
  w[NET_W2 + 4] += 1.f;   // W2[0][0][1][1]
  w[NET_W3 + 4] += 1.f;   // W3[0][1][1]
  return w;
}

// Corner of the training window of Adam update k: a splitmix64 hash of k
// mapped onto the field.
void crop_corner(long long k, int nx, int ny, int* ox, int* oy) {
  uint64_t x = 0x9E3779B97F4A7C15ULL * (uint64_t)(k + 1);
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  x ^= x >> 31;
  *ox = (int)((x & 0xFFFFFFFFULL) % (uint64_t)nx);
  *oy = (int)((x >> 32) % (uint64_t)ny);
}

}  // namespace

extern "C" {

int32_t pic_plan(const pic_run_desc* runs, int32_t n_runs, const pic_options* opt,
                 pic_plan_info* out) {
  if (!out) return PIC_E_INVAL;
  Tiling tl;
  std::string msg;
  return plan_impl(runs, n_runs, opt, out, &tl, &msg);
}

int32_t pic_init(const pic_run_desc* runs, int32_t n_runs, const pic_options* opt,
                 void* d_workspace, size_t ws_bytes, void* hip_stream, pic_ctx** out) {
  if (!out) return PIC_E_INVAL;
  *out = nullptr;
  g_init_err.clear();
  pic_ctx* c = new pic_ctx();
  std::string msg;
  int rc = plan_impl(runs, n_runs, opt, &c->plan, &c->tl, &msg);
  if (rc) {
    delete c;
    g_init_err = msg;
    return rc;
  }
  if (!d_workspace || ws_bytes < c->plan.workspace_bytes) {
    delete c;
    g_init_err = "workspace missing or smaller than pic_plan's workspace_bytes";
    return PIC_E_NOMEM;
  }
  c->runs.assign(runs, runs + n_runs);
  c->opt = *opt;
  if (c->opt.history_cap <= 0) c->opt.history_cap = 1;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (uint8_t*)d_workspace;
  c->ws_bytes = ws_bytes;
  c->fast = opt->precision == PIC_FP32_FAST;
  c->ids = opt->track_ids != 0;
  c->pair_slots = pair_slots_of(opt);
  c->learned = c->pair_slots > 0;
  std::vector<long long> net_cells;
  if (c->learned) {
    group_nets(runs, n_runs, &c->net_of_run, &c->net_first_run);
    for (int r : c->net_first_run) {
      net_cells.push_back((long long)runs[r].nx * runs[r].ny);
      c->train_cells = std::max(c->train_cells, net_cells.back());
    }
  }
  c->use_learned = c->learned;
  const long long ic = inject_cap_of(runs, n_runs);
  if (c->fast)
    carve<float>(c->ws, c->tl, c->plan, n_runs, true, c->split, c->ids, c->opt.history_cap,
                 c->pair_slots, net_cells, ic, c, &c->sf);
  else
    carve<double>(c->ws, c->tl, c->plan, n_runs, false, c->split, c->ids, c->opt.history_cap,
                  c->pair_slots, net_cells, ic, c, &c->sd);
  c->next_id.assign(n_runs, std::array<long long, PIC_MAXS>{0, 0});
  c->sf.nodal = c->sd.nodal = opt->gather == PIC_GATHER_NODAL ? 1 : 0;
  c->fa.learned_form = opt->learned_form;
  c->fa.cg_x0 = opt->cg_x0 == PIC_X0_PREV ? 1 : 0;
  c->fa.explicit_fdtd = opt->field_scheme == PIC_SCHEME_EXPLICIT ? 1 : 0;
  c->fa.coop = 1;
  c->fa.any_shock = 0;
  for (int r = 0; r < n_runs; ++r)
    if (runs[r].bc == PIC_BC_SHOCK) c->fa.any_shock = 1;
  c->fa.learned_maxit = opt->learned_maxit > 0 ? opt->learned_maxit : kDefaultLearnedMaxit;

  // CG work-groups: as many as can be co-resident, split over runs by cells
  int dev = 0, n_cu = 0;
  // an error left pending by an earlier runtime call of the process (not by
  // this library) is reported with the message, then cleared
  const hipError_t pending = hipGetLastError();
  hipError_t he = hipGetDevice(&dev);
  const char* what = "hipGetDevice";
  if (he == hipSuccess) {
    he = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    what = "hipDeviceGetAttribute";
  }
  if (he != hipSuccess) {
    delete c;
    g_init_err = std::string(what) + ": " + hipGetErrorString(he) +
                 (pending != hipSuccess ? std::string(" (pending before pic_init: ") +
                                              hipGetErrorString(pending) + ")"
                                        : std::string());
    return PIC_E_HIP;
  }
  if (pending != hipSuccess)
    c->err = std::string("note: an error was pending before pic_init and was cleared: ") +
             hipGetErrorString(pending);
  // the plain and the learned variant must both fit the same grid
  int maxb = pic_field_solve_max_blocks(n_cu, 0, 0);
  if (c->learned)
    maxb = std::min(maxb, pic_field_solve_max_blocks(n_cu, 1, opt->learned_form));
  if (maxb < n_runs) {
    delete c;
    g_init_err = "fewer co-resident field-solve work-groups than runs";
    return PIC_E_HIP;
  }
  c->max_cg_blocks = std::min(maxb, kMaxCgBlocks);
  c->device = dev;
  c->h_stats.assign((size_t)n_runs * PIC_STAT_WORDS, 0.0);
  // this device's copy of the allocation-free field solve's scratch
  he = pic_noalloc_scratch_init(dev);
  if (he != hipSuccess) {
    delete c;
    g_init_err = std::string("hipGetSymbolAddress of the field-solve scratch: ") +
                 hipGetErrorString(he);
    return PIC_E_HIP;
  }
  c->hruns.resize(n_runs);
  for (int r = 0; r < n_runs; ++r) {
    const pic_run_desc& d = runs[r];
    DevRun& h = c->hruns[r];
    memset(&h, 0, sizeof h);
    h.nx = d.nx;
    h.ny = d.ny;
    h.order = d.shape_order;
    h.nspecies = d.n_species;
    h.bc = d.bc;
    h.x_out = d.bc == PIC_BC_SHOCK ? d.nx - PIC_WALL_GAP : d.nx;
    h.ntx = c->tl.ntx[r];
    h.nty = c->tl.nty[r];
    h.tile0 = c->tl.tile0[r];
    h.cell0 = c->tl.cell0[r];
    h.dx = d.dx;
    h.dy = d.dy;
    h.dt = d.cfl * d.dx;
    h.theta = d.theta;
    h.cg_rtol = d.cg_rtol;
    h.cg_maxit = d.cg_maxit;
    if (c->learned) {
      h.net_id = c->net_of_run[r];
      if (c->net_first_run[h.net_id] == r) h.pairs = c->net_pairs[h.net_id];
    }
    for (int s = 0; s < d.n_species; ++s) {
      h.q[s] = d.species[s].q;
      h.m[s] = d.species[s].m;
    }
  }
  // By default the field solve launches every work-group that can be
  // co-resident (at most one per PIC_CG_THREADS cells of each run): its
  // sweeps stream some twenty arrays and need the whole chip (plain CG at
  // 8192 x 2048: 18.7 ms with 256 work-groups, 31.2 ms with 128), while the
  // grid barrier costs about 5.5 us at 256. pic_tune measures other counts.
  assign_cg_blocks(c, opt->cg_blocks > 0 ? opt->cg_blocks : c->max_cg_blocks);
  std::vector<int> tile_run(c->tl.n_tiles);
  for (int r = 0; r < n_runs; ++r)
    for (int t = 0; t < c->tl.ntx[r] * c->tl.nty[r]; ++t) tile_run[c->tl.tile0[r] + t] = r;

  hipStream_t S = c->stream;
  const char* step = "workspace clear";
  hipError_t e = hipMemsetAsync(c->ws, 0, c->plan.workspace_bytes, S);
  if (e == hipSuccess) {
    step = "run table upload";
    e = hipMemcpyAsync(c->d_runs, c->hruns.data(), sizeof(DevRun) * n_runs, hipMemcpyHostToDevice, S);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->d_tile_run, tile_run.data(), sizeof(int) * tile_run.size(),
                       hipMemcpyHostToDevice, S);
  if (e == hipSuccess && c->learned) {
    step = "network set-up";
    const std::vector<float> w0 = initial_weights();   // copies complete before the sync below
    std::vector<NetWeights> hn;
    for (auto& nt : c->nets) {
      if (e == hipSuccess)
        e = hipMemcpyAsync(nt.w, w0.data(), w0.size() * sizeof(float), hipMemcpyHostToDevice, S);
      if (e == hipSuccess) e = pic_net_refresh(nt, S);
      hn.push_back(NetWeights{nt.w, nt.w2b, nt.k49});
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->d_nets, hn.data(), hn.size() * sizeof(NetWeights),
                         hipMemcpyHostToDevice, S);
    if (e == hipSuccess) e = hipStreamSynchronize(S);
  }
  if (e == hipSuccess) {
    step = "initial synchronisation";
    e = hipStreamSynchronize(S);
  }
  if (e != hipSuccess) {
    delete c;
    g_init_err = std::string(step) + ": " + hipGetErrorString(e);
    return PIC_E_HIP;
  }
  *out = c;
  return PIC_OK;
}

int32_t pic_load_particles(pic_ctx* c, int32_t run, int32_t species, int64_t n, const int32_t* ix,
                           const int32_t* iy, const double* fx, const double* fy, const double* ux,
                           const double* uy, const double* uz) {
  if (!c) return PIC_E_INVAL;
  if (run < 0 || run >= (int)c->runs.size() || species < 0 ||
      species >= c->runs[run].n_species || n < 0 || (n > 0 && (!ix || !iy || !fx || !fy || !ux || !uy || !uz)))
    return fail(c, PIC_E_INVAL, "bad run/species/arguments");
  if (c->phase != 0) return fail(c, PIC_E_STATE, "load during a split step");
  return c->fast ? load_impl<float>(c, run, species, n, ix, iy, fx, fy, ux, uy, uz)
                 : load_impl<double>(c, run, species, n, ix, iy, fx, fy, ux, uy, uz);
}

int32_t pic_load_plasma(pic_ctx* c, int32_t run, int32_t species, const pic_plasma_desc* d) {
  if (!c || !d) return PIC_E_INVAL;
  if (run < 0 || run >= (int)c->runs.size() || species < 0 || species >= c->runs[run].n_species)
    return fail(c, PIC_E_INVAL, "bad run/species");
  if (c->phase != 0) return fail(c, PIC_E_STATE, "load during a split step");
  const pic_run_desc& rd = c->runs[run];
  const int xmax = rd.bc == PIC_BC_SHOCK ? rd.nx - PIC_WALL_GAP : rd.nx;
  const int xc = d->x_cells > 0 ? d->x_cells : rd.nx;
  if (d->ppc < 0 || xc > xmax || !(d->gamma0 >= 1.0) || !(d->T >= 0.0) ||
      (d->direction != 1 && d->direction != -1))
    return fail(c, PIC_E_INVAL, "plasma load needs ppc >= 0, x_cells within the particle "
                                "region, gamma0 >= 1, T >= 0, direction +-1");
  const Tiling& tl = c->tl;
  // capacity: the fullest tile holds widest x tallest cells
  const long long per_tile = (long long)tl.TXA * tl.TYA * d->ppc;
  if (per_tile > c->plan.tile_slots[species])
    return fail(c, PIC_E_CAPACITY, "tile slots smaller than ppc x tile cells; raise slack or ppc");
  const long long n = (long long)xc * rd.ny * d->ppc;
  if (n > (long long)INT32_MAX) return fail(c, PIC_E_INVAL, "too many particles for int32 ids");
  const PlasmaLoad L = plasma_load(d->seed, d->ppc, xc, rd.ny, d->gamma0, d->T, d->direction);
  const int nt = tl.ntx[run] * tl.nty[run];
  hipError_t e = c->fast
                     ? pic_launch_load_plasma<float>(c->sf, run, species, L, nt, c->stream)
                     : pic_launch_load_plasma<double>(c->sd, run, species, L, nt, c->stream);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("plasma load: ") + hipGetErrorString(e));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->next_id[run][species] = n;
  return PIC_OK;
}

int32_t pic_inject_particles(pic_ctx* c, int32_t run, int32_t species, int64_t n,
                             const int32_t* ix, const int32_t* iy, const double* fx,
                             const double* fy, const double* ux, const double* uy,
                             const double* uz) {
  if (!c) return PIC_E_INVAL;
  if (run < 0 || run >= (int)c->runs.size() || species < 0 ||
      species >= c->runs[run].n_species || n < 0 ||
      (n > 0 && (!ix || !iy || !fx || !fy || !ux || !uy || !uz)))
    return fail(c, PIC_E_INVAL, "bad run/species/arguments");
  if (c->runs[run].bc != PIC_BC_SHOCK)
    return fail(c, PIC_E_INVAL, "injection is for shock runs (PIC_BC_SHOCK)");
  if (c->phase != 0) return fail(c, PIC_E_STATE, "inject during a split step");
  return c->fast ? inject_impl<float>(c, run, species, n, ix, iy, fx, fy, ux, uy, uz)
                 : inject_impl<double>(c, run, species, n, ix, iy, fx, fy, ux, uy, uz);
}

int32_t pic_set_inflow(pic_ctx* c, int32_t run, const pic_inflow_desc* d) {
  if (!c || run < 0 || run >= (int)c->runs.size()) return PIC_E_INVAL;
  if (c->phase != 0) return fail(c, PIC_E_STATE, "set_inflow during a split step");
  const pic_run_desc& rd = c->runs[run];
  InflowDev f{};
  long long step0 = 0;
  if (d) {
    if (rd.bc != PIC_BC_SHOCK) return fail(c, PIC_E_INVAL, "inflow needs a PIC_BC_SHOCK run");
    if (d->ppc < 1 || !(d->gamma0 > 1.0) || !(d->T >= 0.0) || d->first_step < 0)
      return fail(c, PIC_E_INVAL, "inflow needs ppc >= 1, gamma0 > 1, T >= 0, first_step >= 0");
    const int x_out = rd.nx - PIC_WALL_GAP;
    const double beta0 = std::sqrt(1.0 - 1.0 / (d->gamma0 * d->gamma0));
    f.on = 1;
    f.w = beta0 * rd.cfl;
    f.ppc_w = (double)d->ppc * f.w;
    f.item0 = (long long)x_out * rd.ny * d->ppc;
    f.L = plasma_load(d->seed, d->ppc, x_out, rd.ny, d->gamma0, d->T, -1);
    // a step adds at most ceil(ppc w) particles per row to the tiles of the
    // entry column: the fullest tile must hold them on top of a full load
    const long long per_tile =
        (long long)c->tl.TXA * c->tl.TYA * d->ppc + (long long)std::ceil(f.ppc_w) * c->tl.TYA;
    for (int s = 0; s < rd.n_species; ++s)
      if (per_tile > c->plan.tile_slots[s])
        return fail(c, PIC_E_CAPACITY, "tile slots too few for the inflow; raise slack");
    step0 = d->first_step;
  }
  if (c->inflow.empty()) c->inflow.assign(c->runs.size(), InflowDev{});
  c->inflow[run] = f;
  c->any_inflow = false;
  for (const InflowDev& v : c->inflow) c->any_inflow = c->any_inflow || v.on;
  HIPCHK(c, hipMemcpyAsync(c->d_inflow + run, &c->inflow[run], sizeof(InflowDev),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_inflow_step + run, &step0, sizeof(long long),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // captured graphs hold the step's launches: capture again
  for (int k = 0; k < 8; ++k) c->gkey[k] = -1;
  return PIC_OK;
}

int32_t pic_read_particles(pic_ctx* c, int32_t run, int32_t species, int64_t cap, int32_t* ix,
                           int32_t* iy, double* fx, double* fy, double* ux, double* uy,
                           double* uz, int64_t* n_out) {
  if (!c || !n_out) return PIC_E_INVAL;
  if (run < 0 || run >= (int)c->runs.size() || species < 0 || species >= c->runs[run].n_species)
    return fail(c, PIC_E_INVAL, "bad run/species");
  return c->fast ? read_impl<float>(c, run, species, cap, ix, iy, fx, fy, ux, uy, uz, n_out)
                 : read_impl<double>(c, run, species, cap, ix, iy, fx, fy, ux, uy, uz, n_out);
}

// device array of a field of one run; the particle moments (charge, species
// densities) are deposited on demand into the density buffer
const double* field_src(pic_ctx* c, int run, int id, int* rc) {
  *rc = PIC_OK;
  if (id >= PIC_RHO) {
    if (id > PIC_RHO && id - PIC_N0 >= c->runs[run].n_species) {
      *rc = fail(c, PIC_E_INVAL, "no such species");
      return nullptr;
    }
    const int sp = id == PIC_RHO ? -1 : id - PIC_N0;
    *rc = c->fast ? rho_impl<float>(c, run, sp) : rho_impl<double>(c, run, sp);
    return *rc ? nullptr : c->d_rho;
  }
  return field_ptr(c, id) + c->tl.cell0[run];
}

int32_t pic_get_field(pic_ctx* c, int32_t run, int32_t id, double* host) {
  if (!c || !host || run < 0 || run >= (int)c->runs.size() || id < PIC_EX || id > PIC_N1)
    return fail(c, PIC_E_INVAL, "bad run/field/pointer");
  const long long n = (long long)c->runs[run].nx * c->runs[run].ny;
  int rc = PIC_OK;
  const double* src = field_src(c, run, id, &rc);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(host, src, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

int32_t pic_field_spectrum(pic_ctx* c, int32_t run, int32_t id, double* host) {
  if (!c || !host || run < 0 || run >= (int)c->runs.size() || id < PIC_EX || id > PIC_N1)
    return fail(c, PIC_E_INVAL, "bad run/field/pointer");
  if (c->phase != 0) return fail(c, PIC_E_STATE, "spectrum during a split step");
  const int nx = c->runs[run].nx, ny = c->runs[run].ny;
  const long long n = (long long)nx * ny;
  const long long o = c->tl.cell0[run];
  int rc = PIC_OK;
  const double* src = field_src(c, run, id, &rc);
  if (rc) return rc;
  // scratch: CG vectors, unused between field solves
  double* xr = c->fa.w0[0] + o;
  double* xi = c->fa.w0[1] + o;
  double* pw = c->fa.w1[0] + o;
  hipError_t e = pic_launch_spectrum(src, nx, ny, xr, xi, pw, c->stream);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("spectrum: ") + hipGetErrorString(e));
  HIPCHK(c, hipMemcpyAsync(host, pw, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

int32_t pic_transverse_average(pic_ctx* c, int32_t run, int32_t id, double* host) {
  if (!c || !host || run < 0 || run >= (int)c->runs.size() || id < PIC_EX || id > PIC_N1)
    return fail(c, PIC_E_INVAL, "bad run/field/pointer");
  if (c->phase != 0) return fail(c, PIC_E_STATE, "average during a split step");
  const int nx = c->runs[run].nx, ny = c->runs[run].ny;
  int rc = PIC_OK;
  const double* src = field_src(c, run, id, &rc);
  if (rc) return rc;
  double* out = c->fa.w1[1] + c->tl.cell0[run];   // CG vector, unused between solves
  hipError_t e = pic_launch_transverse_mean(src, nx, ny, out, c->stream);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("average: ") + hipGetErrorString(e));
  HIPCHK(c, hipMemcpyAsync(host, out, nx * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

int32_t pic_set_field(pic_ctx* c, int32_t run, int32_t id, const double* host) {
  if (!c || !host || run < 0 || run >= (int)c->runs.size() || id < PIC_EX || id > PIC_JZ)
    return fail(c, PIC_E_INVAL, "bad run/field/pointer");
  if (c->phase != 0) return fail(c, PIC_E_STATE, "set_field during a split step");
  const long long n = (long long)c->runs[run].nx * c->runs[run].ny;
  const long long o = c->tl.cell0[run];
  HIPCHK(c, hipMemcpyAsync(field_ptr(c, id) + o, host, n * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  if (c->fast && id <= PIC_BZ) {
    std::vector<float> h(n);
    for (long long k = 0; k < n; ++k) h[k] = (float)host[k];
    HIPCHK(c, hipMemcpyAsync(c->fa.Ef[id] + o, h.data(), n * sizeof(float), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

int32_t pic_gather_push(pic_ctx* c) {
  if (!c) return PIC_E_INVAL;
  if (c->phase != 0) return fail(c, PIC_E_STATE, "gather_push needs a completed step");
  int rc = c->fast ? do_gather_push<float>(c) : do_gather_push<double>(c);
  if (rc == PIC_OK) c->phase = 1;
  return rc;
}

int32_t pic_deposit(pic_ctx* c) {
  if (!c) return PIC_E_INVAL;
  if (c->phase != 1) return fail(c, PIC_E_STATE, "deposit must follow gather_push");
  int rc = c->fast ? do_deposit<float>(c) : do_deposit<double>(c);
  if (rc == PIC_OK) c->phase = 2;
  return rc;
}

int32_t pic_field_solve(pic_ctx* c, pic_solve_stats* stats) {
  if (!c) return PIC_E_INVAL;
  if (c->phase != 2) return fail(c, PIC_E_STATE, "field_solve must follow deposit");
  int rc = launch_field(c, diag_step(c) ? 1 : 0);
  if (rc) return rc;
  c->phase = 0;
  c->step += 1;
  rc = check_err(c);
  if (rc) return rc;
  return read_stats(c, stats);
}

int32_t pic_field_solve_noalloc(pic_ctx* c, pic_solve_stats* stats) {
  if (!c) return PIC_E_INVAL;
  if (c->phase != 2) return fail(c, PIC_E_STATE, "field_solve must follow deposit");
  int rc = launch_field(c, diag_step(c) ? 1 : 0, true);
  if (rc) return rc;
  c->phase = 0;
  c->step += 1;
  rc = check_err(c);
  if (rc) return rc;
  return read_stats(c, stats);
}

int32_t pic_step(pic_ctx* c, int32_t nsteps, pic_solve_stats* last) {
  if (!c || nsteps < 0) return PIC_E_INVAL;
  if (c->phase != 0) return fail(c, PIC_E_STATE, "pic_step during a split step");
  for (int k = 0; k < nsteps;) {
    if (nsteps - k >= 2 && graph_usable(c)) {
      int rc = c->fast ? graph_two_steps<float>(c) : graph_two_steps<double>(c);
      if (rc == PIC_OK) {
        k += 2;
        continue;
      }
      if (c->graph_ok) return rc;   // a launch error; otherwise fall through to eager
    }
    int rc = c->fast ? do_step<float>(c) : do_step<double>(c);
    if (rc) return rc;
    k += 1;
  }
  int rc = check_err(c);
  if (rc) return rc;
  return read_stats(c, last);
}

int32_t pic_history(pic_ctx* c, int32_t run, pic_diag_out* out, int32_t cap, int32_t* n_out) {
  if (!c || !n_out || run < 0 || run >= (int)c->runs.size()) return PIC_E_INVAL;
  const int hc = c->opt.history_cap;
  const long long have = std::min<long long>(c->diag_count, hc);
  std::vector<double> h((size_t)hc * PIC_REC_WORDS);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->d_history + (size_t)run * hc * PIC_REC_WORDS,
                           h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const long long first = c->diag_count - have;
  int n = 0;
  for (long long k = first; k < c->diag_count && n < cap; ++k, ++n) {
    const double* r = h.data() + (size_t)(k % hc) * PIC_REC_WORDS;
    pic_diag_out& o = out[n];
    memset(&o, 0, sizeof o);
    o.step = (int64_t)r[0];
    o.t = r[1];
    o.W_E = r[2];
    o.W_B = r[3];
    o.W_K_minus = r[4];
    o.W_K_plus = r[5];
    for (int q = 0; q < 3; ++q) {
      o.cg_iters[q] = (int)r[6 + q];
      o.cg_relres[q] = r[9 + q];
    }
  }
  *n_out = n;
  return PIC_OK;
}

int32_t pic_diag(pic_ctx* c, int32_t run, pic_diag_out* out) {
  if (!c || !out || run < 0 || run >= (int)c->runs.size()) return PIC_E_INVAL;
  if (c->phase != 0) return fail(c, PIC_E_STATE, "diag during a split step");
  memset(out, 0, sizeof *out);
  out->step = -1;
  if (c->diag_count > 0) {
    int n = 0;
    std::vector<pic_diag_out> all(std::min<long long>(c->diag_count, c->opt.history_cap));
    int rc = pic_history(c, run, all.data(), (int)all.size(), &n);
    if (rc) return rc;
    if (n > 0) *out = all[n - 1];
  }
  const Tiling& tl = c->tl;
  const int nt = tl.ntx[run] * tl.nty[run];
  for (int s = 0; s < c->runs[run].n_species; ++s) {
    std::vector<int> cnt(nt);
    int* src = c->fast ? c->sf.cnt[s] : c->sd.cnt[s];
    HIPCHK(c, hipMemcpyAsync(cnt.data(), src + tl.tile0[run], nt * sizeof(int),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    long long tot = 0;
    for (int v : cnt) tot += v;
    out->n_particles[s] = tot;
  }
  std::vector<double> st(PIC_STAT_WORDS);
  HIPCHK(c, hipMemcpyAsync(st.data(), c->d_stats + (size_t)run * PIC_STAT_WORDS,
                           st.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  int rc = c->fast ? rho_impl<float>(c, run) : rho_impl<double>(c, run);
  if (rc) return rc;
  const double* E[3] = {c->fa.E[0], c->fa.E[1], c->fa.E[2]};
  const double* B[3] = {c->fa.B[0], c->fa.B[1], c->fa.B[2]};
  hipError_t e = pic_launch_divergences(c->d_runs, run,
                                        (long long)c->runs[run].nx * c->runs[run].ny, E, B,
                                        c->d_rho, c->d_divpart, kDivBlocks, c->stream);
  if (e != hipSuccess) return fail(c, PIC_E_HIP, hipGetErrorString(e));
  std::vector<double> h(kDivBlocks * kDivWords);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->d_divpart, h.size() * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // maxima (NaN wins), the charge in block order, non-finite field values
  double g = 0, d = 0, q = 0, bad = 0;
  for (int b = 0; b < kDivBlocks; ++b) {
    const double* p = h.data() + (size_t)b * kDivWords;
    if (p[0] > g || std::isnan(p[0])) g = p[0];
    if (p[1] > d || std::isnan(p[1])) d = p[1];
    q += p[2];
    bad += p[3];
  }
  const pic_run_desc& rd = c->runs[run];
  out->gauss_max = g;
  out->divb_max = d;
  out->total_charge = q * rd.dx * rd.dy;
  out->fallbacks = (int64_t)st[13];
  out->solves = (int64_t)st[14];
  if (bad > 0) return fail(c, PIC_E_NAN, "non-finite E or B value");
  if (!std::isfinite(g) || !std::isfinite(d) || !std::isfinite(out->total_charge))
    return fail(c, PIC_E_NAN, "non-finite Gauss residual, div B or charge");
  if (out->step >= 0 && (!std::isfinite(out->W_E) || !std::isfinite(out->W_B) ||
                         !std::isfinite(out->W_K_minus) || !std::isfinite(out->W_K_plus)))
    return fail(c, PIC_E_NAN, "non-finite energy");
  return PIC_OK;
}

int32_t pic_timing(pic_ctx* c, int32_t on) {
  if (!c) return PIC_E_INVAL;
  t_resolve(c);
  c->timing = on != 0;
  for (int k = 0; k < kTimingClasses; ++k) {
    c->t_ms[k] = 0;
    c->t_n[k] = 0;
  }
  return PIC_OK;
}

int32_t pic_get_timing(pic_ctx* c, pic_timing_out* out) {
  if (!c || !out) return PIC_E_INVAL;
  t_resolve(c);
  for (int k = 0; k < kTimingClasses; ++k) {
    out->ms[k] = c->t_ms[k];
    out->launches[k] = c->t_n[k];
  }
  out->graph_replays = c->graph_replays;
  return PIC_OK;
}

int32_t pic_precond_collect(pic_ctx* c, int32_t on, int32_t* n_pairs) {
  if (!c) return PIC_E_INVAL;
  if (!c->learned) return fail(c, PIC_E_STATE, "collection needs solver PIC_SOLVER_LEARNED_PCG");
  c->collect = on != 0;
  if (n_pairs) *n_pairs = (int32_t)std::min<long long>(c->pairs_written, c->pair_slots);
  return PIC_OK;
}

int32_t pic_precond_use(pic_ctx* c, int32_t on) {
  if (!c) return PIC_E_INVAL;
  if (!c->learned) return fail(c, PIC_E_STATE, "the learned path needs solver PIC_SOLVER_LEARNED_PCG");
  c->use_learned = on != 0;
  return PIC_OK;
}

int32_t pic_precond_train(pic_ctx* c, const pic_train_opts* o, pic_train_stats* out) {
  if (!c || !o) return PIC_E_INVAL;
  if (!c->learned) return fail(c, PIC_E_STATE, "training needs solver PIC_SOLVER_LEARNED_PCG");
  if (o->epochs < 1) return fail(c, PIC_E_INVAL, "epochs must be >= 1");
  if (o->crop > kMaxTrainCrop) return fail(c, PIC_E_INVAL, "crop must be <= 128");
  const int crop = o->crop == 0 ? kDefaultTrainCrop : o->crop;
  const long long have = std::min<long long>(c->pairs_written, c->pair_slots);
  if (have < 1) return fail(c, PIC_E_STATE, "no training pairs recorded");
  const float lr = (float)(o->lr > 0 ? o->lr : 1e-3);
  hipStream_t S = c->stream;
  const long long oldest = c->pairs_written - have;
  const int n_nets = (int)c->nets.size();
  double first = 0, last = 0;
  int updates = 0;
  for (int ep = 0; ep < o->epochs; ++ep) {
    double sum = 0;
    // each network on the pairs of its first run, oldest pair first
    for (int g = 0; g < n_nets; ++g) {
      const NetTrain& T = c->nets[g];
      const pic_run_desc& d = c->runs[c->net_first_run[g]];
      const long long n1 = (long long)d.nx * d.ny;
      HIPCHK(c, hipMemsetAsync(T.scal, 0, 4 * sizeof(double), S));
      // a window, unless it would cover the whole field
      const bool whole = crop < 0 || (crop >= d.nx && crop >= d.ny);
      const int cx = whole ? 0 : std::min(crop, d.nx), cy = whole ? 0 : std::min(crop, d.ny);
      for (long long k = oldest; k < c->pairs_written; ++k) {
        const double* pb = c->net_pairs[g] + (size_t)(k % c->pair_slots) * 6 * n1;
        for (int comp = 0; comp < 3; ++comp) {
          int ox = 0, oy = 0;
          crop_corner(c->adam_step, d.nx, d.ny, &ox, &oy);
          HIPCHK(c, pic_net_grad(T, pb + (size_t)(2 * comp) * n1, pb + (size_t)(2 * comp + 1) * n1,
                                 d.nx, d.ny, ox, oy, cx, cy, S));
          HIPCHK(c, pic_net_adam(T, lr, ++c->adam_step, S));
          ++updates;
        }
      }
      double scal[4];
      HIPCHK(c, hipMemcpyAsync(scal, T.scal, sizeof scal, hipMemcpyDeviceToHost, S));
      HIPCHK(c, hipStreamSynchronize(S));
      sum += scal[2];
    }
    const double mean = sum / (double)(have * 3 * n_nets);
    if (ep == 0) first = mean;
    last = mean;
  }
  for (auto& T : c->nets) HIPCHK(c, pic_net_refresh(T, S));
  HIPCHK(c, hipStreamSynchronize(S));
  if (out) {
    out->loss_first = first;
    out->loss_last = last;
    out->samples = (int32_t)(have * 3 * n_nets);
    out->updates = updates;
    out->networks = n_nets;
  }
  if (!std::isfinite(last)) return fail(c, PIC_E_NAN, "non-finite training loss");
  return PIC_OK;
}

int32_t pic_precond_get_weights(pic_ctx* c, float* host, size_t n) {
  if (!c || !host) return PIC_E_INVAL;
  if (!c->learned) return fail(c, PIC_E_STATE, "no network (solver is not PIC_SOLVER_LEARNED_PCG)");
  if (n != (size_t)NET_NW * c->nets.size())
    return fail(c, PIC_E_INVAL, "weight count must be 9792 per network");
  for (size_t g = 0; g < c->nets.size(); ++g)
    HIPCHK(c, hipMemcpyAsync(host + g * NET_NW, c->nets[g].w, NET_NW * sizeof(float),
                             hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

int32_t pic_precond_set_weights(pic_ctx* c, const float* host, size_t n) {
  if (!c || !host) return PIC_E_INVAL;
  if (!c->learned) return fail(c, PIC_E_STATE, "no network (solver is not PIC_SOLVER_LEARNED_PCG)");
  if (n != (size_t)NET_NW * c->nets.size())
    return fail(c, PIC_E_INVAL, "weight count must be 9792 per network");
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(host[k])) return fail(c, PIC_E_INVAL, "non-finite weight");
  for (size_t g = 0; g < c->nets.size(); ++g) {
    HIPCHK(c, hipMemcpyAsync(c->nets[g].w, host + g * NET_NW, NET_NW * sizeof(float),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, pic_net_refresh(c->nets[g], c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

int32_t pic_precond_apply(pic_ctx* c, int32_t form, int32_t nx, int32_t ny, const double* d_in,
                          double* d_out) {
  if (!c || !d_in || !d_out) return PIC_E_INVAL;
  if (!c->learned) return fail(c, PIC_E_STATE, "no network (solver is not PIC_SOLVER_LEARNED_PCG)");
  if (form != PIC_NET_COLLAPSED && form != PIC_NET_MFMA)
    return fail(c, PIC_E_INVAL, "form must be PIC_NET_COLLAPSED or PIC_NET_MFMA");
  if (nx < 3 || ny < 3 || (long long)nx * ny > c->train_cells)
    return fail(c, PIC_E_INVAL, "need nx, ny >= 3 and nx * ny <= the largest first run's cells");
  HIPCHK(c, pic_net_apply(c->nets[0], form, d_in, d_out, nx, ny, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

int32_t pic_precond_grad(pic_ctx* c, int32_t nx, int32_t ny, const double* d_b, const double* d_t,
                         const int32_t* window, float* host_grad, size_t n, double* loss) {
  if (!c || !d_b || !d_t || !host_grad) return PIC_E_INVAL;
  if (!c->learned) return fail(c, PIC_E_STATE, "no network (solver is not PIC_SOLVER_LEARNED_PCG)");
  if (n != (size_t)NET_NW) return fail(c, PIC_E_INVAL, "gradient count must be 9792");
  if (nx < 3 || ny < 3)
    return fail(c, PIC_E_INVAL, "need nx, ny >= 3");
  int ox = 0, oy = 0, cx = 0, cy = 0;
  if (window) {
    ox = window[0];
    oy = window[1];
    cx = window[2];
    cy = window[3];
    if (ox < 0 || ox >= nx || oy < 0 || oy >= ny || cx < 1 || cy < 1 || cx > nx || cy > ny ||
        cx > kMaxTrainCrop || cy > kMaxTrainCrop)
      return fail(c, PIC_E_INVAL, "window corner outside the field or size outside [1, min(n, 128)]");
  } else if ((long long)nx * ny > c->train_cells) {
    return fail(c, PIC_E_INVAL, "need nx * ny <= the largest first run's cells");
  }
  const NetTrain& T = c->nets[0];
  HIPCHK(c, hipMemsetAsync(T.scal, 0, 4 * sizeof(double), c->stream));
  HIPCHK(c, pic_net_grad(T, d_b, d_t, nx, ny, ox, oy, cx, cy, c->stream));
  double scal[4];
  HIPCHK(c, hipMemcpyAsync(scal, T.scal, sizeof scal, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(host_grad, T.grad, n * sizeof(float), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = scal[1];
  return PIC_OK;
}

int32_t pic_tune(pic_ctx* c, const pic_tune_opts* o, pic_tune_out* out) {
  if (!c || !o) return PIC_E_INVAL;
  if (c->phase != 0) return fail(c, PIC_E_STATE, "pic_tune during a split step");
  if (o->steps < 1 || o->n_split < 0 || o->n_split > 8 || o->n_cg < 0 || o->n_cg > 8)
    return fail(c, PIC_E_INVAL, "steps >= 1 and at most 8 candidates per parameter");
  std::vector<int> ks, cgs;
  if (o->n_split == 0) {
    for (int k = 1; k <= 8; k *= 2)
      if (k <= c->plan.tile_split) ks.push_back(k);
  } else {
    for (int q = 0; q < o->n_split; ++q) {
      if (o->split[q] < 1 || o->split[q] > c->plan.tile_split)
        return fail(c, PIC_E_INVAL, "split candidate outside [1, planned tile_split]");
      ks.push_back(o->split[q]);
    }
  }
  if (o->n_cg == 0) {
    for (int b = 64; b <= 512; b *= 2)
      if (b <= c->max_cg_blocks) cgs.push_back(b);
    if (cgs.empty()) cgs.push_back(c->max_cg_blocks);
  } else {
    for (int q = 0; q < o->n_cg; ++q) {
      if (o->cg_blocks[q] < 1) return fail(c, PIC_E_INVAL, "cg_blocks candidate must be >= 1");
      cgs.push_back(o->cg_blocks[q]);
    }
  }
  const bool timing0 = c->timing;
  auto timed = [&](int cls, double* ms) -> int {
    t_resolve(c);
    c->timing = true;
    for (int k = 0; k < kTimingClasses; ++k) c->t_ms[k] = c->t_n[k] = 0;
    for (int q = 0; q < o->steps; ++q) {
      int rc = c->fast ? do_step<float>(c) : do_step<double>(c);
      if (rc) return rc;
    }
    t_resolve(c);
    *ms = c->t_ms[cls] / o->steps;
    return check_err(c);
  };
  auto set_split = [&](int K) {
    c->sf.K = K;
    c->sd.K = K;
    c->fa.K = K;
  };
  pic_tune_out res{};
  int best_k = ks[0];
  double best = 1e300;
  for (size_t q = 0; q < ks.size(); ++q) {
    set_split(ks[q]);
    double ms = 0;
    int rc = timed(0, &ms);
    if (rc) return rc;
    res.split[q] = ks[q];
    res.particle_ms[q] = ms;
  }
  // within kTuneTie of the fastest counts as equal: the earliest candidate wins
  for (size_t q = 0; q < ks.size(); ++q) best = std::min(best, res.particle_ms[q]);
  for (size_t q = 0; q < ks.size(); ++q)
    if (res.particle_ms[q] <= best * (1.0 + kTuneTie)) {
      best_k = ks[q];
      break;
    }
  res.n_split = (int)ks.size();
  set_split(best_k);
  res.tile_split = best_k;
  int best_cap = cgs[0];
  best = 1e300;
  for (size_t q = 0; q < cgs.size(); ++q) {
    assign_cg_blocks(c, cgs[q]);
    HIPCHK(c, hipMemcpyAsync(c->d_runs, c->hruns.data(), sizeof(DevRun) * c->runs.size(),
                             hipMemcpyHostToDevice, c->stream));
    double ms = 0;
    int rc = timed(5, &ms);
    if (rc) return rc;
    res.cg_blocks_tried[q] = c->fa.n_blocks;
    res.field_ms[q] = ms;
  }
  for (size_t q = 0; q < cgs.size(); ++q) best = std::min(best, res.field_ms[q]);
  for (size_t q = 0; q < cgs.size(); ++q)
    if (res.field_ms[q] <= best * (1.0 + kTuneTie)) {
      best_cap = cgs[q];
      break;
    }
  res.n_cg = (int)cgs.size();
  assign_cg_blocks(c, best_cap);
  HIPCHK(c, hipMemcpyAsync(c->d_runs, c->hruns.data(), sizeof(DevRun) * c->runs.size(),
                           hipMemcpyHostToDevice, c->stream));
  res.cg_blocks = c->fa.n_blocks;
  // captured graphs hold the old grids
  for (auto& g : c->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  t_resolve(c);
  c->timing = timing0;
  for (int k = 0; k < kTimingClasses; ++k) c->t_ms[k] = c->t_n[k] = 0;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (out) *out = res;
  return PIC_OK;
}

int32_t pic_sync(pic_ctx* c) {
  if (!c) return PIC_E_INVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return check_err(c);
}

int32_t pic_destroy(pic_ctx* c) {
  if (!c) return PIC_OK;
  (void)hipStreamSynchronize(c->stream);
  for (auto& g : c->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
  return PIC_OK;
}

const char* pic_last_error(const pic_ctx* c) {
  if (c) return c->err.c_str();
  return g_init_err.empty() ? "null context" : g_init_err.c_str();
}

const char* pic_status_str(int32_t s) {
  switch (s) {
    case PIC_OK: return "PIC_OK";
    case PIC_E_INVAL: return "PIC_E_INVAL";
    case PIC_E_NOMEM: return "PIC_E_NOMEM";
    case PIC_E_HIP: return "PIC_E_HIP";
    case PIC_E_NOCONV: return "PIC_E_NOCONV";
    case PIC_E_CAPACITY: return "PIC_E_CAPACITY";
    case PIC_E_NAN: return "PIC_E_NAN";
    case PIC_E_STATE: return "PIC_E_STATE";
    default: return "unknown status";
  }
}

}  // extern "C"
