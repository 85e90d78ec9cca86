// Host-side launch interfaces between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "net_dev.h"
#include "pic_dev.h"

#define PIC_REC_WORDS 16   // doubles per history record

#define PIC_CG_THREADS 512    // work-group size of the persistent field solve
// grid barrier of the persistent field solve: arrival groups, and its words
// (group counters, top counter and generation, each on its own 128-byte line)
constexpr unsigned kBarGroups = 16;
constexpr int kBarWords = 32 * (kBarGroups + 2);
// doubles per run of solve statistics: 0-2 iterations, 3-5 true relative
// residual, 6-8 ||b||, 9-11 learned iterations, 12 fallback, 13 fallbacks and
// 14 solves since initialisation, 16-18 recursive relative residual
#define PIC_STAT_WORDS 24
// doubles of the solve's partial-sum buffer the true-residual sweep may use
// (the buffer holds 24 per field-solve work-group, at least 4096 of them)
#define PIC_RES_PART_DOUBLES 98304

struct FieldArgs {
  int n_runs, n_blocks, diag;
  const DevRun* runs;
  double* E[3];
  double* B[3];
  double* J[3];
  float* Ef[6];            // FP32 copies (null pointers in the FP64 form)
  double* x[3];            // dB
  double* p[3];
  double* r0[3];           // r, w = A r and s = A p, double-buffered
  double* r1[3];
  double* w0[3];
  double* w1[3];
  double* s0[3];
  double* s1[3];
  double* bsv[3];          // b of Eq. (7), kept for the true residual and the pairs
  double* part;            // per-block partial sums, 3 x [block][8]
  int* g_active;           // active-run counters (3)
  unsigned* bar;           // grid barrier: counter at [0], generation at [32]
  int* err;                // error bits
  double* stats;           // [run][PIC_STAT_WORDS]: iters, relres, ||b||, learned iters, fallback
  const double* wk_part;   // [tile][K][species][2] kinetic partials
  int K;                   // work-groups per tile in the particle kernel
  double* history;         // [run][hist_cap][PIC_REC_WORDS]
  int hist_cap, hist_slot;
  long long step;
  int learned;             // x0 = N(b) and flexible CG preconditioned by N
  int learned_form;        // 0: collapsed 7 x 7 filter (FP64), 1: BF16 network
  int learned_maxit;       // iteration budget of the learned solver
  const NetWeights* nets;  // one network per distinct operator (DevRun::net_id)
  int collect;             // record (b, dB) of each network's first run into its ring
  int pair_slot;           // ring slot: pairs + pair_slot * 6 * ncell, [component][b | dB]
  int coop;                // 1: cooperative launch; 0: ordinary launch (graph capture)
  int any_shock;           // some run has shock walls (selects the kernel variant)
  int cg_x0;               // 1: plain CG starts from the previous step's dB
  int explicit_fdtd;       // 1: explicit Yee advance of Eqs. (3)-(4) instead of the solve
};

// The allocation-free field solve: largest total cells of a context and
// largest field-solve grid it serves; its scratch is a device array of the
// library (about 57 MB per GPU).
#define PIC_NOALLOC_MAX_CELLS (1LL << 18)
#define PIC_NOALLOC_MAX_BLOCKS 4096
// once per device, with it current: look up this GPU's copy of the array
hipError_t pic_noalloc_scratch_init(int dev);
// point the scratch of the solve's arguments into it: 0, or -1 (not set up
// on this device), -2 (more cells or work-groups than it holds)
int pic_field_args_noalloc(FieldArgs& a, int dev, long long n_cells);

size_t pic_field_solve_smem(int learned, int form);
// co-resident work-groups of the solve kernel variant (plain, or learned in
// the given form) over n_cu compute units
int pic_field_solve_max_blocks(int n_cu, int learned, int form);
hipError_t pic_launch_field_solve(const FieldArgs& a, hipStream_t s);

enum PicParticleMode { PIC_MODE_FUSED = 0, PIC_MODE_PUSH = 1, PIC_MODE_DEPOSIT = 2 };

template <typename R>
hipError_t pic_launch_particles(const DevState<R>& st, int mode, int diag, int threads,
                                hipStream_t s);
template <typename R>
hipError_t pic_launch_rebin(const DevState<R>& st, int n_species, hipStream_t s);
// reorder every tile's current particles into the next store (cell-sorted,
// one contiguous run per wavefront lane); max_tile_cells = widest tile's cells
template <typename R>
hipError_t pic_launch_sort(const DevState<R>& st, int n_species, int max_tile_cells,
                           hipStream_t s);
// append staged particles (list of (tile, first, count)) to the current store
template <typename R>
hipError_t pic_launch_inject(const DevState<R>& st, int s, int n_entries, const int* list,
                             const int* cell, const R* ox, const R* oy, const R* ux, const R* uy,
                             const R* uz, const int* id, hipStream_t stream);
template <typename R>
hipError_t pic_launch_current_sum(const DevState<R>& st, long long max_cells, hipStream_t s);
template <typename R>
hipError_t pic_launch_charge_sum(const DevState<R>& st, int run, long long ncell, double* rho,
                                 hipStream_t s);
template <typename R>
size_t pic_particle_smem(const DevState<R>& st, int mode);
// node density of one species (species >= 0: particles per unit area) or the
// charge density (species < 0) into the current patches; pic_launch_charge_sum
// then sums them
template <typename R>
hipError_t pic_launch_density(const DevState<R>& st, int species, int threads, hipStream_t s);
// profile(i) = mean over j of one [ny][nx] field
hipError_t pic_launch_transverse_mean(const double* f, int nx, int ny, double* out,
                                      hipStream_t s);

hipError_t pic_launch_divergences(const DevRun* runs, int run, long long ncell,
                                  const double* const* E, const double* const* B,
                                  const double* rho, double* partial_max, int n_blocks,
                                  hipStream_t s);

// Training state of the learned aid: FP32 weights and Adam moments, the BF16
// copy used by the matrix cores, and whole-field activation buffers of the
// largest training grid.
struct NetTrain {
  float* w;              // [NET_NW]
  __bf16* w2b;           // [9][NET_C][NET_C]
  double* k49;           // collapsed filter [7][7]
  float *grad, *m, *v;   // [NET_NW]
  float* part;           // [wg_blocks][NET_C * NET_C * 9]
  float *xin, *y, *gy;   // [ncell]
  double* tc;            // [ncell]: target of a training crop
  float *h1, *h2, *gh1, *gh2;   // [NET_C][ncell]
  double* dpart;         // [256][2]
  double* scal;          // [4]: sum t^2, loss, loss accumulator
  int wg_blocks;
};

// BF16 copy of W2 and the collapsed filter, after any change of the weights
hipError_t pic_net_refresh(const NetTrain& T, hipStream_t s);
// out = N(in) on an nx x ny periodic field (form 0 collapsed, 1 network)
hipError_t pic_net_apply(const NetTrain& T, int form, const double* in, double* out, int nx,
                         int ny, hipStream_t s);
// loss and weight gradient of one sample: the whole nx x ny periodic field
// (cx <= 0) or the cx x cy window at (ox, oy); the training buffers must hold
// (cx + 6) (cy + 6) cells
hipError_t pic_net_grad(const NetTrain& T, const double* b, const double* t, int nx, int ny,
                        int ox, int oy, int cx, int cy, hipStream_t s);
hipError_t pic_net_adam(const NetTrain& T, float lr, int step, hipStream_t s);

// power spectrum |F(k)|^2 / (nx ny)^2 of one [ny][nx] field (DFT order);
// xr, xi: nx * ny doubles of scratch each
hipError_t pic_launch_spectrum(const double* f, int nx, int ny, double* xr, double* xi,
                               double* power, hipStream_t s);

// Device-side seeded plasma load (same items as the host generator)
struct PlasmaLoad {
  unsigned long long seed;
  int ppc, x_cells, ny;
  double gamma0, beta, T;
  // rejection envelope of the rest-frame Maxwell-Juettner speed
  double pa, s, uc, gc, vc, lam, mix0, mix1;
};
template <typename R>
hipError_t pic_launch_load_plasma(const DevState<R>& st, int run, int s, const PlasmaLoad& L,
                                  int n_tiles_run, hipStream_t stream);

// Inflow of a shock run, injected on the device before every step
struct InflowDev {
  int on;
  double ppc_w;          // ppc * beta0 * cfl: particles per row per step, accumulated
  double w;              // beta0 * cfl: the slab width in cells
  long long item0;       // x_out * ny * ppc: first item after the initial load
  PlasmaLoad L;          // momentum draw (direction -x)
};
template <typename R>
hipError_t pic_launch_inject_flow(const DevState<R>& st, const InflowDev* tab, long long* step_ctr,
                                  int n_runs, int max_nty, int n_species, hipStream_t stream);
