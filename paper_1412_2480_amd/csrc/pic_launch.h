// Host-side launch interfaces between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "pic_dev.h"

#define PIC_REC_WORDS 16   // doubles per history record

#define PIC_CG_THREADS 512    // work-group size of the persistent field solve

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
  double* part;            // per-block partial sums, 2 x [block][8]
  int* g_active;           // active-run counters (3)
  unsigned* bar;           // grid barrier: counter at [0], generation at [32]
  int* err;                // error bits
  double* stats;           // [run][9]: iters, relres, ||b||
  const double* wk_part;   // [tile][K][species][2] kinetic partials
  int K;                   // work-groups per tile in the particle kernel
  double* history;         // [run][hist_cap][PIC_REC_WORDS]
  int hist_cap, hist_slot;
  long long step;
};

int pic_field_solve_max_blocks(int n_cu);
hipError_t pic_launch_field_solve(const FieldArgs& a, hipStream_t s);

enum PicParticleMode { PIC_MODE_FUSED = 0, PIC_MODE_PUSH = 1, PIC_MODE_DEPOSIT = 2 };

template <typename R>
hipError_t pic_launch_particles(const DevState<R>& st, int mode, int diag, int threads,
                                hipStream_t s);
template <typename R>
hipError_t pic_launch_rebin(const DevState<R>& st, int n_species, hipStream_t s);
template <typename R>
hipError_t pic_launch_current_sum(const DevState<R>& st, long long max_cells, hipStream_t s);
template <typename R>
hipError_t pic_launch_charge_sum(const DevState<R>& st, int run, long long ncell, double* rho,
                                 hipStream_t s);
template <typename R>
size_t pic_particle_smem(const DevState<R>& st, int mode);

hipError_t pic_launch_divergences(const DevRun* runs, int run, long long ncell,
                                  const double* const* E, const double* const* B,
                                  const double* rho, double* partial_max, int n_blocks,
                                  hipStream_t s);
