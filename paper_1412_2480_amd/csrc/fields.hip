// Implicit field solve of Ikeya & Matsumoto (PASJ 2015), Sec. 2:
//   Eq. (7):  [1 - (theta c dt)^2 L] dB = theta (c dt)^2 (L B^n + (4 pi/c) curl J^{n+1/2})
//                                       - c dt curl E^n
//   solved by conjugate gradients (the paper cites Hoshino 2013 for CG), then
//   Eqs. (5)-(6): E^{n+1} = E^n + c dt curl(B^n + theta dB) - 4 pi dt J,
//                 B^{n+1} = B^n + dB.
//
// One persistent kernel per step does all of it for every run of the
// context: each run owns a contiguous range of work-groups, the three B
// components are solved together (three recurrences sharing one sweep), and
// grid-wide barriers separate the phases. All arithmetic of the solve is FP64;
// block reductions are deterministic and are summed across a run's blocks in
// a fixed order, so every block of a run holds bit-identical scalars.
//
// Plain solver: the Chronopoulos-Gear form of CG (Chronopoulos & Gear 1989),
// which produces the iterates of CG in exact arithmetic with a single global
// reduction, <r,r> and <Ar,r> together, per iteration. The residual at a
// neighbour, r_{k+1} = r_k - alpha_k (w_k + beta_k s_{k-1}), is recomputed
// from the previous iteration's buffers, so each iteration is one sweep and one
// barrier:
//   p_k = r_k + beta_k p_{k-1},  s_k = w_k + beta_k s_{k-1}   (s = A p)
//   x_{k+1} = x_k + alpha_k p_k, r_{k+1} = r_k - alpha_k s_k, w_{k+1} = A r_{k+1}
//   gamma = <r,r>, delta = <w,r>, beta = gamma_{k+1}/gamma_k,
//   alpha_{k+1} = gamma_{k+1} / (delta_{k+1} - beta_{k+1} gamma_{k+1}/alpha_k).
//
// Explicit variant (the Yee FDTD of Eqs. (3)-(4), which the paper contrasts
// with the implicit solver): B carried at integer times for the particle push,
// advanced in three sweeps separated by grid barriers,
//   B^{n+1/2} = B^n - (c dt/2) curl E^n,
//   E^{n+1}   = E^n + c dt curl B^{n+1/2} - 4 pi dt J^{n+1/2},
//   B^{n+1}   = B^{n+1/2} - (c dt/2) curl E^{n+1},
// whose half-step values are the leapfrog of Eqs. (3)-(4).
//
// Learned solver (an addition to the method): x_0 = N(b) and flexible CG
// with z = N(r) as preconditioner and the Polak-Ribiere beta,
// beta = <z_{k+1}, r_{k+1} - r_k>/<z_k, r_k> = -alpha_k <z_{k+1}, q_k>/<z_k, r_k>,
// to the same relative residual; if it has not converged within its
// iteration budget the plain solver restarts from the current iterate. N is
// applied either as the BF16 network on the matrix cores or as its exact
// collapsed 7 x 7 filter in FP64.
#include <math.h>

#include "net_dev.h"
#include "pic_dev.h"
#include "pic_launch.h"

namespace {

constexpr int kThreads = PIC_CG_THREADS;
constexpr int kWaves = kThreads / 64;
constexpr double kFourPi = 12.566370614359172953850573533118;
constexpr long kSpinLimit = 1L << 26;   // about seconds of polling: a stalled grid errors out

struct Loc {
  long long base;   // cell0 of the run
  int nx, ny;
};

__device__ __forceinline__ long long lidx(const Loc& L, int i, int j) {
  return L.base + (long long)pic_wrap(j, L.ny) * L.nx + pic_wrap(i, L.nx);
}

// Grid barrier in two levels: every block makes its writes visible (release
// fence) and arrives on the counter of its group (blockIdx % kBarGroups); the
// last block of a group arrives on the top counter, and the last group's
// releases the generation word, which every block polls with relaxed loads
// (one acquire fence follows; relaxed polling avoids a cache invalidation per
// poll). Splitting the arrivals over 16 counters takes 256 work-groups from
// 7.5 to 5.5 us per barrier on this chip. Counters reset themselves, so no
// memset is needed between launches. A block that polls for longer than
// kSpinLimit raises an error bit and continues, so a grid that cannot
// complete still terminates.
// Layout of the barrier words (kBarWords, 128-byte lines): group counters at
// 32 g, the top counter at 32 kBarGroups, the generation at 32 (kBarGroups+1).
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned nb, unsigned& my_gen,
                                             int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    constexpr unsigned G = kBarGroups;
    unsigned* const top = bar + 32 * G;
    unsigned* const gen = bar + 32 * (G + 1);
    const unsigned g = my_gen;
    const unsigned grp = blockIdx.x % G;
    const unsigned gsize = (nb - grp + G - 1) / G;   // blocks of this group
    const unsigned ngrp = nb < G ? nb : G;           // non-empty groups
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned old =
        __hip_atomic_fetch_add(bar + 32 * grp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool released = false;
    if (old == gsize - 1) {
      __hip_atomic_store(bar + 32 * grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned t = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (t == ngrp - 1) {
        __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        released = true;
      }
    }
    if (!released) {
      long spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          atomicOr(err, PIC_ERRBIT_BARRIER);
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    my_gen = g + 1;
  }
  __syncthreads();
}

// deterministic block reduction of N doubles; result valid in all threads
// Every lane of the block holds the same value: tell the compiler so (scalar
// registers and branches for the solve's coefficients and decisions).
__device__ __forceinline__ double uniform(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* sm) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double x = v[k];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) sm[wave * N + k] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += sm[w * N + k];
    v[k] = uniform(s);
  }
  __syncthreads();
}

// Sum of the per-block partials (N values each, stride 8) of one run,
// computed cooperatively by the block: thread t adds partials blo+t,
// blo+t+kThreads, ... in order, then the fixed reduction tree of block_sum.
template <int N>
__device__ __forceinline__ void run_sum(const double* part, int blo, int bhi, double (&s)[N],
                                        double* sm) {
#pragma unroll
  for (int k = 0; k < N; ++k) s[k] = 0.0;
  for (int b = blo + (int)threadIdx.x; b < bhi; b += kThreads)
#pragma unroll
    for (int k = 0; k < N; ++k) s[k] += part[(size_t)b * 8 + k];
  block_sum<N>(s, sm);
}

template <int N>
__device__ __forceinline__ void put_part(double* part, const double (&v)[N]) {
  if (threadIdx.x == 0)
    for (int k = 0; k < N; ++k) part[(size_t)blockIdx.x * 8 + k] = v[k];
}

// curl with forward differences at the B points (Eq. (5)), F co-located with E
__device__ __forceinline__ void curl_fwd(const Loc& L, double* const* F, int i, int j,
                                         double idx_, double idy_, double out[3]) {
  const double fz = F[2][lidx(L, i, j)];
  out[0] = (F[2][lidx(L, i, j + 1)] - fz) * idy_;
  out[1] = -(F[2][lidx(L, i + 1, j)] - fz) * idx_;
  out[2] = (F[1][lidx(L, i + 1, j)] - F[1][lidx(L, i, j)]) * idx_ -
           (F[0][lidx(L, i, j + 1)] - F[0][lidx(L, i, j)]) * idy_;
}

// kMode: 0 plain CG, 1 learned with the collapsed filter, 2 learned with the
// BF16 network, 3 explicit FDTD (no solve). kShock: some run of the context has shock walls (the wall
// rows are then tested per run; without it they compile away).
template <int kMode, bool kShock>
__global__ void __launch_bounds__(kThreads)
k_field_solve(FieldArgs a) {
  __shared__ double sm[kWaves * 8];
  __shared__ int s_run;
  extern __shared__ __align__(16) unsigned char net_lds[];

  if (threadIdx.x == 0) {
    int r = 0;
    while (r + 1 < a.n_runs && (int)blockIdx.x >= a.runs[r].cg_blk_hi) ++r;
    s_run = r;
  }
  __syncthreads();
  const int run = __builtin_amdgcn_readfirstlane(s_run);
  const DevRun& R = a.runs[run];
  const int blo = R.cg_blk_lo, bhi = R.cg_blk_hi;
  const int lb = blockIdx.x - blo, nb = bhi - blo;
  const bool leader = (int)blockIdx.x == blo;
  const Loc L{R.cell0, R.nx, R.ny};
  const int ncell = R.nx * R.ny;
  const double dt = R.dt, th = R.theta;
  const double idx_ = 1.0 / R.dx, idy_ = 1.0 / R.dy;
  const double idx2 = idx_ * idx_, idy2 = idy_ * idy_;
  const double ax = (th * dt) * (th * dt) * idx2, ay = (th * dt) * (th * dt) * idy2;
  const int stride = nb * kThreads;
  const int first = lb * kThreads + (int)threadIdx.x;
  const unsigned nblocks = gridDim.x;
  // the generation word persists across launches; it cannot move before every
  // block has arrived at the first barrier, so all blocks read the same value
  unsigned my_gen =
      __hip_atomic_load(a.bar + 32 * (kBarGroups + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  auto barrier = [&]() { grid_barrier(a.bar, nblocks, my_gen, a.err); };
  // per-block partial sums, three sets of [block][8]
  double* const part0 = a.part;
  double* const part1 = a.part + (size_t)a.n_blocks * 8;
  double* const part2 = a.part + (size_t)a.n_blocks * 16;
  // Shock runs (conducting walls at x = 0 and x = (nx-1) dx): fixed rows
  // (Bx on both wall lines, the outside column of By and Bz) are identity rows
  // holding zero, so a fixed neighbour of Bx reads zero; behind a wall the
  // tangential By, Bz take the row's own value.
  const bool shock = kShock && R.bc == 1;
  auto fixed_row = [&](int c, int i) {
    return shock && (c == 0 ? (i == 0 || i == R.nx - 1) : i == R.nx - 1);
  };
  // A v of component c at (i, j) for a vector given by a functor of the index
  auto applyA = [&](auto&& v, int c, int i, long long g, long long gxp, long long gxm,
                    long long gyp, long long gym) {
    if (shock) {
      if (fixed_row(c, i)) return v(g);
      if (c > 0) {
        if (i == 0) gxm = g;
        if (i == R.nx - 2) gxp = g;
      }
    }
    const double cc = v(g);
    return cc - ax * (v(gxp) - 2.0 * cc + v(gxm)) - ay * (v(gyp) - 2.0 * cc + v(gym));
  };
  // right-hand side of Eq. (7) for component c at (i, j)
  auto rhs_b = [&](int c, int i, int j, const double (&cj)[3], const double (&ce)[3]) {
    if (fixed_row(c, i)) return 0.0;
    const double* f = a.B[c];
    const long long g = lidx(L, i, j);
    long long gxp = lidx(L, i + 1, j), gxm = lidx(L, i - 1, j);
    if (shock && c > 0) {
      if (i == 0) gxm = g;
      if (i == R.nx - 2) gxp = g;
    }
    const double v = f[g];
    const double lb = (f[gxp] - 2.0 * v + f[gxm]) * idx2 +
                      (f[lidx(L, i, j + 1)] - 2.0 * v + f[lidx(L, i, j - 1)]) * idy2;
    return th * dt * dt * (lb + kFourPi * cj[c]) - dt * ce[c];
  };
  // Global "does any run still iterate" decisions: round k adds into
  // g_active[k % 3] before a barrier and reads it after; block 0 clears the
  // next round's slot (its previous readers finished two barriers earlier).
  int round = 0;
  auto count_active = [&](bool any) {
    if (leader && threadIdx.x == 0) atomicAdd(&a.g_active[round % 3], any ? 1 : 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.g_active[(round + 1) % 3] = 0;
  };
  auto read_active = [&]() {
    const int t = __hip_atomic_load(&a.g_active[round % 3], __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    ++round;
    return __builtin_amdgcn_readfirstlane(t);
  };
  // z = N(v) over every tile of every active component, items spread over the
  // run's blocks: rd(c, i, j) gives the input at any cell, wr(c, i, j, z) sees
  // each output of the run's own cells
  // this run's network (runs that share an operator share it)
  const NetWeights net = (kMode == 1 || kMode == 2) ? a.nets[R.net_id] : NetWeights{};
  constexpr bool collapsed = kMode == 1;
  constexpr int TE = collapsed ? NET_KT : NET_T;
  const int ntx = (R.nx + TE - 1) / TE, nty = (R.ny + TE - 1) / TE;
  auto net_sweep = [&](const bool (&act)[3], auto&& rd, auto&& wr) {
    if constexpr (collapsed) {
      // one item = one tile, all three components
      for (int t = lb; t < ntx * nty; t += nb)
        net_apply_tile_collapsed<3>(net, (t % ntx) * TE, (t / ntx) * TE, R.nx, R.ny, act, rd,
                                    wr, net_lds);
    } else {
      for (int item = lb; item < ntx * nty * 3; item += nb) {
        const int c = item % 3, t = item / 3;
        if (!act[c]) continue;
        auto rd_c = [&](int i, int j) { return rd(c, i, j); };
        auto wr_c = [&](int i, int j, double v) { wr(c, i, j, v); };
        net_apply_tile(net, (t % ntx) * TE, (t / ntx) * TE, R.nx, R.ny, rd_c, wr_c, net_lds);
      }
    }
  };

  // per-run record (leader block, thread 0): solve statistics and the
  // energies of step n; tr = squared true residual norms
  auto write_record = [&](const double (&tr)[3], const int (&its)[3], const double (&b2)[3],
                          const double (&g2)[3], const int (&lits)[3], int fb, double we,
                          double wb) {
    double* st = a.stats + (size_t)run * PIC_STAT_WORDS;
    for (int c = 0; c < 3; ++c) {
      st[c] = (double)its[c];
      st[3 + c] = b2[c] > 0.0 ? sqrt(tr[c] / b2[c]) : 0.0;
      st[6 + c] = sqrt(b2[c]);
      st[9 + c] = (double)lits[c];
      st[16 + c] = b2[c] > 0.0 ? sqrt(g2[c] / b2[c]) : 0.0;
    }
    st[12] = (double)fb;
    st[13] += (double)fb;   // cumulative counters since initialisation
    st[14] += 1.0;
    if (a.diag) {
      double wk[PIC_MAXS][2] = {{0.0, 0.0}, {0.0, 0.0}};
      const int nt = R.ntx * R.nty;
      for (int t = R.tile0 * a.K; t < (R.tile0 + nt) * a.K; ++t)
        for (int s = 0; s < R.nspecies; ++s) {
          wk[s][0] += a.wk_part[((size_t)t * PIC_MAXS + s) * 2 + 0];
          wk[s][1] += a.wk_part[((size_t)t * PIC_MAXS + s) * 2 + 1];
        }
      const double cellv = R.dx * R.dy / (2.0 * kFourPi);
      double* rec = a.history + ((size_t)run * a.hist_cap + a.hist_slot) * PIC_REC_WORDS;
      rec[0] = (double)a.step;
      rec[1] = (double)a.step * dt;
      rec[2] = we * cellv;
      rec[3] = wb * cellv;
      rec[4] = wk[0][0] + wk[1][0];
      rec[5] = wk[0][1] + wk[1][1];
      for (int c = 0; c < 3; ++c) {
        rec[6 + c] = (double)its[c];
        rec[9 + c] = st[3 + c];
      }
    }
  };
  // FP32 copies of E and B for the fast particle path
  auto write_shadow = [&](long long g) {
    if (a.Ef[0]) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a.Ef[c][g] = (float)a.E[c][g];
        a.Ef[3 + c][g] = (float)a.B[c][g];
      }
    }
  };

  if constexpr (kMode == 3) {
    // ---- X1: B^{n+1/2} = B^n - (dt/2) curl E^n into x; energies of step n
    double en[2] = {0.0, 0.0};
    for (int k = first; k < ncell; k += stride) {
      const int j = k / R.nx, i = k - j * R.nx;
      double ce[3];
      curl_fwd(L, a.E, i, j, idx_, idy_, ce);
      const long long g = L.base + k;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double bb = a.B[c][g];
        a.x[c][g] = bb - 0.5 * dt * ce[c];
        if (a.diag) {
          const double e = a.E[c][g];
          en[0] += e * e;
          en[1] += bb * bb;
        }
      }
    }
    block_sum<2>(en, sm);
    put_part<2>(part0, en);
    barrier();
    // ---- X2: E^{n+1} = E^n + dt curl B^{n+1/2} - 4 pi dt J^{n+1/2}
    for (int k = first; k < ncell; k += stride) {
      const int j = k / R.nx, i = k - j * R.nx;
      const long long g = L.base + k;
      const long long gxm = lidx(L, i - 1, j), gym = lidx(L, i, j - 1);
      const double cx = (a.x[2][g] - a.x[2][gym]) * idy_;
      const double cy = -(a.x[2][g] - a.x[2][gxm]) * idx_;
      const double cz = (a.x[1][g] - a.x[1][gxm]) * idx_ - (a.x[0][g] - a.x[0][gym]) * idy_;
      a.E[0][g] += dt * cx - kFourPi * dt * a.J[0][g];
      a.E[1][g] += dt * cy - kFourPi * dt * a.J[1][g];
      a.E[2][g] += dt * cz - kFourPi * dt * a.J[2][g];
    }
    barrier();
    // ---- X3: B^{n+1} = B^{n+1/2} - (dt/2) curl E^{n+1}; FP32 copies
    for (int k = first; k < ncell; k += stride) {
      const int j = k / R.nx, i = k - j * R.nx;
      double ce[3];
      curl_fwd(L, a.E, i, j, idx_, idy_, ce);
      const long long g = L.base + k;
#pragma unroll
      for (int c = 0; c < 3; ++c) a.B[c][g] = a.x[c][g] - 0.5 * dt * ce[c];
      write_shadow(g);
    }
    if (leader) {
      double e2[2];
      run_sum<2>(part0, blo, bhi, e2, sm);
      if (threadIdx.x == 0) {
        const double z3[3] = {0.0, 0.0, 0.0};
        const int zi[3] = {0, 0, 0};
        write_record(z3, zi, z3, z3, zi, 0, e2[0], e2[1]);
      }
    }
    return;
  }

  // plain CG from the previous step's dB (kept in x) instead of zero
  const bool warm = kMode == 0 && a.cg_x0 != 0;
  // ---- P0: right-hand side of Eq. (7): b into r0, r1 and bsv (kept), x = 0
  // (or the previous dB); energies
  {
    double en[2] = {0.0, 0.0};
    for (int k = first; k < ncell; k += stride) {
      const int j = k / R.nx, i = k - j * R.nx;
      double cj[3], ce[3];
      curl_fwd(L, a.J, i, j, idx_, idy_, cj);
      curl_fwd(L, a.E, i, j, idx_, idy_, ce);
      const long long g = L.base + k;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double b = rhs_b(c, i, j, cj, ce);
        a.r0[c][g] = b;
        a.r1[c][g] = b;
        a.bsv[c][g] = b;
        if (!warm) a.x[c][g] = 0.0;
      }
      if (a.diag) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double e = a.E[c][g], bb = a.B[c][g];
          en[0] += e * e;
          en[1] += bb * bb;
        }
      }
    }
    block_sum<2>(en, sm);
    if (threadIdx.x == 0) {
      part0[(size_t)blockIdx.x * 8 + 6] = en[0];
      part0[(size_t)blockIdx.x * 8 + 7] = en[1];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.g_active[0] = 0;
  }
  barrier();
  double we_tot = 0.0, wb_tot = 0.0;
  if (leader && a.diag) {
    // energies of step n; later phases never write words 6 and 7 of part0
    double e2[2];
    run_sum<2>(part0 + 6, blo, bhi, e2, sm);
    we_tot = e2[0];
    wb_tot = e2[1];
  }

  double bn2[3] = {0, 0, 0}, gam[3] = {0, 0, 0};
  int iters[3] = {0, 0, 0}, learned_iters[3] = {0, 0, 0};
  bool need_plain[3] = {true, true, true};
  bool x_nonzero = warm;
  int fallback = 0;

  if constexpr (kMode != 0) {
    // ---- L1: x0 = N(b); ||b||^2
    {
      const bool all3[3] = {true, true, true};
      double d[3] = {0, 0, 0};
      net_sweep(all3, [&](int c, int i, int j) { return a.r1[c][L.base + (long long)j * R.nx + i]; },
                [&](int c, int i, int j, double v) {
                  const long long g = L.base + (long long)j * R.nx + i;
                  a.x[c][g] = fixed_row(c, i) ? 0.0 : v;
                  const double b = a.r1[c][g];
                  d[c] += b * b;
                });
      block_sum<3>(d, sm);
      put_part<3>(part2, d);
    }
    barrier();
    bool act[3];
    {
      double s[3];
      run_sum<3>(part2, blo, bhi, s, sm);
      for (int c = 0; c < 3; ++c) {
        bn2[c] = s[c];
        act[c] = bn2[c] > 0.0;
      }
    }
    x_nonzero = true;
    // ---- L2: r0 = b - A x0 (recomputed at the halo), z0 = N(r0); p_old = 0;
    // <r0, r0>, <z0, r0>
    auto resid0 = [&](int c, int i, int j) {
      const long long g = lidx(L, i, j);
      const double* xc = a.x[c];
      return a.r1[c][g] - applyA([&](long long q) { return xc[q]; }, c, i, g, lidx(L, i + 1, j),
                                 lidx(L, i - 1, j), lidx(L, i, j + 1), lidx(L, i, j - 1));
    };
    {
      double d[6] = {0, 0, 0, 0, 0, 0};
      net_sweep(act, resid0, [&](int c, int i, int j, double v) {
        const long long g = L.base + (long long)j * R.nx + i;
        const double r = resid0(c, i, j);
        if (fixed_row(c, i)) v = 0.0;
        a.r0[c][g] = r;
        a.w0[c][g] = v;
        a.s0[c][g] = 0.0;
        d[c] += r * r;
        d[3 + c] += v * r;
      });
      block_sum<6>(d, sm);
      put_part<6>(part1, d);
    }
    barrier();
    double rr[3] = {0, 0, 0}, rho[3] = {0, 0, 0}, beta[3] = {0, 0, 0}, alpha[3] = {0, 0, 0};
    const int budget = R.cg_maxit < a.learned_maxit ? R.cg_maxit : a.learned_maxit;
    {
      double s[6];
      run_sum<6>(part1, blo, bhi, s, sm);
      for (int c = 0; c < 3; ++c) {
        rr[c] = s[c];
        rho[c] = s[3 + c];
        act[c] = act[c] && budget > 0 && sqrt(rr[c]) > R.cg_rtol * sqrt(bn2[c]);
      }
    }
    // Flexible PCG, two grid barriers per iteration:
    //   A:  p = z + beta p_old, q = A p (p recomputed at the halo); <p, q>
    //   BC: alpha; x += alpha p; r' = r - alpha q (recomputed at the halo);
    //       z = N(r'); <r', r'>, <z, r'>, <z, q>
    for (int it = 0;; ++it) {
      bool any = act[0] || act[1] || act[2];
      count_active(any);
      double* const* rc = (it & 1) ? a.p : a.r0;    // r_k
      double* const* rn = (it & 1) ? a.r0 : a.p;    // r_{k+1}
      double* const* po = (it & 1) ? a.s1 : a.s0;   // p_{k-1}
      double* const* pn = (it & 1) ? a.s0 : a.s1;   // p_k
      {
        double d[3] = {0, 0, 0};
        if (any) {
          for (int k = first; k < ncell; k += stride) {
            const int j = k / R.nx, i = k - j * R.nx;
            const long long g = L.base + k;
            const long long gxp = lidx(L, i + 1, j), gxm = lidx(L, i - 1, j);
            const long long gyp = lidx(L, i, j + 1), gym = lidx(L, i, j - 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              if (!act[c]) continue;
              const double* z_ = a.w0[c];
              const double* p_ = po[c];
              const double be = beta[c];
              auto pv = [&](long long q) { return z_[q] + be * p_[q]; };
              const double p = pv(g);
              const double qv = applyA(pv, c, i, g, gxp, gxm, gyp, gym);
              pn[c][g] = p;
              a.w1[c][g] = qv;
              d[c] += p * qv;
            }
          }
        }
        block_sum<3>(d, sm);
        put_part<3>(part0, d);
      }
      barrier();
      if (read_active() == 0) break;
      {
        double s[3];
        run_sum<3>(part0, blo, bhi, s, sm);
        for (int c = 0; c < 3; ++c) alpha[c] = (act[c] && s[c] != 0.0) ? rho[c] / s[c] : 0.0;
        double d[6] = {0, 0, 0, 0, 0, 0}, e[3] = {0, 0, 0};
        auto rnext = [&](int c, int i, int j) {
          const long long g = L.base + (long long)j * R.nx + i;
          return rc[c][g] - alpha[c] * a.w1[c][g];
        };
        net_sweep(act, rnext, [&](int c, int i, int j, double v) {
          const long long g = L.base + (long long)j * R.nx + i;
          const double r = rnext(c, i, j);
          if (fixed_row(c, i)) v = 0.0;
          rn[c][g] = r;
          a.x[c][g] += alpha[c] * pn[c][g];
          a.w0[c][g] = v;
          d[c] += r * r;
          d[3 + c] += v * r;
          e[c] += v * a.w1[c][g];
        });
        block_sum<6>(d, sm);
        block_sum<3>(e, sm);
        put_part<6>(part1, d);
        put_part<3>(part2, e);
      }
      barrier();
      {
        double s[6], s2[3];
        run_sum<6>(part1, blo, bhi, s, sm);
        run_sum<3>(part2, blo, bhi, s2, sm);
        for (int c = 0; c < 3; ++c) {
          if (!act[c]) continue;
          rr[c] = s[c];
          learned_iters[c] = it + 1;
          beta[c] = rho[c] != 0.0 ? -alpha[c] * s2[c] / rho[c] : 0.0;
          rho[c] = s[3 + c];
          act[c] = sqrt(rr[c]) > R.cg_rtol * sqrt(bn2[c]) && it + 1 < budget;
        }
      }
    }
    for (int c = 0; c < 3; ++c) {
      gam[c] = rr[c];
      iters[c] = learned_iters[c];
      need_plain[c] = bn2[c] > 0.0 && sqrt(rr[c]) > R.cg_rtol * sqrt(bn2[c]);
      fallback |= need_plain[c] ? 1 : 0;
    }
  }

  // every block must agree whether the plain solver runs (it has barriers)
  bool run_plain = true;
  if constexpr (kMode != 0) {
    count_active(need_plain[0] || need_plain[1] || need_plain[2]);
    barrier();
    run_plain = read_active() > 0;
  }
  if (run_plain) {
    if (x_nonzero) {
      // restart from the current iterate: r0 = b - A x
      for (int k = first; k < ncell; k += stride) {
        const int j = k / R.nx, i = k - j * R.nx;
        const long long g = L.base + k;
        const long long gxp = lidx(L, i + 1, j), gxm = lidx(L, i - 1, j);
        const long long gyp = lidx(L, i, j + 1), gym = lidx(L, i, j - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (!need_plain[c]) continue;
          const double* xc = a.x[c];
          a.r0[c][g] = a.r1[c][g] - applyA([&](long long q) { return xc[q]; }, c, i, g, gxp, gxm,
                                           gyp, gym);
        }
      }
      barrier();
    }
    // ---- P1: w0 = A r0; gamma0 = <r0,r0>, delta0 = <w0,r0>, <b,b>; s_{-1} = p_{-1} = 0
    {
      double d[6] = {0, 0, 0, 0, 0, 0};
      double bb[3] = {0, 0, 0};
      for (int k = first; k < ncell; k += stride) {
        const int j = k / R.nx, i = k - j * R.nx;
        const long long g = L.base + k;
        const long long gxp = lidx(L, i + 1, j), gxm = lidx(L, i - 1, j);
        const long long gyp = lidx(L, i, j + 1), gym = lidx(L, i, j - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (!need_plain[c]) continue;
          const double* rc = a.r0[c];
          const double w = applyA([&](long long q) { return rc[q]; }, c, i, g, gxp, gxm, gyp, gym);
          const double r = rc[g];
          const double b = a.r1[c][g];
          a.w0[c][g] = w;
          a.s0[c][g] = 0.0;
          a.p[c][g] = 0.0;
          d[c] += r * r;
          d[3 + c] += w * r;
          bb[c] += b * b;
        }
      }
      block_sum<6>(d, sm);
      block_sum<3>(bb, sm);
      put_part<6>(part1, d);
      put_part<3>(part2, bb);
    }
    barrier();
    double alpha[3], beta[3];
    bool act[3];
    {
      double s[6], sb[3];
      run_sum<6>(part1, blo, bhi, s, sm);
      run_sum<3>(part2, blo, bhi, sb, sm);
      for (int c = 0; c < 3; ++c) {
        alpha[c] = beta[c] = 0.0;
        act[c] = false;
        if (!need_plain[c]) continue;
        bn2[c] = sb[c];
        gam[c] = s[c];
        alpha[c] = s[3 + c] > 0.0 ? s[c] / s[3 + c] : 0.0;
        act[c] = R.cg_maxit > iters[c] && bn2[c] > 0.0;
      }
    }
    const int done0[3] = {iters[0], iters[1], iters[2]};
    for (int it = 0;; ++it) {
      // all blocks of all runs take the same number of passes; a run whose
      // components have all converged sweeps nothing
      bool any = false;
      for (int c = 0; c < 3; ++c) {
        act[c] = act[c] && done0[c] + it < R.cg_maxit && sqrt(gam[c]) > R.cg_rtol * sqrt(bn2[c]);
        if (act[c]) iters[c] = done0[c] + it + 1;
        any |= act[c];
      }
      count_active(any);
      double* const* rc = (it & 1) ? a.r1 : a.r0;
      double* const* rn = (it & 1) ? a.r0 : a.r1;
      double* const* wc = (it & 1) ? a.w1 : a.w0;
      double* const* wn = (it & 1) ? a.w0 : a.w1;
      double* const* sc = (it & 1) ? a.s1 : a.s0;   // s_{k-1}
      double* const* sn = (it & 1) ? a.s0 : a.s1;   // s_k
      double d[6] = {0, 0, 0, 0, 0, 0};
      if (any) {
        for (int k = first; k < ncell; k += stride) {
          const int j = k / R.nx, i = k - j * R.nx;
          const long long g = L.base + k;
          const long long gxp = lidx(L, i + 1, j), gxm = lidx(L, i - 1, j);
          const long long gyp = lidx(L, i, j + 1), gym = lidx(L, i, j - 1);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const double* r_ = rc[c];
            const double* w_ = wc[c];
            const double* s_ = sc[c];
            const double al = alpha[c], be = beta[c];
            // r_{k+1} at any point from the previous buffers
            auto rnext = [&](long long q) { return r_[q] - al * (w_[q] + be * s_[q]); };
            const double sk = w_[g] + be * s_[g];
            const double pk = r_[g] + be * a.p[c][g];
            const double r1 = r_[g] - al * sk;
            const double w1 = applyA(rnext, c, i, g, gxp, gxm, gyp, gym);
            a.p[c][g] = pk;
            sn[c][g] = sk;
            a.x[c][g] += al * pk;
            rn[c][g] = r1;
            wn[c][g] = w1;
            d[c] += r1 * r1;
            d[3 + c] += w1 * r1;
          }
        }
      }
      double* const pw = (it & 1) ? part1 : part0;
      block_sum<6>(d, sm);
      put_part<6>(pw, d);
      barrier();
      if (read_active() == 0) break;
      double s[6];
      run_sum<6>(pw, blo, bhi, s, sm);
      for (int c = 0; c < 3; ++c) {
        if (!act[c]) continue;
        const double gnew = s[c], dnew = s[3 + c];
        const double bnew = gnew / gam[c];
        const double den = dnew - bnew * gnew / alpha[c];
        beta[c] = bnew;
        alpha[c] = den != 0.0 ? gnew / den : 0.0;
        gam[c] = gnew;
      }
    }
  }

  // ---- E update, Eq. (6): E += dt curl_B(B^n + theta dB) - 4 pi dt J; in the
  // same sweep the training pairs (b, dB) of each network's first run (b kept
  // from P0). dB is complete (the solve ended on a barrier) and this sweep
  // writes only E at its own cells.
  const bool rec_pairs = a.collect && R.pairs;
  double* const pb = rec_pairs ? R.pairs + (size_t)a.pair_slot * 6 * ncell : nullptr;
  for (int k = first; k < ncell; k += stride) {
    const int j = k / R.nx, i = k - j * R.nx;
    const long long g = L.base + k;
    const long long gxm = lidx(L, i - 1, j), gym = lidx(L, i, j - 1);
    if (rec_pairs) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pb[(size_t)(2 * c) * ncell + k] = a.bsv[c][g];
        pb[(size_t)(2 * c + 1) * ncell + k] = a.x[c][g];
      }
    }
    const double bz = a.B[2][g] + th * a.x[2][g];
    const double bz_ym = a.B[2][gym] + th * a.x[2][gym];
    const double bz_xm = a.B[2][gxm] + th * a.x[2][gxm];
    const double by = a.B[1][g] + th * a.x[1][g];
    const double by_xm = a.B[1][gxm] + th * a.x[1][gxm];
    const double bx = a.B[0][g] + th * a.x[0][g];
    const double bx_ym = a.B[0][gym] + th * a.x[0][gym];
    const double cx = (bz - bz_ym) * idy_;
    const double cy = -(bz - bz_xm) * idx_;
    const double cz = (by - by_xm) * idx_ - (bx - bx_ym) * idy_;
    a.E[0][g] += dt * cx - kFourPi * dt * a.J[0][g];
    a.E[1][g] += dt * cy - kFourPi * dt * a.J[1][g];
    a.E[2][g] += dt * cz - kFourPi * dt * a.J[2][g];
    if (shock) {
      // E nodes on the conductors (Ey, Ez on both wall lines, the outside
      // column's Ex) stay zero
      if (i == 0 || i == R.nx - 1) a.E[1][g] = a.E[2][g] = 0.0;
      if (i == R.nx - 1) a.E[0][g] = 0.0;
    }
  }
  barrier();

  // ---- per-run record: solve statistics and energies of step n (the true
  // residual words are written by k_true_residual_final after this kernel)
  if (leader && threadIdx.x == 0)
    write_record(gam, iters, bn2, gam, learned_iters, fallback, we_tot, wb_tot);

  // ---- B update, Eq. (5) through dB; FP32 copies for the fast particle path
  for (int k = first; k < ncell; k += stride) {
    const long long g = L.base + k;
#pragma unroll
    for (int c = 0; c < 3; ++c) a.B[c][g] += a.x[c][g];
    write_shadow(g);
  }
}

}  // namespace

namespace {

// The operator of Eq. (7), (1 - (theta dt)^2 L) v, for component c at cell
// (i, j) of run R, with the shock runs' wall rows (the solve's operator).
__device__ double op_at(const DevRun& R, const double* v, int c, int i, int j) {
  const Loc L{R.cell0, R.nx, R.ny};
  const long long g = lidx(L, i, j);
  long long gxp = lidx(L, i + 1, j), gxm = lidx(L, i - 1, j);
  if (R.bc == 1) {
    const bool fixed = c == 0 ? (i == 0 || i == R.nx - 1) : i == R.nx - 1;
    if (fixed) return v[g];
    if (c > 0) {
      if (i == 0) gxm = g;
      if (i == R.nx - 2) gxp = g;
    }
  }
  const double a2 = (R.theta * R.dt) * (R.theta * R.dt);
  const double ax = a2 / (R.dx * R.dx), ay = a2 / (R.dy * R.dy);
  const double cc = v[g];
  return cc - ax * (v[gxp] - 2.0 * cc + v[gxm]) -
         ay * (v[lidx(L, i, j + 1)] - 2.0 * cc + v[lidx(L, i, j - 1)]);
}

constexpr int kResThreads = 256;
// work-groups per run of the residual sweep: partials of all runs must fit the
// solve's partial-sum buffer (PIC_RES_PART_DOUBLES doubles, 4 per work-group)
inline int res_blocks(int n_runs) {
  const int b = PIC_RES_PART_DOUBLES / (4 * n_runs);
  return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

// True residual ||b - A dB||^2 of the applied dB per component, after the
// solve: per (work-group, run) partial sums in a fixed reduction tree.
__global__ void __launch_bounds__(kResThreads) k_true_residual(FieldArgs a) {
  const int run = blockIdx.y;
  const DevRun& R = a.runs[run];
  const int ncell = R.nx * R.ny;
  double d[3] = {0.0, 0.0, 0.0};
  for (int k = blockIdx.x * kResThreads + threadIdx.x; k < ncell;
       k += (int)gridDim.x * kResThreads) {
    const int j = k / R.nx, i = k - j * R.nx;
    const long long g = R.cell0 + k;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double r = a.bsv[c][g] - op_at(R, a.x[c], c, i, j);
      d[c] += r * r;
    }
  }
  __shared__ double sm[3][kResThreads];
  for (int c = 0; c < 3; ++c) sm[c][threadIdx.x] = d[c];
  __syncthreads();
  for (int off = kResThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int c = 0; c < 3; ++c) sm[c][threadIdx.x] += sm[c][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 3)
    a.part[((size_t)run * gridDim.x + blockIdx.x) * 4 + threadIdx.x] = sm[threadIdx.x][0];
}

// sum of the partials (each thread a strided subset in block order, then a
// fixed tree over the threads); relres = ||b - A dB|| / ||b|| into the solve
// statistics and the step's history record
__global__ void __launch_bounds__(kResThreads) k_true_residual_final(FieldArgs a, int nblk) {
  const int run = blockIdx.x;
  const double* part = a.part + (size_t)run * nblk * 4;
  double d[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += kResThreads)
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] += part[(size_t)b * 4 + c];
  __shared__ double sm[3][kResThreads];
  for (int c = 0; c < 3; ++c) sm[c][threadIdx.x] = d[c];
  __syncthreads();
  for (int off = kResThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int c = 0; c < 3; ++c) sm[c][threadIdx.x] += sm[c][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x >= 3) return;
  const int c = threadIdx.x;
  double* st = a.stats + (size_t)run * PIC_STAT_WORDS;
  const double bn = st[6 + c];
  const double rel = bn > 0.0 ? sqrt(sm[c][0]) / bn : 0.0;
  st[3 + c] = rel;
  if (a.diag) a.history[((size_t)run * a.hist_cap + a.hist_slot) * PIC_REC_WORDS + 9 + c] = rel;
}

}  // namespace

// ---- allocation-free field solve: its scratch (the CG vectors, per-block
// partial sums, active-run counters and grid-barrier words) lives in this
// file-scope device array instead of the context's workspace. One copy per
// GPU, held until the process ends; calls that overlap on one GPU race on it.
namespace {
constexpr long long kScratchCells = PIC_NOALLOC_MAX_CELLS;
constexpr int kScratchVecs = 27;   // x, p, r0, r1, w0, w1, s0, s1, bsv; 3 components each
constexpr size_t kScratchPart = (size_t)PIC_NOALLOC_MAX_BLOCKS * 24;   // doubles
constexpr size_t kScratchBytes = (size_t)kScratchVecs * kScratchCells * sizeof(double) +
                                 kScratchPart * sizeof(double) + 256 + kBarWords * 4;
constexpr int kScratchDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
void* g_scratch[kScratchDevices] = {};
}

hipError_t pic_noalloc_scratch_init(int dev) {
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  if (__atomic_load_n(&g_scratch[dev], __ATOMIC_ACQUIRE)) return hipSuccess;
  void* ptr = nullptr;
  // the array's name is a host-side stand-in: its device address (this GPU's
  // copy) comes from the runtime, with the device current
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  __atomic_store_n(&g_scratch[dev], ptr, __ATOMIC_RELEASE);
  return hipSuccess;
}

int pic_field_args_noalloc(FieldArgs& a, int dev, long long n_cells) {
  if (dev < 0 || dev >= kScratchDevices) return -1;
  unsigned char* base = (unsigned char*)__atomic_load_n(&g_scratch[dev], __ATOMIC_ACQUIRE);
  if (!base) return -1;
  if (n_cells > kScratchCells || a.n_blocks > PIC_NOALLOC_MAX_BLOCKS) return -2;
  double* v = reinterpret_cast<double*>(base);
  double** vecs[9] = {a.x, a.p, a.r0, a.r1, a.w0, a.w1, a.s0, a.s1, a.bsv};
  for (int q = 0; q < 9; ++q)
    for (int c = 0; c < 3; ++c) vecs[q][c] = v + (size_t)(3 * q + c) * kScratchCells;
  a.part = v + (size_t)kScratchVecs * kScratchCells;
  unsigned char* tail = reinterpret_cast<unsigned char*>(a.part + kScratchPart);
  a.g_active = reinterpret_cast<int*>(tail);
  a.bar = reinterpret_cast<unsigned*>(tail + 256);
  a.cg_x0 = 0;   // the previous dB is not kept: every call starts from x0 = 0
  return 0;
}

size_t pic_field_solve_smem(int learned, int form) {
  return learned ? (form == 0 ? NET_K_LDS_BYTES : NET_LDS_BYTES) : 0;
}

namespace {
const void* solve_kernel(int learned, int form, int shock, int explicit_fdtd) {
  if (explicit_fdtd) return (const void*)k_field_solve<3, false>;
  if (shock) {
    if (!learned) return (const void*)k_field_solve<0, true>;
    return form == 0 ? (const void*)k_field_solve<1, true> : (const void*)k_field_solve<2, true>;
  }
  if (!learned) return (const void*)k_field_solve<0, false>;
  return form == 0 ? (const void*)k_field_solve<1, false> : (const void*)k_field_solve<2, false>;
}
}  // namespace

int pic_field_solve_max_blocks(int n_cu, int learned, int form) {
  int nb = 0;
  for (int variant = 0; variant < 3; ++variant) {
    // periodic, shock walls, explicit FDTD
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &v, solve_kernel(learned, form, variant == 1, variant == 2), kThreads,
            pic_field_solve_smem(learned, form)) != hipSuccess)
      return -1;
    nb = variant == 0 ? v : (v < nb ? v : nb);
  }
  return nb * n_cu;
}

hipError_t pic_launch_field_solve(const FieldArgs& a, hipStream_t s) {
  FieldArgs copy = a;
  void* args[] = {(void*)&copy};
  const void* k = solve_kernel(a.learned, a.learned_form, a.any_shock, a.explicit_fdtd);
  const size_t smem = pic_field_solve_smem(a.learned, a.learned_form);
  hipError_t e;
  if (a.coop)
    e = hipLaunchCooperativeKernel(k, dim3(a.n_blocks), dim3(kThreads), args, smem, s);
  else
    // ordinary launch (inside a captured graph): the grid is no larger than
    // the co-resident maximum and the kernel runs alone in its stream, so all
    // work-groups are resident; a grid that is not still ends through the
    // barrier's bounded spin with an error bit
    e = hipLaunchKernel(k, dim3(a.n_blocks), dim3(kThreads), args, smem, s);
  if (e != hipSuccess || a.explicit_fdtd) return e;
  // the true residual of the applied dB: a separate sweep of two small
  // kernels (inside the persistent solve the same stencil sweep costs about
  // 0.2 ms at 1024 x 256, measured)
  const int nblk = res_blocks(a.n_runs);
  k_true_residual<<<dim3(nblk, a.n_runs), kResThreads, 0, s>>>(copy);
  k_true_residual_final<<<a.n_runs, kResThreads, 0, s>>>(copy, nblk);
  return hipGetLastError();
}
