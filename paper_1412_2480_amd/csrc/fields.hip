// Implicit field solve of Ikeya & Matsumoto (PASJ 2015), Sec. 2:
//   Eq. (7):  [1 - (theta c dt)^2 L] dB = theta (c dt)^2 (L B^n + (4 pi/c) curl J^{n+1/2})
//                                       - c dt curl E^n
//   solved by conjugate gradients (the paper cites Hoshino 2013 for CG), then
//   Eqs. (5)-(6): E^{n+1} = E^n + c dt curl(B^n + theta dB) - 4 pi dt J,
//                 B^{n+1} = B^n + dB.
//
// One persistent, cooperatively launched kernel per step does all of it for
// every run of the context: each run owns a contiguous range of work-groups,
// the three B components are solved together (three independent CG
// recurrences sharing one stencil sweep), and grid-wide barriers separate the
// phases. All arithmetic is FP64; block reductions are deterministic and are
// summed across a run's blocks in a fixed order, so every block of a run holds
// bit-identical CG scalars.
//
// Phases: P0 right-hand side (+ field-energy partials) | per iteration
// {A: p = r + beta p_old, q = A p, <p,q>} | {B: x += alpha p, r -= alpha q,
// <r,r>} | E update | B update and FP32 field copy ("|" = grid barrier).
#include <hip/hip_cooperative_groups.h>
#include <math.h>

#include "pic_dev.h"
#include "pic_launch.h"

namespace cg = cooperative_groups;

namespace {

constexpr int kThreads = 256;
constexpr double kFourPi = 12.566370614359172953850573533118;

struct Loc {
  long long base;   // cell0 of the run
  int nx, ny;
};

__device__ __forceinline__ long long lidx(const Loc& L, int i, int j) {
  return L.base + (long long)pic_wrap(j, L.ny) * L.nx + pic_wrap(i, L.nx);
}

// deterministic block reduction of N doubles; result valid in all threads
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
    for (int w = 0; w < kThreads / 64; ++w) s += sm[w * N + k];
    v[k] = s;
  }
  __syncthreads();
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

__device__ __forceinline__ double lap5(const Loc& L, const double* f, int i, int j,
                                       double idx2, double idy2) {
  const double c = f[lidx(L, i, j)];
  return (f[lidx(L, i + 1, j)] - 2.0 * c + f[lidx(L, i - 1, j)]) * idx2 +
         (f[lidx(L, i, j + 1)] - 2.0 * c + f[lidx(L, i, j - 1)]) * idy2;
}

// Sum of the per-block partials of one run, computed cooperatively by the
// block: thread t adds partials blo+t, blo+t+256, ... in order, then a fixed
// reduction tree combines the threads. Every block of the run obtains the
// same bits.
__device__ __forceinline__ void run_sum3(const double* part, int blo, int bhi, double s[3],
                                         double* sm) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int b = blo + (int)threadIdx.x; b < bhi; b += kThreads) {
    v[0] += part[(size_t)b * 4 + 0];
    v[1] += part[(size_t)b * 4 + 1];
    v[2] += part[(size_t)b * 4 + 2];
  }
  block_sum<3>(v, sm);
  s[0] = v[0];
  s[1] = v[1];
  s[2] = v[2];
}

__global__ void __launch_bounds__(kThreads)
k_field_solve(FieldArgs a) {
  cg::grid_group grid = cg::this_grid();
  __shared__ double sm[(kThreads / 64) * 4];
  __shared__ int s_run;

  if (threadIdx.x == 0) {
    int r = 0;
    while (r + 1 < a.n_runs && (int)blockIdx.x >= a.runs[r].cg_blk_hi) ++r;
    s_run = r;
  }
  __syncthreads();
  const int run = s_run;
  const DevRun& R = a.runs[run];
  const int blo = R.cg_blk_lo, bhi = R.cg_blk_hi;
  const bool mine = (int)blockIdx.x >= blo && (int)blockIdx.x < bhi;
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
  double* const part_pq = a.part;
  double* const part_rr = a.part + (size_t)a.n_blocks * 4;
  double* const part_en = a.part + (size_t)a.n_blocks * 8;

  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.g_active[0] = 0;
    a.g_active[1] = 0;
  }

  // ---- P0: right-hand side of Eq. (7); x = 0, r = p = b; <b,b>; energies
  {
    double acc[3] = {0.0, 0.0, 0.0};
    double en[2] = {0.0, 0.0};
    if (mine) {
      for (int k = first; k < ncell; k += stride) {
        const int j = k / R.nx, i = k - j * R.nx;
        double cj[3], ce[3];
        curl_fwd(L, a.J, i, j, idx_, idy_, cj);
        curl_fwd(L, a.E, i, j, idx_, idy_, ce);
        const long long g = L.base + k;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double lb_ = lap5(L, a.B[c], i, j, idx2, idy2);
          const double b = th * dt * dt * (lb_ + kFourPi * cj[c]) - dt * ce[c];
          a.x[c][g] = 0.0;
          a.r[c][g] = b;
          a.p0[c][g] = b;   // p_old of iteration 0 (beta = 0 there)
          acc[c] += b * b;
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
    }
    block_sum<3>(acc, sm);
    block_sum<2>(en, sm);
    if (threadIdx.x == 0) {
      double* pp = part_rr + (size_t)blockIdx.x * 4;
      pp[0] = acc[0]; pp[1] = acc[1]; pp[2] = acc[2];
      part_en[(size_t)blockIdx.x * 2 + 0] = en[0];
      part_en[(size_t)blockIdx.x * 2 + 1] = en[1];
    }
  }
  grid.sync();

  double bn2[3], rr[3], rr_old[3] = {1.0, 1.0, 1.0};
  bool act[3] = {true, true, true};
  int iters[3] = {0, 0, 0};
  int it = 0;
  for (;; ++it) {
    // ---- phase A: residual norms, convergence, p and q = A p, <p,q>
    {
      double s[3];
      run_sum3(part_rr, blo, bhi, s, sm);
      for (int c = 0; c < 3; ++c) {
        if (it == 0) bn2[c] = s[c];
        if (act[c]) rr[c] = s[c];   // inactive components keep their last norm
      }
    }
    int nact = 0;
    for (int c = 0; c < 3; ++c) {
      act[c] = it < R.cg_maxit && bn2[c] > 0.0 && sqrt(rr[c]) > R.cg_rtol * sqrt(bn2[c]);
      nact += act[c];
      if (act[c]) iters[c] = it + 1;
    }
    if (leader && threadIdx.x == 0) atomicAdd(&a.g_active[it & 1], nact);
    double* const* pold = (it & 1) ? a.p1 : a.p0;
    double* const* pnew = (it & 1) ? a.p0 : a.p1;
    double beta[3];
    for (int c = 0; c < 3; ++c) beta[c] = (it == 0 || !act[c]) ? 0.0 : rr[c] / rr_old[c];
    double pq[3] = {0.0, 0.0, 0.0};
    if (mine && nact > 0) {
      for (int k = first; k < ncell; k += stride) {
        const int j = k / R.nx, i = k - j * R.nx;
        const long long g = L.base + k;
        const long long gxp = lidx(L, i + 1, j), gxm = lidx(L, i - 1, j);
        const long long gyp = lidx(L, i, j + 1), gym = lidx(L, i, j - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (!act[c]) continue;
          const double* rc = a.r[c];
          const double* po = pold[c];
          const double bc = beta[c];
          const double p = rc[g] + bc * po[g];
          const double pxp = rc[gxp] + bc * po[gxp], pxm = rc[gxm] + bc * po[gxm];
          const double pyp = rc[gyp] + bc * po[gyp], pym = rc[gym] + bc * po[gym];
          const double q = p - ax * (pxp - 2.0 * p + pxm) - ay * (pyp - 2.0 * p + pym);
          pnew[c][g] = p;
          a.q[c][g] = q;
          pq[c] += p * q;
        }
      }
    }
    block_sum<3>(pq, sm);
    if (threadIdx.x == 0) {
      double* pp = part_pq + (size_t)blockIdx.x * 4;
      pp[0] = pq[0]; pp[1] = pq[1]; pp[2] = pq[2];
    }
    for (int c = 0; c < 3; ++c) rr_old[c] = rr[c];
    grid.sync();

    // ---- phase B: step length, x and r updates, <r,r>
    const int total = __hip_atomic_load(&a.g_active[it & 1], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    if (total == 0) break;
    if (leader && threadIdx.x == 0) a.g_active[(it + 1) & 1] = 0;
    double alpha[3];
    {
      double s[3];
      run_sum3(part_pq, blo, bhi, s, sm);
      for (int c = 0; c < 3; ++c) alpha[c] = act[c] ? rr[c] / s[c] : 0.0;
    }
    double rn[3] = {0.0, 0.0, 0.0};
    if (mine && nact > 0) {
      for (int k = first; k < ncell; k += stride) {
        const long long g = L.base + k;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (!act[c]) continue;
          const double p = pnew[c][g];
          a.x[c][g] += alpha[c] * p;
          const double r = a.r[c][g] - alpha[c] * a.q[c][g];
          a.r[c][g] = r;
          rn[c] += r * r;
        }
      }
    }
    block_sum<3>(rn, sm);
    if (threadIdx.x == 0) {
      double* pp = part_rr + (size_t)blockIdx.x * 4;
      pp[0] = rn[0]; pp[1] = rn[1]; pp[2] = rn[2];
    }
    grid.sync();
  }

  // ---- per-run record: CG statistics and energies of step n
  if (leader && threadIdx.x == 0) {
    double* st = a.stats + (size_t)run * 9;
    for (int c = 0; c < 3; ++c) {
      st[c] = (double)iters[c];
      st[3 + c] = bn2[c] > 0.0 ? sqrt(rr[c] / bn2[c]) : 0.0;
      st[6 + c] = sqrt(bn2[c]);
    }
    if (a.diag) {
      double we = 0.0, wb = 0.0;
      for (int b = blo; b < bhi; ++b) {   // one thread, once per step
        we += part_en[(size_t)b * 2 + 0];
        wb += part_en[(size_t)b * 2 + 1];
      }
      double wk[PIC_MAXS][2] = {{0.0, 0.0}, {0.0, 0.0}};
      const int nt = R.ntx * R.nty;
      for (int t = R.tile0; t < R.tile0 + nt; ++t)
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
        rec[6 + c] = (double)iters[c];
        rec[9 + c] = st[3 + c];
      }
    }
  }

  // ---- E update, Eq. (6): E += dt curl_B(B^n + theta dB) - 4 pi dt J
  if (mine) {
    for (int k = first; k < ncell; k += stride) {
      const int j = k / R.nx, i = k - j * R.nx;
      const long long g = L.base + k;
      const long long gxm = lidx(L, i - 1, j), gym = lidx(L, i, j - 1);
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
    }
  }
  grid.sync();
  // ---- B update, Eq. (5) through dB; FP32 copies for the fast particle path
  if (mine) {
    for (int k = first; k < ncell; k += stride) {
      const long long g = L.base + k;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double bnew = a.B[c][g] + a.x[c][g];
        a.B[c][g] = bnew;
        if (a.Ef[0]) {
          a.Ef[3 + c][g] = (float)bnew;
          a.Ef[c][g] = (float)a.E[c][g];
        }
      }
    }
  }
}

}  // namespace

int pic_field_solve_max_blocks(int n_cu) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_field_solve, kThreads, 0) != hipSuccess)
    return -1;
  return nb * n_cu;
}

hipError_t pic_launch_field_solve(const FieldArgs& a, hipStream_t s) {
  FieldArgs copy = a;
  void* args[] = {(void*)&copy};
  return hipLaunchCooperativeKernel((const void*)k_field_solve, dim3(a.n_blocks),
                                    dim3(kThreads), args, 0, s);
}
