/*
 * Plain FP64 CPU oracle of the 2D3V implicit-FDTD PIC step.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference the GPU
 * library is checked against. Only tests, the smoke check and the benchmark's
 * CPU-baseline leg load it. Shares no code with the GPU library.
 *
 * Paper: Ikeya & Matsumoto, PASJ 2015 (arXiv:1412.2480). Each function cites
 * the passage it follows; the layout and units are described in oracle.h.
 * Written for clarity, not speed: loops run over fixed windows that contain
 * the shape supports, and zero weights are simply added.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Threads: particle loops and grid loops run over OpenMP threads with a
 * static schedule (independent iterations). Sums into shared arrays (the
 * deposit, the charge) go to one buffer per thread, which are then added in
 * thread order; dot products add per-thread partial sums in thread order.
 * The result is therefore a fixed function of the thread count. */
static int g_default_threads = 0;   /* OMP_NUM_THREADS or the cores, as at first use */
void ora_set_threads(int n) {
  if (g_default_threads == 0) g_default_threads = omp_get_max_threads();
  omp_set_num_threads(n > 0 ? n : g_default_threads);
}
int ora_get_threads(void) { return omp_get_max_threads(); }

/* loops shorter than this run on one thread (thread start-up would dominate) */
#define ORA_PAR_MIN 32768

/* sum of nt per-thread buffers of n values into out (out += buf[0] + ...) */
static void add_buffers(int64_t n, int nt, double* const* buf, double* out) {
#pragma omp parallel for schedule(static) if (n >= ORA_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) {
    double v = out[k];
    for (int t = 0; t < nt; ++t) v += buf[t][k];
    out[k] = v;
  }
}

static inline int wrapi(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }
static inline int64_t at(int nx, int ny, int i, int j) {
  return (int64_t)wrapi(j, ny) * nx + wrapi(i, nx);
}

/* B-spline of degree p (p = 1: linear, 2: quadratic, 3: cubic); the paper's
 * first- and second-order shape functions (Sec. 3.2-3.3) are p = 1 and 2. */
double ora_shape(int order, double d) {
  double a = fabs(d);
  switch (order) {
    case 1:
      return a < 1.0 ? 1.0 - a : 0.0;
    case 2:
      if (a < 0.5) return 0.75 - a * a;
      if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
      return 0.0;
    case 3:
      if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
      if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
      return 0.0;
    default:
      return 0.0;
  }
}

/* staggered offsets (in cells) of Ex, Ey, Ez, Bx, By, Bz on the Yee grid */
static const double STAG_X[6] = {0.5, 0.0, 0.0, 0.0, 0.5, 0.5};
static const double STAG_Y[6] = {0.0, 0.5, 0.0, 0.5, 0.0, 0.5};

/* Staggered gather (the alternative reading of the interpolation, kept for
 * comparison): field value at the particle = sum over the component's own
 * grid points of F(i+sx, j+sy) * S(X - i - sx) * S(Y - j - sy). The window i
 * in [ix-2, ix+2] contains the support of every order for both staggers. */
void ora_gather(int nx, int ny, int order, const double* const* f6,
                int64_t np, const int32_t* ix, const int32_t* iy,
                const double* fx, const double* fy, double* out6) {
#pragma omp parallel for schedule(static) if (np >= ORA_PAR_MIN)
  for (int64_t k = 0; k < np; ++k) {
    for (int c = 0; c < 6; ++c) {
      double sum = 0.0;
      for (int j = iy[k] - 2; j <= iy[k] + 2; ++j) {
        double wy = ora_shape(order, (double)(iy[k] - j) + fy[k] - STAG_Y[c]);
        for (int i = ix[k] - 2; i <= ix[k] + 2; ++i) {
          double wx = ora_shape(order, (double)(ix[k] - i) + fx[k] - STAG_X[c]);
          sum += f6[c][at(nx, ny, i, j)] * wx * wy;
        }
      }
      out6[(int64_t)c * np + k] = sum;
    }
  }
}

/* Momentum-conserving gather in the sense of Birdsall & Langdon ch. 8 (the
 * reading adopted for the paper's method, Sec. 1 and Sec. 3): the force is
 * interpolated from the charge nodes with the charge-assignment weights, so
 * every component is first averaged from its Yee points onto the node (i, j):
 *   Ex, By (half-integer x): (F(i-1, j) + F(i, j)) / 2
 *   Ey, Bx (half-integer y): (F(i, j-1) + F(i, j)) / 2
 *   Ez (node):               F(i, j)
 *   Bz (half-integer x, y):  (F(i-1, j-1) + F(i, j-1) + F(i-1, j) + F(i, j)) / 4
 * and then interpolated as sum_{i,j} N(i, j) S(X - i) S(Y - j). fetch gives the
 * Yee value at any (i, j) (periodic wrap, or the conductor images). */
typedef double (*ora_fetch)(int nx, int ny, const double* f, int c, int i, int j);

static double node_value(int nx, int ny, const double* f, int c, int i, int j, ora_fetch get) {
  switch (c) {
    case 0:
    case 4:
      return 0.5 * (get(nx, ny, f, c, i - 1, j) + get(nx, ny, f, c, i, j));
    case 1:
    case 3:
      return 0.5 * (get(nx, ny, f, c, i, j - 1) + get(nx, ny, f, c, i, j));
    case 2:
      return get(nx, ny, f, c, i, j);
    default:
      return 0.25 * (get(nx, ny, f, c, i - 1, j - 1) + get(nx, ny, f, c, i, j - 1) +
                     get(nx, ny, f, c, i - 1, j) + get(nx, ny, f, c, i, j));
  }
}

static double periodic_field(int nx, int ny, const double* f, int c, int i, int j) {
  (void)c;
  return f[at(nx, ny, i, j)];
}

static void gather_nodal(int nx, int ny, int order, const double* const* f6, int64_t np,
                         const int32_t* ix, const int32_t* iy, const double* fx,
                         const double* fy, double* out6, ora_fetch get) {
#pragma omp parallel for schedule(static) if (np >= ORA_PAR_MIN)
  for (int64_t k = 0; k < np; ++k) {
    for (int c = 0; c < 6; ++c) {
      double sum = 0.0;
      for (int j = iy[k] - 2; j <= iy[k] + 2; ++j) {
        double wy = ora_shape(order, (double)(iy[k] - j) + fy[k]);
        if (wy == 0.0) continue;
        for (int i = ix[k] - 2; i <= ix[k] + 2; ++i) {
          double wx = ora_shape(order, (double)(ix[k] - i) + fx[k]);
          if (wx == 0.0) continue;
          sum += node_value(nx, ny, f6[c], c, i, j, get) * wx * wy;
        }
      }
      out6[(int64_t)c * np + k] = sum;
    }
  }
}

void ora_gather_nodal(int nx, int ny, int order, const double* const* f6,
                      int64_t np, const int32_t* ix, const int32_t* iy,
                      const double* fx, const double* fy, double* out6) {
  gather_nodal(nx, ny, order, f6, np, ix, iy, fx, fy, out6, periodic_field);
}

/* Relativistic Boris push, c = 1:
 *   u-  = u + (q dt/2m) E
 *   t   = (q dt/(2m gamma-)) B,  gamma- = sqrt(1 + |u-|^2)
 *   s   = 2 t/(1 + |t|^2)
 *   u'  = u- + u- x t
 *   u+  = u- + u' x s
 *   u   = u+ + (q dt/2m) E                                                   */
void ora_boris(int64_t np, double qdt_2m, const double* e3, const double* b3,
               double* ux, double* uy, double* uz) {
#pragma omp parallel for schedule(static) if (np >= ORA_PAR_MIN)
  for (int64_t k = 0; k < np; ++k) {
    double ex = e3[k], ey = e3[np + k], ez = e3[2 * np + k];
    double bx = b3[k], by = b3[np + k], bz = b3[2 * np + k];
    double umx = ux[k] + qdt_2m * ex;
    double umy = uy[k] + qdt_2m * ey;
    double umz = uz[k] + qdt_2m * ez;
    double gm = sqrt(1.0 + umx * umx + umy * umy + umz * umz);
    double tx = qdt_2m * bx / gm, ty = qdt_2m * by / gm, tz = qdt_2m * bz / gm;
    double t2 = tx * tx + ty * ty + tz * tz;
    double sx = 2.0 * tx / (1.0 + t2), sy = 2.0 * ty / (1.0 + t2), sz = 2.0 * tz / (1.0 + t2);
    double upx = umx + (umy * tz - umz * ty);
    double upy = umy + (umz * tx - umx * tz);
    double upz = umz + (umx * ty - umy * tx);
    double uplx = umx + (upy * sz - upz * sy);
    double uply = umy + (upz * sx - upx * sz);
    double uplz = umz + (upx * sy - upy * sx);
    ux[k] = uplx + qdt_2m * ex;
    uy[k] = uply + qdt_2m * ey;
    uz[k] = uplz + qdt_2m * ez;
  }
}

/* advance one coordinate held as cell + offset by a displacement of less
 * than one cell; an offset that rounds to exactly 1 moves to the next cell */
static void advance(int32_t* cell, double* off, double disp) {
  double f = *off + disp;
  int32_t c = *cell;
  if (f >= 1.0) {
    f -= 1.0;
    c += 1;
  } else if (f < 0.0) {
    f += 1.0;
    c -= 1;
  }
  if (f >= 1.0) {
    f -= 1.0;
    c += 1;
  }
  *cell = c;
  *off = f;
}

void ora_move(int64_t np, double dt, double dx, double dy,
              const double* ux, const double* uy, const double* uz,
              int32_t* ix, int32_t* iy, double* fx, double* fy) {
#pragma omp parallel for schedule(static) if (np >= ORA_PAR_MIN)
  for (int64_t k = 0; k < np; ++k) {
    double g = sqrt(1.0 + ux[k] * ux[k] + uy[k] * uy[k] + uz[k] * uz[k]);
    advance(&ix[k], &fx[k], dt * ux[k] / (g * dx));
    advance(&iy[k], &fy[k], dt * uy[k] / (g * dy));
  }
}

/* Esirkepov (2001) charge-conserving deposit in 2D with a z velocity:
 * with node shapes S0 (old position) and S1 (new), DS = S1 - S0,
 *   Wx = DSx (S0y + DSy/2),  Wy = DSy (S0x + DSx/2),
 *   Wz = S0x S0y + DSx S0y/2 + S0x DSy/2 + DSx DSy/3,
 *   Jx(i+1/2, j) = -(q/(dy dt)) sum_{i' <= i} Wx(i', j)
 *   Jy(i, j+1/2) = -(q/(dx dt)) sum_{j' <= j} Wy(i, j')
 *   Jz(i, j)     =  q vz Wz(i, j)/(dx dy).
 * The window of 6 nodes per axis, [i0-2, i0+3], holds both supports for all
 * orders because a particle moves less than one cell per step. */
static void deposit_range(int nx, int ny, int order, double dx, double dy, double dt,
                          double q, int64_t k0, int64_t k1,
                 const int32_t* ix0, const int32_t* iy0, const double* fx0, const double* fy0,
                 const int32_t* ix1, const int32_t* iy1, const double* fx1, const double* fy1,
                 const double* ux, const double* uy, const double* uz,
                 double* jx, double* jy, double* jz) {
  enum { W = 6 };
  for (int64_t k = k0; k < k1; ++k) {
    double s0x[W], s1x[W], dsx[W], s0y[W], s1y[W], dsy[W];
    int bi = ix0[k] - 2, bj = iy0[k] - 2;
    for (int a = 0; a < W; ++a) {
      int i = bi + a, j = bj + a;
      s0x[a] = ora_shape(order, (double)(ix0[k] - i) + fx0[k]);
      s1x[a] = ora_shape(order, (double)(ix1[k] - i) + fx1[k]);
      s0y[a] = ora_shape(order, (double)(iy0[k] - j) + fy0[k]);
      s1y[a] = ora_shape(order, (double)(iy1[k] - j) + fy1[k]);
      dsx[a] = s1x[a] - s0x[a];
      dsy[a] = s1y[a] - s0y[a];
    }
    double g = sqrt(1.0 + ux[k] * ux[k] + uy[k] * uy[k] + uz[k] * uz[k]);
    double vz = uz[k] / g;
    double cx = -q / (dy * dt), cy = -q / (dx * dt), cz = q * vz / (dx * dy);
    for (int b = 0; b < W; ++b) {
      double acc = 0.0;
      for (int a = 0; a < W; ++a) {
        acc += dsx[a] * (s0y[b] + 0.5 * dsy[b]);
        jx[at(nx, ny, bi + a, bj + b)] += cx * acc;
      }
    }
    for (int a = 0; a < W; ++a) {
      double acc = 0.0;
      for (int b = 0; b < W; ++b) {
        acc += dsy[b] * (s0x[a] + 0.5 * dsx[a]);
        jy[at(nx, ny, bi + a, bj + b)] += cy * acc;
      }
    }
    for (int b = 0; b < W; ++b)
      for (int a = 0; a < W; ++a) {
        double wz = s0x[a] * s0y[b] + 0.5 * dsx[a] * s0y[b] + 0.5 * s0x[a] * dsy[b] +
                    dsx[a] * dsy[b] / 3.0;
        jz[at(nx, ny, bi + a, bj + b)] += cz * wz;
      }
  }
}

void ora_deposit(int nx, int ny, int order, double dx, double dy, double dt,
                 double q, int64_t np,
                 const int32_t* ix0, const int32_t* iy0, const double* fx0, const double* fy0,
                 const int32_t* ix1, const int32_t* iy1, const double* fx1, const double* fy1,
                 const double* ux, const double* uy, const double* uz,
                 double* jx, double* jy, double* jz) {
  const int nt = np >= ORA_PAR_MIN ? omp_get_max_threads() : 1;
  if (nt == 1) {
    deposit_range(nx, ny, order, dx, dy, dt, q, 0, np, ix0, iy0, fx0, fy0, ix1, iy1, fx1, fy1,
                  ux, uy, uz, jx, jy, jz);
    return;
  }
  /* thread t deposits the particles [t np/nt, (t+1) np/nt) into its own
   * zeroed copies of Jx, Jy, Jz; the copies are then added in thread order */
  const int64_t n = (int64_t)nx * ny;
  double** buf = malloc(sizeof(double*) * 3 * nt);
  for (int t = 0; t < 3 * nt; ++t) buf[t] = calloc((size_t)n, sizeof(double));
#pragma omp parallel num_threads(nt)
  {
    const int t = omp_get_thread_num();
    deposit_range(nx, ny, order, dx, dy, dt, q, np * t / nt, np * (t + 1) / nt, ix0, iy0, fx0,
                  fy0, ix1, iy1, fx1, fy1, ux, uy, uz, buf[3 * t], buf[3 * t + 1],
                  buf[3 * t + 2]);
  }
  double* const out[3] = {jx, jy, jz};
  for (int c = 0; c < 3; ++c) {
    double* bc[nt];
    for (int t = 0; t < nt; ++t) bc[t] = buf[3 * t + c];
    add_buffers(n, nt, bc, out[c]);
  }
  for (int t = 0; t < 3 * nt; ++t) free(buf[t]);
  free(buf);
}

void ora_wrap_periodic(int nx, int ny, int64_t np, int32_t* ix, int32_t* iy) {
  for (int64_t k = 0; k < np; ++k) {
    ix[k] = wrapi(ix[k], nx);
    iy[k] = wrapi(iy[k], ny);
  }
}

/* 5-point Laplacian of a periodic array at (i, j) */
static double lap(int nx, int ny, double dx, double dy, const double* f, int i, int j) {
  double c = f[at(nx, ny, i, j)];
  return (f[at(nx, ny, i + 1, j)] - 2.0 * c + f[at(nx, ny, i - 1, j)]) / (dx * dx) +
         (f[at(nx, ny, i, j + 1)] - 2.0 * c + f[at(nx, ny, i, j - 1)]) / (dy * dy);
}

/* curl with forward differences, evaluated at the B points (Eq. (5)):
 * (cE F)x(i, j+1/2) = dFz/dy, (cE F)y(i+1/2, j) = -dFz/dx,
 * (cE F)z(i+1/2, j+1/2) = dFy/dx - dFx/dy, for F co-located with E */
static void curl_e(int nx, int ny, double dx, double dy, const double* const* f, int i, int j,
                   double* out3) {
  out3[0] = (f[2][at(nx, ny, i, j + 1)] - f[2][at(nx, ny, i, j)]) / dy;
  out3[1] = -(f[2][at(nx, ny, i + 1, j)] - f[2][at(nx, ny, i, j)]) / dx;
  out3[2] = (f[1][at(nx, ny, i + 1, j)] - f[1][at(nx, ny, i, j)]) / dx -
            (f[0][at(nx, ny, i, j + 1)] - f[0][at(nx, ny, i, j)]) / dy;
}

/* curl with backward differences, evaluated at the E points (Eq. (6)):
 * (cB F)x(i+1/2, j) = dFz/dy, (cB F)y(i, j+1/2) = -dFz/dx,
 * (cB F)z(i, j) = dFy/dx - dFx/dy, for F co-located with B */
static void curl_b(int nx, int ny, double dx, double dy, const double* const* f, int i, int j,
                   double* out3) {
  out3[0] = (f[2][at(nx, ny, i, j)] - f[2][at(nx, ny, i, j - 1)]) / dy;
  out3[1] = -(f[2][at(nx, ny, i, j)] - f[2][at(nx, ny, i - 1, j)]) / dx;
  out3[2] = (f[1][at(nx, ny, i, j)] - f[1][at(nx, ny, i - 1, j)]) / dx -
            (f[0][at(nx, ny, i, j)] - f[0][at(nx, ny, i, j - 1)]) / dy;
}

/* Eq. (7) right-hand side, c = 1:
 * b = theta dt^2 (L B^n + 4 pi curl J^{n+1/2}) - dt curl E^n */
void ora_rhs(int nx, int ny, double dx, double dy, double dt, double theta,
             const double* const* e3, const double* const* b3, const double* const* j3,
             double* const* b_out) {
  const double four_pi = 4.0 * M_PI;
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny >= ORA_PAR_MIN)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double cj[3], ce[3];
      curl_e(nx, ny, dx, dy, j3, i, j, cj);
      curl_e(nx, ny, dx, dy, e3, i, j, ce);
      for (int c = 0; c < 3; ++c) {
        double lb = lap(nx, ny, dx, dy, b3[c], i, j);
        b_out[c][at(nx, ny, i, j)] = theta * dt * dt * (lb + four_pi * cj[c]) - dt * ce[c];
      }
    }
}

/* the operator of Eq. (7): A = 1 - (theta c dt)^2 L */
void ora_apply_A(int nx, int ny, double dx, double dy, double dt, double theta,
                 const double* x, double* y) {
  double a = (theta * dt) * (theta * dt);
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny >= ORA_PAR_MIN)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      y[at(nx, ny, i, j)] = x[at(nx, ny, i, j)] - a * lap(nx, ny, dx, dy, x, i, j);
}

static double dot(int64_t n, const double* a, const double* b) {
  const int nt = n >= ORA_PAR_MIN ? omp_get_max_threads() : 1;
  if (nt == 1) {
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k) s += a[k] * b[k];
    return s;
  }
  /* per-thread partial sums over contiguous ranges, added in thread order */
  double part[nt];
#pragma omp parallel num_threads(nt)
  {
    const int t = omp_get_thread_num();
    double s = 0.0;
    for (int64_t k = n * t / nt; k < n * (t + 1) / nt; ++k) s += a[k] * b[k];
    part[t] = s;
  }
  double s = 0.0;
  for (int t = 0; t < nt; ++t) s += part[t];
  return s;
}

/* Conjugate gradient (Hestenes-Stiefel) for a symmetric positive definite
 * operator given as a callback; the paper solves Eq. (7) by CG (Sec. 2,
 * citing Hoshino 2013). Starts from the x passed in; stops when
 * ||r||_2 <= rtol ||b||_2 (recursive residual) or after maxit iterations. */
static int cg_generic(int64_t n, void (*apply)(const void*, const double*, double*),
                      const void* ctx, const double* b, double* x, double rtol, int maxit,
                      double* relres) {
  double bnorm = sqrt(dot(n, b, b));
  if (bnorm == 0.0) {
    memset(x, 0, sizeof(double) * n);
    if (relres) *relres = 0.0;
    return 0;
  }
  double* r = malloc(sizeof(double) * n);
  double* p = malloc(sizeof(double) * n);
  double* q = malloc(sizeof(double) * n);
  apply(ctx, x, q);
#pragma omp parallel for schedule(static) if (n >= ORA_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) {
    r[k] = b[k] - q[k];
    p[k] = r[k];
  }
  double rr = dot(n, r, r);
  int it = 0;
  while (it < maxit && sqrt(rr) > rtol * bnorm) {
    apply(ctx, p, q);
    double alpha = rr / dot(n, p, q);
#pragma omp parallel for schedule(static) if (n >= ORA_PAR_MIN)
    for (int64_t k = 0; k < n; ++k) {
      x[k] += alpha * p[k];
      r[k] -= alpha * q[k];
    }
    double rr_new = dot(n, r, r);
    double beta = rr_new / rr;
#pragma omp parallel for schedule(static) if (n >= ORA_PAR_MIN)
    for (int64_t k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
    rr = rr_new;
    ++it;
  }
  if (relres) {
    apply(ctx, x, q);
    for (int64_t k = 0; k < n; ++k) r[k] = b[k] - q[k];
    *relres = sqrt(dot(n, r, r)) / bnorm;
  }
  free(r);
  free(p);
  free(q);
  return it;
}

struct periodic_op {
  int nx, ny;
  double dx, dy, dt, theta;
};
static void periodic_apply(const void* ctx, const double* x, double* y) {
  const struct periodic_op* o = (const struct periodic_op*)ctx;
  ora_apply_A(o->nx, o->ny, o->dx, o->dy, o->dt, o->theta, x, y);
}

int ora_cg(int nx, int ny, double dx, double dy, double dt, double theta,
           const double* b, double* x, double rtol, int maxit, double* relres) {
  struct periodic_op o = {nx, ny, dx, dy, dt, theta};
  return cg_generic((int64_t)nx * ny, periodic_apply, &o, b, x, rtol, maxit, relres);
}

/* Eqs. (5)-(6) with dB known:
 * E^{n+1} = E^n + dt curl_B(B^n + theta dB) - 4 pi dt J^{n+1/2}, B^{n+1} = B^n + dB */
void ora_update(int nx, int ny, double dx, double dy, double dt, double theta,
                double* const* e3, double* const* b3, const double* const* db3,
                const double* const* j3) {
  int64_t n = (int64_t)nx * ny;
  double* bt[3];
  for (int c = 0; c < 3; ++c) {
    bt[c] = malloc(sizeof(double) * n);
    for (int64_t k = 0; k < n; ++k) bt[c][k] = b3[c][k] + theta * db3[c][k];
  }
  const double four_pi = 4.0 * M_PI;
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny >= ORA_PAR_MIN)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double cb[3];
      curl_b(nx, ny, dx, dy, (const double* const*)bt, i, j, cb);
      for (int c = 0; c < 3; ++c) {
        int64_t k = at(nx, ny, i, j);
        e3[c][k] += dt * cb[c] - four_pi * dt * j3[c][k];
      }
    }
  for (int c = 0; c < 3; ++c) {
    for (int64_t k = 0; k < n; ++k) b3[c][k] += db3[c][k];
    free(bt[c]);
  }
}

/* Explicit FDTD (Yee) variant of the field advance, Eqs. (3)-(4): leapfrog
 * with B at half steps, B^{n+1/2} = B^{n-1/2} - c dt curl E^n and
 * E^{n+1} = E^n + c dt curl B^{n+1/2} - 4 pi dt J^{n+1/2}. The particles are
 * pushed with B at integer time, carried here as B^n = (B^{n-1/2} +
 * B^{n+1/2})/2, so the advance from (E^n, B^n) is three sweeps:
 *   B^{n+1/2} = B^n - (c dt/2) curl_E E^n
 *   E^{n+1}   = E^n + c dt curl_B B^{n+1/2} - 4 pi dt J^{n+1/2}
 *   B^{n+1}   = B^{n+1/2} - (c dt/2) curl_E E^{n+1}
 * whose half-step values satisfy Eqs. (3)-(4) exactly. */
void ora_update_explicit(int nx, int ny, double dx, double dy, double dt, double* const* e3,
                         double* const* b3, const double* const* j3) {
  const int64_t n = (int64_t)nx * ny;
  const double four_pi = 4.0 * M_PI;
  double* bh[3];
  for (int c = 0; c < 3; ++c) bh[c] = malloc(sizeof(double) * n);
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny >= ORA_PAR_MIN)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double ce[3];
      curl_e(nx, ny, dx, dy, (const double* const*)e3, i, j, ce);
      for (int c = 0; c < 3; ++c) bh[c][at(nx, ny, i, j)] = b3[c][at(nx, ny, i, j)] - 0.5 * dt * ce[c];
    }
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny >= ORA_PAR_MIN)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double cb[3];
      curl_b(nx, ny, dx, dy, (const double* const*)bh, i, j, cb);
      for (int c = 0; c < 3; ++c) {
        const int64_t k = at(nx, ny, i, j);
        e3[c][k] += dt * cb[c] - four_pi * dt * j3[c][k];
      }
    }
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny >= ORA_PAR_MIN)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double ce[3];
      curl_e(nx, ny, dx, dy, (const double* const*)e3, i, j, ce);
      for (int c = 0; c < 3; ++c) b3[c][at(nx, ny, i, j)] = bh[c][at(nx, ny, i, j)] - 0.5 * dt * ce[c];
    }
  for (int c = 0; c < 3; ++c) free(bh[c]);
}

static void charge_range(int nx, int ny, int order, double dx, double dy, double q, int64_t k0,
                         int64_t k1, const int32_t* ix, const int32_t* iy, const double* fx,
                         const double* fy, double* rho) {
  for (int64_t k = k0; k < k1; ++k)
    for (int j = iy[k] - 2; j <= iy[k] + 3; ++j) {
      double wy = ora_shape(order, (double)(iy[k] - j) + fy[k]);
      for (int i = ix[k] - 2; i <= ix[k] + 3; ++i) {
        double wx = ora_shape(order, (double)(ix[k] - i) + fx[k]);
        rho[at(nx, ny, i, j)] += q * wx * wy / (dx * dy);
      }
    }
}

void ora_charge(int nx, int ny, int order, double dx, double dy, double q, int64_t np,
                const int32_t* ix, const int32_t* iy, const double* fx, const double* fy,
                double* rho) {
  const int nt = np >= ORA_PAR_MIN ? omp_get_max_threads() : 1;
  if (nt == 1) {
    charge_range(nx, ny, order, dx, dy, q, 0, np, ix, iy, fx, fy, rho);
    return;
  }
  const int64_t n = (int64_t)nx * ny;
  double** buf = malloc(sizeof(double*) * nt);
  for (int t = 0; t < nt; ++t) buf[t] = calloc((size_t)n, sizeof(double));
#pragma omp parallel num_threads(nt)
  {
    const int t = omp_get_thread_num();
    charge_range(nx, ny, order, dx, dy, q, np * t / nt, np * (t + 1) / nt, ix, iy, fx, fy,
                 buf[t]);
  }
  add_buffers(n, nt, buf, rho);
  for (int t = 0; t < nt; ++t) free(buf[t]);
  free(buf);
}

void ora_div_e(int nx, int ny, double dx, double dy, const double* ex, const double* ey,
               double* out) {
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      out[at(nx, ny, i, j)] = (ex[at(nx, ny, i, j)] - ex[at(nx, ny, i - 1, j)]) / dx +
                              (ey[at(nx, ny, i, j)] - ey[at(nx, ny, i, j - 1)]) / dy;
}

void ora_div_b(int nx, int ny, double dx, double dy, const double* bx, const double* by,
               double* out) {
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      out[at(nx, ny, i, j)] = (bx[at(nx, ny, i + 1, j)] - bx[at(nx, ny, i, j)]) / dx +
                              (by[at(nx, ny, i, j + 1)] - by[at(nx, ny, i, j)]) / dy;
}

double ora_kinetic(int64_t np, double m, const double* ux, const double* uy, const double* uz) {
  const int nt = np >= ORA_PAR_MIN ? omp_get_max_threads() : 1;
  double part[nt];
#pragma omp parallel num_threads(nt)
  {
    const int t = omp_get_thread_num();
    double s = 0.0;
    for (int64_t k = np * t / nt; k < np * (t + 1) / nt; ++k)
      s += m * (sqrt(1.0 + ux[k] * ux[k] + uy[k] * uy[k] + uz[k] * uz[k]) - 1.0);
    part[t] = s;
  }
  double s = 0.0;
  for (int t = 0; t < nt; ++t) s += part[t];
  return s;
}

/* ------------------------------------------------------------------------
 * Shock set-up (a reading: the paper only says that the shock runs inject
 * the flow at one side and reflect it at the other, Sec. 4). x = 0 and
 * x = (nx-1) dx are conducting walls: Ey, Ez and Bx are zero on those node
 * lines, and the half-integer components (Ex, By, Bz, Jx) of the last column
 * lie outside and are zero. Particles reflect specularly at x = 0 and leave
 * the run when they reach x_out = (nx - ORA_WALL_GAP) dx, where new flow is
 * injected. y stays periodic.
 * ---------------------------------------------------------------------- */

/* field value at column i (any integer) of component c with the conductor
 * images behind x = 0: integer-x components (Ey, Ez, Bx) are odd about the
 * wall node line, half-integer ones (Ex, By, Bz) even */
static double wall_field(int nx, int ny, const double* f, int c, int i, int j) {
  if (i < 0) {
    if (STAG_X[c] > 0.0) return f[at(nx, ny, -i - 1, j)];
    return -f[at(nx, ny, -i, j)];
  }
  if (i >= nx) abort();   /* particles stay ORA_WALL_GAP cells from the right wall */
  return f[at(nx, ny, i, j)];
}

void ora_gather_wall(int nx, int ny, int order, const double* const* f6,
                     int64_t np, const int32_t* ix, const int32_t* iy,
                     const double* fx, const double* fy, double* out6) {
  for (int64_t k = 0; k < np; ++k) {
    for (int c = 0; c < 6; ++c) {
      double sum = 0.0;
      for (int j = iy[k] - 2; j <= iy[k] + 2; ++j) {
        double wy = ora_shape(order, (double)(iy[k] - j) + fy[k] - STAG_Y[c]);
        for (int i = ix[k] - 2; i <= ix[k] + 2; ++i) {
          double wx = ora_shape(order, (double)(ix[k] - i) + fx[k] - STAG_X[c]);
          if (wx == 0.0 || wy == 0.0) continue;
          sum += wall_field(nx, ny, f6[c], c, i, j) * wx * wy;
        }
      }
      out6[(int64_t)c * np + k] = sum;
    }
  }
}

void ora_gather_nodal_wall(int nx, int ny, int order, const double* const* f6,
                           int64_t np, const int32_t* ix, const int32_t* iy,
                           const double* fx, const double* fy, double* out6) {
  gather_nodal(nx, ny, order, f6, np, ix, iy, fx, fy, out6, wall_field);
}

/* add v to component c (0 Jx, 1 Jy, 2 Jz, 3 rho) at column i, folding a
 * column behind the wall onto its mirror: rho, Jy and Jz keep their sign,
 * Jx (half-integer x, the normal current) changes sign. The fold keeps the
 * discrete continuity equation exact at every node off the wall line. */
static void wall_add(int nx, int ny, double* f, int c, int i, int j, double v) {
  if (i < 0) {
    if (c == 0) {
      i = -i - 1;
      v = -v;
    } else {
      i = -i;
    }
  }
  if (i >= nx) abort();
  f[at(nx, ny, i, j)] += v;
}

/* Esirkepov deposit (same arithmetic as ora_deposit) of the unreflected
 * displacement, with the wall fold */
void ora_deposit_wall(int nx, int ny, int order, double dx, double dy, double dt,
                      double q, int64_t np,
                      const int32_t* ix0, const int32_t* iy0, const double* fx0,
                      const double* fy0, const int32_t* ix1, const int32_t* iy1,
                      const double* fx1, const double* fy1, const double* ux,
                      const double* uy, const double* uz, double* jx, double* jy, double* jz) {
  enum { W = 6 };
  for (int64_t k = 0; k < np; ++k) {
    double s0x[W], s1x[W], dsx[W], s0y[W], s1y[W], dsy[W];
    int bi = ix0[k] - 2, bj = iy0[k] - 2;
    for (int a = 0; a < W; ++a) {
      int i = bi + a, j = bj + a;
      s0x[a] = ora_shape(order, (double)(ix0[k] - i) + fx0[k]);
      s1x[a] = ora_shape(order, (double)(ix1[k] - i) + fx1[k]);
      s0y[a] = ora_shape(order, (double)(iy0[k] - j) + fy0[k]);
      s1y[a] = ora_shape(order, (double)(iy1[k] - j) + fy1[k]);
      dsx[a] = s1x[a] - s0x[a];
      dsy[a] = s1y[a] - s0y[a];
    }
    double g = sqrt(1.0 + ux[k] * ux[k] + uy[k] * uy[k] + uz[k] * uz[k]);
    double vz = uz[k] / g;
    double cx = -q / (dy * dt), cy = -q / (dx * dt), cz = q * vz / (dx * dy);
    for (int b = 0; b < W; ++b) {
      double acc = 0.0;
      for (int a = 0; a < W; ++a) {
        acc += dsx[a] * (s0y[b] + 0.5 * dsy[b]);
        if (acc != 0.0) wall_add(nx, ny, jx, 0, bi + a, bj + b, cx * acc);
      }
    }
    for (int a = 0; a < W; ++a) {
      double acc = 0.0;
      for (int b = 0; b < W; ++b) {
        acc += dsy[b] * (s0x[a] + 0.5 * dsx[a]);
        if (acc != 0.0) wall_add(nx, ny, jy, 1, bi + a, bj + b, cy * acc);
      }
    }
    for (int b = 0; b < W; ++b)
      for (int a = 0; a < W; ++a) {
        double wz = s0x[a] * s0y[b] + 0.5 * dsx[a] * s0y[b] + 0.5 * s0x[a] * dsy[b] +
                    dsx[a] * dsy[b] / 3.0;
        if (wz != 0.0) wall_add(nx, ny, jz, 2, bi + a, bj + b, cz * wz);
      }
  }
}

/* currents on the conductors drive no field: Jy, Jz on both wall node lines
 * and Jx of the last (outside) column are set to zero */
void ora_mask_wall_currents(int nx, int ny, double* jx, double* jy, double* jz) {
  for (int j = 0; j < ny; ++j) {
    jy[at(nx, ny, 0, j)] = 0.0;
    jz[at(nx, ny, 0, j)] = 0.0;
    jy[at(nx, ny, nx - 1, j)] = 0.0;
    jz[at(nx, ny, nx - 1, j)] = 0.0;
    jx[at(nx, ny, nx - 1, j)] = 0.0;
  }
}

/* after the deposit: specular reflection of particles behind x = 0
 * (x -> -x, ux -> -ux) and removal of those at or beyond x_out; keep[k] = 0
 * marks a removed particle. y is wrapped periodically. */
void ora_boundary_wall(int nx, int ny, int64_t np, int32_t* ix, int32_t* iy, double* fx,
                       double* ux, uint8_t* keep) {
  for (int64_t k = 0; k < np; ++k) {
    if (ix[k] < 0) {
      /* x = ix + fx with ix = -1: -x = (-ix - 1) + (1 - fx) */
      double f = 1.0 - fx[k];
      int32_t c = -ix[k] - 1;
      if (f >= 1.0) {
        f -= 1.0;
        c += 1;
      }
      ix[k] = c;
      fx[k] = f;
      ux[k] = -ux[k];
    }
    keep[k] = ix[k] < nx - ORA_WALL_GAP ? 1 : 0;
    iy[k] = wrapi(iy[k], ny);
  }
}

/* row class of component c at column i: 0 free, 1 fixed (zero). Bx lives on
 * integer x and is zero on both wall lines; By, Bz live on half-integer x and
 * the last column is outside. */
static int wall_fixed(int nx, int c, int i) {
  if (c == 0) return i == 0 || i == nx - 1;
  return i == nx - 1;
}

/* x-neighbour value for the Laplacian of component c at free row i: a fixed
 * neighbour is zero (Dirichlet); behind a conductor the tangential By, Bz take
 * the row's own value (their normal derivative vanishes at the wall) */
static double wall_xnb(int nx, int ny, const double* f, int c, int i, int j, int di) {
  int n = i + di;
  if (c == 0) {
    if (n <= 0 || n >= nx - 1) return 0.0;
    return f[at(nx, ny, n, j)];
  }
  if (n < 0 || n >= nx - 1) return f[at(nx, ny, i, j)];
  return f[at(nx, ny, n, j)];
}

static double lap_wall(int nx, int ny, double dx, double dy, const double* f, int c, int i,
                       int j) {
  double v = f[at(nx, ny, i, j)];
  return (wall_xnb(nx, ny, f, c, i, j, 1) - 2.0 * v + wall_xnb(nx, ny, f, c, i, j, -1)) /
             (dx * dx) +
         (f[at(nx, ny, i, j + 1)] - 2.0 * v + f[at(nx, ny, i, j - 1)]) / (dy * dy);
}

void ora_rhs_wall(int nx, int ny, double dx, double dy, double dt, double theta,
                  const double* const* e3, const double* const* b3, const double* const* j3,
                  double* const* b_out) {
  const double four_pi = 4.0 * M_PI;
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny >= ORA_PAR_MIN)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double cj[3], ce[3];
      curl_e(nx, ny, dx, dy, j3, i, j, cj);
      curl_e(nx, ny, dx, dy, e3, i, j, ce);
      for (int c = 0; c < 3; ++c) {
        double v = 0.0;
        if (!wall_fixed(nx, c, i)) {
          double lb = lap_wall(nx, ny, dx, dy, b3[c], c, i, j);
          v = theta * dt * dt * (lb + four_pi * cj[c]) - dt * ce[c];
        }
        b_out[c][at(nx, ny, i, j)] = v;
      }
    }
}

void ora_apply_A_wall(int nx, int ny, double dx, double dy, double dt, double theta, int c,
                      const double* x, double* y) {
  double a = (theta * dt) * (theta * dt);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int64_t k = at(nx, ny, i, j);
      y[k] = wall_fixed(nx, c, i) ? x[k] : x[k] - a * lap_wall(nx, ny, dx, dy, x, c, i, j);
    }
}

struct wall_op {
  int nx, ny, c;
  double dx, dy, dt, theta;
};
static void wall_apply(const void* ctx, const double* x, double* y) {
  const struct wall_op* o = (const struct wall_op*)ctx;
  ora_apply_A_wall(o->nx, o->ny, o->dx, o->dy, o->dt, o->theta, o->c, x, y);
}

int ora_cg_wall(int nx, int ny, double dx, double dy, double dt, double theta, int c,
                const double* b, double* x, double rtol, int maxit, double* relres) {
  struct wall_op o = {nx, ny, c, dx, dy, dt, theta};
  return cg_generic((int64_t)nx * ny, wall_apply, &o, b, x, rtol, maxit, relres);
}

/* Eqs. (5)-(6) with the walls: E nodes on a conductor (Ey, Ez on both wall
 * lines, Ex of the outside column) stay zero; B += dB (dB is zero on fixed rows) */
void ora_update_wall(int nx, int ny, double dx, double dy, double dt, double theta,
                     double* const* e3, double* const* b3, const double* const* db3,
                     const double* const* j3) {
  ora_update(nx, ny, dx, dy, dt, theta, e3, b3, db3, j3);
  for (int j = 0; j < ny; ++j) {
    e3[1][at(nx, ny, 0, j)] = 0.0;
    e3[2][at(nx, ny, 0, j)] = 0.0;
    e3[0][at(nx, ny, nx - 1, j)] = 0.0;
    e3[1][at(nx, ny, nx - 1, j)] = 0.0;
    e3[2][at(nx, ny, nx - 1, j)] = 0.0;
  }
}

/* charge density with the wall fold (rho keeps its sign behind x = 0) */
void ora_charge_wall(int nx, int ny, int order, double dx, double dy, double q, int64_t np,
                     const int32_t* ix, const int32_t* iy, const double* fx, const double* fy,
                     double* rho) {
  for (int64_t k = 0; k < np; ++k)
    for (int j = iy[k] - 2; j <= iy[k] + 3; ++j) {
      double wy = ora_shape(order, (double)(iy[k] - j) + fy[k]);
      for (int i = ix[k] - 2; i <= ix[k] + 3; ++i) {
        double wx = ora_shape(order, (double)(ix[k] - i) + fx[k]);
        if (wx == 0.0 || wy == 0.0) continue;
        wall_add(nx, ny, rho, 3, i, j, q * wx * wy / (dx * dy));
      }
    }
}
