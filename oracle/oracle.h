/*
 * Plain FP64 CPU oracle of the 2D3V implicit-FDTD PIC step.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, obviously correct
 * reference the GPU library is checked against. Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU product path never does. It shares no source with the GPU library.
 *
 * Paper: Ikeya & Matsumoto, PASJ 2015 (arXiv:1412.2480).
 *
 * Grid (standard 2D Yee layout; the paper's Fig. 1 is not reproduced, so the
 * textbook arrangement is taken): nx*ny cells, row-major arrays [ny][nx],
 * index k = j*nx + i, periodic in both directions.
 *   Ex(i+1/2, j)   Ey(i, j+1/2)   Ez(i, j)
 *   Bx(i, j+1/2)   By(i+1/2, j)   Bz(i+1/2, j+1/2)
 *   Jx, Jy, Jz co-located with Ex, Ey, Ez; rho at nodes (i, j).
 * Units: Gaussian with c = 1 (Maxwell equations of Sec. 2, Eqs. (1)-(2)).
 *
 * Particles: cell index (ix, iy) and in-cell offset (fx, fy) in [0, 1), so
 * the position in cell units is X = ix + fx; momentum u = gamma v (ux, uy, uz)
 * at the half step n-1/2, position at step n (leapfrog implied by J^{n+1/2}
 * in Eq. (6)).
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* OpenMP threads of the following calls (n <= 0: back to the default,
 * OMP_NUM_THREADS or the host's cores); results are a fixed function of the
 * thread count. */
void ora_set_threads(int n);
int ora_get_threads(void);

/* B-spline shape of degree `order` (1, 2 or 3), evaluated at distance d in
 * cell units; shared by gather and charge assignment (Sec. 1, Sec. 3). */
double ora_shape(int order, double d);

/* Momentum-conserving gather (Sec. 1 and Sec. 3, citing Birdsall & Langdon
 * ch. 8), the method's reading: the force is interpolated from the charge
 * nodes with the charge-assignment weights, every component first averaged
 * from its Yee points onto the nodes (Ex, By along x; Ey, Bx along y; Bz over
 * the four surrounding points; Ez is a node value). f6 = {Ex, Ey, Ez, Bx, By,
 * Bz}, each [ny][nx]. out6[c*np + k]. */
void ora_gather_nodal(int nx, int ny, int order, const double* const* f6,
                      int64_t np, const int32_t* ix, const int32_t* iy,
                      const double* fx, const double* fy, double* out6);

/* The alternative reading, kept for comparison: every field component is
 * interpolated from its own staggered points with the same order-p shape in
 * x and y as the charge assignment (no averaging onto the nodes). */
void ora_gather(int nx, int ny, int order, const double* const* f6,
                int64_t np, const int32_t* ix, const int32_t* iy,
                const double* fx, const double* fy, double* out6);

/* Relativistic Boris rotation (the paper names no pusher; read as the
 * standard Boris scheme, with gamma from the half-kicked momentum).
 * qdt_2m = q*dt/(2m). e3/b3 point at per-particle Ex..Ez and Bx..Bz columns
 * (stride np). Updates ux, uy, uz in place from n-1/2 to n+1/2. */
void ora_boris(int64_t np, double qdt_2m, const double* e3, const double* b3,
               double* ux, double* uy, double* uz);

/* Position advance x^{n+1} = x^n + dt u^{n+1/2}/gamma (2D; z untracked).
 * Writes the unwrapped new cell index and offset. */
void ora_move(int64_t np, double dt, double dx, double dy,
              const double* ux, const double* uy, const double* uz,
              int32_t* ix, int32_t* iy, double* fx, double* fy);

/* Esirkepov (2001) density-decomposition current deposit of J^{n+1/2} from
 * the displacement (ix0+fx0, iy0+fy0) -> (ix1+fx1, iy1+fy1), cited in Sec. 1
 * and Sec. 3. Adds into jx, jy, jz ([ny][nx], periodic wrap). */
void ora_deposit(int nx, int ny, int order, double dx, double dy, double dt,
                 double q, int64_t np,
                 const int32_t* ix0, const int32_t* iy0, const double* fx0, const double* fy0,
                 const int32_t* ix1, const int32_t* iy1, const double* fx1, const double* fy1,
                 const double* ux, const double* uy, const double* uz,
                 double* jx, double* jy, double* jz);

/* Periodic wrap of cell indices into [0, nx) x [0, ny). */
void ora_wrap_periodic(int nx, int ny, int64_t np, int32_t* ix, int32_t* iy);

/* Right-hand side of Eq. (7) on each B component's own grid:
 * b = theta dt^2 (L B^n + 4 pi curl_E J) - dt curl_E E^n. */
void ora_rhs(int nx, int ny, double dx, double dy, double dt, double theta,
             const double* const* e3, const double* const* b3, const double* const* j3,
             double* const* b_out);

/* Apply A = I - (theta dt)^2 L (5-point Laplacian, periodic). */
void ora_apply_A(int nx, int ny, double dx, double dy, double dt, double theta,
                 const double* x, double* y);

/* Plain unpreconditioned conjugate gradient for A x = b (Eq. (7) is solved
 * by CG in the paper, Sec. 2). Starts from the x passed in. Stops when
 * ||r||_2 <= rtol ||b||_2 (recursive residual) or after maxit iterations.
 * Returns the iteration count; *relres receives ||b - A x||_2 / ||b||_2
 * recomputed from scratch (0 when b = 0). */
int ora_cg(int nx, int ny, double dx, double dy, double dt, double theta,
           const double* b, double* x, double rtol, int maxit, double* relres);

/* Field update from Eqs. (5)-(6) given dB = B^{n+1} - B^n:
 * E^{n+1} = E^n + dt curl_B(B^n + theta dB) - 4 pi dt J;  B^{n+1} = B^n + dB. */
void ora_update(int nx, int ny, double dx, double dy, double dt, double theta,
                double* const* e3, double* const* b3, const double* const* db3,
                const double* const* j3);

/* Explicit FDTD (Yee) field advance of Eqs. (3)-(4) (the scheme the paper
 * contrasts with the implicit one, Sec. 2): B carried at integer times for
 * the particle push as the mean of the half-step values; E^n, B^n -> E^{n+1},
 * B^{n+1} with J^{n+1/2}, periodic. Stable for c dt sqrt(1/dx^2 + 1/dy^2) <= 1;
 * a vacuum mode's amplification obeys Eq. (16). */
void ora_update_explicit(int nx, int ny, double dx, double dy, double dt, double* const* e3,
                         double* const* b3, const double* const* j3);

/* Charge density at nodes, rho(i,j) += q S(X-i) S(Y-j)/(dx dy). */
void ora_charge(int nx, int ny, int order, double dx, double dy, double q, int64_t np,
                const int32_t* ix, const int32_t* iy, const double* fx, const double* fy,
                double* rho);

/* Discrete divergences: divE at nodes (backward differences of Ex, Ey),
 * divB at cell centres (forward differences of Bx, By). */
void ora_div_e(int nx, int ny, double dx, double dy, const double* ex, const double* ey, double* out);
void ora_div_b(int nx, int ny, double dx, double dy, const double* bx, const double* by, double* out);

/* ---- Shock set-up (a reading; the paper only says the shock runs inject the
 * flow at one side and reflect it at the other, Sec. 4): conducting walls at
 * x = 0 and x = (nx-1) dx, specular particle reflection at x = 0, particles
 * removed at x >= (nx - ORA_WALL_GAP) dx where the flow is injected, y
 * periodic. Tangential E (Ey, Ez) and normal B (Bx) vanish on the wall node
 * lines; the half-integer components of the last column lie outside. */
#define ORA_WALL_GAP 4

/* gather with the conductor images behind x = 0 (Ey, Ez, Bx odd; Ex, By, Bz
 * even about the wall line) */
void ora_gather_wall(int nx, int ny, int order, const double* const* f6,
                     int64_t np, const int32_t* ix, const int32_t* iy,
                     const double* fx, const double* fy, double* out6);

/* the node-averaged gather with the same conductor images */
void ora_gather_nodal_wall(int nx, int ny, int order, const double* const* f6,
                           int64_t np, const int32_t* ix, const int32_t* iy,
                           const double* fx, const double* fy, double* out6);

/* Esirkepov deposit of the unreflected displacement; columns behind the wall
 * fold onto their mirrors (rho, Jy, Jz with their sign, Jx negated) */
void ora_deposit_wall(int nx, int ny, int order, double dx, double dy, double dt,
                      double q, int64_t np,
                      const int32_t* ix0, const int32_t* iy0, const double* fx0,
                      const double* fy0, const int32_t* ix1, const int32_t* iy1,
                      const double* fx1, const double* fy1, const double* ux,
                      const double* uy, const double* uz, double* jx, double* jy, double* jz);

/* zero Jy, Jz on both wall lines and Jx of the outside column */
void ora_mask_wall_currents(int nx, int ny, double* jx, double* jy, double* jz);

/* reflect particles behind x = 0 (x -> -x, ux -> -ux); keep[k] = 0 for those
 * at or beyond x_out; wrap y */
void ora_boundary_wall(int nx, int ny, int64_t np, int32_t* ix, int32_t* iy, double* fx,
                       double* ux, uint8_t* keep);

/* Eq. (7) with the walls, component by component (c = 0 Bx, 1 By, 2 Bz):
 * fixed rows (Bx on both wall lines, the outside column of By and Bz) have
 * b = 0 and an identity row; a fixed x-neighbour reads zero; behind a wall By
 * and Bz take the row's own value. */
void ora_rhs_wall(int nx, int ny, double dx, double dy, double dt, double theta,
                  const double* const* e3, const double* const* b3, const double* const* j3,
                  double* const* b_out);
void ora_apply_A_wall(int nx, int ny, double dx, double dy, double dt, double theta, int c,
                      const double* x, double* y);
int ora_cg_wall(int nx, int ny, double dx, double dy, double dt, double theta, int c,
                const double* b, double* x, double rtol, int maxit, double* relres);

/* charge density at nodes with the same fold as the deposit */
void ora_charge_wall(int nx, int ny, int order, double dx, double dy, double q, int64_t np,
                     const int32_t* ix, const int32_t* iy, const double* fx, const double* fy,
                     double* rho);

/* Eqs. (5)-(6) with the conductor E nodes held at zero */
void ora_update_wall(int nx, int ny, double dx, double dy, double dt, double theta,
                     double* const* e3, double* const* b3, const double* const* db3,
                     const double* const* j3);

/* sum m (gamma - 1) over particles */
double ora_kinetic(int64_t np, double m, const double* ux, const double* uy, const double* uz);

#ifdef __cplusplus
}
#endif
#endif
