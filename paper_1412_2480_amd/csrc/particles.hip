// Particle loop of the implicit-FDTD PIC method of Ikeya & Matsumoto
// (PASJ 2015): momentum-conserving gather with order-p B-spline shapes,
// relativistic Boris push, move, and Esirkepov (2001) density-decomposition
// deposit of J^{n+1/2} (Sec. 1 and Sec. 3 name these ingredients; Eq. (6)
// puts J at the half step).
//
// Layout: particles are kept sorted by cell tile (TX x TY cells). One
// work-group owns one tile: it stages the tile's E and B (+ guard nodes) in
// LDS, pushes every particle of every species of the tile, accumulates the
// current of the tile (+ guard nodes) in LDS, and writes that patch out whole.
// A second pass sums the overlapping patches node by node in a fixed order
// (no global atomics on J). The particle store is double-buffered: every
// particle is written once into its (new) tile's region of the next buffer,
// at a slot taken from that tile's counter (one global atomic per wavefront
// and destination tile), so a particle that changes tile costs no more than
// one that stays; the re-binning kernel only commits the counts.
#include <math.h>

#include <type_traits>

#include "pic_dev.h"
#include "pic_launch.h"

namespace {

constexpr int G = PIC_GUARD_LO;
constexpr double kFourPi = 12.566370614359172953850573533118;

enum { MODE_FUSED = PIC_MODE_FUSED, MODE_PUSH = PIC_MODE_PUSH, MODE_DEPOSIT = PIC_MODE_DEPOSIT,
       MODE_CHARGE = 3 };

// largest displacement per step, in cells: the Esirkepov window assumes a
// particle crosses at most one cell boundary per axis per step
template <typename R> __device__ __forceinline__ R max_disp();
template <> __device__ __forceinline__ float max_disp<float>() { return 1.0f - 0x1p-20f; }
template <> __device__ __forceinline__ double max_disp<double>() { return 1.0 - 0x1p-40; }

// B-spline weights of degree P for a point at offset t (in cells) from node 0
// of the component's grid, t in [-1/2, 1). Returns the first node index
// (relative to node 0) and the P+1 non-trivial weights. Every sum is an
// explicit fused multiply-add, so the weights of a position round the same
// way wherever the function is inlined: the new shape a step deposits with is
// then bit for bit the old shape of the next step (and of the charge
// density), which the discrete continuity equation needs.
template <int P, typename R>
__device__ __forceinline__ int bspline_weights(R t, R (&w)[P + 1]) {
  if constexpr (P == 1) {
    const int fl = t < R(0) ? -1 : 0;
    const R d = t - R(fl);
    w[0] = R(1) - d;
    w[1] = d;
    return fl;
  } else if constexpr (P == 2) {
    const int r = t >= R(0.5) ? 1 : 0;     // nearest node
    const R d = t - R(r);                  // in [-1/2, 1/2)
    const R a = R(0.5) - d, b = R(0.5) + d;
    w[0] = R(0.5) * a * a;
    w[1] = fma(-d, d, R(0.75));
    w[2] = R(0.5) * b * b;
    return r - 1;
  } else {
    const int fl = t < R(0) ? -1 : 0;
    const R d = t - R(fl);                 // in [0, 1)
    const R d2 = d * d, d3 = d2 * d, e = R(1) - d;
    const R sixth = R(1) / R(6);
    w[0] = e * e * e * sixth;
    w[1] = fma(R(3), d3, fma(R(-6), d2, R(4))) * sixth;
    w[2] = fma(R(-3), d3, fma(R(3), d2, fma(R(3), d, R(1)))) * sixth;
    w[3] = d3 * sixth;
    return fl - 1;
  }
}

// 1/sqrt(x) and 1/x: in the FP32 form the hardware's approximations (1 ulp,
// against the 6e-8 unit roundoff the form already carries); in FP64 exact
template <typename R> __device__ __forceinline__ R inv_sqrt(R x);
template <> __device__ __forceinline__ float inv_sqrt<float>(float x) {
  return __builtin_amdgcn_rsqf(x);
}
template <> __device__ __forceinline__ double inv_sqrt<double>(double x) { return 1.0 / sqrt(x); }
template <typename R> __device__ __forceinline__ R recip(R x);
template <> __device__ __forceinline__ float recip<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
template <> __device__ __forceinline__ double recip<double>(double x) { return 1.0 / x; }

// sum_{jj,ii} F(x0+ii, y0+jj) wx[ii] wy[jj] from an LDS plane with pitch PW
template <int P, typename R, typename F>
__device__ __forceinline__ R interp(const F* f, int PW, int x0, int y0, const R (&wx)[P + 1],
                                    const R (&wy)[P + 1]) {
  R s = R(0);
#pragma unroll
  for (int jj = 0; jj <= P; ++jj) {
    const F* row = f + (y0 + jj) * PW + x0;
    R acc = R(0);
#pragma unroll
    for (int ii = 0; ii <= P; ++ii) acc += R(row[ii]) * wx[ii];
    s += acc * wy[jj];
  }
  return s;
}

// advance an in-cell offset by a displacement of at most one cell; returns
// the cell change; an offset that rounds to exactly 1 moves to the next cell
template <typename R>
__device__ __forceinline__ int advance(R& f, R disp) {
  R g = f + disp;
  int d = 0;
  if (g >= R(1)) {
    g -= R(1);
    d = 1;
  } else if (g < R(0)) {
    g += R(1);
    d = -1;
  }
  if (g >= R(1)) {
    g -= R(1);
    d += 1;
  }
  f = g;
  return d;
}

// Node shapes on the Esirkepov window. A particle moves less than one cell,
// so the first support node of the new position differs from that of the old
// one by at most one node and both supports fit in P + 2 nodes starting at the
// smaller first node. off is 0 or 1: where the P + 1 weights start.
template <int P, typename R>
__device__ __forceinline__ R place(const R (&w)[P + 1], int off, int a) {
  const R v0 = (a <= P) ? w[a > P ? P : a] : R(0);
  const R v1 = (a >= 1) ? w[a < 1 ? 0 : a - 1] : R(0);
  return off == 0 ? v0 : v1;
}

// The FP64 values of a shape's weights, the last taken as one minus the
// others so that the shape sums to exactly one. The charge density and the
// current are both formed from these: a shape whose weights summed to one
// only to rounding (the FP32 form's, to about 6e-8) would change the
// particle's charge from step to step, and the window's last node, where
// the running sum of the shape change ends, would not receive it.
template <int P, typename R>
__device__ __forceinline__ void unit_weights(const R (&w)[P + 1], double (&d)[P + 1]) {
  double sum = 0.0;
#pragma unroll
  for (int a = 0; a < P; ++a) {
    d[a] = (double)w[a];
    sum += d[a];
  }
  d[P] = 1.0 - sum;
}

// reserve slots in counters[key] for every lane with want set, one atomic per
// wavefront and distinct key; returns the lane's slot (or -1)
__device__ __forceinline__ int wave_reserve(bool want, int key, int* counters) {
  const int lane = __lane_id();
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int slot = -1;
  bool pending = want;
  while (true) {
    const unsigned long long m = __ballot(pending);
    if (m == 0ull) break;
    const int leader = __ffsll((unsigned long long)m) - 1;
    const int k = __shfl(key, leader);
    const bool mine = pending && key == k;
    const unsigned long long mm = __ballot(mine);
    int base = 0;
    if (lane == leader) base = atomicAdd(&counters[k], __popcll(mm));
    base = __shfl(base, leader);
    if (mine) {
      slot = base + __popcll(mm & below);
      pending = false;
    }
  }
  return slot;
}

template <typename R, typename F, int P, int MODE, bool DIAG, bool NODAL>
__device__ void tile_body(const DevState<R>& st, const DevRun& run, int tile, int tx, int ty,
                          int x0, int y0, int tw, int th, const F* sF, double* sJ, int part,
                          int sel, double (&wk)[PIC_MAXS][2]) {
  constexpr int W = P + 2;   // Esirkepov window: union of old and new supports
  const int PW = st.PW, PH = st.PH;
  const int plane = PW * PH;
  const R dt = R(run.dt);
  const R dtdx = R(run.dt / run.dx), dtdy = R(run.dt / run.dy);
  const R lim = max_disp<R>();

  for (int s = 0; s < run.nspecies; ++s) {
    // the charge mode deposits one species' number density when sel >= 0
    if (MODE == MODE_CHARGE && sel >= 0 && s != sel) continue;
    const int n_all = st.cnt[s][tile];
    // this work-group's share of the tile's particles
    const int lo = (int)(((long long)n_all * part) / st.K);
    const int n = (int)(((long long)n_all * (part + 1)) / st.K);
    const long long base = (long long)tile * st.tile_slots[s];
    const R qdt_2m = R(run.q[s] * run.dt / (2.0 * run.m[s]));
    // current factors in FP64 in both forms: rounded to FP32 they would
    // scale each species' current by its own rounding error, which Gauss's
    // law would see at 1e-6 of the charge density per step
    const double cjx = -run.q[s] / (run.dy * run.dt);
    const double cjy = -run.q[s] / (run.dx * run.dt);
    const double cjz = run.q[s] / (run.dx * run.dy);
    const double mass = run.m[s];
    for (int k0 = lo; k0 < n; k0 += blockDim.x) {
      const int k = k0 + threadIdx.x;
      const bool active = k < n;
      bool leave = false;
      bool gone = false;   // left a shock run through its outflow line
      int dest = 0;
      int gcell = 0;
      R fx1 = R(0), fy1 = R(0), ux = R(0), uy = R(0), uz = R(0);
      int pid = 0;
      if (active) {
        const long long idx = base + k;
        int cell0, dcx = 0, dcy = 0;
        R fx, fy;
        if constexpr (MODE == MODE_DEPOSIT) {
          cell0 = st.old_cell[s][idx];
          fx = st.old_ox[s][idx];
          fy = st.old_oy[s][idx];
          const int c1 = st.cell[s][idx];
          fx1 = st.ox[s][idx];
          fy1 = st.oy[s][idx];
          ux = st.ux[s][idx];
          uy = st.uy[s][idx];
          uz = st.uz[s][idx];
          dcx = pic_cell_ix(c1) - pic_cell_ix(cell0);
          dcy = pic_cell_iy(c1) - pic_cell_iy(cell0);
          if (dcx > 1) dcx -= run.nx;
          if (dcx < -1) dcx += run.nx;
          if (dcy > 1) dcy -= run.ny;
          if (dcy < -1) dcy += run.ny;
        } else {
          cell0 = st.cell[s][idx];
          fx = st.ox[s][idx];
          fy = st.oy[s][idx];
          ux = st.ux[s][idx];
          uy = st.uy[s][idx];
          uz = st.uz[s][idx];
        }
        const int lx = pic_cell_ix(cell0) - x0;
        const int ly = pic_cell_iy(cell0) - y0;
        R w0x[P + 1], w0y[P + 1];
        const int f0x = bspline_weights<P, R>(fx, w0x);
        const int f0y = bspline_weights<P, R>(fy, w0y);

        if constexpr (MODE == MODE_CHARGE) {
          // from the same unit-sum FP64 weights as the deposit
          const double cq = (sel >= 0 ? 1.0 : run.q[s]) / (run.dx * run.dy);
          const int ax0 = lx + f0x + G, ay0 = ly + f0y + G;
          double ux_[P + 1], uy_[P + 1];
          unit_weights<P, R>(w0x, ux_);
          unit_weights<P, R>(w0y, uy_);
#pragma unroll
          for (int b = 0; b <= P; ++b)
#pragma unroll
            for (int a = 0; a <= P; ++a)
              atomicAdd(&sJ[(ay0 + b) * PW + ax0 + a], cq * (ux_[a] * uy_[b]));
        }

        if constexpr (MODE == MODE_FUSED || MODE == MODE_PUSH) {
          // ---- gather: NODAL, every component from the charge nodes (staged
          // node averages) with the charge-assignment weights; otherwise each
          // component from its own staggered points
          const int gx0 = lx + f0x + G, gy0 = ly + f0y + G;
          R ex, ey, ez, bx, by, bz;
          if constexpr (NODAL) {
            ex = interp<P, R, F>(sF + 0 * plane, PW, gx0, gy0, w0x, w0y);
            ey = interp<P, R, F>(sF + 1 * plane, PW, gx0, gy0, w0x, w0y);
            ez = interp<P, R, F>(sF + 2 * plane, PW, gx0, gy0, w0x, w0y);
            bx = interp<P, R, F>(sF + 3 * plane, PW, gx0, gy0, w0x, w0y);
            by = interp<P, R, F>(sF + 4 * plane, PW, gx0, gy0, w0x, w0y);
            bz = interp<P, R, F>(sF + 5 * plane, PW, gx0, gy0, w0x, w0y);
          } else {
            R whx[P + 1], why[P + 1];
            const int fhx = bspline_weights<P, R>(fx - R(0.5), whx);
            const int fhy = bspline_weights<P, R>(fy - R(0.5), why);
            const int gxh = lx + fhx + G, gyh = ly + fhy + G;
            ex = interp<P, R, F>(sF + 0 * plane, PW, gxh, gy0, whx, w0y);
            ey = interp<P, R, F>(sF + 1 * plane, PW, gx0, gyh, w0x, why);
            ez = interp<P, R, F>(sF + 2 * plane, PW, gx0, gy0, w0x, w0y);
            bx = interp<P, R, F>(sF + 3 * plane, PW, gx0, gyh, w0x, why);
            by = interp<P, R, F>(sF + 4 * plane, PW, gxh, gy0, whx, w0y);
            bz = interp<P, R, F>(sF + 5 * plane, PW, gxh, gyh, whx, why);
          }
          if constexpr (DIAG)
            wk[s][0] += mass * (sqrt(1.0 + (double)ux * ux + (double)uy * uy +
                                     (double)uz * uz) - 1.0);
          // ---- relativistic Boris push u^{n-1/2} -> u^{n+1/2}
          const R umx = ux + qdt_2m * ex, umy = uy + qdt_2m * ey, umz = uz + qdt_2m * ez;
          R tf;
          if constexpr (std::is_same<R, float>::value)
            tf = qdt_2m * inv_sqrt<R>(R(1) + umx * umx + umy * umy + umz * umz);
          else
            tf = qdt_2m / sqrt(R(1) + umx * umx + umy * umy + umz * umz);
          const R tx_ = tf * bx, ty_ = tf * by, tz_ = tf * bz;
          R sf;
          if constexpr (std::is_same<R, float>::value)
            sf = R(2) * recip<R>(R(1) + tx_ * tx_ + ty_ * ty_ + tz_ * tz_);
          else
            sf = R(2) / (R(1) + tx_ * tx_ + ty_ * ty_ + tz_ * tz_);
          const R sx = sf * tx_, sy = sf * ty_, sz = sf * tz_;
          const R upx = umx + (umy * tz_ - umz * ty_);
          const R upy = umy + (umz * tx_ - umx * tz_);
          const R upz = umz + (umx * ty_ - umy * tx_);
          ux = umx + (upy * sz - upz * sy) + qdt_2m * ex;
          uy = umy + (upz * sx - upx * sz) + qdt_2m * ey;
          uz = umz + (upx * sy - upy * sx) + qdt_2m * ez;
          // ---- move x^n -> x^{n+1}
          const R ig = inv_sqrt<R>(R(1) + ux * ux + uy * uy + uz * uz);
          if constexpr (DIAG)
            wk[s][1] += mass * (sqrt(1.0 + (double)ux * ux + (double)uy * uy +
                                     (double)uz * uz) - 1.0);
          R dx_ = ux * ig * dtdx, dy_ = uy * ig * dtdy;
          dx_ = dx_ > lim ? lim : (dx_ < -lim ? -lim : dx_);
          dy_ = dy_ > lim ? lim : (dy_ < -lim ? -lim : dy_);
          fx1 = fx;
          fy1 = fy;
          dcx = advance(fx1, dx_);
          dcy = advance(fy1, dy_);
        }

        if constexpr (MODE == MODE_PUSH) {
          st.old_cell[s][idx] = cell0;
          st.old_ox[s][idx] = fx;
          st.old_oy[s][idx] = fy;
          const int ix1 = pic_wrap(pic_cell_ix(cell0) + dcx, run.nx);
          const int iy1 = pic_wrap(pic_cell_iy(cell0) + dcy, run.ny);
          st.cell[s][idx] = pic_cell_pack(ix1, iy1);
          st.ox[s][idx] = fx1;
          st.oy[s][idx] = fy1;
          st.ux[s][idx] = ux;
          st.uy[s][idx] = uy;
          st.uz[s][idx] = uz;
        }

        if constexpr (MODE == MODE_FUSED || MODE == MODE_DEPOSIT) {
          // ---- Esirkepov deposit of J^{n+1/2} into the LDS patch
          R w1x[P + 1], w1y[P + 1];
          const int f1x = bspline_weights<P, R>(fx1, w1x);
          const int f1y = bspline_weights<P, R>(fy1, w1y);
          // first support nodes (relative to the old cell) of old and new shapes
          const int n1x = dcx + f1x, n1y = dcy + f1y;
          const int Ax = f0x < n1x ? f0x : n1x, Ay = f0y < n1y ? f0y : n1y;
          const int o0x = f0x - Ax, o1x = n1x - Ax, o0y = f0y - Ay, o1y = n1y - Ay;
          double u0x[P + 1], u1x[P + 1], u0y[P + 1], u1y[P + 1];
          unit_weights<P, R>(w0x, u0x);
          unit_weights<P, R>(w1x, u1x);
          unit_weights<P, R>(w0y, u0y);
          unit_weights<P, R>(w1y, u1y);
          const int ax0 = lx + Ax + G, ay0 = ly + Ay + G;
          R vz;
          if constexpr (std::is_same<R, float>::value)
            vz = uz * inv_sqrt<R>(R(1) + ux * ux + uy * uy + uz * uz);
          else
            vz = uz / sqrt(R(1) + ux * ux + uy * uy + uz * uz);
          double* jx = sJ;
          double* jy = sJ + plane;
          double* jz = sJ + 2 * plane;
          // The sums run in FP64 from the window weights converted once (an
          // FP64 FMA issues at the rate of an FP32 one here) into FP64 LDS
          // accumulators in both forms: measured on gfx950 in this kernel, the
          // native FP32 LDS atomic add (ds_add_f32) takes the 1024 x 256
          // order-3 push from 1.3 ms to 10.3 ms, while ds_add_f64 runs near
          // the LDS bandwidth. Jx(i+1/2) is the running sum of Wx along x (the
          // last node's sum is zero); the constant factors of Jx, Jy, Jz are
          // folded into the per-row and per-column weights. The shapes are
          // the unit-sum FP64 weights the charge density uses (the next
          // step's old shape is this step's new one bit for bit), so the
          // current carries exactly the change of that density and Gauss's
          // law holds to FP64 rounding in the FP32 form too.
          double s0x[W], dsx[W], s0y[W], dsy[W];
#pragma unroll
          for (int a = 0; a < W; ++a) {
            s0x[a] = place<P, double>(u0x, o0x, a);
            dsx[a] = place<P, double>(u1x, o1x, a) - s0x[a];
            s0y[a] = place<P, double>(u0y, o0y, a);
            dsy[a] = place<P, double>(u1y, o1y, a) - s0y[a];
          }
          const double cx = cjx, cy = cjy, cz = cjz * (double)vz;
          // The window's last row (column) holds weights only for a lane
          // whose support moved along y (x) this step; when no lane of the
          // wavefront did, its Jx and Jz row (Jy and Jz column) is exactly
          // zero and the wavefront skips those atomics as a whole.
          const bool row_last = __any(o0y != o1y);
          const bool col_last = __any(o0x != o1x);
          double* const bx_ = jx + ay0 * PW + ax0;
          double* const by_ = jy + ay0 * PW + ax0;
          double* const bz_ = jz + ay0 * PW + ax0;
          auto jx_row = [&](int b) {
            const double wy = (s0y[b] + 0.5 * dsy[b]) * cx;
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < W - 1; ++a) {
              acc += dsx[a] * wy;
              if (acc != 0.0) atomicAdd(&bx_[b * PW + a], acc);
            }
          };
#pragma unroll
          for (int b = 0; b < W - 1; ++b) jx_row(b);
          if (row_last) jx_row(W - 1);
          // Wz = S0x S0y + DSx S0y/2 + S0x DSy/2 + DSx DSy/3, grouped as
          // (S0x + DSx/2) S0y + (S0x/2 + DSx/3) DSy; the first factor is Jy's
          double hy[W], hz[W], zz[W];
#pragma unroll
          for (int a = 0; a < W; ++a) {
            const double hx = s0x[a] + 0.5 * dsx[a];
            hy[a] = hx * cy;
            hz[a] = hx * cz;
            zz[a] = (0.5 * s0x[a] + dsx[a] * (1.0 / 3.0)) * cz;
          }
          auto jy_col = [&](int a) {
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < W - 1; ++b) {
              acc += dsy[b] * hy[a];
              if (acc != 0.0) atomicAdd(&by_[b * PW + a], acc);
            }
          };
#pragma unroll
          for (int a = 0; a < W - 1; ++a) jy_col(a);
          if (col_last) jy_col(W - 1);
          auto jz_at = [&](int a, int b) {
            const double wz = hz[a] * s0y[b] + zz[a] * dsy[b];
            if (wz != 0.0) atomicAdd(&bz_[b * PW + a], wz);
          };
#pragma unroll
          for (int b = 0; b < W - 1; ++b)
#pragma unroll
            for (int a = 0; a < W - 1; ++a) jz_at(a, b);
          if (col_last) {
#pragma unroll
            for (int b = 0; b < W - 1; ++b) jz_at(W - 1, b);
          }
          if (row_last) {
#pragma unroll
            for (int a = 0; a < W - 1; ++a) jz_at(a, W - 1);
            if (col_last) jz_at(W - 1, W - 1);
          }

          // ---- boundaries: a shock run reflects at x = 0 (after the deposit
          // of the unreflected displacement, whose ghost columns the current
          // reduction folds back) and drops particles reaching x_out
          int lx1 = lx + dcx;
          const int ly1 = ly + dcy;
          int ix1;
          if (run.bc == 1) {
            int gx1 = x0 + lx1;
            if (gx1 < 0) {
              R f = R(1) - fx1;
              int c = -gx1 - 1;
              if (f >= R(1)) {
                f -= R(1);
                c += 1;
              }
              gx1 = c;
              fx1 = f;
              ux = -ux;
            }
            gone = gx1 >= run.x_out;
            ix1 = gx1;
            lx1 = gx1 - x0;
          } else {
            ix1 = pic_wrap(x0 + lx1, run.nx);
          }
          // ---- tile membership after the move
          const int iy1 = pic_wrap(y0 + ly1, run.ny);
          gcell = pic_cell_pack(ix1, iy1);
          int dest_t = tile;
          if (lx1 < 0 || lx1 >= tw || ly1 < 0 || ly1 >= th) {
            int ttx = tx + (lx1 < 0 ? -1 : (lx1 >= tw ? 1 : 0));
            int tty = ty + (ly1 < 0 ? -1 : (ly1 >= th ? 1 : 0));
            ttx = ttx < 0 ? run.ntx - 1 : (ttx >= run.ntx ? 0 : ttx);
            tty = tty < 0 ? run.nty - 1 : (tty >= run.nty ? 0 : tty);
            dest_t = run.tile0 + tty * run.ntx + ttx;
          }
          if (dest_t != tile && !gone) {
            leave = true;
            dest = dest_t;
          }
          if (st.id[s]) pid = st.id[s][idx];
        }
      }
      if constexpr (MODE == MODE_FUSED || MODE == MODE_DEPOSIT) {
        // Every particle goes straight to its tile's region of the next
        // buffer: stayers and arrivals from the neighbours take slots from
        // the same per-tile counter (one atomic per wavefront and distinct
        // tile), so no separate exchange buffer and no second copy exist. A
        // tile whose slots run out drops the surplus and flags the run.
        const int cap = st.tile_slots[s];
        const bool stay = active && !leave && !gone;
        const unsigned long long m = __ballot(stay);
        int wbase = 0;
        if (__lane_id() == 0 && m) wbase = atomicAdd(&st.stay_cnt[s][tile], __popcll(m));
        wbase = __shfl(wbase, 0);
        const int lane = __lane_id();
        const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        const int moved = wave_reserve(leave, dest, st.stay_cnt[s]);
        const int slot = stay ? wbase + __popcll(m & below) : moved;
        if (stay || leave) {
          if (slot < cap) {
            const long long o = (long long)(stay ? tile : dest) * cap + slot;
            st.ncell[s][o] = gcell;
            st.nox[s][o] = fx1;
            st.noy[s][o] = fy1;
            st.nux[s][o] = ux;
            st.nuy[s][o] = uy;
            st.nuz[s][o] = uz;
            if (st.nid[s]) st.nid[s][o] = pid;
          } else {
            atomicOr(st.err, PIC_ERRBIT_TILE);
          }
        }
      }
    }
  }
}

// DIAG: the step records the kinetic energies W_K(n -/+ 1/2) (a compile-time
// variant, so that the ordinary step carries no FP64 accumulators)
template <typename R, typename F, int MODE, bool DIAG, bool NODAL>
__global__ void __launch_bounds__(256) k_particles(DevState<R> st, int sel) {
  // XCD-aware order: consecutive (tile, part) items go to the same XCD
  const int per = gridDim.x / 8;
  const int item = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (item >= st.n_tiles * st.K) return;
  const int tile = item / st.K, part = item % st.K;
  const int ri = st.tile_run[tile];
  const DevRun& run = st.runs[ri];
  const int lt = tile - run.tile0;
  const int tx = lt % run.ntx, ty = lt / run.ntx;
  const int x0 = tx * st.TX, y0 = ty * st.TY;
  const int tw = pic_tile_width(tx, st.TX, run.ntx, run.nx);
  const int th = pic_tile_width(ty, st.TY, run.nty, run.ny);
  const int PW = st.PW, PH = st.PH, plane = PW * PH;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  F* sF = reinterpret_cast<F*>(smem_raw);
  const size_t fbytes = (MODE == MODE_FUSED || MODE == MODE_PUSH) ? 6 * plane * sizeof(F) : 0;
  // currents (and rho) accumulate in FP64 LDS in both forms
  double* sJ = reinterpret_cast<double*>(smem_raw + fbytes);
  const int nj = (MODE == MODE_PUSH) ? 0 : (MODE == MODE_CHARGE ? 1 : 3);
  __shared__ double s_red[4][PIC_MAXS * 2];

  if constexpr (MODE == MODE_FUSED || MODE == MODE_PUSH) {
    // Yee value of component c at column gx, row gy: periodic wrap, or behind
    // a shock run's wall at x = 0 the conductor images (integer-x components
    // Ey, Ez, Bx odd, half-integer ones Ex, By, Bz even); columns at or beyond
    // the far wall's outside column hold zero
    auto yee = [&](int c, int gx, int gy) -> F {
      const bool half = c == 0 || c >= 4;
      int col = pic_wrap(gx, run.nx);
      F sign = F(1);
      if (run.bc == 1) {
        if (gx < 0) {
          col = half ? -gx - 1 : -gx;
          if (!half) sign = F(-1);
        } else if (gx >= run.nx) {
          return F(0);
        }
      }
      const long long g = run.cell0 + (long long)pic_wrap(gy, run.ny) * run.nx + col;
      F v;
      if constexpr (sizeof(F) == 4)
        v = st.Ef[c][g];
      else
        v = (c < 3) ? st.E[c][g] : st.B[c - 3][g];
      return sign * v;
    };
    for (int e = threadIdx.x; e < plane; e += blockDim.x) {
      const int ly = e / PW - G, lx = e % PW - G;
      const bool in = lx <= tw + PIC_GUARD_HI - 1 && ly <= th + PIC_GUARD_HI - 1;
      const int gx = x0 + lx, gy = y0 + ly;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        F v = F(0);
        if (in) {
          if constexpr (NODAL) {
            // momentum-conserving interpolation: the component averaged from
            // its Yee points onto the charge node (gx, gy)
            if (c == 0 || c == 4)
              v = F(0.5) * (yee(c, gx - 1, gy) + yee(c, gx, gy));
            else if (c == 1 || c == 3)
              v = F(0.5) * (yee(c, gx, gy - 1) + yee(c, gx, gy));
            else if (c == 2)
              v = yee(c, gx, gy);
            else
              v = F(0.25) * (yee(c, gx - 1, gy - 1) + yee(c, gx, gy - 1) + yee(c, gx - 1, gy) +
                             yee(c, gx, gy));
          } else {
            v = yee(c, gx, gy);
          }
        }
        sF[c * plane + e] = v;
      }
    }
  }
  for (int e = threadIdx.x; e < nj * plane; e += blockDim.x) sJ[e] = 0.0;
  __syncthreads();

  double wk[PIC_MAXS][2] = {{0.0, 0.0}, {0.0, 0.0}};
  switch (run.order) {
    case 1:
      tile_body<R, F, 1, MODE, DIAG, NODAL>(st, run, tile, tx, ty, x0, y0, tw, th, sF, sJ, part, sel, wk);
      break;
    case 2:
      tile_body<R, F, 2, MODE, DIAG, NODAL>(st, run, tile, tx, ty, x0, y0, tw, th, sF, sJ, part, sel, wk);
      break;
    default:
      tile_body<R, F, 3, MODE, DIAG, NODAL>(st, run, tile, tx, ty, x0, y0, tw, th, sF, sJ, part, sel, wk);
      break;
  }
  __syncthreads();

  if constexpr (MODE != MODE_PUSH) {
    for (int c = 0; c < nj; ++c) {
      double* out = st.patch[c] + (size_t)item * plane;
      for (int e = threadIdx.x; e < plane; e += blockDim.x) out[e] = sJ[c * plane + e];
    }
  }
  if constexpr ((MODE == MODE_FUSED || MODE == MODE_PUSH) && DIAG) {
    {
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
      for (int s = 0; s < PIC_MAXS; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          double v = wk[s][h];
          for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
          if (lane == 0) s_red[wave][s * 2 + h] = v;
        }
      __syncthreads();
      if (threadIdx.x < PIC_MAXS * 2) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += s_red[w][threadIdx.x];
        st.wk_part[(size_t)item * PIC_MAXS * 2 + threadIdx.x] = v;
      }
    }
  }
}

// Re-binning: the particle kernel has already written every particle into its
// tile's region of the next buffer; the tile's new count is what its counter
// handed out (at most the tile's slots), and the counter is cleared for the
// next pass.
template <typename R>
__global__ void __launch_bounds__(256) k_rebin(DevState<R> st) {
  const int tile = blockIdx.x * blockDim.x + threadIdx.x;
  if (tile >= st.n_tiles) return;
  const int s = blockIdx.y;
  if (s >= st.runs[st.tile_run[tile]].nspecies) return;
  const int cap = st.tile_slots[s];
  int n = st.stay_cnt[s][tile];
  if (n > cap) {
    atomicOr(st.err, PIC_ERRBIT_TILE);
    n = cap;   // the surplus was dropped; the run is flagged
  }
  st.cnt[s][tile] = n;
  st.stay_cnt[s][tile] = 0;
}

// Reordering of a tile's particles (every sort_every steps, after the
// re-binning): the compaction of stayers mixes the storage order over the
// steps, so that the 64 lanes of a wavefront land on random cells of the tile
// and the particle kernel's LDS atomics and gathers collide in banks more and
// more. A counting sort by cell gives each particle a position p in
// cell-major order; lane l of every wavefront then takes the l-th contiguous
// 1/64 of that order (run length L or L - 1), so one wavefront covers 64
// distinct cells spread over the tile: storage q = w * 64 + l for the w-th
// particle of lane l's run. The current store is read, the next one written
// in storage order (the reads gather through the inverse permutation).
constexpr int kSortBatch = 8;
// dynamic LDS of the staged reordering, leaving room for the static words
// within the 64 KB a work-group may hold
constexpr size_t kSortStageBytes = 63 * 1024;
constexpr long long kSortMaxPasses = 4;   // staging passes per array at most
// one work-group per (tile, species); the staging LDS (up to 63 KB) admits two
// work-groups per CU, so 16 wavefronts each fill the CU's wavefront slots
// (0.36 ms per launch at 1024 x 256 against 0.41 with 512 threads and 0.60
// with 256)
constexpr int kSortThreads = 1024;

// Staged form: with max_slots (the largest tile's slots) small enough, the
// permutation (16 bit) lives in LDS and each array's tile region is staged
// there too, `chunk` elements at a time (one pass per chunk writes the
// destinations whose source lies in it), so the gathers read LDS and every
// global access is contiguous.
template <typename R>
__global__ void __launch_bounds__(kSortThreads) k_sort(DevState<R> st, int max_cells, int max_slots,
                                              int staged, int chunk) {
  // dynamic LDS: [max_cells] counts then cursors; staged: [max_slots] u16
  // permutation, then [max_slots] elements of the array being moved
  extern __shared__ __align__(16) int s_cell[];
  __shared__ int s_carry;
  const int per = gridDim.x / 8;
  const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= st.n_tiles) return;
  const int s = blockIdx.y;
  const DevRun& run = st.runs[st.tile_run[tile]];
  if (s >= run.nspecies) return;
  const int lt = tile - run.tile0;
  const int tx = lt % run.ntx, ty = lt / run.ntx;
  const int x0 = tx * st.TX, y0 = ty * st.TY;
  const int tw = pic_tile_width(tx, st.TX, run.ntx, run.nx);
  const int th = pic_tile_width(ty, st.TY, run.nty, run.ny);
  const int nc = tw * th;
  const int n = st.cnt[s][tile];
  const long long base = (long long)tile * st.tile_slots[s];
  __shared__ int s_bad;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) s_cell[c] = 0;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  // kSortBatch loads in flight per thread before their LDS updates
  const int stride = (int)blockDim.x * kSortBatch;
  for (int k0 = threadIdx.x; k0 < n; k0 += stride) {
    int cell[kSortBatch];
#pragma unroll
    for (int u = 0; u < kSortBatch; ++u) {
      const int k = k0 + u * (int)blockDim.x;
      cell[u] = k < n ? st.cell[s][base + k] : -1;
    }
#pragma unroll
    for (int u = 0; u < kSortBatch; ++u) {
      if (cell[u] < 0) continue;
      const int lx = pic_cell_ix(cell[u]) - x0, ly = pic_cell_iy(cell[u]) - y0;
      if (lx < 0 || lx >= tw || ly < 0 || ly >= th)
        s_bad = 1;   // not in this tile: the store is inconsistent
      else
        atomicAdd(&s_cell[ly * tw + lx], 1);
    }
  }
  __syncthreads();
  if (s_bad) {
    // keep the order (copy) and flag the run
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const long long i = base + k;
      st.ncell[s][i] = st.cell[s][i];
      st.nox[s][i] = st.ox[s][i];
      st.noy[s][i] = st.oy[s][i];
      st.nux[s][i] = st.ux[s][i];
      st.nuy[s][i] = st.uy[s][i];
      st.nuz[s][i] = st.uz[s][i];
      if (st.id[s]) st.nid[s][i] = st.id[s][i];
    }
    if (threadIdx.x == 0) atomicOr(st.err, PIC_ERRBIT_TILE);
    return;
  }
  // exclusive scan of the counts, blockDim cells at a time: a shuffle scan
  // per wavefront, the wavefront totals, and a carry over the chunks
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nc; c0 += blockDim.x) {
    const int c = c0 + threadIdx.x;
    const int v = c < nc ? s_cell[c] : 0;
    // inclusive scan within the wavefront
    int x = v;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    __shared__ int s_wave[kSortThreads / 64];
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int before = s_carry;
    for (int w = 0; w < wave; ++w) before += s_wave[w];
    if (c < nc) s_cell[c] = before + x - v;   // exclusive start = cursor
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) s_carry = before + x;
    __syncthreads();
  }
  // the source of every destination, in the split path's old-cell array
  // (free during pic_step): cell-sorted position p is the w-th particle of
  // lane l's run (runs of L or L - 1, the longer first), destination 64 w + l
  const int L = (n + 63) / 64;
  const int full = n - 64 * (L - 1);   // lanes whose run has L particles
  int* const inv = st.old_cell[s] + base;
  // region offsets rounded to 16 bytes (the staged elements may be FP64)
  unsigned char* const lds = reinterpret_cast<unsigned char*>(s_cell);
  unsigned short* const inv16 =
      reinterpret_cast<unsigned short*>(lds + (((size_t)max_cells * 4 + 15) & ~(size_t)15));
  unsigned char* const stage = reinterpret_cast<unsigned char*>(inv16) +
                               (((size_t)max_slots * 2 + 15) & ~(size_t)15);
  for (int k0 = threadIdx.x; k0 < n; k0 += stride) {
    int cell[kSortBatch];
#pragma unroll
    for (int u = 0; u < kSortBatch; ++u) {
      const int k = k0 + u * (int)blockDim.x;
      cell[u] = k < n ? st.cell[s][base + k] : -1;
    }
#pragma unroll
    for (int u = 0; u < kSortBatch; ++u) {
      if (cell[u] < 0) continue;
      const int c = (pic_cell_iy(cell[u]) - y0) * tw + pic_cell_ix(cell[u]) - x0;
      const int p = atomicAdd(&s_cell[c], 1);
      int l, w;
      if (p < full * L) {
        l = p / L;
        w = p - l * L;
      } else {
        const int p2 = p - full * L;   // here L >= 2, since p < n
        l = full + p2 / (L - 1);
        w = p2 - (l - full) * (L - 1);
      }
      if (staged)
        inv16[w * 64 + l] = (unsigned short)(k0 + u * (int)blockDim.x);
      else
        inv[w * 64 + l] = k0 + u * (int)blockDim.x;
    }
  }
  __syncthreads();
  if (staged) {
    // one array at a time: contiguous load of the tile region into LDS, then
    // contiguous stores of the permuted elements
    auto move_lds = [&](auto* dst, const auto* srcp) {
      using T = typename std::remove_const<typename std::remove_pointer<decltype(srcp)>::type>::type;
      T* const buf = reinterpret_cast<T*>(stage);
      for (int c0 = 0; c0 < n; c0 += chunk) {
        const int cn = n - c0 < chunk ? n - c0 : chunk;
        for (int k0 = threadIdx.x; k0 < cn; k0 += stride) {
          T v[kSortBatch];
#pragma unroll
          for (int u = 0; u < kSortBatch; ++u) {
            const int k = k0 + u * (int)blockDim.x;
            if (k < cn) v[u] = srcp[base + c0 + k];
          }
#pragma unroll
          for (int u = 0; u < kSortBatch; ++u) {
            const int k = k0 + u * (int)blockDim.x;
            if (k < cn) buf[k] = v[u];
          }
        }
        __syncthreads();
        if (cn == n) {
          for (int q = threadIdx.x; q < n; q += blockDim.x) dst[base + q] = buf[inv16[q]];
        } else {
          for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int k = (int)inv16[q] - c0;
            if (k >= 0 && k < cn) dst[base + q] = buf[k];
          }
        }
        __syncthreads();
      }
    };
    move_lds(st.ncell[s], st.cell[s]);
    move_lds(st.nox[s], st.ox[s]);
    move_lds(st.noy[s], st.oy[s]);
    move_lds(st.nux[s], st.ux[s]);
    move_lds(st.nuy[s], st.uy[s]);
    move_lds(st.nuz[s], st.uz[s]);
    if (st.id[s]) move_lds(st.nid[s], st.id[s]);
    return;
  }
  // destination order, one array at a time (the gathers of a work-group then
  // stay within one array's region of the tile): contiguous stores
  auto move = [&](auto* dst, const auto* srcp) {
    for (int q0 = threadIdx.x; q0 < n; q0 += (int)blockDim.x * kSortBatch) {
      int from[kSortBatch];
#pragma unroll
      for (int u = 0; u < kSortBatch; ++u) {
        const int q = q0 + u * (int)blockDim.x;
        from[u] = q < n ? inv[q] : -1;
      }
#pragma unroll
      for (int u = 0; u < kSortBatch; ++u)
        if (from[u] >= 0) dst[base + q0 + u * (int)blockDim.x] = srcp[base + from[u]];
    }
  };
  move(st.ncell[s], st.cell[s]);
  move(st.nox[s], st.ox[s]);
  move(st.noy[s], st.oy[s]);
  move(st.nux[s], st.ux[s]);
  move(st.nuy[s], st.uy[s]);
  move(st.nuz[s], st.uz[s]);
  if (st.id[s]) move(st.nid[s], st.id[s]);
}

// Injection: staged particles (sorted by tile) are appended to the current
// store of their tile; entry e of the list is (tile, first staged index,
// count) and each tile appears once, so one work-group owns a tile's count.
template <typename R>
__global__ void __launch_bounds__(256) k_inject(DevState<R> st, int s, const int* list,
                                                const int* cell, const R* ox, const R* oy,
                                                const R* ux, const R* uy, const R* uz,
                                                const int* id) {
  const int t = list[3 * blockIdx.x], o = list[3 * blockIdx.x + 1];
  int k = list[3 * blockIdx.x + 2];
  const int cap = st.tile_slots[s];
  const int n0 = st.cnt[s][t];
  if (n0 + k > cap) {
    if (threadIdx.x == 0) atomicOr(st.err, PIC_ERRBIT_TILE);
    k = cap - n0;
  }
  const long long base = (long long)t * cap + n0;
  for (int e = threadIdx.x; e < k; e += blockDim.x) {
    st.cell[s][base + e] = cell[o + e];
    st.ox[s][base + e] = ox[o + e];
    st.oy[s][base + e] = oy[o + e];
    st.ux[s][base + e] = ux[o + e];
    st.uy[s][base + e] = uy[o + e];
    st.uz[s][base + e] = uz[o + e];
    if (st.id[s]) st.id[s][base + e] = id[o + e];
  }
  __syncthreads();
  if (threadIdx.x == 0) st.cnt[s][t] = n0 + k;
}

// Sum of the overlapping tile patches at every node, in a fixed tile order.
template <typename R>
__global__ void __launch_bounds__(256) k_current_sum(DevState<R> st, int ncomp, double* out0,
                                                     int only_run) {
  const int ri = only_run >= 0 ? only_run : blockIdx.y;
  const DevRun& run = st.runs[ri];
  const long long ncell = (long long)run.nx * run.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncell) return;
  const int i = (int)(k % run.nx), j = (int)(k / run.nx);
  const int TX = st.TX, TY = st.TY, PW = st.PW, plane = PW * st.PH;
  const int tx = pic_tile_of(i, TX, run.ntx), ty = pic_tile_of(j, TY, run.nty);
  const bool shock = run.bc == 1;
  double acc[3] = {0.0, 0.0, 0.0};
  // a patch reaches PIC_GUARD_LO nodes below its tile and PIC_GUARD_HI - 1
  // above it, so tiles narrower than the guard have patches reaching past
  // their neighbours: look as many tiles out as the guard spans
  constexpr int GMAX = G > PIC_GUARD_HI ? G : PIC_GUARD_HI;
  const int RX = (GMAX + TX - 1) / TX, RY = (GMAX + TY - 1) / TY;
  for (int dy = -RY; dy <= RY; ++dy) {
    // tile row ty + dy, wrapped periodically: origin t_y TY + my ny
    int t_y = ty + dy, my = 0;
    while (t_y < 0) { t_y += run.nty; --my; }
    while (t_y >= run.nty) { t_y -= run.nty; ++my; }
    const int oy = t_y * TY + my * run.ny;
    const int hy = pic_tile_width(t_y, TY, run.nty, run.ny);
    const int ly = j - oy;
    if (ly < -G || ly > hy + PIC_GUARD_HI - 1) continue;
    for (int dx = -RX; dx <= RX; ++dx) {
      int t_x = tx + dx, mx = 0;
      while (t_x < 0) { t_x += run.ntx; --mx; }
      while (t_x >= run.ntx) { t_x -= run.ntx; ++mx; }
      if (shock && mx != 0) continue;
      const int ox = t_x * TX + mx * run.nx;
      const int hx = pic_tile_width(t_x, TX, run.ntx, run.nx);
      const int lx = i - ox;
      if (lx < -G || lx > hx + PIC_GUARD_HI - 1) continue;
      const size_t t = (size_t)(run.tile0 + t_y * run.ntx + t_x);
      const size_t in_patch = (size_t)(ly + G) * PW + (lx + G);
      for (int pk = 0; pk < st.K; ++pk) {
        const size_t off = (t * st.K + pk) * plane + in_patch;
        for (int c = 0; c < ncomp; ++c) acc[c] += st.patch[c][off];
      }
    }
    if (shock) {
      // fold of the ghost columns of the wall tiles (x0 = 0): column -i of
      // rho, Jy, Jz adds with its sign; Jx(-i-1/2) adds negated to Jx(i+1/2)
      const size_t t = (size_t)(run.tile0 + t_y * run.ntx);
      for (int c = 0; c < ncomp; ++c) {
        const bool jx = out0 == nullptr && c == 0;
        const int lxg = jx ? -i - 1 : -i;
        if (lxg < -G || lxg >= 0) continue;
        const size_t in_patch = (size_t)(ly + G) * PW + (lxg + G);
        double f = 0.0;
        for (int pk = 0; pk < st.K; ++pk) f += st.patch[c][(t * st.K + pk) * plane + in_patch];
        acc[c] += jx ? -f : f;
      }
    }
  }
  const long long g = run.cell0 + k;
  if (out0) {
    out0[k] = acc[0];
  } else {
    if (shock) {
      // currents on the conductors drive no field
      if (i == run.nx - 1) acc[0] = 0.0;
      if (i == 0 || i == run.nx - 1) acc[1] = acc[2] = 0.0;
    }
    for (int c = 0; c < ncomp; ++c) st.J[c][g] = acc[c];
  }
}

// Diagnostics of the current state of one run, per work-group: max Gauss
// residual |div E - 4 pi rho| at the nodes, max |div B| at the cell centres,
// sum of rho (fixed reduction tree) and the number of non-finite E or B
// values (any of the six components)
__global__ void __launch_bounds__(256)
k_divergences(const DevRun* runs, int ri, const double* ex, const double* ey, const double* ez,
              const double* bx, const double* by, const double* bz, const double* rho,
              double* part) {
  const DevRun& run = runs[ri];
  const long long ncell = (long long)run.nx * run.ny;
  double g = 0.0, d = 0.0, q = 0.0, bad = 0.0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < ncell;
       k += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(k % run.nx), j = (int)(k / run.nx);
    const long long c0 = run.cell0;
    const long long kk = c0 + k;
    const long long xm = c0 + (long long)j * run.nx + pic_wrap(i - 1, run.nx);
    const long long ym = c0 + (long long)pic_wrap(j - 1, run.ny) * run.nx + i;
    const long long xp = c0 + (long long)j * run.nx + pic_wrap(i + 1, run.nx);
    const long long yp = c0 + (long long)pic_wrap(j + 1, run.ny) * run.nx + i;
    const double dive = (ex[kk] - ex[xm]) / run.dx + (ey[kk] - ey[ym]) / run.dy;
    double gr = fabs(dive - kFourPi * rho[k]);
    // shock runs: the wall line carries the conductor's surface charge and
    // particles leave near x_out, so Gauss's law is checked in between
    if (run.bc == 1 && (i < 1 || i > run.x_out - 4)) gr = 0.0;
    const double divb = fabs((bx[xp] - bx[kk]) / run.dx + (by[yp] - by[kk]) / run.dy);
    g = (gr > g || gr != gr) ? gr : g;
    d = (divb > d || divb != divb) ? divb : d;
    q += rho[k];
    const double f6[6] = {ex[kk], ey[kk], ez[kk], bx[kk], by[kk], bz[kk]};
#pragma unroll
    for (int c = 0; c < 6; ++c) bad += isfinite(f6[c]) ? 0.0 : 1.0;
  }
  __shared__ double sg[256], sd[256], sq[256], sb[256];
  sg[threadIdx.x] = g;
  sd[threadIdx.x] = d;
  sq[threadIdx.x] = q;
  sb[threadIdx.x] = bad;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const double a = sg[threadIdx.x + off], b = sd[threadIdx.x + off];
      if (a > sg[threadIdx.x] || a != a) sg[threadIdx.x] = a;
      if (b > sd[threadIdx.x] || b != b) sd[threadIdx.x] = b;
      sq[threadIdx.x] += sq[threadIdx.x + off];
      sb[threadIdx.x] += sb[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4 + 0] = sg[0];
    part[blockIdx.x * 4 + 1] = sd[0];
    part[blockIdx.x * 4 + 2] = sq[0];
    part[blockIdx.x * 4 + 3] = sb[0];
  }
}

inline int grid_tiles(int n_tiles) { return ((n_tiles + 7) / 8) * 8; }

}  // namespace

template <typename R>
size_t pic_particle_smem(const DevState<R>& st, int mode) {
  using F = typename std::conditional<sizeof(R) == 4, float, double>::type;
  const size_t plane = (size_t)st.PW * st.PH;
  size_t b = 0;
  if (mode == MODE_FUSED || mode == MODE_PUSH) b += 6 * plane * sizeof(F);
  if (mode == MODE_FUSED || mode == MODE_DEPOSIT) b += 3 * plane * sizeof(double);
  if (mode == MODE_CHARGE) b += plane * sizeof(double);
  return b;
}

template <typename R>
hipError_t pic_launch_particles(const DevState<R>& st, int mode, int diag, int threads,
                                hipStream_t s) {
  using F = typename std::conditional<sizeof(R) == 4, float, double>::type;
  const size_t smem = pic_particle_smem(st, mode);
  const dim3 grid(grid_tiles(st.n_tiles * st.K)), block(threads);
  // the gather variant (node-averaged or staggered) is a compile-time choice
  // of the gathering modes
  auto gathering = [&](auto mode_c, auto diag_c) {
    constexpr int M = decltype(mode_c)::value;
    constexpr bool D = decltype(diag_c)::value;
    if (st.nodal)
      k_particles<R, F, M, D, true><<<grid, block, smem, s>>>(st, -1);
    else
      k_particles<R, F, M, D, false><<<grid, block, smem, s>>>(st, -1);
  };
  using std::integral_constant;
  switch (mode) {
    case MODE_FUSED:
      if (diag)
        gathering(integral_constant<int, MODE_FUSED>{}, integral_constant<bool, true>{});
      else
        gathering(integral_constant<int, MODE_FUSED>{}, integral_constant<bool, false>{});
      break;
    case MODE_PUSH:
      if (diag)
        gathering(integral_constant<int, MODE_PUSH>{}, integral_constant<bool, true>{});
      else
        gathering(integral_constant<int, MODE_PUSH>{}, integral_constant<bool, false>{});
      break;
    case MODE_DEPOSIT:
      k_particles<R, F, MODE_DEPOSIT, false, false><<<grid, block, smem, s>>>(st, -1);
      break;
    default:
      k_particles<R, F, MODE_CHARGE, false, false><<<grid, block, smem, s>>>(st, -1);
      break;
  }
  return hipGetLastError();
}

template <typename R>
hipError_t pic_launch_density(const DevState<R>& st, int species, int threads, hipStream_t s) {
  using F = typename std::conditional<sizeof(R) == 4, float, double>::type;
  const size_t smem = pic_particle_smem(st, MODE_CHARGE);
  const dim3 grid(grid_tiles(st.n_tiles * st.K)), block(threads);
  k_particles<R, F, MODE_CHARGE, false, false><<<grid, block, smem, s>>>(st, species);
  return hipGetLastError();
}

// Transverse average of one run's [ny][nx] field: profile(i) = mean_j f(i, j)
__global__ void __launch_bounds__(256) k_transverse_mean(const double* f, int nx, int ny,
                                                         double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx) return;
  double s = 0.0;
  for (int j = 0; j < ny; ++j) s += f[(long long)j * nx + i];
  out[i] = s / ny;
}

hipError_t pic_launch_transverse_mean(const double* f, int nx, int ny, double* out,
                                      hipStream_t s) {
  k_transverse_mean<<<(nx + 255) / 256, 256, 0, s>>>(f, nx, ny, out);
  return hipGetLastError();
}

template <typename R>
hipError_t pic_launch_sort(const DevState<R>& st, int n_species, int max_tile_cells,
                           hipStream_t s) {
  int max_slots = 0;
  for (int k = 0; k < n_species; ++k) max_slots = st.tile_slots[k] > max_slots ? st.tile_slots[k] : max_slots;
  const size_t cells_b = (size_t)max_tile_cells * sizeof(int);
  const size_t fixed_b = ((cells_b + 15) & ~(size_t)15) + (((size_t)max_slots * 2 + 15) & ~(size_t)15);
  const size_t elem = sizeof(R) > sizeof(int) ? sizeof(R) : sizeof(int);
  // staging chunk: what the remaining LDS holds, in whole 256-element blocks;
  // staged when the permutation is 16-bit and at most kSortMaxPasses passes
  // cover the largest tile
  long long chunk = fixed_b < kSortStageBytes ? (long long)((kSortStageBytes - fixed_b) / elem) : 0;
  chunk = chunk / 256 * 256;
  if (chunk > max_slots) chunk = max_slots;
  const int staged = max_slots <= 65535 && chunk >= 256 &&
                     chunk * kSortMaxPasses >= max_slots ? 1 : 0;
  const size_t smem = staged ? fixed_b + (size_t)chunk * elem : cells_b;
  k_sort<R><<<dim3(grid_tiles(st.n_tiles), n_species), dim3(kSortThreads), smem, s>>>(
      st, max_tile_cells, max_slots, staged, staged ? (int)chunk : 0);
  return hipGetLastError();
}

template <typename R>
hipError_t pic_launch_rebin(const DevState<R>& st, int n_species, hipStream_t s) {
  k_rebin<R><<<dim3((st.n_tiles + 255) / 256, n_species), dim3(256), 0, s>>>(st);
  return hipGetLastError();
}

template <typename R>
hipError_t pic_launch_inject(const DevState<R>& st, int s, int n_entries, const int* list,
                             const int* cell, const R* ox, const R* oy, const R* ux, const R* uy,
                             const R* uz, const int* id, hipStream_t stream) {
  if (n_entries <= 0) return hipSuccess;
  k_inject<R><<<n_entries, 256, 0, stream>>>(st, s, list, cell, ox, oy, ux, uy, uz, id);
  return hipGetLastError();
}

template <typename R>
hipError_t pic_launch_current_sum(const DevState<R>& st, long long max_cells, hipStream_t s) {
  const dim3 grid((unsigned)((max_cells + 255) / 256), st.n_runs);
  k_current_sum<R><<<grid, dim3(256), 0, s>>>(st, 3, nullptr, -1);
  return hipGetLastError();
}

template <typename R>
hipError_t pic_launch_charge_sum(const DevState<R>& st, int run, long long ncell, double* rho,
                                 hipStream_t s) {
  k_current_sum<R><<<dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s>>>(st, 1, rho, run);
  return hipGetLastError();
}

hipError_t pic_launch_divergences(const DevRun* runs, int run, long long ncell,
                                  const double* const* E, const double* const* B,
                                  const double* rho, double* partial_max, int n_blocks,
                                  hipStream_t s) {
  k_divergences<<<dim3(n_blocks), dim3(256), 0, s>>>(runs, run, E[0], E[1], E[2], B[0], B[1],
                                                     B[2], rho, partial_max);
  return hipGetLastError();
}

template size_t pic_particle_smem<float>(const DevState<float>&, int);
template size_t pic_particle_smem<double>(const DevState<double>&, int);
template hipError_t pic_launch_particles<float>(const DevState<float>&, int, int, int, hipStream_t);
template hipError_t pic_launch_particles<double>(const DevState<double>&, int, int, int, hipStream_t);
template hipError_t pic_launch_density<float>(const DevState<float>&, int, int, hipStream_t);
template hipError_t pic_launch_density<double>(const DevState<double>&, int, int, hipStream_t);
template hipError_t pic_launch_rebin<float>(const DevState<float>&, int, hipStream_t);
template hipError_t pic_launch_sort<float>(const DevState<float>&, int, int, hipStream_t);
template hipError_t pic_launch_sort<double>(const DevState<double>&, int, int, hipStream_t);
template hipError_t pic_launch_rebin<double>(const DevState<double>&, int, hipStream_t);
template hipError_t pic_launch_inject<float>(const DevState<float>&, int, int, const int*,
                                             const int*, const float*, const float*,
                                             const float*, const float*, const float*,
                                             const int*, hipStream_t);
template hipError_t pic_launch_inject<double>(const DevState<double>&, int, int, const int*,
                                              const int*, const double*, const double*,
                                              const double*, const double*, const double*,
                                              const int*, hipStream_t);
template hipError_t pic_launch_current_sum<float>(const DevState<float>&, long long, hipStream_t);
template hipError_t pic_launch_current_sum<double>(const DevState<double>&, long long, hipStream_t);
template hipError_t pic_launch_charge_sum<float>(const DevState<float>&, int, long long, double*, hipStream_t);
template hipError_t pic_launch_charge_sum<double>(const DevState<double>&, int, long long, double*, hipStream_t);
