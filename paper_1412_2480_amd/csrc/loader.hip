// Device-side plasma loader: the seeded synthetic load (positions stratified
// ppc per cell, momenta drifting Maxwell-Juettner) generated on the GPU and
// written straight into the tile store, for loads too large to build on the
// host. Not part of the method: it produces the same inputs as the seeded
// host generator, item by item.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): a
// 4 x 32-bit counter block mixed by ten rounds, each multiplying two words by
// fixed 32-bit constants and mixing the high and low product halves with the
// other words and the key, the key bumped by two Weyl constants per round.
// Key = (seed low word, seed high word xor tag * 0x85EBCA6B); counter =
// (item low, item high, draw block, 0); one block gives two doubles in (0, 1)
// from 53 bits each (27 + 26 bits of two words, plus half an ulp).
//
// Momenta: the rest-frame speed by exact rejection from a two-piece envelope
// (a chi-3 below u_c, a three-term Gamma mixture above; constants computed on
// the host), an isotropic direction, then the flipping method of Zenitani
// (2015) and a Lorentz boost along x. Item k sits in cell k / ppc (row-major
// over the loaded columns), rank k % ppc.
#include <math.h>

#include "pic_dev.h"
#include "pic_launch.h"

namespace {

__device__ __forceinline__ void philox_round(unsigned (&c)[4], unsigned k0, unsigned k1) {
  const unsigned long long p0 = 0xD2511F53ull * c[0];
  const unsigned long long p1 = 0xCD9E8D57ull * c[2];
  const unsigned n0 = (unsigned)(p1 >> 32) ^ c[1] ^ k0;
  const unsigned n1 = (unsigned)p1;
  const unsigned n2 = (unsigned)(p0 >> 32) ^ c[3] ^ k1;
  const unsigned n3 = (unsigned)p0;
  c[0] = n0;
  c[1] = n1;
  c[2] = n2;
  c[3] = n3;
}

struct Stream {
  unsigned k0, k1;
  __device__ Stream(unsigned long long seed, unsigned tag) {
    k0 = (unsigned)(seed & 0xFFFFFFFFull);
    k1 = (unsigned)(seed >> 32) ^ (unsigned)(tag * 0x85EBCA6Bu);
  }
  // two uniforms in (0, 1) for (item, block)
  __device__ void u01(long long item, unsigned block, double& a, double& b) const {
    unsigned c[4] = {(unsigned)(item & 0xFFFFFFFFll), (unsigned)((unsigned long long)item >> 32),
                     block, 0u};
    unsigned x0 = k0, x1 = k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
      if (r > 0) {
        x0 += 0x9E3779B9u;
        x1 += 0xBB67AE85u;
      }
      philox_round(c, x0, x1);
    }
    const unsigned long long ia = ((unsigned long long)(c[0] >> 5) << 26) | (c[1] >> 6);
    const unsigned long long ib = ((unsigned long long)(c[2] >> 5) << 26) | (c[3] >> 6);
    const double scale = 1.0 / 9007199254740992.0;
    a = ((double)ia + 0.5) * scale;
    b = ((double)ib + 0.5) * scale;
  }
};

constexpr unsigned kTagPos = 1, kTagMom = 2;
constexpr double kTwoPi = 6.283185307179586;   // 2 * 3.141592653589793 rounded to double

// rest-frame momentum magnitude of item k (attempts use blocks 2 + 3a .. 4 + 3a)
__device__ double mj_speed(const Stream& st, long long k, const PlasmaLoad& L) {
#pragma clang fp contract(off)
  for (int attempt = 0; attempt <= 200; ++attempt) {
    const unsigned blk = 2u + 3u * (unsigned)attempt;
    double a0, a1, b0, b1, c0, c1;
    st.u01(k, blk, a0, a1);
    st.u01(k, blk + 1, b0, b1);
    st.u01(k, blk + 2, c0, c1);
    const bool pa = a0 < L.pa;
    const double la1 = log(a1);
    if (pa) {
      const double r1 = sqrt(-2.0 * log(b0));
      const double n1 = r1 * cos(kTwoPi * b1);
      const double n2 = r1 * sin(kTwoPi * b1);
      const double n3 = sqrt(-2.0 * log(c0)) * cos(kTwoPi * c1);
      const double ua = L.s * sqrt(n1 * n1 + n2 * n2 + n3 * n3);
      const double ga = sqrt(1.0 + ua * ua);
      const double loga = -(ga - 1.0) / L.T + ua * ua / ((1.0 + L.gc) * L.T);
      if (ua <= L.uc && la1 <= loga) return ua;
    } else {
      const double e1 = -log(b1), e2 = -log(c0), e3 = -log(c1);
      const int kk = b0 < L.mix0 ? 1 : (b0 < L.mix1 ? 2 : 3);
      const double w = (e1 + (kk >= 2 ? e2 : 0.0) + (kk >= 3 ? e3 : 0.0)) / L.lam;
      const double ub = L.uc + w;
      const double gb = sqrt(1.0 + ub * ub);
      const double logb = -(gb - L.gc - L.vc * w) / L.T;
      if (la1 <= logb) return ub;
    }
  }
  return 0.0;   // not reached in practice (acceptance is about one half per attempt)
}

// lab-frame momentum of item k: rest-frame magnitude (blocks 2, ...), an
// isotropic direction (block 0), the flip decision (block 1) and the boost
// along x with velocity L.beta (Zenitani's flipping method)
__device__ void draw_momentum(const Stream& mom, long long k, const PlasmaLoad& L, double& ux,
                              double& uy, double& uz) {
#pragma clang fp contract(off)
  const double umag = L.T > 0.0 ? mj_speed(mom, k, L) : 0.0;
  double d0, d1, f0, unused;
  mom.u01(k, 0, d0, d1);
  mom.u01(k, 1, f0, unused);
  const double mu = 2.0 * d0 - 1.0;
  const double phi = kTwoPi * d1;
  const double stt = sqrt(fmax(0.0, 1.0 - mu * mu));
  ux = umag * mu;
  uy = umag * stt * cos(phi);
  uz = umag * stt * sin(phi);
  if (L.gamma0 > 1.0) {
    const double gp = sqrt(1.0 + umag * umag);
    const double vx = ux / gp;
    if (-L.beta * vx > f0) ux = -ux;
    ux = L.gamma0 * (ux + L.beta * gp);
  }
}

template <typename R>
__device__ __forceinline__ R offset_below_one(double f) {
  const R r = (R)f;
  return r < R(1) ? r : R(1) - R(sizeof(R) == 4 ? 0x1p-24 : 0x1p-53);
}

template <typename R>
__global__ void __launch_bounds__(256) k_load_plasma(DevState<R> st, int run, int s,
                                                     PlasmaLoad L) {
#pragma clang fp contract(off)
  const DevRun& rd = st.runs[run];
  const long long n = (long long)L.x_cells * rd.ny * L.ppc;
  const Stream pos(L.seed, kTagPos), mom(L.seed, kTagMom + 16u * (unsigned)s);
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const long long cell = k / L.ppc;
    const int r = (int)(k - cell * L.ppc);
    const int ix = (int)(cell % L.x_cells), iy = (int)(cell / L.x_cells);
    const int tx = pic_tile_of(ix, st.TX, rd.ntx), ty = pic_tile_of(iy, st.TY, rd.nty);
    const int x0 = tx * st.TX, y0 = ty * st.TY;
    const int tw = pic_tile_width(tx, st.TX, rd.ntx, rd.nx);
    const int th = pic_tile_width(ty, st.TY, rd.nty, rd.ny);
    int fw = L.x_cells - x0;
    fw = fw < tw ? fw : tw;                     // filled columns of this tile
    const int tile = rd.tile0 + ty * rd.ntx + tx;
    // interleaved order: the r-th particle of every cell before the (r+1)-th
    const long long o = (long long)tile * st.tile_slots[s] + (long long)r * fw * th +
                        (long long)(iy - y0) * fw + (ix - x0);
    double fx, fy;
    pos.u01(k, 0, fx, fy);
    double ux, uy, uz;
    draw_momentum(mom, k, L, ux, uy, uz);
    // an offset that rounds up to 1 in FP32 is clamped to the largest value
    // below 1, so the particle stays in the cell and tile it is stored in (as
    // in the host load)
    const R ox = offset_below_one<R>(fx), oy = offset_below_one<R>(fy);
    st.cell[s][o] = pic_cell_pack(ix, iy);
    st.ox[s][o] = ox;
    st.oy[s][o] = oy;
    st.ux[s][o] = (R)ux;
    st.uy[s][o] = (R)uy;
    st.uz[s][o] = (R)uz;
    if (st.id[s]) st.id[s][o] = (int)k;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_load_counts(DevState<R> st, int run, int s,
                                                     PlasmaLoad L) {
  const DevRun& rd = st.runs[run];
  const int nt = rd.ntx * rd.nty;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) {
    const int tx = t % rd.ntx, ty = t / rd.ntx;
    const int x0 = tx * st.TX;
    const int tw = pic_tile_width(tx, st.TX, rd.ntx, rd.nx);
    const int th = pic_tile_width(ty, st.TY, rd.nty, rd.ny);
    int fw = L.x_cells - x0;
    fw = fw < 0 ? 0 : (fw < tw ? fw : tw);
    st.cnt[s][rd.tile0 + t] = fw * th * L.ppc;
  }
}

// Inflow of a shock run: before every step the flow entering through x_out
// is appended to the tiles of the cell column x_out - 1, as the seeded host
// generator of the injection slabs draws it. The stream moves w = beta0 cfl
// cells per step, so before step n each row receives
// floor(ppc w (n+1)) - floor(ppc w n) particles at x = x_out - w r0 (r0, and
// y's offset r1, from the item's position block), momenta drifting
// Maxwell-Juettner towards -x; the items continue after the x_out * ny * ppc
// of the initial load (item = first + row * per_row + j), electrons and
// positrons co-located. One work-group per (tile row, run, species): the
// tile's count is read, its rows' particles written after it, the count
// raised. The step index lives in device memory (graph replay reads it).
template <typename R>
__global__ void __launch_bounds__(256) k_inject_flow(DevState<R> st, const InflowDev* tab,
                                                     const long long* step_ctr) {
#pragma clang fp contract(off)
  const int ri = blockIdx.y;
  const InflowDev& F = tab[ri];
  if (!F.on) return;
  const DevRun& rd = st.runs[ri];
  const int s = blockIdx.z;
  const int ty = blockIdx.x;
  if (s >= rd.nspecies || ty >= rd.nty) return;
  const long long step = step_ctr[ri];
  const double done = floor(F.ppc_w * (double)step);
  const int per_row = (int)(floor(F.ppc_w * (double)(step + 1)) - done);
  const long long first = F.item0 + (long long)done * rd.ny;
  const int x_out = rd.x_out;
  const int tx = pic_tile_of(x_out - 1, st.TX, rd.ntx);
  const int y0 = ty * st.TY;
  const int th = pic_tile_width(ty, st.TY, rd.nty, rd.ny);
  const int tile = rd.tile0 + ty * rd.ntx + tx;
  const int cap = st.tile_slots[s];
  const int n0 = st.cnt[s][tile];
  int add = per_row * th;
  if (n0 + add > cap) {
    if (threadIdx.x == 0) atomicOr(st.err, PIC_ERRBIT_TILE);
    add = cap - n0;
  }
  const Stream pos(F.L.seed, kTagPos), mom(F.L.seed, kTagMom + 16u * (unsigned)s);
  const long long base = (long long)tile * cap + n0;
  for (int e = threadIdx.x; e < add; e += blockDim.x) {
    const int row = y0 + e / per_row;
    const long long k = first + (long long)row * per_row + (e - (e / per_row) * per_row);
    double r0, r1;
    pos.u01(k, 0, r0, r1);
    const double X = (double)x_out - F.w * r0;
    int ix = (int)floor(X);
    double fx = X - (double)ix;
    if (ix > x_out - 1) {   // r0 rounds the position onto x_out itself
      ix = x_out - 1;
      fx = 1.0;
    }
    double ux, uy, uz;
    draw_momentum(mom, k, F.L, ux, uy, uz);
    st.cell[s][base + e] = pic_cell_pack(ix, row);
    st.ox[s][base + e] = offset_below_one<R>(fx);
    st.oy[s][base + e] = offset_below_one<R>(r1);
    st.ux[s][base + e] = (R)ux;
    st.uy[s][base + e] = (R)uy;
    st.uz[s][base + e] = (R)uz;
    if (st.id[s]) st.id[s][base + e] = (int)k;
  }
  __syncthreads();
  if (threadIdx.x == 0 && add > 0) st.cnt[s][tile] = n0 + add;
}

// the inflow step counters advance once per step, after the injection
__global__ void k_inflow_advance(const InflowDev* tab, long long* step_ctr, int n_runs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_runs && tab[r].on) step_ctr[r] += 1;
}

}  // namespace

template <typename R>
hipError_t pic_launch_inject_flow(const DevState<R>& st, const InflowDev* tab, long long* step_ctr,
                                  int n_runs, int max_nty, int n_species, hipStream_t stream) {
  k_inject_flow<R><<<dim3(max_nty, n_runs, n_species), 256, 0, stream>>>(st, tab, step_ctr);
  k_inflow_advance<<<(n_runs + 63) / 64, 64, 0, stream>>>(tab, step_ctr, n_runs);
  return hipGetLastError();
}

template hipError_t pic_launch_inject_flow<float>(const DevState<float>&, const InflowDev*,
                                                  long long*, int, int, int, hipStream_t);
template hipError_t pic_launch_inject_flow<double>(const DevState<double>&, const InflowDev*,
                                                   long long*, int, int, int, hipStream_t);

template <typename R>
hipError_t pic_launch_load_plasma(const DevState<R>& st, int run, int s, const PlasmaLoad& L,
                                  int n_tiles_run, hipStream_t stream) {
  const long long n = (long long)L.x_cells * L.ny * L.ppc;
  const long long want = (n + 255) / 256;
  const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
  k_load_counts<R><<<(n_tiles_run + 255) / 256, 256, 0, stream>>>(st, run, s, L);
  if (n > 0) k_load_plasma<R><<<grid, 256, 0, stream>>>(st, run, s, L);
  return hipGetLastError();
}

template hipError_t pic_launch_load_plasma<float>(const DevState<float>&, int, int,
                                                  const PlasmaLoad&, int, hipStream_t);
template hipError_t pic_launch_load_plasma<double>(const DevState<double>&, int, int,
                                                   const PlasmaLoad&, int, hipStream_t);
