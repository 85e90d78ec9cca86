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
    // momentum: direction (block 0), flip decision (block 1), magnitude (2, ...)
    const double umag = L.T > 0.0 ? mj_speed(mom, k, L) : 0.0;
    double d0, d1, f0, unused;
    mom.u01(k, 0, d0, d1);
    mom.u01(k, 1, f0, unused);
    const double mu = 2.0 * d0 - 1.0;
    const double phi = kTwoPi * d1;
    const double stt = sqrt(fmax(0.0, 1.0 - mu * mu));
    double ux = umag * mu;
    const double uy = umag * stt * cos(phi);
    const double uz = umag * stt * sin(phi);
    if (L.gamma0 > 1.0) {
      const double gp = sqrt(1.0 + umag * umag);
      const double vx = ux / gp;
      if (-L.beta * vx > f0) ux = -ux;
      ux = L.gamma0 * (ux + L.beta * gp);
    }
    int cx = ix, cy = iy;
    R ox = (R)fx, oy = (R)fy;
    // an offset that rounds up to 1 moves to the next cell (as in the host load)
    if (ox >= R(1)) {
      ox = R(0);
      cx = ix + 1;
    }
    if (oy >= R(1)) {
      oy = R(0);
      cy = iy + 1 < rd.ny ? iy + 1 : 0;
    }
    st.cell[s][o] = pic_cell_pack(cx, cy);
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

}  // namespace

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
