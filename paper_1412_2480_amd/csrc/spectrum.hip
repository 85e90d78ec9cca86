// k-space diagnostic of the numerical Cherenkov instability: the power
// spectrum |F(kx, ky)|^2 of one field component of a run, the quantity whose
// maps show where the instability grows (Sec. 3.1, Fig. 3: B_z in Fourier
// space against the resonance locus of Eq. (17)).
//
// A direct separable DFT in FP64 (the diagnostic grids of the paper's scans
// are 128 x 128; at 1024 x 256 it is about 3e8 complex multiply-adds):
//   pass 1: X(kx, j)  = sum_i F(i, j) exp(-2 pi i kx i / nx)   one thread per (kx, j)
//   pass 2: P(kx, ky) = |sum_j X(kx, j) exp(-2 pi i ky j / ny)|^2 / (nx ny)^2
// The phase angles are reduced exactly in integers, (kx i) mod nx, before the
// sine and cosine. Outputs are in the order of a discrete Fourier transform
// (index m = 0 .. n-1 for wavenumber 2 pi m / (n dx), aliased above n/2).
#include <math.h>

#include "pic_launch.h"

namespace {

constexpr int kSpecThreads = 256;

__global__ void __launch_bounds__(kSpecThreads)
k_dft_rows(const double* f, int nx, int ny, double* xr, double* xi) {
  const int kx = blockIdx.x * kSpecThreads + threadIdx.x;
  const int j = blockIdx.y;
  if (kx >= nx || j >= ny) return;
  const double* row = f + (long long)j * nx;
  double sr = 0.0, si = 0.0;
  long long m = 0;   // (kx * i) mod nx, advanced by kx each step
  for (int i = 0; i < nx; ++i) {
    double s, c;
    sincospi(2.0 * (double)m / (double)nx, &s, &c);
    const double v = row[i];
    sr += v * c;
    si -= v * s;
    m += kx;
    if (m >= nx) m -= nx;
  }
  xr[(long long)j * nx + kx] = sr;
  xi[(long long)j * nx + kx] = si;
}

__global__ void __launch_bounds__(kSpecThreads)
k_dft_cols_power(const double* xr, const double* xi, int nx, int ny, double* power) {
  const int kx = blockIdx.x * kSpecThreads + threadIdx.x;
  const int ky = blockIdx.y;
  if (kx >= nx || ky >= ny) return;
  double sr = 0.0, si = 0.0;
  long long m = 0;   // (ky * j) mod ny
  for (int j = 0; j < ny; ++j) {
    double s, c;
    sincospi(2.0 * (double)m / (double)ny, &s, &c);
    const double ar = xr[(long long)j * nx + kx], ai = xi[(long long)j * nx + kx];
    // (ar + i ai)(c - i s)
    sr += ar * c + ai * s;
    si += ai * c - ar * s;
    m += ky;
    if (m >= ny) m -= ny;
  }
  const double norm = 1.0 / ((double)nx * (double)ny);
  power[(long long)ky * nx + kx] = (sr * sr + si * si) * norm * norm;
}

}  // namespace

hipError_t pic_launch_spectrum(const double* f, int nx, int ny, double* xr, double* xi,
                               double* power, hipStream_t s) {
  const dim3 grid((nx + kSpecThreads - 1) / kSpecThreads, ny);
  k_dft_rows<<<grid, kSpecThreads, 0, s>>>(f, nx, ny, xr, xi);
  k_dft_cols_power<<<grid, kSpecThreads, 0, s>>>(xr, xi, nx, ny, power);
  return hipGetLastError();
}
