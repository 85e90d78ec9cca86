// Training and test-inference kernels of the learned CG aid (net_dev.h).
// Training runs in FP32 on the vector ALUs, on a whole periodic field of one
// run or on a crop of it: forward through the three linear 3x3 layers, the
// relative squared error against the recorded solution dB, backward through
// the adjoint convolutions, weight gradients reduced per block and then in a
// fixed block order, and an Adam update. A crop is the cx x cy window plus a
// 3-cell halo, taken with the field's periodic wrap and treated as a periodic
// field of its own; the three layers reach 3 cells, so the wrap of the window
// only affects its halo, which the loss leaves out: the loss and gradient are
// exactly those of the network on the window's cx x cy cells. Inference inside the solver uses net_apply_tile
// (BF16 matrix cores); k_net_apply runs that same routine on a whole field.
#include <math.h>

#include "net_dev.h"
#include "pic_dev.h"
#include "pic_launch.h"

namespace {

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// out[co][cell] = sum_ci sum_tap W[co][ci][tap] in[ci][cell + (dx-1, dy-1)]
__global__ void __launch_bounds__(256) k_conv_fwd(const float* in, int Cin, const float* W,
                                                  int Cout, float* out, int nx, int ny) {
  const long long n = (long long)nx * ny;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * Cout) return;
  const int co = (int)(e / n);
  const int cell = (int)(e - (long long)co * n);
  const int j = cell / nx, i = cell - j * nx;
  float acc = 0.f;
  for (int ci = 0; ci < Cin; ++ci) {
    const float* w = W + ((size_t)co * Cin + ci) * 9;
    const float* src = in + (size_t)ci * n;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const int jj = wrapc(j + dy - 1, ny);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) acc += w[dy * 3 + dx] * src[(size_t)jj * nx + wrapc(i + dx - 1, nx)];
    }
  }
  out[e] = acc;
}

// adjoint in the input: out[ci][cell] = sum_co sum_tap W[co][ci][tap] g[co][cell - (dx-1, dy-1)]
__global__ void __launch_bounds__(256) k_conv_adj(const float* g, int Cout, const float* W,
                                                  int Cin, float* out, int nx, int ny) {
  const long long n = (long long)nx * ny;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * Cin) return;
  const int ci = (int)(e / n);
  const int cell = (int)(e - (long long)ci * n);
  const int j = cell / nx, i = cell - j * nx;
  float acc = 0.f;
  for (int co = 0; co < Cout; ++co) {
    const float* w = W + ((size_t)co * Cin + ci) * 9;
    const float* src = g + (size_t)co * n;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const int jj = wrapc(j - dy + 1, ny);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) acc += w[dy * 3 + dx] * src[(size_t)jj * nx + wrapc(i - dx + 1, nx)];
    }
  }
  out[e] = acc;
}

// per-block partial weight gradients: part[b][co][ci][tap] =
// sum over the block's cells of g[co][cell] in[ci][cell + (dx-1, dy-1)];
// one thread per (co, ci) pair keeps the 9 taps as independent sums
__global__ void __launch_bounds__(256) k_conv_wgrad(const float* in, int Cin, const float* g,
                                                    int Cout, float* part, int nx, int ny,
                                                    int cells_per_block) {
  const int n = nx * ny;
  const int c0 = blockIdx.x * cells_per_block;
  const int c1 = min(n, c0 + cells_per_block);
  const int nw = Cout * Cin * 9;
  for (int pr = threadIdx.x; pr < Cout * Cin; pr += blockDim.x) {
    const int co = pr / Cin, ci = pr - co * Cin;
    const float* gs = g + (size_t)co * n;
    const float* xs = in + (size_t)ci * n;
    float acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.f;
    int j = c0 / nx, i = c0 - (c0 / nx) * nx;
    for (int cell = c0; cell < c1; ++cell) {
      const float gv = gs[cell];
      const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
      const float* rm = xs + (size_t)(j == 0 ? ny - 1 : j - 1) * nx;
      const float* r0 = xs + (size_t)j * nx;
      const float* rp = xs + (size_t)(j == ny - 1 ? 0 : j + 1) * nx;
      acc[0] += gv * rm[im];
      acc[1] += gv * rm[i];
      acc[2] += gv * rm[ip];
      acc[3] += gv * r0[im];
      acc[4] += gv * r0[i];
      acc[5] += gv * r0[ip];
      acc[6] += gv * rp[im];
      acc[7] += gv * rp[i];
      acc[8] += gv * rp[ip];
      if (++i == nx) {
        i = 0;
        ++j;
      }
    }
    float* out = part + (size_t)blockIdx.x * nw + (size_t)pr * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) out[k] = acc[k];
  }
}

// grad[w] = sum_b part[b][w] for 32 weights per work-group: 8 threads per
// weight each sum a strided eighth of the blocks, then the eight partial sums
// are added in a fixed order (deterministic)
constexpr int kRedW = 32, kRedT = 8;
__global__ void __launch_bounds__(kRedW * kRedT) k_reduce_parts(const float* part, int nblk,
                                                                int nw, float* grad) {
  __shared__ float acc[kRedT][kRedW];
  const int wl = threadIdx.x % kRedW, t = threadIdx.x / kRedW;
  const int w = blockIdx.x * kRedW + wl;
  float s = 0.f;
  if (w < nw) {
#pragma unroll 4
    for (int b = t; b < nblk; b += kRedT) s += part[(size_t)b * nw + w];
  }
  acc[t][wl] = s;
  __syncthreads();
  if (t == 0 && w < nw) {
    float r = acc[0][wl];
#pragma unroll
    for (int k = 1; k < kRedT; ++k) r += acc[k][wl];
    grad[w] = r;
  }
}

__global__ void __launch_bounds__(256) k_to_float(const double* a, float* b, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (float)a[e];
}

// the w x h window with corner (ox, oy) of an nx x ny periodic field: b as
// FP32 network input, t copied
__global__ void __launch_bounds__(256) k_crop(const double* b, const double* t, int nx, int ny,
                                              int ox, int oy, int w, int h, float* xin,
                                              double* tc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= w * h) return;
  const int i = e % w, j = e / w;
  const long long src = (long long)((oy + j) % ny) * nx + (ox + i) % nx;
  xin[e] = (float)b[src];
  tc[e] = t[src];
}

// cells of a w x h field that enter the loss: all but a border of bw cells
__device__ __forceinline__ bool in_loss(long long e, int w, int h, int bw) {
  const int i = (int)(e % w), j = (int)(e / w);
  return i >= bw && i < w - bw && j >= bw && j < h - bw;
}

// partial sums of t^2 (slot 0) and (y - t)^2 (slot 1) per block
__global__ void __launch_bounds__(256) k_sums(const float* y, const double* t, double* part,
                                              int w, int h, int bw) {
  __shared__ double s0[256], s1[256];
  double a0 = 0.0, a1 = 0.0;
  const long long n = (long long)w * h;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    if (!in_loss(e, w, h, bw)) continue;
    const double tv = t[e];
    const double r = (double)y[e] - tv;
    a0 += tv * tv;
    a1 += r * r;
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s0[threadIdx.x] += s0[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x * 2 + 0] = s0[0];
    part[blockIdx.x * 2 + 1] = s1[0];
  }
}

// scal[0] = sum t^2, scal[1] = loss = sum (y-t)^2 / sum t^2, added into
// scal[2]; one wavefront: each lane sums a strided share of the block
// partials, then a fixed butterfly adds the lanes (deterministic)
__global__ void __launch_bounds__(64) k_finish_sums(const double* part, int nblk, double* scal) {
  double t2 = 0.0, r2 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) {
    t2 += part[2 * b];
    r2 += part[2 * b + 1];
  }
  for (int off = 32; off > 0; off >>= 1) {
    t2 += __shfl_xor(t2, off, 64);
    r2 += __shfl_xor(r2, off, 64);
  }
  if (threadIdx.x == 0) {
    scal[0] = t2;
    scal[1] = t2 > 0.0 ? r2 / t2 : 0.0;
    scal[2] += scal[1];
  }
}

// gy = 2 (y - t) / sum t^2 on the loss cells, 0 on the border
__global__ void __launch_bounds__(256) k_loss_grad(const float* y, const double* t,
                                                   const double* scal, float* gy, int w, int h,
                                                   int bw) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)w * h) return;
  const double t2 = scal[0];
  gy[e] = t2 > 0.0 && in_loss(e, w, h, bw) ? (float)(2.0 * ((double)y[e] - t[e]) / t2) : 0.f;
}

__global__ void __launch_bounds__(256) k_adam(float* w, const float* g, float* m, float* v, int n,
                                              float lr, float b1, float b2, float eps, int step) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gv = g[e];
  const float mv = b1 * m[e] + (1.f - b1) * gv;
  const float vv = b2 * v[e] + (1.f - b2) * gv * gv;
  m[e] = mv;
  v[e] = vv;
  const float mh = mv / (1.f - powf(b1, (float)step));
  const float vh = vv / (1.f - powf(b2, (float)step));
  w[e] -= lr * mh / (sqrtf(vh) + eps);
}

// BF16 copy of W2 as [tap][co][ci] for the matrix cores
__global__ void __launch_bounds__(256) k_w2b(const float* w, __bf16* w2b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NET_C * NET_C * 9) return;
  const int ci = e % NET_C, co = (e / NET_C) % NET_C, tap = e / (NET_C * NET_C);
  w2b[e] = (__bf16)w[NET_W2 + ((size_t)co * NET_C + ci) * 9 + tap];
}

// Collapsed filter of the three layers, in FP64. With offsets o = (dx-1, dy-1)
// per 3 x 3 tap, N(x)(p) = sum W3 W2 W1 x(p + o1 + o2 + o3); first
// U[c2][o1 + o2] = sum_c1 W2[c2][c1][o2] W1[c1][o1] (5 x 5 per channel), then
// K[o] = sum_c2 sum_{o3} W3[c2][o3] U[c2][o - o3].
__global__ void __launch_bounds__(1024) k_collapse(const float* w, double* k49) {
  __shared__ double U[NET_C * 25];
  const int tid = threadIdx.x;
  if (tid < NET_C * 25) {
    const int c2 = tid / 25, o12 = tid % 25;
    const int oy = o12 / 5 - 2, ox = o12 % 5 - 2;
    double acc = 0.0;
    for (int t2 = 0; t2 < 9; ++t2) {
      const int ox1 = ox - (t2 % 3 - 1), oy1 = oy - (t2 / 3 - 1);
      if (ox1 < -1 || ox1 > 1 || oy1 < -1 || oy1 > 1) continue;
      const int t1 = (oy1 + 1) * 3 + (ox1 + 1);
      for (int c1 = 0; c1 < NET_C; ++c1)
        acc += (double)w[NET_W2 + (c2 * NET_C + c1) * 9 + t2] * (double)w[NET_W1 + c1 * 9 + t1];
    }
    U[tid] = acc;
  }
  __syncthreads();
  if (tid < 49) {
    const int oy = tid / 7 - 3, ox = tid % 7 - 3;
    double acc = 0.0;
    for (int t3 = 0; t3 < 9; ++t3) {
      const int ox12 = ox - (t3 % 3 - 1), oy12 = oy - (t3 / 3 - 1);
      if (ox12 < -2 || ox12 > 2 || oy12 < -2 || oy12 > 2) continue;
      const int o12 = (oy12 + 2) * 5 + (ox12 + 2);
      for (int c2 = 0; c2 < NET_C; ++c2)
        acc += (double)w[NET_W3 + c2 * 9 + t3] * U[c2 * 25 + o12];
    }
    k49[tid] = acc;
  }
}

template <bool kCollapsed>
__global__ void __launch_bounds__(PIC_CG_THREADS) k_net_apply(NetWeights W, const double* in,
                                                              double* out, int nx, int ny) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int TE = kCollapsed ? NET_KT : NET_T;
  const int ntx = (nx + TE - 1) / TE, nty = (ny + TE - 1) / TE;
  auto rd = [&](int i, int j) { return in[(long long)j * nx + i]; };
  auto wr = [&](int i, int j, double v) { out[(long long)j * nx + i] = v; };
  const bool one[1] = {true};
  for (int t = blockIdx.x; t < ntx * nty; t += gridDim.x) {
    if constexpr (kCollapsed)
      net_apply_tile_collapsed<1>(W, (t % ntx) * TE, (t / ntx) * TE, nx, ny, one,
                                  [&](int, int i, int j) { return rd(i, j); },
                                  [&](int, int i, int j, double v) { wr(i, j, v); }, lds);
    else
      net_apply_tile(W, (t % ntx) * TE, (t / ntx) * TE, nx, ny, rd, wr, lds);
  }
}

inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t pic_net_refresh(const NetTrain& T, hipStream_t s) {
  k_w2b<<<nblk(NET_C * NET_C * 9), 256, 0, s>>>(T.w, T.w2b);
  k_collapse<<<1, 1024, 0, s>>>(T.w, T.k49);
  return hipGetLastError();
}

hipError_t pic_net_apply(const NetTrain& T, int form, const double* in, double* out, int nx,
                         int ny, hipStream_t s) {
  NetWeights W{T.w, T.w2b, T.k49};
  const int TE = form == 0 ? NET_KT : NET_T;
  const int tiles = ((nx + TE - 1) / TE) * ((ny + TE - 1) / TE);
  const dim3 grid(tiles < 2048 ? tiles : 2048), block(PIC_CG_THREADS);
  if (form == 0)
    k_net_apply<true><<<grid, block, NET_K_LDS_BYTES, s>>>(W, in, out, nx, ny);
  else
    k_net_apply<false><<<grid, block, NET_LDS_BYTES, s>>>(W, in, out, nx, ny);
  return hipGetLastError();
}

// One loss/gradient evaluation on the sample (b, t) of an nx x ny periodic
// field, whole (cx <= 0) or on the cx x cy window with corner (ox, oy) and its
// 3-cell halo; grad receives dL/dW (all 9792 weights); scal[1] the loss,
// scal[2] accumulates it.
hipError_t pic_net_grad(const NetTrain& T, const double* b, const double* t, int nx, int ny,
                        int ox, int oy, int cx, int cy, hipStream_t s) {
  int w = nx, h = ny, bw = 0;
  const double* tt = t;
  if (cx > 0) {
    constexpr int H = 3;   // receptive-field radius of the three layers
    w = cx + 2 * H;
    h = cy + 2 * H;
    bw = H;
    k_crop<<<nblk((long long)w * h), 256, 0, s>>>(b, t, nx, ny, ((ox - H) % nx + nx) % nx,
                                                   ((oy - H) % ny + ny) % ny, w, h, T.xin, T.tc);
    tt = T.tc;
  } else {
    k_to_float<<<nblk((long long)w * h), 256, 0, s>>>(b, T.xin, (long long)w * h);
  }
  nx = w;
  ny = h;
  const long long n = (long long)nx * ny;
  const int C = NET_C;
  const float* W1 = T.w + NET_W1;
  const float* W2 = T.w + NET_W2;
  const float* W3 = T.w + NET_W3;
  k_conv_fwd<<<nblk(n * C), 256, 0, s>>>(T.xin, 1, W1, C, T.h1, nx, ny);
  k_conv_fwd<<<nblk(n * C), 256, 0, s>>>(T.h1, C, W2, C, T.h2, nx, ny);
  k_conv_fwd<<<nblk(n), 256, 0, s>>>(T.h2, C, W3, 1, T.y, nx, ny);
  k_sums<<<256, 256, 0, s>>>(T.y, tt, T.dpart, w, h, bw);
  k_finish_sums<<<1, 64, 0, s>>>(T.dpart, 256, T.scal);
  k_loss_grad<<<nblk(n), 256, 0, s>>>(T.y, tt, T.scal, T.gy, w, h, bw);
  const int cpb = (int)((n + T.wg_blocks - 1) / T.wg_blocks);
  // layer 3
  k_conv_wgrad<<<T.wg_blocks, 256, 0, s>>>(T.h2, C, T.gy, 1, T.part, nx, ny, cpb);
  k_reduce_parts<<<nblk(C * 9, kRedW), kRedW * kRedT, 0, s>>>(T.part, T.wg_blocks, C * 9,
                                                               T.grad + NET_W3);
  k_conv_adj<<<nblk(n * C), 256, 0, s>>>(T.gy, 1, W3, C, T.gh2, nx, ny);
  // layer 2
  k_conv_wgrad<<<T.wg_blocks, 256, 0, s>>>(T.h1, C, T.gh2, C, T.part, nx, ny, cpb);
  k_reduce_parts<<<nblk(C * C * 9, kRedW), kRedW * kRedT, 0, s>>>(T.part, T.wg_blocks,
                                                                   C * C * 9, T.grad + NET_W2);
  k_conv_adj<<<nblk(n * C), 256, 0, s>>>(T.gh2, C, W2, C, T.gh1, nx, ny);
  // layer 1
  k_conv_wgrad<<<T.wg_blocks, 256, 0, s>>>(T.xin, 1, T.gh1, C, T.part, nx, ny, cpb);
  k_reduce_parts<<<nblk(C * 9, kRedW), kRedW * kRedT, 0, s>>>(T.part, T.wg_blocks, C * 9,
                                                               T.grad + NET_W1);
  return hipGetLastError();
}

hipError_t pic_net_adam(const NetTrain& T, float lr, int step, hipStream_t s) {
  k_adam<<<nblk(NET_NW), 256, 0, s>>>(T.w, T.grad, T.m, T.v, NET_NW, lr, 0.9f, 0.999f, 1e-12f,
                                      step);
  return hipGetLastError();
}
