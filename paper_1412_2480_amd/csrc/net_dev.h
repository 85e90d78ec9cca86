// Learned initial guess / preconditioner for the field CG (an addition to the
// paper's method, which solves Eq. (7) by plain CG): a linear convolutional
// network N of three 3x3 layers, 1 -> 32 -> 32 -> 1 channels, periodic
// padding, no activation (the target A^{-1} is linear). N is applied to one
// 16 x 16 output tile at a time by a work-group: the input with a 3-cell halo
// is staged in LDS, layer 1 (1 -> 32) and layer 3 (32 -> 1) run on the vector
// ALUs in FP32, layer 2 (32 -> 32, 92% of the arithmetic) runs on the matrix
// cores as an implicit GEMM in BF16 with FP32 accumulation
// (v_mfma_f32_32x32x16_bf16: 32 cells x 32 output channels x 16 input
// channels per instruction, 2 instructions per tap).
//
// Because every layer is linear and shift-invariant, N is exactly one 7 x 7
// periodic filter K (the three 3 x 3 kernels composed, summed over channels).
// The collapsed form applies K in FP64 to 32 x 32 tiles staged in LDS; K is
// recomputed from the FP32 weights whenever they change.
#pragma once

#include <hip/hip_runtime.h>

#define NET_C 32                       // hidden channels
#define NET_T 16                       // output tile edge
#define NET_W1 0                       // offsets in the FP32 weight vector
#define NET_W2 (NET_C * 9)
#define NET_W3 (NET_C * 9 + NET_C * NET_C * 9)
#define NET_NW (NET_C * 9 * 2 + NET_C * NET_C * 9)   // 9792 weights

typedef __bf16 net_bf16x8 __attribute__((ext_vector_type(8)));
typedef float net_f32x16 __attribute__((ext_vector_type(16)));

// LDS footprint of one tile application (bytes)
#define NET_X_E ((NET_T + 6) * (NET_T + 6))        // input with 3-cell halo
#define NET_H1_E ((NET_T + 4) * (NET_T + 4))       // layer-1 output, 2-cell halo
#define NET_H2_E (((((NET_T + 2) * (NET_T + 2)) + 31) / 32) * 32)  // layer-2 output, padded
#define NET_W1_PITCH 12                            // W1 row of 9 taps padded to 12 in LDS
#define NET_LDS_BYTES (NET_X_E * 4 + NET_H1_E * NET_C * 2 + NET_H2_E * NET_C * 2 + \
                       (NET_C * NET_W1_PITCH + 9 * NET_C) * 4)

#define NET_KT 32                                     // output tile edge, collapsed form
#define NET_KE (NET_KT + 6)                           // staged edge (3-cell halo)
#define NET_K_LDS_BYTES ((64 + 3 * NET_KE * NET_KE) * 8)   // filter + 3 staged components

struct NetWeights {
  const float* w;        // FP32 weights: W1[co][tap], W2[co][ci][tap], W3[ci][tap]
  const __bf16* w2b;     // BF16 copy of W2 as [tap][co][ci] (matrix-core B operand)
  const double* k49;     // collapsed filter: N(x)(p) = sum_o K[(oy+3)*7 + ox+3] x(p + o)
};

// i mod n for i within a few periods of [0, n) (the staged halo is at most
// 3 cells; a loop keeps grids narrower than the halo correct)
__device__ __forceinline__ int net_mod(int i, int n) {
  while (i < 0) i += n;
  while (i >= n) i -= n;
  return i;
}

// z(tile) = N(r) for the 16 x 16 output tile at (X0, Y0) of a periodic nx x ny
// grid. rd(i, j) reads the input at any (wrapped) cell; wr(i, j, v) writes the
// output of an in-grid cell (i < nx, j < ny). All threads of the block call it.
template <typename Rd, typename Wr>
__device__ void net_apply_tile(const NetWeights& W, int X0, int Y0, int nx, int ny, Rd&& rd,
                               Wr&& wr, unsigned char* lds) {
  float* sx = reinterpret_cast<float*>(lds);
  __bf16* h1 = reinterpret_cast<__bf16*>(lds + NET_X_E * 4);
  __bf16* h2 = h1 + NET_H1_E * NET_C;
  float* w1 = reinterpret_cast<float*>(h2 + NET_H2_E * NET_C);   // [co][NET_W1_PITCH]
  float* w3 = w1 + NET_C * NET_W1_PITCH;                           // [tap][ci]
  const int tid = threadIdx.x, nthr = blockDim.x;
  constexpr int XE = NET_T + 6, HE1 = NET_T + 4, HE2 = NET_T + 2;

  for (int e = tid; e < NET_C * 9; e += nthr) {
    const int co = e / 9, t = e % 9;
    w1[co * NET_W1_PITCH + t] = W.w[NET_W1 + e];
    w3[t * NET_C + co] = W.w[NET_W3 + e];     // W3 is [ci][tap]; e = ci * 9 + tap
  }
  for (int e = tid; e < XE * XE; e += nthr) {
    const int i = net_mod(X0 + e % XE - 3, nx), j = net_mod(Y0 + e / XE - 3, ny);
    sx[e] = (float)rd(i, j);
  }
  __syncthreads();
  // layer 1: one cell of the (T+4)^2 region per thread, all channels; the
  // weights are read as broadcasts, the 32 outputs stored as four 16-byte rows
  for (int cell = tid; cell < NET_H1_E; cell += nthr) {
    const int u = cell % HE1, v = cell / HE1;   // region origin at tile -2
    float xv[9];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) xv[dy * 3 + dx] = sx[(v + dy) * XE + (u + dx)];
    __bf16* dst = h1 + cell * NET_C;
#pragma unroll
    for (int c8 = 0; c8 < NET_C; c8 += 8) {
      net_bf16x8 pack;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float* w = w1 + (c8 + q) * NET_W1_PITCH;
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc += w[t] * xv[t];
        pack[q] = (__bf16)acc;
      }
      *reinterpret_cast<net_bf16x8*>(dst + c8) = pack;
    }
  }
  __syncthreads();
  // layer 2 on the matrix cores: rows = 32 cells of the (T+2)^2 region
  {
    const int lane = tid & 63, wave = tid >> 6, nwave = nthr >> 6;
    const int row = lane & 31, kg = lane >> 5;
    constexpr int nblk = NET_H2_E / 32;
    for (int cb = wave; cb < nblk; cb += nwave) {
      int cell = cb * 32 + row;
      const int valid_max = HE2 * HE2 - 1;
      const int cc = cell > valid_max ? valid_max : cell;   // padded rows read a valid cell
      const int u = cc % HE2, v = cc / HE2;                  // region origin at tile -1
      net_f32x16 acc = {};
#pragma unroll 1
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int tap = dy * 3 + dx;
          const __bf16* arow = h1 + ((v + dy) * HE1 + (u + dx)) * NET_C;
          const __bf16* brow = W.w2b + (tap * NET_C + row) * NET_C;
#pragma unroll
          for (int kc = 0; kc < 2; ++kc) {
            const net_bf16x8 a = *reinterpret_cast<const net_bf16x8*>(arow + kc * 16 + kg * 8);
            const net_bf16x8 b = *reinterpret_cast<const net_bf16x8*>(brow + kc * 16 + kg * 8);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
          }
        }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int r_ = (q >> 2) * 8 + kg * 4 + (q & 3);
        const int oc = cb * 32 + r_;
        if (oc < HE2 * HE2) h2[oc * NET_C + row] = (__bf16)acc[q];
      }
    }
  }
  __syncthreads();
  // layer 3: two threads per output cell, 16 channels each, read as two
  // 16-byte rows per tap; the halves are combined across the lane pair
  for (int base = 0; base < NET_T * NET_T * 2; base += nthr) {
    const int e = base + tid;
    const bool live = e < NET_T * NET_T * 2;
    const int cell = e >> 1, half = e & 1;
    const int u = cell % NET_T, v = cell / NET_T;
    float acc = 0.f;
    if (live) {
#pragma unroll 1
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const __bf16* hp = h2 + ((v + dy) * HE2 + (u + dx)) * NET_C + half * 16;
          const float* w = w3 + (dy * 3 + dx) * NET_C + half * 16;
          const net_bf16x8 a0 = *reinterpret_cast<const net_bf16x8*>(hp);
          const net_bf16x8 a1 = *reinterpret_cast<const net_bf16x8*>(hp + 8);
#pragma unroll
          for (int q = 0; q < 8; ++q) acc += w[q] * (float)a0[q];
#pragma unroll
          for (int q = 0; q < 8; ++q) acc += w[8 + q] * (float)a1[q];
        }
    }
    acc += __shfl_xor(acc, 1, 64);
    const int i = X0 + u, j = Y0 + v;
    if (live && half == 0 && i < nx && j < ny) wr(i, j, (double)acc);
  }
  __syncthreads();
}

// Collapsed form: z_c = K * x_c on the NET_KT x NET_KT output tile at
// (X0, Y0) for every component c < NC with act[c], in FP64. The components
// share one staging pass, so their loads are in flight together.
// rd(c, i, j) reads component c at an in-grid cell; wr(c, i, j, z) receives
// each output of an in-grid cell. All threads of the block call it.
template <int NC, typename Rd, typename Wr>
__device__ void net_apply_tile_collapsed(const NetWeights& W, int X0, int Y0, int nx, int ny,
                                         const bool (&act)[NC], Rd&& rd, Wr&& wr,
                                         unsigned char* lds) {
  constexpr int E = NET_KE;
  double* sk = reinterpret_cast<double*>(lds);
  double* sx = sk + 64;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int e = tid; e < 49; e += nthr) sk[e] = W.k49[e];
  for (int e = tid; e < E * E; e += nthr) {
    const int i = net_mod(X0 + e % E - 3, nx), j = net_mod(Y0 + e / E - 3, ny);
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (act[c]) sx[c * E * E + e] = rd(c, i, j);
  }
  __syncthreads();
  // each thread forms two vertically adjacent outputs from 8 staged rows:
  // per row 7 values and that row's 7 filter weights are read once, the
  // previous row's weights serve the lower output (112 LDS reads for 2 x 49
  // products instead of 196); each sum keeps a single output's order
  for (int pr = tid; pr < NET_KT * NET_KT / 2; pr += nthr) {
    const int u = pr % NET_KT, v = 2 * (pr / NET_KT);
    const int i = X0 + u, j = Y0 + v;
    if (i >= nx || j >= ny) continue;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (!act[c]) continue;
      const double* x = sx + c * E * E;
      double a0 = 0.0, a1 = 0.0;
      double kp[7];
#pragma unroll 1
      for (int dy = 0; dy < 8; ++dy) {
        double row[7], kc[7];
#pragma unroll
        for (int dx = 0; dx < 7; ++dx) {
          row[dx] = x[(v + dy) * E + (u + dx)];
          kc[dx] = dy < 7 ? sk[dy * 7 + dx] : 0.0;
        }
        if (dy < 7) {
#pragma unroll
          for (int dx = 0; dx < 7; ++dx) a0 += kc[dx] * row[dx];
        }
        if (dy >= 1) {
#pragma unroll
          for (int dx = 0; dx < 7; ++dx) a1 += kp[dx] * row[dx];
        }
#pragma unroll
        for (int dx = 0; dx < 7; ++dx) kp[dx] = kc[dx];
      }
      wr(c, i, j, a0);
      if (j + 1 < ny) wr(c, i, j + 1, a1);
    }
  }
  __syncthreads();
}
