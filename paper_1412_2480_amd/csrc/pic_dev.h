// Internal device-side layout of the PIC library (not part of the C-ABI).
//
// All runs of a context live in one workspace. Field arrays of every run are
// concatenated (run r starts at cell0[r]); the particle store of a species is
// one SoA region cut into fixed-size tile segments (slot k of global tile t is
// t * tile_slots + k). Tiles are TX x TY cells; the last tile of a row/column
// may be up to 2 cells wider so that no tile is narrower than 3 cells.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PIC_MAXS 2
#define PIC_GUARD_LO 2   // patch / LDS nodes below the tile origin
#define PIC_GUARD_HI 3   // patch / LDS nodes at or above the tile end

// error bits raised by kernels (read back by the host)
#define PIC_ERRBIT_TILE 4       // a tile's slots ran out
#define PIC_ERRBIT_BARRIER 8    // a grid barrier timed out

#define PIC_WALL_GAP 4   // shock runs: particles leave at x >= (nx - PIC_WALL_GAP) dx

struct DevRun {
  int nx, ny, order, nspecies;
  int bc;             // 0 periodic, 1 shock (conducting walls in x, reflection at x = 0)
  int x_out;          // shock runs: first cell column where particles leave
  int ntx, nty;       // tiles per row / column of this run
  int tile0;          // first global tile index
  long long cell0;    // first cell in the concatenated field arrays
  int cg_blk_lo, cg_blk_hi;  // CG work-group range owned by this run
  int cg_maxit;
  double cg_rtol;
  double dx, dy, dt, theta;
  double q[PIC_MAXS], m[PIC_MAXS];
  int net_id;         // learned solver: network of this run's operator
  double* pairs;      // learned solver: (b, dB) ring of the network, in its first run only
};

template <typename R>
struct DevState {
  int n_runs, n_tiles;
  int TX, TY, TXA, TYA, PW, PH;  // tile shape, widest tile, patch pitch/rows
  int tile_slots[PIC_MAXS];
  int K;                          // work-groups per tile (each takes 1/K of its particles)
  int nodal;                      // 1: gather from node-averaged fields (momentum-conserving)
  const DevRun* runs;
  const int* tile_run;            // run index of each global tile

  // fields, FP64 masters (Yee positions), all runs concatenated
  double* E[3];
  double* B[3];
  double* J[3];
  float* Ef[6];                   // FP32 copy of Ex..Bz for the fast path

  // particle store (per species), double-buffered: the particle kernel reads
  // the current arrays and writes the particles that stay in their tile,
  // compacted, into the next arrays; re-binning appends the arrivals there
  // and the host swaps the two sets. id arrays are null when ids are off.
  int* cell[PIC_MAXS];            // (iy << 16) | ix, run-local cell
  R* ox[PIC_MAXS];
  R* oy[PIC_MAXS];
  R* ux[PIC_MAXS];
  R* uy[PIC_MAXS];
  R* uz[PIC_MAXS];
  int* id[PIC_MAXS];
  int* ncell[PIC_MAXS];
  R* nox[PIC_MAXS];
  R* noy[PIC_MAXS];
  R* nux[PIC_MAXS];
  R* nuy[PIC_MAXS];
  R* nuz[PIC_MAXS];
  int* nid[PIC_MAXS];
  int* cnt[PIC_MAXS];             // live particles per tile (current arrays)
  int* stay_cnt[PIC_MAXS];        // slots handed out in the next arrays by the running pass

  // split path: positions before the move
  int* old_cell[PIC_MAXS];
  R* old_ox[PIC_MAXS];
  R* old_oy[PIC_MAXS];

  double* patch[3];               // current patches [tile][K][PH][PW] (FP64)
  double* wk_part;                // [tile][K][species][2] kinetic energy partials
  int* err;                       // error bits
};

__device__ __forceinline__ int pic_cell_ix(int c) { return c & 0xffff; }
__device__ __forceinline__ int pic_cell_iy(int c) { return c >> 16; }
__device__ __forceinline__ int pic_cell_pack(int ix, int iy) { return (iy << 16) | ix; }

// tile index along one axis for cell i; the last tile absorbs a short tail
__device__ __forceinline__ int pic_tile_of(int i, int T, int nt) {
  int t = i / T;
  return t < nt ? t : nt - 1;
}
__device__ __forceinline__ int pic_tile_width(int t, int T, int nt, int n) {
  return t == nt - 1 ? n - t * T : T;
}
__device__ __forceinline__ int pic_wrap(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}
