/*
 * pic.h -- C-ABI of the MI355X (gfx950) library for the data-parallel hot path
 * of the 2D3V relativistic PIC method of Ikeya & Matsumoto, "Stability Property
 * of Numerical Cherenkov Radiation and its Application to Relativistic Shock
 * Simulations", PASJ 2015 (arXiv:1412.2480).
 *
 * One time step, as the paper states the problem (Sec. 2, Eqs. (5)-(7), and the
 * PIC ingredients named in Sec. 1 and Sec. 3):
 *   1. momentum-conserving gather of E^n, B^n to x^n with the order-p shape,
 *   2. relativistic Boris push u^{n-1/2} -> u^{n+1/2}, move x^n -> x^{n+1},
 *   3. Esirkepov density-decomposition deposit of J^{n+1/2},
 *   4. implicit theta-weighted field solve: CG for dB of Eq. (7), then the
 *      update of Eqs. (5)-(6).
 *
 * Conventions
 *   Units: Gaussian, c = 1. dt = cfl * dx (cfl is the paper's sigma, Sec. 3.1).
 *   Grid: nx*ny cells, arrays row-major [ny][nx] (index j*nx + i), standard 2D
 *   Yee staggering: Ex(i+1/2,j) Ey(i,j+1/2) Ez(i,j) Bx(i,j+1/2) By(i+1/2,j)
 *   Bz(i+1/2,j+1/2); J co-located with E; rho at nodes.
 *   Particles: cell index (ix, iy) plus in-cell offset (fx, fy) in [0, 1), so
 *   x = (ix + fx) dx; momentum u = gamma v; positions at integer steps,
 *   momenta at half steps.
 *
 * Ownership: the caller allocates one device workspace of
 * pic_plan_info.workspace_bytes (e.g. a torch uint8 tensor) and owns a HIP
 * stream; both must outlive the context. The library allocates no device
 * memory; it only keeps host-side bookkeeping in the opaque context. Host arrays
 * passed in are borrowed for the duration of the call and copied.
 *
 * Errors: every call returns an int32 status (PIC_OK = 0, negative on error);
 * no exception crosses the ABI. pic_last_error() gives a message (with a
 * null context: that of the last failed pic_init on this thread). EINVAL
 * leaves the state unchanged. Kernel faults surface at the next call that
 * synchronises (pic_sync, pic_diag, reads, the end of pic_step).
 * Threading: one context per host thread; all work is ordered on the
 * context's stream.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_MAX_SPECIES 2
#define PIC_MAX_RUNS 256

enum pic_status {
  PIC_OK = 0,
  PIC_E_INVAL = -1,    /* bad argument or descriptor */
  PIC_E_NOMEM = -2,    /* workspace smaller than the plan requires */
  PIC_E_HIP = -3,      /* HIP runtime error */
  PIC_E_NOCONV = -4,   /* CG hit cg_maxit; the best iterate was applied */
  PIC_E_CAPACITY = -5, /* a tile's particle slots overflowed (raise slack) */
  PIC_E_NAN = -6,      /* non-finite value found by a diagnostic */
  PIC_E_STATE = -7     /* calls out of order (e.g. deposit before gather_push) */
};

/* Boundaries. PIC_BC_SHOCK is the shock set-up (a reading: the paper only says
 * the flow is injected at one side and reflected at the other, Sec. 4):
 * conducting walls at x = 0 and x = (nx-1) dx (Ey, Ez, Bx zero on those node
 * lines; Ex, By, Bz of the last column lie outside and are zero), specular
 * reflection of particles at x = 0 (x -> -x, ux -> -ux; the deposit folds the
 * part of a shape behind the wall back, rho/Jy/Jz with their sign and Jx
 * negated), removal of particles reaching x_out = (nx - PIC_WALL_GAP) dx,
 * where new flow enters through pic_inject_particles; y periodic. */
enum pic_bc { PIC_BC_PERIODIC = 0, PIC_BC_SHOCK = 1 };
#define PIC_WALL_GAP 4
enum pic_precision { PIC_FP64 = 0, PIC_FP32_FAST = 1 };
enum pic_solver {
  PIC_SOLVER_CG = 0,          /* plain CG on Eq. (7) (the paper's solver) */
  PIC_SOLVER_LEARNED_PCG = 1  /* learned x0 + flexible PCG, plain-CG fallback (an addition) */
};
enum pic_learned_form {
  PIC_NET_COLLAPSED = 0,      /* the network's exact 7 x 7 composite filter, FP64 */
  PIC_NET_MFMA = 1            /* the network itself, BF16 matrix cores, FP32 accumulation */
};
/* Field ids. PIC_RHO (charge density) and PIC_N0, PIC_N1 (number density of
 * species 0, 1: particles per unit area, the density profiles of the shock
 * runs, Sec. 4, Figs. 7-8) are deposited on demand from the particles with
 * the order-p shape at the nodes; they are read only. */
enum pic_field_id {
  PIC_EX = 0, PIC_EY, PIC_EZ, PIC_BX, PIC_BY, PIC_BZ, PIC_JX, PIC_JY, PIC_JZ, PIC_RHO,
  PIC_N0, PIC_N1
};

typedef struct pic_species_desc {
  double q;           /* macro-particle charge (Gaussian units) */
  double m;           /* macro-particle mass */
  double ppc;         /* expected particles per cell, sizes the tile slots */
} pic_species_desc;

/* One simulation. All runs of a context share precision and tile shape. */
typedef struct pic_run_desc {
  int32_t nx, ny;        /* cells; each >= 8 and <= 32767 */
  double dx, dy;         /* cell sizes (c/omega_pe) */
  double cfl;            /* sigma = c dt/dx, 0 < sigma <= 1 (Esirkepov needs < 1 cell/step) */
  double theta;          /* implicitness factor of Eqs. (5)-(6), 0.5 <= theta <= 1 */
  int32_t shape_order;   /* B-spline degree 1, 2 or 3 */
  int32_t bc;            /* PIC_BC_PERIODIC (both directions) or PIC_BC_SHOCK (nx >= 16) */
  int32_t n_species;     /* 1 .. PIC_MAX_SPECIES */
  pic_species_desc species[PIC_MAX_SPECIES];
  double cg_rtol;        /* relative residual target of the field CG (e.g. 1e-8) */
  int32_t cg_maxit;      /* iteration cap of the field CG (e.g. 200) */
} pic_run_desc;

typedef struct pic_options {
  int32_t precision;     /* PIC_FP64 or PIC_FP32_FAST (particles in FP32, fields FP64) */
  int32_t solver;        /* PIC_SOLVER_CG or PIC_SOLVER_LEARNED_PCG */
  int32_t tile_x, tile_y;/* tile shape in cells, at least 2 each (PIC_E_INVAL otherwise);
                            0 picks a default (16) */
  double slack;          /* extra tile slots over ppc*cells (default 0.25 if <= 0); a
                            relativistic drift that goes unstable to numerical Cherenkov
                            radiation bunches the density: the 2000-step gamma0 = 40 run
                            of 1024 x 256 cells needs 0.5 (PIC_E_CAPACITY near step 500
                            at 0.25) */
  double exchange_frac;  /* ignored: particles that change tile are written straight into
                            the destination tile's slots, so no exchange buffer exists */
  int32_t diag_every;    /* record energies every n steps into the history (0 = never) */
  int32_t history_cap;   /* history records kept per run (ring buffer) */
  int32_t cg_blocks;     /* work-groups of the persistent field solve; 0 = as many as
                            can be co-resident (at most one per 512 cells of a run) */
  int32_t track_ids;     /* 1: particles carry ids and reads return them ordered by id;
                            0: no ids (8 B less traffic per particle-step), reads return
                            storage order */
  int32_t tile_split;    /* work-groups per tile in the particle kernel; 0 = 4 */
  int32_t learned_form;  /* PIC_NET_COLLAPSED or PIC_NET_MFMA (learned solver only) */
  int32_t learned_maxit; /* iteration budget of the learned PCG before the plain-CG
                            fallback; 0 = 30 */
  int32_t precond_slots; /* (b, dB) training pairs kept (ring); 0 = 16 */
  int32_t graph;         /* 1: pic_step replays HIP graphs of two captured steps (one
                            per buffer parity, reordering pattern and solver variant)
                            whenever no diagnostics record, timing or pair collection
                            falls in them; 0: plain launches */
  int32_t sort_every;    /* pic_step reorders every tile's particles by cell every
                            this many steps (0 = never); see pic_step */
  int32_t cg_x0;         /* initial iterate of the plain field CG: PIC_X0_ZERO (the
                            paper's solve, the default) or PIC_X0_PREV (the previous
                            step's dB; the stopping test is the same relative residual).
                            The learned solver always starts from N(b). */
  int32_t field_scheme;  /* PIC_SCHEME_IMPLICIT: the theta-weighted implicit solve of
                            Eqs. (5)-(7) (the paper's method, the default);
                            PIC_SCHEME_EXPLICIT: the explicit Yee FDTD of Eqs. (3)-(4)
                            (the scheme the paper contrasts it with, Sec. 2), B carried at
                            integer times for the push as the mean of its half-step
                            values; periodic runs, solver PIC_SOLVER_CG, and the Courant
                            condition cfl^2 (1 + dx^2/dy^2) <= 1 (dispersion Eq. (16));
                            theta and the CG fields are not used */
  int32_t gather;        /* field interpolation to the particles: PIC_GATHER_NODAL, the
                            momentum-conserving interpolation of Sec. 1 and Sec. 3
                            (Birdsall & Langdon ch. 8: every component averaged from its
                            Yee points onto the charge nodes, then interpolated with the
                            charge-assignment weights; the default), or
                            PIC_GATHER_STAGGERED (each component from its own Yee points
                            with the same weights; an alternative reading, kept for
                            comparison) */
} pic_options;

enum pic_cg_x0 { PIC_X0_ZERO = 0, PIC_X0_PREV = 1 };
enum pic_gather { PIC_GATHER_NODAL = 0, PIC_GATHER_STAGGERED = 1 };
enum pic_field_scheme { PIC_SCHEME_IMPLICIT = 0, PIC_SCHEME_EXPLICIT = 1 };

typedef struct pic_plan_info {
  uint64_t workspace_bytes;
  int32_t tile_x, tile_y;
  int32_t n_tiles;                         /* over all runs */
  int32_t tile_slots[PIC_MAX_SPECIES];     /* particle slots per tile per species */
  int32_t exchange_slots;                  /* always 0 (no exchange buffer) */
  int32_t tile_split;                      /* work-groups per tile */
  int64_t particle_slots[PIC_MAX_SPECIES]; /* total slots per species */
  int64_t n_cells;                         /* over all runs */
} pic_plan_info;

/* Statistics of the last field solve of one run (Eq. (7), per B component). */
typedef struct pic_solve_stats {
  int32_t iters[3];      /* CG iterations per B component (learned + plain) */
  double relres[3];      /* true relative residual ||b - A dB||_2/||b||_2 of the applied dB,
                            recomputed in FP64 from E^n, B^n, J after the solve */
  double bnorm[3];       /* ||b||_2 of Eq. (7)'s right-hand side */
  int32_t learned_iters[3]; /* iterations of the learned PCG (0 with plain CG) */
  int32_t fallback;      /* 1 if the learned PCG missed cg_rtol and plain CG finished */
  double relres_recursive[3]; /* the solver's recursive residual ||r_k||/||b|| at exit,
                            which its stopping test compares with cg_rtol */
} pic_solve_stats;

/* Diagnostics of one run. The energy record (step .. cg_relres) is written
 * by the field solve every diag_every steps; the energy balance it allows is
 * the one the paper reports its runs by (total energy within 1%, Sec. 3.2):
 * W_E(n) + W_B(n) + (W_K(n-1/2) + W_K(n+1/2))/2. pic_diag fills the fields
 * after n_particles from the current state; history records leave them 0. */
typedef struct pic_diag_out {
  int64_t step;          /* step index n of the record (-1: none recorded yet) */
  double t;              /* n dt */
  double W_E, W_B;       /* field energies at step n: sum |F|^2 dx dy/(8 pi) */
  double W_K_minus;      /* sum m (gamma - 1) at n - 1/2 */
  double W_K_plus;       /* sum m (gamma - 1) at n + 1/2 */
  int32_t cg_iters[3];
  double cg_relres[3];   /* true relative residual of the step's solve */
  int64_t n_particles[PIC_MAX_SPECIES];
  double gauss_max;      /* max |div E - 4 pi rho| over the nodes (Gauss's law, which
                            the Esirkepov deposit and Eqs. (5)-(6) keep at its initial
                            value); a shock run is measured on node columns
                            1 .. x_out - 4 (the wall line carries the conductor's surface
                            charge and particles leave at x_out) */
  double divb_max;       /* max |div B| over the cells */
  double total_charge;   /* sum rho dx dy of the particles' charge density */
  int64_t fallbacks;     /* learned-solver solves finished by plain CG, since pic_init */
  int64_t solves;        /* field solves since pic_init */
} pic_diag_out;

typedef struct pic_timing_out {
  /* accumulated device time (ms) and launch counts per kernel class since
     timing was switched on: 0 particle push (fused or split), 1 deposit
     (split path), 2 rebin, 3 current reduction, 4 field RHS, 5 CG,
     6 field update, 7 diagnostics, 8 particle reordering */
  double ms[9];
  int64_t launches[9];
  int64_t graph_replays; /* two-step graph replays since pic_init (graph mode) */
} pic_timing_out;

typedef struct pic_ctx pic_ctx;

/* Validate runs/options and size the workspace (host only, no HIP calls). */
int32_t pic_plan(const pic_run_desc* runs, int32_t n_runs, const pic_options* opt,
                 pic_plan_info* out);

/* Create a context on the caller's workspace and stream (hipStream_t passed
 * as void*; NULL is the default stream). Fields start at zero, as in the
 * paper's runs (Sec. 3, first paragraph); particle counts start at zero. */
int32_t pic_init(const pic_run_desc* runs, int32_t n_runs, const pic_options* opt,
                 void* d_workspace, size_t ws_bytes, void* hip_stream, pic_ctx** out);

/* Replace the particles of (run, species) with n host particles: cell index
 * (ix, iy), offset (fx, fy) in [0, 1) and momentum (ux, uy, uz) at n - 1/2.
 * Particle k gets id k. PIC_E_CAPACITY if a tile's slots overflow (state unchanged). */
int32_t pic_load_particles(pic_ctx* ctx, int32_t run, int32_t species, int64_t n,
                           const int32_t* ix, const int32_t* iy, const double* fx,
                           const double* fy, const double* ux, const double* uy,
                           const double* uz);

/* Seeded synthetic plasma generated on the device (for loads too large for
 * the host): ppc particles per cell in the cell columns i < x_cells (0 = all
 * columns; a shock run's load must stop at x_out), uniform inside the cell,
 * momenta drifting Maxwell-Juettner with rest-frame temperature T (m c^2) and
 * bulk Lorentz factor gamma0 along direction * x. Item k (cell k / ppc,
 * row-major over the loaded columns) draws its numbers from Philox4x32-10
 * counters keyed by (seed, tag): positions from tag 1, momenta from tag
 * 2 + 16 * species; this is the recipe of the repository's seeded host
 * generator, item by item. Replaces the particles of (run, species); ids are
 * the item numbers. */
typedef struct pic_plasma_desc {
  int32_t ppc;
  int32_t x_cells;
  double gamma0;
  double T;
  int32_t direction;     /* +1 or -1 */
  uint64_t seed;
} pic_plasma_desc;

int32_t pic_load_plasma(pic_ctx* ctx, int32_t run, int32_t species, const pic_plasma_desc* desc);

/* Append n host particles to (run, species) of a PIC_BC_SHOCK run between
 * steps (same arrays as pic_load_particles; ix < nx - PIC_WALL_GAP). They get
 * the next ids of the species. At most four cell columns' worth of the run
 * (4 ny ppc) per call; PIC_E_CAPACITY if a tile's slots would overflow (state
 * unchanged). Synchronises. */
int32_t pic_inject_particles(pic_ctx* ctx, int32_t run, int32_t species, int64_t n,
                             const int32_t* ix, const int32_t* iy, const double* fx,
                             const double* fy, const double* ux, const double* uy,
                             const double* uz);

/* Inflow of a PIC_BC_SHOCK run generated on the device (the shock set-up of
 * Sec. 4: the flow is injected at one side; a reading of its details): from
 * the next step on, every step (pic_step, and pic_gather_push of the split
 * path) first appends the flow entering through x_out = (nx - PIC_WALL_GAP) dx
 * to the tiles of the cell column x_out - 1, for every species of the run,
 * with no host transfer (graph replay included). The stream moves
 * w = beta0 cfl cells per step (beta0 = sqrt(1 - 1/gamma0^2)); before the
 * run's injection step n each row receives floor(ppc w (n+1)) -
 * floor(ppc w n) particles at x = x_out - w r0, y uniform in the row,
 * momenta drifting Maxwell-Juettner at (gamma0, T) towards -x; electrons and
 * positrons co-located. The numbers come from the Philox streams of
 * pic_load_plasma with items continuing after x_out * ny * ppc (the initial
 * load of the flow region), item = first + row * per_row + j; ids are the item
 * numbers (int32: meaningful while the items stay below 2^31). This is the recipe of the repository's seeded host generator of
 * injection slabs, item by item. first_step: the injection step index of the
 * next step (0 after a fresh load); it advances on the device. d = NULL
 * switches the inflow off. Do not mix with pic_inject_particles on one run
 * (their ids would collide). PIC_E_CAPACITY if a tile could not hold a full
 * load plus one step's inflow. */
typedef struct pic_inflow_desc {
  int32_t ppc;           /* particles per cell per species of the flow */
  double gamma0;         /* bulk Lorentz factor, > 1 (the flow moves towards -x) */
  double T;              /* rest-frame temperature (m c^2) */
  uint64_t seed;         /* Philox key (as for pic_load_plasma) */
  int64_t first_step;    /* injection step index of the next step */
} pic_inflow_desc;

int32_t pic_set_inflow(pic_ctx* ctx, int32_t run, const pic_inflow_desc* d);

/* Copy the particles of (run, species) to the host, with n_out = count (at
 * most cap), in ascending id order when ids are tracked (ids are load order,
 * then injection order; removed particles leave gaps), storage order
 * otherwise. Any output pointer may be NULL. */
int32_t pic_read_particles(pic_ctx* ctx, int32_t run, int32_t species, int64_t cap,
                           int32_t* ix, int32_t* iy, double* fx, double* fy, double* ux,
                           double* uy, double* uz, int64_t* n_out);

/* Field arrays of one run, [ny][nx] FP64 at their Yee positions. Setting E or B
 * also refreshes the FP32 copy used by the fast particle path. PIC_RHO is
 * computed on demand from the particles (read only). */
int32_t pic_set_field(pic_ctx* ctx, int32_t run, int32_t id, const double* host);
int32_t pic_get_field(pic_ctx* ctx, int32_t run, int32_t id, double* host);

/* Transverse average of a field of one run, profile(i) = (1/ny) sum_j f(i, j)
 * for i = 0 .. nx-1 (the x profiles of the shock runs, Sec. 4, Figs. 7c and
 * 8c: density and B_z averaged across the flow); host array of nx doubles.
 * Synchronises. */
int32_t pic_transverse_average(pic_ctx* ctx, int32_t run, int32_t id, double* host);

/* k-space diagnostic of the numerical Cherenkov instability (Sec. 3.1,
 * Fig. 3: B_z in Fourier space, with the resonance locus of Eq. (17)): the
 * power |F(kx, ky)|^2 / (nx ny)^2 of one field of a run (any field id), F(kx, ky) = sum_{i,j} f(i, j) exp(-2 pi i (kx i / nx + ky j / ny))
 * in FP64 on the device; host array [ny][nx] in discrete-Fourier-transform
 * order (index m for wavenumber 2 pi m / (n dx), m > n/2 aliased to m - n).
 * The staggering of a component changes only phases, not the power.
 * Synchronises. */
int32_t pic_field_spectrum(pic_ctx* ctx, int32_t run, int32_t id, double* host);

/* Split step, for parity checks. gather_push: gather, Boris push and move of
 * every particle of every run, keeping x^n (Sec. 1, Sec. 3). deposit:
 * Esirkepov deposit of J^{n+1/2} from x^n -> x^{n+1}, periodic wrap and tile
 * re-binning. field_solve: RHS of Eq. (7), CG for dB, update of Eqs. (5)-(6).
 * stats may be NULL or point at n_runs entries. */
int32_t pic_gather_push(pic_ctx* ctx);
int32_t pic_deposit(pic_ctx* ctx);
int32_t pic_field_solve(pic_ctx* ctx, pic_solve_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * field solve as pic_field_solve, with its scratch (CG vectors, per-block
 * partial sums, barrier words) in a device array of the library instead of
 * the context's workspace. The array holds a context of at most 262144 cells
 * over all runs and 4096 field-solve work-groups (about 57 MB per GPU, kept
 * until the process ends); larger contexts get PIC_E_INVAL. It calls no
 * device allocator. Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other contexts or threads) race. The plain CG starts
 * from x0 = 0 here (cg_x0 is not honoured); no event timing. */
int32_t pic_field_solve_noalloc(pic_ctx* ctx, pic_solve_stats* stats);

/* nsteps fused steps, each one time step n -> n+1 of the method as the paper
 * states it (Sec. 2, Eqs. (5)-(7): particles advanced with J^{n+1/2}
 * deposited, then the implicit solve; the PIC ingredients of Sec. 1 and
 * Sec. 3): gather+push+move+deposit in one kernel per tile, then re-binning,
 * the current reduction and the field solve. Equal to pic_gather_push,
 * pic_deposit, pic_field_solve in turn. Synchronises once at the end to
 * report overflow and CG status. last: NULL or n_runs entries.
 * With sort_every = K > 0, after the re-binning of every K-th step each
 * tile's particles are reordered: sorted by cell, then dealt out so that each
 * wavefront of the particle kernel takes 64 distinct cells spread over the
 * tile (the order the loaders produce; compaction mixes it step by step).
 * This changes storage order only; reads with track_ids return id order. */
int32_t pic_step(pic_ctx* ctx, int32_t nsteps, pic_solve_stats* last);

/* Diagnostics of one run (synchronises): the energy record of the last
 * recorded step, and from the current state the particle counts, Gauss's law
 * residual with rho deposited by the order-p shape, div B, the total charge
 * and the solve counters (the quantities by which the paper judges its runs:
 * energy conservation, Sec. 3.2; and the field energy whose growth measures
 * the numerical Cherenkov instability, Figs. 4-6). Returns PIC_E_NAN, with out
 * filled, if any field value, energy, residual or charge is not finite. */
int32_t pic_diag(pic_ctx* ctx, int32_t run, pic_diag_out* out);

/* History records collected every diag_every steps (oldest first). */
int32_t pic_history(pic_ctx* ctx, int32_t run, pic_diag_out* out, int32_t cap, int32_t* n_out);

/* Event timing per kernel class (on the context stream). */
int32_t pic_timing(pic_ctx* ctx, int32_t on);
int32_t pic_get_timing(pic_ctx* ctx, pic_timing_out* out);

/* ---- Learned CG aid (solver PIC_SOLVER_LEARNED_PCG; an addition to the
 * paper, which solves Eq. (7) by plain CG). A linear network N of three 3 x 3
 * periodic convolutions, 1 -> 32 -> 32 -> 1 channels (9792 FP32 weights,
 * layout W1[32][3][3], W2[32][32][3][3], W3[32][3][3], taps [dy][dx] with
 * offset (dx-1, dy-1)), approximates the inverse of Eq. (7)'s operator. Runs
 * that share dx, dy, cfl and theta share one network; each distinct operator
 * of the context has its own, trained on the pairs of the first run that uses
 * it. The field solve starts from x0 = N(b) and runs flexible PCG with z = N(r) to
 * cg_rtol; plain CG from the current iterate finishes any component that
 * misses it within learned_maxit, so the result always meets cg_rtol as plain
 * CG would. The weights start at the identity map plus small fixed noise. */
typedef struct pic_train_opts {
  int32_t epochs;        /* passes over the recorded pairs (>= 1) */
  double lr;             /* Adam step size; <= 0 picks 1e-3 */
  int32_t crop;          /* cells per side of the training window: 0 picks 64,
                            < 0 trains on whole fields, at most 128 */
} pic_train_opts;

typedef struct pic_train_stats {
  double loss_first;     /* mean of sum (N(b) - dB)^2 / sum dB^2 over the first epoch */
  double loss_last;      /* the same over the last epoch */
  int32_t samples;       /* (pair, component, network) samples per epoch */
  int32_t updates;       /* Adam updates made */
  int32_t networks;      /* networks trained (one per distinct operator) */
} pic_train_stats;

/* Record (b, dB) of each network's first run from every following field
 * solve (on != 0) into the network's ring of precond_slots pairs; n_pairs
 * (nullable) receives the number held per network. */
int32_t pic_precond_collect(pic_ctx* ctx, int32_t on, int32_t* n_pairs);

/* Train every network on its recorded pairs: per epoch one Adam update per
 * (pair, component) sample, oldest pair first, all in FP32 on the device;
 * then refresh the BF16 copies and collapsed filters. Each update sees one
 * crop x crop window of the sample (its corner a fixed hash of the update
 * count, the periodic field wrapped), with the loss on the window's cells
 * only; the network's 7 x 7 reach is inside the window plus a 3-cell halo,
 * so this is the exact loss of those cells. A window at least as large as the
 * field in both directions means the whole field. Synchronises. */
int32_t pic_precond_train(pic_ctx* ctx, const pic_train_opts* opts, pic_train_stats* out);

/* Use the learned path in the following field solves (on != 0, the default
 * for PIC_SOLVER_LEARNED_PCG) or plain CG (on == 0). */
int32_t pic_precond_use(pic_ctx* ctx, int32_t on);

/* Copy the FP32 weights of all networks out / in, network after network in
 * the order of their first runs (n must be 9792 x networks). set_weights
 * refreshes the derived BF16 copies and collapsed filters. */
int32_t pic_precond_get_weights(pic_ctx* ctx, float* host, size_t n);
int32_t pic_precond_set_weights(pic_ctx* ctx, const float* host, size_t n);

/* For parity checks. apply: d_out = N(d_in) on one nx x ny periodic FP64
 * device field ([ny][nx]) in the given form (PIC_NET_COLLAPSED or
 * PIC_NET_MFMA). grad: FP32 loss and weight gradient of one sample (d_b, d_t
 * device FP64 fields), host_grad receiving n = 9792 floats; window (nullable)
 * = {ox, oy, cx, cy} restricts it to the cx x cy cells from corner (ox, oy),
 * as training does (0 <= ox < nx, 0 <= oy < ny, 1 <= cx <= min(nx, 128),
 * 1 <= cy <= min(ny, 128)). Both use the first network (that of run 0), need
 * nx, ny >= 3 and, for whole fields, nx * ny no larger than the largest first
 * run's cell count, and synchronise. */
int32_t pic_precond_apply(pic_ctx* ctx, int32_t form, int32_t nx, int32_t ny, const double* d_in,
                          double* d_out);
int32_t pic_precond_grad(pic_ctx* ctx, int32_t nx, int32_t ny, const double* d_b,
                         const double* d_t, const int32_t* window, float* host_grad, size_t n,
                         double* loss);

/* ---- Autotuning of the launch schedule on a live context (the runs advance
 * by the timed steps). Work-groups per tile of the particle kernel and
 * work-groups of the persistent field solve are tried one after the other,
 * each for `steps` steps timed with events, and the fastest is kept (the two
 * kernels are independent). Tile shapes change the layout and are chosen by
 * building one context per shape (paper_1412_2480_amd.tune). */
typedef struct pic_tune_opts {
  int32_t steps;         /* timed steps per candidate, >= 1 */
  int32_t n_split;       /* 0: 1, 2, 4, 8 up to the planned tile_split */
  int32_t split[8];
  int32_t n_cg;          /* 0: 64, 128, 256, 512 up to the co-resident limit */
  int32_t cg_blocks[8];
} pic_tune_opts;

typedef struct pic_tune_out {
  int32_t tile_split;    /* chosen work-groups per tile */
  int32_t cg_blocks;     /* chosen field-solve work-groups (as launched) */
  int32_t n_split, n_cg; /* candidates tried */
  int32_t split[8], cg_blocks_tried[8];
  double particle_ms[8]; /* mean particle-kernel ms per step of each split candidate */
  double field_ms[8];    /* mean field-solve ms per step of each cg candidate */
} pic_tune_out;

int32_t pic_tune(pic_ctx* ctx, const pic_tune_opts* opts, pic_tune_out* out);

int32_t pic_sync(pic_ctx* ctx);
int32_t pic_destroy(pic_ctx* ctx);
const char* pic_last_error(const pic_ctx* ctx);
const char* pic_status_str(int32_t status);

#ifdef __cplusplus
}
#endif
#endif
