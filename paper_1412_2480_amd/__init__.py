"""MI355X (gfx950) hot path of the implicit-FDTD relativistic PIC method of
Ikeya & Matsumoto, PASJ 2015 (arXiv:1412.2480).

This module is a thin ctypes binding of libpic.so (C-ABI in include/pic.h):
it only marshals arguments. PyTorch provides the device workspace and the
stream; every step of the method runs in the library's HIP kernels. There is
no CPU fallback: importing works without the library, but creating a Sim
raises if libpic.so is missing or no GPU is visible.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_MAX_SPECIES = 2
PIC_FP64, PIC_FP32_FAST = 0, 1
PIC_SOLVER_CG, PIC_SOLVER_LEARNED_PCG = 0, 1
PIC_NET_COLLAPSED, PIC_NET_MFMA = 0, 1
NET_NW = 9792
PIC_BC_PERIODIC, PIC_BC_SHOCK = 0, 1
PIC_X0_ZERO, PIC_X0_PREV = 0, 1
PIC_SCHEME_IMPLICIT, PIC_SCHEME_EXPLICIT = 0, 1
PIC_GATHER_NODAL, PIC_GATHER_STAGGERED = 0, 1
PIC_WALL_GAP = 4
FIELD_IDS = {"Ex": 0, "Ey": 1, "Ez": 2, "Bx": 3, "By": 4, "Bz": 5, "Jx": 6, "Jy": 7, "Jz": 8,
             "rho": 9, "n0": 10, "n1": 11}
PIC_E_NOCONV, PIC_E_CAPACITY, PIC_E_NAN = -4, -5, -6
STATUS = {0: "PIC_OK", -1: "PIC_E_INVAL", -2: "PIC_E_NOMEM", -3: "PIC_E_HIP",
          -4: "PIC_E_NOCONV", -5: "PIC_E_CAPACITY", -6: "PIC_E_NAN", -7: "PIC_E_STATE"}
EXPORTS = ["pic_plan", "pic_init", "pic_load_particles", "pic_load_plasma", "pic_inject_particles",
           "pic_set_inflow",
           "pic_read_particles", "pic_set_field", "pic_get_field", "pic_field_spectrum", "pic_transverse_average", "pic_gather_push",
           "pic_deposit", "pic_field_solve", "pic_field_solve_noalloc", "pic_step", "pic_diag", "pic_history",
           "pic_timing", "pic_get_timing", "pic_precond_collect", "pic_precond_train",
           "pic_precond_use", "pic_precond_get_weights", "pic_precond_set_weights",
           "pic_precond_apply", "pic_precond_grad", "pic_tune", "pic_sync", "pic_destroy",
           "pic_last_error", "pic_status_str"]


class SpeciesDesc(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("m", ctypes.c_double), ("ppc", ctypes.c_double)]


class RunDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("cfl", ctypes.c_double), ("theta", ctypes.c_double),
                ("shape_order", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("n_species", ctypes.c_int32),
                ("species", SpeciesDesc * PIC_MAX_SPECIES),
                ("cg_rtol", ctypes.c_double), ("cg_maxit", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("solver", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("slack", ctypes.c_double), ("exchange_frac", ctypes.c_double),
                ("diag_every", ctypes.c_int32), ("history_cap", ctypes.c_int32),
                ("cg_blocks", ctypes.c_int32), ("track_ids", ctypes.c_int32),
                ("tile_split", ctypes.c_int32), ("learned_form", ctypes.c_int32),
                ("learned_maxit", ctypes.c_int32), ("precond_slots", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("sort_every", ctypes.c_int32),
                ("cg_x0", ctypes.c_int32), ("field_scheme", ctypes.c_int32),
                ("gather", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_uint64), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("tile_slots", ctypes.c_int32 * PIC_MAX_SPECIES),
                ("exchange_slots", ctypes.c_int32), ("tile_split", ctypes.c_int32),
                ("particle_slots", ctypes.c_int64 * PIC_MAX_SPECIES),
                ("n_cells", ctypes.c_int64)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32 * 3), ("relres", ctypes.c_double * 3),
                ("bnorm", ctypes.c_double * 3), ("learned_iters", ctypes.c_int32 * 3),
                ("fallback", ctypes.c_int32), ("relres_recursive", ctypes.c_double * 3)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("lr", ctypes.c_double), ("crop", ctypes.c_int32)]


class TrainStats(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("samples", ctypes.c_int32), ("updates", ctypes.c_int32),
                ("networks", ctypes.c_int32)]


class PlasmaDesc(ctypes.Structure):
    _fields_ = [("ppc", ctypes.c_int32), ("x_cells", ctypes.c_int32), ("gamma0", ctypes.c_double),
                ("T", ctypes.c_double), ("direction", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class InflowDesc(ctypes.Structure):
    _fields_ = [("ppc", ctypes.c_int32), ("gamma0", ctypes.c_double), ("T", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("first_step", ctypes.c_int64)]


class TuneOpts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("n_split", ctypes.c_int32),
                ("split", ctypes.c_int32 * 8), ("n_cg", ctypes.c_int32),
                ("cg_blocks", ctypes.c_int32 * 8)]


class TuneOut(ctypes.Structure):
    _fields_ = [("tile_split", ctypes.c_int32), ("cg_blocks", ctypes.c_int32),
                ("n_split", ctypes.c_int32), ("n_cg", ctypes.c_int32),
                ("split", ctypes.c_int32 * 8), ("cg_blocks_tried", ctypes.c_int32 * 8),
                ("particle_ms", ctypes.c_double * 8), ("field_ms", ctypes.c_double * 8)]


class DiagOut(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double), ("W_E", ctypes.c_double),
                ("W_B", ctypes.c_double), ("W_K_minus", ctypes.c_double),
                ("W_K_plus", ctypes.c_double), ("cg_iters", ctypes.c_int32 * 3),
                ("cg_relres", ctypes.c_double * 3),
                ("n_particles", ctypes.c_int64 * PIC_MAX_SPECIES),
                ("gauss_max", ctypes.c_double), ("divb_max", ctypes.c_double),
                ("total_charge", ctypes.c_double), ("fallbacks", ctypes.c_int64),
                ("solves", ctypes.c_int64)]


class TimingOut(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 9), ("launches", ctypes.c_int64 * 9),
                ("graph_replays", ctypes.c_int64)]


TIMING_CLASSES = ["push", "deposit", "rebin", "current_sum", "rhs", "field_solve", "update", "diag",
                  "sort"]

_lib = None


def lib():
    """Load libpic.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        # torch first: its HIP runtime is then the one libpic.so binds to (the
        # same soname). Loaded the other way round, torch would bring a second
        # HIP/HSA runtime into the process and one of the two sees no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.pic_plan.argtypes = [P(RunDesc), ctypes.c_int32, P(Options), P(PlanInfo)]
        L.pic_init.argtypes = [P(RunDesc), ctypes.c_int32, P(Options), ctypes.c_void_p,
                               ctypes.c_size_t, ctypes.c_void_p, P(ctypes.c_void_p)]
        L.pic_load_particles.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64] + [ctypes.c_void_p] * 7
        L.pic_load_plasma.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                      P(PlasmaDesc)]
        L.pic_inject_particles.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int64] + [ctypes.c_void_p] * 7
        L.pic_set_inflow.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        L.pic_read_particles.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64] + [ctypes.c_void_p] * 7 + \
                                        [P(ctypes.c_int64)]
        L.pic_set_field.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_void_p]
        L.pic_get_field.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_void_p]
        L.pic_field_spectrum.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p]
        L.pic_transverse_average.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_void_p]
        L.pic_gather_push.argtypes = [ctypes.c_void_p]
        L.pic_deposit.argtypes = [ctypes.c_void_p]
        L.pic_field_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.pic_field_solve_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.pic_step.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        L.pic_diag.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(DiagOut)]
        L.pic_history.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_int32, P(ctypes.c_int32)]
        L.pic_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.pic_get_timing.argtypes = [ctypes.c_void_p, P(TimingOut)]
        L.pic_precond_collect.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_int32)]
        L.pic_precond_train.argtypes = [ctypes.c_void_p, P(TrainOpts), P(TrainStats)]
        L.pic_precond_use.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.pic_precond_get_weights.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
        L.pic_precond_set_weights.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
        L.pic_precond_apply.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        L.pic_precond_grad.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, P(ctypes.c_int32),
                                       ctypes.c_void_p, ctypes.c_size_t, P(ctypes.c_double)]
        L.pic_tune.argtypes = [ctypes.c_void_p, P(TuneOpts), P(TuneOut)]
        L.pic_sync.argtypes = [ctypes.c_void_p]
        L.pic_destroy.argtypes = [ctypes.c_void_p]
        L.pic_last_error.argtypes = [ctypes.c_void_p]
        L.pic_last_error.restype = ctypes.c_char_p
        L.pic_status_str.argtypes = [ctypes.c_int32]
        L.pic_status_str.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("pic_last_error", "pic_status_str"):
                getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def run_desc(nx, ny, dx, cfl, theta, order, species, dy=None, cg_rtol=1e-8, cg_maxit=200,
             bc="periodic"):
    """species: list of (q, m, ppc); bc: "periodic" or "shock"."""
    d = RunDesc()
    d.nx, d.ny = int(nx), int(ny)
    d.dx = float(dx)
    d.dy = float(dx if dy is None else dy)
    d.cfl, d.theta = float(cfl), float(theta)
    d.shape_order = int(order)
    d.bc = PIC_BC_SHOCK if bc in ("shock", PIC_BC_SHOCK) else PIC_BC_PERIODIC
    d.n_species = len(species)
    for k, (q, m, ppc) in enumerate(species):
        d.species[k].q, d.species[k].m, d.species[k].ppc = float(q), float(m), float(ppc)
    d.cg_rtol, d.cg_maxit = float(cg_rtol), int(cg_maxit)
    return d


def make_options(precision="fp64", tile=(16, 16), slack=0.25, exchange_frac=0.25,
                 diag_every=0, history_cap=1, cg_blocks=0, track_ids=True, tile_split=0,
                 solver="cg", learned_form="collapsed", learned_maxit=0, precond_slots=0,
                 graph=False, sort_every=0, cg_x0="zero", scheme="implicit", gather="nodal"):
    """solver: "cg" or "learned"; learned_form: "collapsed" or "mfma";
    cg_x0: "zero" or "prev" (plain CG from the previous step's dB);
    scheme: "implicit" (Eqs. (5)-(7)) or "explicit" (Yee FDTD, Eqs. (3)-(4));
    gather: "nodal" (momentum-conserving: fields averaged onto the charge nodes,
    the default) or "staggered" (each component from its own Yee points);
    exchange_frac: ignored by the library (kept in pic_options)."""
    o = Options()
    o.precision = PIC_FP32_FAST if precision in ("fp32", PIC_FP32_FAST) else PIC_FP64
    o.solver = PIC_SOLVER_LEARNED_PCG if solver in ("learned", PIC_SOLVER_LEARNED_PCG) \
        else PIC_SOLVER_CG
    o.learned_form = PIC_NET_MFMA if learned_form in ("mfma", PIC_NET_MFMA) \
        else PIC_NET_COLLAPSED
    o.learned_maxit = int(learned_maxit)
    o.precond_slots = int(precond_slots)
    o.graph = 1 if graph else 0
    o.sort_every = int(sort_every)
    o.cg_x0 = PIC_X0_PREV if cg_x0 in ("prev", PIC_X0_PREV) else PIC_X0_ZERO
    o.field_scheme = PIC_SCHEME_EXPLICIT if scheme in ("explicit", PIC_SCHEME_EXPLICIT) \
        else PIC_SCHEME_IMPLICIT
    if gather not in ("nodal", "staggered", PIC_GATHER_NODAL, PIC_GATHER_STAGGERED):
        raise ValueError(f"gather must be 'nodal' or 'staggered', not {gather!r}")
    o.gather = PIC_GATHER_STAGGERED if gather in ("staggered", PIC_GATHER_STAGGERED) \
        else PIC_GATHER_NODAL
    o.tile_x, o.tile_y = int(tile[0]), int(tile[1])
    o.slack, o.exchange_frac = float(slack), float(exchange_frac)
    o.diag_every, o.history_cap = int(diag_every), int(history_cap)
    o.cg_blocks = int(cg_blocks)
    o.track_ids = 1 if track_ids else 0
    o.tile_split = int(tile_split)
    return o


def plan(runs, options):
    arr = (RunDesc * len(runs))(*runs)
    info = PlanInfo()
    rc = lib().pic_plan(arr, len(runs), ctypes.byref(options), ctypes.byref(info))
    if rc != 0:
        raise PicError(rc, "pic_plan rejected the configuration")
    return info


def _ptr(a):
    return None if a is None else a.ctypes.data


# Contexts still open when the interpreter exits are destroyed by an exit
# handler, before the HIP runtime and any profiling tool attached to it tear
# down: a context left to the garbage collector at interpreter shutdown would
# otherwise release its graph execs and events after the runtime is gone.
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for s in list(_live):
        try:
            s.close()
        except Exception:
            pass


class Sim:
    """A context of one or more runs on the current torch CUDA (HIP) device."""

    def __init__(self, runs, options, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the PIC library has no CPU path")
        self.L = lib()
        self.runs = list(runs)
        self.options = options
        self.info = plan(self.runs, options)
        self.device = torch.device("cuda" if device is None else device)
        self.workspace = torch.empty(int(self.info.workspace_bytes), dtype=torch.uint8,
                                     device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        arr = (RunDesc * len(self.runs))(*self.runs)
        ctx = ctypes.c_void_p()
        rc = self.L.pic_init(arr, len(self.runs), ctypes.byref(options),
                             ctypes.c_void_p(self.workspace.data_ptr()),
                             int(self.info.workspace_bytes),
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if rc != 0:
            raise PicError(rc, f"pic_init failed: {self.L.pic_last_error(None).decode()}")
        self.ctx = ctx
        _live.add(self)

    def _check(self, rc, what, allow=()):
        if rc != 0 and rc not in allow:
            raise PicError(rc, f"{what}: {self.L.pic_last_error(self.ctx).decode()}")
        return rc

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.L.pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- data
    def load_particles(self, run, species, ix, iy, fx, fy, ux, uy, uz):
        a = [np.ascontiguousarray(v, dtype=t) for v, t in
             ((ix, np.int32), (iy, np.int32), (fx, np.float64), (fy, np.float64),
              (ux, np.float64), (uy, np.float64), (uz, np.float64))]
        n = a[0].size
        self._check(self.L.pic_load_particles(self.ctx, run, species, n, *[_ptr(v) for v in a]),
                    "load_particles")

    def load_plasma(self, run, species, ppc, gamma0, T, seed, direction=1, x_cells=0):
        """Seeded synthetic plasma generated on the device (pic_load_plasma)."""
        d = PlasmaDesc()
        d.ppc, d.x_cells, d.gamma0, d.T = int(ppc), int(x_cells), float(gamma0), float(T)
        d.direction, d.seed = int(direction), int(seed)
        self._check(self.L.pic_load_plasma(self.ctx, run, species, ctypes.byref(d)),
                    "load_plasma")

    def inject_particles(self, run, species, ix, iy, fx, fy, ux, uy, uz):
        a = [np.ascontiguousarray(v, dtype=t) for v, t in
             ((ix, np.int32), (iy, np.int32), (fx, np.float64), (fy, np.float64),
              (ux, np.float64), (uy, np.float64), (uz, np.float64))]
        self._check(self.L.pic_inject_particles(self.ctx, run, species, a[0].size,
                                                *[_ptr(v) for v in a]), "inject_particles")

    def set_inflow(self, run, ppc, gamma0, T, seed, first_step=0):
        """Device-generated inflow of a shock run before every step
        (pic_set_inflow); ppc=None switches it off."""
        if ppc is None:
            self._check(self.L.pic_set_inflow(self.ctx, run, None), "set_inflow")
            return
        d = InflowDesc()
        d.ppc, d.gamma0, d.T, d.seed, d.first_step = (int(ppc), float(gamma0), float(T),
                                                      int(seed), int(first_step))
        self._check(self.L.pic_set_inflow(self.ctx, run, ctypes.byref(d)), "set_inflow")

    def read_particles(self, run, species, cap):
        out = dict(ix=np.empty(cap, np.int32), iy=np.empty(cap, np.int32),
                   fx=np.empty(cap), fy=np.empty(cap), ux=np.empty(cap), uy=np.empty(cap),
                   uz=np.empty(cap))
        n = ctypes.c_int64(0)
        self._check(self.L.pic_read_particles(self.ctx, run, species, cap,
                                              *[_ptr(out[k]) for k in
                                                ("ix", "iy", "fx", "fy", "ux", "uy", "uz")],
                                              ctypes.byref(n)), "read_particles")
        return {k: v[:n.value] for k, v in out.items()}

    def get_field(self, run, name):
        d = self.runs[run]
        out = np.empty((d.ny, d.nx))
        self._check(self.L.pic_get_field(self.ctx, run, FIELD_IDS[name], _ptr(out)), "get_field")
        return out

    def spectrum(self, run, name):
        """|F(kx, ky)|^2 / (nx ny)^2 of one field ([ny][nx], DFT order)."""
        d = self.runs[run]
        out = np.empty((d.ny, d.nx))
        self._check(self.L.pic_field_spectrum(self.ctx, run, FIELD_IDS[name], _ptr(out)),
                    "field_spectrum")
        return out

    def transverse_average(self, run, name):
        """mean over y of one field: an x profile of nx values"""
        out = np.empty(self.runs[run].nx)
        self._check(self.L.pic_transverse_average(self.ctx, run, FIELD_IDS[name], _ptr(out)),
                    "transverse_average")
        return out

    def set_field(self, run, name, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        d = self.runs[run]
        assert a.shape == (d.ny, d.nx)
        self._check(self.L.pic_set_field(self.ctx, run, FIELD_IDS[name], _ptr(a)), "set_field")

    # ---- step calls
    def gather_push(self):
        self._check(self.L.pic_gather_push(self.ctx), "gather_push")

    def deposit(self):
        self._check(self.L.pic_deposit(self.ctx), "deposit")

    def _stats(self, st):
        return [dict(iters=list(s.iters), relres=list(s.relres), bnorm=list(s.bnorm),
                     learned_iters=list(s.learned_iters), fallback=s.fallback,
                     relres_recursive=list(s.relres_recursive)) for s in st]

    def field_solve(self, allow_noconv=False):
        st = (SolveStats * len(self.runs))()
        self._check(self.L.pic_field_solve(self.ctx, st), "field_solve",
                    allow=(-4,) if allow_noconv else ())
        return self._stats(st)

    def field_solve_noalloc(self, allow_noconv=False):
        """pic_field_solve_noalloc: the same solve with the library's static
        device scratch instead of the workspace (no device allocation)."""
        st = (SolveStats * len(self.runs))()
        self._check(self.L.pic_field_solve_noalloc(self.ctx, st), "field_solve_noalloc",
                    allow=(-4,) if allow_noconv else ())
        return self._stats(st)

    def step(self, n=1, allow_noconv=False):
        st = (SolveStats * len(self.runs))()
        self._check(self.L.pic_step(self.ctx, int(n), st), "step",
                    allow=(-4,) if allow_noconv else ())
        return self._stats(st)

    def step_async(self, n=1):
        """Enqueue n steps; returns the status without reading anything back
        except the end-of-call overflow and CG checks."""
        return self.L.pic_step(self.ctx, int(n), None)

    def sync(self):
        self._check(self.L.pic_sync(self.ctx), "sync")

    # ---- diagnostics
    @staticmethod
    def _rec(o):
        return dict(step=o.step, t=o.t, W_E=o.W_E, W_B=o.W_B, W_K_minus=o.W_K_minus,
                    W_K_plus=o.W_K_plus, cg_iters=list(o.cg_iters),
                    cg_relres=list(o.cg_relres), n_particles=list(o.n_particles))

    def diag_status(self, run=0):
        """(status, record) of pic_diag without raising on PIC_E_NAN."""
        o = DiagOut()
        rc = self._check(self.L.pic_diag(self.ctx, run, ctypes.byref(o)), "diag", allow=(-6,))
        r = self._rec(o)
        r.update(gauss_max=o.gauss_max, divb_max=o.divb_max, total_charge=o.total_charge,
                 fallbacks=o.fallbacks, solves=o.solves)
        return rc, r

    def diag(self, run=0):
        """pic_diag: the last energy record plus the current state's particle
        counts, Gauss residual, div B, total charge and solve counters."""
        o = DiagOut()
        self._check(self.L.pic_diag(self.ctx, run, ctypes.byref(o)), "diag")
        r = self._rec(o)
        r.update(gauss_max=o.gauss_max, divb_max=o.divb_max, total_charge=o.total_charge,
                 fallbacks=o.fallbacks, solves=o.solves)
        return r

    def history(self, run=0):
        cap = max(1, self.options.history_cap)
        out = (DiagOut * cap)()
        n = ctypes.c_int32(0)
        self._check(self.L.pic_history(self.ctx, run, out, cap, ctypes.byref(n)), "history")
        return [self._rec(out[k]) for k in range(n.value)]

    # ---- learned CG aid
    def precond_collect(self, on=True):
        n = ctypes.c_int32(0)
        self._check(self.L.pic_precond_collect(self.ctx, 1 if on else 0, ctypes.byref(n)),
                    "precond_collect")
        return n.value

    def precond_train(self, epochs=1, lr=0.0, crop=0):
        o = TrainOpts()
        o.epochs, o.lr, o.crop = int(epochs), float(lr), int(crop)
        st = TrainStats()
        self._check(self.L.pic_precond_train(self.ctx, ctypes.byref(o), ctypes.byref(st)),
                    "precond_train")
        return dict(loss_first=st.loss_first, loss_last=st.loss_last, samples=st.samples,
                    updates=st.updates, networks=st.networks)

    def precond_use(self, on=True):
        self._check(self.L.pic_precond_use(self.ctx, 1 if on else 0), "precond_use")

    def get_weights(self, networks=1):
        w = np.empty(NET_NW * networks, np.float32)
        self._check(self.L.pic_precond_get_weights(self.ctx, _ptr(w), w.size), "get_weights")
        return w

    def set_weights(self, w):
        a = np.ascontiguousarray(w, dtype=np.float32).ravel()
        self._check(self.L.pic_precond_set_weights(self.ctx, _ptr(a), a.size), "set_weights")

    def _device_field(self, a):
        import torch
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)

    def precond_apply(self, x, form="collapsed"):
        """N(x) for one [ny][nx] periodic field (host array in, host array out)."""
        xd = self._device_field(x)
        yd = torch_empty_like(xd)
        f = PIC_NET_MFMA if form in ("mfma", PIC_NET_MFMA) else PIC_NET_COLLAPSED
        ny, nx = xd.shape
        self.stream.synchronize()
        self._check(self.L.pic_precond_apply(self.ctx, f, nx, ny, ctypes.c_void_p(xd.data_ptr()),
                                             ctypes.c_void_p(yd.data_ptr())), "precond_apply")
        return yd.cpu().numpy()

    def precond_grad(self, b, t, window=None):
        """(loss, dL/dW) of one sample, L = sum (N(b) - t)^2 / sum t^2 over the
        field or over the window (ox, oy, cx, cy) of it."""
        bd, td = self._device_field(b), self._device_field(t)
        ny, nx = bd.shape
        g = np.empty(NET_NW, np.float32)
        loss = ctypes.c_double(0.0)
        win = None if window is None else (ctypes.c_int32 * 4)(*[int(v) for v in window])
        self.stream.synchronize()
        self._check(self.L.pic_precond_grad(self.ctx, nx, ny, ctypes.c_void_p(bd.data_ptr()),
                                            ctypes.c_void_p(td.data_ptr()), win, _ptr(g),
                                            NET_NW, ctypes.byref(loss)), "precond_grad")
        return loss.value, g

    def tune(self, steps=3, splits=(), cg_blocks=()):
        """Pick work-groups per tile and field-solve work-groups by timing
        `steps` real steps per candidate (pic_tune); returns the table."""
        o = TuneOpts()
        o.steps = int(steps)
        o.n_split = len(splits)
        for k, v in enumerate(splits):
            o.split[k] = int(v)
        o.n_cg = len(cg_blocks)
        for k, v in enumerate(cg_blocks):
            o.cg_blocks[k] = int(v)
        r = TuneOut()
        self._check(self.L.pic_tune(self.ctx, ctypes.byref(o), ctypes.byref(r)), "tune")
        return dict(tile_split=r.tile_split, cg_blocks=r.cg_blocks,
                    split_ms={r.split[k]: r.particle_ms[k] for k in range(r.n_split)},
                    cg_ms={r.cg_blocks_tried[k]: r.field_ms[k] for k in range(r.n_cg)})

    def timing(self, on=True):
        self._check(self.L.pic_timing(self.ctx, 1 if on else 0), "timing")

    def get_timing(self):
        t = TimingOut()
        self._check(self.L.pic_get_timing(self.ctx, ctypes.byref(t)), "get_timing")
        out = {name: dict(ms=t.ms[k], launches=t.launches[k])
               for k, name in enumerate(TIMING_CLASSES)}
        out["graph_replays"] = t.graph_replays
        return out


def torch_empty_like(t):
    import torch
    return torch.empty_like(t)


def exported_symbols():
    return list(EXPORTS)
