"""FP64 CPU oracle of the paper's implicit-FDTD PIC step (Ikeya & Matsumoto,
PASJ 2015, arXiv:1412.2480).

TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users. The GPU library never imports it, and it
imports nothing from the GPU package.

The arithmetic lives in oracle.c (plain C, FP64); this module marshals numpy
arrays and strings the per-step functions together in the paper's order:
gather -> push -> move -> deposit J^{n+1/2} -> wrap -> RHS of Eq. (7) ->
CG for dB -> update of Eqs. (5)-(6).

Numerical helpers that are closed forms (exact FFT solve of Eq. (7), the
dispersion relation Eq. (10) and its printed forms) are in spectral.py; the
growth-rate fit of the magnetic-energy history is in growth.py.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)
_DP = ctypes.POINTER(_D)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(
                os.path.join(_build.HERE, "oracle.c")):
            _build.build()
        L = ctypes.CDLL(path)
        L.ora_shape.restype = ctypes.c_double
        L.ora_shape.argtypes = [ctypes.c_int, ctypes.c_double]
        L.ora_cg.restype = ctypes.c_int
        L.ora_kinetic.restype = ctypes.c_double
        _lib = L
    return _lib


def set_threads(n):
    """OpenMP threads of the oracle's loops (results depend on the count only
    through the fixed order of the per-thread partial sums)."""
    lib().ora_set_threads(int(n))


def get_threads():
    return int(lib().ora_get_threads())


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _i(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I)


def _dpp(arrs):
    ptrs = (_D * len(arrs))(*[_d(a) for a in arrs])
    return ctypes.cast(ptrs, _DP)


def shape(order, d):
    return lib().ora_shape(int(order), float(d))


WALL_GAP = 4   # particles leave shock runs at x >= (nx - WALL_GAP) dx


class Particles:
    """One species: cell index + in-cell offset, momentum u = gamma v, and an
    id per particle (load order, then injection order; kept sorted)."""

    def __init__(self, ix, iy, fx, fy, ux, uy, uz, q, m, ids=None):
        self.ix = np.array(ix, dtype=np.int32, copy=True, order="C")
        self.iy = np.array(iy, dtype=np.int32, copy=True, order="C")
        self.fx = np.array(fx, dtype=np.float64, copy=True, order="C")
        self.fy = np.array(fy, dtype=np.float64, copy=True, order="C")
        self.ux = np.array(ux, dtype=np.float64, copy=True, order="C")
        self.uy = np.array(uy, dtype=np.float64, copy=True, order="C")
        self.uz = np.array(uz, dtype=np.float64, copy=True, order="C")
        self.q = float(q)
        self.m = float(m)
        self.ids = (np.arange(self.ix.size, dtype=np.int64) if ids is None
                    else np.array(ids, dtype=np.int64, copy=True))

    @classmethod
    def from_xy(cls, x, y, ux, uy, uz, q, m, dx, dy):
        X = np.asarray(x, dtype=np.float64) / dx
        Y = np.asarray(y, dtype=np.float64) / dy
        ix = np.floor(X)
        iy = np.floor(Y)
        return cls(ix.astype(np.int32), iy.astype(np.int32), X - ix, Y - iy, ux, uy, uz, q, m)

    @property
    def n(self):
        return self.ix.size

    def copy(self):
        return Particles(self.ix.copy(), self.iy.copy(), self.fx.copy(), self.fy.copy(),
                         self.ux.copy(), self.uy.copy(), self.uz.copy(), self.q, self.m,
                         self.ids.copy())

    def select(self, keep):
        """drop the particles with keep == 0 (order kept)"""
        keep = np.asarray(keep, dtype=bool)
        for name in ("ix", "iy", "fx", "fy", "ux", "uy", "uz", "ids"):
            setattr(self, name, np.ascontiguousarray(getattr(self, name)[keep]))

    def append(self, ix, iy, fx, fy, ux, uy, uz, first_id):
        n = len(ix)
        self.ix = np.concatenate([self.ix, np.asarray(ix, np.int32)])
        self.iy = np.concatenate([self.iy, np.asarray(iy, np.int32)])
        self.fx = np.concatenate([self.fx, np.asarray(fx, np.float64)])
        self.fy = np.concatenate([self.fy, np.asarray(fy, np.float64)])
        self.ux = np.concatenate([self.ux, np.asarray(ux, np.float64)])
        self.uy = np.concatenate([self.uy, np.asarray(uy, np.float64)])
        self.uz = np.concatenate([self.uz, np.asarray(uz, np.float64)])
        self.ids = np.concatenate([self.ids, first_id + np.arange(n, dtype=np.int64)])

    def x(self, dx):
        return (self.ix + self.fx) * dx

    def y(self, dy):
        return (self.iy + self.fy) * dy


GATHER_MODES = ("nodal", "staggered")


def gather(nx, ny, order, fields6, p, mode="nodal"):
    """E, B at the particles: "nodal" (the method's momentum-conserving
    interpolation: fields averaged onto the charge nodes, then the
    charge-assignment weights) or "staggered" (each component from its own
    Yee points)."""
    assert mode in GATHER_MODES
    out = np.zeros(6 * p.n)
    fn = lib().ora_gather_nodal if mode == "nodal" else lib().ora_gather
    fn(nx, ny, order, _dpp(fields6), ctypes.c_int64(p.n), _i(p.ix), _i(p.iy),
       _d(p.fx), _d(p.fy), _d(out))
    return out.reshape(6, p.n)


def boris(p, dt, e3, b3):
    e3 = np.ascontiguousarray(e3, dtype=np.float64)
    b3 = np.ascontiguousarray(b3, dtype=np.float64)
    lib().ora_boris(ctypes.c_int64(p.n), ctypes.c_double(p.q * dt / (2.0 * p.m)), _d(e3), _d(b3),
                    _d(p.ux), _d(p.uy), _d(p.uz))


def move(p, dt, dx, dy):
    lib().ora_move(ctypes.c_int64(p.n), ctypes.c_double(dt), ctypes.c_double(dx),
                   ctypes.c_double(dy), _d(p.ux), _d(p.uy), _d(p.uz), _i(p.ix), _i(p.iy),
                   _d(p.fx), _d(p.fy))


def deposit(nx, ny, order, dx, dy, dt, old, new, j3):
    lib().ora_deposit(nx, ny, order, ctypes.c_double(dx), ctypes.c_double(dy),
                      ctypes.c_double(dt), ctypes.c_double(new.q), ctypes.c_int64(new.n),
                      _i(old.ix), _i(old.iy), _d(old.fx), _d(old.fy),
                      _i(new.ix), _i(new.iy), _d(new.fx), _d(new.fy),
                      _d(new.ux), _d(new.uy), _d(new.uz), _d(j3[0]), _d(j3[1]), _d(j3[2]))


def wrap(nx, ny, p):
    lib().ora_wrap_periodic(nx, ny, ctypes.c_int64(p.n), _i(p.ix), _i(p.iy))


def rhs(nx, ny, dx, dy, dt, theta, e3, b3, j3):
    out = [np.zeros((ny, nx)) for _ in range(3)]
    lib().ora_rhs(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy), ctypes.c_double(dt),
                  ctypes.c_double(theta), _dpp(e3), _dpp(b3), _dpp(j3), _dpp(out))
    return out


def apply_A(nx, ny, dx, dy, dt, theta, x):
    y = np.zeros((ny, nx))
    lib().ora_apply_A(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy), ctypes.c_double(dt),
                      ctypes.c_double(theta), _d(np.ascontiguousarray(x, dtype=np.float64)),
                      _d(y))
    return y


def cg(nx, ny, dx, dy, dt, theta, b, rtol=1e-8, maxit=200, x0=None):
    """Plain CG for Eq. (7); returns (x, iterations, true relative residual)."""
    x = np.zeros((ny, nx)) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    rel = ctypes.c_double(0.0)
    it = lib().ora_cg(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy), ctypes.c_double(dt),
                      ctypes.c_double(theta), _d(np.ascontiguousarray(b, dtype=np.float64)),
                      _d(x), ctypes.c_double(rtol), int(maxit), ctypes.byref(rel))
    return x, it, rel.value


def update(nx, ny, dx, dy, dt, theta, e3, b3, db3, j3):
    lib().ora_update(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy), ctypes.c_double(dt),
                     ctypes.c_double(theta), _dpp(e3), _dpp(b3), _dpp(db3), _dpp(j3))


def update_explicit(nx, ny, dx, dy, dt, e3, b3, j3):
    """Explicit FDTD advance of Eqs. (3)-(4) in place (B at integer times)."""
    lib().ora_update_explicit(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy),
                              ctypes.c_double(dt), _dpp(e3), _dpp(b3), _dpp(j3))


def charge(nx, ny, order, dx, dy, p, rho=None):
    rho = np.zeros((ny, nx)) if rho is None else rho
    lib().ora_charge(nx, ny, order, ctypes.c_double(dx), ctypes.c_double(dy),
                     ctypes.c_double(p.q), ctypes.c_int64(p.n), _i(p.ix), _i(p.iy),
                     _d(p.fx), _d(p.fy), _d(rho))
    return rho


def div_e(nx, ny, dx, dy, ex, ey):
    out = np.zeros((ny, nx))
    lib().ora_div_e(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy), _d(ex), _d(ey), _d(out))
    return out


def div_b(nx, ny, dx, dy, bx, by):
    out = np.zeros((ny, nx))
    lib().ora_div_b(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy), _d(bx), _d(by), _d(out))
    return out


# ---- shock set-up: conducting walls at x = 0 and x = (nx-1) dx, reflection
# at x = 0, outflow/injection at x = (nx - WALL_GAP) dx (see oracle.h)
def gather_wall(nx, ny, order, fields6, p, mode="nodal"):
    assert mode in GATHER_MODES
    out = np.zeros(6 * p.n)
    fn = lib().ora_gather_nodal_wall if mode == "nodal" else lib().ora_gather_wall
    fn(nx, ny, order, _dpp(fields6), ctypes.c_int64(p.n), _i(p.ix), _i(p.iy), _d(p.fx),
       _d(p.fy), _d(out))
    return out.reshape(6, p.n)


def deposit_wall(nx, ny, order, dx, dy, dt, old, new, j3):
    lib().ora_deposit_wall(nx, ny, order, ctypes.c_double(dx), ctypes.c_double(dy),
                           ctypes.c_double(dt), ctypes.c_double(new.q), ctypes.c_int64(new.n),
                           _i(old.ix), _i(old.iy), _d(old.fx), _d(old.fy),
                           _i(new.ix), _i(new.iy), _d(new.fx), _d(new.fy),
                           _d(new.ux), _d(new.uy), _d(new.uz), _d(j3[0]), _d(j3[1]), _d(j3[2]))


def mask_wall_currents(nx, ny, j3):
    lib().ora_mask_wall_currents(nx, ny, _d(j3[0]), _d(j3[1]), _d(j3[2]))


def boundary_wall(nx, ny, p):
    """reflect at x = 0, drop particles at or beyond the outflow line, wrap y;
    returns the number removed"""
    keep = np.zeros(p.n, dtype=np.uint8)
    lib().ora_boundary_wall(nx, ny, ctypes.c_int64(p.n), _i(p.ix), _i(p.iy), _d(p.fx),
                            _d(p.ux), keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    removed = int(p.n - keep.sum())
    if removed:
        p.select(keep)
    return removed


def rhs_wall(nx, ny, dx, dy, dt, theta, e3, b3, j3):
    out = [np.zeros((ny, nx)) for _ in range(3)]
    lib().ora_rhs_wall(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy), ctypes.c_double(dt),
                       ctypes.c_double(theta), _dpp(e3), _dpp(b3), _dpp(j3), _dpp(out))
    return out


def apply_A_wall(nx, ny, dx, dy, dt, theta, c, x):
    y = np.zeros((ny, nx))
    lib().ora_apply_A_wall(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy),
                           ctypes.c_double(dt), ctypes.c_double(theta), int(c),
                           _d(np.ascontiguousarray(x, dtype=np.float64)), _d(y))
    return y


def cg_wall(nx, ny, dx, dy, dt, theta, c, b, rtol=1e-8, maxit=200):
    x = np.zeros((ny, nx))
    rel = ctypes.c_double(0.0)
    it = lib().ora_cg_wall(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy),
                           ctypes.c_double(dt), ctypes.c_double(theta), int(c),
                           _d(np.ascontiguousarray(b, dtype=np.float64)), _d(x),
                           ctypes.c_double(rtol), int(maxit), ctypes.byref(rel))
    return x, it, rel.value


def update_wall(nx, ny, dx, dy, dt, theta, e3, b3, db3, j3):
    lib().ora_update_wall(nx, ny, ctypes.c_double(dx), ctypes.c_double(dy),
                          ctypes.c_double(dt), ctypes.c_double(theta), _dpp(e3), _dpp(b3),
                          _dpp(db3), _dpp(j3))


def charge_wall(nx, ny, order, dx, dy, p, rho=None):
    rho = np.zeros((ny, nx)) if rho is None else rho
    lib().ora_charge_wall(nx, ny, order, ctypes.c_double(dx), ctypes.c_double(dy),
                          ctypes.c_double(p.q), ctypes.c_int64(p.n), _i(p.ix), _i(p.iy),
                          _d(p.fx), _d(p.fy), _d(rho))
    return rho


def kinetic(p):
    return lib().ora_kinetic(ctypes.c_int64(p.n), ctypes.c_double(p.m), _d(p.ux), _d(p.uy),
                             _d(p.uz))


class Sim:
    """One run of the scheme, step n -> n+1 in the paper's order.

    State: E^n, B^n (6 arrays [ny][nx]); per species x^n, u^{n-1/2}.
    After step(): J holds J^{n+1/2} of the step just taken, `last` holds that
    step's record (energies, CG iterations and residuals).
    bc: "periodic" (both directions) or "shock" (walls in x, see oracle.h).
    scheme: "implicit" (Eqs. (5)-(7), the paper's solver) or "explicit"
    (the Yee FDTD of Eqs. (3)-(4), periodic only; theta is not used).
    gather: "nodal" (the method's momentum-conserving interpolation) or
    "staggered" (the alternative reading, see gather()).
    """

    def __init__(self, nx, ny, dx, dy, cfl, theta, order, species, rtol=1e-8, maxit=200,
                 bc="periodic", scheme="implicit", gather="nodal"):
        self.nx, self.ny, self.dx, self.dy = nx, ny, float(dx), float(dy)
        self.dt = cfl * dx        # sigma = c dt/dx with c = 1 (Sec. 3.1)
        self.theta, self.order = float(theta), int(order)
        self.species = species
        self.rtol, self.maxit = rtol, maxit
        assert bc in ("periodic", "shock")
        assert scheme in ("implicit", "explicit")
        assert scheme == "implicit" or bc == "periodic"
        self.bc = bc
        self.scheme = scheme
        assert gather in GATHER_MODES
        self.gather = gather
        self.next_id = [p.n for p in species]
        self.E = [np.zeros((ny, nx)) for _ in range(3)]
        self.B = [np.zeros((ny, nx)) for _ in range(3)]
        self.J = [np.zeros((ny, nx)) for _ in range(3)]
        self.n = 0
        self.last = None

    def field_energy(self):
        cell = self.dx * self.dy / (8.0 * np.pi)
        we = sum(float(np.sum(a * a)) for a in self.E) * cell
        wb = sum(float(np.sum(a * a)) for a in self.B) * cell
        return we, wb

    def inject(self, s, ix, iy, fx, fy, ux, uy, uz):
        """append particles to species s (ids continue the species' count)"""
        self.species[s].append(ix, iy, fx, fy, ux, uy, uz, self.next_id[s])
        self.next_id[s] += len(ix)

    def push_deposit(self):
        """Gather, Boris, move, Esirkepov deposit and boundaries for every species."""
        nx, ny, dx, dy, dt = self.nx, self.ny, self.dx, self.dy, self.dt
        wall = self.bc == "shock"
        for a in self.J:
            a[...] = 0.0
        wk_minus = wk_plus = 0.0
        for p in self.species:
            wk_minus += kinetic(p)
            f = (gather_wall if wall else gather)(nx, ny, self.order, self.E + self.B, p,
                                                  self.gather)
            boris(p, dt, f[0:3], f[3:6])
            wk_plus += kinetic(p)
            old = p.copy()
            move(p, dt, dx, dy)
            if wall:
                deposit_wall(nx, ny, self.order, dx, dy, dt, old, p, self.J)
                boundary_wall(nx, ny, p)
            else:
                deposit(nx, ny, self.order, dx, dy, dt, old, p, self.J)
                wrap(nx, ny, p)
        if wall:
            mask_wall_currents(nx, ny, self.J)
        return wk_minus, wk_plus

    def field_solve(self, x0=None):
        nx, ny, dx, dy, dt, th = self.nx, self.ny, self.dx, self.dy, self.dt, self.theta
        if self.scheme == "explicit":
            B0 = [a.copy() for a in self.B]
            update_explicit(nx, ny, dx, dy, dt, self.E, self.B, self.J)
            return [b - a for a, b in zip(B0, self.B)], [0, 0, 0], [0.0, 0.0, 0.0]
        wall = self.bc == "shock"
        b = (rhs_wall if wall else rhs)(nx, ny, dx, dy, dt, th, self.E, self.B, self.J)
        db, its, rels = [], [], []
        for c in range(3):
            if wall:
                x, it, rel = cg_wall(nx, ny, dx, dy, dt, th, c, b[c], self.rtol, self.maxit)
            else:
                x, it, rel = cg(nx, ny, dx, dy, dt, th, b[c], self.rtol, self.maxit,
                                None if x0 is None else x0[c])
            db.append(x)
            its.append(it)
            rels.append(rel)
        (update_wall if wall else update)(nx, ny, dx, dy, dt, th, self.E, self.B, db, self.J)
        return db, its, rels

    def step(self):
        we, wb = self.field_energy()
        wkm, wkp = self.push_deposit()
        _, its, rels = self.field_solve()
        self.last = dict(step=self.n, W_E=we, W_B=wb, W_K_minus=wkm, W_K_plus=wkp,
                         cg_iters=its, cg_relres=rels)
        self.n += 1
        return self.last

    def rho(self):
        r = np.zeros((self.ny, self.nx))
        for p in self.species:
            (charge_wall if self.bc == "shock" else charge)(self.nx, self.ny, self.order,
                                                             self.dx, self.dy, p, r)
        return r

    def gauss_residual(self):
        return div_e(self.nx, self.ny, self.dx, self.dy, self.E[0], self.E[1]) - 4.0 * np.pi * self.rho()
