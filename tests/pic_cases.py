"""Shared set-up for parity tests: the same seeded synthetic load goes to the
FP64 oracle and to the GPU library (helper module, not a test file)."""
import numpy as np

import oracle
from synth import loads


def relerr(a, b):
    """normwise relative error ||a - b||_inf / ||b||_inf"""
    d = float(np.abs(np.asarray(a) - np.asarray(b)).max())
    s = float(np.abs(np.asarray(b)).max())
    return d / s if s > 0 else d


class Case:
    def __init__(self, nx, ny, order, ppc, gamma0=20.0, T=0.01, cfl=1.0, theta=0.6, seed=0,
                 dx=0.1, dy=None, field_amp=0.0, n_species=2, rtol=1e-8, maxit=200,
                 gather="nodal"):
        self.nx, self.ny, self.order, self.ppc = nx, ny, order, ppc
        self.gather = gather
        self.dx, self.dy = dx, (dx if dy is None else dy)
        self.cfl, self.theta, self.rtol, self.maxit = cfl, theta, rtol, maxit
        Q = loads.macro_charge(max(gamma0, 1.0), self.dx, self.dy, ppc)
        self.Q = Q
        sp = loads.pair_plasma(nx, ny, self.dx, self.dy, ppc, gamma0, T, seed)
        self.species = []
        for s in range(n_species):
            q = -Q if s == 0 else Q
            self.species.append(oracle.Particles.from_xy(sp[s]["x"], sp[s]["y"], sp[s]["ux"],
                                                         sp[s]["uy"], sp[s]["uz"], q, Q,
                                                         self.dx, self.dy))
        rng = np.random.default_rng(1000 + seed)
        self.fields = {k: field_amp * rng.standard_normal((ny, nx))
                       for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")}

    def species_desc(self):
        return [(p.q, p.m, self.ppc) for p in self.species]

    def oracle_sim(self, rtol=None):
        sim = oracle.Sim(self.nx, self.ny, self.dx, self.dy, self.cfl, self.theta, self.order,
                         [p.copy() for p in self.species],
                         rtol=self.rtol if rtol is None else rtol, maxit=self.maxit,
                         gather=self.gather)
        for k, n in enumerate(("Ex", "Ey", "Ez")):
            sim.E[k][...] = self.fields[n]
        for k, n in enumerate(("Bx", "By", "Bz")):
            sim.B[k][...] = self.fields[n]
        return sim

    def run_desc(self, rtol=None):
        import paper_1412_2480_amd as pic
        return pic.run_desc(self.nx, self.ny, self.dx, self.cfl, self.theta, self.order,
                            self.species_desc(), dy=self.dy,
                            cg_rtol=self.rtol if rtol is None else rtol, cg_maxit=self.maxit)

    def load_into(self, sim, run=0):
        for s, p in enumerate(self.species):
            sim.load_particles(run, s, p.ix, p.iy, p.fx, p.fy, p.ux, p.uy, p.uz)
        for n, a in self.fields.items():
            sim.set_field(run, n, a)

    def gpu_sim(self, precision="fp64", tile=(16, 16), rtol=None, **opt):
        import paper_1412_2480_amd as pic
        opt.setdefault("gather", self.gather)
        sim = pic.Sim([self.run_desc(rtol)], pic.make_options(precision, tile=tile, **opt))
        self.load_into(sim)
        return sim


def compare_particles(gpu, ref, nx, ny):
    """max position difference (cells, periodic) and relative momentum error"""
    X = gpu["ix"] + gpu["fx"]
    Y = gpu["iy"] + gpu["fy"]
    Xr = ref.ix + ref.fx
    Yr = ref.iy + ref.fy
    dxp = np.abs((X - Xr + nx / 2) % nx - nx / 2).max()
    dyp = np.abs((Y - Yr + ny / 2) % ny - ny / 2).max()
    u = np.stack([gpu["ux"], gpu["uy"], gpu["uz"]])
    ur = np.stack([ref.ux, ref.uy, ref.uz])
    return max(dxp, dyp), relerr(u, ur)
