"""Batching: several uneven runs in one context (one launch per kernel for all
runs) give the same results as each run alone."""
import sys

import numpy as np
import pytest

from pic_cases import Case, relerr

pytestmark = pytest.mark.gpu

NAMES = ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz")


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


CASES = [
    dict(nx=40, ny=36, order=1, ppc=3, cfl=0.5, theta=0.5, seed=1),
    dict(nx=64, ny=32, order=3, ppc=2, cfl=1.0, theta=0.6, seed=2),
    dict(nx=34, ny=24, order=2, ppc=4, cfl=0.8, theta=0.6, seed=3),
    dict(nx=16, ny=48, order=3, ppc=3, cfl=0.7, theta=0.5, seed=4),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_equals_unbatched(precision):
    import paper_1412_2480_amd as pic
    _say(f"batched vs unbatched {precision}")
    cases = [Case(c["nx"], c["ny"], c["order"], c["ppc"], gamma0=5.0, T=0.05, cfl=c["cfl"],
                  theta=c["theta"], seed=c["seed"], field_amp=0.3, rtol=1e-12) for c in CASES]
    opts = pic.make_options(precision, tile=(16, 16))
    batched = pic.Sim([c.run_desc() for c in cases], opts)
    for r, c in enumerate(cases):
        c.load_into(batched, run=r)
    batched.step(4)
    tol = 1e-11 if precision == "fp64" else 1e-5
    for r, c in enumerate(cases):
        alone = c.gpu_sim(precision, tile=(16, 16))
        alone.step(4)
        for n in NAMES:
            e = relerr(batched.get_field(r, n), alone.get_field(0, n))
            assert e <= tol, (r, n, e)
        for s in range(2):
            a = batched.read_particles(r, s, c.species[s].n)
            b = alone.read_particles(0, s, c.species[s].n)
            assert np.array_equal(a["ix"], b["ix"]) and np.array_equal(a["iy"], b["iy"])
            for k in ("fx", "fy", "ux", "uy", "uz"):
                assert np.abs(a[k] - b[k]).max() <= tol * max(1.0, np.abs(b[k]).max()), (r, k)
        alone.close()
    batched.close()


def test_sweep_table_runs_in_one_context():
    """The 48-run sweep table (uneven grids 128x64 ... 512x128, orders 1-3,
    CFL 0.5-1.0, theta 0.5/0.6), reduced to 4 ppc and 3 steps, runs in one
    context; every run keeps its particles and its CG converges."""
    import paper_1412_2480_amd as pic
    from synth import configs, loads
    _say("sweep table")
    table = configs.sweep_runs()
    descs, loads_ = [], []
    for t in table:
        Q = loads.macro_charge(t["gamma0"], t["dx"], t["dx"], t["ppc"])
        descs.append(pic.run_desc(t["nx"], t["ny"], t["dx"], t["cfl"], t["theta"], t["order"],
                                  [(-Q, Q, 4), (Q, Q, 4)], cg_rtol=1e-8))
    sim = pic.Sim(descs, pic.make_options("fp32", tile=(16, 16)))
    counts = []
    for r, t in enumerate(table):
        ld = loads.pair_plasma_cells(t["nx"], t["ny"], 4, t["gamma0"], t["T"], t["seed"])
        for s in range(2):
            d = ld[s]
            sim.load_particles(r, s, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"])
        counts.append(d["ix"].size)
    st = sim.step(3)
    for r in range(len(table)):
        assert max(st[r]["relres"]) <= 1e-8
        d = sim.diag(r)
        assert d["n_particles"][:2] == [counts[r], counts[r]]
    sim.close()
