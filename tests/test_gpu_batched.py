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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_runs_match_their_oracle_runs(precision):
    """Every run of the mixed 4-run context (uneven grids, orders 1-3, CFL
    0.5-1.0, theta 0.5/0.6) against its own FP64 oracle run after 4 steps:
    fields and particles at 1e-12 in the FP64 form (CG at rtol 1e-14), at
    FP32 roundoff bounds in the fast form."""
    import paper_1412_2480_amd as pic
    from pic_cases import compare_particles
    _say(f"batched vs oracle {precision}")
    cases = [Case(c["nx"], c["ny"], c["order"], c["ppc"], gamma0=5.0, T=0.05, cfl=c["cfl"],
                  theta=c["theta"], seed=c["seed"], field_amp=0.3, rtol=1e-14, maxit=500)
             for c in CASES]
    batched = pic.Sim([c.run_desc() for c in cases], pic.make_options(precision, tile=(16, 16)))
    for r, c in enumerate(cases):
        c.load_into(batched, run=r)
    batched.step(4)
    tol = 1e-12 if precision == "fp64" else 2e-5
    for r, c in enumerate(cases):
        ref = c.oracle_sim()
        for _ in range(4):
            ref.step()
        for k, n in enumerate(("Ex", "Ey", "Ez")):
            assert relerr(batched.get_field(r, n), ref.E[k]) <= tol, (r, n)
        for k, n in enumerate(("Bx", "By", "Bz")):
            assert relerr(batched.get_field(r, n), ref.B[k]) <= tol, (r, n)
        for s, p in enumerate(ref.species):
            g = batched.read_particles(r, s, p.n)
            pos, mom = compare_particles(g, p, c.nx, c.ny)
            assert pos <= tol and mom <= tol, (r, s, pos, mom)
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


def test_batched_learned_solver_one_network_per_operator():
    """The learned aid in a batched context whose runs use four operators
    (dx, dy, cfl, theta): one network each, trained on the pairs of the
    operator's first run (the fifth run shares the second run's network).
    After training every run reaches the plain-CG residual without the
    fallback, in fewer iterations over the batch, and its fields agree with
    plain CG's to the solver tolerance."""
    import paper_1412_2480_amd as pic
    _say("batched learned solver, four operators")
    specs = CASES + [dict(nx=48, ny=40, order=2, ppc=3, cfl=1.0, theta=0.6, seed=5)]
    cases = [Case(c["nx"], c["ny"], c["order"], c["ppc"], gamma0=20.0, T=0.01, cfl=c["cfl"],
                  theta=c["theta"], seed=c["seed"], rtol=1e-8) for c in specs]
    descs = [c.run_desc() for c in cases]
    a = pic.Sim(descs, pic.make_options("fp64", tile=(16, 16)))
    b = pic.Sim(descs, pic.make_options("fp64", tile=(16, 16), solver="learned",
                                        precond_slots=8))
    for r, c in enumerate(cases):
        c.load_into(a, run=r)
        c.load_into(b, run=r)
    b.precond_use(False)
    b.precond_collect(True)
    a.step(8)
    b.step(8)
    assert b.precond_collect(False) == 8
    tr = b.precond_train(epochs=20)
    _say(f"  training: {tr}")
    assert tr["networks"] == 4 and tr["samples"] == 8 * 3 * 4
    assert tr["loss_last"] < 0.1 * tr["loss_first"]
    w = b.get_weights(networks=4).reshape(4, -1)
    assert all(not np.array_equal(w[0], w[g]) for g in range(1, 4))
    b.precond_use(True)
    it_a = it_b = 0
    for step in range(6):
        sa = a.step(1)
        sb = b.step(1)
        for r in range(len(cases)):
            assert sb[r]["fallback"] == 0 and max(sb[r]["relres"]) <= 1e-8, (step, r)
            it_a += sum(sa[r]["iters"])
            it_b += sum(sb[r]["iters"])
    _say(f"  CG iterations over 6 steps: plain {it_a}, learned {it_b}")
    assert it_b < it_a
    for r in range(len(cases)):
        for n in NAMES[:6]:
            e = relerr(b.get_field(r, n), a.get_field(r, n))
            assert e <= 1e-6, (r, n, e)
    a.close()
    b.close()


def test_sweep_table_full_length():
    """The 48-run sweep at its full size and length (8-32 ppc/species, 500
    steps) in one context on the schedule the sweep benchmark uses (4 x 32
    tiles, reordering every 8 steps, slack 0.5): no tile overflows, every
    run keeps its particles, the last
    solve of every run meets the 1e-8 residual and the field energies stay
    finite."""
    import paper_1412_2480_amd as pic
    from synth import configs, loads
    table = configs.sweep_runs()
    descs = []
    for t in table:
        Q = loads.macro_charge(t["gamma0"], t["dx"], t["dx"], t["ppc"])
        descs.append(pic.run_desc(t["nx"], t["ny"], t["dx"], t["cfl"], t["theta"], t["order"],
                                  [(-Q, Q, t["ppc"]), (Q, Q, t["ppc"])], cg_rtol=1e-8))
    sim = pic.Sim(descs, pic.make_options("fp32", tile=(4, 32), tile_split=2, sort_every=8, slack=0.5, track_ids=False,
                                          graph=True))
    for r, t in enumerate(table):
        for s in range(2):
            sim.load_plasma(r, s, t["ppc"], t["gamma0"], t["T"], t["seed"])
    for chunk in range(5):
        st = sim.step(100)
        _say(f"  step {100 * (chunk + 1)}: max relres {max(max(x['relres']) for x in st):.1e}")
        assert all(max(x["relres"]) <= 1e-8 for x in st)
    for r, t in enumerate(table):
        d = sim.diag(r)
        n = t["nx"] * t["ny"] * t["ppc"]
        assert d["n_particles"][:2] == [n, n], r
        assert np.isfinite(d["W_E"]) and np.isfinite(d["W_B"]), r
    sim.close()
