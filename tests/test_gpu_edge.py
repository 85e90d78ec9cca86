"""Degenerate inputs through the C-ABI against the FP64 oracle: a context
with no particles loaded (the field equations of Sec. 2 alone, Eqs. (5)-(7),
from nonzero fields; and with zero fields a zero right-hand side, which the
solve meets with no iterations), one species empty while the other is not,
particles at rest in zero fields (no current, nothing moves), and a batched
context one of whose runs holds no particles."""
import sys

import numpy as np
import pytest

import oracle
from pic_cases import Case, compare_particles, relerr

pytestmark = pytest.mark.gpu

EN, BN, JN = ("Ex", "Ey", "Ez"), ("Bx", "By", "Bz"), ("Jx", "Jy", "Jz")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _empty(p):
    """the species p with no particles (same charge and mass)"""
    z = np.zeros(0)
    return oracle.Particles(z.astype(np.int32), z.astype(np.int32), z, z, z, z, z, p.q, p.m)


def _fields_match(sim, ref, run=0, tol=1e-12):
    for k, n in enumerate(EN):
        assert relerr(sim.get_field(run, n), ref.E[k]) <= tol, n
    for k, n in enumerate(BN):
        assert relerr(sim.get_field(run, n), ref.B[k]) <= tol, n


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_no_particles_fields_alone(precision):
    """Nothing loaded: the step is the implicit field update with J = 0."""
    import paper_1412_2480_amd as pic
    _say(f"no particles, nonzero fields, {precision}")
    case = Case(40, 36, 3, ppc=2, field_amp=0.5, seed=4, rtol=1e-14, maxit=500)
    sim = pic.Sim([case.run_desc()], pic.make_options(precision, tile=(16, 16)))
    for n, a in case.fields.items():
        sim.set_field(0, n, a)
    ref = case.oracle_sim()
    ref.species = [_empty(p) for p in ref.species]
    for step in range(3):
        st = sim.step(1)[0]
        its = ref.step()["cg_iters"]
        for c in range(3):
            assert abs(st["iters"][c] - its[c]) <= 1, (step, c)
        for k, n in enumerate(JN):
            assert not np.any(sim.get_field(0, n)), (step, n)
        _fields_match(sim, ref)
    d = sim.diag(0)
    assert d["n_particles"][:2] == [0, 0] and d["total_charge"] == 0.0
    sim.close()


def test_no_particles_zero_fields():
    """A zero right-hand side: no CG iterations, the fields stay exactly zero."""
    import paper_1412_2480_amd as pic
    _say("no particles, zero fields")
    case = Case(34, 12, 1, ppc=2, field_amp=0.0, seed=2)
    for solver in ("cg", "learned"):
        sim = pic.Sim([case.run_desc()], pic.make_options("fp32", tile=(16, 16), solver=solver,
                                                         precond_slots=2))
        st = sim.step(2)[0]
        assert list(st["iters"]) == [0, 0, 0] and max(st["relres"]) == 0.0, solver
        for n in EN + BN + JN:
            assert not np.any(sim.get_field(0, n)), (solver, n)
        sim.close()


def test_one_species_empty_fp64():
    """Electrons loaded, positrons declared but empty: per-step parity."""
    _say("one species empty, fp64")
    case = Case(40, 36, 2, ppc=3, gamma0=5.0, T=0.05, field_amp=0.3, seed=6, rtol=1e-14,
                maxit=500)
    import paper_1412_2480_amd as pic
    sim = pic.Sim([case.run_desc()], pic.make_options("fp64", tile=(16, 16)))
    p = case.species[0]
    sim.load_particles(0, 0, p.ix, p.iy, p.fx, p.fy, p.ux, p.uy, p.uz)
    for n, a in case.fields.items():
        sim.set_field(0, n, a)
    ref = case.oracle_sim()
    ref.species[1] = _empty(ref.species[1])
    for step in range(2):
        sim.step(1)
        ref.step()
        g = sim.read_particles(0, 0, p.n)
        pos, mom = compare_particles(g, ref.species[0], case.nx, case.ny)
        assert pos <= 1e-12 and mom <= 1e-12, (step, pos, mom)
        assert len(sim.read_particles(0, 1, 4)["ix"]) == 0
        for k, n in enumerate(JN):
            assert relerr(sim.get_field(0, n), ref.J[k]) <= 1e-12, (step, n)
        _fields_match(sim, ref)
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_particles_at_rest(precision):
    """u = 0 in zero fields: no displacement, so every current node is
    exactly zero, the fields stay zero and the particles stay put."""
    import paper_1412_2480_amd as pic
    _say(f"particles at rest, {precision}")
    case = Case(34, 20, 3, ppc=4, gamma0=1.0, T=0.0, field_amp=0.0, seed=8)
    sim = pic.Sim([case.run_desc()], pic.make_options(precision, tile=(16, 16)))
    for s, p in enumerate(case.species):
        z = np.zeros(p.n)
        sim.load_particles(0, s, p.ix, p.iy, p.fx, p.fy, z, z, z)
    before = [sim.read_particles(0, s, p.n) for s, p in enumerate(case.species)]
    sim.step(2)
    for n in EN + BN + JN:
        assert not np.any(sim.get_field(0, n)), n
    for s, p in enumerate(case.species):
        g = sim.read_particles(0, s, p.n)
        for k in ("ix", "iy", "fx", "fy"):
            assert np.array_equal(g[k], before[s][k]), (s, k)
        for k in ("ux", "uy", "uz"):
            assert not np.any(g[k]), (s, k)
    sim.close()


def test_batched_context_with_an_empty_run():
    """Two runs in one context, the second with no particles: the first
    matches its own oracle run, the second evolves its fields alone."""
    import paper_1412_2480_amd as pic
    _say("batched context, second run empty")
    a = Case(40, 36, 2, ppc=3, gamma0=5.0, T=0.05, field_amp=0.3, seed=9, rtol=1e-14,
             maxit=500)
    b = Case(34, 12, 2, ppc=3, gamma0=5.0, T=0.05, field_amp=0.3, seed=10, rtol=1e-14,
             maxit=500)
    sim = pic.Sim([a.run_desc(), b.run_desc()], pic.make_options("fp64", tile=(16, 16)))
    a.load_into(sim, 0)
    for n, v in b.fields.items():
        sim.set_field(1, n, v)
    ra, rb = a.oracle_sim(), b.oracle_sim()
    rb.species = [_empty(p) for p in rb.species]
    for step in range(2):
        sim.step(1)
        ra.step()
        rb.step()
        for s, p in enumerate(ra.species):
            g = sim.read_particles(0, s, p.n)
            pos, mom = compare_particles(g, p, a.nx, a.ny)
            assert pos <= 1e-12 and mom <= 1e-12, (step, s)
        _fields_match(sim, ra, 0)
        _fields_match(sim, rb, 1)
        assert sim.diag(1)["n_particles"][:2] == [0, 0]
    sim.close()
