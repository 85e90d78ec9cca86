"""Boundary behaviour of the C-ABI on the GPU: the diagnostics record
(Gauss's law, div B, total charge, solve counters), the PIC_E_NAN path, the
true FP64 residual reported by the field solve (checked against the oracle's
operator of Eq. (7) on the fields read back), the warm-started plain CG, and
FP32 offsets that round up to 1 when loaded."""
import sys

import numpy as np
import pytest

import oracle
from pic_cases import Case, relerr

pytestmark = pytest.mark.gpu

EN = ("Ex", "Ey", "Ez")
BN = ("Bx", "By", "Bz")
JN = ("Jx", "Jy", "Jz")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_diag_fields_and_nan_status():
    import paper_1412_2480_amd as pic
    _say("diag fields and PIC_E_NAN")
    case = Case(40, 36, 2, ppc=3, gamma0=5.0, T=0.05, field_amp=0.0, seed=3)
    sim = case.gpu_sim("fp64", tile=(16, 16), diag_every=1, history_cap=4)
    sim.step(3)
    d = sim.diag(0)
    assert d["step"] == 2 and d["solves"] == 3 and d["fallbacks"] == 0
    assert d["n_particles"] == [case.species[0].n, case.species[1].n]
    # co-located pairs: rho = 0 at t = 0 and Gauss's law holds to roundoff after
    assert d["gauss_max"] < 1e-9 and d["divb_max"] < 1e-6
    # total charge: sum of q over both species (zero for the pair plasma), to
    # the roundoff of the node sums
    q = sum(p.q * p.n for p in case.species)
    assert abs(d["total_charge"] - q) <= 1e-12 * case.Q * case.species[0].n
    # a NaN set through pic_set_field is reported as PIC_E_NAN, with the record filled
    bz = sim.get_field(0, "Bz")
    bz[5, 7] = np.nan
    sim.set_field(0, "Bz", bz)
    rc, rec = sim.diag_status(0)
    assert rc == pic.PIC_E_NAN
    assert rec["n_particles"] == d["n_particles"]
    sim.close()


def test_single_species_total_charge():
    _say("total charge of one species")
    case = Case(34, 12, 3, ppc=2, gamma0=3.0, T=0.05, field_amp=0.0, seed=5, n_species=1)
    sim = case.gpu_sim("fp64", tile=(16, 16))
    d = sim.diag(0)
    p = case.species[0]
    assert abs(d["total_charge"] - p.q * p.n) <= 1e-12 * abs(p.q) * p.n
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_true_residual_against_the_operator(precision):
    """relres is ||b - A dB||/||b|| of the applied dB: recomputed on the host
    with the oracle's right-hand side and operator of Eq. (7) from E^n, B^n, J
    and dB = B^{n+1} - B^n read back."""
    _say(f"true residual {precision}")
    case = Case(40, 36, 3, ppc=3, gamma0=5.0, T=0.05, field_amp=0.3, seed=7, rtol=1e-8)
    sim = case.gpu_sim(precision, tile=(16, 16))
    sim.gather_push()
    sim.deposit()
    E0 = [sim.get_field(0, n) for n in EN]
    B0 = [sim.get_field(0, n) for n in BN]
    J = [sim.get_field(0, n) for n in JN]
    st = sim.field_solve()[0]
    B1 = [sim.get_field(0, n) for n in BN]
    nx, ny, dt = case.nx, case.ny, case.cfl * case.dx
    b = oracle.rhs(nx, ny, case.dx, case.dy, dt, case.theta, E0, B0, J)
    for c in range(3):
        db = B1[c] - B0[c]
        r = b[c] - oracle.apply_A(nx, ny, case.dx, case.dy, dt, case.theta, db)
        host = np.sqrt((r * r).sum() / (b[c] * b[c]).sum())
        assert st["relres"][c] <= case.rtol and st["relres_recursive"][c] <= case.rtol
        # B^{n+1} - B^n carries the rounding of B^{n+1} (|B| >> |dB| here)
        assert abs(host - st["relres"][c]) <= 1e-6 * case.rtol + 1e-13, (c, host, st["relres"][c])
    sim.close()


def test_warm_start_previous_db():
    """cg_x0 = prev: plain CG from the previous step's dB meets the same
    relative residual; the fields agree with the zero start to the solve
    tolerance (the iteration counts are printed)."""
    _say("cg_x0 prev")
    case = Case(64, 48, 2, ppc=4, gamma0=10.0, T=0.05, field_amp=0.1, seed=11, rtol=1e-10)
    sims = {x0: case.gpu_sim("fp64", tile=(16, 16), cg_x0=x0) for x0 in ("zero", "prev")}
    its = {x0: 0 for x0 in sims}
    for k in range(6):
        for x0, sim in sims.items():
            st = sim.step(1)[0]
            assert max(st["relres"]) <= case.rtol
            if k > 0:
                its[x0] += sum(st["iters"])
    _say(f"  CG iterations over steps 1-5: {its}")
    for n in EN + BN:
        a, b = sims["prev"].get_field(0, n), sims["zero"].get_field(0, n)
        assert relerr(a, b) <= 1e-7, n
    for sim in sims.values():
        sim.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_offset_rounding_up_keeps_cell_and_tile(precision):
    """An FP64 offset of 1 - 2^-26 rounds to 1 in FP32: it is clamped below 1,
    so the particle keeps its cell (the last cell of the last tile, whose
    neighbour across the periodic edge is tile 0). A step afterwards keeps
    Gauss's law and raises no tile overflow."""
    _say(f"offset clamp {precision}")
    import paper_1412_2480_amd as pic
    from synth import loads
    nx, ny, dx, ppc = 40, 36, 0.1, 1
    Q = loads.macro_charge(1.0, dx, dx, ppc)
    run = pic.run_desc(nx, ny, dx, 1.0, 0.6, 3, [(-Q, Q, ppc), (Q, Q, ppc)], cg_rtol=1e-12,
                       cg_maxit=400)
    sim = pic.Sim([run], pic.make_options(precision, tile=(16, 16)))
    f = 1.0 - 2.0 ** -26
    ix = np.array([nx - 1, 3], np.int32)
    iy = np.array([ny - 1, 5], np.int32)
    fx = np.array([f, 0.25])
    fy = np.array([f, f])
    u = np.array([0.3, -0.2])
    for s in range(2):
        sgn = 1.0 if s == 0 else -1.0   # the species separate: rho is not zero
        sim.load_particles(0, s, ix, iy, fx, fy, sgn * u, -sgn * u, 0.5 * u)
    for s in range(2):
        g = sim.read_particles(0, s, 2)
        assert list(g["ix"]) == [nx - 1, 3] and list(g["iy"]) == [ny - 1, 5]
        assert (g["fx"] < 1.0).all() and (g["fy"] < 1.0).all()
        assert abs(g["fx"][0] - f) <= 2.0 ** -23 and abs(g["fy"][1] - f) <= 2.0 ** -23
    sim.step(2)
    d = sim.diag(0)
    assert d["n_particles"] == [2, 2]
    scale = 4 * np.pi * Q / (dx * dx)   # 4 pi rho of one macro-particle on one node
    assert d["gauss_max"] <= (1e-5 if precision == "fp32" else 1e-11) * scale
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_species_density_and_transverse_average(precision):
    """PIC_N0/PIC_N1: a species' number density deposited with the order-p
    shape at the nodes, against the oracle's charge deposit of that species
    with unit charge; pic_transverse_average against the row mean of the
    field read back."""
    _say(f"species density {precision}")
    case = Case(40, 36, 3, ppc=3, gamma0=5.0, T=0.05, field_amp=0.2, seed=12)
    sim = case.gpu_sim(precision, tile=(16, 16))
    sim.step(2)
    tol = 1e-12 if precision == "fp64" else 1e-5
    for s, name in enumerate(("n0", "n1")):
        g = sim.read_particles(0, s, case.species[s].n)
        p = oracle.Particles(g["ix"], g["iy"], g["fx"], g["fy"], g["ux"], g["uy"], g["uz"], 1.0,
                             1.0)
        ref = oracle.charge(case.nx, case.ny, case.order, case.dx, case.dy, p)
        got = sim.get_field(0, name)
        assert relerr(got, ref) <= tol, name
        # the total is the particle count
        # the total is the particle count (FP32 weights: to their roundoff)
        assert abs(got.sum() * case.dx * case.dy - p.n) <= (1e-9 if precision == "fp64"
                                                            else 1e-6) * p.n
        prof = sim.transverse_average(0, name)
        assert np.allclose(prof, got.mean(axis=0), rtol=1e-13, atol=0)
    bz = sim.get_field(0, "Bz")
    assert np.allclose(sim.transverse_average(0, "Bz"), bz.mean(axis=0), rtol=1e-13,
                       atol=1e-18)
    sim.close()
