"""GPU parity: the HIP library (through its C-ABI) against the FP64 CPU oracle
on the same seeded inputs. Tolerances: FP64 form 1e-12 normwise relative per
kernel step (field solve compared at CG rtol 1e-14); FP32 form against the
FP64 oracle at bounds derived from FP32 rounding."""
import sys

import numpy as np
import pytest

from pic_cases import Case, compare_particles, relerr

pytestmark = pytest.mark.gpu

EN = ("Ex", "Ey", "Ez")
BN = ("Bx", "By", "Bz")
JN = ("Jx", "Jy", "Jz")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# grids with several tiles and ragged tails: 40 = 16+16+8, 34 = 16+18 (last
# tile absorbs a 2-cell tail), 12 < tile (single tile), 36 = 16+16+4
GRIDS = [(40, 36), (34, 12)]


@pytest.mark.parametrize("gather", ["nodal", "staggered"])
@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("grid", GRIDS)
def test_split_step_parity_fp64(order, grid, gather):
    nx, ny = grid
    _say(f"split parity fp64 order={order} grid={grid} gather={gather}")
    case = Case(nx, ny, order, ppc=3, gamma0=5.0, T=0.05, field_amp=0.5, seed=order,
                rtol=1e-14, maxit=500, gather=gather)
    sim = case.gpu_sim("fp64", tile=(16, 16))
    ref = case.oracle_sim()
    # gather + push + move
    sim.gather_push()
    wkm, wkp = 0.0, 0.0
    olds = []
    ref_f = []
    for p in ref.species:
        import oracle
        f = oracle.gather(nx, ny, order, ref.E + ref.B, p, gather)
        oracle.boris(p, ref.dt, f[0:3], f[3:6])
        olds.append(p.copy())
        oracle.move(p, ref.dt, ref.dx, ref.dy)
    for s, p in enumerate(ref.species):
        g = sim.read_particles(0, s, p.n)
        pos, mom = compare_particles(g, p, nx, ny)
        assert mom <= 1e-12, (s, mom)
        assert pos <= 1e-12, (s, pos)
    # deposit J^{n+1/2}
    sim.deposit()
    for a in ref.J:
        a[...] = 0.0
    for s, p in enumerate(ref.species):
        oracle.deposit(nx, ny, order, ref.dx, ref.dy, ref.dt, olds[s], p, ref.J)
        oracle.wrap(nx, ny, p)
    for k, n in enumerate(JN):
        e = relerr(sim.get_field(0, n), ref.J[k])
        assert e <= 1e-12, (n, e)
    # field solve (Eq. (7) by CG, then Eqs. (5)-(6))
    st = sim.field_solve()
    _, its, rels = ref.field_solve()
    for k, n in enumerate(EN):
        e = relerr(sim.get_field(0, n), ref.E[k])
        assert e <= 1e-12, (n, e)
    for k, n in enumerate(BN):
        e = relerr(sim.get_field(0, n), ref.B[k])
        assert e <= 1e-12, (n, e)
    for c in range(3):
        assert abs(st[0]["iters"][c] - its[c]) <= 1
    # particles after re-binning are the oracle's wrapped particles
    for s, p in enumerate(ref.species):
        g = sim.read_particles(0, s, p.n)
        pos, mom = compare_particles(g, p, nx, ny)
        assert pos <= 1e-12 and mom <= 1e-12
    sim.close()


@pytest.mark.parametrize("order", [1, 3])
def test_fused_step_equals_split(order):
    _say(f"fused vs split order={order}")
    case = Case(40, 36, order, ppc=3, gamma0=5.0, T=0.05, field_amp=0.5, seed=7, rtol=1e-13)
    a = case.gpu_sim("fp64")
    b = case.gpu_sim("fp64")
    a.step(1)
    b.gather_push()
    b.deposit()
    b.field_solve()
    for n in EN + BN + JN:
        assert relerr(a.get_field(0, n), b.get_field(0, n)) <= 1e-13, n
    for s in range(2):
        ga = a.read_particles(0, s, case.species[s].n)
        gb = b.read_particles(0, s, case.species[s].n)
        for k in ("ix", "iy"):
            assert np.array_equal(ga[k], gb[k])
        for k in ("fx", "fy", "ux", "uy", "uz"):
            assert np.abs(ga[k] - gb[k]).max() <= 1e-13 * max(1.0, np.abs(gb[k]).max())
    a.close()
    b.close()


def test_multistep_64x64_fp64_energy_history():
    """The 64x64 configuration (16 ppc/species, gamma0 = 20, T = 0.01, order 1,
    sigma = 1, theta = 0.6) for 12 steps: per-step energies and final fields."""
    _say("multistep 64x64 fp64")
    case = Case(64, 64, 1, ppc=16, gamma0=20.0, T=0.01, seed=0, rtol=1e-8)
    sim = case.gpu_sim("fp64", diag_every=1, history_cap=64)
    ref = case.oracle_sim()
    rec = [ref.step() for _ in range(12)]
    sim.step(12)
    hist = sim.history(0)
    assert len(hist) == 12
    for h, r in zip(hist, rec):
        assert h["step"] == r["step"]
        for key in ("W_K_minus", "W_K_plus"):
            assert abs(h[key] - r[key]) <= 1e-11 * abs(r[key]), key
        for key in ("W_E", "W_B"):
            assert abs(h[key] - r[key]) <= 1e-8 * max(abs(r[key]), 1e-300), (key, h[key], r[key])
    for k, n in enumerate(EN):
        assert relerr(sim.get_field(0, n), ref.E[k]) <= 1e-8, n
    for k, n in enumerate(BN):
        assert relerr(sim.get_field(0, n), ref.B[k]) <= 1e-8, n
    sim.close()


@pytest.mark.parametrize("gather", ["nodal", "staggered"])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_one_step_fp32_fast_form(order, gather):
    """FP32 particles (int cell + FP32 offset, FP32 current) against the FP64
    oracle after one step; bounds from FP32 rounding (unit roundoff 6e-8)."""
    _say(f"fp32 one step order={order} gather={gather}")
    case = Case(40, 36, order, ppc=4, gamma0=20.0, T=0.01, field_amp=0.5, seed=11,
                rtol=1e-12, gather=gather)
    import oracle
    sim = case.gpu_sim("fp32")
    ref = case.oracle_sim()
    # absolute current scale: the same deposit with |q| for every species, so
    # the electron and positron contributions add instead of cancelling
    jabs = [np.zeros((case.ny, case.nx)) for _ in range(3)]
    for p in ref.species:
        a = p.copy()
        f = oracle.gather(case.nx, case.ny, order, ref.E + ref.B, a, gather)
        oracle.boris(a, ref.dt, f[0:3], f[3:6])
        old = a.copy()
        oracle.move(a, ref.dt, ref.dx, ref.dy)
        a.q = abs(a.q)
        oracle.deposit(case.nx, case.ny, order, ref.dx, ref.dy, ref.dt, old, a, jabs)
    sim.step(1)
    ref.step()
    for s, p in enumerate(ref.species):
        g = sim.read_particles(0, s, p.n)
        pos, mom = compare_particles(g, p, case.nx, case.ny)
        assert pos <= 2e-6, (s, pos)
        assert mom <= 2e-6, (s, mom)
    # FP32 forms S0 and S1 separately, so DS = S1 - S0 carries an absolute
    # error of order u32 = 6e-8 whatever the displacement; the natural scale
    # is the current every particle would carry moving one full cell:
    # |q|/(dy dt) * (sum of node weights) for Jx (likewise Jy), and
    # |q| max|vz| * (sum of node weights)/(dx dy) for Jz.
    count = np.zeros((case.ny, case.nx))
    vzmax = 0.0
    for p in ref.species:
        a = p.copy()
        a.q = 1.0
        oracle.charge(case.nx, case.ny, order, 1.0, 1.0, a, count)
        vzmax = max(vzmax, float(np.abs(p.uz / np.sqrt(1 + p.ux ** 2 + p.uy ** 2 + p.uz ** 2)).max()))
    nmax = count.max()
    jscale = [case.Q / (case.dy * ref.dt) * nmax, case.Q / (case.dx * ref.dt) * nmax,
              case.Q * vzmax * nmax / (case.dx * case.dy)]
    for k, n in enumerate(JN):
        err = np.abs(sim.get_field(0, n) - ref.J[k]).max()
        _say(f"  {n}: err/scale = {err / jscale[k]:.3e}, err/|J|abs = "
             f"{err / np.abs(jabs[k]).max():.3e}")
        assert err <= 1e-6 * jscale[k], (n, err / jscale[k])
    escale = max(np.abs(ref.E[k]).max() for k in range(3))
    for k, n in enumerate(EN):
        err = np.abs(sim.get_field(0, n) - ref.E[k]).max()
        assert err <= 1e-5 * (escale + 4 * np.pi * ref.dt * jscale[k]), n
    bscale = max(np.abs(ref.B[k]).max() for k in range(3))
    for k, n in enumerate(BN):
        assert np.abs(sim.get_field(0, n) - ref.B[k]).max() <= 1e-5 * bscale, n
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_exchange_keeps_every_particle(precision):
    """Thirty steps of a gamma0 = 40 drift (about one cell per step in x): no
    particle is lost or duplicated moving between tiles, and positions follow
    the oracle."""
    _say(f"exchange {precision}")
    case = Case(48, 40, 2, ppc=4, gamma0=40.0, T=0.05, seed=3, rtol=1e-10)
    sim = case.gpu_sim(precision, tile=(8, 8))
    ref = case.oracle_sim(rtol=1e-10)
    sim.step(30)
    for _ in range(30):
        ref.step()
    tol = 1e-9 if precision == "fp64" else 1e-3
    for s, p in enumerate(ref.species):
        g = sim.read_particles(0, s, p.n)
        assert g["ix"].size == p.n
        assert g["ix"].min() >= 0 and g["ix"].max() < case.nx
        assert g["iy"].min() >= 0 and g["iy"].max() < case.ny
        pos, mom = compare_particles(g, p, case.nx, case.ny)
        assert pos <= tol and mom <= tol, (pos, mom)
    d = sim.diag(0)
    assert d["n_particles"][:2] == [case.species[0].n, case.species[1].n]
    sim.close()


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("tile", [(2, 8), (2, 2), (3, 5)])
def test_narrow_tiles_match_oracle(tile, order):
    """Tiles narrower than the current patch's guard (2 nodes below a tile, 3
    at and above its end): a node's current then comes from patches of tiles
    two or more tiles away, which the reduction must include. A gamma0 = 40
    drift moves every particle about one cell per step, so particles change
    tile every step; fields, currents and particles follow the oracle."""
    _say(f"narrow tiles {tile} order {order}")
    case = Case(40, 36, order, ppc=3, gamma0=40.0, T=0.05, field_amp=0.3, seed=11 + order,
                rtol=1e-14, maxit=500)
    sim = case.gpu_sim("fp64", tile=tile, tile_split=2, slack=1.0)
    ref = case.oracle_sim()
    g0 = sim.diag(0)["gauss_max"]
    for step in range(4):
        sim.step(1)
        ref.step()
        for k, n in enumerate(JN):
            e = relerr(sim.get_field(0, n), ref.J[k])
            assert e <= 1e-11, (step, n, e)
        for k, n in enumerate(EN + BN):
            a = ref.E[k] if k < 3 else ref.B[k - 3]
            e = relerr(sim.get_field(0, n), a)
            assert e <= 1e-11, (step, n, e)
    for s, p in enumerate(ref.species):
        g = sim.read_particles(0, s, p.n)
        pos, mom = compare_particles(g, p, case.nx, case.ny)
        assert pos <= 1e-11 and mom <= 1e-11, (s, pos, mom)
    # the Gauss residual of the random initial fields is carried unchanged
    scale = 4 * np.pi * case.Q / (case.dx * case.dy)
    assert abs(sim.diag(0)["gauss_max"] - g0) <= 1e-10 * scale
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gauss_law_constant_on_gpu(precision):
    """div E - 4 pi rho stays at its initial value (zero for the neutral load)
    up to FP64 roundoff in both forms: Esirkepov's J satisfies discrete
    continuity, and the FP32 form forms charge and current from the same
    unit-sum FP64 weights of its FP32 positions."""
    _say(f"gauss {precision}")
    case = Case(32, 32, 3, ppc=4, gamma0=20.0, T=0.01, seed=5, rtol=1e-6)
    sim = case.gpu_sim(precision)
    d0 = sim.diag(0)
    sim.step(10)
    d1 = sim.diag(0)
    scale = 4 * np.pi * case.Q / (case.dx * case.dy)
    tol = 1e-11
    assert d0["gauss_max"] <= tol * scale
    assert d1["gauss_max"] <= tol * scale, d1["gauss_max"] / scale
    sim.close()


def test_noconv_status_and_best_iterate():
    import paper_1412_2480_amd as pic
    _say("noconv")
    case = Case(24, 24, 2, ppc=2, gamma0=5.0, T=0.05, field_amp=0.5, seed=9, rtol=1e-12,
                maxit=1)
    sim = case.gpu_sim("fp64")
    with pytest.raises(pic.PicError) as ei:
        sim.step(1)
    assert ei.value.code == -4
    sim.close()


def test_capacity_and_state_errors():
    import paper_1412_2480_amd as pic
    _say("capacity/state")
    case = Case(24, 24, 2, ppc=4, gamma0=5.0, T=0.05, seed=2)
    sim = pic.Sim([case.run_desc()], pic.make_options("fp64", tile=(8, 8), slack=0.01))
    p = case.species[0]
    # eight times the density in one tile cannot fit its slots
    ix = np.full(p.n, 1, np.int32)
    iy = np.full(p.n, 1, np.int32)
    with pytest.raises(pic.PicError) as ei:
        sim.load_particles(0, 0, ix, iy, p.fx, p.fy, p.ux, p.uy, p.uz)
    assert ei.value.code == -5
    with pytest.raises(pic.PicError) as ei:
        sim.deposit()
    assert ei.value.code == -7
    with pytest.raises(pic.PicError) as ei:
        sim.field_solve()
    assert ei.value.code == -7
    sim.close()


def test_64x64_full_run_fp64():
    """The plain-method configuration at full length: 64x64, 16 ppc/species,
    gamma0 = 20, T = 0.01, order 1, sigma = 1, theta = 0.6, 200 steps, seed 0,
    FP64 on both sides. The two CG implementations stop at 1e-8 with different
    iterates, and the instability amplifies such differences, so the history is
    compared on the field energy relative to its running maximum and on the
    kinetic energy (measured: 3e-15 and 2e-14). The drifting beam loses total
    energy to the instability and the theta-damping (about 8% here), unlike the
    thermal plasma of Sec. 3 whose 1% bound the oracle tests pin; the drift is
    reported, and equal on both sides by the energy parity."""
    _say("64x64 full run, 200 steps fp64")
    case = Case(64, 64, 1, ppc=16, gamma0=20.0, T=0.01, seed=0, rtol=1e-8)
    sim = case.gpu_sim("fp64", diag_every=1, history_cap=256)
    ref = case.oracle_sim()
    rec = [ref.step() for _ in range(200)]
    sim.step(200)
    hist = sim.history(0)
    assert [h["step"] for h in hist] == list(range(200))
    wf = np.array([h["W_E"] + h["W_B"] for h in hist])
    wf_ref = np.array([r["W_E"] + r["W_B"] for r in rec])
    runmax = np.maximum.accumulate(wf_ref)
    ok = runmax > 0
    e = np.abs(wf - wf_ref)[ok] / runmax[ok]
    wk = np.array([h["W_K_plus"] for h in hist])
    wk_ref = np.array([r["W_K_plus"] for r in rec])
    ek = np.abs(wk - wk_ref).max() / np.abs(wk_ref).max()
    tot = wf + 0.5 * np.array([h["W_K_minus"] + h["W_K_plus"] for h in hist])
    drift = np.abs(tot - tot[0]).max() / tot[0]
    _say(f"64x64 200 steps: field-energy e max {e.max():.3e}, kinetic {ek:.3e}, "
         f"total-energy drift {drift:.3e}")
    assert e.max() <= 1e-10
    assert ek <= 1e-10
    sim.close()
