"""GPU parity of the shock set-up (PIC_BC_SHOCK: conducting walls in x,
specular reflection at x = 0, outflow and injection at x_out) against the
FP64 oracle on the same seeded inputs, including the injected flow."""
import sys

import numpy as np
import pytest

import oracle
from pic_cases import compare_particles, relerr
from synth import loads

pytestmark = pytest.mark.gpu

EN, BN, JN = ("Ex", "Ey", "Ez"), ("Bx", "By", "Bz"), ("Jx", "Jy", "Jz")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class Shock:
    def __init__(self, nx, ny, order, ppc, gamma0=5.0, T=0.05, cfl=1.0, theta=0.6, seed=0,
                 field_amp=0.0, rtol=1e-8, maxit=300, gather="nodal"):
        self.nx, self.ny, self.order, self.ppc = nx, ny, order, ppc
        self.gather = gather
        self.gamma0, self.T, self.cfl, self.theta, self.seed = gamma0, T, cfl, theta, seed
        self.rtol, self.maxit = rtol, maxit
        self.x_out = nx - oracle.WALL_GAP
        self.Q = loads.macro_charge(gamma0, 0.1, 0.1, ppc)
        self.load = loads.shock_load(self.x_out, ny, ppc, gamma0, T, seed)
        rng = np.random.default_rng(500 + seed)
        f = {k: field_amp * rng.standard_normal((ny, nx)) for k in EN + BN}
        # conductor nodes hold zero; Bx is made divergence-free from a stream
        # function that vanishes on both wall lines
        psi = field_amp * rng.standard_normal((ny, nx)) * 0.1
        psi[:, 0] = psi[:, nx - 1] = 0.0
        f["Bx"] = (np.roll(psi, -1, axis=0) - psi) / 0.1
        f["By"] = -(np.roll(psi, -1, axis=1) - psi) / 0.1
        f["Ey"][:, 0] = f["Ez"][:, 0] = 0.0
        for k in EN + ("By", "Bz"):
            f[k][:, nx - 1] = 0.0
        self.fields = f

    def injection(self, step):
        return loads.shock_injection(self.x_out, self.ny, self.ppc, self.gamma0, self.T,
                                     self.seed, step, self.cfl)

    def oracle_sim(self, rtol=None):
        sp = [oracle.Particles(d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"],
                               q, self.Q) for d, q in zip(self.load, (-self.Q, self.Q))]
        sim = oracle.Sim(self.nx, self.ny, 0.1, 0.1, self.cfl, self.theta, self.order, sp,
                         rtol=self.rtol if rtol is None else rtol, maxit=self.maxit, bc="shock",
                         gather=self.gather)
        for k, n in enumerate(EN):
            sim.E[k][...] = self.fields[n]
        for k, n in enumerate(BN):
            sim.B[k][...] = self.fields[n]
        return sim

    def gpu_sim(self, precision="fp64", rtol=None, **opt):
        import paper_1412_2480_amd as pic
        run = pic.run_desc(self.nx, self.ny, 0.1, self.cfl, self.theta, self.order,
                           [(-self.Q, self.Q, self.ppc), (self.Q, self.Q, self.ppc)],
                           cg_rtol=self.rtol if rtol is None else rtol, cg_maxit=self.maxit,
                           bc="shock")
        opt.setdefault("gather", self.gather)
        sim = pic.Sim([run], pic.make_options(precision, slack=2.0, **opt))
        for s, d in enumerate(self.load):
            sim.load_particles(0, s, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"],
                               d["uz"])
        for n, a in self.fields.items():
            sim.set_field(0, n, a)
        return sim


def _inject_both(case, step, gpu, ref):
    inj = case.injection(step)
    for s, d in enumerate(inj):
        if gpu is not None:
            gpu.inject_particles(0, s, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"],
                                 d["uz"])
        if ref is not None:
            ref.inject(s, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"])


@pytest.mark.parametrize("order,tile,gather",
                         [(1, (16, 16), "nodal"), (2, (16, 16), "nodal"), (3, (16, 16), "nodal"),
                          (2, (2, 8), "nodal"), (3, (2, 4), "nodal"),
                          (1, (16, 16), "staggered"), (3, (2, 4), "staggered")])
def test_shock_steps_match_oracle_fp64(order, tile, gather):
    """Split steps with reflection, outflow and injection against the oracle;
    the 2-cell-wide tiles put the wall's ghost columns and the patches that
    reach two tiles out through the current reduction."""
    _say(f"shock split steps vs oracle, order {order}, tile {tile}, gather {gather}")
    case = Shock(40, 20, order, ppc=3, seed=order, field_amp=0.3, rtol=1e-14, gather=gather)
    ref = case.oracle_sim()
    sim = case.gpu_sim("fp64", tile=tile)
    reflected = 0
    for step in range(4):
        _inject_both(case, step, sim, ref)
        sim.gather_push()
        sim.deposit()
        sim.field_solve()
        before = [p.ux.copy() for p in ref.species]
        ref.step()
        for s, p in enumerate(ref.species):
            g = sim.read_particles(0, s, p.n + 10)
            assert len(g["ix"]) == p.n, (step, s)
            pos, mom = compare_particles(g, p, case.nx, case.ny)
            assert pos <= 1e-12 and mom <= 1e-12, (step, s, pos, mom)
        reflected += sum(int(np.sum(u < 0)) for u in before) - sum(
            int(np.sum(p.ux < 0)) for p in ref.species)
        for k, n in enumerate(JN):
            assert relerr(sim.get_field(0, n), ref.J[k]) <= 1e-12, (step, n)
        for k, n in enumerate(EN):
            assert relerr(sim.get_field(0, n), ref.E[k]) <= 1e-12, (step, n)
        for k, n in enumerate(BN):
            assert relerr(sim.get_field(0, n), ref.B[k]) <= 1e-12, (step, n)
    assert reflected > 0   # the wall was exercised
    sim.close()


def test_shock_fused_equals_split():
    _say("shock fused == split")
    case = Shock(48, 24, 2, ppc=4, seed=5, field_amp=0.2)
    a = case.gpu_sim("fp64")
    b = case.gpu_sim("fp64")
    for step in range(5):
        _inject_both(case, step, a, None)
        _inject_both(case, step, b, None)
        a.step(1)
        b.gather_push()
        b.deposit()
        b.field_solve()
    for n in EN + BN:
        assert relerr(a.get_field(0, n), b.get_field(0, n)) <= 1e-13, n
    for s in range(2):
        ga = a.read_particles(0, s, 1 << 20)
        gb = b.read_particles(0, s, 1 << 20)
        assert len(ga["ix"]) == len(gb["ix"])
        for k in ("ix", "iy"):
            assert np.array_equal(ga[k], gb[k])
        for k in ("fx", "fy", "ux", "uy", "uz"):
            assert np.abs(ga[k] - gb[k]).max() <= 1e-13
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shock_run_keeps_gauss_law(precision):
    """Co-located pairs start and enter with zero charge density, so with a
    charge-conserving deposit the Gauss residual stays at roundoff between the
    wall line and the outflow region."""
    _say(f"shock run Gauss law, {precision}")
    case = Shock(96, 32, 2, ppc=8, gamma0=20.0, T=0.01)
    sim = case.gpu_sim(precision)
    for step in range(40):
        _inject_both(case, step, sim, None)
        st = sim.step(1)
        assert max(st[0]["relres"]) <= case.rtol
    d = sim.diag(0)
    rho_scale = 4 * np.pi * case.Q / (0.1 * 0.1)     # one particle per cell
    tol = (1e-10 if precision == "fp64" else 1e-4) * rho_scale
    assert d["gauss_max"] <= tol, d["gauss_max"]
    n0 = case.x_out * case.ny * case.ppc
    for s in range(2):
        assert 0.8 * n0 <= d["n_particles"][s] <= 2.5 * n0
    sim.close()


@pytest.mark.parametrize("form", ["collapsed", "mfma"])
def test_shock_learned_solver(form):
    """The learned aid on a walled run: trained on the run's own pairs, it
    reaches the plain-CG residual without the fallback in fewer iterations,
    and its fields agree with plain CG's to the solver tolerance."""
    _say(f"shock run with the learned solver ({form})")
    case = Shock(96, 32, 2, ppc=8, gamma0=20.0, T=0.01)
    a = case.gpu_sim("fp64")
    b = case.gpu_sim("fp64", solver="learned", learned_form=form, precond_slots=8)
    b.precond_use(False)
    b.precond_collect(True)
    for step in range(8):
        _inject_both(case, step, a, None)
        _inject_both(case, step, b, None)
        a.step(1)
        b.step(1)
    assert b.precond_collect(False) == 8
    tr = b.precond_train(epochs=20)
    assert tr["loss_last"] < 0.1 * tr["loss_first"]
    b.precond_use(True)
    for step in range(8, 14):
        _inject_both(case, step, a, None)
        _inject_both(case, step, b, None)
        sa = a.step(1)[0]
        sb = b.step(1)[0]
        assert sb["fallback"] == 0 and max(sb["relres"]) <= case.rtol
        assert sum(sb["iters"]) < sum(sa["iters"])
    for n in EN + BN:
        assert relerr(b.get_field(0, n), a.get_field(0, n)) <= 1e-6, n
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_device_inflow_matches_host_slabs(precision):
    """pic_set_inflow generates on the device, before every step, the flow
    that the seeded host slab generator produces for that step, item by item
    (ids = item numbers, so in id order the newest particles are the slab in
    its order). Each step's injected particles are compared after the push of
    that step with the host slab pushed by the oracle's gather, Boris and move
    on the same fields (read back before the step)."""
    _say(f"device inflow vs host slabs, {precision}")
    import paper_1412_2480_amd as pic
    case = Shock(40, 24, 2, ppc=5, gamma0=20.0, T=0.01, seed=7)
    run = pic.run_desc(case.nx, case.ny, 0.1, case.cfl, case.theta, case.order,
                       [(-case.Q, case.Q, case.ppc), (case.Q, case.Q, case.ppc)], bc="shock")
    # no initial load: every particle of the run comes from the inflow
    sim = pic.Sim([run], pic.make_options(precision, slack=2.0))
    sim.set_inflow(0, case.ppc, case.gamma0, case.T, case.seed)
    # FP64: transcendental functions of the momentum draw differ in the last
    # bits between the device and numpy; FP32: the particle precision
    tol = 1e-13 if precision == "fp64" else 4e-6
    dt = 0.1 * case.cfl
    for step in range(6):
        n_before = [sim.diag(0)["n_particles"][s] for s in range(2)]
        F = [sim.get_field(0, n) for n in EN + BN]
        sim.gather_push()          # the injection of this step comes first
        inj = case.injection(step)
        for s in range(2):
            d = inj[s]
            p = oracle.Particles(d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"],
                                 (-1) ** (s + 1) * case.Q, case.Q)
            if precision == "fp32":
                for k in ("fx", "fy", "ux", "uy", "uz"):
                    setattr(p, k, getattr(p, k).astype(np.float32).astype(np.float64))
            f = oracle.gather_wall(case.nx, case.ny, case.order, F, p)
            oracle.boris(p, dt, f[0:3], f[3:6])
            oracle.move(p, dt, 0.1, 0.1)
            g = sim.read_particles(0, s, 1 << 16)
            assert g["ix"].size == n_before[s] + p.n, (step, s)
            new = {k: v[n_before[s]:] for k, v in g.items()}
            X = new["ix"] + new["fx"] - (p.ix + p.fx)
            Y = new["iy"] + new["fy"] - (p.iy + p.fy)
            assert np.abs(X).max() <= tol * case.nx and np.abs(Y).max() <= tol * case.ny, step
            for k in ("ux", "uy", "uz"):
                ref = getattr(p, k)
                assert np.abs(new[k] - ref).max() <= tol * max(1.0, np.abs(ref).max()), (step, k)
        sim.deposit()
        sim.field_solve()
    sim.close()


def test_device_inflow_run_matches_oracle_fp64():
    """A walled run whose flow enters through the device inflow equals the
    oracle run fed with the host slabs, step by step (FP64 form, 1e-12)."""
    _say("device inflow run vs oracle")
    case = Shock(40, 20, 2, ppc=3, seed=2, field_amp=0.3, rtol=1e-14)
    ref = case.oracle_sim()
    sim = case.gpu_sim("fp64")
    sim.set_inflow(0, case.ppc, case.gamma0, case.T, case.seed)
    for step in range(6):
        _inject_both(case, step, None, ref)
        sim.step(1)
        ref.step()
        for s, p in enumerate(ref.species):
            g = sim.read_particles(0, s, p.n + 10)
            assert len(g["ix"]) == p.n, (step, s)
            pos, mom = compare_particles(g, p, case.nx, case.ny)
            assert pos <= 1e-12 and mom <= 1e-12, (step, s, pos, mom)
        for k, n in enumerate(EN):
            assert relerr(sim.get_field(0, n), ref.E[k]) <= 1e-12, (step, n)
    sim.close()


def test_device_inflow_graph_replay_equals_plain():
    """Graph replay of steps with the device inflow (the step counter lives on
    the device) equals plain launches."""
    _say("device inflow with graphs")
    case = Shock(48, 24, 2, ppc=4, gamma0=20.0, T=0.01, seed=3)
    a = case.gpu_sim("fp32", graph=True, sort_every=3)
    b = case.gpu_sim("fp32", graph=False, sort_every=3)
    for sim in (a, b):
        sim.set_inflow(0, case.ppc, case.gamma0, case.T, case.seed)
    a.step(12)
    b.step(12)
    assert a.get_timing()["graph_replays"] > 0
    for n in EN + BN:
        assert relerr(a.get_field(0, n), b.get_field(0, n)) <= 1e-12, n
    for s in range(2):
        ga = a.read_particles(0, s, 1 << 20)
        gb = b.read_particles(0, s, 1 << 20)
        assert len(ga["ix"]) == len(gb["ix"])
        # the current sums may add in another order (LDS atomics): FP32 roundoff
        X = ga["ix"] + ga["fx"] - gb["ix"] - gb["fx"]
        Y = ga["iy"] + ga["fy"] - gb["iy"] - gb["fy"]
        assert np.abs(X).max() <= 1e-5 and np.abs((Y + 12) % 24 - 12).max() <= 1e-5
        assert np.abs(ga["ux"] - gb["ux"]).max() <= 1e-5 * np.abs(gb["ux"]).max()
    a.close()
    b.close()
