"""Parity at full size on outputs the FP64 oracle can compute piecewise.

* The benchmark workload (periodic 1024 x 256, pair plasma at gamma0 = 40,
  64 particles/cell/species, cubic shape, CFL 1, theta 0.6, FP32 particle
  path, in the launch configurations bench.py's tuner picks among: 2 x 64
  and 4 x 32 tiles, two work-groups per tile, particles reordered by cell
  (here every 2 steps, so that the measured step starts from a reordered
  store and ends with a reordering), slack 0.5; and 16 x 32 tiles, one
  work-group per tile, without reordering): a sample of
  particles pushed one by one, the
  current on sampled node boxes from the particles that can reach them, and
  the field solve on the whole grid from the GPU's own current.
* The shock workload (4096 x 512 with walls, flow at gamma0 = 40 towards the
  wall, 32 particles/cell/species, order 2, CFL 1, theta 0.6, FP32 particles,
  learned CG aid trained on the run's own first pairs): properties that hold
  at any size (conductor nodes, Gauss's law in the interior, particle
  bookkeeping with injection and outflow, learned solves at the plain-CG
  residual)."""
import sys

import numpy as np
import pytest

import oracle
from pic_cases import relerr

pytestmark = pytest.mark.gpu

NX, NY, PPC, G0, ORDER, DX = 1024, 256, 64, 40.0, 3, 0.1


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("tile,split,sort_every,slack",
                         [((2, 64), 2, 2, 0.5), ((4, 32), 2, 2, 0.5), ((16, 32), 1, 0, 0.25)])
def test_fullsize_fp32_step_sampled_parity(tile, split, sort_every, slack):
    import paper_1412_2480_amd as pic
    from synth import loads
    _say(f"fullsize: generating load (tile {tile}, sort_every {sort_every})")
    Q = loads.macro_charge(G0, DX, DX, PPC)
    ld = loads.pair_plasma_cells(NX, NY, PPC, G0, 0.01, seed=0)
    run = pic.run_desc(NX, NY, DX, 1.0, 0.6, ORDER, [(-Q, Q, PPC), (Q, Q, PPC)], cg_rtol=1e-8)
    sim = pic.Sim([run], pic.make_options("fp32", tile=tile, tile_split=split,
                                          sort_every=sort_every, slack=slack))
    for s in range(2):
        d = ld[s]
        sim.load_particles(0, s, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"])
    n = NX * NY * PPC
    del ld
    _say("fullsize: 3 warm steps")
    sim.step(3)   # fields grow from noise so the push below is not trivial
    F0 = {k: sim.get_field(0, k) for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")}
    P0 = [sim.read_particles(0, s, n) for s in range(2)]
    _say("fullsize: one measured step")
    sim.step(1)
    J1 = [sim.get_field(0, k) for k in ("Jx", "Jy", "Jz")]
    F1 = {k: sim.get_field(0, k) for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")}
    P1 = [sim.read_particles(0, s, n) for s in range(2)]
    sim.close()
    dt = DX
    # the GPU gathers from an FP32 copy of the FP64 fields
    fields32 = [F0[k].astype(np.float32).astype(np.float64)
                for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")]
    rng = np.random.default_rng(0)

    # ---- sampled particles pushed one by one
    for s, q in enumerate((-Q, Q)):
        idx = rng.choice(n, 4000, replace=False)
        p = oracle.Particles(P0[s]["ix"][idx], P0[s]["iy"][idx], P0[s]["fx"][idx],
                             P0[s]["fy"][idx], P0[s]["ux"][idx], P0[s]["uy"][idx],
                             P0[s]["uz"][idx], q, Q)
        f = oracle.gather(NX, NY, ORDER, fields32, p)
        oracle.boris(p, dt, f[0:3], f[3:6])
        oracle.move(p, dt, DX, DX)
        oracle.wrap(NX, NY, p)
        u = np.stack([P1[s]["ux"][idx], P1[s]["uy"][idx], P1[s]["uz"][idx]])
        ur = np.stack([p.ux, p.uy, p.uz])
        mom = np.abs(u - ur).max() / np.abs(ur).max()
        X = P1[s]["ix"][idx] + P1[s]["fx"][idx]
        Xr = p.ix + p.fx
        pos = np.abs((X - Xr + NX / 2) % NX - NX / 2).max()
        _say(f"  species {s}: momentum err {mom:.2e}, position err {pos:.2e} cells")
        assert mom <= 2e-6 and pos <= 1e-5

    # ---- current on sampled 8x8 node boxes from every particle within reach
    jscale = None
    for b in range(4):
        i0 = int(rng.integers(8, NX - 16))
        j0 = int(rng.integers(8, NY - 16))
        Jr = [np.zeros((NY, NX)) for _ in range(3)]
        count = np.zeros((NY, NX))
        for s, q in enumerate((-Q, Q)):
            sel = ((P0[s]["ix"] >= i0 - 5) & (P0[s]["ix"] < i0 + 13) &
                   (P0[s]["iy"] >= j0 - 5) & (P0[s]["iy"] < j0 + 13))
            p = oracle.Particles(*(P0[s][k][sel] for k in ("ix", "iy", "fx", "fy", "ux", "uy",
                                                            "uz")), q, Q)
            f = oracle.gather(NX, NY, ORDER, fields32, p)
            oracle.boris(p, dt, f[0:3], f[3:6])
            old = p.copy()
            oracle.move(p, dt, DX, DX)
            oracle.deposit(NX, NY, ORDER, DX, DX, dt, old, p, Jr)
            one = old.copy()
            one.q = 1.0
            oracle.charge(NX, NY, ORDER, 1.0, 1.0, one, count)
        nmax = count[j0:j0 + 8, i0:i0 + 8].max()
        jscale = [Q / (DX * dt) * nmax, Q / (DX * dt) * nmax, Q * nmax / (DX * DX)]
        for c in range(3):
            err = np.abs(J1[c][j0:j0 + 8, i0:i0 + 8] - Jr[c][j0:j0 + 8, i0:i0 + 8]).max()
            _say(f"  box {b} J{'xyz'[c]}: err/scale {err / jscale[c]:.2e}")
            assert err <= 1e-6 * jscale[c]

    # ---- field solve on the whole grid, from the GPU's current, in FP64
    ref = oracle.Sim(NX, NY, DX, DX, 1.0, 0.6, ORDER, [], rtol=1e-8)
    for k, name in enumerate(("Ex", "Ey", "Ez")):
        ref.E[k][...] = F0[name]
    for k, name in enumerate(("Bx", "By", "Bz")):
        ref.B[k][...] = F0[name]
    for c in range(3):
        ref.J[c][...] = J1[c]
    ref.field_solve()
    for k, name in enumerate(("Ex", "Ey", "Ez")):
        e = relerr(F1[name] - F0[name], ref.E[k] - F0[name])
        _say(f"  {name} increment relerr {e:.2e}")
        assert e <= 1e-6
    for k, name in enumerate(("Bx", "By", "Bz")):
        e = relerr(F1[name] - F0[name], ref.B[k] - F0[name])
        _say(f"  {name} increment relerr {e:.2e}")
        assert e <= 1e-6


def test_fullsize_shock_fp32_learned():
    import paper_1412_2480_amd as pic
    from synth import loads
    nx, ny, ppc, g0 = 4096, 512, 32, 40.0
    x_out = nx - pic.PIC_WALL_GAP
    Q = loads.macro_charge(g0, DX, DX, ppc)
    _say("fullsize shock: generating load")
    ld = loads.shock_load(x_out, ny, ppc, g0, 0.01, 0)
    run = pic.run_desc(nx, ny, DX, 1.0, 0.6, 2, [(-Q, Q, ppc), (Q, Q, ppc)], cg_rtol=1e-8,
                       bc="shock")
    sim = pic.Sim([run], pic.make_options("fp32", tile=(16, 32), tile_split=1, slack=1.5, track_ids=False, solver="learned",
                                          precond_slots=4))
    for s in range(2):
        d = ld[s]
        sim.load_particles(0, s, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"])
    n0 = x_out * ny * ppc
    del ld
    injected = 0

    def inject(step):
        nonlocal injected
        for s, d in enumerate(loads.shock_injection(x_out, ny, ppc, g0, 0.01, 0, step, 1.0)):
            sim.inject_particles(0, s, d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"],
                                 d["uz"])
        injected += len(d["ix"])

    _say("fullsize shock: 4 plain-CG steps recording pairs")
    sim.precond_use(False)
    sim.precond_collect(True)
    plain_iters = []
    for step in range(4):
        inject(step)
        st = sim.step(1)[0]
        plain_iters.append(sum(st["iters"]))
    assert sim.precond_collect(False) == 4
    tr = sim.precond_train(epochs=8)
    _say(f"fullsize shock: trained {tr}")
    assert tr["loss_last"] < 0.1 * tr["loss_first"]
    sim.precond_use(True)
    for step in range(4, 8):
        inject(step)
        st = sim.step(1)[0]
        assert st["fallback"] == 0 and max(st["relres"]) <= 1e-8
        assert sum(st["iters"]) < min(plain_iters)
    _say(f"fullsize shock: plain {plain_iters}, learned last {st['iters']}")
    d = sim.diag(0)
    rho_scale = 4 * np.pi * Q / (DX * DX)
    _say(f"fullsize shock: gauss {d['gauss_max']:.3e} (scale {rho_scale:.3e}), "
         f"particles {d['n_particles']}")
    assert d["gauss_max"] <= 1e-4 * rho_scale
    for s in range(2):
        assert 0.95 * n0 <= d["n_particles"][s] <= n0 + injected
    F = {k: sim.get_field(0, k) for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")}
    for k in ("Ey", "Ez", "Bx"):
        assert np.all(F[k][:, 0] == 0) and np.all(F[k][:, nx - 1] == 0), k
    for k in ("Ex", "By", "Bz"):
        assert np.all(F[k][:, nx - 1] == 0), k
    assert np.abs(F["Bz"]).max() > 0
    sim.close()


def test_fullsize_tuned_schedule_full_length():
    """The benchmark workload for its full run length (2000 steps) in the
    timed configuration: 4 x 32 tiles, two work-groups per tile, half again
    the mean tile occupancy as slots (the bunching of the later phase, where
    the slow numerical instability of this set-up has grown, overflows the
    default quarter), reordering every 3 steps,
    graph replay, the learned aid trained on the first 8 solves. No tile
    overflows in 2000 steps, the last solve of every 249-step stretch meets
    the plain-CG residual without the fallback, every particle is kept, Gauss's
    law holds at FP64 roundoff and the energies stay finite."""
    import paper_1412_2480_amd as pic
    from synth import loads
    Q = loads.macro_charge(G0, DX, DX, PPC)
    run = pic.run_desc(NX, NY, DX, 1.0, 0.6, ORDER, [(-Q, Q, PPC), (Q, Q, PPC)], cg_rtol=1e-8)
    sim = pic.Sim([run], pic.make_options("fp32", tile=(4, 32), tile_split=2, sort_every=3, slack=0.5, track_ids=False,
                                          graph=True,
                                          solver="learned", precond_slots=8, diag_every=250,
                                          history_cap=16))
    for s in range(2):
        sim.load_plasma(0, s, PPC, G0, 0.01, 0)
    sim.precond_use(False)
    sim.precond_collect(True)
    sim.step(8)
    sim.precond_collect(False)
    tr = sim.precond_train(epochs=50)
    assert tr["loss_last"] < 1e-3 * tr["loss_first"]
    sim.precond_use(True)
    for chunk in range(8):
        st = sim.step(249)[0]
        _say(f"  step {8 + 249 * (chunk + 1)}: learned {st['learned_iters']}, relres "
             f"{max(st['relres']):.1e}, fallback {st['fallback']}")
        assert st["fallback"] == 0 and max(st["relres"]) <= 1e-8
    assert sim.get_timing()["graph_replays"] > 500
    d = sim.diag(0)
    rho_scale = 4 * np.pi * Q / (DX * DX)
    _say(f"  gauss {d['gauss_max']:.2e} (scale {rho_scale:.2e}), particles {d['n_particles']}")
    assert d["n_particles"][:2] == [NX * NY * PPC] * 2
    # charge and current from the same unit-sum FP64 weights: FP64 roundoff
    assert d["gauss_max"] <= 1e-9 * rho_scale
    h = sim.history(0)
    assert len(h) >= 8
    for r in h:
        tot = r["W_E"] + r["W_B"] + 0.5 * (r["W_K_minus"] + r["W_K_plus"])
        assert np.isfinite(tot) and tot > 0
    _say("  energy history: " + ", ".join(
        f"{r['step']}: {r['W_E'] + r['W_B']:.3e}" for r in h))
    sim.close()
